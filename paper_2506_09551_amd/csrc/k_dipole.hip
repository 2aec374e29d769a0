// Electron-number-changing site operators between two fixed-(N_up, N_dn)
// sectors of one lattice (the dipole-type O_1 / O_2 of Sec. III for edges
// that add or remove a valence electron):
//   y[v] = sum_j coef_j c+_{j s} x[v]   or   sum_j coef_j c_{j s} x[v].
// The operator changes one spin's configuration only, so every output
// element (u', d') gathers at most n_sites input elements of the same d'
// (up-spin operator: rows of the input) or the same u' (down-spin operator:
// columns within one input row).  The host tabulates, per site and output
// configuration of that spin, the input rank and the Jordan-Wigner sign.
#include "k_common.h"

namespace msb {

__global__ __launch_bounds__(kBlock) void k_dipole(DipoleArgs a) {
  const int v = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= a.D_dst) return;
  const int u = (int)(i / a.nd_dst), d = (int)(i % a.nd_dst);
  const int c = (a.spin == 0) ? u : d;
  const void* x = Access<double, true>::offset(a.x, (int64_t)v * a.D_src);
  cv<double> acc = {0.0, 0.0};
  for (int j = 0; j < a.n_sites; ++j) {
    const int e = a.table[(int64_t)j * a.n_conf + c];   // input rank << 1 | negative, or -1
    if (e < 0) continue;
    const int r = e >> 1;
    const int64_t src = (a.spin == 0) ? (int64_t)r * a.nd_src + d : (int64_t)u * a.nd_src + r;
    const cv<double> xv = Access<double, true>::template load<double>(x, src);
    const double s = (e & 1) ? -1.0 : 1.0;
    const cv<double> cf = {s * a.coef_re[j], s * a.coef_im[j]};
    acc = cadd(acc, cmul(cf, xv));
  }
  void* y = Access<double, true>::offset(a.y, (int64_t)v * a.D_dst);
  if (a.accumulate) acc = cadd(acc, Access<double, true>::template load<double>(y, i));
  Access<double, true>::store(y, i, acc);
}

hipError_t launch_dipole(const DipoleArgs& a, int nvec, hipStream_t st) {
  const int nb = (int)((a.D_dst + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_dipole, dim3(nb, nvec), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

}  // namespace msb
