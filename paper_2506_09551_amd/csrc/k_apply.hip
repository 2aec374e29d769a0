// Matrix-free Hamiltonian apply  v = (H' - c) x  for a batch of systems.
//
// H' = H_up (x) I + I (x) H_dn + diag(U * #double + U_c n_core) (Sec. III,
// Eqs. Hubbard and intermediate_H) acting on the layout x[u * n_dn + d].
// One workgroup owns one up-spin row u of one system:
//   * the row x[u, :] is staged once in LDS; the I (x) H_dn hops and the
//     diagonal read it from there;
//   * the H_up (x) I hops read whole neighbour rows x[u', :] with coalesced
//     global loads (the hop list of u is uniform across the workgroup);
//   * the diagonal is recomputed from the occupation bits.
// Rows are assigned so that each XCD (workgroups are dispatched round-robin
// over the 8 XCDs) works on one contiguous range of u, which keeps
// neighbouring rows u' that differ only in low sites inside that XCD's L2.
// Optional fused reductions feed the COCG step (sigma = r^T A p), the
// Lanczos coefficient a_k = <q|H q>, or the true residual |E - (A - w) Psi|.
#include "k_common.h"

namespace msb {

template <typename S, typename Tc, bool CPLX, int EPT, int MODE>
__global__ __launch_bounds__(kBlock) void k_apply(ApplyArgs a) {
  using Ax = Access<S, CPLX>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cv<Tc>* row = reinterpret_cast<cv<Tc>*>(smem_raw);
  __shared__ Tc s_amp[MSB_MAX_BOND_TYPES];

  const int tid = threadIdx.x;
  const int s = blockIdx.y;
  const int bx = blockIdx.x;
  const int nd = a.T.n_dn;
  // rows of this XCD: [xcd * rows_per_xcd, (xcd + 1) * rows_per_xcd), walked by
  // the nbx / 8 workgroups of this system that the hardware places on it
  const int xcd = bx % kNumXcd, q = bx / kNumXcd, nq = a.nbx / kNumXcd;
  const int r0 = xcd * a.rows_per_xcd;
  const int r1 = min(r0 + a.rows_per_xcd, a.T.n_up);

  double part[3] = {0.0, 0.0, 0.0};
  int64_t aux_off = (int64_t)(s / a.aux_div) * a.D;
  bool work = (r0 + q < r1);
  if (work && a.status) work = (a.status[(int64_t)s * a.status_stride] == kActive);
  if (work && a.aux_m)
    aux_off = ((int64_t)s * a.aux_cap + (a.aux_m[(int64_t)s * a.status_stride] - *a.aux_base)) * a.D;

  if (work) {
    const SysDev* sd = a.sys + s;
    if (tid < MSB_MAX_BOND_TYPES) s_amp[tid] = (Tc)sd->amp[tid];
    const void* x = Ax::offset(a.x, (int64_t)s * a.D);
    const Tc Uv = (Tc)sd->U, Uc = (Tc)sd->Uc, dre = (Tc)sd->d_re, dim = (Tc)sd->d_im;
    const int core = sd->core;

    for (int u = r0 + q; u < r1; u += nq) {
      const int64_t row0 = (int64_t)u * nd;
      __syncthreads();                       // previous row fully consumed
#pragma unroll 4
      for (int i = tid; i < nd; i += kBlock) row[i] = Ax::template load<Tc>(x, row0 + i);
      __syncthreads();

      const uint32_t cu = a.T.conf_up[u];
      const Tc nu_core = (core >= 0) ? (Tc)((cu >> core) & 1u) : (Tc)0;
      cv<Tc> acc[EPT];
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int d = tid + e * kBlock;
        acc[e] = {(Tc)0, (Tc)0};
        if (d < nd) {
          const uint32_t cd = a.T.conf_dn[d];
          Tc dg = Uv * (Tc)__builtin_popcount(cu & cd) + dre;
          if (core >= 0) dg += Uc * (nu_core + (Tc)((cd >> core) & 1u));
          const cv<Tc> xd = row[d];
          acc[e].re = dg * xd.re - dim * xd.im;
          acc[e].im = dg * xd.im + dim * xd.re;
          const uint32_t k0 = a.T.off_dn[d], k1 = a.T.off_dn[d + 1];
          for (uint32_t k = k0; k < k1; ++k) {
            const uint32_t h = a.T.hop_dn[k];
            Tc c = s_amp[(h >> 1) & 127u];
            c = (h & 1u) ? c : -c;
            const cv<Tc> xn = row[h >> 16];
            acc[e].re += c * xn.re;
            acc[e].im += c * xn.im;
          }
        }
      }

      const uint32_t h0 = a.T.off_up[u], h1 = a.T.off_up[u + 1];
      for (uint32_t k = h0; k < h1; ++k) {
        const uint32_t h = a.T.hop_up[k];
        Tc c = s_amp[(h >> 1) & 127u];
        c = (h & 1u) ? c : -c;
        const int64_t nrow = (int64_t)(h >> 16) * nd;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          const int d = tid + e * kBlock;
          if (d < nd) {
            const cv<Tc> xn = Ax::template load<Tc>(x, nrow + d);
            acc[e].re += c * xn.re;
            acc[e].im += c * xn.im;
          }
        }
      }

#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int d = tid + e * kBlock;
        if (d >= nd) continue;
        const int64_t gi = row0 + d;
        const cv<Tc> vv = acc[e];
        if constexpr (MODE != kModeResid) {
          Ax::store(a.v, (int64_t)s * a.D + gi, vv);
        }
        if constexpr (MODE == kModeBilinear) {
          // sigma = sum r_i v_i (unconjugated, r^T v) with r the stored residual
          const cv<double> r = Ax::template load<double>(a.aux, aux_off + gi);
          const cv<double> vs = {(double)(S)vv.re, (double)(S)vv.im};   // value as stored
          part[0] += r.re * vs.re - r.im * vs.im;
          part[1] += r.re * vs.im + r.im * vs.re;
          part[2] += vs.re * vs.re + vs.im * vs.im;
        } else if constexpr (MODE == kModeHerm) {
          const cv<Tc> qv = row[d];
          part[0] += (double)qv.re * (double)vv.re + (double)qv.im * (double)vv.im;
          part[1] += (double)qv.re * (double)vv.im - (double)qv.im * (double)vv.re;
          part[2] += (double)vv.re * (double)vv.re + (double)vv.im * (double)vv.im;
        } else if constexpr (MODE == kModeResid) {
          const cv<double> ee = Access<double, true>::template load<double>(a.aux, aux_off + gi);
          const double dr = ee.re - (double)vv.re, di = ee.im - (double)vv.im;
          part[2] += dr * dr + di * di;
        }
      }
    }
  }
  if constexpr (MODE != kModePlain) {
    publish_partials<3>(part, a.partials, a.counter, a.red, a.nbx, s, bx);
  }
}

int apply_rows_per_xcd(int n_up) { return (n_up + kNumXcd - 1) / kNumXcd; }
int apply_nbx(int n_up, int nsys) {
  const int rpx = apply_rows_per_xcd(n_up);
  int per_xcd = (2048 / kNumXcd + nsys - 1) / nsys;   // about 2048 workgroups in total
  if (per_xcd < 1) per_xcd = 1;
  if (per_xcd > rpx) per_xcd = rpx;
  return per_xcd * kNumXcd;
}

template <typename S, typename Tc, bool CPLX, int MODE>
static hipError_t launch_ept(const ApplyArgs& a, hipStream_t st) {
  const int nd = a.T.n_dn;
  const int need = (nd + kBlock - 1) / kBlock;
  dim3 grid(a.nbx, a.nsys);
  const size_t lds = (size_t)nd * sizeof(cv<Tc>);
#define MSB_EPT_CASE(E)                                                             \
  if (need <= E) {                                                                  \
    hipLaunchKernelGGL((k_apply<S, Tc, CPLX, E, MODE>), grid, dim3(kBlock), lds, st, a); \
    return hipGetLastError();                                                       \
  }
  MSB_EPT_CASE(1)
  MSB_EPT_CASE(2)
  MSB_EPT_CASE(4)
  MSB_EPT_CASE(8)
  MSB_EPT_CASE(16)
  MSB_EPT_CASE(24)
#undef MSB_EPT_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_apply(Elem e, int mode, const ApplyArgs& a, hipStream_t st) {
  switch (e) {
    case Elem::R64:
      if (mode == kModePlain) return launch_ept<double, double, false, kModePlain>(a, st);
      if (mode == kModeHerm) return launch_ept<double, double, false, kModeHerm>(a, st);
      break;
    case Elem::C128:
      if (mode == kModePlain) return launch_ept<double, double, true, kModePlain>(a, st);
      if (mode == kModeBilinear) return launch_ept<double, double, true, kModeBilinear>(a, st);
      if (mode == kModeHerm) return launch_ept<double, double, true, kModeHerm>(a, st);
      if (mode == kModeResid) return launch_ept<double, double, true, kModeResid>(a, st);
      break;
    case Elem::C64:
      if (mode == kModePlain) return launch_ept<float, float, true, kModePlain>(a, st);
      if (mode == kModeBilinear) return launch_ept<float, float, true, kModeBilinear>(a, st);
      if (mode == kModeResid) return launch_ept<float, double, true, kModeResid>(a, st);
      break;
  }
  return hipErrorInvalidValue;
}

}  // namespace msb
