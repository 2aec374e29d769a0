// Multi-shift assembly of the shifted solutions (Appendix C/D: Eqs.
// shift_coeffs, search_dir_, solution_ket_).
//
// For shift w the algorithm updates, for m = 0, 1, ...,
//   p_m^w   = r_m / zeta_m + bw_m p_{m-1}^w,   bw_m = (zeta_{m-1}/zeta_m)^2 beta_{m-1}
//   Psi_{m+1}^w = Psi_m^w + aw_m p_m^w,        aw_m = (zeta_m/zeta_{m+1}) alpha_m
// so over a block of iterations [base, end) the result is linear in the seed
// residuals r_l kept in the bank:
//   Psi_end = Psi_base + (bw_base S_base) p_{base-1} + sum_l (S_l / zeta_l) r_l,
//   S_l = aw_l + bw_{l+1} S_{l+1},  S_end = 0,
// and, if the shift keeps iterating after the block,
//   p_{end-1} = (bw_base G_base) p_{base-1} + sum_l (G_l / zeta_l) r_l,
//   G_l = bw_{l+1} G_{l+1},  G_{end-1} = 1.
// k_coef evaluates these scalar recurrences (one thread per shift); k_flush
// then forms the dense contraction out[k] += sum_l C[k][l] r_l for all shifts
// at once, which replaces per-iteration sweeps over the n_shift x D vectors
// p^w and Psi^w by a single pass over them.
#include "k_common.h"

namespace msb {

__global__ __launch_bounds__(kBlock) void k_coef(CoefArgs a, double* scratch) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int total = a.nsys * a.n_list;
  if (tid >= total) return;
  const int s = tid / a.n_list;
  const int j = tid % a.n_list;
  double* crow = a.coef + (int64_t)tid * a.K * 2;
  double* grow = a.gcoef ? a.gcoef + (int64_t)tid * a.K * 2 : nullptr;
  double* zrow = scratch + (int64_t)tid * a.K * 4;    // (zeta_l, bw_l)
  const int k = a.list[tid];
  const int lend = (k >= 0) ? a.lend[tid] : 0;
  for (int l = lend; l < a.K; ++l) {
    crow[2 * l] = crow[2 * l + 1] = 0.0;
    if (grow) grow[2 * l] = grow[2 * l + 1] = 0.0;
  }
  double* ab = a.ab + (int64_t)tid * 4;
  ab[0] = ab[1] = ab[2] = ab[3] = 0.0;
  if (k < 0 || lend <= 0) return;

  const double w = a.wshift[k];
  const int end = a.base + lend;                       // absolute end of the range
  const int Mw = a.conv_iter[(int64_t)s * a.n_shift + k];
  const bool carry = (grow != nullptr) && (Mw < 0 || Mw > end);
  const double* al = a.alpha_log + (int64_t)s * a.maxit * 2;
  const double* be = a.beta_log + (int64_t)s * a.maxit * 2;

  // forward: zeta_m, aw_m, bw_m for m < end; stash the block part
  cv<double> z = {1.0, 0.0}, zp = {1.0, 0.0};          // zeta_0, zeta_{-1}
  cv<double> ap = {1.0, 0.0}, bp = {0.0, 0.0};         // alpha_{-1}, beta_{-1}
  for (int m = 0; m < end; ++m) {
    const cv<double> alpha = {al[2 * m], al[2 * m + 1]};
    const cv<double> cshift = cdiv(cmul(alpha, bp), ap);
    const cv<double> f = {1.0 - alpha.re * w, -alpha.im * w};
    const cv<double> zn = cadd(cmul(f, z), cmul(cshift, csub(z, zp)));
    if (m >= a.base) {
      const int l = m - a.base;
      const cv<double> aw = cmul(cdiv(z, zn), alpha);
      const cv<double> q = cdiv(zp, z);
      const cv<double> bw = cmul(cmul(q, q), bp);
      crow[2 * l] = aw.re;
      crow[2 * l + 1] = aw.im;
      zrow[4 * l + 0] = z.re;
      zrow[4 * l + 1] = z.im;
      zrow[4 * l + 2] = bw.re;
      zrow[4 * l + 3] = bw.im;
    }
    zp = z;
    z = zn;
    ap = alpha;
    bp = {be[2 * m], be[2 * m + 1]};
  }
  // backward accumulation
  cv<double> S = {0.0, 0.0}, G = {1.0, 0.0};
  for (int l = lend - 1; l >= 0; --l) {
    const cv<double> aw = {crow[2 * l], crow[2 * l + 1]};
    if (l < lend - 1) {
      const cv<double> bnext = {zrow[4 * (l + 1) + 2], zrow[4 * (l + 1) + 3]};
      S = cadd(aw, cmul(bnext, S));
      if (carry) G = cmul(bnext, G);
    } else {
      S = aw;
    }
    const cv<double> zl = {zrow[4 * l], zrow[4 * l + 1]};
    const cv<double> c = cdiv(S, zl);
    crow[2 * l] = c.re;
    crow[2 * l + 1] = c.im;
    if (grow) {
      const cv<double> g = carry ? cdiv(G, zl) : cv<double>{0.0, 0.0};
      grow[2 * l] = g.re;
      grow[2 * l + 1] = g.im;
    }
  }
  if (a.base > 0) {
    const cv<double> b0 = {zrow[2], zrow[3]};
    const cv<double> aps = cmul(b0, S);
    ab[0] = aps.re;
    ab[1] = aps.im;
    if (carry) {
      const cv<double> hp = cmul(b0, G);
      ab[2] = hp.re;
      ab[3] = hp.im;
    }
  }
}

hipError_t launch_coef(const CoefArgs& a, double* scratch, hipStream_t st) {
  const int total = a.nsys * a.n_list;
  const int blocks = (total + kBlock - 1) / kBlock;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_coef, dim3(blocks), dim3(kBlock), 0, st, a, scratch);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Flush: out[s][k][i] = ow_k * out[s][k][i] + pw_k * X[s][k][i] + sum_l C[s][j][l] r_l[i]
// One workgroup: 4 wavefronts x TS shifts (a shift tile) times 64*EPL
// elements; the residual tile is staged through LDS and shared by the four
// wavefronts, the coefficients are wave-uniform (scalar loads).
// Workgroups of one element tile are issued back to back on one XCD so the
// residual tile is read from HBM once and from that XCD's L2 afterwards.
constexpr int kFlushTS = 8;
constexpr int kFlushEPL = 4;
constexpr int kFlushKT = 8;
int flush_shifts_per_tile() { return kFlushTS * (kBlock / kWave); }
int flush_elems_per_tile() { return kWave * kFlushEPL; }

template <typename SB, typename SO>
__global__ __launch_bounds__(kBlock) void k_flush(FlushArgs a, int ow_mode) {
  constexpr int TS = kFlushTS, EPL = kFlushEPL, KT = kFlushKT;
  constexpr int TILE = kWave * EPL;
  using AB = Access<SB, true>;
  using AO = Access<SO, true>;
  __shared__ cv<double> rt[KT][TILE];

  const int s = blockIdx.y;
  const int b = blockIdx.x;
  const int xcd = b % kNumXcd, q = b / kNumXcd;
  const int et = xcd + kNumXcd * (q / a.n_stiles);
  const int stt = q % a.n_stiles;
  if (et >= a.n_etiles) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int slot0 = stt * (TS * (kBlock / kWave)) + wave * TS;
  const int Kext = a.tile_k[s * a.n_stiles + stt];
  const int64_t e0 = (int64_t)et * TILE;
  const void* bank_s = AB::offset(a.bank, (int64_t)s * a.cap * a.D);
  const double* crow = a.coef + ((int64_t)s * a.n_list + slot0) * a.K * 2;

  cv<double> acc[TS][EPL];
#pragma unroll
  for (int t = 0; t < TS; ++t)
#pragma unroll
    for (int e = 0; e < EPL; ++e) acc[t][e] = {0.0, 0.0};

  const int64_t my_i = e0 + threadIdx.x;
  for (int kb = 0; kb < Kext; kb += KT) {
#pragma unroll
    for (int kk = 0; kk < KT; ++kk) {
      const int l = kb + kk;
      cv<double> v = {0.0, 0.0};
      if (l < Kext && my_i < a.D) v = AB::template load<double>(bank_s, (int64_t)l * a.D + my_i);
      rt[kk][threadIdx.x] = v;
    }
    __syncthreads();
    const int kn = min(KT, Kext - kb);
    for (int kk = 0; kk < kn; ++kk) {
      cv<double> r[EPL];
#pragma unroll
      for (int e = 0; e < EPL; ++e) r[e] = rt[kk][lane + kWave * e];
#pragma unroll
      for (int t = 0; t < TS; ++t) {
        const double cr = crow[((int64_t)t * a.K + kb + kk) * 2];
        const double ci = crow[((int64_t)t * a.K + kb + kk) * 2 + 1];
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
          acc[t][e].re = fma(cr, r[e].re, acc[t][e].re);
          acc[t][e].re = fma(-ci, r[e].im, acc[t][e].re);
          acc[t][e].im = fma(cr, r[e].im, acc[t][e].im);
          acc[t][e].im = fma(ci, r[e].re, acc[t][e].im);
        }
      }
    }
    __syncthreads();
  }

#pragma unroll
  for (int t = 0; t < TS; ++t) {
    const int slot = slot0 + t;
    const int k = a.list[s * a.n_list + slot];
    if (k < 0) continue;
    cv<double> ow = {0.0, 0.0}, pw = {0.0, 0.0};
    if (ow_mode == 1) ow = {1.0, 0.0};
    if (ow_mode == 2) {
      const double* o = a.ow + ((int64_t)s * a.n_list + slot) * a.ow_stride;
      ow = {o[0], o[1]};
    }
    if (a.pw) {
      const double* p = a.pw + ((int64_t)s * a.n_list + slot) * a.pw_stride;
      pw = {p[0], p[1]};
    }
    const int64_t obase = ((int64_t)s * a.n_shift + k) * a.D;
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      const int64_t i = e0 + lane + kWave * e;
      if (i >= a.D) continue;
      cv<double> v = acc[t][e];
      if (ow_mode != 0) v = cadd(v, cmul(ow, AO::template load<double>(a.out, obase + i)));
      if (a.X) v = cadd(v, cmul(pw, AO::template load<double>(a.X, obase + i)));
      AO::store(a.out, obase + i, v);
    }
  }
}

hipError_t launch_flush(Elem eb, Elem eo, const FlushArgs& a, int ow_mode, hipStream_t st) {
  const int per_xcd = (a.n_etiles + kNumXcd - 1) / kNumXcd;
  dim3 grid(per_xcd * kNumXcd * a.n_stiles, a.nsys);
  if (eb == Elem::C128 && eo == Elem::C128)
    hipLaunchKernelGGL((k_flush<double, double>), grid, dim3(kBlock), 0, st, a, ow_mode);
  else if (eb == Elem::C64 && eo == Elem::C64)
    hipLaunchKernelGGL((k_flush<float, float>), grid, dim3(kBlock), 0, st, a, ow_mode);
  else if (eb == Elem::C64 && eo == Elem::C128)
    hipLaunchKernelGGL((k_flush<float, double>), grid, dim3(kBlock), 0, st, a, ow_mode);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace msb
