// Matrix-free Hamiltonian apply  v = (H' - c) x  for a batch of vectors.
//
// H' = H_up (x) I + I (x) H_dn + diag(U * #double + U_c n_core) (Sec. III,
// Eqs. Hubbard and intermediate_H) acting on the layout x[u * n_dn + d].
// One workgroup owns one up-spin row u of NV vectors (systems):
//   * the NV rows x_v[u, :] are staged once in LDS; the I (x) H_dn hops and
//     the diagonal read them from there.  The down-spin hops come from a
//     padded, transposed hop table (every lane runs the same unrolled loop with
//     coalesced table loads), and one table entry serves all NV vectors;
//   * the H_up (x) I hops read whole neighbour rows x_v[u', :] with coalesced
//     global loads (the hop list of u is uniform across the workgroup);
//   * the diagonal is recomputed from the occupation bits.
// Rows are assigned so that each XCD (workgroups are dispatched round-robin
// over the 8 XCDs) works on one contiguous range of u, which keeps
// neighbouring rows u' that differ only in low sites inside that XCD's L2.
// Optional fused reductions feed the COCG step (sigma = r^T A p), the
// Lanczos coefficient a_k = <q|H q>, or the true residual |E - (A - w) Psi|;
// their per-workgroup partials are summed by a finalize launch.
#include "k_common.h"

namespace msb {

template <typename S, typename Tc, bool CPLX, int EPT, int MODE, int NV>
__global__ __launch_bounds__(kBlock) void k_apply(ApplyArgs a) {
  using Ax = Access<S, CPLX>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cv<Tc>* rows = reinterpret_cast<cv<Tc>*>(smem_raw);    // [NV][nd]
  __shared__ Tc s_amp[NV][MSB_MAX_BOND_TYPES];

  const int tid = threadIdx.x;
  const int bx = blockIdx.x;
  const int s0 = blockIdx.y * NV;
  const int nd = a.T.n_dn;
  const int u = (bx % kNumXcd) * a.rows_per_xcd + bx / kNumXcd;
  const bool row_ok = u < a.T.n_up;

  bool act[NV];
  int64_t aux_off[NV];
  Tc Uv[NV], Ucv[NV], dre[NV], dim[NV];
  int core[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int s = s0 + v;
    act[v] = row_ok && s < a.nsys;
    if (act[v] && a.status) act[v] = (a.status[(int64_t)s * a.status_stride] == kActive);
    aux_off[v] = (int64_t)(s / a.aux_div) * a.D;
    if (act[v] && a.aux_m)
      aux_off[v] = ((int64_t)s * a.aux_cap + (a.aux_m[(int64_t)s * a.status_stride] - *a.aux_base)) * a.D;
    Uv[v] = Ucv[v] = dre[v] = dim[v] = (Tc)0;
    core[v] = -1;
    if (act[v]) {
      const SysDev* sd = a.sys + s;
      Uv[v] = (Tc)sd->U;
      Ucv[v] = (Tc)sd->Uc;
      dre[v] = (Tc)sd->d_re;
      dim[v] = (Tc)sd->d_im;
      core[v] = sd->core;
      if (tid < MSB_MAX_BOND_TYPES) s_amp[v][tid] = (Tc)sd->amp[tid];
    }
  }
  bool any = false;
#pragma unroll
  for (int v = 0; v < NV; ++v) any |= act[v];

  double part[NV][3];
#pragma unroll
  for (int v = 0; v < NV; ++v) part[v][0] = part[v][1] = part[v][2] = 0.0;

  if (any) {
    const int64_t row0 = (int64_t)u * nd;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if (!act[v]) continue;
      const void* x = Ax::offset(a.x, (int64_t)(s0 + v) * a.D);
#pragma unroll 4
      for (int i = tid; i < nd; i += kBlock) rows[v * nd + i] = Ax::template load<Tc>(x, row0 + i);
    }
    __syncthreads();

    const uint32_t cu = a.T.conf_up[u];
    cv<Tc> acc[NV][EPT];
    // diagonal
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int d = tid + e * kBlock;
      const uint32_t cd = (d < nd) ? a.T.conf_dn[d] : 0u;
      const Tc pc = (Tc)__builtin_popcount(cu & cd);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        acc[v][e] = {(Tc)0, (Tc)0};
        if (d < nd && act[v]) {
          Tc dg = Uv[v] * pc + dre[v];
          if (core[v] >= 0) dg += Ucv[v] * (Tc)(((cu >> core[v]) & 1u) + ((cd >> core[v]) & 1u));
          const cv<Tc> xd = rows[v * nd + d];
          acc[v][e].re = dg * xd.re - dim[v] * xd.im;
          acc[v][e].im = dg * xd.im + dim[v] * xd.re;
        }
      }
    }
    // I (x) H_dn: padded transposed hop table, one entry for all NV vectors
    const int kdn = a.T.k_dn;
#pragma unroll 2
    for (int k = 0; k < kdn; ++k) {
      uint32_t h[EPT];
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int d = tid + e * kBlock;
        h[e] = (d < nd) ? a.T.ell_dn[(int64_t)k * nd + d] : kNoHop;
      }
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        if (h[e] == kNoHop) continue;
        const uint32_t tgt = h[e] >> 16, ty = (h[e] >> 1) & 127u;
        const bool neg = (h[e] & 1u) == 0u;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          if (!act[v]) continue;
          Tc c = s_amp[v][ty];
          c = neg ? -c : c;
          const cv<Tc> xn = rows[v * nd + tgt];
          acc[v][e].re += c * xn.re;
          acc[v][e].im += c * xn.im;
        }
      }
    }
    // H_up (x) I: whole neighbour rows from global memory
    const uint32_t h0 = a.T.off_up[u], h1 = a.T.off_up[u + 1];
    for (uint32_t k = h0; k < h1; ++k) {
      const uint32_t h = a.T.hop_up[k];
      const uint32_t ty = (h >> 1) & 127u;
      const bool neg = (h & 1u) == 0u;
      const int64_t nrow = (int64_t)(h >> 16) * nd;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if (!act[v]) continue;
        Tc c = s_amp[v][ty];
        c = neg ? -c : c;
        const void* x = Ax::offset(a.x, (int64_t)(s0 + v) * a.D);
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          const int d = tid + e * kBlock;
          if (d < nd) {
            const cv<Tc> xn = Ax::template load<Tc>(x, nrow + d);
            acc[v][e].re += c * xn.re;
            acc[v][e].im += c * xn.im;
          }
        }
      }
    }
    // outputs
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if (!act[v]) continue;
      const int64_t vbase = (int64_t)(s0 + v) * a.D;
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int d = tid + e * kBlock;
        if (d >= nd) continue;
        const int64_t gi = row0 + d;
        const cv<Tc> vv = acc[v][e];
        if constexpr (MODE != kModeResid) Ax::store(a.v, vbase + gi, vv);
        if constexpr (MODE == kModeBilinear) {
          // sigma = sum r_i v_i (unconjugated, r^T v) with r the stored residual
          const cv<double> r = Ax::template load<double>(a.aux, aux_off[v] + gi);
          const cv<double> vs = {(double)(S)vv.re, (double)(S)vv.im};   // value as stored
          part[v][0] += r.re * vs.re - r.im * vs.im;
          part[v][1] += r.re * vs.im + r.im * vs.re;
          part[v][2] += vs.re * vs.re + vs.im * vs.im;
        } else if constexpr (MODE == kModeHerm) {
          const cv<Tc> qv = rows[v * nd + d];
          part[v][0] += (double)qv.re * (double)vv.re + (double)qv.im * (double)vv.im;
          part[v][1] += (double)qv.re * (double)vv.im - (double)qv.im * (double)vv.re;
          part[v][2] += (double)vv.re * (double)vv.re + (double)vv.im * (double)vv.im;
        } else if constexpr (MODE == kModeResid) {
          const cv<double> ee = Access<double, true>::template load<double>(a.aux, aux_off[v] + gi);
          const double dr = ee.re - (double)vv.re, di = ee.im - (double)vv.im;
          part[v][2] += dr * dr + di * di;
        }
      }
    }
  }
  if constexpr (MODE != kModePlain) {
    // every workgroup writes the partials of all its vectors (zeros if idle)
    __shared__ double sh[3 * NV][kBlock / kWave];
    double flat[3 * NV];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int i = 0; i < 3; ++i) flat[3 * v + i] = part[v][i];
    block_sum<3 * NV>(flat, sh);
    if (tid == 0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if (s0 + v >= a.nsys) continue;
#pragma unroll
        for (int i = 0; i < 3; ++i) a.partials[((int64_t)(s0 + v) * a.nbx + bx) * 4 + i] = flat[3 * v + i];
      }
    }
  }
}

int apply_rows_per_xcd(int n_up) { return (n_up + kNumXcd - 1) / kNumXcd; }
int apply_nbx(int n_up, int nsys) {
  (void)nsys;
  return apply_rows_per_xcd(n_up) * kNumXcd;   // one row per workgroup
}

// Vectors per workgroup: as many as keep the staged rows within 40 KB of LDS
// (four workgroups per CU), at most 4 and at most the number of systems.
static int pick_nv(int nd, size_t elem, int nsys, int ept) {
  if (ept > 8) return 1;
  int nv = 4;
  while (nv > 1 && ((size_t)nv * nd * elem > 40 * 1024 || nv > nsys)) nv /= 2;
  return nv;
}

template <typename S, typename Tc, bool CPLX, int MODE>
static hipError_t launch_ept(const ApplyArgs& a0, hipStream_t st) {
  ApplyArgs a = a0;
  const int nd = a.T.n_dn;
  const int need = (nd + kBlock - 1) / kBlock;
  const int nv = pick_nv(nd, sizeof(cv<Tc>), a.nsys, need);
  a.nvec = nv;
  dim3 grid(a.nbx, (a.nsys + nv - 1) / nv);
  const size_t lds = (size_t)nv * nd * sizeof(cv<Tc>);
  hipError_t err = hipErrorInvalidValue;
#define MSB_EPT_CASE(E, NVV)                                                              \
  else if (need <= E && nv == NVV) {                                                      \
    hipLaunchKernelGGL((k_apply<S, Tc, CPLX, E, MODE, NVV>), grid, dim3(kBlock), lds, st, a); \
    err = hipGetLastError();                                                              \
  }
  if (false) {}
  MSB_EPT_CASE(1, 4) MSB_EPT_CASE(1, 2) MSB_EPT_CASE(1, 1)
  MSB_EPT_CASE(2, 4) MSB_EPT_CASE(2, 2) MSB_EPT_CASE(2, 1)
  MSB_EPT_CASE(4, 4) MSB_EPT_CASE(4, 2) MSB_EPT_CASE(4, 1)
  MSB_EPT_CASE(8, 4) MSB_EPT_CASE(8, 2) MSB_EPT_CASE(8, 1)
  MSB_EPT_CASE(16, 1)
  MSB_EPT_CASE(24, 1)
#undef MSB_EPT_CASE
  if (err != hipSuccess || MODE == kModePlain) return err;
  return launch_reduce(a.partials, a.nbx, a.nsys, a.red, st);
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
