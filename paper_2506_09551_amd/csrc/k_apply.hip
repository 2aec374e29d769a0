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
// The ordered form instead lists the rows of all systems in level order
// (TablesDev::order_up) and gives each XCD one contiguous eighth of that
// list: on chains a row's up-spin neighbours lie in the adjacent levels, so
// they are still in the XCD's L2 from the rows just before.
// Optional fused reductions feed the COCG step (sigma = r^T A p), the
// Lanczos coefficient a_k = <q|H q>, or the true residual |E - (A - w) Psi|;
// their per-workgroup partials are summed by a finalize launch.
#include "k_common.h"

namespace msb {

// Amplitude with its sign flipped when bit 31 of `sb` is set (sign bits of
// the hop entries; no branch and no select).
__device__ __forceinline__ float flip_sign(float a, uint32_t sb) {
  return __int_as_float(__float_as_int(a) ^ (int)sb);
}
__device__ __forceinline__ double flip_sign(double a, uint32_t sb) {
  return __longlong_as_double(__double_as_longlong(a) ^ ((long long)sb << 32));
}

// 1024-thread shapes with few elements per thread ask for 8 waves per SIMD
// (at most 64 VGPRs), so that two workgroups share a CU.
template <typename S, typename Tc, bool CPLX, int EPT, int MODE, int NV, int BLK>
__global__ __launch_bounds__(BLK, (BLK >= 1024 && EPT * NV <= 5) ? 8 : 1) void k_apply(ApplyArgs a) {
  using Ax = Access<S, CPLX>;
  constexpr bool kSelf = MODE == kModeSelf;   // operand = the aux bank slot, in place
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cv<Tc>* rows = reinterpret_cast<cv<Tc>*>(smem_raw);    // [NV][nd + 1], element nd = 0

  const int tid = threadIdx.x;
  const int nd = a.T.n_dn;
  const int ldr = nd + 1;
  // (system group, row) of this workgroup and its column in the partials
  int s0, u, bx;
  if (a.ordered) {
    const int per_xcd = gridDim.x / kNumXcd;            // grid.x = groups * nbx, nbx % 8 == 0
    const int item = (blockIdx.x % kNumXcd) * per_xcd + blockIdx.x / kNumXcd;
    bx = item % a.nbx;
    s0 = (item / a.nbx) * NV;
    u = bx < a.T.n_up ? (int)a.T.order_up[bx] : a.T.n_up;
  } else {
    bx = blockIdx.x;
    s0 = blockIdx.y * NV;
    u = (bx % kNumXcd) * a.rows_per_xcd + bx / kNumXcd;
  }
  const bool row_ok = u < a.T.n_up;

  bool act[NV];
  int64_t aux_off[NV];
  Tc Uv[NV], Ucv[NV], dre[NV], dim[NV];
  int core[NV];
  // status and bank slot are loaded side by side (neither waits for the
  // other): every operand load of the workgroup waits for them
  const int abase = a.aux_m ? *a.aux_base : 0;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int s = s0 + v;
    const bool in = row_ok && s < a.nsys;
    const int stv = (in && a.status) ? a.status[(int64_t)s * a.status_stride] : (int)kActive;
    const int mv = (in && a.aux_m) ? a.aux_m[(int64_t)s * a.status_stride] : 0;
    act[v] = in && stv == (int)kActive;
    aux_off[v] = (int64_t)(s / a.aux_div) * a.D;
    if (in && a.aux_m) {
      // clamped: an idle system's m may lie past the bank (its slot is read
      // with coefficient 0 or not at all)
      int slot = mv - abase;
      slot = slot < 0 ? 0 : (slot >= a.aux_cap ? a.aux_cap - 1 : slot);
      aux_off[v] = ((int64_t)s * a.aux_cap + slot) * a.D;
    }
    Uv[v] = Ucv[v] = dre[v] = dim[v] = (Tc)0;
    core[v] = -1;
    if (act[v]) {
      const SysDev* sd = a.sys + s;
      Uv[v] = (Tc)sd->U;
      Ucv[v] = (Tc)sd->Uc;
      dre[v] = (Tc)sd->d_re;
      dim[v] = (Tc)sd->d_im;
      core[v] = sd->core;
    }
  }
  bool any = false;
#pragma unroll
  for (int v = 0; v < NV; ++v) any |= act[v];
  // operand of each vector: x[s] or, when the operand is the aux bank slot
  // itself, that slot; a ragged last group's slots past the last system
  // point at system s0 (always present) and are added with coefficient 0
  int64_t xoff[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const bool in = s0 + v < a.nsys;
    xoff[v] = kSelf ? aux_off[in ? v : 0] : (int64_t)(in ? s0 + v : s0) * a.D;
  }

  double part[NV][3];
#pragma unroll
  for (int v = 0; v < NV; ++v) part[v][0] = part[v][1] = part[v][2] = 0.0;

  if (any) {
    const int64_t row0 = (int64_t)u * nd;
    // columns d = tid + e * BLK; idle lanes (d >= nd) read column nd - 1 and
    // store nothing, so every load below is unconditional
    uint32_t voff[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int d = tid + e * BLK;
      voff[e] = (uint32_t)(d < nd ? d : nd - 1);
    }
    // own row elements in registers (diagonal, staging)
    cv<Tc> xs[NV][EPT];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const void* x = Ax::offset(kSelf ? a.aux : a.x, xoff[v] + row0);
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        xs[v][e] = act[v] ? Ax::template load<Tc>(x, voff[e]) : cv<Tc>{(Tc)0, (Tc)0};
      }
    }
    // the operand of the fused reduction (r for sigma, E for the residual) is
    // requested now, so that its latency hides behind the hops
    constexpr bool kAuxEarly = (MODE == kModeBilinear || MODE == kModeResid) && EPT * NV <= 8 && BLK < 1024;
    cv<double> auxv[kAuxEarly ? NV : 1][kAuxEarly ? EPT : 1];
    if constexpr (kAuxEarly) {
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          auxv[v][e] = {0.0, 0.0};
          if (v > 0 && act[v] && aux_off[v] == aux_off[v - 1]) {
            auxv[v][e] = auxv[v - 1][e];       // shifts of one system share their right-hand side
          } else if (act[v]) {
            if constexpr (MODE == kModeBilinear)
              auxv[v][e] = Ax::template load_nt<double>(a.aux, aux_off[v] + row0 + voff[e]);
            else
              auxv[v][e] = Access<double, true>::template load_nt<double>(a.aux, aux_off[v] + row0 + voff[e]);
          }
        }
    }
    const bool second_pass = a.vin != nullptr;   // diagonal and up-spin hops already in vin
    // kModeSelf: the old v (added as beta v) is requested now as well; with
    // beta = 0 (first iteration) the loaded values are not used
    constexpr bool kOldEarly = kSelf && EPT * NV <= 8 && BLK < 1024;
    cv<Tc> vold[kOldEarly ? NV : 1][kOldEarly ? EPT : 1];
    if constexpr (kOldEarly) {
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          vold[v][e] = {(Tc)0, (Tc)0};
          if (act[v] && a.beta && !second_pass)
            vold[v][e] = Ax::template load_nt<Tc>(a.v, (int64_t)(s0 + v) * a.D + row0 + voff[e]);
        }
    }
    const uint32_t cu = a.T.conf_up[u];
    cv<Tc> acc[NV][EPT];
    // diagonal
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int d = tid + e * BLK;
      const uint32_t cd = a.T.conf_dn[voff[e]];
      const Tc pc = (Tc)__builtin_popcount(cu & cd);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if (second_pass) {
          acc[v][e] = act[v] ? Ax::template load<Tc>(Ax::offset(a.vin, (int64_t)(s0 + v) * a.D + row0), voff[e])
                             : cv<Tc>{(Tc)0, (Tc)0};
        } else {
          Tc dg = Uv[v] * pc + dre[v];
          if (core[v] >= 0) dg += Ucv[v] * (Tc)(((cu >> core[v]) & 1u) + ((cd >> core[v]) & 1u));
          acc[v][e].re = dg * xs[v][e].re - dim[v] * xs[v][e].im;
          acc[v][e].im = dg * xs[v][e].im + dim[v] * xs[v][e].re;
        }
        if (d < nd) rows[v * ldr + d] = xs[v][e];
      }
    }
    if (tid < NV) rows[tid * ldr + nd] = cv<Tc>{(Tc)0, (Tc)0};
    // H_up (x) I: whole neighbour rows from global memory.  The hop list of u
    // is uniform across the workgroup (scalar loads; the coefficient is a
    // scalar), and HG hops are loaded before their FMAs are issued.
    // (256-thread shapes have the registers for twice as many)
    constexpr int kLoadsInFlight = (sizeof(Tc) == 4 ? 12 : 8) * (BLK >= 1024 ? 1 : 2);
    constexpr int HG = (EPT * NV >= kLoadsInFlight) ? 1 : kLoadsInFlight / (EPT * NV);
    const void* xsrc = kSelf ? a.aux : a.x;
    const int h0 = second_pass ? 0 : (int)a.T.off_up[u];
    const int nh = second_pass ? 0 : (int)a.T.off_up[u + 1] - h0;
    auto up_hops = [&](auto G, int k) {
      constexpr int NG = decltype(G)::value;
      cv<Tc> xn[NG][NV][EPT];
      Tc cf[NG][NV];
#pragma unroll
      for (int j = 0; j < NG; ++j) {
        const uint32_t h = a.T.hop_up[h0 + k + j];
        const uint32_t ty = (h >> 1) & (MSB_MAX_BOND_TYPES - 1);
        const uint32_t sb = (h & 1u) ? 0u : 0x80000000u;      // parity 0: -t
        const int64_t nrow = (int64_t)(h >> 16) * nd;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          cf[j][v] = act[v] ? flip_sign((Tc)a.sys[s0 + v].amp[ty], sb) : (Tc)0;
          const void* x = Ax::offset(xsrc, xoff[v] + nrow);
#pragma unroll
          for (int e = 0; e < EPT; ++e) xn[j][v][e] = Ax::template load<Tc>(x, voff[e]);
        }
      }
#pragma unroll
      for (int j = 0; j < NG; ++j)
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
          for (int e = 0; e < EPT; ++e) {
            acc[v][e].re += cf[j][v] * xn[j][v][e].re;
            acc[v][e].im += cf[j][v] * xn[j][v][e].im;
          }
    };
    int k = 0;
    for (; k + HG <= nh; k += HG) up_hops(std::integral_constant<int, HG>{}, k);
    for (; k < nh; ++k) up_hops(std::integral_constant<int, 1>{}, k);
    __syncthreads();   // staged rows complete
    // I (x) H_dn: one padded, transposed hop table per bond type; a 64-bit
    // word holds four hops of a state as 16-bit entries (target column, the
    // parity-0 sign in bit 15), padding points at the zero element nd.  The
    // next word (four hops ahead) is prefetched.
    const uint64_t* ell = a.T.ell_dn;
    for (int t = 0; t < a.T.n_types; ++t) {
      const int kq = a.T.k_type[t];
      Tc amp[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) amp[v] = act[v] ? (Tc)a.sys[s0 + v].amp[t] : (Tc)0;
      uint64_t hn[EPT];
      if (kq > 0) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) hn[e] = ell[voff[e]];
      }
      for (int g = 0; g < kq; ++g) {
        uint32_t hw[EPT][2];
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          hw[e][0] = (uint32_t)hn[e];
          hw[e][1] = (uint32_t)(hn[e] >> 32);
        }
        if (g + 1 < kq) {
          const uint64_t* nxt = ell + (int64_t)(g + 1) * nd;
#pragma unroll
          for (int e = 0; e < EPT; ++e) hn[e] = nxt[voff[e]];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int e = 0; e < EPT; ++e) {
            const uint32_t ent = (hw[e][j >> 1] >> (16 * (j & 1))) & 0xFFFFu;
            const uint32_t sb = (ent & 0x8000u) << 16;
            const int tgt = (int)(ent & 0x7FFFu);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
              const Tc c = flip_sign(amp[v], sb);
              const cv<Tc> xv = rows[v * ldr + tgt];
              acc[v][e].re += c * xv.re;
              acc[v][e].im += c * xv.im;
            }
          }
      }
      ell += (int64_t)kq * nd;
    }
    // outputs
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if (!act[v]) continue;
      const int64_t vbase = (int64_t)(s0 + v) * a.D;
      // kModeSelf: v = A x + beta_s v (loaded here, so it holds no register
      // through the hops; 0: the old v is not read)
      cv<Tc> bacc = {(Tc)0, (Tc)0};
      if (kSelf && a.beta)
        bacc = {(Tc)a.beta[(int64_t)(s0 + v) * a.beta_stride], (Tc)a.beta[(int64_t)(s0 + v) * a.beta_stride + 1]};
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int d = tid + e * BLK;
        if (d >= nd) continue;
        const int64_t gi = row0 + d;
        cv<Tc> vv = acc[v][e];
        if constexpr (kSelf) {
          // v_m = A r_m + beta_{m-1} v_{m-1}, in place (the first pass already added it)
          if (!second_pass && (bacc.re != (Tc)0 || bacc.im != (Tc)0)) {
            cv<Tc> vo;
            if constexpr (kOldEarly) vo = vold[v][e];
            else vo = Ax::template load_nt<Tc>(a.v, vbase + gi);
            vv.re += bacc.re * vo.re - bacc.im * vo.im;
            vv.im += bacc.re * vo.im + bacc.im * vo.re;
          }
        }
        if constexpr (MODE != kModeResid) Ax::store_nt(a.v, vbase + gi, vv);
        if constexpr (MODE == kModeBilinear || kSelf) {
          // sigma = sum r_i v_i (unconjugated, r^T v) with r the stored residual
          // (the staged row when the operand is r itself)
          cv<double> r;
          if constexpr (kSelf) {
            const cv<Tc> q = rows[v * ldr + d];
            r = {(double)q.re, (double)q.im};
          } else if constexpr (kAuxEarly) {
            r = auxv[v][e];
          } else {
            r = Ax::template load_nt<double>(a.aux, aux_off[v] + gi);
          }
          const cv<double> vs = {(double)(S)vv.re, (double)(S)vv.im};   // value as stored
          part[v][0] += r.re * vs.re - r.im * vs.im;
          part[v][1] += r.re * vs.im + r.im * vs.re;
          part[v][2] += vs.re * vs.re + vs.im * vs.im;
        } else if constexpr (MODE == kModeHerm) {
          const cv<Tc> qv = rows[v * ldr + d];   // the staged operand (frees xs early)
          part[v][0] += (double)qv.re * (double)vv.re + (double)qv.im * (double)vv.im;
          part[v][1] += (double)qv.re * (double)vv.im - (double)qv.im * (double)vv.re;
          part[v][2] += (double)vv.re * (double)vv.re + (double)vv.im * (double)vv.im;
        } else if constexpr (MODE == kModeResid) {
          cv<double> ee;
          if constexpr (kAuxEarly) ee = auxv[v][e];
          else ee = Access<double, true>::template load_nt<double>(a.aux, aux_off[v] + gi);
          const double dr = ee.re - (double)vv.re, di = ee.im - (double)vv.im;
          part[v][2] += dr * dr + di * di;
        }
      }
    }
  }
  if constexpr (MODE != kModePlain) {
    // every workgroup writes the partials of all its vectors (zeros if idle)
    __shared__ double sh[3 * NV][BLK / kWave];
    double flat[3 * NV];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int i = 0; i < 3; ++i) flat[3 * v + i] = part[v][i];
    block_sum<3 * NV, BLK>(flat, sh);
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

// ---- first pass of the two-pass apply: diagonal and H_up (x) I ------------
// v[u][d] = diag(u, d) x[u][d] + sum_u' T_up[u][u'] x[u'][d] on column panels
// of kPanel down-spin states.  The panels are dealt to the XCDs round robin
// (panel p on XCD p % 8) and one XCD works through a panel before the next, so
// the panel (n_up x kPanel elements, 2.2 MB for 4368 rows in complex64) stays
// in that XCD's L2 while every row gathers its up-spin neighbours from it.
// A workgroup takes kRowsPerWg consecutive rows of one panel: it first lists
// their work items in LDS (per row the diagonal, then every up-spin hop with
// its signed amplitude), then each wavefront walks the items of its own rows
// (one column per lane) with the neighbour-row load kPrefetch items ahead of
// its use, across row boundaries, so the gathers stay in flight.  The row
// kernel then adds I (x) H_dn in place (ApplyArgs::vin).
constexpr int kPanel = 64, kRowsPerWg = 16, kPanelItems = 1024, kPrefetch = 8;
constexpr uint32_t kDiagItem = 0x80000000u;

int panel_nbx(int n_up, int n_dn) {
  const int n_panels = (n_dn + kPanel - 1) / kPanel;
  const int chunks = (n_up + kRowsPerWg - 1) / kRowsPerWg;
  return kNumXcd * ((n_panels + kNumXcd - 1) / kNumXcd) * chunks;
}
bool panel_fits(int k_up_max) { return kRowsPerWg * (1 + k_up_max) <= kPanelItems; }

template <typename S, typename Tc, bool CPLX>
__global__ __launch_bounds__(256) void k_apply_up(ApplyArgs a) {
  using Ax = Access<S, CPLX>;
  __shared__ int s_off[kRowsPerWg + 1];
  __shared__ uint32_t s_tgt[kPanelItems];     // input row (kDiagItem | u for a row's diagonal)
  __shared__ Tc s_cf[kPanelItems];            // signed hop amplitude
  const int s = blockIdx.y;
  const int nd = a.T.n_dn, nu = a.T.n_up;
  const int chunks = (nu + kRowsPerWg - 1) / kRowsPerWg;
  const int x = blockIdx.x % kNumXcd, l = blockIdx.x / kNumXcd;
  const int panel = x + kNumXcd * (l / chunks), chunk = l % chunks;
  if (panel * kPanel >= nd) return;
  if (a.status && a.status[(int64_t)s * a.status_stride] != kActive) return;
  const SysDev* sd = a.sys + s;
  const int r0 = chunk * kRowsPerWg;
  const int nrows = min(kRowsPerWg, nu - r0);
  if (threadIdx.x == 0) {
    int o = 0;
    for (int r = 0; r < nrows; ++r) {
      s_off[r] = o;
      o += 1 + (int)(a.T.off_up[r0 + r + 1] - a.T.off_up[r0 + r]);
    }
    s_off[nrows] = o;                          // <= kPanelItems (panel_fits on the host)
  }
  __syncthreads();
  const int n_items = s_off[nrows];
  for (int t = threadIdx.x; t < n_items; t += blockDim.x) {
    int r = 0;
    while (t >= s_off[r + 1]) ++r;
    const int u = r0 + r, k = t - s_off[r];
    if (k == 0) {
      s_tgt[t] = kDiagItem | (uint32_t)u;
      s_cf[t] = (Tc)0;
    } else {
      const uint32_t h = a.T.hop_up[a.T.off_up[u] + k - 1];
      s_tgt[t] = h >> 16;
      s_cf[t] = flip_sign((Tc)sd->amp[(h >> 1) & (MSB_MAX_BOND_TYPES - 1)], (h & 1u) ? 0u : 0x80000000u);
    }
  }
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rows_per_wave = kRowsPerWg / 4;
  const int i0 = s_off[min(wave * rows_per_wave, nrows)];
  const int i1 = s_off[min((wave + 1) * rows_per_wave, nrows)];
  const int d = panel * kPanel + lane;
  const bool ok = d < nd;
  const uint32_t dc = (uint32_t)(ok ? d : nd - 1);        // idle lanes read a valid column
  const uint32_t cd = a.T.conf_dn[dc];
  const Tc U = (Tc)sd->U, Uc = (Tc)sd->Uc, dre = (Tc)sd->d_re, dim = (Tc)sd->d_im;
  const int core = sd->core;
  // the operand: x[s], or the aux bank slot of an active system
  const int64_t xo = (a.x_from_aux && a.aux_m)
                         ? ((int64_t)s * a.aux_cap + (a.aux_m[(int64_t)s * a.status_stride] - *a.aux_base)) * a.D
                         : (int64_t)s * a.D;
  const void* xsys = Ax::offset(a.x_from_aux ? a.aux : a.x, xo);
  void* vv = Ax::offset(a.v, (int64_t)s * a.D);
  // kModeSelf: v = A x + beta_s v, the old v added here (the row pass does not)
  cv<Tc> bs = {(Tc)0, (Tc)0};
  if (a.x_from_aux && a.beta) bs = {(Tc)a.beta[(int64_t)s * a.beta_stride], (Tc)a.beta[(int64_t)s * a.beta_stride + 1]};
  const bool badd = bs.re != (Tc)0 || bs.im != (Tc)0;
  auto put = [&](int r, cv<Tc> v) {
    const int64_t o = (int64_t)r * nd + d;
    if (badd) {
      const cv<Tc> vo = Ax::template load<Tc>(vv, o);
      v.re += bs.re * vo.re - bs.im * vo.im;
      v.im += bs.re * vo.im + bs.im * vo.re;
    }
    Ax::store(vv, o, v);
  };
  cv<Tc> buf[kPrefetch];
#pragma unroll
  for (int j = 0; j < kPrefetch; ++j)
    if (i0 + j < i1) buf[j] = Ax::template load<Tc>(xsys, (int64_t)(s_tgt[i0 + j] & ~kDiagItem) * nd + dc);
  int row = -1;
  cv<Tc> acc = {(Tc)0, (Tc)0};
  for (int i = i0; i < i1; i += kPrefetch) {
#pragma unroll
    for (int j = 0; j < kPrefetch; ++j) {
      const int it = i + j;
      if (it < i1) {                          // uniform across the wavefront
        const uint32_t tg = s_tgt[it];
        const cv<Tc> xv = buf[j];
        if (it + kPrefetch < i1)
          buf[j] = Ax::template load<Tc>(xsys, (int64_t)(s_tgt[it + kPrefetch] & ~kDiagItem) * nd + dc);
        if (tg & kDiagItem) {
          if (row >= 0 && ok) put(row, acc);
          row = (int)(tg & ~kDiagItem);
          const uint32_t cu = a.T.conf_up[row];
          Tc dg = U * (Tc)__builtin_popcount(cu & cd) + dre;
          if (core >= 0) dg += Uc * (Tc)(((cu >> core) & 1u) + ((cd >> core) & 1u));
          acc = {dg * xv.re - dim * xv.im, dg * xv.im + dim * xv.re};
        } else {
          const Tc c = s_cf[it];
          acc.re += c * xv.re;
          acc.im += c * xv.im;
        }
      }
    }
  }
  if (row >= 0 && ok) put(row, acc);
}

// ---- first pass on LDS-staged column panels (passes = 3) --------------------
// One workgroup stages the panel x[:, c0 .. c0 + W) of one system -- every
// up-spin row, W down-spin columns, and a zero row at index n_up -- in LDS
// (global_load_lds, 16 bytes per lane straight from memory), then each thread
// forms whole rows of the panel: the diagonal and every up-spin hop, read from
// LDS through the padded, transposed up-spin table, so one table word and one
// LDS read of W elements serve W columns and no neighbour row is fetched from
// the caches again.  The Q panels that share a 128-byte line run side by side
// on one XCD, so the line leaves HBM once.  The row kernel then adds
// I (x) H_dn in place (ApplyArgs::vin); in the recurred mode (x_from_aux) the
// old v is added here with its beta, as in k_apply_up.
template <int W, typename S>
constexpr int pan_lines() {
  return (W * (int)sizeof(cv<S>) >= 128) ? 1 : 128 / (W * (int)sizeof(cv<S>));
}
size_t pan_lds_bytes(int n_up, int W, size_t es) {
  const size_t units = ((size_t)n_up * W * es + 15) / 16;
  const size_t staged = (units + kWave - 1) / kWave * kWave * 16;   // whole wavefront loads
  const size_t need = (size_t)(n_up + 1) * W * es;
  return staged > need ? staged : need;
}
// 1024 threads (16 wavefronts to hide the LDS latency) unless the rows are
// few or a row of W elements needs more registers than 1024 threads have
int pan_block(int n_up, int W, size_t es) { return (n_up > 600 && W * es <= 64) ? 1024 : 256; }

template <typename S, int W, int BLK>
__global__ __launch_bounds__(BLK) void k_apply_pan(ApplyArgs a) {
  using V16 = typename std::conditional<std::is_same<S, double>::value, double2, float4>::type;
  constexpr int ES = (int)sizeof(cv<S>);
  constexpr int CPR = W * ES / 16;                         // 16-byte units of a panel row
  static_assert(CPR >= 1 && (W * ES) % 16 == 0, "panel rows are whole 16-byte units");
  constexpr int Q = pan_lines<W, S>();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cv<S>* pan = reinterpret_cast<cv<S>*>(smem_raw);         // [n_up + 1][W]
  const int nd = a.T.n_dn, nu = a.T.n_up;
  const int s = blockIdx.y;
  const int xq = blockIdx.x % kNumXcd, l = blockIdx.x / kNumXcd;
  const int c0 = ((l % Q) + Q * (xq + kNumXcd * (l / Q))) * W;
  if (c0 >= nd) return;
  if (a.status && a.status[(int64_t)s * a.status_stride] != kActive) return;
  const SysDev* sd = a.sys + s;
  const int tid = threadIdx.x;
  int64_t xo = (int64_t)s * a.D;
  if (a.x_from_aux && a.aux_m) {
    int slot = a.aux_m[(int64_t)s * a.status_stride] - *a.aux_base;
    slot = slot < 0 ? 0 : (slot >= a.aux_cap ? a.aux_cap - 1 : slot);
    xo = ((int64_t)s * a.aux_cap + slot) * a.D;
  }
  const cv<S>* xs = reinterpret_cast<const cv<S>*>(a.x_from_aux ? a.aux : a.x) + xo;
  cv<S>* vs = reinterpret_cast<cv<S>*>(a.v) + (int64_t)s * a.D;
  // whole 16-byte units: a full panel, rows of whole units, aligned vectors
  const bool fast = c0 + W <= nd && ((int64_t)nd * ES) % 16 == 0 &&
                    ((reinterpret_cast<uintptr_t>(xs) | reinterpret_cast<uintptr_t>(vs)) & 15) == 0;
  if (fast) {
    const int n_units = nu * CPR;
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave), lane = tid % kWave;
    for (int i0 = wave * kWave; i0 < n_units; i0 += BLK) {
      // lanes past the panel reload its last unit into the space of the zero
      // row (written below) or the whole-wavefront tail of the allocation
      const int i = min(i0 + lane, n_units - 1);
      const V16* src = reinterpret_cast<const V16*>(xs + (int64_t)(i / CPR) * nd + c0) + i % CPR;
      __builtin_amdgcn_global_load_lds(static_cast<const void*>(src),
                                       (__attribute__((address_space(3))) void*)(smem_raw + (size_t)i0 * 16),
                                       16, 0, 0);
    }
    __builtin_amdgcn_s_waitcnt(0);
  } else {
    for (int i = tid; i < nu * W; i += BLK) {
      const int d = c0 + i % W;
      pan[i] = d < nd ? xs[(int64_t)(i / W) * nd + d] : cv<S>{(S)0, (S)0};
    }
  }
  __syncthreads();
  if (tid < W) pan[nu * W + tid] = cv<S>{(S)0, (S)0};
  __syncthreads();

  const S U = (S)sd->U, Uc = (S)sd->Uc, dre = (S)sd->d_re, dim = (S)sd->d_im;
  const int core = sd->core;
  uint32_t cdw[W];
#pragma unroll
  for (int w = 0; w < W; ++w) cdw[w] = a.T.conf_dn[min(c0 + w, nd - 1)];
  cv<S> bs = {(S)0, (S)0};
  if (a.x_from_aux && a.beta) bs = {(S)a.beta[(int64_t)s * a.beta_stride], (S)a.beta[(int64_t)s * a.beta_stride + 1]};
  const bool badd = bs.re != (S)0 || bs.im != (S)0;
  // one panel row: the diagonal, the up-spin hops (four 16-bit entries per
  // table word; the four hops' panel rows are requested before their FMAs),
  // the store
  auto diag = [&](int u, cv<S> (&acc)[W]) {
    const uint32_t cu = a.T.conf_up[u < nu ? u : nu - 1];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      S dg = U * (S)__builtin_popcount(cu & cdw[w]) + dre;
      if (core >= 0) dg += Uc * (S)(((cu >> core) & 1u) + ((cdw[w] >> core) & 1u));
      const cv<S> xv = pan[(u < nu ? u : nu) * W + w];
      acc[w] = {dg * xv.re - dim * xv.im, dg * xv.im + dim * xv.re};
    }
  };
  auto hops = [&](cv<S> (&acc)[W], uint64_t hw, auto amp_of, uint32_t tmask) {
    cv<S> xv[4][W];
    S c[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t ent = (uint32_t)(hw >> (16 * j)) & 0xFFFFu;
      c[j] = flip_sign(amp_of(ent), (ent & 0x8000u) << 16);
      const cv<S>* src = pan + (ent & tmask) * W;
#pragma unroll
      for (int w = 0; w < W; ++w) xv[j][w] = src[w];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int w = 0; w < W; ++w) {
        acc[w].re += c[j] * xv[j][w].re;
        acc[w].im += c[j] * xv[j][w].im;
      }
  };
  auto store = [&](int u, cv<S> (&acc)[W]) {
    cv<S>* out = vs + (int64_t)u * nd + c0;
    if (badd) {
#pragma unroll
      for (int w = 0; w < W; ++w)
        if (fast || c0 + w < nd) {
          const cv<S> vo = out[w];
          acc[w].re += bs.re * vo.re - bs.im * vo.im;
          acc[w].im += bs.re * vo.im + bs.im * vo.re;
        }
    }
    if (fast) {
      V16* o16 = reinterpret_cast<V16*>(out);
#pragma unroll
      for (int j = 0; j < CPR; ++j) {
        if constexpr (std::is_same<S, double>::value) {
          o16[j] = make_double2(acc[j].re, acc[j].im);
        } else {
          o16[j] = make_float4(acc[2 * j].re, acc[2 * j].im, acc[2 * j + 1].re, acc[2 * j + 1].im);
        }
      }
    } else {
#pragma unroll
      for (int w = 0; w < W; ++w)
        if (c0 + w < nd) out[w] = acc[w];
    }
  };
  if (a.T.pan_ell) {
    // rows in hop-count order: each wavefront's words are padded only to its
    // own longest row; the entry carries the bond type (at most two types)
    const S am0 = (S)sd->amp[0], am1 = a.T.n_types > 1 ? (S)sd->amp[1] : (S)0;
    auto amp_of = [&](uint32_t ent) { return (ent & 0x4000u) ? am1 : am0; };
    const int npos = (nu + kWave - 1) / kWave * kWave;
    for (int p = tid; p < npos; p += BLK) {
      const int wv = p / kWave, lane = p % kWave;
      const int u = (int)a.T.pan_perm[p];                 // nu past the last row
      const int q0 = a.T.pan_woff[wv], nq = a.T.pan_woff[wv + 1] - q0;
      const uint64_t* ell = a.T.pan_ell + (int64_t)q0 * kWave + lane;
      cv<S> acc[W];
      diag(u, acc);
      uint64_t hn = nq > 0 ? ell[0] : 0;
      for (int q = 0; q < nq; ++q) {
        const uint64_t hw = hn;
        if (q + 1 < nq) hn = ell[(int64_t)(q + 1) * kWave];
        hops(acc, hw, amp_of, 0x3FFFu);
      }
      if (u < nu) store(u, acc);
    }
  } else {
    // one padded, transposed table per bond type, the amplitude uniform per type
    for (int u = tid; u < nu; u += BLK) {
      cv<S> acc[W];
      diag(u, acc);
      const uint64_t* ell = a.T.ell_up;
      for (int t = 0; t < a.T.n_types; ++t) {
        const int kq = a.T.k_type_up[t];
        const S am = (S)sd->amp[t];
        auto amp_of = [&](uint32_t) { return am; };
        uint64_t hn = kq > 0 ? ell[u] : 0;
        for (int q = 0; q < kq; ++q) {
          const uint64_t hw = hn;
          if (q + 1 < kq) hn = ell[(int64_t)(q + 1) * nu + u];
          hops(acc, hw, amp_of, 0x7FFFu);
        }
        ell += (int64_t)kq * nu;
      }
      store(u, acc);
    }
  }
}

// Panel widths compiled for the LDS-staged first pass, by storage type.
static bool pan_compiled(size_t es, int W) {
  if (es == 16) return W == 1 || W == 2 || W == 4 || W == 8;
  if (es == 8) return W == 2 || W == 4 || W == 8 || W == 16;
  return false;
}
// Widest compiled panel whose staged rows fit the LDS (0: none).
int pan_width_max(int n_up, size_t es, size_t lds_max) {
  int best = 0;
  for (int W = 1; W <= 16; W *= 2)
    if (pan_compiled(es, W) && pan_lds_bytes(n_up, W, es) <= lds_max) best = W;
  return best;
}

template <typename S>
static hipError_t launch_pan(const ApplyArgs& a, int W, hipStream_t st) {
  const int nu = a.T.n_up, nd = a.T.n_dn;
  const size_t es = sizeof(cv<S>);
  if (!a.T.ell_up || nu >= 32768 || !pan_compiled(es, W) || pan_lds_bytes(nu, W, es) > a.lds_max)
    return hipErrorInvalidValue;
  const int Q = (W * (int)es >= 128) ? 1 : 128 / (W * (int)es);
  const int n_panels = (nd + W - 1) / W;
  const int per = kNumXcd * Q;
  const dim3 grid((unsigned)(per * ((n_panels + per - 1) / per)), (unsigned)a.nsys);
  const size_t lds = pan_lds_bytes(nu, W, es);
  const int blk = pan_block(nu, W, es);
#define MSB_PAN_CASE(WW)                                                                        \
  if (W == WW) {                                                                               \
    if constexpr ((WW) * sizeof(cv<S>) % 16 == 0) {                                            \
      if (blk == 1024) hipLaunchKernelGGL((k_apply_pan<S, WW, 1024>), grid, dim3(1024), lds, st, a); \
      else hipLaunchKernelGGL((k_apply_pan<S, WW, 256>), grid, dim3(256), lds, st, a);          \
      return hipGetLastError();                                                                \
    }                                                                                          \
  }
  MSB_PAN_CASE(1) MSB_PAN_CASE(2) MSB_PAN_CASE(4) MSB_PAN_CASE(8)
  if constexpr (sizeof(S) == 4) { MSB_PAN_CASE(16) }
#undef MSB_PAN_CASE
  return hipErrorInvalidValue;
}

int apply_rows_per_xcd(int n_up) { return (n_up + kNumXcd - 1) / kNumXcd; }
int apply_nbx(int n_up, int nsys) {
  (void)nsys;
  return apply_rows_per_xcd(n_up) * kNumXcd;   // one row per workgroup
}

// Compiled launch shapes (threads per workgroup, elements per thread,
// vectors per workgroup).  A row of n_dn elements needs BLK * EPT >= n_dn.
// Large workgroups put more waves on one staged row: with a 55 KB row only
// two workgroups fit a CU's LDS, and 1024 threads each give 32 waves per CU
// instead of 8, which is what hides the latency of the neighbour-row loads.
#define MSB_APPLY_SHAPES(X)                                              \
  X(256, 1, 4) X(256, 1, 2) X(256, 1, 1)                                 \
  X(256, 2, 4) X(256, 2, 2) X(256, 2, 1)                                 \
  X(256, 4, 4) X(256, 4, 2) X(256, 4, 1)                                 \
  X(256, 8, 4) X(256, 8, 2) X(256, 8, 1)                                 \
  X(256, 16, 1) X(256, 24, 1)                                            \
  X(1024, 1, 2) X(1024, 1, 1)                                            \
  X(1024, 4, 4) X(1024, 4, 2) X(1024, 4, 1)                              \
  X(1024, 5, 4) X(1024, 5, 2) X(1024, 5, 1) X(1024, 8, 1) X(1024, 16, 1)

static const ApplyShape kShapes[] = {
#define MSB_SHAPE_ENTRY(B, E, N) {B, E, N, 1, 0},
    MSB_APPLY_SHAPES(MSB_SHAPE_ENTRY)
#undef MSB_SHAPE_ENTRY
};
static constexpr int kNumShapes = (int)(sizeof(kShapes) / sizeof(kShapes[0]));

static bool compiled(const ApplyShape& sh) {
  for (int i = 0; i < kNumShapes; ++i)
    if (kShapes[i].blk == sh.blk && kShapes[i].ept == sh.ept && kShapes[i].nv == sh.nv) return true;
  return false;
}

// Shape usable for rows of nd elements of `row_bytes` bytes each: the row
// fits, the staged rows fit the workgroup's LDS limit, and EPT is the
// smallest compiled one for this (BLK, NV) (larger ones only add idle lanes).
// A panel first pass (passes = 3) also needs its panel of pw columns of
// pan_nu rows (elements of pan_es bytes) to fit; pan_nu = 0: not available.
static bool usable(const ApplyShape& sh, int nd, size_t row_bytes, int nsys, size_t lds_max, int pan_nu,
                   size_t pan_es) {
  if (!compiled(sh) || sh.passes < 1 || sh.passes > 3 || (sh.order != 0 && sh.order != 1)) return false;
  if (sh.passes == 3 && (pan_nu <= 0 || pan_nu >= 32768 || !pan_compiled(pan_es, sh.pw) ||
                         pan_lds_bytes(pan_nu, sh.pw, pan_es) > lds_max))
    return false;
  if ((int64_t)sh.blk * sh.ept < nd) return false;
  if ((size_t)sh.nv * (nd + 1) * row_bytes > lds_max) return false;
  if (sh.nv > 1 && sh.nv > nsys) return false;
  for (int i = 0; i < kNumShapes; ++i) {
    const ApplyShape& o = kShapes[i];
    if (o.blk == sh.blk && o.nv == sh.nv && o.ept < sh.ept && (int64_t)o.blk * o.ept >= nd) return false;
  }
  if (sh.blk > 256 && 2 * nd < sh.blk * sh.ept) return false;   // mostly idle lanes
  return true;
}

int apply_candidates(int nd, size_t row_bytes, int nsys, size_t lds_max, int k_up_max, int pan_nu,
                     size_t pan_es, ApplyShape* out, int max_out) {
  int n = 0;
  for (int order = 0; order <= 1; ++order)
    for (int passes = 1; passes <= (panel_fits(k_up_max) ? 2 : 1); ++passes)
      for (int i = 0; i < kNumShapes && n < max_out; ++i) {
        ApplyShape sh = kShapes[i];
        sh.passes = passes;
        sh.order = order;
        if (usable(sh, nd, row_bytes, nsys, lds_max, 0, 0)) out[n++] = sh;
      }
  // LDS panel first pass: the widest panel and the half-width one (two
  // workgroups per CU); the row kernel after it gathers nothing from other
  // rows, so the row order does not matter
  const int wmax = pan_nu > 0 ? pan_width_max(pan_nu, pan_es, lds_max) : 0;
  for (int W : {wmax, wmax / 2}) {
    if (W <= 0 || (W == wmax / 2 && W == wmax)) continue;
    for (int i = 0; i < kNumShapes && n < max_out; ++i) {
      ApplyShape sh = kShapes[i];
      sh.passes = 3;
      sh.order = 0;
      sh.pw = W;
      if (usable(sh, nd, row_bytes, nsys, lds_max, pan_nu, pan_es)) out[n++] = sh;
    }
  }
  return n;
}

// Default shape when nothing was tuned: 256 threads (1024 if no 256-thread
// shape covers the row), as many vectors per workgroup as keep the staged
// rows within 40 KB (at most 4).  ept == 0: no shape fits.
static ApplyShape default_shape(int nd, size_t row_bytes, int nsys, size_t lds_max) {
  for (int blk : {256, 1024}) {
    ApplyShape sh{blk, 0, 1, 1, 0};
    for (int i = 0; i < kNumShapes; ++i) {
      const ApplyShape& o = kShapes[i];
      if (o.blk == blk && o.nv == 1 && (int64_t)o.blk * o.ept >= nd && (sh.ept == 0 || o.ept < sh.ept)) sh.ept = o.ept;
    }
    if (sh.ept == 0 || (size_t)(nd + 1) * row_bytes > lds_max) continue;
    for (int nv = 4; nv > 1; nv /= 2) {
      ApplyShape c{blk, sh.ept, nv, 1, 0};
      if (compiled(c) && nv <= nsys && (size_t)nv * (nd + 1) * row_bytes <= 40 * 1024) return c;
    }
    return sh;
  }
  return ApplyShape{256, 0, 1, 1, 0};
}

// The requested shape if usable for this kernel's row type, else the same
// shape with fewer vectors per workgroup, else the default.
// The residual mode writes no v, so it has no buffer for the first pass and
// runs the single-pass form of the requested shape.
static ApplyShape resolve_shape(const ApplyArgs& a, size_t row_bytes, bool allow_two, int pan_nu, size_t pan_es) {
  const int nd = a.T.n_dn;
  ApplyShape sh = a.shape;
  if (sh.blk > 0) {
    if (sh.passes == 2 && (!allow_two || !panel_fits(a.T.k_up_max))) sh.passes = 1;
    if (sh.passes == 3 && (!allow_two || pan_nu <= 0)) sh.passes = 1;
    for (; sh.nv >= 1; sh.nv /= 2)
      if (usable(sh, nd, row_bytes, a.nsys, a.lds_max, pan_nu, pan_es)) return sh;
  }
  return default_shape(nd, row_bytes, a.nsys, a.lds_max);
}

// rows of the LDS panel pass for storage S (0: not available)
template <typename S, bool CPLX>
static int pan_rows(const ApplyArgs& a) {
  return (CPLX && a.T.ell_up && a.T.n_up < 32768) ? a.T.n_up : 0;
}

template <typename S, typename Tc, bool CPLX, int MODE>
static hipError_t launch_mode(const ApplyArgs& a0, hipStream_t st) {
  ApplyArgs a = a0;
  const int nd = a.T.n_dn;
  // an operand read from the bank needs the slot of every active system
  a.x_from_aux = MODE == kModeSelf ? 1 : 0;
  if (MODE == kModeSelf && (!a.aux || !a.aux_m || !a.aux_base || !a.status)) return hipErrorInvalidValue;
  const ApplyShape sh = resolve_shape(a, sizeof(cv<Tc>), MODE != kModeResid, pan_rows<S, CPLX>(a), sizeof(cv<S>));
  if (sh.ept == 0 || (int64_t)sh.blk * sh.ept < nd || (size_t)sh.nv * (nd + 1) * sizeof(cv<Tc>) > a.lds_max)
    return hipErrorInvalidValue;
  a.nvec = sh.nv;
  a.vin = nullptr;
  a.ordered = sh.order;
  if (sh.passes == 2) {
    hipLaunchKernelGGL((k_apply_up<S, Tc, CPLX>), dim3(panel_nbx(a.T.n_up, nd), a.nsys), dim3(256), 0, st, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    a.vin = a.v;   // the row kernel adds the down-spin hops in place
  } else if (sh.passes == 3) {
    if constexpr (CPLX) {
      const hipError_t e = launch_pan<S>(a, sh.pw, st);
      if (e != hipSuccess) return e;
      a.vin = a.v;
    } else {
      return hipErrorInvalidValue;
    }
  }
  const int groups = (a.nsys + sh.nv - 1) / sh.nv;
  const dim3 grid = sh.order ? dim3(a.nbx * groups, 1) : dim3(a.nbx, groups);
  const size_t lds = (size_t)sh.nv * (nd + 1) * sizeof(cv<Tc>);
  hipError_t err = hipErrorInvalidValue;
#define MSB_SHAPE_CASE(B, E, N)                                                             \
  else if (sh.blk == B && sh.ept == E && sh.nv == N) {                                      \
    hipLaunchKernelGGL((k_apply<S, Tc, CPLX, E, MODE, N, B>), grid, dim3(B), lds, st, a);     \
    err = hipGetLastError();                                                                \
  }
  if (false) {}
  MSB_APPLY_SHAPES(MSB_SHAPE_CASE)
#undef MSB_SHAPE_CASE
  if (err != hipSuccess || MODE == kModePlain) return err;
  return launch_reduce(a.partials, a.nbx, a.nsys, a.red, st);
}

ApplyShape apply_shape_used(Elem e, int mode, const ApplyArgs& a) {
  // bytes of one staged element: complex64 residual mode accumulates in FP64
  size_t b = 16;
  if (e == Elem::R64) b = 8;
  else if (e == Elem::C64) b = (mode == kModeResid) ? 16 : 8;
  const size_t pes = e == Elem::C128 ? 16 : 8;
  const int pnu = (e != Elem::R64 && a.T.ell_up && a.T.n_up < 32768) ? a.T.n_up : 0;
  return resolve_shape(a, b, mode != kModeResid, pnu, pes);
}

hipError_t launch_apply(Elem e, int mode, const ApplyArgs& a, hipStream_t st) {
  switch (e) {
    case Elem::R64:
      if (mode == kModePlain) return launch_mode<double, double, false, kModePlain>(a, st);
      if (mode == kModeHerm) return launch_mode<double, double, false, kModeHerm>(a, st);
      break;
    case Elem::C128:
      if (mode == kModePlain) return launch_mode<double, double, true, kModePlain>(a, st);
      if (mode == kModeBilinear) return launch_mode<double, double, true, kModeBilinear>(a, st);
      if (mode == kModeSelf) return launch_mode<double, double, true, kModeSelf>(a, st);
      if (mode == kModeHerm) return launch_mode<double, double, true, kModeHerm>(a, st);
      if (mode == kModeResid) return launch_mode<double, double, true, kModeResid>(a, st);
      break;
    case Elem::C64:
      if (mode == kModePlain) return launch_mode<float, float, true, kModePlain>(a, st);
      if (mode == kModeBilinear) return launch_mode<float, float, true, kModeBilinear>(a, st);
      if (mode == kModeSelf) return launch_mode<float, float, true, kModeSelf>(a, st);
      if (mode == kModeResid) return launch_mode<float, double, true, kModeResid>(a, st);
      break;
  }
  return hipErrorInvalidValue;
}


// ---- interleaved block apply (the batched form's SpMM) ----------------------
// G systems stored interleaved, x[g][D][G] (the element (row u, column d) of
// system g*G + s at ((g * D + u * n_dn + d) * G + s)), so one neighbour-row
// gather brings the same element of all G right-hand sides in one contiguous
// load and one hop-table word serves them all.  Two passes:
//  * k_apply_up_il: the diagonal and H_up (x) I on column panels of 64 / G
//    columns x G systems (one lane per (column, system), the panel of every
//    row stays in one XCD's L2 while the rows gather from it; work items as
//    in k_apply_up, with one signed amplitude per system);
//  * k_apply_dn_il: one workgroup per row stages the G interleaved rows in
//    LDS, adds I (x) H_dn to the first pass's output in place and fuses the
//    COCG partial sums sigma = r^T v, |v|^2 (r from the residual bank, one
//    vector per system).
template <typename S, typename Tc, int G>
__global__ __launch_bounds__(256) void k_apply_up_il(ApplyArgs a) {
  using Ax = Access<S, true>;
  constexpr int W = kWave / G;                           // columns of a panel
  __shared__ int s_off[kRowsPerWg + 1];
  __shared__ uint32_t s_tgt[kPanelItems];
  __shared__ Tc s_cf[kPanelItems][G];
  const int grp = blockIdx.y;
  const int nd = a.T.n_dn, nu = a.T.n_up;
  const int chunks = (nu + kRowsPerWg - 1) / kRowsPerWg;
  const int xq = blockIdx.x % kNumXcd, l = blockIdx.x / kNumXcd;
  const int panel = xq + kNumXcd * (l / chunks), chunk = l % chunks;
  if (panel * W >= nd) return;
  const int r0 = chunk * kRowsPerWg;
  const int nrows = min(kRowsPerWg, nu - r0);
  if (threadIdx.x == 0) {
    int o = 0;
    for (int r = 0; r < nrows; ++r) {
      s_off[r] = o;
      o += 1 + (int)(a.T.off_up[r0 + r + 1] - a.T.off_up[r0 + r]);
    }
    s_off[nrows] = o;                                   // <= kPanelItems (panel_fits on the host)
  }
  __syncthreads();
  const int n_items = s_off[nrows];
  for (int t = threadIdx.x; t < n_items; t += blockDim.x) {
    int r = 0;
    while (t >= s_off[r + 1]) ++r;
    const int u = r0 + r, k = t - s_off[r];
    if (k == 0) {
      s_tgt[t] = kDiagItem | (uint32_t)u;
#pragma unroll
      for (int g = 0; g < G; ++g) s_cf[t][g] = (Tc)0;
    } else {
      const uint32_t h = a.T.hop_up[a.T.off_up[u] + k - 1];
      s_tgt[t] = h >> 16;
      const uint32_t ty = (h >> 1) & (MSB_MAX_BOND_TYPES - 1), sb = (h & 1u) ? 0u : 0x80000000u;
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int s = min(grp * G + g, a.nsys - 1);
        s_cf[t][g] = flip_sign((Tc)a.sys[s].amp[ty], sb);
      }
    }
  }
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rows_per_wave = kRowsPerWg / 4;
  const int i0 = s_off[min(wave * rows_per_wave, nrows)];
  const int i1 = s_off[min((wave + 1) * rows_per_wave, nrows)];
  const int gs = lane % G, col = lane / G;
  const int s = grp * G + gs;
  const int d = panel * W + col;
  const bool ok = d < nd && s < a.nsys &&
                  (!a.status || a.status[(int64_t)min(s, a.nsys - 1) * a.status_stride] == kActive);
  const uint32_t dc = (uint32_t)(d < nd ? d : nd - 1);   // idle lanes read a valid column
  const uint32_t cd = a.T.conf_dn[dc];
  const SysDev* sd = a.sys + min(s, a.nsys - 1);
  const Tc U = (Tc)sd->U, Uc = (Tc)sd->Uc, dre = (Tc)sd->d_re, dim = (Tc)sd->d_im;
  const int core = sd->core;
  const void* xg = Ax::offset(a.x, (int64_t)grp * a.D * G);
  void* vg = Ax::offset(a.v, (int64_t)grp * a.D * G);
  auto idx = [&](int row) { return ((int64_t)row * nd + dc) * G + gs; };
  cv<Tc> buf[kPrefetch];
#pragma unroll
  for (int j = 0; j < kPrefetch; ++j)
    if (i0 + j < i1) buf[j] = Ax::template load<Tc>(xg, idx((int)(s_tgt[i0 + j] & ~kDiagItem)));
  int row = -1;
  cv<Tc> acc = {(Tc)0, (Tc)0};
  for (int i = i0; i < i1; i += kPrefetch) {
#pragma unroll
    for (int j = 0; j < kPrefetch; ++j) {
      const int it = i + j;
      if (it < i1) {                                    // uniform across the wavefront
        const uint32_t tg = s_tgt[it];
        const cv<Tc> xv = buf[j];
        if (it + kPrefetch < i1)
          buf[j] = Ax::template load<Tc>(xg, idx((int)(s_tgt[it + kPrefetch] & ~kDiagItem)));
        if (tg & kDiagItem) {
          if (row >= 0 && ok) Ax::store(vg, idx(row), acc);
          row = (int)(tg & ~kDiagItem);
          const uint32_t cu = a.T.conf_up[row];
          Tc dg = U * (Tc)__builtin_popcount(cu & cd) + dre;
          if (core >= 0) dg += Uc * (Tc)(((cu >> core) & 1u) + ((cd >> core) & 1u));
          acc = {dg * xv.re - dim * xv.im, dg * xv.im + dim * xv.re};
        } else {
          const Tc c = s_cf[it][gs];
          acc.re += c * xv.re;
          acc.im += c * xv.im;
        }
      }
    }
  }
  if (row >= 0 && ok) Ax::store(vg, idx(row), acc);
}

// G consecutive complex values (one element of the G systems of a group).
template <typename S, typename Tc, int G>
struct GroupIO {
  static __device__ __forceinline__ void load(const void* base, int64_t i, cv<Tc> (&out)[G]) {
    if constexpr (std::is_same<S, float>::value && G % 2 == 0) {
      const float4* p = reinterpret_cast<const float4*>(reinterpret_cast<const cv<float>*>(base) + i);
#pragma unroll
      for (int h = 0; h < G / 2; ++h) {
        const float4 t = p[h];
        out[2 * h] = {(Tc)t.x, (Tc)t.y};
        out[2 * h + 1] = {(Tc)t.z, (Tc)t.w};
      }
    } else {
#pragma unroll
      for (int g = 0; g < G; ++g) out[g] = Access<S, true>::template load<Tc>(base, i + g);
    }
  }
  static __device__ __forceinline__ void store(void* base, int64_t i, const cv<Tc> (&v)[G]) {
    if constexpr (std::is_same<S, float>::value && G % 2 == 0) {
      float4* p = reinterpret_cast<float4*>(reinterpret_cast<cv<float>*>(base) + i);
#pragma unroll
      for (int h = 0; h < G / 2; ++h)
        p[h] = make_float4((float)v[2 * h].re, (float)v[2 * h].im, (float)v[2 * h + 1].re, (float)v[2 * h + 1].im);
    } else {
#pragma unroll
      for (int g = 0; g < G; ++g) Access<S, true>::store(base, i + g, v[g]);
    }
  }
};

template <typename S, typename Tc, int G, int EPT, int BLK, int MODE>
__global__ __launch_bounds__(BLK) void k_apply_dn_il(ApplyArgs a) {
  using Ax = Access<S, true>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cv<Tc>* rows = reinterpret_cast<cv<Tc>*>(smem_raw);     // [nd + 1][G], element nd = 0
  const int tid = threadIdx.x;
  const int nd = a.T.n_dn;
  const int bx = blockIdx.x, grp = blockIdx.y;
  const int u = (bx % kNumXcd) * a.rows_per_xcd + bx / kNumXcd;
  const bool row_ok = u < a.T.n_up;
  bool act[G];
  int64_t aux_off[G];
  const int abase = a.aux_m ? *a.aux_base : 0;
  bool any = false;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int s = grp * G + g;
    const bool in = row_ok && s < a.nsys;
    act[g] = in && (!a.status || a.status[(int64_t)s * a.status_stride] == (int)kActive);
    any |= act[g];
    aux_off[g] = 0;
    if (in && a.aux_m) {
      int slot = a.aux_m[(int64_t)s * a.status_stride] - abase;
      slot = slot < 0 ? 0 : (slot >= a.aux_cap ? a.aux_cap - 1 : slot);
      aux_off[g] = ((int64_t)s * a.aux_cap + slot) * a.D;
    } else if (in) {
      aux_off[g] = (int64_t)s * a.D;
    }
  }
  double part[G][3];
#pragma unroll
  for (int g = 0; g < G; ++g) part[g][0] = part[g][1] = part[g][2] = 0.0;
  if (any) {
    const int64_t row0 = (int64_t)u * nd;
    const void* xg = Ax::offset(a.x, (int64_t)grp * a.D * G);
    void* vg = Ax::offset(a.v, (int64_t)grp * a.D * G);
    uint32_t voff[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int d = tid + e * BLK;
      voff[e] = (uint32_t)(d < nd ? d : nd - 1);
    }
    cv<Tc> acc[EPT][G];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int d = tid + e * BLK;
      cv<Tc> xs[G];
      GroupIO<S, Tc, G>::load(xg, (row0 + voff[e]) * G, xs);
      GroupIO<S, Tc, G>::load(vg, (row0 + voff[e]) * G, acc[e]);   // diagonal and up-spin hops
      if (d < nd) {
#pragma unroll
        for (int g = 0; g < G; ++g) rows[d * G + g] = xs[g];
      }
    }
    if (tid < G) rows[nd * G + tid] = cv<Tc>{(Tc)0, (Tc)0};
    __syncthreads();
    const uint64_t* ell = a.T.ell_dn;
    for (int t = 0; t < a.T.n_types; ++t) {
      const int kq = a.T.k_type[t];
      Tc amp[G];
#pragma unroll
      for (int g = 0; g < G; ++g) amp[g] = act[g] ? (Tc)a.sys[grp * G + g].amp[t] : (Tc)0;
      uint64_t hn[EPT];
      if (kq > 0) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) hn[e] = ell[voff[e]];
      }
      for (int q = 0; q < kq; ++q) {
        uint32_t hw[EPT][2];
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          hw[e][0] = (uint32_t)hn[e];
          hw[e][1] = (uint32_t)(hn[e] >> 32);
        }
        if (q + 1 < kq) {
          const uint64_t* nxt = ell + (int64_t)(q + 1) * nd;
#pragma unroll
          for (int e = 0; e < EPT; ++e) hn[e] = nxt[voff[e]];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int e = 0; e < EPT; ++e) {
            const uint32_t ent = (hw[e][j >> 1] >> (16 * (j & 1))) & 0xFFFFu;
            const uint32_t sb = (ent & 0x8000u) << 16;
            const int tgt = (int)(ent & 0x7FFFu);
#pragma unroll
            for (int g = 0; g < G; ++g) {
              const Tc c = flip_sign(amp[g], sb);
              const cv<Tc> xv = rows[tgt * G + g];
              acc[e][g].re += c * xv.re;
              acc[e][g].im += c * xv.im;
            }
          }
      }
      ell += (int64_t)kq * nd;
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int d = tid + e * BLK;
      if (d >= nd) continue;
      cv<Tc> vs[G];
#pragma unroll
      for (int g = 0; g < G; ++g) vs[g] = act[g] ? acc[e][g] : cv<Tc>{(Tc)0, (Tc)0};
      GroupIO<S, Tc, G>::store(vg, (row0 + d) * G, vs);
      if constexpr (MODE == kModeBilinear) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
          if (!act[g]) continue;
          const cv<double> r = Ax::template load_nt<double>(a.aux, aux_off[g] + row0 + d);
          const cv<double> w = {(double)(S)vs[g].re, (double)(S)vs[g].im};   // value as stored
          part[g][0] += r.re * w.re - r.im * w.im;
          part[g][1] += r.re * w.im + r.im * w.re;
          part[g][2] += w.re * w.re + w.im * w.im;
        }
      }
    }
  }
  if constexpr (MODE != kModePlain) {
    __shared__ double sh[3 * G][BLK / kWave];
    double flat[3 * G];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int i = 0; i < 3; ++i) flat[3 * g + i] = part[g][i];
    block_sum<3 * G, BLK>(flat, sh);
    if (tid == 0) {
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int s = grp * G + g;
        if (s >= a.nsys) continue;
#pragma unroll
        for (int i = 0; i < 3; ++i) a.partials[((int64_t)s * a.nbx + bx) * 4 + i] = flat[3 * g + i];
      }
    }
  }
}

// LDS the row pass takes besides the staged rows (its reduction buffer)
constexpr size_t kIlStaticLds = 4096;

int apply_il_width(int nd, size_t elem_bytes, int nsys, size_t lds_max, int k_up_max) {
  if (!panel_fits(k_up_max)) return 0;
  for (int g : {4, 2})
    if (nsys >= g && (size_t)g * (nd + 1) * elem_bytes + kIlStaticLds <= lds_max && nd <= 1024 * 10) return g;
  return 0;
}

template <typename S, typename Tc, int G, int MODE>
static hipError_t launch_il_mode(const ApplyArgs& a, hipStream_t st) {
  const int nd = a.T.n_dn;
  if ((size_t)G * (nd + 1) * sizeof(cv<Tc>) + kIlStaticLds > a.lds_max) return hipErrorInvalidValue;
  const int groups = (a.nsys + G - 1) / G;
  const int W = kWave / G;
  const int n_panels = (nd + W - 1) / W;
  const int chunks = (a.T.n_up + kRowsPerWg - 1) / kRowsPerWg;
  const int pnbx = kNumXcd * ((n_panels + kNumXcd - 1) / kNumXcd) * chunks;
  hipLaunchKernelGGL((k_apply_up_il<S, Tc, G>), dim3(pnbx, groups), dim3(256), 0, st, a);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  const dim3 grid(a.nbx, groups);
  const size_t lds = (size_t)G * (nd + 1) * sizeof(cv<Tc>);
  err = hipErrorInvalidValue;
  // rows that fit the LDS: at most 5 elements per thread of a 1024-thread
  // workgroup (10 for pairs of complex64 systems, 3 for quadruples of complex128)
  constexpr int kMaxE = (sizeof(S) == 4 && G == 2) ? 10 : (sizeof(S) == 8 && G == 4) ? 3 : 5;
#define MSB_IL_CASE(B, E)                                                                  \
  else if (((B) == 256) == (nd <= 1024) && (int64_t)(B) * (E) >= nd &&                      \
           (int64_t)(B) * ((E) - 1) < nd) {                                                 \
    if constexpr ((E) <= kMaxE) {                                                           \
      hipLaunchKernelGGL((k_apply_dn_il<S, Tc, G, E, B, MODE>), grid, dim3(B), lds, st, a); \
      err = hipGetLastError();                                                              \
    }                                                                                       \
  }
  if (false) {}
  MSB_IL_CASE(256, 1) MSB_IL_CASE(256, 2) MSB_IL_CASE(256, 3) MSB_IL_CASE(256, 4)
  MSB_IL_CASE(1024, 2) MSB_IL_CASE(1024, 3) MSB_IL_CASE(1024, 4) MSB_IL_CASE(1024, 5)
  MSB_IL_CASE(1024, 6) MSB_IL_CASE(1024, 7) MSB_IL_CASE(1024, 8) MSB_IL_CASE(1024, 9) MSB_IL_CASE(1024, 10)
#undef MSB_IL_CASE
  if (err != hipSuccess || MODE == kModePlain) return err;
  return launch_reduce(a.partials, a.nbx, a.nsys, a.red, st);
}

hipError_t launch_apply_il(Elem e, int mode, int G, const ApplyArgs& a, hipStream_t st) {
  if (a.aux_m && !a.aux) return hipErrorInvalidValue;
#define MSB_IL_DISPATCH(S, TC)                                                          \
  if (G == 4 && mode == kModePlain) return launch_il_mode<S, TC, 4, kModePlain>(a, st);       \
  if (G == 4 && mode == kModeBilinear) return launch_il_mode<S, TC, 4, kModeBilinear>(a, st); \
  if (G == 2 && mode == kModePlain) return launch_il_mode<S, TC, 2, kModePlain>(a, st);       \
  if (G == 2 && mode == kModeBilinear) return launch_il_mode<S, TC, 2, kModeBilinear>(a, st);
  if (e == Elem::C128) { MSB_IL_DISPATCH(double, double) }
  if (e == Elem::C64) { MSB_IL_DISPATCH(float, float) }
#undef MSB_IL_DISPATCH
  return hipErrorInvalidValue;
}
}  // namespace msb
