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
  // coefficient tables are slot-major, [s][l][j] complex: for one slot the
  // shifts of a tile are adjacent (one scalar load serves a wavefront's shifts)
  // entries of ncomp doubles: (c_re, c_im), or for the three-product assembly
  // (c_re, c_re + c_im, c_im - c_re)
  const int nc = a.ncomp;
  const int64_t cstride = (int64_t)a.n_list * nc;
  double* crow = a.coef + ((int64_t)s * a.K * a.n_list + j) * nc;
  double* grow = a.gcoef ? a.gcoef + ((int64_t)s * a.K * a.n_list + j) * nc : nullptr;
  double* zrow = scratch + (int64_t)tid * a.K * 4;    // (zeta_l, bw_l)
  const int k = a.list[tid];
  const int lend = (k >= 0) ? a.lend[tid] : 0;
  for (int l = lend; l < a.K; ++l)
    for (int c = 0; c < nc; ++c) {
      crow[cstride * l + c] = 0.0;
      if (grow) grow[cstride * l + c] = 0.0;
    }
  auto put = [nc](double* e, cv<double> v) {
    e[0] = v.re;
    e[1] = nc == 3 ? v.re + v.im : v.im;
    if (nc == 3) e[2] = v.im - v.re;
  };
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
      crow[cstride * l] = aw.re;
      crow[cstride * l + 1] = aw.im;
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
    const cv<double> aw = {crow[cstride * l], crow[cstride * l + 1]};
    if (l < lend - 1) {
      const cv<double> bnext = {zrow[4 * (l + 1) + 2], zrow[4 * (l + 1) + 3]};
      S = cadd(aw, cmul(bnext, S));
      if (carry) G = cmul(bnext, G);
    } else {
      S = aw;
    }
    const cv<double> zl = {zrow[4 * l], zrow[4 * l + 1]};
    put(crow + cstride * l, cdiv(S, zl));
    if (grow) put(grow + cstride * l, carry ? cdiv(G, zl) : cv<double>{0.0, 0.0});
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
// The sum is a dense complex contraction (shifts x slots) . (slots x elements),
// evaluated with FP64 matrix-core instructions: v_mfma_f64_16x16x4f64 computes
// D(16x16) += A(16x4) B(4x16) with A[i][k] in lane i+16k, B[k][j] in lane j+16k
// and D[i][j] in lane j+16(i%4), register i/4.  A complex product takes four
// real products (re*re - im*im, re*im + im*re).  A wavefront owns 16 shifts x
// 64 elements (four 16x16 tiles); the four wavefronts of a workgroup take 64
// consecutive shift slots over the same 64 elements, so residual loads are
// shared through L1.  Workgroups of one element tile are issued back to back on
// one XCD so the residual tile is read from HBM once and from L2 afterwards.
constexpr int kFlushM = 16;       // shifts per wavefront (MFMA rows)
constexpr int kFlushNT = 4;       // 16-element MFMA tiles per wavefront
constexpr int kFlushWaves = kBlock / kWave;
// Three-product (default) engine variants: shift slots per wavefront,
// elements per lane and wavefronts per workgroup.  Every VALU engine covers
// 32 shift slots per workgroup.
struct GaussShape {
  int M, EPL, NW;
};
__host__ __device__ constexpr GaussShape gauss_shape(int engine) {
  return engine == 3 ? GaussShape{8, 2, 8} : engine == 4 ? GaussShape{4, 4, 8} : GaussShape{8, 2, 4};
}
int flush_shifts_per_tile(int engine) {
  if (engine == 5) return 256;     // k_flush_oz.hip: shift slots per workgroup
  if (engine == 6) return 16;      // k_flush_mf64.hip: one wavefront per 16-shift tile
  if (engine == 1) return kFlushM * kFlushWaves;
  if (engine == 2) return 8 * kFlushWaves;
  const GaussShape g = gauss_shape(engine);
  return g.M * g.NW;
}
int flush_elems_per_tile(int engine) {
  if (engine == 5) return 32;      // k_flush_oz.hip: elements per workgroup
  if (engine == 6) return 32;      // k_flush_mf64.hip
  if (engine == 1) return 16 * kFlushNT;
  if (engine == 2) return kWave * 4;
  return kWave * gauss_shape(engine).EPL;
}
int flush_coef_comps(int engine) { return (engine == 1 || engine == 2) ? 2 : 3; }

typedef double v4d __attribute__((ext_vector_type(4)));

template <typename SB, typename SO>
__global__ __launch_bounds__(kBlock) void k_flush_mfma(FlushArgs a, int ow_mode) {
  using AB = Access<SB, true>;
  using AO = Access<SO, true>;
  constexpr int TILE = 16 * kFlushNT;

  const int s = blockIdx.y;
  const int b = blockIdx.x;
  const int xcd = b % kNumXcd, q = b / kNumXcd;
  const int et = xcd + kNumXcd * (q / a.n_stiles);
  const int stt = q % a.n_stiles;
  if (et >= a.n_etiles) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int li = lane % 16, lk = lane / 16;
  const int slot0 = stt * (kFlushM * kFlushWaves) + wave * kFlushM;
  const int Kext = a.tile_k[s * a.n_stiles + stt];
  const int64_t e0 = (int64_t)et * TILE;
  const void* bank_s = AB::offset(a.bank, (int64_t)s * a.cap * a.D);
  // this lane's A-operand row: shift slot0 + li
  const double* crow = a.coef + ((int64_t)s * a.K * a.n_list + slot0 + li) * 2;   // slot-major
  const int64_t cstride = (int64_t)a.n_list * 2;

  v4d accr[kFlushNT], acci[kFlushNT];
#pragma unroll
  for (int t = 0; t < kFlushNT; ++t) {
    accr[t] = v4d{0.0, 0.0, 0.0, 0.0};
    acci[t] = v4d{0.0, 0.0, 0.0, 0.0};
  }
  // operands of one K-step (4 residual slots); the next step's operands are
  // loaded while the matrix instructions of the current step run
  struct Ops {
    double ar, ai;
    cv<double> rv[kFlushNT];
  };
  // Branch-free loads (so the compiler can keep the prefetch in flight): slot
  // and element indices are clamped into written memory; a clamped slot gets a
  // zero coefficient, a clamped element only feeds an output that is not stored.
  const int64_t last_e = a.D - 1;
  auto load_ops = [&](int kb, Ops& o) {
    const int kk = kb + lk;
    const bool kin = kk < Kext;
    const int kc = kin ? kk : Kext - 1;
    const double cr = crow[cstride * kc], ci = crow[cstride * kc + 1];
    o.ar = kin ? cr : 0.0;
    o.ai = kin ? ci : 0.0;
    const void* rs = AB::offset(bank_s, (int64_t)kc * a.D);
#pragma unroll
    for (int t = 0; t < kFlushNT; ++t) {
      int64_t e = e0 + t * 16 + li;
      e = e < last_e ? e : last_e;
      o.rv[t] = AB::template load<double>(rs, e);
    }
  };
  Ops cur, nxt;
  // an empty tile (every listed shift froze before this block) has Kext = 0:
  // nothing is loaded and the zero sums are stored (or added to the old output)
  if (Kext > 0) load_ops(0, cur);
  for (int kb = 0; kb < Kext; kb += 4) {
    if (kb + 4 < Kext) load_ops(kb + 4, nxt);
#pragma unroll
    for (int t = 0; t < kFlushNT; ++t) {
      accr[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(cur.ar, cur.rv[t].re, accr[t], 0, 0, 0);
      accr[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(-cur.ai, cur.rv[t].im, accr[t], 0, 0, 0);
      acci[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(cur.ar, cur.rv[t].im, acci[t], 0, 0, 0);
      acci[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(cur.ai, cur.rv[t].re, acci[t], 0, 0, 0);
    }
    cur = nxt;
  }

#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int slot = slot0 + 4 * r + lk;            // D row i = 4r + lane/16
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
    for (int t = 0; t < kFlushNT; ++t) {
      const int64_t i = e0 + t * 16 + li;           // D column j = lane%16
      if (i >= a.D) continue;
      cv<double> v = {accr[t][r], acci[t][r]};
      if (ow_mode != 0) v = cadd(v, cmul(ow, AO::template load<double>(a.out, obase + i)));
      if (a.X) v = cadd(v, cmul(pw, AO::template load<double>(a.X, obase + i)));
      AO::store(a.out, obase + i, v);
    }
  }
}


// VALU form of the same contraction (the default: on MI355X FP64 FMA issues
// faster from the vector ALUs than from the FP64 matrix instructions).  A
// workgroup owns 32 shift slots (8 per wavefront) x 256 elements (4 per lane).
// Residual slots are staged in LDS in chunks of 6; with a complex128 bank the
// chunks go straight from memory to LDS and the next one is in flight while
// the FMAs of the current one run (two 24 KB buffers: three workgroups still
// fit a CU's LDS, as many as the registers allow).  The coefficients are
// wave-uniform and come through the scalar cache, so they cost neither LDS
// nor vector-memory bandwidth; the next slot's coefficients are requested
// before the current slot's FMAs so the scalar-cache misses overlap with them.
constexpr int kValuM = 8;         // shift slots per wavefront
constexpr int kValuEPL = 4;       // elements per lane
constexpr int kValuKT = 6;        // residual slots per staged chunk

template <typename SB, typename SO>
__global__ __launch_bounds__(kBlock) void k_flush_valu(FlushArgs a, const double* __restrict__ coef,
                                                       int ow_mode) {
  using AB = Access<SB, true>;
  using AO = Access<SO, true>;
  constexpr int EPL = kValuEPL, KT = kValuKT, M = kValuM;
  constexpr int TILE = kWave * EPL;                       // 256 elements
  constexpr int NS = M * kFlushWaves;                     // 32 shift slots
  constexpr int RPT = KT;                                 // residual slots staged per thread per chunk
  static_assert(TILE == kBlock, "one staged element per thread");
  __shared__ cv<double> rt[KT][TILE];
  // second chunk buffer of the complex128 form (an empty array otherwise)
  __shared__ cv<double> rt2[std::is_same<SB, double>::value ? KT : 1][TILE];

  const int s = blockIdx.y;
  const int b = blockIdx.x;
  const int xcd = b % kNumXcd, q = b / kNumXcd;
  const int et = xcd + kNumXcd * (q / a.n_stiles);
  const int stt = q % a.n_stiles;
  if (et >= a.n_etiles) return;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
  const int lane = tid % kWave;
  const int Kext = a.tile_k[s * a.n_stiles + stt];
  const int64_t e0 = (int64_t)et * TILE;
  const int64_t last_e = a.D - 1;
  const void* bank_s = AB::offset(a.bank, (int64_t)s * a.cap * a.D);
  const int slot0 = stt * NS + wave * M;
  // the list is sorted by descending range, so the wavefront's first slot has
  // its longest one: chunks beyond it are staged for the other wavefronts only
  const int Kw = a.lend ? __builtin_amdgcn_readfirstlane(a.lend[s * a.n_list + slot0]) : Kext;
  // uniform address in the constant address space: read through the scalar cache
  typedef __attribute__((address_space(4))) const double cdouble;
  cdouble* crow = (cdouble*)(coef + ((int64_t)s * a.K * a.n_list + slot0) * 2);   // slot-major

  cv<double> acc[M][EPL];
#pragma unroll
  for (int t = 0; t < M; ++t)
#pragma unroll
    for (int e = 0; e < EPL; ++e) acc[t][e] = {0.0, 0.0};

  // coefficients of slot l for this wavefront's M shifts (scalar registers);
  // the next slot's are requested before the current slot's FMAs are issued
  auto load_c = [&](int l, cv<double> (&c)[M]) {
#pragma unroll
    for (int t = 0; t < M; ++t) c[t] = {crow[((int64_t)l * a.n_list + t) * 2], crow[((int64_t)l * a.n_list + t) * 2 + 1]};
  };
  int64_t my_e = e0 + tid;
  my_e = my_e < last_e ? my_e : last_e;                   // clamped: feeds only unstored outputs
  // the FMAs of the slots [kb, kb + kn) staged in buf
  auto run = [&](const cv<double> (*buf)[TILE], int kb, int kn) {
    cv<double> c_cur[M], c_nxt[M];
    const int kw = min(kn, Kw - kb);                      // wave-uniform; may be <= 0
    if (kw > 0) load_c(kb, c_cur);
    for (int kk = 0; kk < kw; ++kk) {
      if (kk + 1 < kw) load_c(kb + kk + 1, c_nxt);
      cv<double> r[EPL];
#pragma unroll
      for (int e = 0; e < EPL; ++e) r[e] = buf[kk][lane + kWave * e];
#pragma unroll
      for (int t = 0; t < M; ++t) {
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
          acc[t][e].re = fma(c_cur[t].re, r[e].re, acc[t][e].re);
          acc[t][e].re = fma(-c_cur[t].im, r[e].im, acc[t][e].re);
          acc[t][e].im = fma(c_cur[t].re, r[e].im, acc[t][e].im);
          acc[t][e].im = fma(c_cur[t].im, r[e].re, acc[t][e].im);
        }
      }
#pragma unroll
      for (int t = 0; t < M; ++t) c_cur[t] = c_nxt[t];
    }
  };
  if constexpr (std::is_same<SB, double>::value) {
    // complex128 bank: each chunk goes straight from memory to LDS
    // (global_load_lds, 16 bytes per lane at the wavefront's LDS base), and
    // chunk kb + KT is in flight while the FMAs of chunk kb run
    const cv<double>* bank_c = reinterpret_cast<const cv<double>*>(bank_s);
    auto stage = [&](cv<double> (*buf)[TILE], int kb) {
      const int kn = min(KT, Kext - kb);
#pragma unroll
      for (int j = 0; j < KT; ++j) {
        const int kc = kb + (j < kn ? j : kn - 1);        // clamped: its coefficient is never used
        __builtin_amdgcn_global_load_lds(static_cast<const void*>(bank_c + (int64_t)kc * a.D + my_e),
                                         (__attribute__((address_space(3))) void*)&buf[j][wave * kWave],
                                         16, 0, 0);
      }
    };
    if (Kext > 0) stage(rt, 0);
    for (int kb = 0; kb < Kext; kb += 2 * KT) {
      __builtin_amdgcn_s_waitcnt(0);                      // this wavefront's part of chunk kb landed
      __syncthreads();                                    // every part; rt2 no longer read
      if (kb + KT < Kext) stage(rt2, kb + KT);
      run(rt, kb, min(KT, Kext - kb));
      if (kb + KT >= Kext) break;
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (kb + 2 * KT < Kext) stage(rt, kb + 2 * KT);
      run(rt2, kb + KT, min(KT, Kext - kb - KT));
    }
  } else {
    for (int kb = 0; kb < Kext; kb += KT) {
      const int kn = min(KT, Kext - kb);
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        const int kc = kb + (j < kn ? j : kn - 1);        // clamped: its coefficient is never used
        rt[j][tid] = AB::template load<double>(bank_s, (int64_t)kc * a.D + my_e);
      }
      __syncthreads();
      run(rt, kb, kn);
      __syncthreads();
    }
  }

#pragma unroll
  for (int t = 0; t < M; ++t) {
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

// Three-product form (the default engine).  With s = r_re + r_im per element
// (one add, shared by the wavefront's shifts) and the table entry
// (c_re, c_re + c_im, c_im - c_re) precomputed by k_coef,
//   c r = [c_re s - (c_re + c_im) r_im] + i [c_re s + (c_im - c_re) r_re],
// so each (shift, element, slot) costs three FMAs into three accumulators
// (A1 += c_re s, A2 += (c_re + c_im) r_im, A3 += (c_im - c_re) r_re;
// re = A1 - A2, im = A1 + A3) instead of the four of the plain complex
// product.  A workgroup owns M * NW shift slots and 64 * EPL elements.  The
// residual slots go straight from memory to LDS in their storage precision
// (global_load_lds, 16 bytes per lane: one complex128 or two complex64
// elements), in chunks of kValuKT slots, double-buffered so that the next
// chunk is in flight while the FMAs of the current one run; complex64 values
// are widened to FP64 as they are read from LDS.  Lane l owns the elements
// l + 64 e (complex128 bank) or 2 l + 128 (e / 2) + e % 2 (complex64 bank,
// one 16-byte LDS read per pair).  Table entries are wave-uniform scalar
// loads (the next slot's requested early when M <= 4).
template <typename SB>
__device__ __forceinline__ int gauss_elem(int lane, int e) {
  if constexpr (std::is_same<SB, double>::value) return lane + kWave * e;
  else return 2 * kWave * (e / 2) + 2 * lane + (e % 2);
}

template <typename SB, typename SO, int M, int EPL, int NW>
__global__ __launch_bounds__(NW * kWave) void k_flush_gauss(FlushArgs a, const double* __restrict__ coef,
                                                             int ow_mode) {
  using AO = Access<SO, true>;
  using VB = typename std::conditional<std::is_same<SB, double>::value, double2, float4>::type;
  constexpr int KT = kValuKT;
  constexpr int TILE = kWave * EPL;                       // elements of the workgroup
  constexpr int NS = M * NW;                              // shift slots of the workgroup
  constexpr int PER16 = 16 / (int)sizeof(cv<SB>);         // elements per 16-byte lane load
  constexpr int LROWS = EPL / PER16;                      // wave loads per slot
  constexpr int ROWS = KT * LROWS;                        // wave loads per chunk
  static_assert(EPL % PER16 == 0, "whole 16-byte loads per lane");
  // two chunk buffers, 16-byte units, as two objects: the compiler then
  // knows that the DMA into one does not write the other, and reads the
  // current chunk while the next one is in flight
  __shared__ VB rt0[KT][TILE / PER16];
  __shared__ VB rt1[KT][TILE / PER16];

  const int s = blockIdx.y;
  const int b = blockIdx.x;
  const int xcd = b % kNumXcd, q = b / kNumXcd;
  const int et = xcd + kNumXcd * (q / a.n_stiles);
  const int stt = q % a.n_stiles;
  if (et >= a.n_etiles) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int Kext = a.tile_k[s * a.n_stiles + stt];
  const int64_t e0 = (int64_t)et * TILE;
  const cv<SB>* bank_s = reinterpret_cast<const cv<SB>*>(a.bank) + (int64_t)s * a.cap * a.D;
  const int slot0 = stt * NS + wave * M;
  const int Kw = a.lend ? __builtin_amdgcn_readfirstlane(a.lend[s * a.n_list + slot0]) : Kext;
  typedef __attribute__((address_space(4))) const double cdouble;
  cdouble* crow = (cdouble*)(coef + ((int64_t)s * a.K * a.n_list + slot0) * 3);   // slot-major

  // 16-byte units a lane loads for one wave load: clamped into the vector
  // (the D % PER16 tail of a complex64 bank reads its last whole unit; such
  // elements feed only outputs that are not stored)
  const int64_t n_units = a.D / PER16;                    // whole 16-byte units of one slot
  double A1[M][EPL], A2[M][EPL], A3[M][EPL];
#pragma unroll
  for (int t = 0; t < M; ++t)
#pragma unroll
    for (int e = 0; e < EPL; ++e) A1[t][e] = A2[t][e] = A3[t][e] = 0.0;

  auto stage = [&](VB (&rt)[KT][TILE / PER16], int kb) {
    const int kn = min(KT, Kext - kb);
    for (int row = wave; row < ROWS; row += NW) {
      const int j = row / LROWS, g = row % LROWS;
      const int kc = kb + (j < kn ? j : kn - 1);          // clamped: its coefficient is never used
      int64_t unit = (e0 / PER16) + (int64_t)g * kWave + lane;
      unit = unit < n_units - 1 ? unit : n_units - 1;
      const VB* src = reinterpret_cast<const VB*>(bank_s + (int64_t)kc * a.D) + unit;
      __builtin_amdgcn_global_load_lds(static_cast<const void*>(src),
                                       (__attribute__((address_space(3))) void*)&rt[j][g * kWave],
                                       16, 0, 0);
    }
  };
  struct C3 {
    double r, sum, dif;
  };
  auto load_c = [&](int l, C3 (&c)[M]) {
#pragma unroll
    for (int t = 0; t < M; ++t) {
      const int64_t o = ((int64_t)l * a.n_list + t) * 3;
      c[t] = {crow[o], crow[o + 1], crow[o + 2]};
    }
  };
  constexpr bool kPrefetch = M <= 4;
  auto run = [&](const VB (&rt)[KT][TILE / PER16], int kb, int kn) {
    C3 c_cur[M], c_nxt[kPrefetch ? M : 1];
    const int kw = min(kn, Kw - kb);                      // wave-uniform; may be <= 0
    if (kPrefetch && kw > 0) load_c(kb, c_cur);
    for (int kk = 0; kk < kw; ++kk) {
      if constexpr (kPrefetch) {
        if (kk + 1 < kw) load_c(kb + kk + 1, c_nxt);
      } else {
        load_c(kb + kk, c_cur);
      }
      double rr[EPL], ri[EPL], sm[EPL];
      if constexpr (std::is_same<SB, double>::value) {
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
          const double2 r = rt[kk][lane + kWave * e];
          rr[e] = r.x;
          ri[e] = r.y;
        }
      } else {
#pragma unroll
        for (int g = 0; g < EPL / 2; ++g) {
          const float4 r = rt[kk][g * kWave + lane];
          rr[2 * g] = (double)r.x;
          ri[2 * g] = (double)r.y;
          rr[2 * g + 1] = (double)r.z;
          ri[2 * g + 1] = (double)r.w;
        }
      }
#pragma unroll
      for (int e = 0; e < EPL; ++e) sm[e] = rr[e] + ri[e];
#pragma unroll
      for (int t = 0; t < M; ++t)
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
          A1[t][e] = fma(c_cur[t].r, sm[e], A1[t][e]);
          A2[t][e] = fma(c_cur[t].sum, ri[e], A2[t][e]);
          A3[t][e] = fma(c_cur[t].dif, rr[e], A3[t][e]);
        }
      if constexpr (kPrefetch) {
#pragma unroll
        for (int t = 0; t < M; ++t) c_cur[t] = c_nxt[t];
      }
    }
  };
  if (Kext > 0) stage(rt0, 0);
  for (int kb = 0; kb < Kext; kb += 2 * KT) {
    __builtin_amdgcn_s_waitcnt(0);                        // this wavefront's part of chunk kb landed
    __syncthreads();                                      // every part; the other buffer is free
    if (kb + KT < Kext) stage(rt1, kb + KT);
    run(rt0, kb, min(KT, Kext - kb));
    if (kb + KT >= Kext) break;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (kb + 2 * KT < Kext) stage(rt0, kb + 2 * KT);
    run(rt1, kb + KT, min(KT, Kext - kb - KT));
  }

#pragma unroll
  for (int t = 0; t < M; ++t) {
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
      const int64_t i = e0 + gauss_elem<SB>(lane, e);
      if (i >= a.D) continue;
      cv<double> v = {A1[t][e] - A2[t][e], A1[t][e] + A3[t][e]};
      // outputs stream through the caches (non-temporal): they must not
      // evict the residual chunks that the other shift tiles still read
      if (ow_mode != 0) v = cadd(v, cmul(ow, AO::template load_nt<double>(a.out, obase + i)));
      if (a.X) v = cadd(v, cmul(pw, AO::template load_nt<double>(a.X, obase + i)));
      AO::store_nt(a.out, obase + i, v);
    }
  }
}

hipError_t launch_flush(Elem eb, Elem eo, const FlushArgs& a, int ow_mode, int engine,
                        hipStream_t st) {
  const int per_xcd = (a.n_etiles + kNumXcd - 1) / kNumXcd;
  dim3 grid(per_xcd * kNumXcd * a.n_stiles, a.nsys);
  if (engine < 0 || engine >= kNumFlushEngines) return hipErrorInvalidValue;
  // 16-byte staging of complex64 slots needs an even D (the caller picks engine 2 otherwise)
  if (eb == Elem::C64 && (a.D & 1) && flush_coef_comps(engine) == 3) return hipErrorInvalidValue;
  if (engine == 5) {
    // the digit planes go to a.work
    if (!a.work) return hipErrorInvalidValue;
    return launch_flush_oz(eb, eo, a, grid, ow_mode, st);
  }
  if (engine == 6) {
    if (eb != Elem::C128) return hipErrorInvalidValue;     // complex128 bank
    return launch_flush_mf64(eo, a, ow_mode, st);
  }
#define MSB_GAUSS(SB, SO, E)                                                                   \
  hipLaunchKernelGGL((k_flush_gauss<SB, SO, gauss_shape(E).M, gauss_shape(E).EPL, gauss_shape(E).NW>), grid, \
                     dim3(gauss_shape(E).NW * kWave), 0, st, a, a.coef, ow_mode);
#define MSB_FLUSH(SB, SO)                                                                      \
  if (engine == 1) hipLaunchKernelGGL((k_flush_mfma<SB, SO>), grid, dim3(kBlock), 0, st, a, ow_mode); \
  else if (engine == 2) hipLaunchKernelGGL((k_flush_valu<SB, SO>), grid, dim3(kBlock), 0, st, a, a.coef, ow_mode); \
  else if (engine == 3) { MSB_GAUSS(SB, SO, 3) }                                               \
  else if (engine == 4) { MSB_GAUSS(SB, SO, 4) }                                               \
  else { MSB_GAUSS(SB, SO, 0) }
  if (eb == Elem::C128 && eo == Elem::C128) {
    MSB_FLUSH(double, double)
  } else if (eb == Elem::C64 && eo == Elem::C64) {
    MSB_FLUSH(float, float)
  } else if (eb == Elem::C64 && eo == Elem::C128) {
    MSB_FLUSH(float, double)
  } else {
    return hipErrorInvalidValue;
  }
#undef MSB_FLUSH
#undef MSB_GAUSS
  return hipGetLastError();
}

}  // namespace msb
