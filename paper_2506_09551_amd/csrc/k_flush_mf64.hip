// Multi-shift assembly on the FP64 matrix cores in the three-product form
// (assembly engine 6): the contraction out[k] += sum_l C[k][l] r_l of the
// other engines (Appendix C/D: Eqs. shift_coeffs, search_dir_,
// solution_ket_), evaluated with v_mfma_f64_16x16x4f64.
//
// With s = r_re + r_im per element and the table entry (c_re, c_re + c_im,
// c_im - c_re) written by k_coef,
//   c r = [c_re s - (c_re + c_im) r_im] + i [c_re s + (c_im - c_re) r_re],
// three real matrix products (P1 = C_re S, P2 = C_sum R_im, P3 = C_dif R_re)
// give re = P1 - P2 and im = P1 + P3.
//
// v_mfma_f64_16x16x4f64: D(16 x 16) += A(16 x 4) B(4 x 16), A[i][k] in lane
// i + 16 k, B[k][j] in lane j + 16 k, D[i][j] in lane j + 16 (i % 4),
// register i / 4.  Rows are shifts, the depth is residual slots, columns
// are elements.
//
// A workgroup owns kMfNE elements and one group of at most kMfMaxWaves
// 16-shift tiles of one system: the bank slice of the group is read from
// memory once, in chunks of kMfKT slots that go straight to LDS
// (global_load_lds, double-buffered), and every wavefront runs a tile over
// both column tiles from there.  With T tiles in the group and
// W = min(kMfMaxWaves, T + min(T, kMfMaxSplit)) wavefronts, the first W - T
// tiles (the longest: the list is sorted by descending range) are shared by
// two wavefronts, each taking half of the depth steps of every chunk, whose
// sums are added through LDS at the end; the others take one wavefront
// each.  The four SIMDs then get nearly equal shares of the matrix
// instructions between two barriers.  A wavefront's coefficients of the
// next chunk are requested before the current chunk's matrix instructions.
#include "k_common.h"

namespace msb {

constexpr int kMfNE = 32;          // elements per workgroup (column tiles of 16)
constexpr int kMfCT = kMfNE / 16;  // column tiles
constexpr int kMfKT = 16;          // slots per staged chunk
constexpr int kMfKS = kMfKT / 4;   // matrix-instruction depth steps per chunk
constexpr int kMfMaxWaves = 16;
constexpr int kMfMaxSplit = 4;    // tiles shared by two wavefronts, at most

typedef double v4d __attribute__((ext_vector_type(4)));

template <typename SO>
__global__ __launch_bounds__(kMfMaxWaves * kWave, 4) void k_flush_mf64(FlushArgs a, int n_groups, int tg,
                                                                      int ow_mode) {
  using AO = Access<SO, true>;
  // two chunk buffers as two objects: the DMA into one does not make the
  // compiler wait before reads of the other
  __shared__ double2 st0[kMfKT][kMfNE];
  __shared__ double2 st1[kMfKT][kMfNE];
  __shared__ double red[kMfMaxSplit][kMfCT * 3 * 4][kWave];   // odd-chunk sums of shared tiles

  const int s = blockIdx.y;
  const int b = blockIdx.x;
  const int xcd = b % kNumXcd, q = b / kNumXcd;
  const int et = xcd + kNumXcd * (q / n_groups);
  const int grp = q % n_groups;
  if (et >= a.n_etiles) return;
  const int nw = blockDim.x / kWave;                       // wavefronts (uniform)
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
  const int lane = tid % kWave;
  const int li = lane % 16, lk = lane / 16;
  const int n_tiles = a.n_list / 16;
  const int n_split = nw - tg;                             // shared tiles of the group
  const int tile0 = grp * tg;
  // this wavefront's tile, and its half of the depth steps (-1: all)
  const int tile = tile0 + (wave < 2 * n_split ? wave / 2 : wave - n_split);
  const int parity = wave < 2 * n_split ? wave % 2 : -1;
  auto ks_on = [&](int ks) { return parity < 0 || (ks >= kMfKS / 2) == (parity == 1); };
  // slots of the group (first tile: the list is sorted by descending range)
  // and of this wavefront's tile
  const int Kext = a.tile_k[s * a.n_stiles + tile0];
  const int kw = tile < n_tiles ? __builtin_amdgcn_readfirstlane(a.tile_k[s * a.n_stiles + tile]) : 0;
  const int64_t e0 = (int64_t)et * kMfNE;
  const double2* bank_s = reinterpret_cast<const double2*>(a.bank) + (int64_t)s * a.cap * a.D;

  // DMA of chunk c: kMfKT slots x kMfNE elements, 16 bytes per lane, the
  // wave loads of the workgroup in turn
  auto stage = [&](double2 (&buf)[kMfKT][kMfNE], int c) {
    constexpr int kRows = kMfKT * kMfNE / kWave;           // wave loads per chunk
    for (int row = wave; row < kRows; row += nw) {
      const int k = row * (kWave / kMfNE) + lane / kMfNE;  // slot within the chunk
      int l = kMfKT * c + k;
      l = l < Kext ? l : Kext - 1;                         // clamped: zero coefficients there
      int64_t e = e0 + lane % kMfNE;
      e = e < a.D - 1 ? e : a.D - 1;                       // clamped: feeds only unstored outputs
      __builtin_amdgcn_global_load_lds(static_cast<const void*>(bank_s + (int64_t)l * a.D + e),
                                       (__attribute__((address_space(3))) void*)&buf[row * (kWave / kMfNE)][0],
                                       16, 0, 0);
    }
  };
  // this lane's A operands of chunk c: row li (shift 16 tile + li), slot
  // 16 c + 4 ks + lk, three components; zero past the table
  struct COps {
    double c[kMfKS][3];
  };
  const double* crow = a.coef + ((int64_t)s * a.K * a.n_list + 16 * (int64_t)tile + li) * 3;
  auto load_c = [&](int c, COps& o) {
#pragma unroll
    for (int ks = 0; ks < kMfKS; ++ks) {
      if (!ks_on(ks)) continue;
      const int l = kMfKT * c + 4 * ks + lk;
      const bool in = l < a.K && tile < n_tiles;
      const double* e = crow + (int64_t)(in ? l : 0) * a.n_list * 3;
#pragma unroll
      for (int p = 0; p < 3; ++p) o.c[ks][p] = in ? e[p] : 0.0;
    }
  };

  v4d A1[kMfCT], A2[kMfCT], A3[kMfCT];
#pragma unroll
  for (int t = 0; t < kMfCT; ++t) A1[t] = A2[t] = A3[t] = v4d{0.0, 0.0, 0.0, 0.0};

  auto run = [&](const double2 (&buf)[kMfKT][kMfNE], const COps& co) {
#pragma unroll
    for (int ks = 0; ks < kMfKS; ++ks) {
      if (!ks_on(ks)) continue;
#pragma unroll
      for (int t = 0; t < kMfCT; ++t) {
        // B[k][j]: slot 4 ks + lk, element 16 t + li
        const double2 r = buf[4 * ks + lk][16 * t + li];
        const double sm = r.x + r.y;
        A1[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(co.c[ks][0], sm, A1[t], 0, 0, 0);
        A2[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(co.c[ks][1], r.y, A2[t], 0, 0, 0);
        A3[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(co.c[ks][2], r.x, A3[t], 0, 0, 0);
      }
    }
  };

  const int nck = (Kext + kMfKT - 1) / kMfKT;
  COps cur, nxt;
  if (nck > 0) {
    if (kw > 0) load_c(0, cur);
    stage(st0, 0);
  }
  for (int c = 0; c < nck; c += 2) {
    __builtin_amdgcn_s_waitcnt(0);                         // this wavefront's part of chunk c landed
    __syncthreads();                                       // every part; st1 no longer read
    if (c + 1 < nck) {
      stage(st1, c + 1);
      if (kMfKT * (c + 1) < kw) load_c(c + 1, nxt);
    }
    if (kMfKT * c < kw) run(st0, cur);
    if (c + 1 >= nck) break;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (c + 2 < nck) {
      stage(st0, c + 2);
      if (kMfKT * (c + 2) < kw) load_c(c + 2, cur);
    }
    if (kMfKT * (c + 1) < kw) run(st1, nxt);
  }

  // shared tiles: the second half's sums go through LDS to the first half's wavefront
  if (n_split > 0) {
    if (parity == 1) {
#pragma unroll
      for (int t = 0; t < kMfCT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          red[wave / 2][(t * 3 + 0) * 4 + r][lane] = A1[t][r];
          red[wave / 2][(t * 3 + 1) * 4 + r][lane] = A2[t][r];
          red[wave / 2][(t * 3 + 2) * 4 + r][lane] = A3[t][r];
        }
    }
    __syncthreads();
    if (parity == 1) return;
    if (parity == 0) {
#pragma unroll
      for (int t = 0; t < kMfCT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          A1[t][r] += red[wave / 2][(t * 3 + 0) * 4 + r][lane];
          A2[t][r] += red[wave / 2][(t * 3 + 1) * 4 + r][lane];
          A3[t][r] += red[wave / 2][(t * 3 + 2) * 4 + r][lane];
        }
    }
  }

  if (tile >= n_tiles) return;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int slot = 16 * tile + 4 * r + lk;               // D row i = 4 r + lane / 16
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
    for (int t = 0; t < kMfCT; ++t) {
      const int64_t i = e0 + 16 * t + li;                  // D column j = lane % 16
      if (i >= a.D) continue;
      cv<double> v = {A1[t][r] - A2[t][r], A1[t][r] + A3[t][r]};
      // outputs stream through the caches (non-temporal)
      if (ow_mode != 0) v = cadd(v, cmul(ow, AO::template load_nt<double>(a.out, obase + i)));
      if (a.X) v = cadd(v, cmul(pw, AO::template load_nt<double>(a.X, obase + i)));
      AO::store_nt(a.out, obase + i, v);
    }
  }
}

hipError_t launch_flush_mf64(Elem eo, const FlushArgs& a, int ow_mode, hipStream_t st) {
  const int n_tiles = a.n_list / 16;
  if (n_tiles <= 0 || a.n_stiles != n_tiles) return hipErrorInvalidValue;
  // groups of nearly equal size, at most kMfMaxWaves tiles each, and the
  // wavefronts of a group (its first nw - tg tiles shared by two)
  const int n_groups = (n_tiles + kMfMaxWaves - 1) / kMfMaxWaves;
  const int tg = (n_tiles + n_groups - 1) / n_groups;
  const int nw = std::min(kMfMaxWaves, tg + std::min(tg, kMfMaxSplit));
  const int per_xcd = (a.n_etiles + kNumXcd - 1) / kNumXcd;
  const dim3 grid(per_xcd * kNumXcd * n_groups, a.nsys);
  if (eo == Elem::C128)
    hipLaunchKernelGGL(k_flush_mf64<double>, grid, dim3(nw * kWave), 0, st, a, n_groups, tg, ow_mode);
  else if (eo == Elem::C64)
    hipLaunchKernelGGL(k_flush_mf64<float>, grid, dim3(nw * kWave), 0, st, a, n_groups, tg, ow_mode);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace msb
