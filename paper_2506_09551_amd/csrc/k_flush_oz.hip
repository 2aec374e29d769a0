// Multi-shift assembly on the int8 matrix cores (assembly engine 5): the
// contraction out[k] += sum_l C[k][l] r_l of the FP64 engines (Appendix C/D:
// Eqs. shift_coeffs, search_dir_, solution_ket_), in its three-product form,
// evaluated exactly in integer arithmetic on digit planes of the operands.
#include "k_common.h"

namespace msb {

// Engine 5: the three-product contraction on the int8 matrix cores, with
// every FP64 operand split into 8-bit digit planes (the error-free splitting
// of Ozaki, Ogita, Oishi and Rump, 2012, in its integer form).
//
// Slot l is first rescaled exactly: its coefficients by 2^(e_l) and its bank
// vector by 2^(-e_l), e_l the exponent of |r_l| (the products are unchanged;
// the operands of one chunk then have comparable magnitudes).  Within a chunk
// of 64 slots each coefficient row (shift, product) and each bank column
// (element, product) gets its own power-of-two scale 2^E with every |v| <
// 2^E; with NP planes, Y = trunc(v 2^(8 NP - 2 - E)) is an integer with
// |Y| < 2^(8 NP - 2), written in balanced digits
// Y = sum_p d_p 2^(8 (NP - 1 - p)), p = 0..NP-1: the bytes of Y plus 128 in
// each lower byte, minus 128, the top digit (in [-64, 64]) taking the carry.
// A digit product has weight 2^(-8(p + q)); the NP (NP + 1) / 2 pairs with
// p + q < NP are summed exactly in 32-bit integers over the chunk by
// v_mfma_i32_16x16x64_i8, one integer sum per level t = p + q, and the level
// sums become one FP64 value scaled by the two chunk exponents.  The dropped
// pairs and the truncation leave an error of order 2^-(8 NP - 3) of the
// chunk's largest product per term, with no bias (balanced digits).  A
// complex128 bank takes NP = 6 (21 pairs; on Krylov banks of the 8- and
// 10-site rings the assembled solutions differ from the FP64 sums by at
// most 2.2e-11 relative), a complex64 bank, whose values carry 24 bits,
// NP = 5 (15 pairs, 256 times that).
//
// MFMA operand layout: lane l holds row l % 16 of A and column l % 16 of B
// for the 16 depth indices 16 (l / 16) .. + 15 (one byte each); the 16 x 16
// result holds row 4 (l / 16) + r, column l % 16 in register r.
constexpr int kOzPlanes = 6;      // digit planes per operand, at most (workspace size)
constexpr int kOzKC = 64;         // slots per chunk (one MFMA depth)
constexpr int kOzNE = 32;         // elements per workgroup (two 16-column tiles)
constexpr int kOzWaves = 8;
constexpr int kOzTPW = 2;         // 16-shift tiles per wavefront
constexpr int kOzShifts = kOzWaves * kOzTPW * 16;   // shift slots per workgroup
static_assert(kOzShifts == 256 && kOzNE == 32, "flush_shifts_per_tile(5), flush_elems_per_tile(5)");
constexpr size_t kOzPlaneBytes = 64 * 16;          // one operand plane of one MFMA
constexpr int kOzNone = -100000;  // exponent of an all-zero row or column
typedef int v4i __attribute__((ext_vector_type(4)));

// biased exponent field of |v| plus de, or kOzNone for zero (and subnormals)
__device__ __forceinline__ int oz_bexp(double v, int de) {
  const int b = (int)((uint32_t)(__double_as_longlong(v) >> 52) & 0x7FFu);
  return b == 0 ? kOzNone : b + de;
}
// Y + bias for Y = trunc(v 2^de 2^(8 NP - 2 - E)), eb the biased chunk
// exponent (every |v 2^de| < 2^(eb - 1022)): the 53-bit significand shifted
// right by 55 - 8 NP + eb - (b + de); the bias is 128 in each of the NP - 1
// lower bytes
template <int NP>
__device__ __forceinline__ int64_t oz_fixed(double v, int eb, int de) {
  const uint64_t bits = (uint64_t)__double_as_longlong(v);
  const int b = (int)((bits >> 52) & 0x7FFu);
  const int sh = 55 - 8 * NP + eb - (b + de);
  const uint64_t m = (bits & 0xFFFFFFFFFFFFFull) | 0x10000000000000ull;
  int64_t y = (b == 0 || sh > 60) ? 0 : (int64_t)(m >> sh);
  y = (bits >> 63) ? -y : y;
  return y + (NP == 6 ? 0x8080808080ll : 0x80808080ll);
}
// the NP digit planes of four biased values as signed bytes, value j in
// byte j: plane 0 is byte NP - 1 of each (the top digit), planes 1..NP-1
// bytes NP-2..0 with 128 subtracted (a byte transpose by v_perm)
template <int NP>
__device__ __forceinline__ void oz_planes4(const int64_t (&y)[4], int (&pl)[NP]) {
  static_assert(NP == 5 || NP == 6, "five or six planes");
  uint32_t lo[4], hi[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    lo[j] = (uint32_t)y[j];
    hi[j] = (uint32_t)((uint64_t)y[j] >> 32);
  }
  // perm(a, b, sel): selector bytes 0-3 pick bytes of b, 4-7 bytes of a
  const uint32_t t0 = __builtin_amdgcn_perm(lo[1], lo[0], 0x05010400u);
  const uint32_t t1 = __builtin_amdgcn_perm(lo[1], lo[0], 0x07030602u);
  const uint32_t t2 = __builtin_amdgcn_perm(lo[3], lo[2], 0x05010400u);
  const uint32_t t3 = __builtin_amdgcn_perm(lo[3], lo[2], 0x07030602u);
  const uint32_t h0 = __builtin_amdgcn_perm(hi[1], hi[0], 0x05010400u);
  const uint32_t h2 = __builtin_amdgcn_perm(hi[3], hi[2], 0x05010400u);
  constexpr int o = NP - 5;                                                   // planes above byte 4
  if constexpr (NP == 6) pl[0] = (int)__builtin_amdgcn_perm(h2, h0, 0x07060302u);   // byte 5
  pl[o] = (int)(__builtin_amdgcn_perm(h2, h0, 0x05040100u) ^ (NP == 6 ? 0x80808080u : 0u));  // byte 4
  pl[o + 1] = (int)(__builtin_amdgcn_perm(t3, t1, 0x07060302u) ^ 0x80808080u);    // byte 3
  pl[o + 2] = (int)(__builtin_amdgcn_perm(t3, t1, 0x05040100u) ^ 0x80808080u);    // byte 2
  pl[o + 3] = (int)(__builtin_amdgcn_perm(t2, t0, 0x07060302u) ^ 0x80808080u);    // byte 1
  pl[o + 4] = (int)(__builtin_amdgcn_perm(t2, t0, 0x05040100u) ^ 0x80808080u);    // byte 0
}
// exponent e_l of slot l (|r_l| in [2^e_l, 2^(e_l + 1))), 0 without norms
__device__ __forceinline__ int oz_slot_exp(const FlushArgs& a, int s, int l) {
  if (!a.rnorm) return 0;
  const double n = a.rnorm[(int64_t)s * a.rn_stride + a.rn_base + l];
  const int b = (int)((uint32_t)(__double_as_longlong(n) >> 52) & 0x7FFu);
  return b == 0 ? 0 : b - 1023;
}

// Coefficient digit planes: one wavefront per (system, 16-shift tile, chunk,
// product); lane l takes row l % 16 (list slot 16 T + l % 16) and the slots
// 64 c + 16 (l / 16) .. + 15.  Writes planes [s][T][c][P][p][64 lanes][16 B]
// and the biased row exponents [s][T][c][P][16].
template <int NP>
__global__ __launch_bounds__(256) void k_oz_coef(FlushArgs a, int n_chunks, v4i* __restrict__ planes,
                                                 int* __restrict__ rexp) {
  const int n_tiles = a.n_list / 16;
  const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int lane = threadIdx.x % kWave;
  const int64_t total = (int64_t)a.nsys * n_tiles * n_chunks * 3;
  if (w >= total) return;
  const int P = (int)(w % 3);
  const int c = (int)((w / 3) % n_chunks);
  const int T = (int)((w / 3 / n_chunks) % n_tiles);
  const int s = (int)(w / 3 / n_chunks / n_tiles);
  const int row = lane % 16, g = lane / 16;
  const int j = 16 * T + row;
  double v[16];
  int de[16];
  int eb = kOzNone;
#pragma unroll
  for (int b = 0; b < 16; ++b) {
    const int l = kOzKC * c + 16 * g + b;
    v[b] = l < a.K ? a.coef[(((int64_t)s * a.K + l) * a.n_list + j) * 3 + P] : 0.0;
    de[b] = l < a.K ? oz_slot_exp(a, s, l) : 0;
    eb = max(eb, oz_bexp(v[b], de[b]));
  }
  eb = max(eb, __shfl_xor(eb, 16));
  eb = max(eb, __shfl_xor(eb, 32));
  int pl[4][NP];
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const int64_t y[4] = {oz_fixed<NP>(v[4 * d], eb, de[4 * d]), oz_fixed<NP>(v[4 * d + 1], eb, de[4 * d + 1]),
                          oz_fixed<NP>(v[4 * d + 2], eb, de[4 * d + 2]), oz_fixed<NP>(v[4 * d + 3], eb, de[4 * d + 3])};
    oz_planes4<NP>(y, pl[d]);
  }
  v4i* dst = planes + (w * NP) * 64;
#pragma unroll
  for (int p = 0; p < NP; ++p) dst[p * 64 + lane] = v4i{pl[0][p], pl[1][p], pl[2][p], pl[3][p]};
  if (lane < 16) rexp[w * 16 + lane] = eb;
}

// The contraction.  A workgroup (8 wavefronts) owns 32 elements and 256
// shift slots of one system; wavefront w takes the 16-shift tiles w and
// w + 8 over both 16-element column tiles.  Per chunk of 64 slots the
// workgroup loads the bank slice (thread t: element t % 32, slots
// 4 (t / 32) .. + 3), finds each element's exponent per product (the values
// re + im, im, re of the three-product form; one barrier), splits the
// values into digit planes in LDS, and every wavefront runs its 2 x 2 tiles
// x 3 products x 21 digit pairs from LDS (bank) and global memory
// (coefficients, cache-resident; the next chunk's first planes are
// requested before the split).  Planes are double-buffered: chunk c + 1 is
// split, and chunk c + 2 is in flight, while the matrix instructions of
// chunk c run.
template <typename SB, typename SO, int NP>
__global__ __launch_bounds__(kOzWaves * kWave) void k_flush_oz(FlushArgs a, const v4i* __restrict__ cplanes,
                                                                const int* __restrict__ crexp, int n_chunks,
                                                                int ow_mode) {
  using AB = Access<SB, true>;
  using AO = Access<SO, true>;
  __shared__ v4i bpl[2][2][3][NP][64];             // [buffer][column tile][product][plane][lane]
  __shared__ int wexp[2][kOzWaves][kOzNE][3];             // per-wavefront maxima of the biased exponents
  __shared__ int cexp[2][kOzNE][3];                       // chunk exponent per element and product

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
  const int64_t e0 = (int64_t)et * kOzNE;
  const void* bank_s = AB::offset(a.bank, (int64_t)s * a.cap * a.D);
  const int n_tiles = a.n_list / 16;
  // this wavefront's shift tiles (list tiles) and their slot extents
  int tile[kOzTPW], kw[kOzTPW];
#pragma unroll
  for (int u = 0; u < kOzTPW; ++u) {
    tile[u] = stt * (kOzShifts / 16) + wave + kOzWaves * u;
    kw[u] = (a.lend && tile[u] < n_tiles) ? __builtin_amdgcn_readfirstlane(a.lend[s * a.n_list + 16 * tile[u]])
                                          : (tile[u] < n_tiles ? Kext : 0);
  }
  const int nck = (Kext + kOzKC - 1) / kOzKC;

  // slicing role of this thread
  const int ie = tid % kOzNE, sq = tid / kOzNE;           // element, slot quad
  int64_t my_e = e0 + ie;
  my_e = my_e < a.D - 1 ? my_e : a.D - 1;                 // clamped: feeds only unstored outputs
  cv<double> rv[4];
  int rde[4];                                             // -e_l of the four slots
  auto load_chunk = [&](int c) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int l = kOzKC * c + 4 * sq + j;
      rv[j] = l < Kext ? AB::template load_nt<double>(bank_s, (int64_t)l * a.D + my_e) : cv<double>{0.0, 0.0};
      rde[j] = l < Kext ? -oz_slot_exp(a, s, l) : 0;
    }
  };
  // exponents of chunk c (values in rv) -> wexp[buf]
  auto chunk_exp = [&](int buf) {
    int m0 = kOzNone, m1 = kOzNone, m2 = kOzNone;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      m0 = max(m0, oz_bexp(rv[j].re + rv[j].im, rde[j]));
      m1 = max(m1, oz_bexp(rv[j].im, rde[j]));
      m2 = max(m2, oz_bexp(rv[j].re, rde[j]));
    }
    m0 = max(m0, __shfl_xor(m0, 32));
    m1 = max(m1, __shfl_xor(m1, 32));
    m2 = max(m2, __shfl_xor(m2, 32));
    if (lane < 32) {
      wexp[buf][wave][ie][0] = m0;
      wexp[buf][wave][ie][1] = m1;
      wexp[buf][wave][ie][2] = m2;
    }
  };
  // digit planes of chunk (values in rv) -> bpl[buf], after the exponents are complete
  auto chunk_split = [&](int buf) {
    int eb[3] = {kOzNone, kOzNone, kOzNone};
#pragma unroll
    for (int w = 0; w < kOzWaves; ++w)
#pragma unroll
      for (int P = 0; P < 3; ++P) eb[P] = max(eb[P], wexp[buf][w][ie][P]);
    if (sq == 0) {
#pragma unroll
      for (int P = 0; P < 3; ++P) cexp[buf][ie][P] = eb[P];
    }
    const int ct = ie / 16, col = ie % 16;
    const int L = col + 16 * (sq / 4), dw = sq % 4;      // lane and dword of the operand
#pragma unroll
    for (int P = 0; P < 3; ++P) {
      int64_t y[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double v = P == 0 ? rv[j].re + rv[j].im : (P == 1 ? rv[j].im : rv[j].re);
        y[j] = oz_fixed<NP>(v, eb[P], rde[j]);
      }
      int pl[NP];
      oz_planes4<NP>(y, pl);
#pragma unroll
      for (int p = 0; p < NP; ++p) reinterpret_cast<int*>(&bpl[buf][ct][P][p][L])[dw] = pl[p];
    }
  };

  // FP64 sums: [tile][column tile][re/im][row r]
  double acc[kOzTPW][2][2][4];
#pragma unroll
  for (int u = 0; u < kOzTPW; ++u)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[u][ct][0][r] = acc[u][ct][1][r] = 0.0;

  // coefficient planes and row exponents of (chunk c, product P, tile u),
  // walked in the order (c, P, u)
  struct AOps {
    v4i A[NP];
    v4i ea;
  };
  auto load_a = [&](int c, int P, int u, AOps& o) {
    if (c < nck && kOzKC * c < kw[u]) {
      const int64_t w = (((int64_t)s * n_tiles + tile[u]) * n_chunks + c) * 3 + P;
#pragma unroll
      for (int p = 0; p < NP; ++p) o.A[p] = cplanes[(w * NP + p) * 64 + lane];
      o.ea = *reinterpret_cast<const v4i*>(crexp + w * 16 + 4 * (lane / 16));
    }
  };
  AOps cur;
  // the matrix instructions of chunk c (planes in bpl[buf]); cur holds the
  // operands of (c, 0, 0) on entry and of (c + 1, 0, 0) on exit
  auto run = [&](int c, int buf) {
#pragma unroll
    for (int P = 0; P < 3; ++P)
#pragma unroll
      for (int u = 0; u < kOzTPW; ++u) {
        if (P + u > 0) load_a(c, P, u, cur);
        if (kOzKC * c < kw[u]) {
#pragma unroll
          for (int ct = 0; ct < 2; ++ct) {
            v4i B[NP];
#pragma unroll
            for (int p = 0; p < NP; ++p) B[p] = bpl[buf][ct][P][p][lane];
            const int eb = cexp[buf][16 * ct + lane % 16][P];
            v4i lv[NP];
#pragma unroll
            for (int t = 0; t < NP; ++t) lv[t] = v4i{0, 0, 0, 0};
#pragma unroll
            for (int qb = 0; qb < NP; ++qb)
#pragma unroll
              for (int pa = 0; pa + qb < NP; ++pa)
                lv[pa + qb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(cur.A[pa], B[qb], lv[pa + qb], 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              // levels 0..NP-1 (weights 2^(-8t)) -> one FP64 value in units of
              // 2^(-8 (NP - 1)); adjacent levels are first joined in 32 bits
              double h = 0.0;
#pragma unroll
              for (int t = 0; t < NP; t += 2) {
                if (t + 1 < NP) h = fma(h, 65536.0, (double)(lv[t][r] * 256 + lv[t + 1][r]));
                else h = fma(h, 256.0, (double)lv[t][r]);
              }
              const double x = ldexp(h, cur.ea[r] + eb - 2044 - 12 - 8 * (NP - 1));
              if (P == 0) {
                acc[u][ct][0][r] += x;
                acc[u][ct][1][r] += x;
              } else if (P == 1) {
                acc[u][ct][0][r] -= x;
              } else {
                acc[u][ct][1][r] += x;
              }
            }
          }
        }
      }
    load_a(c + 1, 0, 0, cur);
  };

  // chunk c + 2 is in flight while the matrix instructions of chunk c run,
  // and chunk c + 1 is split into the other plane buffer before them
  if (nck > 0) {
    load_a(0, 0, 0, cur);
    load_chunk(0);
    chunk_exp(0);
    __syncthreads();
    chunk_split(0);
    if (nck > 1) {
      load_chunk(1);
      chunk_exp(1);
    }
  }
  const bool run_first = wave < kOzWaves / 2;
  for (int c = 0; c < nck; ++c) {
    const int buf = c & 1;
    __syncthreads();      // planes of chunk c and the maxima of chunk c + 1 complete
    if (c + 1 < nck) {
      chunk_split(buf ^ 1);
      if (c + 2 < nck) load_chunk(c + 2);
    }
    run(c, buf);
    if (c + 2 < nck) chunk_exp(buf);
  }

#pragma unroll
  for (int u = 0; u < kOzTPW; ++u) {
    if (tile[u] >= n_tiles) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int slot = 16 * tile[u] + 4 * (lane / 16) + r;
      const int k = a.list[s * a.n_list + slot];
      if (k < 0) continue;
      cv<double> ow = {0.0, 0.0}, pw = {0.0, 0.0};
      if (ow_mode == 1) ow = {1.0, 0.0};
      if (ow_mode == 2) {
        const double* o = a.ow + ((int64_t)s * a.n_list + slot) * a.ow_stride;
        ow = {o[0], o[1]};
      }
      if (a.pw) {
        const double* pp = a.pw + ((int64_t)s * a.n_list + slot) * a.pw_stride;
        pw = {pp[0], pp[1]};
      }
      const int64_t obase = ((int64_t)s * a.n_shift + k) * a.D;
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
        const int64_t i = e0 + 16 * ct + lane % 16;
        if (i >= a.D) continue;
        cv<double> v = {acc[u][ct][0][r], acc[u][ct][1][r]};
        if (ow_mode != 0) v = cadd(v, cmul(ow, AO::template load_nt<double>(a.out, obase + i)));
        if (a.X) v = cadd(v, cmul(pw, AO::template load_nt<double>(a.X, obase + i)));
        AO::store_nt(a.out, obase + i, v);
      }
    }
  }
}

size_t flush_work_bytes(int engine, int nsys, int n_list, int K) {
  if (engine != 5) return 0;
  const size_t n_chunks = (size_t)(K + kOzKC - 1) / kOzKC;
  const size_t units = (size_t)nsys * (n_list / 16) * n_chunks * 3;
  return units * (kOzPlanes * kOzPlaneBytes + 16 * sizeof(int));
}

template <typename SB, typename SO, int NP>
static hipError_t launch_oz(const FlushArgs& a, dim3 grid, int ow_mode, hipStream_t st) {
  const int n_chunks = (a.K + kOzKC - 1) / kOzKC;
  const int64_t units = (int64_t)a.nsys * (a.n_list / 16) * n_chunks * 3;
  v4i* planes = static_cast<v4i*>(a.work);
  int* rexp = reinterpret_cast<int*>(static_cast<char*>(a.work) + units * NP * kOzPlaneBytes);
  const int64_t blocks = (units * kWave + 255) / 256;
  if (blocks > 0)
    hipLaunchKernelGGL(k_oz_coef<NP>, dim3((unsigned)blocks), dim3(256), 0, st, a, n_chunks, planes, rexp);
  hipLaunchKernelGGL((k_flush_oz<SB, SO, NP>), grid, dim3(kOzWaves * kWave), 0, st, a, planes, rexp, n_chunks,
                     ow_mode);
  return hipGetLastError();
}

// complex128 banks: six planes (46 bits); complex64 banks (24-bit values):
// five planes (38 bits), 15 digit pairs
hipError_t launch_flush_oz(Elem eb, Elem eo, const FlushArgs& a, dim3 grid, int ow_mode, hipStream_t st) {
  if (eb == Elem::C128 && eo == Elem::C128) return launch_oz<double, double, 6>(a, grid, ow_mode, st);
  if (eb == Elem::C64 && eo == Elem::C64) return launch_oz<float, float, 5>(a, grid, ow_mode, st);
  if (eb == Elem::C64 && eo == Elem::C128) return launch_oz<float, double, 5>(a, grid, ow_mode, st);
  return hipErrorInvalidValue;
}

}  // namespace msb
