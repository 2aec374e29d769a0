// Surrogate network of the learned form: an ensemble of multilayer
// perceptrons 6 -> 512 -> 512 -> 512 -> 1 with GELU, trained with Adam.
//
// Precision: the two 512 x 512 layers (forward, input-gradient and
// weight-gradient products) run on the bfloat16 matrix cores with float32
// accumulation (gfx950 v_mfma_f32_32x32x16_bf16); the activations and the
// back-propagated gradients that feed those products are stored in
// bfloat16, everything else (first and last layer, biases, loss, Adam, the
// master weights) is float32.  Every member of the ensemble is one
// blockIdx.z slice of the same launches.
#include "k_common.h"
#include "mlp_internal.h"

namespace msb {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
// gelu(x) and gelu'(x) from one erf: the forward pass keeps gelu'(z) for the
// backward pass (the only use of the pre-activation z)
__device__ __forceinline__ void gelu_both(float x, float& g, float& gp) {
  const float c = 0.5f * (1.0f + erff(x * 0.70710678118654752f));
  g = x * c;
  gp = c + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

// ---- matrix-core product --------------------------------------------------
// C[M][N] = sum_k A[m][k] B[n][k]: both operands are stored k-contiguous (the
// layers keep bfloat16 copies of W and W^T, and the activations that feed a
// weight gradient are also written transposed), so every tile moves with
// 16-byte loads and stores.  A 256-thread workgroup computes a 128 x 128
// tile, each wave a 64 x 64 quarter as 2 x 2 blocks of 32 x 32 matrix-core
// products.  K advances 64 at a time through two LDS buffers: the next tile
// is loaded into registers while the current one is multiplied.
constexpr int kGM = 128, kGN = 128, kGK = 64, kGPad = 8;

template <int EPI>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  // operand stages; after the K loop the same bytes hold the transposed
  // output tile st[column][row] (128 x (128 + 8) bf16 = 34 KB of the 72 KB)
  __shared__ __align__(16) __bf16 sab[2 * 2 * kGM * (kGK + kGPad)];
  auto& sa = *reinterpret_cast<__bf16 (*)[2][kGM][kGK + kGPad]>(sab);
  auto& sb = *reinterpret_cast<__bf16 (*)[2][kGN][kGK + kGPad]>(sab + 2 * kGM * (kGK + kGPad));
  auto& st = *reinterpret_cast<__bf16 (*)[kGN][kGM + kGPad]>(sab);
  static_assert(kGN * (kGM + kGPad) <= 4 * kGM * (kGK + kGPad), "transposed tile fits the operand stages");
  const int splits = g.splitk > 1 ? g.splitk : 1;
  const int mem = blockIdx.z / splits, ks = blockIdx.z % splits;
  const int klen = g.K / splits, kbeg = ks * klen;
  const __bf16* A = g.A + (int64_t)mem * g.sA + kbeg;
  const __bf16* B = g.B + (int64_t)mem * g.sB + kbeg;
  const int m0 = blockIdx.y * kGM, n0 = blockIdx.x * kGN;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

  // tile chunk c = tid + 256 it: row c / 8, k offset (c % 8) * 8
  bf16x8 ra[4], rb[4];
  auto gload = [&](int k0) {
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int c = tid + it * 256, r = c >> 3, kc = (c & 7) * 8;
      ra[it] = *reinterpret_cast<const bf16x8*>(A + (int64_t)(m0 + r) * g.lda + k0 + kc);
      rb[it] = *reinterpret_cast<const bf16x8*>(B + (int64_t)(n0 + r) * g.ldb + k0 + kc);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int c = tid + it * 256, r = c >> 3, kc = (c & 7) * 8;
      *reinterpret_cast<bf16x8*>(&sa[buf][r][kc]) = ra[it];
      *reinterpret_cast<bf16x8*>(&sb[buf][r][kc]) = rb[it];
    }
  };
  gload(0);
  sstore(0);
  __syncthreads();
  for (int k0 = 0; k0 < klen; k0 += kGK) {
    const int buf = (k0 / kGK) & 1;
    const bool more = k0 + kGK < klen;
    if (more) gload(k0 + kGK);
#pragma unroll
    for (int kk = 0; kk < kGK; kk += 16) {
      bf16x8 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
        a[i] = *reinterpret_cast<const bf16x8*>(&sa[buf][wm + i * 32 + (lane & 31)][kk + 8 * (lane >> 5)]);
#pragma unroll
      for (int j = 0; j < 2; ++j)
        b[j] = *reinterpret_cast<const bf16x8*>(&sb[buf][wn + j * 32 + (lane & 31)][kk + 8 * (lane >> 5)]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (more) sstore(buf ^ 1);   // buf ^ 1 was last read before the previous barrier
    __syncthreads();
  }

  // accumulator lane layout: column lane % 32, row 8 (r / 4) + 4 (lane / 32) + r % 4
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row0 = m0 + wm + i * 32 + 8 * q + 4 * (lane >> 5);
        const int col = n0 + wn + j * 32 + (lane & 31);
        __bf16 hv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = row0 + r;
          const float v = acc[i][j][4 * q + r];
          if constexpr (EPI == kEpiFwd) {
            const float z = v + g.bias[(int64_t)mem * g.sBias + col];
            float h, hp;
            if (g.C) {            // training: keep gelu'(z) for the backward pass
              gelu_both(z, h, hp);
              g.C[(int64_t)mem * g.sC + (int64_t)row * g.ldc + col] = hp;
            } else {
              h = gelu_f(z);
            }
            hv[r] = (__bf16)h;
            g.H[(int64_t)mem * g.sH + (int64_t)row * g.ldh + col] = hv[r];
          } else if constexpr (EPI == kEpiDh) {
            const float zp = g.Zp[(int64_t)mem * g.sZ + (int64_t)row * g.ldz + col];
            hv[r] = (__bf16)(v * zp);
            g.H[(int64_t)mem * g.sH + (int64_t)row * g.ldh + col] = hv[r];
          } else {    // float32 output; a K slice writes its own partial copy
            g.C[(int64_t)ks * g.sCk + (int64_t)mem * g.sC + (int64_t)row * g.ldc + col] = v;
          }
        }
        if constexpr (EPI != kEpiStore) {
          if (g.HT) {   // transposed tile in LDS: four consecutive rows are one 8-byte write
            typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
            bf16x4 t4 = {hv[0], hv[1], hv[2], hv[3]};
            *reinterpret_cast<bf16x4*>(&st[col - n0][row0 - m0]) = t4;
          }
        }
      }
  if constexpr (EPI != kEpiStore) {
    if (g.HT) {
      // the 128 x 128 transposed tile leaves as whole 256-byte rows of H^T
      __syncthreads();
#pragma unroll
      for (int it = 0; it < 8; ++it) {
        const int c = tid + it * 256, cl = c >> 4, rc = (c & 15) * 8;
        *reinterpret_cast<bf16x8*>(g.HT + (int64_t)mem * g.sHT + (int64_t)(n0 + cl) * g.ldht + m0 + rc) =
            *reinterpret_cast<const bf16x8*>(&st[cl][rc]);
      }
    }
  }
}

hipError_t launch_gemm(int epi, const GemmArgs& g, int members, hipStream_t st) {
  const int splits = g.splitk > 1 ? g.splitk : 1;
  if (g.M % kGM || g.N % kGN || g.K % (kGK * splits)) return hipErrorInvalidValue;
  if (splits > 1 && epi != kEpiStore) return hipErrorInvalidValue;
  dim3 grid(g.N / kGN, g.M / kGM, members * splits);
  if (epi == kEpiFwd) hipLaunchKernelGGL(k_gemm<kEpiFwd>, grid, dim3(256), 0, st, g);
  else if (epi == kEpiDh) hipLaunchKernelGGL(k_gemm<kEpiDh>, grid, dim3(256), 0, st, g);
  else if (epi == kEpiStore) hipLaunchKernelGGL(k_gemm<kEpiStore>, grid, dim3(256), 0, st, g);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// ---- first layer: z1 = ((x - shift) * scale) W1 + b1, h1 = gelu(z1) ---------
// Row b of the batch is point perm[b] (perm == nullptr: point base + b).
// A workgroup computes a 64 x 64 tile and writes h1 both row-major and
// transposed (through LDS, so both stores are coalesced).
__global__ __launch_bounds__(256) void k_layer1_fwd(MlpFwdArgs a) {
  __shared__ __bf16 tile[64][66];
  const int mem = blockIdx.z;
  const int n = blockIdx.x * 64 + (threadIdx.x & 63);
  const int b0 = blockIdx.y * 64;
  const float* W1 = a.params + (int64_t)mem * a.pstride + kOffW1;
  const float bias = a.params[(int64_t)mem * a.pstride + kOffB1 + n];
  float w[kMlpIn];
#pragma unroll
  for (int k = 0; k < kMlpIn; ++k) w[k] = W1[k * kMlpH + n] * a.in_scale[k];
  const int* perm = a.perm ? a.perm + (int64_t)mem * a.perm_stride + (int64_t)(*a.step) * a.batch : nullptr;
  for (int r = threadIdx.x >> 6; r < 64; r += 4) {
    const int b = b0 + r;
    float z = bias;
    if (b < a.valid) {            // padding rows see zero inputs
      const int64_t pt = a.base + (perm ? perm[b] : b);
#pragma unroll
      for (int k = 0; k < kMlpIn; ++k) z += (a.X[pt * kMlpIn + k] - a.in_shift[k]) * w[k];
    }
    const int64_t i = (int64_t)mem * a.act_stride + (int64_t)b * kMlpH + n;
    float hf, hp;
    if (a.z1) {                   // training: keep gelu'(z1) for the backward pass
      gelu_both(z, hf, hp);
      a.z1[i] = hp;
    } else {
      hf = gelu_f(z);
    }
    const __bf16 h = (__bf16)hf;
    a.h1[i] = h;
    tile[threadIdx.x & 63][r] = h;
  }
  if (!a.h1T) return;             // inference: no transposed copy
  __syncthreads();
  // transposed: h1T[n][b], 4 threads per column, 16 rows each
  const int c = threadIdx.x >> 2, r0 = (threadIdx.x & 3) * 16;
  __bf16* dst = a.h1T + (int64_t)mem * a.actT_stride + (int64_t)(blockIdx.x * 64 + c) * a.ldT + b0 + r0;
#pragma unroll
  for (int j = 0; j < 16; ++j) dst[j] = tile[c][r0 + j];
}

// ---- output layer: y = h3 W4 + b4; loss gradient g = 2 (y - t) / batch ------
// One wave per batch row; per-workgroup loss partials (deterministic sum).
__global__ __launch_bounds__(256) void k_layer4_fwd(MlpFwdArgs a) {
  const int mem = blockIdx.z;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int b = blockIdx.x * 4 + wave;
  const float* W4 = a.params + (int64_t)mem * a.pstride + kOffW4;
  float s = 0.0f;
  if (b < a.batch) {
    const __bf16* h = a.h3 + (int64_t)mem * a.act_stride + (int64_t)b * kMlpH;
#pragma unroll
    for (int t = 0; t < kMlpH / 64; ++t) s += (float)h[lane + 64 * t] * W4[lane + 64 * t];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  __shared__ double part[4];
  double l2 = 0.0;
  if (b < a.batch && lane == 0) {
    const float y = s + a.params[(int64_t)mem * a.pstride + kOffB4];
    a.y[(int64_t)mem * a.y_stride + b] = y;
    if (a.T) {
      float gv = 0.0f;
      if (b < a.valid) {
        const int* perm = a.perm ? a.perm + (int64_t)mem * a.perm_stride + (int64_t)(*a.step) * a.batch : nullptr;
        const int64_t pt = a.base + (perm ? perm[b] : b);
        const float d = y - a.out_scale * a.T[pt];
        gv = 2.0f * d / (float)a.valid;
        l2 = (double)d * (double)d;
      }
      a.g[(int64_t)mem * a.y_stride + b] = gv;
    }
  }
  if (lane == 0) part[wave] = l2;
  __syncthreads();
  if (threadIdx.x == 0 && a.loss_part)
    a.loss_part[(int64_t)mem * gridDim.x + blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

__global__ __launch_bounds__(kBlock) void k_loss_record(const double* loss_part, int nparts, const int* step,
                                                        double* hist, int64_t hist_stride, int valid) {
  const int mem = blockIdx.x;
  double s[1] = {0.0};
  for (int p = threadIdx.x; p < nparts; p += kBlock) s[0] += loss_part[(int64_t)mem * nparts + p];
  __shared__ double sh[1][kBlock / kWave];
  block_sum<1>(s, sh);
  if (threadIdx.x == 0) hist[(int64_t)mem * hist_stride + *step] = s[0] / valid;
}

hipError_t launch_loss_record(const MlpFwdArgs& a, double* loss_hist, int64_t hist_stride, int members,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_loss_record, dim3(members), dim3(kBlock), 0, st, a.loss_part, (a.batch + 3) / 4, a.step,
                     loss_hist, hist_stride, a.valid);
  return hipGetLastError();
}

// ---- output-layer backward: dz3 = g W4^T * gelu'(z3) (bf16) ----------------
__global__ __launch_bounds__(256) void k_layer4_bwd(MlpFwdArgs a) {
  __shared__ __bf16 tile[64][66];
  const int mem = blockIdx.z;
  const int n = blockIdx.x * 64 + (threadIdx.x & 63);
  const int b0 = blockIdx.y * 64;
  const float w = a.params[(int64_t)mem * a.pstride + kOffW4 + n];
  for (int r = threadIdx.x >> 6; r < 64; r += 4) {
    const int b = b0 + r;
    const int64_t i = (int64_t)mem * a.act_stride + (int64_t)b * kMlpH + n;
    const float gv = a.g[(int64_t)mem * a.y_stride + b];
    const __bf16 d = (__bf16)(gv * w * a.z3[i]);   // z3 holds gelu'(z3)
    a.dz3[i] = d;
    tile[threadIdx.x & 63][r] = d;
  }
  __syncthreads();
  const int c = threadIdx.x >> 2, r0 = (threadIdx.x & 3) * 16;
  __bf16* dst = a.dz3T + (int64_t)mem * a.actT_stride + (int64_t)(blockIdx.x * 64 + c) * a.ldT + b0 + r0;
#pragma unroll
  for (int j = 0; j < 16; ++j) dst[j] = tile[c][r0 + j];
}

// ---- column sums over the batch --------------------------------------------
// out[n] = sum_b w_b * src(b, n) for the bias gradients (src = dz, bf16), the
// output-layer weight gradient (src = h3, weights g) and its bias (src = g).
// A workgroup owns 64 columns and a slice of kRowsPerPart rows: its four
// waves take every fourth row (coalesced 64-column rows) and meet in LDS; a
// second launch adds the slices in order.
__global__ __launch_bounds__(256) void k_colsum_part(ColSumArgs a) {
  __shared__ float red[4][64];
  const int mem = blockIdx.z;
  const int c = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + c;
  const int r0 = blockIdx.y * a.rows_per_part, r1 = min(a.nrows, r0 + a.rows_per_part);
  float s = 0.0f;
  if (n < a.ncols) {
    for (int b = r0 + grp; b < r1; b += 4) {
      float v = a.src_bf16 ? (float)a.src_bf16[(int64_t)mem * a.src_stride + (int64_t)b * a.ld + n]
                           : a.src_f32[(int64_t)mem * a.src_stride + (int64_t)b * a.ld + n];
      if (a.wgt) v *= a.wgt[(int64_t)mem * a.wgt_stride + b];
      s += v;
    }
  }
  red[grp][c] = s;
  __syncthreads();
  if (grp == 0 && n < a.ncols)
    a.part[((int64_t)mem * gridDim.y + blockIdx.y) * a.ncols + n] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
}

__global__ __launch_bounds__(256) void k_colsum_fin(ColSumArgs a, int nparts) {
  const int mem = blockIdx.z;
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= a.ncols) return;
  float s = 0.0f;
  for (int p = 0; p < nparts; ++p) s += a.part[((int64_t)mem * nparts + p) * a.ncols + n];
  a.out[(int64_t)mem * a.out_stride + n] = s;
}

hipError_t launch_colsum(const ColSumArgs& a, int members, hipStream_t st) {
  const int nparts = (a.nrows + a.rows_per_part - 1) / a.rows_per_part;
  if (nparts > a.max_parts) return hipErrorInvalidValue;
  dim3 grid((a.ncols + 63) / 64, nparts, members);
  hipLaunchKernelGGL(k_colsum_part, grid, dim3(256), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_colsum_fin, dim3((a.ncols + 255) / 256, 1, members), dim3(256), 0, st, a, nparts);
  return hipGetLastError();
}

// ---- first-layer weight gradient: dW1[k][n] = sum_b xn(b, k) dz1(b, n) -------
// Same decomposition as the column sums, six sums per column.
__global__ __launch_bounds__(256) void k_layer1_bwd_part(MlpFwdArgs a, float* part, int rows_per_part) {
  __shared__ float red[4][kMlpIn][64];
  const int mem = blockIdx.z;
  const int c = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + c;   // < 512
  const int r0 = blockIdx.y * rows_per_part, r1 = min(a.valid, r0 + rows_per_part);
  const int* perm = a.perm ? a.perm + (int64_t)mem * a.perm_stride + (int64_t)(*a.step) * a.batch : nullptr;
  float s[kMlpIn] = {0, 0, 0, 0, 0, 0};
  for (int b = r0 + grp; b < r1; b += 4) {
    const int64_t pt = a.base + (perm ? perm[b] : b);
    const float d = (float)a.dz1[(int64_t)mem * a.act_stride + (int64_t)b * kMlpH + n];
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k) s[k] += (a.X[pt * kMlpIn + k] - a.in_shift[k]) * a.in_scale[k] * d;
  }
#pragma unroll
  for (int k = 0; k < kMlpIn; ++k) red[grp][k][c] = s[k];
  __syncthreads();
  if (grp == 0) {
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k)
      part[(((int64_t)mem * gridDim.y + blockIdx.y) * kMlpIn + k) * kMlpH + n] =
          ((red[0][k][c] + red[1][k][c]) + red[2][k][c]) + red[3][k][c];
  }
}

__global__ __launch_bounds__(256) void k_layer1_bwd_fin(float* grads, int64_t gstride, const float* part, int nparts) {
  const int mem = blockIdx.z;
  const int i = blockIdx.x * 256 + threadIdx.x;   // over 6 * 512
  if (i >= kMlpIn * kMlpH) return;
  float s = 0.0f;
  for (int p = 0; p < nparts; ++p) s += part[((int64_t)mem * nparts + p) * kMlpIn * kMlpH + i];
  grads[(int64_t)mem * gstride + kOffW1 + i] = s;
}

hipError_t launch_layer1_bwd(const MlpFwdArgs& a, float* part, int max_parts, float* grads, int64_t gstride,
                             int members, hipStream_t st) {
  const int rows_per_part = kRowsPerPart;
  const int nparts = (a.batch + rows_per_part - 1) / rows_per_part;
  if (nparts > max_parts) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_layer1_bwd_part, dim3(kMlpH / 64, nparts, members), dim3(256), 0, st, a, part,
                     rows_per_part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_layer1_bwd_fin, dim3((kMlpIn * kMlpH + 255) / 256, 1, members), dim3(256), 0, st,
                     grads, gstride, part, nparts);
  return hipGetLastError();
}

// ---- split-K reduction of the weight-gradient product ----------------------
__global__ __launch_bounds__(256) void k_splitk_sum(const float* part, int64_t split_stride, int splits,
                                                    float* out, int64_t out_stride, int64_t n) {
  const int mem = blockIdx.z;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  float s = 0.0f;
  for (int k = 0; k < splits; ++k) s += part[(int64_t)k * split_stride + (int64_t)mem * n + i];
  out[(int64_t)mem * out_stride + i] = s;
}

hipError_t launch_splitk_sum(const float* part, int64_t split_stride, int splits, float* out, int64_t out_stride,
                             int64_t n, int members, hipStream_t st) {
  hipLaunchKernelGGL(k_splitk_sum, dim3((unsigned)((n + 255) / 256), 1, members), dim3(256), 0, st, part,
                     split_stride, splits, out, out_stride, n);
  return hipGetLastError();
}

hipError_t launch_layer1_fwd(const MlpFwdArgs& a, int members, hipStream_t st) {
  if (a.batch % 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_layer1_fwd, dim3(kMlpH / 64, a.batch / 64, members), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_layer4_fwd(const MlpFwdArgs& a, int members, hipStream_t st) {
  hipLaunchKernelGGL(k_layer4_fwd, dim3((a.batch + 3) / 4, 1, members), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_layer4_bwd(const MlpFwdArgs& a, int members, hipStream_t st) {
  if (a.batch % 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_layer4_bwd, dim3(kMlpH / 64, a.batch / 64, members), dim3(256), 0, st, a);
  return hipGetLastError();
}

// ---- Adam (float32 master weights) and the bfloat16 operand copies ---------
// The step number lives on the device (advanced here) so that a captured
// training step replays unchanged.
__global__ __launch_bounds__(256) void k_adam(AdamArgs a) {
  const int mem = blockIdx.z;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int k = *a.step + 1;
  if (i < kMlpParams) {
    const int64_t o = (int64_t)mem * a.pstride + i;
    const float g = a.grads[o];
    const float m = a.b1 * a.m[o] + (1.0f - a.b1) * g;
    const float v = a.b2 * a.v[o] + (1.0f - a.b2) * g * g;
    a.m[o] = m;
    a.v[o] = v;
    const float mh = m / (1.0f - powf(a.b1, (float)k));
    const float vh = v / (1.0f - powf(a.b2, (float)k));
    const float p = a.params[o] - a.lr * mh / (sqrtf(vh) + a.eps);
    a.params[o] = p;
    if (i >= kOffW2 && i < kOffW2 + kMlpH * kMlpH) {
      const int64_t e = i - kOffW2;     // W2[in][out]: copies [in][out] and [out][in]
      a.w2b[(int64_t)mem * kMlpH * kMlpH + e] = (__bf16)p;
      a.w2t[(int64_t)mem * kMlpH * kMlpH + (e % kMlpH) * kMlpH + e / kMlpH] = (__bf16)p;
    } else if (i >= kOffW3 && i < kOffW3 + kMlpH * kMlpH) {
      const int64_t e = i - kOffW3;
      a.w3b[(int64_t)mem * kMlpH * kMlpH + e] = (__bf16)p;
      a.w3t[(int64_t)mem * kMlpH * kMlpH + (e % kMlpH) * kMlpH + e / kMlpH] = (__bf16)p;
    }
  }
}

__global__ __launch_bounds__(64) void k_step_advance(int* step, int* call_step) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *step += 1;
    *call_step += 1;
  }
}

hipError_t launch_adam(const AdamArgs& a, int members, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3((kMlpParams + 255) / 256, 1, members), dim3(256), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(64), 0, st, a.step, a.call_step);
  return hipGetLastError();
}

// bfloat16 copies of W2 and W3 from the float32 master weights
__global__ __launch_bounds__(256) void k_weights_bf16(const float* params, int64_t pstride, __bf16* w2b,
                                                      __bf16* w3b, __bf16* w2t, __bf16* w3t) {
  const int mem = blockIdx.z;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= kMlpH * kMlpH) return;
  const int64_t o = (int64_t)mem * kMlpH * kMlpH, t = (e % kMlpH) * kMlpH + e / kMlpH;
  const __bf16 v2 = (__bf16)params[(int64_t)mem * pstride + kOffW2 + e];
  const __bf16 v3 = (__bf16)params[(int64_t)mem * pstride + kOffW3 + e];
  w2b[o + e] = v2;
  w3b[o + e] = v3;
  w2t[o + t] = v2;
  w3t[o + t] = v3;
}

hipError_t launch_weights_bf16(const float* params, int64_t pstride, __bf16* w2b, __bf16* w3b, __bf16* w2t,
                               __bf16* w3t, int members, hipStream_t st) {
  hipLaunchKernelGGL(k_weights_bf16, dim3(kMlpH * kMlpH / 256, 1, members), dim3(256), 0, st, params, pstride,
                     w2b, w3b, w2t, w3t);
  return hipGetLastError();
}

// ---- ensemble statistics: mean and standard deviation over members ---------
__global__ __launch_bounds__(256) void k_ensemble_stats(const float* y, int64_t y_stride, int members, int n,
                                                        float inv_scale, float* mean, float* sd) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double s = 0.0, s2 = 0.0;
  for (int m = 0; m < members; ++m) {
    const double v = (double)y[(int64_t)m * y_stride + i] * inv_scale;
    s += v;
    s2 += v * v;
  }
  const double mu = s / members;
  const double var = members > 1 ? fmax(s2 / members - mu * mu, 0.0) : 0.0;
  mean[i] = (float)mu;
  sd[i] = (float)sqrt(var);
}

hipError_t launch_ensemble_stats(const float* y, int64_t y_stride, int members, int n, float inv_scale,
                                 float* mean, float* sd, hipStream_t st) {
  hipLaunchKernelGGL(k_ensemble_stats, dim3((n + 255) / 256), dim3(256), 0, st, y, y_stride, members, n,
                     inv_scale, mean, sd);
  return hipGetLastError();
}

}  // namespace msb
