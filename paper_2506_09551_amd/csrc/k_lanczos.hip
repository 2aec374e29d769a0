// Lanczos building blocks: the FP64 ground-state Lanczos with full
// reorthogonalisation (the ground state is the precondition of Eq.
// intermediateState) and the block of independent complex Lanczos
// recurrences whose continued fractions give Eq. kramers1.
#include "k_common.h"

namespace msb {

constexpr int kEptL = 4;
constexpr int kPerStepL = kBlock * kEptL;
constexpr int kGramChunk = 2048;     // elements of w staged in LDS per workgroup

int gram_blocks(int64_t D) { return (int)((D + kGramChunk - 1) / kGramChunk); }

// part[i][b] = sum_{e in chunk b} Q[i][e] w[e]  (one wavefront per vector i)
__global__ __launch_bounds__(kBlock) void k_gram_partial(const double* Q, const double* w, int64_t D,
                                                         int k, int nb, double* part) {
  __shared__ double ws[kGramChunk];
  const int b = blockIdx.x;
  const int64_t e0 = (int64_t)b * kGramChunk;
  for (int j = threadIdx.x; j < kGramChunk; j += kBlock)
    ws[j] = (e0 + j < D) ? w[e0 + j] : 0.0;
  __syncthreads();
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int n = (int)((D - e0) < kGramChunk ? (D - e0) : kGramChunk);
  for (int i = wave; i < k; i += kBlock / kWave) {
    const double* q = Q + (int64_t)i * D + e0;
    double acc = 0.0;
    for (int j = lane; j < n; j += kWave) acc = fma(q[j], ws[j], acc);
    acc = wave_sum(acc);
    if (lane == 0) part[(int64_t)i * nb + b] = acc;
  }
}

// out[4 i] = sum_b part[i][b]   (one workgroup per vector, fixed order)
__global__ __launch_bounds__(kBlock) void k_gram_reduce(const double* part, int nb, double* out) {
  __shared__ double sh[1][kBlock / kWave];
  const int i = blockIdx.x;
  double acc[1] = {0.0};
  for (int b = threadIdx.x; b < nb; b += kBlock) acc[0] += part[(int64_t)i * nb + b];
  block_sum<1>(acc, sh);
  if (threadIdx.x == 0) out[4 * i] = acc[0];
}

// c_i = sum_e Q[i][e] w[e], i < k, into out[4 i]; partials: [k][gram_blocks(D)]
hipError_t launch_dot_many(const double* Q, int k, const double* w, int64_t D, double* partials,
                           double* out, hipStream_t st) {
  const int nb = gram_blocks(D);
  hipLaunchKernelGGL(k_gram_partial, dim3(nb), dim3(kBlock), 0, st, Q, w, D, k, nb, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gram_reduce, dim3(k), dim3(kBlock), 0, st, partials, nb, out);
  return hipGetLastError();
}

// w[e] -= sum_i c_i Q[i][e]   (c: device, stride 4 as written by the reductions)
__global__ __launch_bounds__(kBlock) void k_gemv_sub(const double* Q, int k, const double* c,
                                                     double* w, int64_t D) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= D) return;
  double acc = 0.0;
  for (int i = 0; i < k; ++i) acc = fma(c[4 * i], Q[(int64_t)i * D + j], acc);
  w[j] -= acc;
}
hipError_t launch_gemv_sub(const double* Q, int k, const double* c, double* w, int64_t D,
                           hipStream_t st) {
  const int nb = (int)((D + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_gemv_sub, dim3(nb), dim3(kBlock), 0, st, Q, k, c, w, D);
  return hipGetLastError();
}

// out[e] = sum_i c_i Q[i][e]  (c: device, dense)
__global__ __launch_bounds__(kBlock) void k_gemv(const double* Q, int k, const double* c,
                                                 double* out, int64_t D) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= D) return;
  double acc = 0.0;
  for (int i = 0; i < k; ++i) acc = fma(c[i], Q[(int64_t)i * D + j], acc);
  out[j] = acc;
}
hipError_t launch_gemv(const double* Q, int k, const double* c, double* out, int64_t D,
                       hipStream_t st) {
  const int nb = (int)((D + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_gemv, dim3(nb), dim3(kBlock), 0, st, Q, k, c, out, D);
  return hipGetLastError();
}

// w -= a q + b qprev (ab = device {a, b}); partial |w|^2
__global__ __launch_bounds__(kBlock) void k_lanczos_real_update(double* w, const double* q,
                                                                const double* qprev,
                                                                const double* ab, int64_t D,
                                                                int nbx, double* partials) {
  const int bx = blockIdx.x;
  const double a = ab[0], b = ab[1];
  double part[1] = {0.0};
  for (int64_t base = (int64_t)bx * kPerStepL; base < D; base += (int64_t)nbx * kPerStepL) {
#pragma unroll
    for (int e = 0; e < kEptL; ++e) {
      const int64_t j = base + e * kBlock + threadIdx.x;
      if (j < D) {
        double x = w[j] - a * q[j];
        if (qprev) x -= b * qprev[j];
        w[j] = x;
        part[0] = fma(x, x, part[0]);
      }
    }
  }
  block_partial<1>(part, partials, nbx, 0, bx);
}
hipError_t launch_lanczos_real_update(double* w, const double* q, const double* qprev,
                                      const double* ab, int64_t D, double* partials,
                                      double* out, hipStream_t st) {
  const int nbx = stream_nbx(D, 1, kPerStepL);
  hipLaunchKernelGGL(k_lanczos_real_update, dim3(nbx), dim3(kBlock), 0, st, w, q, qprev, ab, D,
                     nbx, partials);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  return launch_reduce(partials, nbx, 1, out, st);
}

// q = w * s[0]
__global__ __launch_bounds__(kBlock) void k_scale_real(const double* w, const double* s, double* q,
                                                       int64_t D) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j < D) q[j] = w[j] * s[0];
}
hipError_t launch_scale_real(const double* w, const double* s, double* q, int64_t D,
                             hipStream_t st) {
  const int nb = (int)((D + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_scale_real, dim3(nb), dim3(kBlock), 0, st, w, s, q, D);
  return hipGetLastError();
}

// ---- block of complex Lanczos recurrences (continued fraction) -------------
// w_j -= a_j q_j + b_j qprev_j, partial |w_j|^2 for active j
__global__ __launch_bounds__(kBlock) void k_block_lanczos_update(BlockLanczosArgs a) {
  using Ax = Access<double, true>;
  const int j = blockIdx.y, bx = blockIdx.x;
  double part[1] = {0.0};
  if (a.active[j] == 0) {
    const double aj = a.a[4 * j];
    const double bj = a.b[j];
    const int64_t off = (int64_t)j * a.D;
    for (int64_t base = (int64_t)bx * kPerStepL; base < a.D; base += (int64_t)a.nbx * kPerStepL) {
#pragma unroll
      for (int e = 0; e < kEptL; ++e) {
        const int64_t i = base + e * kBlock + threadIdx.x;
        if (i < a.D) {
          cv<double> x = Ax::template load<double>(a.w, off + i);
          const cv<double> q = Ax::template load<double>(a.q, off + i);
          const cv<double> qp = Ax::template load<double>(a.qprev, off + i);
          x.re -= aj * q.re + bj * qp.re;
          x.im -= aj * q.im + bj * qp.im;
          Ax::store(a.w, off + i, x);
          part[0] += x.re * x.re + x.im * x.im;
        }
      }
    }
  }
  block_partial<1>(part, a.partials, a.nbx, j, bx);
}
hipError_t launch_block_lanczos_update(const BlockLanczosArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_block_lanczos_update, dim3(a.nbx, a.n), dim3(kBlock), 0, st, a);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  return launch_reduce(a.partials, a.nbx, a.n, a.red, st);
}
int lanczos_nbx(int64_t D, int n) { return stream_nbx(D, n, kPerStepL); }

// One step of the block recurrence on unnormalised Lanczos vectors u_k
// (q_k = u_k / beta_k, beta_k^2 = nrm[j]):
//   a_k = <u_k|H u_k> / beta_k^2,
//   u_{k+1} = v / beta_k - (a_k / beta_k) u_k - (beta_k / beta_{k-1}) u_{k-1},  v = H u_k,
// written over u_{k-1}; partial |u_{k+1}|^2.  Keeping the vectors unnormalised
// removes the separate scaling pass (6 instead of 8 vector passes per step).
__global__ __launch_bounds__(kBlock) void k_block_lanczos_step(BlockStepArgs a) {
  using Ax = Access<double, true>;
  const int j = blockIdx.y, bx = blockIdx.x;
  double part[1] = {0.0};
  if (a.active[j] == 0) {
    const double nrm = a.nrm[j];
    const double inv_b = 1.0 / sqrt(nrm);
    const double ca = a.herm[4 * j] / nrm * inv_b;
    const double bp = a.bprev[j];
    const double cp = bp > 0.0 ? sqrt(nrm) / bp : 0.0;
    const int64_t off = (int64_t)j * a.D;
    for (int64_t base = (int64_t)bx * kPerStepL; base < a.D; base += (int64_t)a.nbx * kPerStepL) {
#pragma unroll
      for (int e = 0; e < kEptL; ++e) {
        const int64_t i = base + e * kBlock + threadIdx.x;
        if (i < a.D) {
          const cv<double> v = Ax::template load_nt<double>(a.v, off + i);
          const cv<double> u = Ax::template load<double>(a.u, off + i);
          cv<double> x = {v.re * inv_b - ca * u.re, v.im * inv_b - ca * u.im};
          if (cp != 0.0) {
            const cv<double> up = Ax::template load<double>(a.up, off + i);
            x.re -= cp * up.re;
            x.im -= cp * up.im;
          }
          Ax::store(a.up, off + i, x);
          part[0] += x.re * x.re + x.im * x.im;
        }
      }
    }
  }
  block_partial<1>(part, a.partials, a.nbx, j, bx);
}

// beta_{k-1} <- beta_k, beta_k^2 <- |u_{k+1}|^2 for active vectors
__global__ __launch_bounds__(kBlock) void k_block_lanczos_rotate(const int* active, const double* red,
                                                                 double* nrm, double* bprev, int n) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= n || active[j] != 0) return;
  bprev[j] = sqrt(nrm[j]);
  nrm[j] = red[4 * j];
}

hipError_t launch_block_lanczos_step(const BlockStepArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_block_lanczos_step, dim3(a.nbx, a.n), dim3(kBlock), 0, st, a);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  err = launch_reduce(a.partials, a.nbx, a.n, a.red, st);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_block_lanczos_rotate, dim3((a.n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, a.active,
                     a.red, a.nrm, a.bprev, a.n);
  return hipGetLastError();
}

// out_j = w_j / b_j for active j
__global__ __launch_bounds__(kBlock) void k_block_scale(const double* w, const double* b,
                                                        const int* active, double* out, int64_t D) {
  using Ax = Access<double, true>;
  const int j = blockIdx.y;
  if (active[j] != 0) return;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= D) return;
  const double inv = 1.0 / b[j];
  cv<double> x = Ax::template load<double>(w, (int64_t)j * D + i);
  x.re *= inv;
  x.im *= inv;
  Ax::store(out, (int64_t)j * D + i, x);
}
hipError_t launch_block_scale(const double* w, const double* b, const int* active, double* out,
                              int64_t D, int n, hipStream_t st) {
  const int nb = (int)((D + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_block_scale, dim3(nb, n), dim3(kBlock), 0, st, w, b, active, out, D);
  return hipGetLastError();
}

// I[j][i] = -(1/pi) Im G_j(E_G + w_i + i eta),
// G_j(z) = norm2_j / (z - a_0 - b_1^2 / (z - a_1 - ... b_{d-1}^2 / (z - a_{d-1}))),
// a = a_log[j][0..d), b = b_log[j][1..d) (b_log[j][0] unused), d = depth[j].
__global__ __launch_bounds__(kBlock) void k_cf_eval(const double* a, const double* b,
                                                    const int* depth, int ld, const double* norm2,
                                                    int n, const double* w, int n_w, double E_G,
                                                    double eta, double* I) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= n * n_w) return;
  const int j = t / n_w, i = t % n_w;
  const int d = depth[j];
  const double zr = E_G + w[i], zi = eta;
  const double* aj = a + (int64_t)j * ld;
  const double* bj = b + (int64_t)j * ld;
  double gr = 0.0, gi = 0.0;                // g = 1 / (z - a_k - b_{k+1}^2 g)
  for (int k = d - 1; k >= 0; --k) {
    const double b2 = (k + 1 < d) ? bj[k + 1] * bj[k + 1] : 0.0;
    const double dr = zr - aj[k] - b2 * gr;
    const double di = zi - b2 * gi;
    const double den = dr * dr + di * di;
    gr = dr / den;
    gi = -di / den;
  }
  I[t] = -norm2[j] * gi / M_PI;
}
hipError_t launch_cf_eval(const double* a, const double* b, const int* depth, int ld,
                          const double* norm2, int n, const double* w, int n_w, double E_G,
                          double eta, double* I, hipStream_t st) {
  const int total = n * n_w;
  const int nb = (total + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_cf_eval, dim3(nb), dim3(kBlock), 0, st, a, b, depth, ld, norm2, n, w, n_w,
                     E_G, eta, I);
  return hipGetLastError();
}

}  // namespace msb
