// Small element-wise kernels: the diagonal site operators O1 / O2, the
// coherent site sum with momentum phases, and bank slot copies.
#include "k_common.h"

namespace msb {

__device__ __forceinline__ double site_weight(const TablesDev& T, int64_t i, int site, double w_up,
                                              double w_dn) {
  if (site < 0) return 1.0;
  const int u = (int)(i / T.n_dn), d = (int)(i % T.n_dn);
  return w_up * (double)((T.conf_up[u] >> site) & 1u) + w_dn * (double)((T.conf_dn[d] >> site) & 1u);
}

__global__ __launch_bounds__(kBlock) void k_number_op(TablesDev T, int64_t D, int site, double w_up,
                                                      double w_dn, int x_real, const void* x,
                                                      double* y) {
  const int c = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= D) return;
  const double wgt = site_weight(T, i, site, w_up, w_dn);
  cv<double> v;
  if (x_real) v = Access<double, false>::template load<double>(x, (int64_t)c * D + i);
  else v = Access<double, true>::template load<double>(x, (int64_t)c * D + i);
  v.re *= wgt;
  v.im *= wgt;
  Access<double, true>::store(y, (int64_t)c * D + i, v);
}

hipError_t launch_number_op(const TablesDev& T, int64_t D, int site, double w_up, double w_dn,
                            int count, int x_real, const void* x, double* y, hipStream_t st) {
  const int nb = (int)((D + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_number_op, dim3(nb, count), dim3(kBlock), 0, st, T, D, site, w_up, w_dn,
                     x_real, x, y);
  return hipGetLastError();
}

// phi[k][i] = sum_s (phase_s * O1_s(i)) psi[s][k][i]
template <typename S>
__global__ __launch_bounds__(kBlock) void k_combine(TablesDev T, int64_t D, int nsys, int n,
                                                    const void* psi, const double* coef,
                                                    const int* site, double* phi) {
  const int k = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= D) return;
  cv<double> acc = {0.0, 0.0};
  for (int s = 0; s < nsys; ++s) {
    const double wgt = site_weight(T, i, site[s], coef[4 * s + 2], coef[4 * s + 3]);
    const cv<double> ph = {coef[4 * s] * wgt, coef[4 * s + 1] * wgt};
    const cv<double> v = Access<S, true>::template load<double>(psi, ((int64_t)s * n + k) * D + i);
    acc = cadd(acc, cmul(ph, v));
  }
  Access<double, true>::store(phi, (int64_t)k * D + i, acc);
}

hipError_t launch_combine(const TablesDev& T, int64_t D, int nsys, int n, Elem e, const void* psi,
                          const double* coef, const int* site, double* phi, hipStream_t st) {
  const int nb = (int)((D + kBlock - 1) / kBlock);
  if (e == Elem::C128)
    hipLaunchKernelGGL(k_combine<double>, dim3(nb, n), dim3(kBlock), 0, st, T, D, nsys, n, psi,
                       coef, site, phi);
  else if (e == Elem::C64)
    hipLaunchKernelGGL(k_combine<float>, dim3(nb, n), dim3(kBlock), 0, st, T, D, nsys, n, psi,
                       coef, site, phi);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// dst[s][i] = src[s][i] for s < nsys (strides in elements)
template <typename S>
__global__ __launch_bounds__(kBlock) void k_copy_slot(const void* src, void* dst, int64_t D,
                                                      int64_t src_stride, int64_t dst_stride) {
  using Ax = Access<S, true>;
  const int s = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= D) return;
  const cv<double> v = Ax::template load<double>(src, (int64_t)s * src_stride + i);
  Ax::store(dst, (int64_t)s * dst_stride + i, v);
}

hipError_t launch_copy_slot(Elem e, const void* src, void* dst, int64_t D, int nsys,
                            int64_t src_stride, int64_t dst_stride, hipStream_t st) {
  const int nb = (int)((D + kBlock - 1) / kBlock);
  if (e == Elem::C128)
    hipLaunchKernelGGL(k_copy_slot<double>, dim3(nb, nsys), dim3(kBlock), 0, st, src, dst, D,
                       src_stride, dst_stride);
  else if (e == Elem::C64)
    hipLaunchKernelGGL(k_copy_slot<float>, dim3(nb, nsys), dim3(kBlock), 0, st, src, dst, D,
                       src_stride, dst_stride);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// red[s][0..4) = sum over workgroups of partials[s][bx][0..4)
__global__ __launch_bounds__(kBlock) void k_reduce(const double* partials, int nbx, double* red) {
  const int s = blockIdx.x;
  __shared__ double out[4];
  reduce_partials<4>(partials, nbx, s, out);
  if (threadIdx.x < 4) red[s * 4 + threadIdx.x] = out[threadIdx.x];
}

hipError_t launch_reduce(const double* partials, int nbx, int nsys, double* red, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce, dim3(nsys), dim3(kBlock), 0, st, partials, nbx, red);
  return hipGetLastError();
}

}  // namespace msb
