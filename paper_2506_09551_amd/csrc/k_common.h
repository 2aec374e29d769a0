// Device helpers shared by the HIP kernels: complex arithmetic, typed vector
// loads/stores and the deterministic last-block reduction.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "msb_internal.h"

namespace msb {

template <typename T>
struct cv {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cv<T> cmul(cv<T> a, cv<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cv<T> cadd(cv<T> a, cv<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cv<T> csub(cv<T> a, cv<T> b) { return {a.re - b.re, a.im - b.im}; }
// a / b computed as a * conj(b) / |b|^2
__device__ __forceinline__ cv<double> cdiv(cv<double> a, cv<double> b) {
  const double d = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
__device__ __forceinline__ double cabs(cv<double> a) { return hypot(a.re, a.im); }

// Typed element access.  S = storage scalar (double / float); CPLX selects
// interleaved complex storage.  Values are returned in compute type Tc.
template <typename S, bool CPLX>
struct Access {
  using V2 = typename std::conditional<std::is_same<S, double>::value, double2, float2>::type;
  template <typename Tc>
  static __device__ __forceinline__ cv<Tc> load(const void* base, int64_t i) {
    if constexpr (CPLX) {
      const V2 t = reinterpret_cast<const V2*>(base)[i];
      return {(Tc)t.x, (Tc)t.y};
    } else {
      return {(Tc) reinterpret_cast<const S*>(base)[i], (Tc)0};
    }
  }
  template <typename Tc>
  static __device__ __forceinline__ void store(void* base, int64_t i, cv<Tc> v) {
    if constexpr (CPLX) {
      V2 t;
      t.x = (S)v.re;
      t.y = (S)v.im;
      reinterpret_cast<V2*>(base)[i] = t;
    } else {
      reinterpret_cast<S*>(base)[i] = (S)v.re;
    }
  }
  // Streaming variants (non-temporal hint): for data touched once, so that it
  // does not evict the re-read neighbour rows from the caches.
  using N2 = S __attribute__((ext_vector_type(2)));
  template <typename Tc>
  static __device__ __forceinline__ cv<Tc> load_nt(const void* base, int64_t i) {
    if constexpr (CPLX) {
      const N2 t = __builtin_nontemporal_load(reinterpret_cast<const N2*>(base) + i);
      return {(Tc)t.x, (Tc)t.y};
    } else {
      return {(Tc)__builtin_nontemporal_load(reinterpret_cast<const S*>(base) + i), (Tc)0};
    }
  }
  template <typename Tc>
  static __device__ __forceinline__ void store_nt(void* base, int64_t i, cv<Tc> v) {
    if constexpr (CPLX) {
      N2 t;
      t.x = (S)v.re;
      t.y = (S)v.im;
      __builtin_nontemporal_store(t, reinterpret_cast<N2*>(base) + i);
    } else {
      __builtin_nontemporal_store((S)v.re, reinterpret_cast<S*>(base) + i);
    }
  }
  static constexpr int64_t kBytes = (int64_t)sizeof(S) * (CPLX ? 2 : 1);
  static __device__ __forceinline__ const void* offset(const void* base, int64_t elems) {
    return reinterpret_cast<const char*>(base) + elems * kBytes;
  }
  static __device__ __forceinline__ void* offset(void* base, int64_t elems) {
    return reinterpret_cast<char*>(base) + elems * kBytes;
  }
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Block-wide sum of NV values into thread 0 (deterministic order).
template <int NV, int BLK = kBlock>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*sh)[BLK / kWave]) {
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) sh[i][wave] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double t = 0.0;
      for (int w = 0; w < BLK / kWave; ++w) t += sh[i][w];
      v[i] = t;
    }
  }
  __syncthreads();
}

// Cross-workgroup reductions are done in two launches: every workgroup of
// system s writes its NV partial sums to partials[s][bx][0..NV) (block_partial),
// and a following finalize launch with one workgroup per system sums them in
// index order (reduce_partials), so the result does not depend on scheduling.
// Device-scope atomics and fences are avoided on purpose: on MI355X they
// serialise across the whole device (about 50 ns each).
template <int NV>
__device__ __forceinline__ void block_partial(double (&v)[NV], double* partials, int nbx, int s,
                                              int bx) {
  __shared__ double sh[NV][kBlock / kWave];
  block_sum<NV>(v, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) partials[((int64_t)s * nbx + bx) * 4 + i] = v[i];
  }
}

// Sum of system s's partials into out[0..NV) (shared memory, all threads see it on return).
template <int NV>
__device__ __forceinline__ void reduce_partials(const double* partials, int nbx, int s,
                                                double* out) {
  __shared__ double sh[NV][kBlock / kWave];
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  for (int j = threadIdx.x; j < nbx; j += kBlock) {
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] += partials[((int64_t)s * nbx + j) * 4 + i];
  }
  block_sum<NV>(acc, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) out[i] = acc[i];
  }
  __syncthreads();
}

// Generic finalize: red[s][0..4) = sum_bx partials[s][bx][0..4), one workgroup per system.
hipError_t launch_reduce(const double* partials, int nbx, int nsys, double* red, hipStream_t st);

// Number of workgroups per system for the streaming kernels: about 2048
// workgroups in flight over the whole launch, each walking its share of the
// vector in steps of `per_block` elements.
inline int stream_nbx(int64_t D, int nsys, int per_block) {
  const int64_t need = (D + per_block - 1) / per_block;
  int64_t want = (2048 + nsys - 1) / nsys;
  if (want < 1) want = 1;
  return (int)(need < want ? need : want);
}

}  // namespace msb
