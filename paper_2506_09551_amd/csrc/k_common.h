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

// Coherent (agent-scope) load used when reading partial sums written by other
// workgroups of the same launch.
__device__ __forceinline__ double coherent_load(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Block-wide sum of NV values into thread 0 (deterministic order).
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*sh)[kBlock / kWave]) {
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
      for (int w = 0; w < kBlock / kWave; ++w) t += sh[i][w];
      v[i] = t;
    }
  }
  __syncthreads();
}

// Every workgroup of system `s` (workgroups bx < nbx of that system)
// contributes NV partial sums.  The workgroup that finishes last for that
// system -- detected with a per-system counter -- sums the system's partials
// in index order (the result does not depend on scheduling), writes
// red[s][0..NV) and out_sh[0..NV) (shared memory of the calling block), resets
// the counter and returns true.  Must be called by all threads of every
// workgroup of the launch.
template <int NV>
__device__ bool publish_partials(double (&v)[NV], double* partials, unsigned* counters,
                                 double* red, int nbx, int s, int bx, double* out_sh = nullptr) {
  __shared__ double sh[NV][kBlock / kWave];
  __shared__ int s_last;
  block_sum<NV>(v, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) partials[((int64_t)s * nbx + bx) * 4 + i] = v[i];
    __threadfence();
    const unsigned t = atomicAdd(&counters[s], 1u);
    s_last = (t == (unsigned)nbx - 1u) ? 1 : 0;
  }
  __syncthreads();
  if (!s_last) return false;
  __threadfence();
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  for (int j = threadIdx.x; j < nbx; j += kBlock) {
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] += coherent_load(&partials[((int64_t)s * nbx + j) * 4 + i]);
  }
  block_sum<NV>(acc, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      if (red) red[s * 4 + i] = acc[i];
      if (out_sh) out_sh[i] = acc[i];
    }
    __hip_atomic_store(&counters[s], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
  }
  __syncthreads();
  return true;
}

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
