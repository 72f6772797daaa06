// Device helpers shared by the scan kernels (gfx950): coherent tile-state access for the
// look-back, input loads, and the constant-table view.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "ff.h"
#include "launch.h"

namespace mk {
namespace {

// ------------------------------------------------------------ coherent tile-state access
__device__ __forceinline__ void st_u64(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_u64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_f64(double* p, double v) {
  st_u64(reinterpret_cast<uint64_t*>(p), (uint64_t)__double_as_longlong(v));
}
__device__ __forceinline__ double ld_f64(const double* p) {
  return __longlong_as_double((long long)ld_u64(reinterpret_cast<const uint64_t*>(p)));
}
// s_waitcnt vmcnt(0): wait for all of this wave's vector memory operations.
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }
__device__ __forceinline__ void release_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  wait_vmem();
}
__device__ __forceinline__ void acquire_order() {
  wait_vmem();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

struct TileState {
  unsigned char* b;
  int K;
  __device__ uint64_t* flag() const { return reinterpret_cast<uint64_t*>(b); }
  __device__ double* agg(int i, int c) const { return reinterpret_cast<double*>(b + 8) + 2 * i + c; }
  __device__ double* inc(int i, int c) const { return reinterpret_cast<double*>(b + 8) + 2 * K + 2 * i + c; }
  __device__ double* gag(int i, int c) const { return reinterpret_cast<double*>(b + 8) + 4 * K + 2 * i + c; }
};

// ------------------------------------------------------------ input loads
__device__ __forceinline__ float cvt_f16(unsigned short h) {
  return (float)__builtin_bit_cast(_Float16, h);
}
__device__ __forceinline__ float cvt_bf16(unsigned short h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float load1(const void* base, int dtype, int64_t j) {
  if (dtype == 0) return static_cast<const float*>(base)[j];
  const unsigned short h = static_cast<const unsigned short*>(base)[j];
  return dtype == 1 ? cvt_f16(h) : cvt_bf16(h);
}

// v[r] = x[j + r] for r < R, zero outside [0, N).
template <int R>
__device__ __forceinline__ void load_run(const void* base, int dtype, int64_t j, int64_t N, float (&v)[R]) {
  if (j >= 0 && j + R <= N) {
    if (dtype == 0) {
      const float* p = static_cast<const float*>(base) + j;
      if ((reinterpret_cast<uintptr_t>(p) & 15) == 0) {
#pragma unroll
        for (int r = 0; r < R; r += 4) {
          const float4 q = *reinterpret_cast<const float4*>(p + r);
          v[r] = q.x; v[r + 1] = q.y; v[r + 2] = q.z; v[r + 3] = q.w;
        }
      } else if ((reinterpret_cast<uintptr_t>(p) & 7) == 0) {
#pragma unroll
        for (int r = 0; r < R; r += 2) {
          const float2 q = *reinterpret_cast<const float2*>(p + r);
          v[r] = q.x; v[r + 1] = q.y;
        }
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = p[r];
      }
    } else {
      const unsigned short* p = static_cast<const unsigned short*>(base) + j;
      if ((reinterpret_cast<uintptr_t>(p) & 15) == 0) {
#pragma unroll
        for (int r = 0; r < R; r += 8) {
          const uint4 q = *reinterpret_cast<const uint4*>(p + r);
          const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
          for (int h = 0; h < 4; ++h) {
            const unsigned short lo = (unsigned short)(w[h] & 0xffffu), hi = (unsigned short)(w[h] >> 16);
            v[r + 2 * h] = dtype == 1 ? cvt_f16(lo) : cvt_bf16(lo);
            v[r + 2 * h + 1] = dtype == 1 ? cvt_f16(hi) : cvt_bf16(hi);
          }
        }
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = dtype == 1 ? cvt_f16(p[r]) : cvt_bf16(p[r]);
      }
    }
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t q = j + r;
      v[r] = (q >= 0 && q < N) ? load1(base, dtype, q) : 0.0f;
    }
  }
}

// v[r] = p[j + r] (float32), zero outside [0, N)
template <int R>
__device__ __forceinline__ void load_run_f32(const float* p, int64_t j, int64_t N, float (&v)[R]) {
  if (j >= 0 && j + R <= N) {
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = p[j + r];
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = (j + r >= 0 && j + r < N) ? p[j + r] : 0.0f;
  }
}

// (re, im)[r] = p[j + r] (complex64), zero outside [0, N)
template <int R>
__device__ __forceinline__ void load_run_c(const float2* p, int64_t j, int64_t N, float (&re)[R], float (&im)[R]) {
  if (j >= 0 && j + R <= N) {
#pragma unroll
    for (int r = 0; r < R; ++r) { const float2 q = p[j + r]; re[r] = q.x; im[r] = q.y; }
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool in = (j + r >= 0 && j + r < N);
      const float2 q = in ? p[j + r] : make_float2(0.f, 0.f);
      re[r] = q.x; im[r] = q.y;
    }
  }
}

// time-reversed runs: v[r] = p[N - 1 - (j + r)], zero where j + r is outside [0, N)
template <int R>
__device__ __forceinline__ void load_run_rev(const float* p, int64_t j, int64_t N, float (&v)[R]) {
  if (j >= 0 && j + R <= N) {
    const float* q = p + (N - j - R);
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = q[R - 1 - r];
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = (j + r >= 0 && j + r < N) ? p[N - 1 - (j + r)] : 0.0f;
  }
}

template <int R>
__device__ __forceinline__ void load_run_rev_c(const float2* p, int64_t j, int64_t N, float (&re)[R], float (&im)[R]) {
  if (j >= 0 && j + R <= N) {
    const float2* q = p + (N - j - R);
#pragma unroll
    for (int r = 0; r < R; ++r) { const float2 z = q[R - 1 - r]; re[r] = z.x; im[r] = z.y; }
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool in = (j + r >= 0 && j + r < N);
      const float2 z = in ? p[N - 1 - (j + r)] : make_float2(0.f, 0.f);
      re[r] = z.x; im[r] = z.y;
    }
  }
}

// ------------------------------------------------------------ four-sample loads
// v[r] = x[j + r], r < 4, zero outside [0, N); 16-byte (8-byte for 16-bit types) loads
// when the quad is inside the signal and aligned
__device__ __forceinline__ void load4(const void* base, int dtype, int64_t j, int64_t N, float (&v)[4]) {
  if (j >= 0 && j + 4 <= N) {
    if (dtype == 0) {
      const float* p = static_cast<const float*>(base) + j;
      if ((reinterpret_cast<uintptr_t>(p) & 15) == 0) {
        const float4 q = *reinterpret_cast<const float4*>(p);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = p[r];
      }
    } else {
      const unsigned short* p = static_cast<const unsigned short*>(base) + j;
      uint32_t w0, w1;
      if ((reinterpret_cast<uintptr_t>(p) & 7) == 0) {
        const uint2 q = *reinterpret_cast<const uint2*>(p);
        w0 = q.x; w1 = q.y;
      } else {
        w0 = (uint32_t)p[0] | ((uint32_t)p[1] << 16);
        w1 = (uint32_t)p[2] | ((uint32_t)p[3] << 16);
      }
      const unsigned short h[4] = {(unsigned short)(w0 & 0xffffu), (unsigned short)(w0 >> 16),
                                   (unsigned short)(w1 & 0xffffu), (unsigned short)(w1 >> 16)};
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] = dtype == 1 ? cvt_f16(h[r]) : cvt_bf16(h[r]);
    }
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = (j + r >= 0 && j + r < N) ? load1(base, dtype, j + r) : 0.0f;
  }
}

__device__ __forceinline__ void load4_f32(const float* p, int64_t j, int64_t N, float (&v)[4]) {
  if (j >= 0 && j + 4 <= N && (reinterpret_cast<uintptr_t>(p + j) & 15) == 0) {
    const float4 q = *reinterpret_cast<const float4*>(p + j);
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = (j + r >= 0 && j + r < N) ? p[j + r] : 0.0f;
  }
}

__device__ __forceinline__ void load4_c(const float2* p, int64_t j, int64_t N, float (&re)[4], float (&im)[4]) {
  if (j >= 0 && j + 4 <= N && (reinterpret_cast<uintptr_t>(p + j) & 15) == 0) {
    const float4 a = *reinterpret_cast<const float4*>(p + j), b = *reinterpret_cast<const float4*>(p + j + 2);
    re[0] = a.x; im[0] = a.y; re[1] = a.z; im[1] = a.w; re[2] = b.x; im[2] = b.y; re[3] = b.z; im[3] = b.w;
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const bool in = j + r >= 0 && j + r < N;
      const float2 z = in ? p[j + r] : make_float2(0.f, 0.f);
      re[r] = z.x; im[r] = z.y;
    }
  }
}

// unchecked quads (the caller has checked range and alignment)
template <int DT>
__device__ __forceinline__ void ld4_fast(const void* base, int64_t j, float (&v)[4]) {
  if constexpr (DT == 0) {
    const float4 q = *reinterpret_cast<const float4*>(static_cast<const float*>(base) + j);
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
  } else {
    const uint2 q = *reinterpret_cast<const uint2*>(static_cast<const unsigned short*>(base) + j);
    const unsigned short h[4] = {(unsigned short)(q.x & 0xffffu), (unsigned short)(q.x >> 16),
                                 (unsigned short)(q.y & 0xffffu), (unsigned short)(q.y >> 16)};
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = DT == 1 ? cvt_f16(h[r]) : cvt_bf16(h[r]);
  }
}

__device__ __forceinline__ void ld4_rev_fast(const float* p, int64_t N, int64_t j, float (&v)[4]) {
  const float4 q = *reinterpret_cast<const float4*>(p + (N - 4 - j));
  v[0] = q.w; v[1] = q.z; v[2] = q.y; v[3] = q.x;
}

__device__ __forceinline__ void ld4c_rev_fast(const float2* p, int64_t N, int64_t j, float (&re)[4], float (&im)[4]) {
  const float2* q = p + (N - 4 - j);
  const float4 a = *reinterpret_cast<const float4*>(q), b = *reinterpret_cast<const float4*>(q + 2);
  re[3] = a.x; im[3] = a.y; re[2] = a.z; im[2] = a.w; re[1] = b.x; im[1] = b.y; re[0] = b.z; im[0] = b.w;
}

// time-reversed quads: v[r] = p[N - 1 - (j + r)], zero where j + r is outside [0, N)
__device__ __forceinline__ void load4_rev(const float* p, int64_t j, int64_t N, float (&v)[4]) {
  float t[4];
  load4_f32(p, N - 4 - j, N, t);   // covers indices N-4-j .. N-1-j, i.e. j+3 .. j reversed
#pragma unroll
  for (int r = 0; r < 4; ++r) v[r] = t[3 - r];
}

__device__ __forceinline__ void load4_rev_c(const float2* p, int64_t j, int64_t N, float (&re)[4], float (&im)[4]) {
  float tr[4], ti[4];
  load4_c(p, N - 4 - j, N, tr, ti);
#pragma unroll
  for (int r = 0; r < 4; ++r) { re[r] = tr[3 - r]; im[r] = ti[3 - r]; }
}

// LDS writes of this wave are visible to its other lanes after this (single-wave exchange)
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
}

// ------------------------------------------------------------ constant table access
// Table reads go through the constant address space: uniform indices become scalar loads
// into SGPRs instead of occupying vector registers.
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;

// A view of one scale's table in the arithmetic T of a kernel: float32 or float64 entries,
// or for float-float arithmetic the float32 entries and their float32 remainders (the third
// section of the table) taken as one value.
template <typename T>
struct TabT {
  cptr<T> p;
  int K;
  __device__ T re(int e, int i) const { return p[(2 * e) * K + i]; }
  __device__ T im(int e, int i) const { return p[(2 * e + 1) * K + i]; }
  __device__ T row(int rrow, int i) const { return p[rrow * K + i]; }
  __device__ T scalar(int s) const { return p[s]; }
};
template <>
struct TabT<ff> {
  cptr<float> h, l;
  int K;
  __device__ ff at(int k) const { return ff(h[k], l[k]); }
  __device__ ff re(int e, int i) const { return at((2 * e) * K + i); }
  __device__ ff im(int e, int i) const { return at((2 * e + 1) * K + i); }
  __device__ ff row(int rrow, int i) const { return at(rrow * K + i); }
  __device__ ff scalar(int s) const { return at(s); }
};
template <bool WIDE>
using Tab = TabT<typename std::conditional<WIDE, double, float>::type>;

// The view of the table at tb (float32 section, float64 section at f64_off, float32
// remainders after it) in arithmetic T.
template <typename T>
__device__ __forceinline__ TabT<T> tab_view(const unsigned char* tb, int64_t f64_off, const TabLayout& lay) {
  if constexpr (std::is_same<T, ff>::value) {
    return TabT<ff>{(cptr<float>)tb, (cptr<float>)(tb + f64_off + (int64_t)lay.f64Bytes()), lay.K};
  } else if constexpr (std::is_same<T, double>::value) {
    return TabT<double>{(cptr<double>)(tb + f64_off), lay.K};
  } else {
    return TabT<float>{(cptr<float>)tb, lay.K};
  }
}

}  // namespace
}  // namespace mk
