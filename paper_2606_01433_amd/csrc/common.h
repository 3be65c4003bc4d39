// Shared definitions of the HIP library: error handling, launch helpers and
// wave64 reductions for CDNA4 (gfx950).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>

namespace gdsw {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& msg) : std::runtime_error(msg), code(c) {}
};

#define GDSW_HIP(expr)                                                                        \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) {                                                                   \
      int code_ = (e_ == hipErrorOutOfMemory) ? -3 : -4;                                      \
      throw ::gdsw::Error(code_, std::string(#expr) + ": " + hipGetErrorString(e_) + " (" +   \
                                     __FILE__ + ":" + std::to_string(__LINE__) + ")");        \
    }                                                                                         \
  } while (0)

#define GDSW_LAUNCH_CHECK() GDSW_HIP(hipGetLastError())

constexpr int WAVE = 64;

inline unsigned blocks_for(int64_t n, int per_block) {
  return (unsigned)((n + per_block - 1) / per_block);
}

// Fixed-shape butterfly sum over the 64 lanes of a wavefront (deterministic).
// Load of data read once per pass (factor, operator and basis streams): a
// nontemporal hint, so the stream does not displace what the caches hold for
// reuse.  Same value as a plain load.
template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
  return __builtin_nontemporal_load(p);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

// Value of v held by lane l (l wave-uniform), via v_readlane.
__device__ __forceinline__ double lane_value(double v, int l) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float lane_value(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ __forceinline__ int lane_value(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

// Workgroups of a 1-D grid are dispatched round-robin over the 8 XCDs (each
// with its own L2).  xcd_remap(b, G) maps hardware workgroup b to a logical
// index so that every XCD receives one contiguous range of logical indices:
// neighbouring tiles (same matrix, shared operand panels) then share an L2.
constexpr int NUM_XCD = 8;
__device__ __forceinline__ unsigned xcd_remap(unsigned b, unsigned G) {
  const unsigned x = b % NUM_XCD, j = b / NUM_XCD;
  const unsigned q = G / NUM_XCD, r = G % NUM_XCD;
  return x * q + (x < r ? x : r) + j;
}

// Leading dimension of a dense column-major block of order n whose columns are
// padded to a multiple of `pad` rows (pad <= 1: none).  Padding to 128 bytes
// keeps every 64-row panel boundary on a cache-line boundary.
__host__ __device__ __forceinline__ int lead_dim(int n, int pad) { return pad > 1 ? (n + pad - 1) / pad * pad : n; }

// Lower bound of `key` in the sorted array a[0..n).
__device__ __forceinline__ int lower_bound_i32(const int* a, int n, int key) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Index of the segment of ptr[0..nseg] (non-decreasing, ptr[0] = 0) holding position k.
__device__ __forceinline__ int segment_of(const int64_t* ptr, int nseg, int64_t k) {
  int lo = 0, hi = nseg;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (ptr[mid] <= k) lo = mid;
    else hi = mid;
  }
  return lo;
}

}  // namespace gdsw
