// Device-side helpers shared by the gfx950 kernels of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hd {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kWave = 64;        // CDNA wavefront width
constexpr int kBlock = 256;      // threads per block in every kernel (4 waves)

// Solver vectors (N x ldb) are node-major: element (i, b) at i * ldb + b, so
// the ldb query columns of one item are one contiguous row (a neighbour
// gather in the SpMM is one coalesced 4*ldb-byte load).
__host__ __device__ __forceinline__ size_t vec_index(int64_t N, int ldb, int64_t i, int b) {
    (void)N;
    return (size_t)i * (size_t)ldb + (size_t)b;
}

// Workgroups of a launch are dealt round-robin to the eight XCDs of the chip
// (block b to XCD b % 8), and each XCD has its own L2. xcd_tile() turns the
// hardware block id of a 1-D launch into a logical tile id such that every
// XCD works through one contiguous range of logical ids. Kernels number
// their tiles so that tiles sharing an operand are neighbours; those then run
// on one XCD and share the operand through its L2 instead of each XCD
// fetching it from memory.
constexpr unsigned kXcd = 8;
__device__ __forceinline__ unsigned xcd_tile() {
    const unsigned h = blockIdx.x, n = gridDim.x;
    const unsigned x = h % kXcd, slot = h / kXcd, q = n / kXcd, rem = n % kXcd;
    return x * q + (x < rem ? x : rem) + slot;
}

// Broadcast lane `lane` (wave-uniform) of v to the whole wavefront.
__device__ __forceinline__ int bcast_i(int v, int lane) {
    return __builtin_amdgcn_readlane(v, lane);
}
__device__ __forceinline__ float bcast_f(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Monotone map float -> uint32: a > b (as floats, no NaN) iff key(a) > key(b).
__device__ __forceinline__ uint32_t float_order_key(float x) {
    uint32_t u = __float_as_uint(x);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float float_from_order_key(uint32_t k) {
    uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(u);
}

// 64-bit ranking key: larger score first, and for equal scores the lower id
// first (the id is stored complemented in the low word).
__device__ __forceinline__ uint64_t rank_key(float score, uint32_t id) {
    return ((uint64_t)float_order_key(score) << 32) | (uint64_t)(0xffffffffu - id);
}
__device__ __forceinline__ uint32_t rank_key_id(uint64_t k) {
    return 0xffffffffu - (uint32_t)(k & 0xffffffffu);
}
__device__ __forceinline__ float rank_key_score(uint64_t k) {
    return float_from_order_key((uint32_t)(k >> 32));
}

// Iteration guard of the CG kernels: true when the previous stopping test
// left no active column (ntile per-tile counts, all zero). Every kernel of an
// iteration returns at once then, so the host can queue an iteration before
// it knows whether it is needed.
__device__ __forceinline__ bool all_stopped(const int32_t *nact, int ntile) {
    if (nact == nullptr) return false;
    int s = 0;
    for (int t = 0; t < ntile; ++t) s += nact[t];
    return s == 0;
}

// x + a p as the x-only update writes it (a = 0: x unchanged)
__device__ __forceinline__ float fold_x(float x, float p, double a) {
    return a != 0.0 ? (float)((double)x + a * (double)p) : x;
}

// Row i is in a row mask (bit i of word i / 32; nullptr: every row is).
__device__ __forceinline__ bool row_live(const uint32_t *m, int64_t i) {
    return !m || ((m[i >> 5] >> (i & 31)) & 1u);
}

// Sum of a double over the 64 lanes of a wavefront (fixed butterfly order).
__device__ __forceinline__ double wave_sum_f64(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

}  // namespace hd
