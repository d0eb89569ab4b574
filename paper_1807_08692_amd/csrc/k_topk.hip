// Top-K selection per row (Section 3: items are ranked by decreasing x; also
// used for the k_y nearest neighbours that form y).
//
// Each element becomes a 64-bit key (order-preserving score bits, then the
// complemented id), so one unsigned comparison orders by score and breaks
// ties toward the lower id, and the result is unique. Rows are cut into
// chunks of 2048 keys; a block sorts a chunk in LDS with a bitonic network
// and keeps its best min(K, 2048). The surviving candidates are chunked and
// sorted again until one chunk per row remains, whose first K keys are the
// answer. Each round shrinks the candidate set by 2048/K.
#include "hd_device.h"
#include "hd_kernels.h"

namespace hd {

constexpr int CH = kTopkChunk;

// Sort CH keys in LDS into descending order (256 threads).
__device__ __forceinline__ void bitonic_desc(uint64_t *s) {
    for (int k = 2; k <= CH; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < CH / 2; t += kBlock) {
                const int i = 2 * t - (t & (j - 1));
                const int p = i + j;
                const uint64_t a = s[i], c = s[p];
                const bool desc = (i & k) == 0;
                if (desc ? (a < c) : (a > c)) {
                    s[i] = c;
                    s[p] = a;
                }
            }
            __syncthreads();
        }
    }
}

// Level 0: scores -> keys. Block (c, b) sorts x[b][c*CH .. c*CH+CH) and
// writes its best kc keys to out[b][c][0..kc).
__global__ __launch_bounds__(kBlock) void k_topk_f32(int64_t n, const float *__restrict__ x,
                                                     int64_t ldx, int kc, int nchunk,
                                                     uint64_t *__restrict__ out) {
    __shared__ uint64_t s[CH];
    const int b = blockIdx.y;
    const int64_t base = (int64_t)blockIdx.x * CH;
    for (int t = threadIdx.x; t < CH; t += kBlock) {
        const int64_t i = base + t;
        s[t] = i < n ? rank_key(x[(size_t)b * ldx + i], (uint32_t)i) : 0ull;
    }
    __syncthreads();
    bitonic_desc(s);
    uint64_t *o = out + ((size_t)b * nchunk + blockIdx.x) * kc;
    for (int t = threadIdx.x; t < kc; t += kBlock) o[t] = s[t];
}

// Level >= 1: keys -> keys (m keys per row).
__global__ __launch_bounds__(kBlock) void k_topk_u64(int64_t m, const uint64_t *__restrict__ in,
                                                     int kc, int nchunk,
                                                     uint64_t *__restrict__ out) {
    __shared__ uint64_t s[CH];
    const int b = blockIdx.y;
    const int64_t base = (int64_t)blockIdx.x * CH;
    for (int t = threadIdx.x; t < CH; t += kBlock) {
        const int64_t i = base + t;
        s[t] = i < m ? in[(size_t)b * m + i] : 0ull;
    }
    __syncthreads();
    bitonic_desc(s);
    uint64_t *o = out + ((size_t)b * nchunk + blockIdx.x) * kc;
    for (int t = threadIdx.x; t < kc; t += kBlock) o[t] = s[t];
}

__global__ void k_topk_decode(int B, int K, const uint64_t *__restrict__ keys,
                              int32_t *__restrict__ ids, float *__restrict__ scores,
                              int transform) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * K) return;
    const uint64_t k = keys[idx];
    if (ids) ids[idx] = (int32_t)rank_key_id(k);
    if (scores) {
        float s = rank_key_score(k);
        if (transform == 1) {
            const float c = s > 0.f ? s : 0.f;
            s = c * c * c;
        }
        scores[idx] = s;
    }
}

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

size_t topk_scratch_bytes(int B, int64_t n, int K) {
    const int kc = K < CH ? K : CH;
    const int64_t n0 = ceil_div(n, CH) * kc;  // keys per row after level 0
    return 2 * (size_t)B * (size_t)n0 * sizeof(uint64_t) + 256;
}

hipError_t launch_topk(int B, int64_t n, const float *x, int64_t ldx, int K, void *scratch,
                       int32_t *ids, float *scores, int transform, hipStream_t s) {
    if (K < 1 || K > kTopkMax || K > n || B < 1) return hipErrorInvalidValue;
    const int kc = K;
    const int64_t n0 = ceil_div(n, CH) * kc;
    uint64_t *buf[2];
    buf[0] = reinterpret_cast<uint64_t *>(scratch);
    buf[1] = buf[0] + (size_t)B * n0;
    int nchunk = (int)ceil_div(n, CH);
    k_topk_f32<<<dim3(nchunk, B), kBlock, 0, s>>>(n, x, ldx, kc, nchunk, buf[0]);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int64_t m = (int64_t)nchunk * kc;
    int cur = 0;
    while (nchunk > 1) {
        nchunk = (int)ceil_div(m, CH);
        k_topk_u64<<<dim3(nchunk, B), kBlock, 0, s>>>(m, buf[cur], kc, nchunk, buf[cur ^ 1]);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        cur ^= 1;
        m = (int64_t)nchunk * kc;
    }
    const int tot = B * K;
    k_topk_decode<<<(tot + 255) / 256, 256, 0, s>>>(B, K, buf[cur], ids, scores, transform);
    return hipGetLastError();
}

}  // namespace hd
