// Top-K selection per row (Section 3: items are ranked by decreasing x; also
// used for the k_y nearest neighbours that form y).
//
// Each element becomes a 64-bit key (order-preserving score bits, then the
// complemented id), so one unsigned comparison orders by score and breaks
// ties toward the lower id: the selected set and its order are unique.
//
// Three kernels per call:
//   thresh : (one block per row) radix-select on a strided sample of
//            m <= 4096 elements: the threshold t is the sample's j-th largest, j a few
//            standard deviations above the number of true top-K elements
//            expected in the sample (K m / n), so that t lies below the K-th
//            best with high probability;
//   filter : one coalesced pass over the rows, 8192 elements per block; each
//            element with score >= t is appended to its block's own list
//            (LDS counter, no global atomics);
//   select : (one block per row) if the lists hold K <= count <= 8192
//            candidates and none overflowed, they contain the top K (at least
//            K elements are >= t, so the K-th best is >= t): gather, sort in
//            LDS, write the first K. Otherwise the block selects exactly on
//            its own: an MSB-first radix select over the row finds the K-th
//            key, then a pass in index order collects the keys above it and
//            the lowest-id ties.
//
// The number of row elements at or above t is about n Beta(j+1, m-j), mean
// (j+1) n / m (about 2000 at K <= 100, n = 1M): a cap of 4096 was exceeded by
// about one row in a hundred, and one such row holds a whole batch for the
// full-row selection; at 8192 it is about one in 10^7. The kernel time of a
// batch is that of its slowest row, so the cap matters more than the mean.
// Candidate order within a list depends on timing; the result does not.
#include "hd_device.h"
#include "hd_kernels.h"

namespace hd {

constexpr int kCap = 8192;        // candidates per row for the final sort (64 KB of LDS)
constexpr int kMaxChunk = 4096;   // filter blocks per row the fast path accepts (n <= 32M)
constexpr int kSample = 4096;     // sampled elements per row
constexpr int kChunk = 8192;      // row elements per filter block
constexpr int kChunkCap = 256;    // candidates kept per filter block
constexpr int kWide = 1024;       // threads of the thresh / select blocks

struct TopkScratch {
    uint64_t *cand;   // [B][nchunk][kChunkCap]
    int32_t *cnt;     // [B][nchunk]
    uint32_t *thr;    // [B]
    int32_t *all;     // [B] 1 = threshold admits every element
    int nchunk;
};

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

static TopkScratch carve(void *scratch, int B, int64_t n) {
    TopkScratch t;
    t.nchunk = (int)ceil_div(n, kChunk);
    char *p = reinterpret_cast<char *>(scratch);
    t.cand = reinterpret_cast<uint64_t *>(p);
    p += (size_t)B * t.nchunk * kChunkCap * sizeof(uint64_t);
    t.cnt = reinterpret_cast<int32_t *>(p);
    p += (size_t)B * t.nchunk * sizeof(int32_t);
    t.thr = reinterpret_cast<uint32_t *>(p);
    p += (size_t)B * sizeof(uint32_t);
    t.all = reinterpret_cast<int32_t *>(p);
    return t;
}

size_t topk_scratch_bytes(int B, int64_t n, int K) {
    (void)K;
    const int64_t nchunk = ceil_div(n, kChunk);
    return (size_t)B * (nchunk * (kChunkCap * sizeof(uint64_t) + sizeof(int32_t)) +
                        sizeof(uint32_t) + sizeof(int32_t)) + 256;
}

template <typename T, int NT>
__device__ __forceinline__ void bitonic_desc(T *s, int size) {
    for (int k = 2; k <= size; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < size / 2; t += NT) {
                const int i = 2 * t - (t & (j - 1));
                const int p = i + j;
                const T a = s[i], c = s[p];
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

__device__ __forceinline__ int pow2_ceil(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

// MSB-first radix select of the need-th largest key (1-based) among the keys
// each thread holds in registers (up to 4 per thread). Per 8-bit digit: an LDS
// histogram of the keys that still match the prefix, then wave 0 scans the 256
// bins from the top (4 bins per lane, shuffle scan) to find the digit.
__device__ __forceinline__ uint32_t block_select_key(const uint32_t *key, int nkey, int need) {
    __shared__ int hist[256];
    __shared__ int sel[2];
    uint32_t prefix = 0, pmask = 0;
    const int lane = threadIdx.x % kWave;
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 24 - 8 * pass;
        for (int t = threadIdx.x; t < 256; t += blockDim.x) hist[t] = 0;
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (u < nkey && (key[u] & pmask) == prefix) atomicAdd(&hist[(key[u] >> shift) & 255], 1);
        __syncthreads();
        if (threadIdx.x < kWave) {
            int c[4], loc = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                c[q] = hist[255 - 4 * lane - q];
                loc += c[q];
            }
            int inc = loc;
            for (int off = 1; off < kWave; off <<= 1) {
                const int v = __shfl_up(inc, off, kWave);
                if (lane >= off) inc += v;
            }
            const uint64_t hit = __ballot(inc >= need);
            const int first = __ffsll((long long)hit) - 1;
            if (lane == first) {
                int above = inc - loc;
                int q = 0;
                while (q < 3 && above + c[q] < need) {
                    above += c[q];
                    ++q;
                }
                sel[0] = 255 - 4 * lane - q;
                sel[1] = need - above;
            }
        }
        __syncthreads();
        prefix |= (uint32_t)sel[0] << shift;
        pmask |= 255u << shift;
        need = sel[1];
        __syncthreads();
    }
    return prefix;
}

__global__ __launch_bounds__(kWide) void k_topk_thresh(int64_t n, const float *__restrict__ x,
                                                       int64_t ldx, int K, int64_t stride,
                                                       TopkScratch ts) {
    const int b = blockIdx.x;
    const int64_t m = (n + stride - 1) / stride;  // sample size, <= kSample = 4 * kWide
    uint32_t key[4];
    int nkey = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t t = threadIdx.x + (int64_t)u * kWide;
        key[u] = 0u;
        if (t < m) {
            key[u] = float_order_key(x[(size_t)b * ldx + (size_t)t * stride]);
            nkey = u + 1;
        }
    }
    // threshold: the sample's (j+1)-th largest, j a few standard deviations
    // above the number e = K m / n of true top-K elements expected in it
    const double e = (double)K * (double)m / (double)n;
    const int64_t j = (int64_t)ceil(e + 4.0 * sqrt(e) + 4.0);
    const bool all = j >= m;
    uint32_t thr = 0u;
    if (!all) thr = block_select_key(key, nkey, (int)j + 1);
    if (threadIdx.x == 0) {
        ts.thr[b] = thr;
        ts.all[b] = all ? 1 : 0;
    }
}

__device__ __forceinline__ void filter_one(float v, int64_t i, uint32_t thr, int *lcount,
                                           uint64_t *cand) {
    if (float_order_key(v) >= thr) {
        const int slot = atomicAdd(lcount, 1);
        if (slot < kChunkCap) cand[slot] = rank_key(v, (uint32_t)i);
    }
}

// V = 4: 16-byte loads (rows 16-byte aligned: x aligned and ldx % 4 == 0).
template <int V>
__global__ __launch_bounds__(kBlock) void k_topk_filter(int64_t n, const float *__restrict__ x,
                                                        int64_t ldx, TopkScratch ts) {
    __shared__ int lcount;
    const int b = blockIdx.y;
    const int c = blockIdx.x;
    if (ts.all[b]) return;  // the select kernel reads such rows directly
    const uint32_t thr = ts.thr[b];
    if (threadIdx.x == 0) lcount = 0;
    __syncthreads();
    uint64_t *cand = ts.cand + ((size_t)b * ts.nchunk + c) * kChunkCap;
    const int64_t base = (int64_t)c * kChunk;
    const float *row = x + (size_t)b * ldx;
    if (V == 4) {
        float4 v[kChunk / (4 * kBlock)];
#pragma unroll
        for (int u = 0; u < kChunk / (4 * kBlock); ++u) {
            const int64_t i = base + (int64_t)(u * kBlock + threadIdx.x) * 4;
            v[u] = i + 3 < n ? *reinterpret_cast<const float4 *>(row + i) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < kChunk / (4 * kBlock); ++u) {
            const int64_t i = base + (int64_t)(u * kBlock + threadIdx.x) * 4;
            if (i + 3 < n) {
                filter_one(v[u].x, i, thr, &lcount, cand);
                filter_one(v[u].y, i + 1, thr, &lcount, cand);
                filter_one(v[u].z, i + 2, thr, &lcount, cand);
                filter_one(v[u].w, i + 3, thr, &lcount, cand);
            } else {
                for (int64_t e = i; e < n && e < i + 4; ++e) filter_one(row[e], e, thr, &lcount, cand);
            }
        }
    } else {
#pragma unroll 4
        for (int u = 0; u < kChunk / kBlock; ++u) {
            const int64_t i = base + u * kBlock + threadIdx.x;
            if (i < n) filter_one(row[i], i, thr, &lcount, cand);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) ts.cnt[(size_t)b * ts.nchunk + c] = lcount;
}

// Exclusive prefix sum over the kWide threads of the block; *total gets the
// sum. wsum: kWide / kWave ints of LDS.
__device__ __forceinline__ int block_excl_scan(int v, int *wsum, int *total) {
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    int inc = v;
    for (int off = 1; off < kWave; off <<= 1) {
        const int t = __shfl_up(inc, off, kWave);
        if (lane >= off) inc += t;
    }
    if (lane == kWave - 1) wsum[w] = inc;
    __syncthreads();
    if (w == 0) {
        int t = lane < kWide / kWave ? wsum[lane] : 0;
        for (int off = 1; off < kWide / kWave; off <<= 1) {
            const int u = __shfl_up(t, off, kWave);
            if (lane >= off) t += u;
        }
        if (lane < kWide / kWave) wsum[lane] = t;  // inclusive per-wave totals
    }
    __syncthreads();
    const int base = w ? wsum[w - 1] : 0;
    *total = wsum[kWide / kWave - 1];
    __syncthreads();
    return base + inc - v;
}

__device__ __forceinline__ void write_out(const uint64_t *s, int K, int b, int32_t *ids,
                                          float *scores, int transform) {
    for (int t = threadIdx.x; t < K; t += kWide) {
        const uint64_t k = s[t];
        if (ids) ids[(size_t)b * K + t] = (int32_t)rank_key_id(k);
        if (scores) {
            float v = rank_key_score(k);
            if (transform == 1) {
                const float c = v > 0.f ? v : 0.f;
                v = c * c * c;
            }
            scores[(size_t)b * K + t] = v;
        }
    }
}

__global__ __launch_bounds__(kWide) void k_topk_select(int64_t n, const float *__restrict__ x,
                                                       int64_t ldx, int K, TopkScratch ts,
                                                       int32_t *__restrict__ ids,
                                                       float *__restrict__ scores, int transform) {
    __shared__ uint64_t s[kCap];
    __shared__ int offs[kMaxChunk + 1];
    __shared__ int hist[256];
    __shared__ int sh_int[8];
    __shared__ int wcount[kWide / kWave];
    const int b = blockIdx.x;
    const float *row = x + (size_t)b * ldx;
    const int nchunk = ts.nchunk;

    // ---- fast paths ----
    int total = -1;
    if (ts.all[b]) {
        if (n <= kCap) total = (int)n;
    } else if (nchunk <= kMaxChunk) {
        // offsets of the per-chunk lists: 4 consecutive chunks per thread
        constexpr int kPer = kMaxChunk / kWide;
        int v[kPer], loc = 0;
        bool bad = false;
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int c = threadIdx.x * kPer + q;
            v[q] = c < nchunk ? ts.cnt[(size_t)b * nchunk + c] : 0;
            bad |= v[q] > kChunkCap;
            loc += v[q];
        }
        int acc;
        int o = block_excl_scan(loc, wcount, &acc);
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int c = threadIdx.x * kPer + q;
            if (c < nchunk) offs[c] = o;
            o += v[q];
        }
        if (threadIdx.x == 0) offs[nchunk] = acc;
        const int anybad = __syncthreads_or(bad ? 1 : 0);
        total = (anybad || acc < K || acc > kCap) ? -1 : acc;
    }
    if (total >= 0) {
        const int size = pow2_ceil(total);
        if (ts.all[b]) {
            for (int t = threadIdx.x; t < size; t += kWide)
                s[t] = t < total ? rank_key(row[t], (uint32_t)t) : 0ull;
        } else {
            // candidate t lives in the list of the chunk c with
            // offs[c] <= t < offs[c + 1] (binary search; empty lists repeat
            // an offset, so take the last such c)
            const uint64_t *src = ts.cand + (size_t)b * nchunk * kChunkCap;
            for (int t = threadIdx.x; t < size; t += kWide) {
                uint64_t key = 0ull;
                if (t < total) {
                    int lo = 0, hi = nchunk;  // offs[lo] <= t < offs[hi]
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (offs[mid] <= t) lo = mid; else hi = mid;
                    }
                    key = src[(size_t)lo * kChunkCap + (t - offs[lo])];
                }
                s[t] = key;
            }
        }
        __syncthreads();
        bitonic_desc<uint64_t, kWide>(s, size);
        write_out(s, K, b, ids, scores, transform);
        return;
    }

    // ---- exact selection within the block ----
    uint32_t prefix = 0, pmask = 0;
    int need = K;  // rank (1-based) of the wanted key among those matching the prefix
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 24 - 8 * pass;
        for (int t = threadIdx.x; t < 256; t += kWide) hist[t] = 0;
        __syncthreads();
        for (int64_t i = threadIdx.x; i < n; i += kWide) {
            const uint32_t key = float_order_key(row[i]);
            if ((key & pmask) == prefix) atomicAdd(&hist[(key >> shift) & 255], 1);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int above = 0, dsel = 0;
            for (int dgt = 255; dgt >= 0; --dgt) {
                if (above + hist[dgt] >= need) {
                    dsel = dgt;
                    break;
                }
                above += hist[dgt];
            }
            sh_int[0] = dsel;
            sh_int[1] = need - above;
        }
        __syncthreads();
        prefix |= (uint32_t)sh_int[0] << shift;
        pmask |= 255u << shift;
        need = sh_int[1];
        __syncthreads();
    }
    // prefix is the K-th largest key; `need` of its equals are taken (lowest
    // ids first) and K - need keys lie strictly above it.
    const int n_above = K - need;
    if (threadIdx.x == 0) {
        sh_int[2] = 0;  // slots used by keys above
        sh_int[3] = 0;  // equal keys taken so far
    }
    __syncthreads();
    for (int64_t i = threadIdx.x; i < n; i += kWide) {
        const float v = row[i];
        if (float_order_key(v) > prefix) {
            const int slot = atomicAdd(&sh_int[2], 1);
            s[slot] = rank_key(v, (uint32_t)i);
        }
    }
    __syncthreads();
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int64_t base = 0; base < n; base += kWide) {
        if (sh_int[3] >= need) break;  // uniform: written before the last barrier
        const int64_t i = base + threadIdx.x;
        const float v = i < n ? row[i] : 0.f;
        const bool eq = i < n && float_order_key(v) == prefix;
        const uint64_t mask = __ballot(eq);
        if (lane == 0) wcount[w] = __popcll(mask);
        __syncthreads();
        int before = sh_int[3];
        for (int q = 0; q < w; ++q) before += wcount[q];
        const int slot = before + __popcll(mask & below);
        if (eq && slot < need) s[n_above + slot] = rank_key(v, (uint32_t)i);
        __syncthreads();
        if (threadIdx.x == 0) {
            int tot = 0;
            for (int q = 0; q < kWide / kWave; ++q) tot += wcount[q];
            sh_int[3] += tot;
        }
        __syncthreads();
    }
    const int size = pow2_ceil(K);
    for (int t = K + threadIdx.x; t < size; t += kWide) s[t] = 0ull;
    __syncthreads();
    bitonic_desc<uint64_t, kWide>(s, size);
    write_out(s, K, b, ids, scores, transform);
}

hipError_t launch_topk(int B, int64_t n, const float *x, int64_t ldx, int K, void *scratch,
                       int32_t *ids, float *scores, int transform, hipStream_t s) {
    if (K < 1 || K > kTopkMax || K > n || B < 1) return hipErrorInvalidValue;
    TopkScratch ts = carve(scratch, B, n);
    const int64_t stride = ceil_div(n, kSample);
    k_topk_thresh<<<B, kWide, 0, s>>>(n, x, ldx, K, stride, ts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 fg((unsigned)ts.nchunk, B);
    if (ldx % 4 == 0 && reinterpret_cast<uintptr_t>(x) % 16 == 0) {
        k_topk_filter<4><<<fg, kBlock, 0, s>>>(n, x, ldx, ts);
    } else {
        k_topk_filter<1><<<fg, kBlock, 0, s>>>(n, x, ldx, ts);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_topk_select<<<B, kWide, 0, s>>>(n, x, ldx, K, ts, ids, scores, transform);
    return hipGetLastError();
}

}  // namespace hd
