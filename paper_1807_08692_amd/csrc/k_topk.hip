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
//
// One-pass form (rows of n >= kTopkFuseMin items): the threshold comes from
// the scores of a fixed sample of the row's items, computed before the full
// scores (launch_topk_prepare); the kernel that produces the scores appends
// the candidates to the lists itself (hd_emit.h) and never writes the score
// matrix; the select step then runs on the lists alone
// (launch_topk_select_lists). A row it cannot finish from its lists is
// flagged instead, and launch_topk_fallback selects the flagged rows exactly
// once a gated second launch of the score kernel has written their scores.
#include "hd_device.h"
#include "hd_kernels.h"
#include "hd_emit.h"

namespace hd {

constexpr int kCap = 8192;        // candidates per row for the final sort (64 KB of LDS)
constexpr int kMaxChunk = 4096;   // filter blocks per row the fast path accepts (n <= 32M)
constexpr int kSample = 4096;     // sampled elements per row
constexpr int kChunk = kTopkChunk;        // row elements per filter block
constexpr int kChunkCap = kTopkChunkCap;  // candidates kept per filter block
constexpr int kWide = 1024;       // threads of the thresh / select blocks

struct TopkScratch {
    uint64_t *cand;   // [B][nchunk][kChunkCap]
    int32_t *cnt;     // [B][nchunk]
    uint32_t *thr;    // [B]
    int32_t *all;     // [B] 1 = threshold admits every element
    int32_t *fb;      // [1 + B] one-pass form: any row flagged, then the row flags
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
    p += (size_t)B * sizeof(int32_t);
    t.fb = reinterpret_cast<int32_t *>(p);
    return t;
}

size_t topk_scratch_bytes(int B, int64_t n, int K) {
    (void)K;
    const int64_t nchunk = ceil_div(n, kChunk);
    return (size_t)B * (nchunk * (kChunkCap * sizeof(uint64_t) + sizeof(int32_t)) +
                        sizeof(uint32_t) + 2 * sizeof(int32_t)) + sizeof(int32_t) + 256;
}

void topk_sample(int64_t n, int64_t *stride, int64_t *m) {
    const int64_t st = ceil_div(n, kSample);
    *stride = st;
    *m = ceil_div(n, st);
}

TopkLists topk_lists(void *scratch, int B, int64_t n) {
    const TopkScratch t = carve(scratch, B, n);
    return TopkLists{t.cand, t.cnt, t.thr, t.nchunk};
}

const int32_t *topk_fallback_gate(void *scratch, int B, int64_t n) { return carve(scratch, B, n).fb; }

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

// Row b's sample: m values at x[b * ldx + t * sstride], t < m, drawn from a
// row of n elements. lists = true (one-pass form) also empties the row's
// candidate lists and clears its fallback flag (block 0 the shared one).
__global__ __launch_bounds__(kWide) void k_topk_thresh(int64_t n, int64_t m, const float *__restrict__ x,
                                                       int64_t ldx, int64_t sstride, int K,
                                                       TopkScratch ts, bool lists) {
    const int b = blockIdx.x;
    uint32_t key[4];
    int nkey = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t t = threadIdx.x + (int64_t)u * kWide;
        key[u] = 0u;
        if (t < m) {
            key[u] = float_order_key(x[(size_t)b * ldx + (size_t)t * sstride]);
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
    if (lists) {
        for (int c = threadIdx.x; c < ts.nchunk; c += kWide) ts.cnt[(size_t)b * ts.nchunk + c] = 0;
        if (threadIdx.x == 0) {
            ts.fb[1 + b] = 0;
            if (b == 0) ts.fb[0] = 0;
        }
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

// mode 0: the two-pass form (fast path from the lists, else exact from x);
// mode 1: the one-pass form, lists only (x is not read: a row the lists
// cannot finish is flagged and left unwritten); mode 2: the flagged rows
// only, exactly from x (every other block returns at once).
__global__ __launch_bounds__(kWide) void k_topk_select(int64_t n, const float *__restrict__ x,
                                                       int64_t ldx, int K, TopkScratch ts,
                                                       int32_t *__restrict__ ids,
                                                       float *__restrict__ scores, int transform,
                                                       int mode) {
    __shared__ uint64_t s[kCap];
    __shared__ int offs[kMaxChunk + 1];
    __shared__ int hist[256];
    __shared__ int sh_int[8];
    __shared__ int wcount[kWide / kWave];
    const int b = blockIdx.x;
    const float *row = x + (size_t)b * ldx;
    const int nchunk = ts.nchunk;

    if (mode == 2 && ts.fb[1 + b] == 0) return;
    // ---- fast paths ----
    int total = -1;
    if (mode == 2) {
        // flagged: straight to the exact selection
    } else if (ts.all[b]) {
        if (n <= kCap && mode == 0) total = (int)n;
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

    if (mode == 1) {
        // the lists cannot give this row's top K: flag it for the fallback
        if (threadIdx.x == 0) {
            ts.fb[1 + b] = 1;
            atomicOr(&ts.fb[0], 1);
        }
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
    k_topk_thresh<<<B, kWide, 0, s>>>(n, ceil_div(n, stride), x, ldx, stride, K, ts, false);
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
    k_topk_select<<<B, kWide, 0, s>>>(n, x, ldx, K, ts, ids, scores, transform, 0);
    return hipGetLastError();
}

hipError_t launch_topk_prepare(int B, int64_t n, const float *S, int64_t ld_row, int64_t ld_item, int K,
                               void *scratch, hipStream_t s) {
    if (K < 1 || K > kTopkMax || K > n || B < 1 || n < kTopkFuseMin) return hipErrorInvalidValue;
    int64_t stride, m;
    topk_sample(n, &stride, &m);
    k_topk_thresh<<<B, kWide, 0, s>>>(n, m, S, ld_row, ld_item, K, carve(scratch, B, n), true);
    return hipGetLastError();
}

hipError_t launch_topk_select_lists(int B, int64_t n, int K, void *scratch, int32_t *ids, float *scores,
                                    int transform, hipStream_t s) {
    if (K < 1 || K > kTopkMax || K > n || B < 1 || n < kTopkFuseMin) return hipErrorInvalidValue;
    k_topk_select<<<B, kWide, 0, s>>>(n, nullptr, 0, K, carve(scratch, B, n), ids, scores, transform, 1);
    return hipGetLastError();
}

hipError_t launch_topk_fallback(int B, int64_t n, const float *x, int64_t ldx, int K, void *scratch,
                                int32_t *ids, float *scores, int transform, hipStream_t s) {
    if (K < 1 || K > kTopkMax || K > n || B < 1 || n < kTopkFuseMin) return hipErrorInvalidValue;
    k_topk_select<<<B, kWide, 0, s>>>(n, x, ldx, K, carve(scratch, B, n), ids, scores, transform, 2);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// One-pass candidates straight from node-major X (plain CG ranks x = X^T):
// a block covers 256 items (64 per wave, so one list chunk) and 64 query
// columns, lane = column; every wave loads its 64 items' column runs before
// testing them.
template <bool FOLD>
__global__ __launch_bounds__(kBlock) void k_topk_emit_nm(int64_t n, int B, int ldb, const float *__restrict__ X,
                                                         TopkLists tl, XFold fold) {
    __shared__ EmitStage es;
    __shared__ uint32_t thr[64];
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    const int b0 = blockIdx.y * 64;
    const int64_t i0 = (int64_t)blockIdx.x * 256;
    if (threadIdx.x < 64) thr[threadIdx.x] = b0 + threadIdx.x < B ? tl.thr[b0 + threadIdx.x] : 0u;
    if (threadIdx.x == 0) es.n = 0;
    __syncthreads();
    const int b = b0 + lane;
    const int64_t ib = i0 + 64 * w;
    const double fa = FOLD && b < B && !all_stopped(fold.g.nact, fold.g.ntile) ? fold.a[b] : 0.0;
    float v[16], pv[16];
    for (int u = 0; u < 64; u += 16) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int64_t i = ib + u + q;
            const size_t o = vec_index(n, ldb, i < n ? i : n - 1, b < B ? b : 0);
            v[q] = X[o];
            if (FOLD) pv[q] = fold.P[o];
        }
        if (FOLD) {
#pragma unroll
            for (int q = 0; q < 16; ++q) v[q] = fold_x(v[q], pv[q], fa);
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int64_t i = ib + u + q;
            if (i < n && b < B) emit_one(es, thr[lane], b, i, v[q]);
        }
    }
    __syncthreads();
    emit_flush(es, tl, (int)(i0 / kTopkChunk), b0, b0 + 64 < B ? b0 + 64 : B);
}

hipError_t launch_topk_emit_nm(int64_t n, int B, int ldb, const float *X, TopkLists tl, hipStream_t s,
                               const XFold *fold) {
    if (n < 1 || B < 1 || B > ldb) return hipErrorInvalidValue;
    const dim3 g((unsigned)ceil_div(n, 256), (unsigned)ceil_div(B, 64));
    if (fold)
        k_topk_emit_nm<true><<<g, kBlock, 0, s>>>(n, B, ldb, X, tl, *fold);
    else
        k_topk_emit_nm<false><<<g, kBlock, 0, s>>>(n, B, ldb, X, tl, XFold{nullptr, nullptr, IterGuard{nullptr, 0}});
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Row samples. Fragment-order matrices (rows padded to 16, ld a multiple of
// 32; elem_bytes 2 for bfloat16, 1 for fp8 codes): dst row t = src row
// t * stride for t < m, zero rows from m to m rounded up to 16. A thread
// copies one 8-element lane piece, contiguous in both layouts.
__global__ __launch_bounds__(kBlock) void k_sample_frag(int64_t m, int64_t m16, int64_t stride, int64_t ld,
                                                        const uint8_t *__restrict__ src,
                                                        uint8_t *__restrict__ dst, int eb) {
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t pieces = ld / 8;
    if (idx >= m16 * pieces) return;
    const int64_t t = idx / pieces, k = 8 * (idx % pieces);
    const size_t od = frag_offset(t, k, ld / 32) * (size_t)eb;
    if (eb == 2) {
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (t < m) v = *reinterpret_cast<const uint4 *>(src + frag_offset(t * stride, k, ld / 32) * 2);
        *reinterpret_cast<uint4 *>(dst + od) = v;
    } else {
        uint2 v = make_uint2(0u, 0u);
        if (t < m) v = *reinterpret_cast<const uint2 *>(src + frag_offset(t * stride, k, ld / 32));
        *reinterpret_cast<uint2 *>(dst + od) = v;
    }
}

hipError_t launch_sample_frag(int64_t m, int64_t stride, int64_t ld, const void *src, void *dst, int elem_bytes,
                              hipStream_t s) {
    if (m < 1 || stride < 1 || ld % 32 != 0 || (elem_bytes != 1 && elem_bytes != 2)) return hipErrorInvalidValue;
    const int64_t m16 = (m + 15) / 16 * 16, tot = m16 * (ld / 8);
    k_sample_frag<<<(unsigned)ceil_div(tot, kBlock), kBlock, 0, s>>>(m, m16, stride, ld,
                                                                     reinterpret_cast<const uint8_t *>(src),
                                                                     reinterpret_cast<uint8_t *>(dst), elem_bytes);
    return hipGetLastError();
}

// Row-major rows: dst[t * ld + c] = src[t * stride * ld + c], t < m, c < ld
// (with the fold: x + a p as the combine will read it).
__global__ __launch_bounds__(kBlock) void k_sample_rows(int64_t m, int64_t stride, int ld,
                                                        const float *__restrict__ src, float *__restrict__ dst,
                                                        XFold fold) {
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= m * ld) return;
    const int64_t t = idx / ld, c = idx % ld;
    const size_t o = (size_t)t * (size_t)stride * (size_t)ld + (size_t)c;
    const bool fo = fold.a && !all_stopped(fold.g.nact, fold.g.ntile);
    dst[idx] = fo ? fold_x(src[o], fold.P[o], fold.a[c]) : src[o];
}

hipError_t launch_sample_rows(int64_t m, int64_t stride, int ld, const float *src, float *dst, hipStream_t s,
                              const XFold *fold) {
    if (m < 1 || stride < 1 || ld < 1) return hipErrorInvalidValue;
    k_sample_rows<<<(unsigned)ceil_div(m * ld, kBlock), kBlock, 0, s>>>(
        m, stride, ld, src, dst, fold ? *fold : XFold{nullptr, nullptr, IterGuard{nullptr, 0}});
    return hipGetLastError();
}

}  // namespace hd
