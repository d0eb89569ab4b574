// Candidate emission of the one-pass top-K (device side): a kernel that
// produces ranking scores offers each of them to its row's candidate lists
// (hd::TopkLists) instead of writing the score matrix. A block stages its
// candidates in LDS and flushes them after a barrier, one global atomic per
// candidate, into the list of the chunk its items lie in (a block's items
// never straddle two chunks of kTopkChunk items).
#pragma once

#include "hd_device.h"
#include "hd_kernels.h"

namespace hd {

constexpr int kEmitCap = 512;  // candidates a block stages before its flush

struct EmitStage {
    uint64_t key[kEmitCap];
    int32_t row[kEmitCap];
    int n;  // candidates offered (may exceed kEmitCap)
};

// Offer score v of item i in row b (thr: the row's threshold key).
__device__ __forceinline__ void emit_one(EmitStage &es, uint32_t thr, int b, int64_t i, float v) {
    if (float_order_key(v) >= thr) {
        const int slot = atomicAdd(&es.n, 1);
        if (slot < kEmitCap) {
            es.key[slot] = rank_key(v, (uint32_t)i);
            es.row[slot] = b;
        }
    }
}

// After a barrier that follows every emit_one of the block: append the
// staged candidates to chunk c of their rows. If the stage overflowed, the
// lists of every row of the block ([b_lo, b_hi)) are marked overfull, so
// those rows go to the exact fallback instead.
__device__ __forceinline__ void emit_flush(EmitStage &es, const TopkLists &tl, int c, int b_lo, int b_hi) {
    const int n = es.n;
    if (n > kEmitCap) {
        for (int b = b_lo + (int)threadIdx.x; b < b_hi; b += (int)blockDim.x)
            atomicAdd(&tl.cnt[(size_t)b * tl.nchunk + c], kTopkChunkCap + 1);
        return;
    }
    for (int t = (int)threadIdx.x; t < n; t += (int)blockDim.x) {
        const size_t list = (size_t)es.row[t] * tl.nchunk + c;
        const int slot = atomicAdd(&tl.cnt[list], 1);
        if (slot < kTopkChunkCap) tl.cand[list * kTopkChunkCap + slot] = es.key[t];
    }
}

}  // namespace hd
