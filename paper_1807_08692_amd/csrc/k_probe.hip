// Memory probes: the rates this chip attains for the access patterns of the
// query path's memory-bound kernels, measured with the library's own kernels
// (the ceilings the sparse product and the vector updates are compared with).
//   stream : every 16-byte word of a buffer read once (grid stride)
//   copy   : a buffer read and written once
//   gather : whole rows (row_bytes each) at pseudo-random row ids over the
//            buffer, read from an id array as the sparse product reads its
//            column ids, 16 gathers in flight per wave
//   graph  : the sparse product's own gathers without its arithmetic: for
//            every edge of the loaded graph the neighbour's row of an
//            N x (row_bytes / 4) matrix, rows in CSR order, one wave per row
// Each wave (or thread) folds what it read into a sum that it stores, so no
// load can be dropped; the stores are a few bytes per wave.
#include "hd_device.h"
#include "hd_internal.h"

namespace hd {

__global__ __launch_bounds__(kBlock) void k_probe_read(const float4 *__restrict__ a, size_t n4,
                                                       float *__restrict__ out) {
    float s = 0.f;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += (size_t)gridDim.x * kBlock) {
        const float4 v = a[i];
        s += (v.x + v.y) + (v.z + v.w);
    }
    out[(size_t)blockIdx.x * kBlock + threadIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_probe_copy(const float4 *__restrict__ a, float4 *__restrict__ b,
                                                       size_t n4) {
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += (size_t)gridDim.x * kBlock) b[i] = a[i];
}

// SplitMix64 finaliser (Steele, Lea, Flood 2014): the row id of gather g.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// The row ids of the gather probe, pseudo-random over [0, rows), written
// once before the timed launches so that the timed kernel does no hashing.
__global__ __launch_bounds__(kBlock) void k_probe_ids(int32_t *__restrict__ ids, int64_t n, int64_t rows,
                                                      uint64_t seed) {
    for (int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x; g < n; g += (int64_t)gridDim.x * kBlock)
        ids[g] = (int32_t)(mix64(seed + (uint64_t)g) % (uint64_t)rows);
}

// One wave per run of 64 ids (read with one coalesced load, as the sparse
// product reads a row's column ids), each id's row (64 V floats) gathered
// whole, 16 gathers in flight.
template <int V>
__global__ __launch_bounds__(kBlock) void k_probe_gather(const float *__restrict__ a,
                                                         const int32_t *__restrict__ ids, int64_t ngather,
                                                         float *__restrict__ out) {
    const int lane = threadIdx.x % kWave;
    const int64_t w0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
    const int64_t nw = (int64_t)gridDim.x * (kBlock / kWave);
    float s = 0.f;
    for (int64_t g0 = w0 * kWave; g0 < ngather; g0 += nw * kWave) {
        const int id = g0 + lane < ngather ? ids[g0 + lane] : 0;
        const int cnt = (int)(ngather - g0 < kWave ? ngather - g0 : kWave);
        int t = 0;
        for (; t + 16 <= cnt; t += 16) {
            float pv[16][V];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const float *p = a + (size_t)bcast_i(id, t + u) * (64 * V) + (size_t)lane * V;
#pragma unroll
                for (int v = 0; v < V; ++v) pv[u][v] = p[v];
            }
#pragma unroll
            for (int u = 0; u < 16; ++u)
#pragma unroll
                for (int v = 0; v < V; ++v) s += pv[u][v];
        }
        for (; t < cnt; ++t) {
            const float *p = a + (size_t)bcast_i(id, t) * (64 * V) + (size_t)lane * V;
#pragma unroll
            for (int v = 0; v < V; ++v) s += p[v];
        }
    }
    out[(size_t)blockIdx.x * kBlock + threadIdx.x] = s;
}

// One wave per graph row: the neighbours' rows of P (64 V floats each), 16
// gathers in flight as in the sparse product.
template <int V>
__global__ __launch_bounds__(kBlock) void k_probe_graph(int64_t N, const int64_t *__restrict__ rowptr,
                                                        const int32_t *__restrict__ col,
                                                        const float *__restrict__ P, float *__restrict__ out) {
    const int lane = threadIdx.x % kWave;
    const int64_t w0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
    const int64_t nw = (int64_t)gridDim.x * (kBlock / kWave);
    const int ld = 64 * V;
    float s = 0.f;
    for (int64_t i = w0; i < N; i += nw) {
        const int64_t e0 = rowptr[i], e1 = rowptr[i + 1];
        for (int64_t eb = e0; eb < e1; eb += kWave) {
            const int64_t me = eb + lane;
            const int cidx = me < e1 ? col[me] : 0;
            const int cnt = (int)(e1 - eb < kWave ? e1 - eb : kWave);
            int t = 0;
            for (; t + 16 <= cnt; t += 16) {
                float pv[16][V];
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const float *p = P + (size_t)bcast_i(cidx, t + u) * ld + (size_t)lane * V;
#pragma unroll
                    for (int v = 0; v < V; ++v) pv[u][v] = p[v];
                }
#pragma unroll
                for (int u = 0; u < 16; ++u)
#pragma unroll
                    for (int v = 0; v < V; ++v) s += pv[u][v];
            }
            for (; t < cnt; ++t) {
                const float *p = P + (size_t)bcast_i(cidx, t) * ld + (size_t)lane * V;
#pragma unroll
                for (int v = 0; v < V; ++v) s += p[v];
            }
        }
    }
    out[(size_t)blockIdx.x * kBlock + threadIdx.x] = s;
}

}  // namespace hd

extern "C" int hd_probe_memory(hd_ctx *c, int32_t mode, int64_t bytes, int32_t row_bytes, int32_t reps,
                               double *ms_out, double *bytes_out) {
    g_err.clear();
    if (!c) return fail(HD_EINVAL, "hd_probe_memory: NULL context");
    if (mode < 0 || mode > 3) return fail(HD_EINVAL, "hd_probe_memory: mode %d not in 0..3", mode);
    if (reps < 1 || reps > 1000) return fail(HD_EINVAL, "hd_probe_memory: reps %d not in [1, 1000]", reps);
    if ((mode >= 2) && (row_bytes != 256 && row_bytes != 512 && row_bytes != 1024))
        return fail(HD_EINVAL, "hd_probe_memory: row_bytes %d not 256, 512 or 1024", row_bytes);
    if (mode == 3 && c->n == 0) return fail(HD_ESTATE, "hd_probe_memory: the graph probe needs a loaded graph");
    if (mode < 3 && (bytes < (1 << 20) || bytes > ((int64_t)64 << 30) || bytes % 4096 != 0))
        return fail(HD_EINVAL, "hd_probe_memory: bytes must be a multiple of 4096 in [1 MiB, 64 GiB]");
    HIP_TRY(hipSetDevice(c->device));
    const int64_t buf_bytes = mode == 3 ? c->n * (int64_t)row_bytes : bytes;
    const int grid = 2048;
    DevBuf a, b, out, ids;
    auto cleanup = [&]() {
        a.release();
        b.release();
        out.release();
        ids.release();
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = HD_OK;
    do {
        hipError_t e;
        if ((e = a.ensure((size_t)buf_bytes)) != hipSuccess ||
            (mode == 1 && (e = b.ensure((size_t)buf_bytes)) != hipSuccess) ||
            (e = out.ensure((size_t)grid * hd::kBlock * sizeof(float))) != hipSuccess) {
            rc = fail(e == hipErrorOutOfMemory ? HD_ENOMEM : HD_EDEVICE, "hd_probe_memory: %s", hipGetErrorString(e));
            break;
        }
        // defined contents (zeros); every value is read
        if ((e = hd::launch_fill_zero(a.as<float>(), (size_t)buf_bytes / 4, nullptr)) != hipSuccess) {
            rc = fail(HD_EDEVICE, "hd_probe_memory: %s", hipGetErrorString(e));
            break;
        }
        const int V = row_bytes / 256;
        const int64_t rows = buf_bytes / row_bytes;
        // as many rows gathered as the buffer holds, and at least 1 GiB of
        // them, so that a buffer small enough to stay in a cache still gives
        // a launch long enough to time
        const int64_t min_rows = ((int64_t)1 << 30) / row_bytes;
        const int64_t ngather = rows > min_rows ? rows : min_rows;
        if (mode == 2) {
            if ((e = ids.ensure((size_t)ngather * sizeof(int32_t))) != hipSuccess) {
                rc = fail(e == hipErrorOutOfMemory ? HD_ENOMEM : HD_EDEVICE, "hd_probe_memory: %s", hipGetErrorString(e));
                break;
            }
            hd::k_probe_ids<<<grid, hd::kBlock>>>(ids.as<int32_t>(), ngather, rows, 12345u);
            if ((e = hipGetLastError()) != hipSuccess) {
                rc = fail(HD_EDEVICE, "hd_probe_memory: %s", hipGetErrorString(e));
                break;
            }
        }
        double moved = 0.0;
        auto launch = [&]() -> hipError_t {
            switch (mode) {
                case 0:
                    hd::k_probe_read<<<grid, hd::kBlock>>>(a.as<float4>(), (size_t)buf_bytes / 16, out.as<float>());
                    break;
                case 1:
                    hd::k_probe_copy<<<grid, hd::kBlock>>>(a.as<float4>(), b.as<float4>(), (size_t)buf_bytes / 16);
                    break;
                case 2:
                    if (V == 1) hd::k_probe_gather<1><<<grid, hd::kBlock>>>(a.as<float>(), ids.as<int32_t>(), ngather, out.as<float>());
                    else if (V == 2) hd::k_probe_gather<2><<<grid, hd::kBlock>>>(a.as<float>(), ids.as<int32_t>(), ngather, out.as<float>());
                    else hd::k_probe_gather<4><<<grid, hd::kBlock>>>(a.as<float>(), ids.as<int32_t>(), ngather, out.as<float>());
                    break;
                default:
                    if (V == 1) hd::k_probe_graph<1><<<grid, hd::kBlock>>>(c->n, c->rowptr.as<int64_t>(), c->col.as<int32_t>(), a.as<float>(), out.as<float>());
                    else if (V == 2) hd::k_probe_graph<2><<<grid, hd::kBlock>>>(c->n, c->rowptr.as<int64_t>(), c->col.as<int32_t>(), a.as<float>(), out.as<float>());
                    else hd::k_probe_graph<4><<<grid, hd::kBlock>>>(c->n, c->rowptr.as<int64_t>(), c->col.as<int32_t>(), a.as<float>(), out.as<float>());
                    break;
            }
            return hipGetLastError();
        };
        switch (mode) {
            case 0: moved = (double)buf_bytes; break;
            case 1: moved = 2.0 * (double)buf_bytes; break;
            case 2: moved = (double)ngather * (row_bytes + 4); break;
            default: moved = (double)c->nnz * row_bytes + 12.0 * (double)c->n + 4.0 * (double)c->nnz; break;
        }
        if ((e = launch()) != hipSuccess || (e = hipDeviceSynchronize()) != hipSuccess) {
            rc = fail(HD_EDEVICE, "hd_probe_memory: %s", hipGetErrorString(e));
            break;
        }
        if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess ||
            (e = hipEventRecord(e0, nullptr)) != hipSuccess) {
            rc = fail(HD_EDEVICE, "hd_probe_memory: %s", hipGetErrorString(e));
            break;
        }
        for (int k = 0; k < reps && e == hipSuccess; ++k) e = launch();
        float ms = 0.f;
        if (e != hipSuccess || (e = hipEventRecord(e1, nullptr)) != hipSuccess ||
            (e = hipEventSynchronize(e1)) != hipSuccess || (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) {
            rc = fail(HD_EDEVICE, "hd_probe_memory: %s", hipGetErrorString(e));
            break;
        }
        if (ms_out) *ms_out = (double)ms / reps;
        if (bytes_out) *bytes_out = moved;
    } while (0);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    cleanup();
    return rc;
}
