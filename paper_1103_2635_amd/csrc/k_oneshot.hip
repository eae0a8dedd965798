// k_oneshot.hip -- one-shot RBC build (Sec. 4, Sec. 5.1): every
// representative owns its s nearest database points.
//
// For a chunk of representatives the tile writes every value (BF(R, X) with
// all distances kept) to a value matrix V[rep][row].  Per representative:
//   1. the s-th smallest value is located by two 12-bit radix histograms over
//      order-preserving keys of the fp32 values (bits 31..20, then 19..8 of the
//      keys under the chosen prefix), giving a value T >= the s-th one;
//   2. every row with value <= T + margin (the tile's rounding bound, so no
//      true member of the list is missed) is collected;
//   3. the candidates are scored again in float64 in the fixed order and
//      sorted by (distance, id); the first s are the list, the s-th distance
//      is psi_r.
#include "rbc_device.h"
#include "rbc_kernels.h"

namespace rbc {

// Order-preserving map of fp32 values to uint32 keys (larger value, larger key).
__device__ __forceinline__ uint32_t okey(float v) {
    const uint32_t b = __float_as_uint(v);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ float okey_value(uint32_t k) {
    const uint32_t b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(b);
}

constexpr int kHistBins = 4096;
constexpr int kHistRows = 65536;  // rows per histogram workgroup

// pass 0: bins of key >> 20; pass 1: bins of (key >> 8) & 0xfff among keys
// whose top 12 bits equal prefix[rep].
__global__ __launch_bounds__(256) void os_hist_kernel(const float* V, int64_t ldv, int32_t n,
                                                      int32_t pass, const uint32_t* prefix,
                                                      uint32_t* hist) {
    __shared__ uint32_t h[kHistBins];
    const int rep = blockIdx.x;
    for (int b = threadIdx.x; b < kHistBins; b += 256) h[b] = 0;
    __syncthreads();
    const float* row = V + (int64_t)rep * ldv;
    const int r0 = blockIdx.y * kHistRows;
    const int r1 = r0 + kHistRows < n ? r0 + kHistRows : n;
    const uint32_t pre = pass ? prefix[rep] : 0u;
    for (int i = r0 + threadIdx.x; i < r1; i += 256) {
        const uint32_t k = okey(row[i]);
        if (pass == 0) {
            atomicAdd(&h[k >> 20], 1u);
        } else if ((k >> 20) == pre) {
            atomicAdd(&h[(k >> 8) & 0xfffu], 1u);
        }
    }
    __syncthreads();
    uint32_t* out = hist + (int64_t)rep * kHistBins;
    for (int b = threadIdx.x; b < kHistBins; b += 256)
        if (h[b]) atomicAdd(out + b, h[b]);
}

// Per representative: the bin holding the need[rep]-th smallest key
// (need = s before pass 0).  Writes the bin into prefix (pass 0) or the final
// bound T into tval (pass 1) and the remaining rank into need.
__global__ __launch_bounds__(256) void os_select_kernel(const uint32_t* hist, int32_t pass,
                                                        uint32_t* prefix, int32_t* need,
                                                        float* tval) {
    __shared__ uint32_t part[256];
    __shared__ uint32_t s_want;
    const int rep = blockIdx.x;
    const int t = threadIdx.x;
    if (t == 0) s_want = (uint32_t)need[rep];
    const uint32_t* h = hist + (int64_t)rep * kHistBins;
    constexpr int per = kHistBins / 256;
    uint32_t local[per];
    uint32_t sum = 0;
#pragma unroll
    for (int j = 0; j < per; ++j) {
        local[j] = h[t * per + j];
        sum += local[j];
    }
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint32_t add = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    const uint32_t before = t ? part[t - 1] : 0;
    const uint32_t want = s_want;
    if (before < want && want <= part[t]) {
        uint32_t run = before;
        for (int j = 0; j < per; ++j) {
            if (run + local[j] >= want) {
                const uint32_t bin = (uint32_t)(t * per + j);
                need[rep] = (int32_t)(want - run);
                if (pass == 0) {
                    prefix[rep] = bin;
                } else {
                    const uint32_t key = (prefix[rep] << 20) | (bin << 8) | 0xffu;
                    tval[rep] = okey_value(key);
                }
                break;
            }
            run += local[j];
        }
    }
}

// Rows whose value is at most bound[rep] go to cand[rep][...] (count in
// cnt[rep]; entries beyond cap are counted, not stored).
__global__ __launch_bounds__(256) void os_collect_kernel(const float* V, int64_t ldv, int32_t n,
                                                         const float* bound, int32_t cap,
                                                         int32_t* cnt, int32_t* cand) {
    const int rep = blockIdx.x;
    const float* row = V + (int64_t)rep * ldv;
    const float b = bound[rep];
    const int r0 = blockIdx.y * kHistRows;
    const int r1 = r0 + kHistRows < n ? r0 + kHistRows : n;
    for (int i = r0 + threadIdx.x; i < r1; i += 256) {
        if (row[i] <= b) {
            const int p = atomicAdd(cnt + rep, 1);
            if (p < cap) cand[(int64_t)rep * cap + p] = i;
        }
    }
}

// bound[rep] = T + margin in the tile's value space:
//   mode 0 (matrix core, ||x||^2 - 2 r.x): T + 2 E, E = 4 (d + 2) u (||r|| + max ||x||)^2
//   mode 1/2 (direct d^2 or rho, non-negative): T (1 + 2 delta)
//   no margin when the tile's values are exact for these inputs (tile_exact)
__global__ void os_bound_kernel(const float* tval, const float* rnorm2, const uint32_t* xmax_bits,
                                const uint32_t* flags, int32_t reps, int32_t d, int32_t mode,
                                double delta, float* bound) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= reps) return;
    const double t = (double)tval[r];
    // exact tile values (matrix-core l2, or l1 sums of integers) need no margin
    const bool exact = mode != 1 && tile_exact(flags, flags, d);
    double b;
    if (exact) {
        b = t;
    } else if (mode == 0) {
        const double sq = __builtin_sqrt((double)rnorm2[r]) + (double)__uint_as_float(*xmax_bits);
        b = t + 2.0 * 4.0 * (d + 2) * 5.9604644775390625e-8 * sq * sq;
    } else {
        b = t * (1.0 + 2.0 * delta);
    }
    bound[r] = exact ? (float)b : (float)b * (1.0f + 1e-6f) + 1e-30f;
}

// Float64 re-score of the candidates and an LDS bitonic sort by (distance,
// id); the first s ids form the list, psi = the s-th distance.  One
// workgroup of 1024 threads per representative; cap <= kOsCap.
__global__ __launch_bounds__(1024) void os_sort_kernel(const float* X, int64_t ldx, int32_t d,
                                                       int32_t metric, const float* R, int64_t ldr,
                                                       const int32_t* cnt, const int32_t* cand,
                                                       int32_t cap, int32_t s, int32_t rep0,
                                                       int32_t* lists, double* psi,
                                                       int32_t* overflow) {
    __shared__ double key[kOsCap];
    __shared__ int32_t id[kOsCap];
    const int rep = blockIdx.x;
    const int count = cnt[rep];
    if (count > cap) {
        if (threadIdx.x == 0) atomicAdd(overflow, 1);
        return;
    }
    int size = 1;
    while (size < count) size <<= 1;
    const float* rp = R + (int64_t)(rep0 + rep) * ldr;
    for (int i = threadIdx.x; i < size; i += blockDim.x) {
        if (i < count) {
            const int row = cand[(int64_t)rep * cap + i];
            key[i] = rho_fp64(rp, X + (int64_t)row * ldx, d, metric);
            id[i] = row;
        } else {
            key[i] = RBC_INF_D;
            id[i] = 0x7fffffff;
        }
    }
    __syncthreads();
    // bitonic network, one compare-exchange pair per thread and pass: pair t
    // joins element i (t with a zero bit inserted at j) and i + j
    for (int kk = 2; kk <= size; kk <<= 1) {
        for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < (size >> 1); t += blockDim.x) {
                const int i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
                const int p = i | j;
                const bool up = (i & kk) == 0;
                const bool gt = key[i] > key[p] || (key[i] == key[p] && id[i] > id[p]);
                if (gt == up) {
                    const double tk = key[i];
                    key[i] = key[p];
                    key[p] = tk;
                    const int32_t ti = id[i];
                    id[i] = id[p];
                    id[p] = ti;
                }
            }
            __syncthreads();
        }
    }
    int32_t* out = lists + (int64_t)(rep0 + rep) * s;
    for (int i = threadIdx.x; i < s; i += blockDim.x) out[i] = id[i];
    if (threadIdx.x == 0) psi[rep0 + rep] = key[s - 1];
}

hipError_t launch_oneshot_select(const float* V, int64_t ldv, int32_t n, int32_t reps, int32_t s,
                                 int32_t mode, double delta, int32_t d, const float* rnorm2,
                                 const uint32_t* xmax_bits, const uint32_t* flags, OneShotWork& w,
                                 hipStream_t st) {
    const dim3 g2(reps, (n + kHistRows - 1) / kHistRows);
    hipError_t e;
    if ((e = launch_fill_i32((int32_t*)w.hist, (int64_t)reps * kHistBins, 0, st))) return e;
    if ((e = launch_fill_i32(w.need, reps, s, st))) return e;
    hipLaunchKernelGGL(os_hist_kernel, g2, dim3(256), 0, st, V, ldv, n, 0, (const uint32_t*)w.prefix,
                       w.hist);
    if ((e = hipGetLastError())) return e;
    hipLaunchKernelGGL(os_select_kernel, dim3(reps), dim3(256), 0, st, (const uint32_t*)w.hist, 0,
                       w.prefix, w.need, w.tval);
    if ((e = hipGetLastError())) return e;
    if ((e = launch_fill_i32((int32_t*)w.hist, (int64_t)reps * kHistBins, 0, st))) return e;
    hipLaunchKernelGGL(os_hist_kernel, g2, dim3(256), 0, st, V, ldv, n, 1, (const uint32_t*)w.prefix,
                       w.hist);
    if ((e = hipGetLastError())) return e;
    hipLaunchKernelGGL(os_select_kernel, dim3(reps), dim3(256), 0, st, (const uint32_t*)w.hist, 1,
                       w.prefix, w.need, w.tval);
    if ((e = hipGetLastError())) return e;
    hipLaunchKernelGGL(os_bound_kernel, dim3((reps + 255) / 256), dim3(256), 0, st,
                       (const float*)w.tval, rnorm2, xmax_bits, flags, reps, d, mode, delta,
                       w.bound);
    if ((e = hipGetLastError())) return e;
    if ((e = launch_fill_i32(w.cnt, reps, 0, st))) return e;
    hipLaunchKernelGGL(os_collect_kernel, g2, dim3(256), 0, st, V, ldv, n,
                       (const float*)w.bound, kOsCap, w.cnt, w.cand);
    return hipGetLastError();
}

hipError_t launch_oneshot_sort(const float* X, int64_t ldx, int32_t d, int32_t metric,
                               const float* R, int64_t ldr, int32_t reps, int32_t s, int32_t rep0,
                               OneShotWork& w, int32_t* lists, double* psi, hipStream_t st) {
    hipLaunchKernelGGL(os_sort_kernel, dim3(reps), dim3(1024), 0, st, X, ldx, d, metric, R, ldr,
                       (const int32_t*)w.cnt, (const int32_t*)w.cand, kOsCap, s, rep0, lists, psi,
                       w.overflow);
    return hipGetLastError();
}

// One-shot search work list: items per representative from the query counts
// (offsets of the queries grouped by nearest representative).
__global__ void os_items_kernel(const int32_t* roff, int32_t nr, int32_t isize, int32_t mult,
                                int32_t* nitems) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nr) nitems[r] = (roff[r + 1] - roff[r] + isize - 1) / isize * mult;
}

hipError_t launch_items_from_offsets(const int32_t* roff, int32_t nr, int32_t isize,
                                     int32_t* ioff, hipStream_t st, int32_t mult) {
    hipLaunchKernelGGL(os_items_kernel, dim3((nr + 255) / 256), dim3(256), 0, st, roff, nr, isize,
                       mult, ioff);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_scan_total(ioff, nr, st);
}

// list_off[r] = r * s (one-shot lists are stored back to back).
__global__ void os_offsets_kernel(int32_t* off, int32_t nr, int32_t s) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r <= nr) off[r] = r * s;
}

hipError_t launch_list_offsets(int32_t* off, int32_t nr, int32_t s, hipStream_t st) {
    hipLaunchKernelGGL(os_offsets_kernel, dim3((nr + 1 + 255) / 256), dim3(256), 0, st, off, nr, s);
    return hipGetLastError();
}

}  // namespace rbc
