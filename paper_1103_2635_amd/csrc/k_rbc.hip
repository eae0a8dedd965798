#include <algorithm>
// k_rbc.hip -- kernels of the Random Ball Cover build and search that are not
// distance tiles: row gathers, a stable counting sort (ownership lists and
// query grouping), the list radii psi_r, the representative distances of
// stage 1, the pruning rules, and the per-query-block union of kept lists.
#include "rbc_device.h"
#include "rbc_kernels.h"

namespace rbc {

// ---------------------------------------------------------------- gathers

// out[i][0 .. ldo) = A[rows[i]][0 .. d) then zeros; ids_out[i] = rows[i].
__global__ void gather_rows_kernel(const float* A, int64_t lda, int32_t d, const int32_t* rows,
                                   int64_t nrows, float* out, int64_t ldo, int64_t* ids_out) {
    const int64_t total = nrows * ldo;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / ldo;
        const int64_t c = e - i * ldo;
        const int64_t src = rows[i];
        out[e] = c < d ? A[src * lda + c] : 0.f;
        if (c == 0 && ids_out) ids_out[i] = src;
    }
}

// Float4 form (d, lda, ldo multiples of 4, A 16-byte aligned): one float4
// per thread.
__global__ void gather_rows4_kernel(const float* A, int64_t lda4, int32_t d4, const int32_t* rows,
                                    int64_t nrows, float* out, int64_t ldo4, int64_t* ids_out) {
    const int64_t total = nrows * ldo4;
    const f4 z = {0.f, 0.f, 0.f, 0.f};
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / ldo4;
        const int64_t c = e - i * ldo4;
        const int64_t src = rows[i];
        ((f4*)out)[e] = c < d4 ? ((const f4*)A)[src * lda4 + c] : z;
        if (c == 0 && ids_out) ids_out[i] = src;
    }
}

hipError_t launch_gather_rows(const float* A, int64_t lda, int32_t d, const int32_t* rows,
                              int64_t nrows, float* out, int64_t ldo, int64_t* ids_out,
                              hipStream_t st) {
    if (nrows <= 0) return hipSuccess;
    if (d % 4 == 0 && lda % 4 == 0 && ldo % 4 == 0 && ((uintptr_t)A & 15) == 0 &&
        ((uintptr_t)out & 15) == 0) {
        int64_t blocks = (nrows * (ldo / 4) + 255) / 256;
        if (blocks > 65536) blocks = 65536;
        hipLaunchKernelGGL(gather_rows4_kernel, dim3((unsigned)blocks), dim3(256), 0, st, A,
                           lda / 4, d / 4, rows, nrows, out, ldo / 4, ids_out);
        return hipGetLastError();
    }
    int64_t blocks = (nrows * ldo + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, st, A, lda, d,
                       rows, nrows, out, ldo, ids_out);
    return hipGetLastError();
}

// int64 column 0 of an [n][k] int64 array (k = 1 owner output) -> int32.
__global__ void narrow_kernel(const int64_t* in, int64_t n, int32_t* out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = (int32_t)in[i];
}

hipError_t launch_narrow(const int64_t* in, int64_t n, int32_t* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(narrow_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, n,
                       out);
    return hipGetLastError();
}

// In-place exclusive scan of v[0 .. n) by one workgroup; v[n] = the total.
__global__ __launch_bounds__(1024) void scan_total_kernel(int32_t* v, int64_t n) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t chunk = (n + 1023) / 1024;
    const int64_t s = t * chunk;
    const int64_t e = s + chunk < n ? s + chunk : n;
    int64_t acc = 0;
    for (int64_t i = s; i < e; ++i) acc += v[i];
    part[t] = acc;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t add = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    int64_t run = t > 0 ? part[t - 1] : 0;
    for (int64_t i = s; i < e; ++i) {
        const int32_t x = v[i];
        v[i] = (int32_t)run;
        run += x;
    }
    if (t == 1023) v[n] = (int32_t)part[1023];
}

// ------------------------------------------------------ stable counting sort
// Items 0..n-1 with keys in [0, nk) are ordered by (key, item).  Block b of
// the item range holds items [b * B, (b + 1) * B) and is handled by one
// wavefront.  cnt[key * nblk + b] counts block b's items with that key; its
// exclusive scan in that (key-major) order is where block b's first item of
// the key goes.

__global__ __launch_bounds__(64) void csort_count_kernel(const int32_t* keys, int64_t n,
                                                         int32_t nk, int32_t B, int32_t nblk,
                                                         int32_t* cnt) {
    extern __shared__ int32_t hist[];
    const int b = blockIdx.x;
    for (int r = threadIdx.x; r < nk; r += 64) hist[r] = 0;
    __syncthreads();
    const int64_t i0 = (int64_t)b * B;
    const int64_t i1 = i0 + B < n ? i0 + B : n;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 64) atomicAdd(&hist[keys[i]], 1);
    __syncthreads();
    for (int r = threadIdx.x; r < nk; r += 64) cnt[(int64_t)r * nblk + b] = hist[r];
}

// Stable scatter: chunks of 64 items in id order; a lane's rank among equal
// keys of its chunk is the number of lower lanes holding the same key, and
// the highest such lane advances the running position of the key.
__global__ __launch_bounds__(64) void csort_scatter_kernel(const int32_t* keys, int64_t n,
                                                           int32_t nk, int32_t B, int32_t nblk,
                                                           const int32_t* start, int32_t* perm) {
    extern __shared__ int32_t run[];
    const int b = blockIdx.x;
    const int t = threadIdx.x;
    for (int r = t; r < nk; r += 64) run[r] = start[(int64_t)r * nblk + b];
    __syncthreads();
    const int64_t i0 = (int64_t)b * B;
    const int64_t i1 = i0 + B < n ? i0 + B : n;
    for (int64_t base = i0; base < i1; base += 64) {
        const int64_t i = base + t;
        const int32_t key = i < i1 ? keys[i] : -1;
        int rank = 0;
        bool last = true;
#pragma unroll
        for (int j = 0; j < 64; ++j) {  // constant source lanes: scalar lane reads
            const int32_t kj = __builtin_amdgcn_readlane(key, j);
            if (kj == key) {
                if (j < t) ++rank;
                if (j > t) last = false;
            }
        }
        wave_lds_sync();
        if (key >= 0) perm[run[key] + rank] = (int32_t)i;
        wave_lds_sync();
        if (key >= 0 && last) run[key] += rank + 1;
        wave_lds_sync();
    }
}

// Parallel exclusive scan of int32 values (totals below 2^31): per-block
// scans of 2048 values, a scan of the block sums, then the block offsets.
constexpr int kScanBlock = 2048;

__global__ __launch_bounds__(256) void scan_local_kernel(int32_t* v, int64_t n, int32_t* sums) {
    __shared__ int32_t part[256];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + t * 8;
    int32_t x[8];
    int32_t acc = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        x[j] = base + j < n ? v[base + j] : 0;
        acc += x[j];
    }
    part[t] = acc;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int32_t add = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    int32_t run = t ? part[t - 1] : 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if (base + j < n) v[base + j] = run;
        run += x[j];
    }
    if (t == 255) sums[blockIdx.x] = part[255];
}

__global__ __launch_bounds__(256) void scan_add_kernel(int32_t* v, int64_t n, const int32_t* sums) {
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * 8;
    const int32_t add = sums[blockIdx.x];
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if (base + j < n) v[base + j] += add;
}

// In-place exclusive scan of n values; v[n] receives the total when
// with_total is set.  sums needs ceil(n / 2048) + 1 entries.
hipError_t launch_scan(int32_t* v, int64_t n, int32_t* sums, bool with_total, hipStream_t st) {
    const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    if (nb <= 1) {
        hipLaunchKernelGGL(scan_total_kernel, dim3(1), dim3(1024), 0, st, v, n);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(scan_local_kernel, dim3((unsigned)nb), dim3(256), 0, st, v, n, sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scan_total_kernel, dim3(1), dim3(1024), 0, st, sums, nb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(scan_add_kernel, dim3((unsigned)nb), dim3(256), 0, st, v, n,
                       (const int32_t*)sums);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (with_total) {
        // v[n] = sums[nb] (the grand total written by the sums scan)
        e = hipMemcpyAsync(v + n, sums + nb, sizeof(int32_t), hipMemcpyDeviceToDevice, st);
    }
    return e;
}

// offsets[r] = first position of key r, offsets[nk] = n.
__global__ void csort_offsets_kernel(const int32_t* start, int32_t nk, int32_t nblk, int64_t n,
                                     int32_t* offsets) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nk) offsets[r] = start[(int64_t)r * nblk];
    if (r == nk) offsets[nk] = (int32_t)n;
}

int csort_blocks(int64_t n) { return (int)((n + kSortBlock - 1) / kSortBlock); }
int64_t csort_scratch(int64_t n, int32_t nk) {
    const int64_t cells = (int64_t)nk * csort_blocks(n);
    return cells + (cells + kScanBlock - 1) / kScanBlock + 2;
}

hipError_t launch_csort(const int32_t* keys, int64_t n, int32_t nk, int32_t* cnt, int32_t* perm,
                        int32_t* offsets, hipStream_t st) {
    const int nblk = csort_blocks(n);
    const int64_t cells = (int64_t)nk * nblk;
    const size_t lds = (size_t)nk * sizeof(int32_t);
    hipLaunchKernelGGL(csort_count_kernel, dim3(nblk), dim3(64), lds, st, keys, n, nk,
                       kSortBlock, nblk, cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = launch_scan(cnt, cells, cnt + cells, false, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(csort_scatter_kernel, dim3(nblk), dim3(64), lds, st, keys, n, nk,
                       kSortBlock, nblk, (const int32_t*)cnt, perm);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (offsets) {
        hipLaunchKernelGGL(csort_offsets_kernel, dim3((nk + 1 + 255) / 256), dim3(256), 0, st,
                           (const int32_t*)cnt, nk, nblk, n, offsets);
        e = hipGetLastError();
    }
    return e;
}

// ------------------------------------------------ grouping without order
// Items 0..n-1 grouped by key: offsets[k] .. offsets[k + 1] hold the items
// of key k, in no particular order inside a group (for groupings whose
// consumers do not depend on that order).  cursor: nk int32 scratch.
__global__ __launch_bounds__(256) void group_count_kernel(const int32_t* keys, int64_t n,
                                                          int32_t* cnt) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        atomicAdd(cnt + keys[i], 1);
}

__global__ __launch_bounds__(256) void group_fill_kernel(const int32_t* keys, int64_t n,
                                                         const int32_t* offsets, int32_t* cursor,
                                                         int32_t* perm) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256) {
        const int32_t k = keys[i];
        perm[offsets[k] + atomicAdd(cursor + k, 1)] = (int32_t)i;
    }
}

hipError_t launch_group(const int32_t* keys, int64_t n, int32_t nk, int32_t* cursor,
                        int32_t* perm, int32_t* offsets, hipStream_t st) {
    hipError_t e;
    if ((e = launch_fill_i32(offsets, nk + 1, 0, st)) != hipSuccess) return e;
    if ((e = launch_fill_i32(cursor, nk, 0, st)) != hipSuccess) return e;
    const int64_t blocks = std::min<int64_t>(1024, (n + 255) / 256);
    if (blocks > 0) {
        hipLaunchKernelGGL(group_count_kernel, dim3((unsigned)blocks), dim3(256), 0, st, keys, n,
                           offsets);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if ((e = launch_scan_total(offsets, nk, st)) != hipSuccess) return e;
    if (blocks > 0) {
        hipLaunchKernelGGL(group_fill_kernel, dim3((unsigned)blocks), dim3(256), 0, st, keys, n,
                           (const int32_t*)offsets, cursor, perm);
        e = hipGetLastError();
    }
    return e;
}

// ------------------------------------------------------------- list radii
// psi_r from the lists sorted by own = rho(x, r) (the fp32 distances of the
// ownership search, relative error <= delta): the float64 maximum can only
// be held by rows with own >= max(own) (1 - 2 delta), a suffix of a sorted
// list (unsorted lists are screened whole); those rows are scored again in
// float64 (the fixed order of rho_fp64) and psi_r is their maximum, equal to
// the maximum over the whole list.  One workgroup per list; empty lists get 0.
__global__ __launch_bounds__(256) void psi_own_kernel(const float* Xp, int64_t ld, int32_t d,
                                                      int32_t metric, const float* own,
                                                      const int32_t* list_off,
                                                      const int32_t* lsorted, const float* R,
                                                      int64_t ldr, double delta, double* psi) {
    __shared__ float s_max[4];
    __shared__ double s_psi[4];
    const int r = blockIdx.x;
    const int b = list_off[r], e = list_off[r + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (b == e) {
        if (tid == 0) psi[r] = 0.0;
        return;
    }
    const bool sorted = lsorted[r] != 0;
    float m32 = 0.f;
    if (sorted) {
        m32 = own[e - 1];
    } else {
        for (int j = b + tid; j < e; j += 256) m32 = fmaxf(m32, own[j]);
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) m32 = fmaxf(m32, __shfl_xor(m32, off));
        if (lane == 0) s_max[wave] = m32;
        __syncthreads();
        m32 = fmaxf(fmaxf(s_max[0], s_max[1]), fmaxf(s_max[2], s_max[3]));
    }
    const double thr = (double)m32 * (1.0 - 2.0 * delta);
    const float* rp = R + (int64_t)r * ldr;
    double best = 0.0;
    if (sorted) {
        for (int j = e - 1 - tid; j >= b; j -= 256) {
            if ((double)own[j] < thr) break;
            best = fmax(best, rho_fp64(Xp + (int64_t)j * ld, rp, d, metric));
        }
    } else {
        for (int j = b + tid; j < e; j += 256)
            if ((double)own[j] >= thr) best = fmax(best, rho_fp64(Xp + (int64_t)j * ld, rp, d, metric));
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) best = fmax(best, __shfl_xor(best, off));
    if (lane == 0) s_psi[wave] = best;
    __syncthreads();
    if (tid == 0) psi[r] = fmax(fmax(s_psi[0], s_psi[1]), fmax(s_psi[2], s_psi[3]));
}

hipError_t launch_psi_own(const float* Xp, int64_t ld, int32_t d, int32_t metric, const float* own,
                          const int32_t* list_off, const int32_t* lsorted, const float* R,
                          int64_t ldr, int32_t nr, double* psi, hipStream_t st) {
    const double delta = 2.0 * (d + 2) * 5.9604644775390625e-8;
    hipLaunchKernelGGL(psi_own_kernel, dim3(nr), dim3(256), 0, st, Xp, ld, d, metric, own,
                       list_off, lsorted, R, ldr, delta, psi);
    return hipGetLastError();
}

// xn[i] = qn[perm[i]] (the squared norms the ownership search computed for
// the rows of X), the largest norm as float bits (atomic max, one per
// workgroup) and a copy of the 3 value-flag words.
__global__ __launch_bounds__(256) void gather_norms_kernel(const float* qn, const int32_t* perm,
                                                           int64_t n, float* xn, uint32_t* maxbits,
                                                           const uint32_t* flags_in,
                                                           uint32_t* flags_out) {
    __shared__ float wmax[4];
    float m = 0.f;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float v = qn[perm[i]];
        xn[i] = v;
        m = fmaxf(m, __builtin_sqrtf(v));
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t v = __float_as_uint(fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3])));
        if (__atomic_load_n(maxbits, __ATOMIC_RELAXED) < v) atomicMax(maxbits, v);  // only grows
        if (blockIdx.x == 0)
            for (int w = 0; w < 3; ++w) flags_out[w] = flags_in[w];
    }
}

hipError_t launch_gather_norms(const float* qn, const int32_t* perm, int64_t n, float* xn,
                               uint32_t* maxbits, const uint32_t* flags_in, uint32_t* flags_out,
                               hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(gather_norms_kernel, dim3((unsigned)blocks), dim3(256), 0, st, qn, perm, n,
                       xn, maxbits, flags_in, flags_out);
    return hipGetLastError();
}

// --------------------------------------------------------------- stage 1
constexpr int kDistReps = 64;  // representatives per workgroup (a multiple of 32)
// DR[q][r] = rho(q, r) for every query and representative, fp32, direct
// differences (the BF(q, R) call of Sec. 5.2 keeps every distance).  One
// thread per query with the query in registers (d <= 128, KS 16-feature
// slabs) and 32 representatives at a time staged in LDS; rows of DR have
// stride ldd (a multiple of 4) and are written as float4.  d > 128 takes the
// generic kernel below (query features read from memory).
template <int METRIC, int KS>
__global__ __launch_bounds__(256) void dist_all_kernel(const float* Q, int64_t ldq, int32_t m,
                                                       const float* R, int64_t ldr, int32_t nr,
                                                       int32_t d, float* DR, int64_t ldd) {
    constexpr int F4 = 4 * KS;
    __shared__ f4 rs[32 * F4];
    const int q = blockIdx.x * 256 + threadIdx.x;
    const bool qv = q < m;
    const int rb0 = blockIdx.y * kDistReps;
    const int rb1 = rb0 + kDistReps < nr ? rb0 + kDistReps : nr;
    f4 qr[F4];
    {
        const float* qp = Q + (int64_t)(qv ? q : 0) * ldq;
#pragma unroll
        for (int j = 0; j < F4; ++j) {
            f4 v = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (4 * j + c < d) v[c] = qp[4 * j + c];
            qr[j] = v;
        }
    }
    for (int r0 = rb0; r0 < rb1; r0 += 32) {
        __syncthreads();
        for (int e = threadIdx.x; e < 32 * F4; e += 256) {
            const int rr = e / F4, cc = e - rr * F4;
            f4 v = {0.f, 0.f, 0.f, 0.f};
            if (r0 + rr < nr && 4 * cc < d) v = *(const f4*)(R + (int64_t)(r0 + rr) * ldr + 4 * cc);
            rs[e] = v;
        }
        __syncthreads();
        if (!qv) continue;
        float acc[32];
#pragma unroll
        for (int t = 0; t < 32; ++t) {
            f4 s4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int j = 0; j < F4; ++j) {
                const f4 df = qr[j] - rs[t * F4 + j];
                if (METRIC == 0) {
                    s4 = df * df + s4;
                } else {
                    s4[0] += __builtin_fabsf(df[0]);
                    s4[1] += __builtin_fabsf(df[1]);
                    s4[2] += __builtin_fabsf(df[2]);
                    s4[3] += __builtin_fabsf(df[3]);
                }
            }
            const float v = (s4[0] + s4[1]) + (s4[2] + s4[3]);
            acc[t] = METRIC == 0 ? __builtin_sqrtf(v) : v;
        }
        float* out = DR + (int64_t)q * ldd + r0;
        if (r0 + 32 <= nr) {
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const f4 v = {acc[4 * t], acc[4 * t + 1], acc[4 * t + 2], acc[4 * t + 3]};
                *(f4*)(out + 4 * t) = v;
            }
        } else {
#pragma unroll
            for (int t = 0; t < 32; ++t)
                if (r0 + t < nr) out[t] = acc[t];
        }
    }
}

template <int METRIC>
__global__ __launch_bounds__(256) void dist_all_generic_kernel(const float* Q, int64_t ldq,
                                                               int32_t m, const float* R,
                                                               int64_t ldr, int32_t nr, int32_t d,
                                                               float* DR, int64_t ldd) {
    __shared__ float rs[32][129];
    const int q = blockIdx.x * 256 + threadIdx.x;
    const bool qv = q < m;
    const float* qp = Q + (int64_t)(qv ? q : 0) * ldq;
    const int rb0 = blockIdx.y * kDistReps;
    const int rb1 = rb0 + kDistReps < nr ? rb0 + kDistReps : nr;
    for (int r0 = rb0; r0 < rb1; r0 += 32) {
        float acc[32];
#pragma unroll
        for (int j = 0; j < 32; ++j) acc[j] = 0.f;
        for (int f0 = 0; f0 < d; f0 += 128) {
            const int fl = d - f0 < 128 ? d - f0 : 128;
            __syncthreads();
            for (int e = threadIdx.x; e < 32 * 128; e += 256) {
                const int rr = e >> 7, ff = e & 127;
                rs[rr][ff] = (r0 + rr < nr && ff < fl) ? R[(int64_t)(r0 + rr) * ldr + f0 + ff] : 0.f;
            }
            __syncthreads();
            if (qv) {
                for (int ff = 0; ff < fl; ++ff) {
                    const float qf = qp[f0 + ff];
#pragma unroll
                    for (int j = 0; j < 32; ++j) {
                        const float t = qf - rs[j][ff];
                        if (METRIC == 0)
                            acc[j] = __builtin_fmaf(t, t, acc[j]);
                        else
                            acc[j] += __builtin_fabsf(t);
                    }
                }
            }
        }
        if (qv) {
#pragma unroll
            for (int j = 0; j < 32; ++j)
                if (r0 + j < nr)
                    DR[(int64_t)q * ldd + r0 + j] = METRIC == 0 ? __builtin_sqrtf(acc[j]) : acc[j];
        }
    }
}

template <int METRIC>
static void launch_dist_ks(int ks, dim3 grid, hipStream_t st, const float* Q, int64_t ldq,
                           int32_t m, const float* R, int64_t ldr, int32_t nr, int32_t d,
                           float* DR, int64_t ldd) {
#define RBC_DIST_CASE(K)                                                                        \
    case K:                                                                                    \
        hipLaunchKernelGGL((dist_all_kernel<METRIC, K>), grid, dim3(256), 0, st, Q, ldq, m, R, \
                           ldr, nr, d, DR, ldd);                                               \
        return;
    switch (ks) {
        RBC_DIST_CASE(1)
        RBC_DIST_CASE(2)
        RBC_DIST_CASE(3)
        RBC_DIST_CASE(4)
        RBC_DIST_CASE(5)
        RBC_DIST_CASE(6)
        RBC_DIST_CASE(7)
        RBC_DIST_CASE(8)
    }
#undef RBC_DIST_CASE
    hipLaunchKernelGGL(dist_all_generic_kernel<METRIC>, grid, dim3(256), 0, st, Q, ldq, m, R, ldr,
                       nr, d, DR, ldd);
}

hipError_t launch_dist_all(int metric, const float* Q, int64_t ldq, int32_t m, const float* R,
                           int64_t ldr, int32_t nr, int32_t d, float* DR, int64_t ldd,
                           hipStream_t st) {
    const dim3 grid((m + 255) / 256, (nr + kDistReps - 1) / kDistReps);
    // the register path needs 16-byte aligned representative rows
    const int ks = (ldr % 4 == 0 && ((uintptr_t)R & 15) == 0) ? (d + 15) / 16 : 0;
    if (metric == 0)
        launch_dist_ks<0>(ks, grid, st, Q, ldq, m, R, ldr, nr, d, DR, ldd);
    else
        launch_dist_ks<1>(ks, grid, st, Q, ldq, m, R, ldr, nr, d, DR, ldd);
    return hipGetLastError();
}

// ------------------------------------------------------- pruning (Sec. 5.2)
// One wavefront per query.  gamma_1 = the smallest representative distance,
// gamma_k = the k-th smallest (+inf when k > n_r) and gamma_c = the c-th
// smallest (the shortlist length), found by a bitwise search over the float
// bit patterns (non-negative floats order like their bits).  The stored fp32
// distances are within a relative delta of the true ones, so the rules are
// applied to lower bounds of rho(q, r) and upper bounds of gamma:
//   prune r when  lo(q, r) - psi_r > gamma_k_up          (rule 1, strict)
//             or  lo(q, r) > 2 gamma_k_up + gamma_1_up    (rule 2, k-NN form)
// A superset of the exactly-kept lists is kept, so the answer is unchanged.
// Since R is a subset of X, gamma_c_up also bounds the distance of q's c-th
// nearest database point; it seeds the stage-2 shortlists.
// Outputs: lrank[q][r] = rank of r among the lists q keeps (-1: pruned),
// nkept[q], gcup[q].
// gamma_1 (the minimum) and the bit patterns of gamma_k and gamma_c: the
// smallest pattern p with count(v <= p) >= k (c).  V > 0: the lane's values
// (r = lane + 64 j, j < V) are held in registers (+inf pads), so the 32
// rounds of the bitwise search read no memory; V = 0: read every round.
template <int V>
__device__ __forceinline__ void select_gammas(const float* row, int nr, int k, int c, int lane,
                                              float& g1, uint32_t& pk, uint32_t& pc) {
    uint32_t vb[V > 0 ? V : 1];
    g1 = RBC_INF;
    if (V > 0) {
#pragma unroll
        for (int j = 0; j < (V > 0 ? V : 1); ++j) {
            const int r = lane + 64 * j;
            const float v = r < nr ? row[r] : RBC_INF;
            vb[j] = __float_as_uint(v);
            g1 = fminf(g1, v);
        }
    } else {
        for (int r = lane; r < nr; r += 64) g1 = fminf(g1, row[r]);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) g1 = fminf(g1, __shfl_xor(g1, off));
    pk = 0;
    pc = 0;
    for (int bit = 31; bit >= 0; --bit) {
        const uint32_t tk = pk | (1u << bit), tc = pc | (1u << bit);
        int ck = 0, cc = 0;
        if (V > 0) {
#pragma unroll
            for (int j = 0; j < (V > 0 ? V : 1); ++j) {
                ck += vb[j] < tk ? 1 : 0;
                cc += vb[j] < tc ? 1 : 0;
            }
        } else {
            for (int r = lane; r < nr; r += 64) {
                const uint32_t b = __float_as_uint(row[r]);
                ck += b < tk ? 1 : 0;
                cc += b < tc ? 1 : 0;
            }
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            ck += __shfl_xor(ck, off);
            cc += __shfl_xor(cc, off);
        }
        if (ck < k) pk = tk;
        if (cc < c) pc = tc;
    }
}

template <int V>
__global__ __launch_bounds__(256) void prune_kernel(const float* DR, int64_t ldd, int32_t m,
                                                    int32_t nr, int32_t k, int32_t c,
                                                    double delta, const double* psi,
                                                    const int32_t* list_off, int32_t* lrank,
                                                    int32_t* nkept, float* gcup, int64_t* stats,
                                                    double shrink, const float* taud) {
    const int lane = threadIdx.x & 63;
    const int q = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (q >= m) return;
    const float* row = DR + (int64_t)q * ldd;
    float g1;
    uint32_t pk, pc;
    select_gammas<V>(row, nr, k, c, lane, g1, pk, pc);
    const float gk = k <= nr ? __uint_as_float(pk) : RBC_INF;
    const float gc = c <= nr ? __uint_as_float(pc) : RBC_INF;
    const double g1_up = (double)g1 * (1.0 + delta);
    // shrink < 1: the approximate variant (bounds divided by 1 + eps)
    double gk_up = (double)gk * (1.0 + delta);
    // taud: a bound on the k-th neighbour distance from the query's nearest
    // list (two-pass search); any such bound may replace gamma_k in both rules
    if (taud && (double)taud[q] < gk_up) gk_up = (double)taud[q];
    const double bound2 = (2.0 * gk_up + g1_up) * shrink;
    const double bound1 = gk_up * shrink;
    int running = 0;
    int64_t ncand = 0;
    for (int base = 0; base < nr; base += 64) {
        const int r = base + lane;
        bool kept = false;
        if (r < nr) {
            const double lo = (double)row[r] * (1.0 - delta);
            const double ps = psi[r] * (1.0 + 1e-15);
            kept = !((lo - ps > bound1) || (lo > bound2));
        }
        const uint64_t bits = __ballot(kept);
        const uint64_t below = lane ? (bits & (~0ull >> (64 - lane))) : 0ull;
        if (r < nr) {
            lrank[(int64_t)q * nr + r] = kept ? running + __popcll(below) : -1;
            if (kept) ncand += list_off[r + 1] - list_off[r];
        }
        running += __popcll(bits);
    }
    if (lane == 0) {
        nkept[q] = running;
        gcup[q] = gc < RBC_INF ? (float)((double)gc * (1.0 + delta)) * (1.0f + 1e-6f) : RBC_INF;
    }
    if (stats) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) ncand += __shfl_xor(ncand, off);
        if (lane == 0) {
            atomicAdd((unsigned long long*)&stats[3], (unsigned long long)running);
            atomicAdd((unsigned long long*)&stats[4], (unsigned long long)ncand);
        }
    }
}

hipError_t launch_prune(const float* DR, int64_t ldd, int32_t m, int32_t nr, int32_t k, int32_t c,
                        double delta, const double* psi, const int32_t* list_off, int32_t* lrank,
                        int32_t* nkept, float* gcup, int64_t* stats, hipStream_t st,
                        double shrink, const float* taud) {
    const dim3 grid((m + 3) / 4);
    if (nr <= 1024)
        hipLaunchKernelGGL(prune_kernel<16>, grid, dim3(256), 0, st, DR, ldd, m, nr, k, c, delta,
                           psi, list_off, lrank, nkept, gcup, stats, shrink, taud);
    else if (nr <= 2048)
        hipLaunchKernelGGL(prune_kernel<32>, grid, dim3(256), 0, st, DR, ldd, m, nr, k, c, delta,
                           psi, list_off, lrank, nkept, gcup, stats, shrink, taud);
    else
        hipLaunchKernelGGL(prune_kernel<0>, grid, dim3(256), 0, st, DR, ldd, m, nr, k, c, delta,
                           psi, list_off, lrank, nkept, gcup, stats, shrink, taud);
    return hipGetLastError();
}

// ------------------------------------------------ two-pass exact search
// home[q] = the nearest representative of q (lowest position among equal
// stage-1 distances).  One wavefront per query.
__global__ __launch_bounds__(256) void nearest_rep_kernel(const float* DR, int64_t ldd, int32_t m,
                                                          int32_t nr, int32_t* home) {
    const int lane = threadIdx.x & 63;
    const int q = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (q >= m) return;
    const float* row = DR + (int64_t)q * ldd;
    float best = RBC_INF;
    int bi = 0x7fffffff;
    for (int r = lane; r < nr; r += 64) {
        const float v = row[r];
        if (v < best || (v == best && r < bi)) {
            best = v;
            bi = r;
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const float ob = __shfl_xor(best, off);
        const int oi = __shfl_xor(bi, off);
        if (ob < best || (ob == best && oi < bi)) {
            best = ob;
            bi = oi;
        }
    }
    if (lane == 0) home[q] = bi < nr ? bi : 0;
}

hipError_t launch_nearest_rep(const float* DR, int64_t ldd, int32_t m, int32_t nr, int32_t* home,
                              hipStream_t st) {
    hipLaunchKernelGGL(nearest_rep_kernel, dim3((m + 3) / 4), dim3(256), 0, st, DR, ldd, m, nr,
                       home);
    return hipGetLastError();
}

// taud[q]: an upper bound on the distance of q's k-th nearest database point,
// from the k-th smallest value v over the nsplit sorted shortlists that cover
// its nearest list (k rows have a tile value <= v): mode 0 (matrix tile, v ~ ||x||^2 - 2 q.x, absolute error <=
// 4 (d + 2) u (||q|| + max ||x||)^2, u = 2^-24): sqrt(v + E + ||q||^2
// (1 + (d + 2) u)); mode 1 (direct squared l2, relative error <= delta):
// sqrt(v / (1 - delta)); mode 2 (direct l1): v / (1 - delta); each widened
// by 1e-6 and rounded up to a float.  +inf when the list has fewer than k rows.

__global__ void tau_home_kernel(const float* hval, int32_t c, int32_t nsplit, int32_t k,
                                int32_t m, int32_t mode, const float* qn,
                                const uint32_t* xmax_bits, int32_t d, double delta, float* taud) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= m) return;
    const double u = 5.9604644775390625e-8;
    // k-way merge of the sorted shortlists: the k-th value taken
    const float* hv = hval + (int64_t)q * nsplit * c;
    int pos[kMaxHomeSplit];
    for (int s = 0; s < nsplit; ++s) pos[s] = 0;
    float v = RBC_INF;
    for (int t = 0; t < k; ++t) {
        int bs = -1;
        float bv = RBC_INF;
        for (int s = 0; s < nsplit; ++s)
            if (pos[s] < c && hv[s * c + pos[s]] < bv) {
                bv = hv[s * c + pos[s]];
                bs = s;
            }
        if (bs < 0) {
            v = RBC_INF;
            break;
        }
        ++pos[bs];
        v = bv;
    }
    double t = RBC_INF_D;
    if (v < RBC_INF) {
        if (mode == 0) {
            const double n2 = (double)qn[q];
            const double sq = __builtin_sqrt(n2) + (double)__uint_as_float(*xmax_bits);
            const double e = 4.0 * (d + 2) * u * sq * sq;
            t = __builtin_sqrt(fmax((double)v + e + n2 * (1.0 + (d + 2) * u), 0.0));
        } else if (mode == 1) {
            t = __builtin_sqrt(fmax((double)v / (1.0 - delta), 0.0));
        } else {
            t = fmax((double)v / (1.0 - delta), 0.0);
        }
        t *= 1.0 + 1e-6;
    }
    taud[q] = t < RBC_INF_D ? round_up_f(t) : RBC_INF;
}

hipError_t launch_tau_home(const float* hval, int32_t c, int32_t nsplit, int32_t k, int32_t m,
                           int32_t mode, const float* qn, const uint32_t* xmax_bits, int32_t d,
                           double delta, float* taud, hipStream_t st) {
    if (nsplit < 1 || nsplit > kMaxHomeSplit) return hipErrorInvalidValue;
    hipLaunchKernelGGL(tau_home_kernel, dim3((m + 255) / 256), dim3(256), 0, st, hval, c, nsplit,
                       k, m, mode, qn, xmax_bits, d, delta, taud);
    return hipGetLastError();
}

// Row range of every stage-2 item (two-pass search): a point x of L_r can be
// one of q's k nearest only when abs(rho(x, r) - rho(q, r)) <= taud[q]
// (triangle inequality).  With own(x) and the stage-1 rho(q, r) both within a
// relative rel of the exact distances, that holds only for own in
// [max(0, rho~/(1 + rel) - t) (1 - rel), (rho~/(1 - rel) + t) (1 + rel)]; a
// list sorted by own (lsorted[r]) keeps those rows in one run, and the item
// scans the run covering all of its queries: irows[2 i], irows[2 i + 1].
// Unsorted lists are scanned whole.  taud null: every query has the bound
// tconst (a range search radius).  One wavefront per item, grid-stride.
// With rec non-null the item's record is written as well (representative,
// first and end query position, row run, item).
// First position j in [L, R) of the ascending own[] with own[j] >= v
// (after_equal: own[j] > v), or R: a 64-way search, each lane probing one
// pivot per round, so a list of up to 262,144 rows needs three rounds of
// loads instead of eighteen dependent ones.
__device__ __forceinline__ int wave_bound(const float* own, int L, int R, double v,
                                          bool after_equal, int lane) {
    while (R - L > 64) {
        const int64_t span = R - L;
        const int s = L + (int)(span * lane / 64);
        const double x = (double)own[s];
        const bool below = after_equal ? x <= v : x < v;
        const int c = __popcll(__ballot(below));  // pivots before the answer (a prefix)
        if (c == 0) return L;                     // own[L] already at or past v
        // answer in (pivot c - 1, pivot c]; pivot 64 is R
        const int nl = L + (int)(span * (c - 1) / 64) + 1;
        const int nr = c < 64 ? L + (int)(span * c / 64) : R;
        L = nl;
        R = nr;
    }
    const int s = L + lane;
    bool below = false;
    if (s < R) {
        const double x = (double)own[s];
        below = after_equal ? x <= v : x < v;
    }
    return L + __popcll(__ballot(below));
}

__device__ __forceinline__ int item_cost(int nq, int lo, int hi) {
    const int c = (nq * ((hi - lo + 31) >> 5)) >> 3;
    return c < kCostBuckets - 1 ? c : kCostBuckets - 1;
}

__global__ __launch_bounds__(256) void item_rows_kernel(
    const int32_t* item_total, const int32_t* irep, const int32_t* ioff, const int32_t* roff,
    const int32_t* qlist, int32_t isize, const int32_t* list_off, const int32_t* lsorted,
    const float* own, const float* DR, int64_t ldd, const float* taud, double tconst,
    double rel, int32_t* irows, int32_t* rec) {
    const int lane = threadIdx.x & 63;
    const int total = *item_total;
    const int nwave = gridDim.x * 4;
    for (int item = blockIdx.x * 4 + (threadIdx.x >> 6); item < total; item += nwave) {
        const int r = irep[item];
        const int b = list_off[r], e = list_off[r + 1];
        int lo = b, hi = e;
        const int q_begin = roff[r] + (item - ioff[r]) * isize;
        const int q_end = min(q_begin + isize, roff[r + 1]);
        if (lsorted[r]) {
            double vlo = RBC_INF_D, vhi = 0.0;
            for (int p = q_begin + lane; p < q_end; p += 64) {
                const int q = qlist[p];
                const double rq = (double)DR[(int64_t)q * ldd + r];
                const double t = taud ? (double)taud[q] : tconst;
                double l = (rq / (1.0 + rel) - t) * (1.0 - rel);
                double h = (rq / (1.0 - rel) + t) * (1.0 + rel);
                if (!(l > 0.0)) l = 0.0;          // also NaN
                if (!(h < RBC_INF_D)) h = RBC_INF_D;
                vlo = fmin(vlo, l);
                vhi = fmax(vhi, h);
            }
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                vlo = fmin(vlo, __shfl_xor(vlo, off));
                vhi = fmax(vhi, __shfl_xor(vhi, off));
            }
            // first row with own >= vlo, first row with own > vhi
            lo = wave_bound(own, b, e, vlo, false, lane);
            hi = wave_bound(own, lo, e, vhi, true, lane);
        }
        if (lane == 0) {
            irows[2 * (int64_t)item] = lo;
            irows[2 * (int64_t)item + 1] = hi;
            if (rec) {
                int32_t* o = rec + (int64_t)kItemRec * item;
                *(int4*)o = make_int4(r, q_begin, q_end, lo);
                *(int4*)(o + 4) = make_int4(hi, item, 0, 0);
            }
        }
    }
}

// The records in descending cost class, one workgroup: class counts in LDS,
// their scan (largest class first), then each record copied to the next free
// position of its class (the order inside a class is not fixed; every item
// writes its own output slots).
__global__ __launch_bounds__(1024) void item_order_kernel(const int32_t* item_total,
                                                          const int32_t* rec, int32_t* srec) {
    __shared__ int32_t hist[kCostBuckets];
    __shared__ int32_t part[1024];
    constexpr int kPer = kCostBuckets / 1024;
    const int t = threadIdx.x;
    const int total = *item_total;
    for (int c = t; c < kCostBuckets; c += 1024) hist[c] = 0;
    __syncthreads();
    for (int item = t; item < total; item += 1024) {
        const int4 a = *(const int4*)(rec + (int64_t)kItemRec * item);
        const int hi = rec[(int64_t)kItemRec * item + 4];
        atomicAdd(&hist[item_cost(a.z - a.y, a.w, hi)], 1);
    }
    __syncthreads();
    // thread t owns classes kCostBuckets - 1 - kPer t - j (descending)
    int v[kPer], sum = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        v[j] = hist[kCostBuckets - 1 - kPer * t - j];
        sum += v[j];
    }
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int add = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    int base = part[t] - sum;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        hist[kCostBuckets - 1 - kPer * t - j] = base;
        base += v[j];
    }
    __syncthreads();
    for (int item = t; item < total; item += 1024) {
        const int4 a = *(const int4*)(rec + (int64_t)kItemRec * item);
        const int4 b = *(const int4*)(rec + (int64_t)kItemRec * item + 4);
        const int pos = atomicAdd(&hist[item_cost(a.z - a.y, a.w, b.x)], 1);
        *(int4*)(srec + (int64_t)kItemRec * pos) = a;
        *(int4*)(srec + (int64_t)kItemRec * pos + 4) = b;
    }
}

hipError_t launch_item_order(const int32_t* item_total, const int32_t* rec, int32_t* srec,
                             hipStream_t st) {
    hipLaunchKernelGGL(item_order_kernel, dim3(1), dim3(1024), 0, st, item_total, rec, srec);
    return hipGetLastError();
}

hipError_t launch_item_rows(const int32_t* item_total, const int32_t* irep, const int32_t* ioff,
                            const int32_t* roff, const int32_t* qlist, int32_t isize,
                            const int32_t* list_off, const int32_t* lsorted, const float* own,
                            const float* DR, int64_t ldd, const float* taud, double tconst,
                            double rel, int32_t* irows, hipStream_t st, int32_t* rec) {
    hipLaunchKernelGGL(item_rows_kernel, dim3(1024), dim3(256), 0, st, item_total, irep, ioff,
                       roff, qlist, isize, list_off, lsorted, own, DR, ldd, taud, tconst, rel,
                       irows, rec);
    return hipGetLastError();
}

// ------------------------------------------------ segmented sort (LDS)
// Segment s = vals[off[s] .. off[s + 1]) is reordered by ascending key, ties
// kept in their current order: key of the element at position j is
// keys[vals[j]] (ldk == 0) or keys[vals[j] * ldk + s] (ldk > 0).  Keys are
// non-negative floats (their bit patterns order like the values).  One
// workgroup per segment, bitonic network over (key bits, position) in LDS;
// segments longer than kSegCap are left as they are and flagged 0 in
// sorted (optional), the others 1.
__global__ __launch_bounds__(1024) void seg_sort_kernel(const int32_t* off, int32_t* vals,
                                                        const float* keys, int64_t ldk,
                                                        int32_t* sorted) {
    __shared__ uint64_t key[kSegCap];
    const int sg = blockIdx.x;
    const int b = off[sg];
    const int len = off[sg + 1] - b;
    if (len > kSegCap) {
        if (sorted && threadIdx.x == 0) sorted[sg] = 0;
        return;
    }
    if (sorted && threadIdx.x == 0) sorted[sg] = 1;
    if (len <= 1) return;
    int size = 1;
    while (size < len) size <<= 1;
    for (int i = threadIdx.x; i < size; i += blockDim.x) {
        uint64_t kv = ~0ull;
        if (i < len) {
            const int64_t v = vals[b + i];
            const float f = ldk > 0 ? keys[v * ldk + sg] : keys[v];
            kv = ((uint64_t)__float_as_uint(f) << 32) | (uint32_t)i;
        }
        key[i] = kv;
    }
    __syncthreads();
    // bitonic network; thread t takes compare-exchange pairs t, t + 1024, ...
    // of each stage: pair t joins element i (t with a zero bit inserted at j)
    // and i + j, so every thread has work in every stage
    const int half = size >> 1;
    for (int kk = 2; kk <= size; kk <<= 1) {
        for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < half; t += blockDim.x) {
                const int i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
                const int p = i | j;
                const bool up = (i & kk) == 0;
                const uint64_t a = key[i], c = key[p];
                if ((a > c) == up) {
                    key[i] = c;
                    key[p] = a;
                }
            }
            __syncthreads();
        }
    }
    // gather the values in key order (all reads before any write)
    int32_t got[kSegCap / 1024];
#pragma unroll
    for (int t = 0; t < kSegCap / 1024; ++t) {
        const int i = threadIdx.x + t * 1024;
        got[t] = i < len ? vals[b + (int)(key[i] & 0xffffffffu)] : 0;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kSegCap / 1024; ++t) {
        const int i = threadIdx.x + t * 1024;
        if (i < len) vals[b + i] = got[t];
    }
}

hipError_t launch_seg_sort(const int32_t* off, int32_t nseg, int32_t* vals, const float* keys,
                           int64_t ldk, int32_t* sorted, hipStream_t st) {
    if (nseg <= 0) return hipSuccess;
    hipLaunchKernelGGL(seg_sort_kernel, dim3(nseg), dim3(1024), 0, st, off, vals, keys, ldk,
                       sorted);
    return hipGetLastError();
}

// ---------------------------------------------------------- range search
// Pruning for a range query (radius eps): a point x of L_r has rho(q, x) >=
// rho(q, r) - rho(x, r) >= rho(q, r) - psi_r, so L_r can hold a point within
// eps only when rho(q, r) - psi_r <= eps; applied to the lower bound of the
// stored fp32 rho(q, r).  One wavefront per query; lrank as for k-NN pruning.
__global__ __launch_bounds__(256) void prune_range_kernel(const float* DR, int64_t ldd, int32_t m,
                                                          int32_t nr, double delta,
                                                          const double* psi, double radius,
                                                          int32_t* lrank, int32_t* nkept,
                                                          int64_t* stats) {
    const int lane = threadIdx.x & 63;
    const int q = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (q >= m) return;
    const float* row = DR + (int64_t)q * ldd;
    int running = 0;
    for (int base = 0; base < nr; base += 64) {
        const int r = base + lane;
        bool kept = false;
        if (r < nr) {
            // lower bound of rho(q, r) from the fp32 value; the float64
            // difference is given a relative 1e-12 of slack (NaN keeps the list)
            const double lo = (double)row[r] * (1.0 - delta), pr = psi[r];
            kept = !(lo - pr > radius + 1e-12 * (lo + pr + radius));
        }
        const uint64_t bits = __ballot(kept);
        const uint64_t below = lane ? (bits & (~0ull >> (64 - lane))) : 0ull;
        if (r < nr) lrank[(int64_t)q * nr + r] = kept ? running + __popcll(below) : -1;
        running += __popcll(bits);
    }
    if (lane == 0) {
        nkept[q] = running;
        if (stats) atomicAdd((unsigned long long*)&stats[3], (unsigned long long)running);
    }
}

hipError_t launch_prune_range(const float* DR, int64_t ldd, int32_t m, int32_t nr, double delta,
                              const double* psi, double radius, int32_t* lrank, int32_t* nkept,
                              int64_t* stats, hipStream_t st) {
    hipLaunchKernelGGL(prune_range_kernel, dim3((m + 3) / 4), dim3(256), 0, st, DR, ldd, m, nr,
                       delta, psi, radius, lrank, nkept, stats);
    return hipGetLastError();
}

// off[0] = 0, off[i + 1] = off[i] + cnt[i] (int64), one workgroup.
__global__ __launch_bounds__(1024) void offsets64_kernel(const int32_t* cnt, int64_t m,
                                                         int64_t* off) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t per = (m + 1023) / 1024;
    const int64_t b = t * per, e = b + per < m ? b + per : m;
    int64_t sum = 0;
    for (int64_t i = b; i < e; ++i) sum += cnt[i];
    part[t] = sum;
    __syncthreads();
    for (int step = 1; step < 1024; step <<= 1) {
        const int64_t v = t >= step ? part[t - step] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = part[t] - sum;  // exclusive
    for (int64_t i = b; i < e; ++i) {
        off[i] = run;
        run += cnt[i];
    }
    if (t == 1023) off[m] = part[1023];
}

hipError_t launch_offsets64(const int32_t* cnt, int64_t m, int64_t* off, hipStream_t st) {
    hipLaunchKernelGGL(offsets64_kernel, dim3(1), dim3(1024), 0, st, cnt, m, off);
    return hipGetLastError();
}

// Each segment off[s] .. off[s + 1] of (dist, idx) pairs sorted by (dist,
// idx) (with cnt: only segments whose length equals cnt[s]; the others are
// counted in *bad and left as they are): keys (dist bits << 32 | idx) with dist >= 0 and 0 <= idx < 2^31.  A
// bitonic network in the form that needs no direction flags (a "flip" step
// then half-cleaners, all ascending), so a non-power-of-two length just skips
// the comparisons with partners beyond the end (virtual +inf there never
// moves).  Segments up to kSegCap run in LDS, longer ones in place in global
// memory (same network, one workgroup).
__global__ __launch_bounds__(1024) void seg_sort_pairs_kernel(const int64_t* off, int64_t* idx,
                                                              float* dist, const int32_t* cnt,
                                                              int32_t* bad) {
    __shared__ uint64_t key[kSegCap];
    const int64_t b = off[blockIdx.x];
    const int64_t len = off[blockIdx.x + 1] - b;
    if (cnt && cnt[blockIdx.x] != len) {  // segment not filled exactly: left unsorted
        if (threadIdx.x == 0) atomicAdd(bad, 1);
        return;
    }
    if (len <= 1) return;
    const bool lds = len <= kSegCap;
    int64_t size = 1;
    while (size < len) size <<= 1;
    auto get = [&](int64_t i) -> uint64_t {
        return ((uint64_t)__float_as_uint(dist[b + i]) << 32) | (uint32_t)idx[b + i];
    };
    if (lds) {
        for (int64_t i = threadIdx.x; i < len; i += blockDim.x) key[i] = get(i);
        __syncthreads();
    }
    for (int64_t kk = 2; kk <= size; kk <<= 1) {
        for (int64_t j = kk >> 1; j > 0; j >>= 1) {
            for (int64_t i = threadIdx.x; i < len; i += blockDim.x) {
                // first step of a stage compares mirrored partners, later ones i ^ j
                const int64_t p = j == (kk >> 1) ? (i ^ (kk - 1)) : (i ^ j);
                if (p > i && p < len) {
                    if (lds) {
                        const uint64_t x = key[i], y = key[p];
                        if (x > y) {
                            key[i] = y;
                            key[p] = x;
                        }
                    } else {
                        const uint64_t x = get(i), y = get(p);
                        if (x > y) {
                            dist[b + i] = __uint_as_float((uint32_t)(y >> 32));
                            idx[b + i] = (int64_t)(uint32_t)y;
                            dist[b + p] = __uint_as_float((uint32_t)(x >> 32));
                            idx[b + p] = (int64_t)(uint32_t)x;
                        }
                    }
                }
            }
            if (!lds) __threadfence_block();
            __syncthreads();
        }
    }
    if (lds)
        for (int64_t i = threadIdx.x; i < len; i += blockDim.x) {
            dist[b + i] = __uint_as_float((uint32_t)(key[i] >> 32));
            idx[b + i] = (int64_t)(uint32_t)key[i];
        }
}

hipError_t launch_seg_sort_pairs(const int64_t* off, int64_t nseg, int64_t* idx, float* dist,
                                 const int32_t* cnt, int32_t* bad, hipStream_t st) {
    if (nseg <= 0) return hipSuccess;
    hipLaunchKernelGGL(seg_sort_pairs_kernel, dim3((unsigned)nseg), dim3(1024), 0, st, off, idx,
                       dist, cnt, bad);
    return hipGetLastError();
}

// keep_rq[r][q] = (lrank[q][r] >= 0), through 64 x 64 LDS tiles so that both
// the reads and the writes are contiguous.
__global__ __launch_bounds__(256) void keep_transpose_kernel(const int32_t* lrank, int32_t m,
                                                             int32_t nr, uint8_t* keep_rq) {
    __shared__ uint8_t tile[64][65];
    const int q0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int qi = e >> 6, ri = e & 63;
        const int q = q0 + qi, r = r0 + ri;
        tile[qi][ri] = (q < m && r < nr && lrank[(int64_t)q * nr + r] >= 0) ? 1 : 0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int ri = e >> 6, qi = e & 63;
        const int q = q0 + qi, r = r0 + ri;
        if (q < m && r < nr) keep_rq[(int64_t)r * m + q] = tile[qi][ri];
    }
}

hipError_t launch_keep_transpose(const int32_t* lrank, int32_t m, int32_t nr, uint8_t* keep_rq,
                                 hipStream_t st) {
    hipLaunchKernelGGL(keep_transpose_kernel, dim3((m + 63) / 64, (nr + 63) / 64), dim3(256), 0, st,
                       lrank, m, nr, keep_rq);
    return hipGetLastError();
}

// ------------------------------------------------ stage-2 work list (items)
// Per representative (one wavefront each): how many queries kept it, and the
// number of isize-query items it makes.
__global__ __launch_bounds__(256) void rep_count_kernel(const uint8_t* keep_rq, int32_t m,
                                                        int32_t nr, int32_t isize, int32_t* cnt,
                                                        int32_t* nitems) {
    const int lane = threadIdx.x & 63;
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= nr) return;
    const uint8_t* kr = keep_rq + (int64_t)r * m;
    int c = 0;
    for (int q = lane; q < m; q += 64) c += kr[q];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off);
    if (lane == 0) {
        cnt[r] = c;
        nitems[r] = (c + isize - 1) / isize;
    }
}

// The queries that kept r, ascending, at qlist[roff[r] ..].
__global__ __launch_bounds__(256) void rep_fill_kernel(const uint8_t* keep_rq, int32_t m,
                                                       int32_t nr, const int32_t* roff,
                                                       int32_t* qlist) {
    const int lane = threadIdx.x & 63;
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= nr) return;
    const uint8_t* kr = keep_rq + (int64_t)r * m;
    int pos = roff[r];
    for (int base = 0; base < m; base += 64) {
        const int q = base + lane;
        const bool kept = q < m && kr[q] != 0;
        const uint64_t bits = __ballot(kept);
        const uint64_t below = lane ? (bits & (~0ull >> (64 - lane))) : 0ull;
        if (kept) qlist[pos + __popcll(below)] = q;
        pos += __popcll(bits);
    }
}

// The same two passes reading 16 keep bytes per lane (m a multiple of 16,
// rows 16-byte aligned): a row of 10^4 queries takes 10 loads per lane
// instead of 157.
__device__ __forceinline__ int bytes_sum(uint32_t w) { return (int)((w * 0x01010101u) >> 24); }

__global__ __launch_bounds__(256) void rep_count16_kernel(const uint8_t* keep_rq, int32_t m,
                                                          int32_t nr, int32_t isize, int32_t* cnt,
                                                          int32_t* nitems) {
    const int lane = threadIdx.x & 63;
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= nr) return;
    const uint4* kr = (const uint4*)(keep_rq + (int64_t)r * m);
    int c = 0;
    for (int j = lane; j < m / 16; j += 64) {
        const uint4 w = kr[j];
        c += bytes_sum(w.x) + bytes_sum(w.y) + bytes_sum(w.z) + bytes_sum(w.w);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off);
    if (lane == 0) {
        cnt[r] = c;
        nitems[r] = (c + isize - 1) / isize;
    }
}

__global__ __launch_bounds__(256) void rep_fill16_kernel(const uint8_t* keep_rq, int32_t m,
                                                         int32_t nr, const int32_t* roff,
                                                         int32_t* qlist) {
    const int lane = threadIdx.x & 63;
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= nr) return;
    const uint4* kr = (const uint4*)(keep_rq + (int64_t)r * m);
    int pos = roff[r];
    for (int base = 0; base < m / 16; base += 64) {
        const int j = base + lane;
        uint4 w = {0u, 0u, 0u, 0u};
        if (j < m / 16) w = kr[j];
        const int c = bytes_sum(w.x) + bytes_sum(w.y) + bytes_sum(w.z) + bytes_sum(w.w);
        // exclusive prefix of the lane counts (queries stay in ascending order)
        int incl = c;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int t = __shfl_up(incl, off);
            if (lane >= off) incl += t;
        }
        int at = pos + incl - c;
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if ((ws[k >> 2] >> (8 * (k & 3))) & 0xffu) qlist[at++] = 16 * j + k;
        }
        pos += __shfl(incl, 63);
    }
}

hipError_t launch_scan_total(int32_t* v, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(scan_total_kernel, dim3(1), dim3(1024), 0, st, v, n);
    return hipGetLastError();
}

hipError_t launch_worklist(const uint8_t* keep_rq, int32_t m, int32_t nr, int32_t isize,
                           int32_t* roff, int32_t* ioff, int32_t* qlist, hipStream_t st) {
    const dim3 grid((nr + 3) / 4);
    const bool w16 = (m % 16) == 0 && ((uintptr_t)keep_rq & 15) == 0;
    if (w16)
        hipLaunchKernelGGL(rep_count16_kernel, grid, dim3(256), 0, st, keep_rq, m, nr, isize, roff,
                           ioff);
    else
        hipLaunchKernelGGL(rep_count_kernel, grid, dim3(256), 0, st, keep_rq, m, nr, isize, roff,
                           ioff);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = launch_scan_total(roff, nr, st)) != hipSuccess) return e;
    if ((e = launch_scan_total(ioff, nr, st)) != hipSuccess) return e;
    if (w16)
        hipLaunchKernelGGL(rep_fill16_kernel, grid, dim3(256), 0, st, keep_rq, m, nr,
                           (const int32_t*)roff, qlist);
    else
        hipLaunchKernelGGL(rep_fill_kernel, grid, dim3(256), 0, st, keep_rq, m, nr,
                           (const int32_t*)roff, qlist);
    return hipGetLastError();
}

// Stage-2 shortlist threshold per query, in the value space of the tile:
//   mode 0 (matrix-core l2, values ||x||^2 - 2 q.x):
//        gc^2 - ||q||^2 + 2 E,  E = 4 (d + 2) u (||q|| + max ||x||)^2
//   mode 1 (direct l2, values d^2):  gc^2 (1 + delta)
//   mode 2 (direct l1, values rho):  gc (1 + delta)
//   mode 3 (matrix core on quantised rows, ||x~||^2 - 2 q~.x~): a row within
//        gc of q is within gc + ||q - q~|| + max ||x - x~|| of q~, so
//        (gc + e_q + e_x)^2 - ||q~||^2 + 2 E with E on the quantised norms
// each widened by a relative 4e-6; +inf when gc is.
__global__ void tau_kernel(const float* gcup, const float* qn, const uint32_t* xmax_bits,
                           const uint32_t* flags_q, const uint32_t* flags_x, int32_t m, int32_t d,
                           int32_t mode, double delta, const float* qerr,
                           const uint32_t* xerr_bits, float* tau) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= m) return;
    const double gc = (double)gcup[q];
    float t = RBC_INF;
    if (gc < RBC_INF_D) {
        double v;
        if (mode == 0) {
            const double n2 = (double)qn[q];
            const double sq = __builtin_sqrt(n2) + (double)__uint_as_float(*xmax_bits);
            const double e = tile_exact(flags_q, flags_x, d)
                                 ? 0.0
                                 : 4.0 * (d + 2) * 5.9604644775390625e-8 * sq * sq;
            v = gc * gc * (1.0 + 4e-6) - n2 + 2.0 * e;
        } else if (mode == 3) {
            const double n2 = (double)qn[q];
            const double sq = __builtin_sqrt(n2) + (double)__uint_as_float(*xmax_bits);
            const double e = 4.0 * (d + 2) * 5.9604644775390625e-8 * sq * sq;
            const double g = gc + (double)qerr[q] + (double)__uint_as_float(*xerr_bits);
            v = g * g * (1.0 + 4e-6) - n2 + 2.0 * e;
        } else if (mode == 1) {
            v = gc * gc * (1.0 + delta) * (1.0 + 4e-6);
        } else {
            v = gc * (1.0 + delta) * (1.0 + 4e-6);
        }
        t = (float)v;
    }
    tau[q] = t;
}

hipError_t launch_tau(const float* gcup, const float* qn, const uint32_t* xmax_bits,
                      const uint32_t* flags_q, const uint32_t* flags_x, int32_t m, int32_t d,
                      int32_t mode, double delta, float* tau, hipStream_t st, const float* qerr,
                      const uint32_t* xerr_bits) {
    hipLaunchKernelGGL(tau_kernel, dim3((m + 255) / 256), dim3(256), 0, st, gcup, qn, xmax_bits,
                       flags_q, flags_x, m, d, mode, delta, qerr, xerr_bits, tau);
    return hipGetLastError();
}

}  // namespace rbc
