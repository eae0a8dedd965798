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

hipError_t launch_gather_rows(const float* A, int64_t lda, int32_t d, const int32_t* rows,
                              int64_t nrows, float* out, int64_t ldo, int64_t* ids_out,
                              hipStream_t st) {
    if (nrows <= 0) return hipSuccess;
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

// ------------------------------------------------------ stable counting sort
// Items 0..n-1 with keys in [0, nk) are ordered by (key, item).  Block b of
// the item range holds items [b * B, (b + 1) * B).  cnt[key * nblk + b] counts
// block b's items with that key; its exclusive scan in that (key-major) order
// is where block b's first item of the key goes.

__global__ __launch_bounds__(256) void csort_count_kernel(const int32_t* keys, int64_t n,
                                                          int32_t nk, int32_t B, int32_t nblk,
                                                          int32_t* cnt) {
    extern __shared__ int32_t hist[];
    const int b = blockIdx.x;
    for (int r = threadIdx.x; r < nk; r += 256) hist[r] = 0;
    __syncthreads();
    const int64_t i0 = (int64_t)b * B;
    const int64_t i1 = i0 + B < n ? i0 + B : n;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) atomicAdd(&hist[keys[i]], 1);
    __syncthreads();
    for (int r = threadIdx.x; r < nk; r += 256) cnt[(int64_t)r * nblk + b] = hist[r];
}

// In-place exclusive scan of total int32 values by one workgroup of 1024
// threads (each thread scans a contiguous chunk).
__global__ __launch_bounds__(1024) void scan_1wg_kernel(int32_t* v, int64_t total) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t chunk = (total + 1023) / 1024;
    const int64_t s = t * chunk;
    const int64_t e = s + chunk < total ? s + chunk : total;
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
}

// Stable scatter: items of block b are placed in id order; inside a chunk of
// 256 items an item's rank among equal keys is the number of lower threads
// holding the same key.
__global__ __launch_bounds__(256) void csort_scatter_kernel(const int32_t* keys, int64_t n,
                                                            int32_t nk, int32_t B, int32_t nblk,
                                                            const int32_t* start, int32_t* perm) {
    extern __shared__ int32_t run[];
    __shared__ int32_t ck[256];
    const int b = blockIdx.x;
    const int t = threadIdx.x;
    for (int r = t; r < nk; r += 256) run[r] = start[(int64_t)r * nblk + b];
    __syncthreads();
    const int64_t i0 = (int64_t)b * B;
    const int64_t i1 = i0 + B < n ? i0 + B : n;
    for (int64_t base = i0; base < i1; base += 256) {
        const int64_t i = base + t;
        const int32_t key = i < i1 ? keys[i] : -1;
        ck[t] = key;
        __syncthreads();
        int rank = 0;
        bool last = true;
        if (key >= 0) {
            for (int j = 0; j < t; ++j) rank += ck[j] == key ? 1 : 0;
            for (int j = t + 1; j < 256; ++j) last = last && ck[j] != key;
            perm[run[key] + rank] = (int32_t)i;
        }
        __syncthreads();
        if (key >= 0 && last) run[key] += rank + 1;
        __syncthreads();
    }
}

// offsets[r] = first position of key r, offsets[nk] = n.
__global__ void csort_offsets_kernel(const int32_t* start, int32_t nk, int32_t nblk, int64_t n,
                                     int32_t* offsets) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nk) offsets[r] = start[(int64_t)r * nblk];
    if (r == nk) offsets[nk] = (int32_t)n;
}

int csort_blocks(int64_t n) { return (int)((n + kSortBlock - 1) / kSortBlock); }

hipError_t launch_csort(const int32_t* keys, int64_t n, int32_t nk, int32_t* cnt, int32_t* perm,
                        int32_t* offsets, hipStream_t st) {
    const int nblk = csort_blocks(n);
    const size_t lds = (size_t)nk * sizeof(int32_t);
    hipLaunchKernelGGL(csort_count_kernel, dim3(nblk), dim3(256), lds, st, keys, n, nk,
                       kSortBlock, nblk, cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scan_1wg_kernel, dim3(1), dim3(1024), 0, st, cnt, (int64_t)nk * nblk);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(csort_scatter_kernel, dim3(nblk), dim3(256), lds, st, keys, n, nk,
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

// ------------------------------------------------------------- list radii
// psi_r = max over the points x owned by r of rho(x, r) (Sec. 4), in float64
// with the fixed summation order; the maximum is taken on the bit patterns of
// non-negative doubles, which order like the values.
__global__ void psi_kernel(const float* X, int64_t ldx, int32_t d, int32_t metric, int64_t n,
                           const int32_t* owner, const float* R, int64_t ldr,
                           unsigned long long* psi_bits) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t r = owner[i];
    const double v = rho_fp64(X + i * ldx, R + (int64_t)r * ldr, d, metric);
    atomicMax(psi_bits + r, (unsigned long long)__double_as_longlong(v));
}

hipError_t launch_psi(const float* X, int64_t ldx, int32_t d, int32_t metric, int64_t n,
                      const int32_t* owner, const float* R, int64_t ldr, double* psi,
                      hipStream_t st) {
    hipLaunchKernelGGL(psi_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, X, ldx, d,
                       metric, n, owner, R, ldr, (unsigned long long*)psi);
    return hipGetLastError();
}

// --------------------------------------------------------------- stage 1
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
    for (int r0 = 0; r0 < nr; r0 += 32) {
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
    for (int r0 = 0; r0 < nr; r0 += 32) {
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
    const dim3 grid((m + 255) / 256);
    // the register path needs 16-byte aligned representative rows
    const int ks = (ldr % 4 == 0 && ((uintptr_t)R & 15) == 0) ? (d + 15) / 16 : 0;
    if (metric == 0)
        launch_dist_ks<0>(ks, grid, st, Q, ldq, m, R, ldr, nr, d, DR, ldd);
    else
        launch_dist_ks<1>(ks, grid, st, Q, ldq, m, R, ldr, nr, d, DR, ldd);
    return hipGetLastError();
}

// ------------------------------------------------------- pruning (Sec. 5.2)
// One wavefront per query.  gamma_1 = the smallest representative distance
// (its position is the query's nearest representative), gamma_k = the k-th
// smallest (+inf when k > n_r), found by a bitwise search over the float bit
// patterns (non-negative floats order like their bits).  The stored fp32
// distances are within a relative delta of the true ones, so the rules are
// applied to lower bounds of rho(q, r) and upper bounds of gamma:
//   prune r when  lo(q, r) - psi_r > gamma_k_up          (rule 1, strict)
//             or  lo(q, r) > 2 gamma_k_up + gamma_1_up    (rule 2, k-NN form)
// A superset of the exactly-kept lists is kept, so the answer is unchanged.
__global__ __launch_bounds__(256) void prune_kernel(const float* DR, int64_t ldd, int32_t m,
                                                    int32_t nr, int32_t k, double delta,
                                                    const double* psi,
                                                    const int32_t* list_off, uint8_t* keep,
                                                    int32_t* nearest, int64_t* stats) {
    const int lane = threadIdx.x & 63;
    const int q = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (q >= m) return;
    const float* row = DR + (int64_t)q * ldd;

    // gamma_1 and its position
    float bv = RBC_INF;
    int32_t bi = 0x7fffffff;
    for (int r = lane; r < nr; r += 64) {
        const float v = row[r];
        if (v < bv) {
            bv = v;
            bi = r;
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const float ov = __shfl_xor(bv, off);
        const int32_t oi = __shfl_xor(bi, off);
        if (ov < bv || (ov == bv && oi < bi)) {
            bv = ov;
            bi = oi;
        }
    }
    const float g1 = bv;
    // gamma_k: smallest bit pattern p with count(v <= p) >= k
    float gk = RBC_INF;
    if (k <= nr) {
        uint32_t prefix = 0;
        for (int bit = 31; bit >= 0; --bit) {
            const uint32_t trial = prefix | (1u << bit);
            // count of values strictly below trial
            int c = 0;
            for (int r = lane; r < nr; r += 64) c += __float_as_uint(row[r]) < trial ? 1 : 0;
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off);
            if (c < k) prefix = trial;
        }
        gk = __uint_as_float(prefix);
    }
    const double g1_up = (double)g1 * (1.0 + delta);
    const double gk_up = (double)gk * (1.0 + delta);
    const double bound2 = 2.0 * gk_up + g1_up;
    int nkept = 0;
    int64_t ncand = 0;
    for (int r = lane; r < nr; r += 64) {
        const double lo = (double)row[r] * (1.0 - delta);
        const double ps = psi[r] * (1.0 + 1e-15);
        const bool prune = (lo - ps > gk_up) || (lo > bound2);
        keep[(int64_t)q * nr + r] = prune ? 0 : 1;
        if (!prune) {
            ++nkept;
            ncand += list_off[r + 1] - list_off[r];
        }
    }
    if (lane == 0) nearest[q] = bi;
    if (stats) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            nkept += __shfl_xor(nkept, off);
            ncand += __shfl_xor(ncand, off);
        }
        if (lane == 0) {
            atomicAdd((unsigned long long*)&stats[3], (unsigned long long)nkept);
            atomicAdd((unsigned long long*)&stats[4], (unsigned long long)ncand);
        }
    }
}

hipError_t launch_prune(const float* DR, int64_t ldd, int32_t m, int32_t nr, int32_t k,
                        double delta, const double* psi, const int32_t* list_off, uint8_t* keep,
                        int32_t* nearest, int64_t* stats, hipStream_t st) {
    hipLaunchKernelGGL(prune_kernel, dim3((m + 3) / 4), dim3(256), 0, st, DR, ldd, m, nr, k, delta,
                       psi, list_off, keep, nearest, stats);
    return hipGetLastError();
}

// ------------------------------------------------- per-block union of lists
// For query block b (slots b*256 ..), the representatives kept by at least one
// of its queries, in ascending order, and the running row count before each.
__global__ __launch_bounds__(256) void block_union_kernel(const uint8_t* keep, const int32_t* qmap,
                                                          int32_t m, int32_t nr,
                                                          const int32_t* list_off,
                                                          int32_t* blk_reps, int32_t* blk_cnt,
                                                          int64_t* blk_pre) {
    extern __shared__ uint8_t flags[];
    __shared__ int32_t cpart[256];
    __shared__ int64_t rpart[256];
    const int b = blockIdx.x;
    const int t = threadIdx.x;
    for (int r = t; r < nr; r += 256) flags[r] = 0;
    __syncthreads();
    const int slot = b * 256 + t;
    if (slot < m) {
        const uint8_t* kr = keep + (int64_t)qmap[slot] * nr;
        for (int r = 0; r < nr; ++r)
            if (kr[r]) flags[r] = 1;
    }
    __syncthreads();
    // thread t owns the representative range [t * chunk, (t + 1) * chunk)
    const int chunk = (nr + 255) / 256;
    const int r0 = t * chunk;
    const int r1 = r0 + chunk < nr ? r0 + chunk : nr;
    int c = 0;
    int64_t rows = 0;
    for (int r = r0; r < r1; ++r)
        if (flags[r]) {
            ++c;
            rows += list_off[r + 1] - list_off[r];
        }
    cpart[t] = c;
    rpart[t] = rows;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int32_t ca = t >= off ? cpart[t - off] : 0;
        const int64_t ra = t >= off ? rpart[t - off] : 0;
        __syncthreads();
        cpart[t] += ca;
        rpart[t] += ra;
        __syncthreads();
    }
    int pos = t > 0 ? cpart[t - 1] : 0;
    int64_t pre = t > 0 ? rpart[t - 1] : 0;
    int32_t* reps = blk_reps + (int64_t)b * nr;
    int64_t* prefix = blk_pre + (int64_t)b * (nr + 1);
    for (int r = r0; r < r1; ++r)
        if (flags[r]) {
            reps[pos] = r;
            prefix[pos] = pre;
            ++pos;
            pre += list_off[r + 1] - list_off[r];
        }
    if (t == 255) {
        blk_cnt[b] = cpart[255];
        prefix[cpart[255]] = rpart[255];
    }
}

hipError_t launch_block_union(const uint8_t* keep, const int32_t* qmap, int32_t m, int32_t nr,
                              const int32_t* list_off, int32_t* blk_reps, int32_t* blk_cnt,
                              int64_t* blk_pre, hipStream_t st) {
    const int nblk = (m + 255) / 256;
    hipLaunchKernelGGL(block_union_kernel, dim3(nblk), dim3(256), (size_t)nr, st, keep, qmap, m, nr,
                       list_off, blk_reps, blk_cnt, blk_pre);
    return hipGetLastError();
}

}  // namespace rbc
