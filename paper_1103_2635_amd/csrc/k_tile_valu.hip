// k_tile_valu.hip -- distance tile on the vector ALUs (l1, and l2 in direct
// form for small d or when the matrix-core path is not used).
//
// One lane per query: the query's d features live in registers, the
// workgroup stages 32 database rows at a time in LDS (coalesced float4 loads),
// and every lane walks the staged rows with broadcast LDS reads, accumulating
// sum (q_i - x_i)^2 (l2, squared distance) or sum |q_i - x_i| (l1) in fp32 --
// two VALU operations per feature.  The per-query top-c shortlist is the same
// register list as on the matrix-core path.
#include "rbc_device.h"

#ifndef RBC_KS
#error "compile with -DRBC_KS=<1..8>"
#endif

namespace rbc {

// Scan database rows [r0, r1): the workgroup stages 32 rows at a time, every
// lane with act scores them against its query.  Called by all 256 threads.
template <int METRIC, int KS, int C>
__device__ __forceinline__ void valu_scan(const f4 (&q)[4 * KS], const float* X, int64_t ldx,
                                          int d, int r0, int r1, bool act, TopC<C>& top,
                                          f4* xs) {
    constexpr int F4 = 4 * KS;
    const int tid = threadIdx.x;
    for (int base = r0; base < r1; base += kRowsValu) {
        __syncthreads();
        for (int e = tid; e < kRowsValu * F4; e += 256) {
            const int rr = e / F4, cc = e - rr * F4;
            const int row = base + rr;
            f4 v = {0.f, 0.f, 0.f, 0.f};
            if (row < r1 && 4 * cc < d) v = *(const f4*)(X + (int64_t)row * ldx + 4 * cc);
            xs[e] = v;
        }
        __syncthreads();
        if (act) {
            const int nrow = r1 - base < kRowsValu ? r1 - base : kRowsValu;
            for (int t = 0; t < nrow; ++t) {
                f4 s = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int j = 0; j < F4; ++j) {
                    const f4 df = q[j] - xs[t * F4 + j];
                    if (METRIC == 0) {
                        s = df * df + s;
                    } else {
                        s[0] += __builtin_fabsf(df[0]);
                        s[1] += __builtin_fabsf(df[1]);
                        s[2] += __builtin_fabsf(df[2]);
                        s[3] += __builtin_fabsf(df[3]);
                    }
                }
                top.push((s[0] + s[1]) + (s[2] + s[3]), base + t);
            }
        }
    }
}

template <int KS>
__device__ __forceinline__ void valu_load_q(f4 (&q)[4 * KS], const float* Q, int64_t ldq, int d,
                                            int row) {
    const float* qp = Q + (int64_t)row * ldq;
#pragma unroll
    for (int j = 0; j < 4 * KS; ++j) {
        f4 v = {0.f, 0.f, 0.f, 0.f};
        if (4 * j < d) v = *(const f4*)(qp + 4 * j);
        q[j] = v;
    }
}

template <int METRIC, int KS, int C>
__global__ __launch_bounds__(256, 2) void tile_valu(TileArgs a) {
    __shared__ f4 xs[kRowsValu * 4 * KS];
    const int myslot = blockIdx.x * kTileQ + threadIdx.x;
    const bool qvalid = myslot < a.m;
    f4 q[4 * KS];
    valu_load_q<KS>(q, a.Q, a.ldq, a.d, qvalid ? myslot : a.m - 1);
    TopC<C> top;
    top.init();
    const int64_t r0 = (int64_t)blockIdx.y * a.rps;
    const int64_t r1 = r0 + a.rps < a.n ? r0 + a.rps : a.n;
    if (r0 < r1) valu_scan<METRIC, KS, C>(q, a.X, a.ldx, a.d, (int)r0, (int)r1, qvalid, top, xs);
    if (qvalid) {
        const int64_t off = ((int64_t)blockIdx.y * a.m + myslot) * C;
        top.store(a.pval + off, a.pidx + off);
    }
}

// Exact RBC stage 2 on the vector ALUs: persistent workgroups take
// (representative, 256-query chunk) items from the queue.
template <int METRIC, int KS, int C>
__global__ __launch_bounds__(256, 2) void tile_valu_items(TileArgs a) {
    __shared__ f4 xs[kRowsValu * 4 * KS];
    __shared__ int s_item;
    const int total = *a.item_total;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(a.item_queue, 1);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);  // scalar loop control
        if (item >= total) break;
        const int r = a.irep ? a.irep[item] : item_rep(a, item);
        int chunk = item - a.ioff[r], split = 0;
        if (a.isplit > 1) {
            split = chunk % a.isplit;
            chunk /= a.isplit;
        }
        const int q_begin = a.roff[r] + chunk * kTileQ;
        const int q_end = a.roff[r + 1];
        const int p = q_begin + (int)threadIdx.x;
        const bool valid = p < q_end;
        const int q = a.qlist[valid ? p : q_end - 1];
        f4 qv[4 * KS];
        valu_load_q<KS>(qv, a.Q, a.ldq, a.d, q);
        TopC<C> top;
        if (a.tau) top.seed(a.tau[q]); else top.init();
        int r0 = a.list_off[r], r1 = a.list_off[r + 1];
        if (a.irows) {  // the same entries for the whole workgroup
            r0 = __builtin_amdgcn_readfirstlane(a.irows[2 * (int64_t)item]);
            r1 = __builtin_amdgcn_readfirstlane(a.irows[2 * (int64_t)item + 1]);
        } else if (a.isplit > 1) {
            const int64_t len = r1 - r0;
            r1 = r0 + (int)(len * (split + 1) / a.isplit);
            r0 = r0 + (int)(len * split / a.isplit);
        }
        if (r0 < r1) valu_scan<METRIC, KS, C>(qv, a.X, a.ldx, a.d, r0, r1, valid, top, xs);
        if (valid) {
            const int64_t pair = a.lrank ? (int64_t)a.qoff[q] + a.lrank[(int64_t)q * a.n_r + r]
                                         : (int64_t)q * (a.isplit > 1 ? a.isplit : 1) + split;
            top.store(a.pval + pair * C, a.pidx + pair * C);
        }
        if (a.stats && threadIdx.x == 0) {
            const int nq = q_end - q_begin < kTileQ ? q_end - q_begin : kTileQ;
            const int nrow = r1 > r0 ? r1 - r0 : 0;
            atomicAdd((unsigned long long*)&a.stats[2], (unsigned long long)nq * nrow);
            atomicAdd((unsigned long long*)&a.stats[6], 1ull);
            atomicAdd((unsigned long long*)&a.stats[7],
                      (unsigned long long)kTileQ * ((nrow + kRowsValu - 1) / kRowsValu * kRowsValu));
        }
    }
}

// Every value written out (one-shot build): out[q * ldo + row] = d^2 (l2) or
// rho (l1), direct fp32, for the rows of split blockIdx.y.
template <int METRIC, int KS>
__global__ __launch_bounds__(256, 2) void tile_valu_all(TileArgs a) {
    constexpr int F4 = 4 * KS;
    __shared__ f4 xs[kRowsValu * F4];
    const int myslot = blockIdx.x * kTileQ + threadIdx.x;
    const bool qvalid = myslot < a.m;
    f4 q[F4];
    valu_load_q<KS>(q, a.Q, a.ldq, a.d, qvalid ? myslot : a.m - 1);
    const int r0 = (int)((int64_t)blockIdx.y * a.rps);
    const int r1 = (int)(r0 + (int64_t)a.rps < a.n ? r0 + a.rps : a.n);
    for (int base = r0; base < r1; base += kRowsValu) {
        __syncthreads();
        for (int e = threadIdx.x; e < kRowsValu * F4; e += 256) {
            const int rr = e / F4, cc = e - rr * F4;
            const int row = base + rr;
            f4 v = {0.f, 0.f, 0.f, 0.f};
            if (row < r1 && 4 * cc < a.d) v = *(const f4*)(a.X + (int64_t)row * a.ldx + 4 * cc);
            xs[e] = v;
        }
        __syncthreads();
        if (!qvalid) continue;
        const int nrow = r1 - base < kRowsValu ? r1 - base : kRowsValu;
        float* op = a.pval + (int64_t)myslot * a.ldo + base;
        for (int t = 0; t < nrow; ++t) {
            f4 s = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int j = 0; j < F4; ++j) {
                const f4 df = q[j] - xs[t * F4 + j];
                if (METRIC == 0) {
                    s = df * df + s;
                } else {
                    s[0] += __builtin_fabsf(df[0]);
                    s[1] += __builtin_fabsf(df[1]);
                    s[2] += __builtin_fabsf(df[2]);
                    s[3] += __builtin_fabsf(df[3]);
                }
            }
            op[t] = (s[0] + s[1]) + (s[2] + s[3]);
        }
    }
}

// Range search on the vector ALUs: persistent workgroups take (representative,
// 256-query chunk) items; every lane scores its query against the list's rows
// (staged 32 at a time in LDS) in fp32 direct form, whose relative error is
// below delta = 2 (d + 2) u for the l2 square and the l1 sum alike.  A row is
// inside when s (1 + delta) <= bound, outside when s (1 - delta) > bound
// (bound = radius^2 for l2, radius for l1); in between, the float64 distance
// in the fixed order of rho_fp64 decides, so membership is that of the
// float64 definition.
template <int METRIC, int KS>
__global__ __launch_bounds__(256, 2) void tile_valu_range(TileArgs a) {
    constexpr int F4 = 4 * KS;
    __shared__ f4 xs[kRowsValu * F4];
    __shared__ int s_item;
    const int total = *a.item_total;
    const double delta = 2.0 * (a.d + 2) * 5.9604644775390625e-8;
    // sv, the fp32 sum, lies within a relative delta of the exact sum, plus an
    // absolute d * 2^-149 for terms that underflow; rows clearly inside
    // (count pass) or clearly outside skip the float64 distance, the rest are
    // decided on it, as the reference computation decides them
    const double bound = METRIC == 0 ? a.range_radius * a.range_radius : a.range_radius;
    const double tiny = a.d * 1e-44;
    const double b_in = bound * (1.0 - 2.0 * delta) - tiny;
    const double b_out = bound * (1.0 + 2.0 * delta) + tiny;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(a.item_queue, 1);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        if (item >= total) break;
        const int r = a.irep ? a.irep[item] : item_rep(a, item);
        const int q_begin = a.roff[r] + (item - a.ioff[r]) * kTileQ;
        const int q_end = a.roff[r + 1];
        const int p = q_begin + (int)threadIdx.x;
        const bool valid = p < q_end;
        const int q = a.qlist[valid ? p : q_end - 1];
        f4 qv[F4];
        valu_load_q<KS>(qv, a.Q, a.ldq, a.d, q);
        const float* qp = a.Q + (int64_t)q * a.ldq;
        int r0 = a.list_off[r], r1 = a.list_off[r + 1];
        if (a.irows) {  // the same entries for the whole workgroup
            r0 = __builtin_amdgcn_readfirstlane(a.irows[2 * (int64_t)item]);
            r1 = __builtin_amdgcn_readfirstlane(a.irows[2 * (int64_t)item + 1]);
        }
        int hits = 0;
        for (int base = r0; base < r1; base += kRowsValu) {
            __syncthreads();
            for (int e = threadIdx.x; e < kRowsValu * F4; e += 256) {
                const int rr = e / F4, cc = e - rr * F4;
                const int row = base + rr;
                f4 v = {0.f, 0.f, 0.f, 0.f};
                if (row < r1 && 4 * cc < a.d) v = *(const f4*)(a.X + (int64_t)row * a.ldx + 4 * cc);
                xs[e] = v;
            }
            __syncthreads();
            if (!valid) continue;
            const int nrow = r1 - base < kRowsValu ? r1 - base : kRowsValu;
            for (int t = 0; t < nrow; ++t) {
                f4 s4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int j = 0; j < F4; ++j) {
                    const f4 df = qv[j] - xs[t * F4 + j];
                    if (METRIC == 0) {
                        s4 = df * df + s4;
                    } else {
                        s4[0] += __builtin_fabsf(df[0]);
                        s4[1] += __builtin_fabsf(df[1]);
                        s4[2] += __builtin_fabsf(df[2]);
                        s4[3] += __builtin_fabsf(df[3]);
                    }
                }
                const double sv = (double)((s4[0] + s4[1]) + (s4[2] + s4[3]));
                if (sv > b_out && sv < __builtin_huge_val()) continue;
                const int row = base + t;
                // both passes take the same decision for every row, so the
                // fill pass meets exactly the counts of the count pass
                const bool sure = sv <= b_in;
                double rho = 0.0;
                if (!sure || a.range_fill) rho = rho_fp64(qp, a.X + (int64_t)row * a.ldx, a.d, METRIC);
                if (!sure && !(rho <= a.range_radius)) continue;
                if (a.range_fill) {
                    // the cursor stays inside the caller's segment of query q;
                    // a hit beyond it (offsets from another radius or index)
                    // is counted in range_cnt[m] instead of written
                    const int64_t pos = a.range_off[q] + atomicAdd(a.range_cnt + q, 1);
                    if (pos < a.range_off[q + 1]) {
                        a.range_idx[pos] = a.ids[row];
                        a.range_dist[pos] = (float)rho;
                    } else {
                        atomicAdd(a.range_cnt + a.m, 1);
                    }
                } else {
                    ++hits;
                }
            }
        }
        if (!a.range_fill && valid && hits) atomicAdd(a.range_cnt + q, hits);
    }
}

template <int METRIC, int C>
static hipError_t launch_c(int mode, dim3 grid, const TileArgs& a, hipStream_t st) {
    if (mode == kTileItems || mode == kTileHome)
        hipLaunchKernelGGL((tile_valu_items<METRIC, RBC_KS, C>), grid, dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((tile_valu<METRIC, RBC_KS, C>), grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

template <int METRIC>
static hipError_t launch_m(int c, int mode, dim3 grid, const TileArgs& a, hipStream_t st) {
    if (mode == kTileAll) {
        hipLaunchKernelGGL((tile_valu_all<METRIC, RBC_KS>), grid, dim3(256), 0, st, a);
        return hipGetLastError();
    }
    if (mode == kTileRange) {
        hipLaunchKernelGGL((tile_valu_range<METRIC, RBC_KS>), grid, dim3(256), 0, st, a);
        return hipGetLastError();
    }
    switch (c) {
        case 4: return launch_c<METRIC, 4>(mode, grid, a, st);
        case 8: return launch_c<METRIC, 8>(mode, grid, a, st);
        case 16: return launch_c<METRIC, 16>(mode, grid, a, st);
        case 32: return launch_c<METRIC, 32>(mode, grid, a, st);
        case 64: return launch_c<METRIC, 64>(mode, grid, a, st);
    }
    return hipErrorInvalidValue;
}

// Compiled once per slab count RBC_KS (1..8).
hipError_t RBC_CAT(launch_tile_valu_ks, RBC_KS)(int metric, int c, int mode, dim3 grid,
                                                const TileArgs& a, hipStream_t st) {
    return metric == 0 ? launch_m<0>(c, mode, grid, a, st) : launch_m<1>(c, mode, grid, a, st);
}

}  // namespace rbc
