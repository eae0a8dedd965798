// k_finalize.hip -- the end of the comparison step: merge the partial
// shortlists of all database splits, re-score the shortlist directly, re-rank
// near-ties in float64, certify the shortlist, write the k results.  Queries
// that cannot be certified are listed for an exhaustive float64 search
// (exact_fp64 below), which is also the path for k or d beyond the tiles.
//
// Certificate.  Every row outside the merged shortlist had a tile value at
// least A_c (the shortlist's c-th value).  With a rigorous bound on the tile's
// rounding error this gives a lower bound on the true distance of any row
// outside the shortlist; if it is strictly above the k-th re-scored distance
// (widened by that value's own error), the k best rows are all inside the
// shortlist.  Error bounds, with u = 2^-24:
//   matrix-core tile (values ||x||^2 - 2 q.x, ||q||^2 added here):
//       |error of d^2| <= 4 (d + 2) u (||q|| + max ||x||)^2
//   direct fp32 (d^2 or l1 sum of non-negative terms): relative 2 (d + 2) u.
// The factor 4 (resp. 2) is a safety margin over the textbook bound of a
// d-term dot product, for any summation order.
#include "rbc_device.h"

namespace rbc {

// Wavefront argmin of (value, id, lane); every lane gets the winner's lane.
__device__ __forceinline__ int wave_argmin(float v, int32_t id, float& bv, int32_t& bi) {
    bv = v;
    bi = id;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const float ov = __shfl_xor(bv, off);
        const int32_t oi = __shfl_xor(bi, off);
        if (ov < bv || (ov == bv && oi < bi)) {
            bv = ov;
            bi = oi;
        }
    }
    const uint64_t m = __ballot(v == bv && id == bi);
    return (int)__builtin_ctzll(m);
}

template <int C>
__device__ __forceinline__ void finalize_slot(const FinArgs& a, int slot, int nsplit, int stride) {
    const int lane = threadIdx.x & 63;
    const int qrow = slot;                               // row of Q (and of qn, qerr)
    const int orow = a.qmap ? a.qmap[slot] : slot;       // output row, reported query

    // 1. merge the sorted partial lists into the c best entries: lane r ends
    //    up holding merged entry r.  Each round takes the smallest head; one
    //    lane (the lowest among equal heads) advances, so copies of a bound
    //    are counted as often as they occur.
    float mv = RBC_INF;
    int32_t mi = -1;
    if (a.qoff == nullptr && nsplit == 1) {
        if (lane < C) {
            mv = a.pval[(int64_t)slot * C + lane];
            mi = a.pidx[(int64_t)slot * C + lane];
        }
    } else {
        // every lane first reduces its share of the lists to one sorted
        // register list of c entries (a list is sorted, so its scan stops at
        // the first entry that cannot enter)
        TopC<C> loc;
        loc.init();
        const int nl = a.qoff ? a.npairs[slot] : nsplit;
        for (int j = lane; j < nl; j += 64) {
            const int64_t base = a.qoff ? ((int64_t)a.qoff[slot] + j) * C
                                        : ((int64_t)j * stride + slot) * C;
            for (int i = 0; i < C; ++i) {
                const float v = a.pval[base + i];
                if (!(v < loc.worst())) break;
                loc.insert(v, a.pidx[base + i]);
            }
        }
        for (int r = 0; r < C; ++r) {
            float bv;
            int32_t bi;
            const int w = wave_argmin(loc.v[0], loc.i[0], bv, bi);
            if (lane == r) {
                mv = bv;
                mi = bi;
            }
            if (lane == w) {
#pragma unroll
                for (int j = 0; j + 1 < C; ++j) {
                    loc.v[j] = loc.v[j + 1];
                    loc.i[j] = loc.i[j + 1];
                }
                loc.v[C - 1] = RBC_INF;
                loc.i[C - 1] = -1;
            }
        }
    }
    const bool valid = lane < C && mi >= 0 && mv < RBC_INF;
    const float a_c = __shfl(mv, C - 1);

    // 2. direct re-score in fp32: 64 / C lanes per candidate, each summing a
    //    strided subset of the features, then a reduction inside the group
    constexpr int LPC = 64 / C;
    const float* qp = a.Q + (int64_t)qrow * a.ldq;
    const int cand = lane / LPC;
    const int sub = lane % LPC;
    const int32_t crow = __shfl(mi, cand);
    const bool cvalid = __shfl((int)valid, cand) != 0;
    float part = 0.f;
    if (cvalid) {
        const float* cp = a.X + (int64_t)crow * a.ldx;
        // rows as float4 runs when both are 16-byte aligned (sub-lane s takes
        // runs s, s + LPC, ...), the tail as single features
        const bool v4 = ((a.ldq | a.ldx) & 3) == 0 && (((uintptr_t)a.Q | (uintptr_t)a.X) & 15) == 0;
        const int d4 = v4 ? a.d & ~3 : 0;
        if (a.metric == 0) {
            for (int f = 4 * sub; f < d4; f += 4 * LPC) {
                const f4 t = *(const f4*)(qp + f) - *(const f4*)(cp + f);
                part = __builtin_fmaf(t[0], t[0], part);
                part = __builtin_fmaf(t[1], t[1], part);
                part = __builtin_fmaf(t[2], t[2], part);
                part = __builtin_fmaf(t[3], t[3], part);
            }
            for (int f = d4 + sub; f < a.d; f += LPC) {
                const float t = qp[f] - cp[f];
                part = __builtin_fmaf(t, t, part);
            }
        } else {
            for (int f = 4 * sub; f < d4; f += 4 * LPC) {
                const f4 t = *(const f4*)(qp + f) - *(const f4*)(cp + f);
                part += __builtin_fabsf(t[0]) + __builtin_fabsf(t[1]) + __builtin_fabsf(t[2]) +
                        __builtin_fabsf(t[3]);
            }
            for (int f = d4 + sub; f < a.d; f += LPC) part += __builtin_fabsf(qp[f] - cp[f]);
        }
    }
#pragma unroll
    for (int off = LPC / 2; off >= 1; off >>= 1) part += __shfl_xor(part, off);
    const float s32 = __shfl(part, (lane < C ? lane : 0) * LPC);
    const float* xp = a.X + (int64_t)(valid ? mi : 0) * a.ldx;
    double rho = RBC_INF_D;
    if (valid) rho = a.metric == 0 ? __builtin_sqrt((double)s32) : (double)s32;

    // 3. float64 re-rank of near-ties
    const double u = 5.9604644775390625e-8;
    const double delta = 2.0 * (a.d + 2) * u;  // relative error of a direct fp32 distance
    const double tol = 2.0 * delta;
    bool flag = false;
    for (int i = 0; i < C; ++i) {
        const double ri = __shfl(rho, i);
        if (i != lane && valid && ri < RBC_INF_D &&
            __builtin_fabs(ri - rho) <= tol * (ri > rho ? ri : rho))
            flag = true;
    }
    if (flag) rho = rho_fp64(qp, xp, a.d, a.metric);
    const uint64_t flagged = __ballot(flag);

    // 4. rank by (distance, reported id)
    const int64_t myid = valid ? (a.id_map ? a.id_map[mi] : (int64_t)mi) : INT64_MAX;
    int rank = 0;
    for (int i = 0; i < C; ++i) {
        const double ri = __shfl(rho, i);
        const int64_t ii = __shfl(myid, i);
        if (i != lane && before(ri, ii, rho, myid)) ++rank;
    }
    const int nvalid = __popcll(__ballot(valid));

    // 5. certificate
    bool ok = nvalid >= a.k;
    if (ok && a_c < RBC_INF) {
        const uint64_t kth = __ballot(valid && rank == a.k - 1);
        const double t_k = __shfl(rho, (int)__builtin_ctzll(kth));
        double lo;
        if (a.approx_mode == 0 || a.approx_mode == 2) {
            const double qn = a.qn[slot];
            const double xmax = (double)__uint_as_float(*a.xmax_bits);
            const double sq = __builtin_sqrt(qn) + xmax;
            const double e =
                tile_exact(a.flags_q, a.flags_x, a.d) ? 0.0 : 4.0 * (a.d + 2) * u * sq * sq;
            const double lo2 = (double)a_c + qn - e;
            lo = lo2 > 0.0 ? __builtin_sqrt(lo2) : 0.0;
            if (a.approx_mode == 2)  // distances of the quantised rows: triangle inequality
                lo -= (double)a.qerr[slot] + (double)__uint_as_float(*a.xerr_max_bits);
        } else if (a.metric == 0) {
            lo = __builtin_sqrt((double)a_c) * (1.0 - delta);
        } else {
            lo = (double)a_c * (1.0 - delta);
        }
        ok = lo > t_k * (1.0 + delta);
    }

    if (!ok) {
        if (lane == 0) {
            const int p = atomicAdd(a.fb_count, 1);
            a.fb_list[p] = orow;
        }
    } else if (valid && rank < a.k) {
        a.out_idx[(int64_t)orow * a.k + rank] = myid;
        a.out_dist[(int64_t)orow * a.k + rank] = (float)rho;
        if (a.out_approx) {
            // the entry's distance in the ranking tile, before re-scoring
            double ap;
            if (a.approx_mode == 1)
                ap = a.metric == 0 ? __builtin_sqrt((double)mv) : (double)mv;
            else
                ap = __builtin_sqrt(fmax((double)mv + (double)a.qn[slot], 0.0));
            a.out_approx[(int64_t)orow * a.k + rank] = (float)ap;
        }
    }
    if (a.stats && lane == 0) {
        if (!ok) atomicAdd((unsigned long long*)&a.stats[a.fail_stat], 1ull);
        if (flagged) atomicAdd((unsigned long long*)&a.stats[1], (unsigned long long)__popcll(flagged));
    }
}

// One wavefront per query.  With a device-side query count (the float32
// cascade of low-precision searches) the grid is bounded and strides over
// the queries, so a launch sized for every query costs nothing when few fail.
template <int C>
__global__ __launch_bounds__(256) void finalize_kernel(FinArgs a) {
    int mact = a.m, nsplit = a.nsplit, stride = a.m;
    if (a.m_dev) {
        mact = *a.m_dev;
        const DevSplit ds = dev_split(mact, a.dev_blocks, a.n);
        nsplit = ds.S;
        stride = ds.M;
    }
    for (int slot = blockIdx.x * 4 + (threadIdx.x >> 6); slot < mact; slot += gridDim.x * 4)
        finalize_slot<C>(a, slot, nsplit, stride);  // uniform per wavefront
}

// The same steps for the common case of one list per query (a single
// database split, no pair lists, c <= 16), with 16 lanes per query and four
// queries per wavefront: 16 / c lanes re-score each candidate.  Shuffles stay
// inside a query's 16 lanes; ballots are masked to them.  Used for the
// ownership search of the build (a million queries) and one-shot searches,
// where one wavefront per query leaves the kernel latency-bound.
template <int C>
__global__ __launch_bounds__(256) void finalize_group_kernel(FinArgs a) {
    constexpr int G = 16;
    constexpr int LPC = G / C;
    const int lane = threadIdx.x & 63;
    const int gl = lane & (G - 1);
    const int sh = lane & ~(G - 1);  // first lane of the group in the wavefront
    const int slot = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 4 + (lane >> 4);
    const bool live = slot < a.m;
    const int qrow = live ? slot : a.m - 1;

    float mv = RBC_INF;
    int32_t mi = -1;
    if (live && gl < C) {
        mv = a.pval[(int64_t)qrow * C + gl];
        mi = a.pidx[(int64_t)qrow * C + gl];
    }
    const bool valid = live && gl < C && mi >= 0 && mv < RBC_INF;
    const float a_c = __shfl(mv, C - 1, G);

    const float* qp = a.Q + (int64_t)qrow * a.ldq;
    const int cand = gl / LPC;
    const int sub = gl % LPC;
    const int32_t crow = __shfl(mi, cand, G);
    const bool cvalid = __shfl((int)valid, cand, G) != 0;
    float part = 0.f;
    if (cvalid) {
        const float* cp = a.X + (int64_t)crow * a.ldx;
        // rows as float4 runs when both are 16-byte aligned (sub-lane s takes
        // runs s, s + LPC, ...), the tail as single features
        const bool v4 = ((a.ldq | a.ldx) & 3) == 0 && (((uintptr_t)a.Q | (uintptr_t)a.X) & 15) == 0;
        const int d4 = v4 ? a.d & ~3 : 0;
        if (a.metric == 0) {
            for (int f = 4 * sub; f < d4; f += 4 * LPC) {
                const f4 t = *(const f4*)(qp + f) - *(const f4*)(cp + f);
                part = __builtin_fmaf(t[0], t[0], part);
                part = __builtin_fmaf(t[1], t[1], part);
                part = __builtin_fmaf(t[2], t[2], part);
                part = __builtin_fmaf(t[3], t[3], part);
            }
            for (int f = d4 + sub; f < a.d; f += LPC) {
                const float t = qp[f] - cp[f];
                part = __builtin_fmaf(t, t, part);
            }
        } else {
            for (int f = 4 * sub; f < d4; f += 4 * LPC) {
                const f4 t = *(const f4*)(qp + f) - *(const f4*)(cp + f);
                part += __builtin_fabsf(t[0]) + __builtin_fabsf(t[1]) + __builtin_fabsf(t[2]) +
                        __builtin_fabsf(t[3]);
            }
            for (int f = d4 + sub; f < a.d; f += LPC) part += __builtin_fabsf(qp[f] - cp[f]);
        }
    }
#pragma unroll
    for (int off = LPC / 2; off >= 1; off >>= 1) part += __shfl_xor(part, off, G);
    const float s32 = __shfl(part, (gl < C ? gl : 0) * LPC, G);
    const float* xp = a.X + (int64_t)(valid ? mi : 0) * a.ldx;
    double rho = RBC_INF_D;
    if (valid) rho = a.metric == 0 ? __builtin_sqrt((double)s32) : (double)s32;

    const double u = 5.9604644775390625e-8;
    const double delta = 2.0 * (a.d + 2) * u;
    const double tol = 2.0 * delta;
    bool flag = false;
    for (int i = 0; i < C; ++i) {
        const double ri = __shfl(rho, i, G);
        if (i != gl && valid && ri < RBC_INF_D &&
            __builtin_fabs(ri - rho) <= tol * (ri > rho ? ri : rho))
            flag = true;
    }
    if (flag) rho = rho_fp64(qp, xp, a.d, a.metric);
    const uint32_t flagged = (uint32_t)((__ballot(flag) >> sh) & 0xffffu);

    const int64_t myid = valid ? (a.id_map ? a.id_map[mi] : (int64_t)mi) : INT64_MAX;
    int rank = 0;
    for (int i = 0; i < C; ++i) {
        const double ri = __shfl(rho, i, G);
        const int64_t ii = __shfl(myid, i, G);
        if (i != gl && before(ri, ii, rho, myid)) ++rank;
    }
    const int nvalid = __popc((uint32_t)((__ballot(valid) >> sh) & 0xffffu));
    const uint32_t kth = (uint32_t)((__ballot(valid && rank == a.k - 1) >> sh) & 0xffffu);

    bool ok = live && nvalid >= a.k;
    if (ok && a_c < RBC_INF) {
        const double t_k = __shfl(rho, (int)__builtin_ctz(kth), G);
        double lo;
        if (a.approx_mode == 0 || a.approx_mode == 2) {
            const double qn = a.qn[qrow];
            const double xmax = (double)__uint_as_float(*a.xmax_bits);
            const double sq = __builtin_sqrt(qn) + xmax;
            const double e =
                tile_exact(a.flags_q, a.flags_x, a.d) ? 0.0 : 4.0 * (a.d + 2) * u * sq * sq;
            const double lo2 = (double)a_c + qn - e;
            lo = lo2 > 0.0 ? __builtin_sqrt(lo2) : 0.0;
            if (a.approx_mode == 2)
                lo -= (double)a.qerr[qrow] + (double)__uint_as_float(*a.xerr_max_bits);
        } else if (a.metric == 0) {
            lo = __builtin_sqrt((double)a_c) * (1.0 - delta);
        } else {
            lo = (double)a_c * (1.0 - delta);
        }
        ok = lo > t_k * (1.0 + delta);
    }

    if (!live) return;
    if (!ok) {
        if (gl == 0) {
            const int p = atomicAdd(a.fb_count, 1);
            a.fb_list[p] = qrow;
        }
    } else if (valid && rank < a.k) {
        a.out_idx[(int64_t)qrow * a.k + rank] = myid;
        a.out_dist[(int64_t)qrow * a.k + rank] = (float)rho;
        if (a.out_approx) {
            double ap;
            if (a.approx_mode == 1)
                ap = a.metric == 0 ? __builtin_sqrt((double)mv) : (double)mv;
            else
                ap = __builtin_sqrt(fmax((double)mv + (double)a.qn[qrow], 0.0));
            a.out_approx[(int64_t)qrow * a.k + rank] = (float)ap;
        }
    }
    if (a.stats && gl == 0) {
        if (!ok) atomicAdd((unsigned long long*)&a.stats[a.fail_stat], 1ull);
        if (flagged) atomicAdd((unsigned long long*)&a.stats[1], (unsigned long long)__popc(flagged));
    }
}

hipError_t launch_finalize(int c, const FinArgs& a, hipStream_t st) {
    if (!a.qoff && a.nsplit == 1 && !a.m_dev && !a.qmap && c <= 16) {
        const dim3 g16((a.m + 15) / 16);
        switch (c) {
            case 4: hipLaunchKernelGGL((finalize_group_kernel<4>), g16, dim3(256), 0, st, a); break;
            case 8: hipLaunchKernelGGL((finalize_group_kernel<8>), g16, dim3(256), 0, st, a); break;
            case 16: hipLaunchKernelGGL((finalize_group_kernel<16>), g16, dim3(256), 0, st, a); break;
        }
        return hipGetLastError();
    }
    const int64_t waves = a.m_dev && a.m > 8192 ? 8192 : a.m;
    const dim3 grid((unsigned)((waves + 3) / 4));
    switch (c) {
        case 4: hipLaunchKernelGGL((finalize_kernel<4>), grid, dim3(256), 0, st, a); break;
        case 8: hipLaunchKernelGGL((finalize_kernel<8>), grid, dim3(256), 0, st, a); break;
        case 16: hipLaunchKernelGGL((finalize_kernel<16>), grid, dim3(256), 0, st, a); break;
        case 32: hipLaunchKernelGGL((finalize_kernel<32>), grid, dim3(256), 0, st, a); break;
        case 64: hipLaunchKernelGGL((finalize_kernel<64>), grid, dim3(256), 0, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Exhaustive float64 search (any k <= kExactKCap) for the listed queries: one
// workgroup per query, rows scored one per thread in float64 (the fixed order
// of rho_fp64), candidates below the current k-th value appended to an LDS
// buffer, buffer and current top-k merged by rank counting when it fills.
constexpr int kExactBuf = 1024;

__global__ __launch_bounds__(256) void exact_fp64_kernel(ExactArgs a) {
    __shared__ double tv[kExactKCap];
    __shared__ int64_t ti[kExactKCap];
    __shared__ double bv[kExactBuf];
    __shared__ int64_t bi[kExactBuf];
    __shared__ int s_kcnt, s_bcnt;
    __shared__ double s_thr;
    __shared__ int64_t s_thr_id;
    const int tid = threadIdx.x;
    const int count = *a.count;

    for (int f = blockIdx.x; f < count; f += gridDim.x) {
        const int qrow = a.list[f];
        const float* qp = a.Q + (int64_t)qrow * a.ldq;
        int row0 = 0, row1 = a.n;
        if (a.qrep) {
            row0 = a.list_off[a.qrep[qrow]];
            row1 = a.list_off[a.qrep[qrow] + 1];
        }
        if (tid == 0) {
            s_kcnt = 0;
            s_bcnt = 0;
            s_thr = RBC_INF_D;
            s_thr_id = INT64_MAX;
        }
        __syncthreads();
        for (int base = row0; base < row1; base += 256) {
            const int row = base + tid;
            if (row < row1) {
                const double r = rho_fp64(qp, a.X + (int64_t)row * a.ldx, a.d, a.metric);
                const int64_t id = a.id_map ? a.id_map[row] : (int64_t)row;
                if (before(r, id, s_thr, s_thr_id)) {
                    const int p = atomicAdd(&s_bcnt, 1);
                    bv[p] = r;
                    bi[p] = id;
                }
            }
            __syncthreads();
            const int bcnt = s_bcnt;
            if (bcnt > kExactBuf - 256 || base + 256 >= row1) {
                // merge: rank every entry of (top, buffer) by counting the
                // entries before it; ranks are distinct, keep ranks < k.
                const int kcnt = s_kcnt;
                const int tot = kcnt + bcnt;
                double myv[8];
                int64_t myi[8];
                int myr[8];
                int nmine = 0;
                for (int e = tid; e < tot; e += 256) {
                    const double v = e < kcnt ? tv[e] : bv[e - kcnt];
                    const int64_t id = e < kcnt ? ti[e] : bi[e - kcnt];
                    int rk = 0;
                    for (int j = 0; j < tot; ++j) {
                        const double vj = j < kcnt ? tv[j] : bv[j - kcnt];
                        const int64_t ij = j < kcnt ? ti[j] : bi[j - kcnt];
                        rk += before(vj, ij, v, id) ? 1 : 0;
                    }
                    myv[nmine] = v;
                    myi[nmine] = id;
                    myr[nmine] = rk;
                    ++nmine;
                }
                __syncthreads();
                for (int t = 0; t < nmine; ++t) {
                    if (myr[t] < a.k) {
                        tv[myr[t]] = myv[t];
                        ti[myr[t]] = myi[t];
                    }
                }
                __syncthreads();
                if (tid == 0) {
                    const int nk = tot < a.k ? tot : a.k;
                    s_kcnt = nk;
                    s_bcnt = 0;
                    s_thr = nk == a.k ? tv[nk - 1] : RBC_INF_D;
                    s_thr_id = nk == a.k ? ti[nk - 1] : INT64_MAX;
                }
            }
            __syncthreads();
        }
        for (int e = tid; e < a.k; e += 256) {
            const bool have = e < s_kcnt;
            a.out_idx[(int64_t)qrow * a.k + e] = have ? ti[e] : -1;
            a.out_dist[(int64_t)qrow * a.k + e] = have ? (float)tv[e] : RBC_INF;
        }
        __syncthreads();
    }
}

hipError_t launch_exact(const ExactArgs& a, int grid, hipStream_t st) {
    hipLaunchKernelGGL(exact_fp64_kernel, dim3(grid), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace rbc
