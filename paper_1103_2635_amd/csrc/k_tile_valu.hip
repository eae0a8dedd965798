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

template <int METRIC, int KS, int C, bool GROUPED>
__global__ __launch_bounds__(256, 2) void tile_valu(TileArgs a) {
    constexpr int F4 = 4 * KS;  // float4 per staged row
    __shared__ f4 xs[kRowsValu * F4];

    const int tid = threadIdx.x;
    const int qblk = blockIdx.x;
    const int split = blockIdx.y;
    const int myslot = qblk * kTileQ + tid;
    const bool qvalid = myslot < a.m;
    const int qs = qvalid ? myslot : a.m - 1;
    const int myrow = a.qmap ? a.qmap[qs] : qs;

    f4 q[F4];
    {
        const float* qp = a.Q + (int64_t)myrow * a.ldq;
#pragma unroll
        for (int j = 0; j < F4; ++j) {
            f4 v = {0.f, 0.f, 0.f, 0.f};
            if (4 * j < a.d) v = *(const f4*)(qp + 4 * j);
            q[j] = v;
        }
    }

    TopC<C> top;
    top.init();
    int64_t pairs = 0;

    for_each_segment(a, qblk, split, [&](int32_t r0, int32_t r1, int32_t rep) {
        bool act = qvalid;
        if (GROUPED) act = act && a.keep[(int64_t)myrow * a.n_r + rep] != 0;
        if (GROUPED) {
            const int n_act = __syncthreads_count(act);
            if (n_act == 0) return;  // uniform: nobody in the block kept this list
            if (tid == 0) pairs += (int64_t)n_act * (r1 - r0);
        }
        for (int32_t base = r0; base < r1; base += kRowsValu) {
            __syncthreads();
            for (int e = tid; e < kRowsValu * F4; e += 256) {
                const int rr = e / F4, cc = e - rr * F4;
                const int row = base + rr;
                f4 v = {0.f, 0.f, 0.f, 0.f};
                if (row < r1 && 4 * cc < a.d) v = *(const f4*)(a.X + (int64_t)row * a.ldx + 4 * cc);
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
    });

    if (qvalid) {
        const int64_t off = ((int64_t)split * a.m + myslot) * C;
        top.store(a.pval + off, a.pidx + off);
    }
    if (GROUPED && a.stats && tid == 0 && pairs) atomicAdd((unsigned long long*)&a.stats[2], (unsigned long long)pairs);
}

template <int METRIC, int C>
static hipError_t launch_c(bool grouped, dim3 grid, const TileArgs& a, hipStream_t st) {
    if (grouped)
        hipLaunchKernelGGL((tile_valu<METRIC, RBC_KS, C, true>), grid, dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((tile_valu<METRIC, RBC_KS, C, false>), grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

template <int METRIC>
static hipError_t launch_m(int c, bool grouped, dim3 grid, const TileArgs& a, hipStream_t st) {
    switch (c) {
        case 4: return launch_c<METRIC, 4>(grouped, grid, a, st);
        case 8: return launch_c<METRIC, 8>(grouped, grid, a, st);
        case 16: return launch_c<METRIC, 16>(grouped, grid, a, st);
        case 32: return launch_c<METRIC, 32>(grouped, grid, a, st);
        case 64: return launch_c<METRIC, 64>(grouped, grid, a, st);
    }
    return hipErrorInvalidValue;
}

// Compiled once per slab count RBC_KS (1..8).
hipError_t RBC_CAT(launch_tile_valu_ks, RBC_KS)(int metric, int c, bool grouped, dim3 grid,
                                                const TileArgs& a, hipStream_t st) {
    return metric == 0 ? launch_m<0>(c, grouped, grid, a, st) : launch_m<1>(c, grouped, grid, a, st);
}

}  // namespace rbc
