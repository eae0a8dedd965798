// k_tile_mfma.hip -- L2 distance tile on the gfx950 matrix cores.
//
// Sec. 3 observes that the distance step of BF(Q, X) is shaped like a
// matrix product.  For the Euclidean metric the ranking of
// database rows for a fixed query q only needs  val(x) = ||x||^2 - 2 q.x
// (||q||^2 is common to all rows), a dense contraction over the d features.
//
// Layout of one wavefront's tile (v_mfma_f32_16x16x4f32, fp32 in / fp32
// accumulate): rows of the MFMA output are 32 database rows (two 16-row
// blocks), columns are the wavefront's 64 queries (four 16-query blocks).  The
// accumulators start at ||x||^2 and the query fragments are pre-scaled by -2
// (exact), so the MFMA result is val directly.  Which feature feeds which
// k-slot of an MFMA is free as long as both operands agree: lane l loads the
// float4 at features 16s + 4(l/16) of its row (one 64-byte segment per row per
// slab) and uses its four components in four consecutive MFMAs.
//
// The comparison step (per-query top-c) needs one query per lane, so each
// 32x64 block of results goes through a wavefront-private LDS tile (written as
// [query][row], read back one query per lane), then every lane pushes its 32
// values into a sorted register shortlist (TopC).
#include "rbc_device.h"

#ifndef RBC_KS
#error "compile with -DRBC_KS=<1..8>"
#endif

namespace rbc {

constexpr int kTStride = 36;  // floats per query row of the transpose tile

// Two workgroups per CU while the register footprint allows it.
template <int KS, int C>
struct MfmaOcc {
    static constexpr int value = (24 * KS + 2 * C + 64 <= 200) ? 2 : 1;
};

template <int KS, int C, bool GROUPED>
__global__ __launch_bounds__(256, (MfmaOcc<KS, C>::value)) void tile_l2_mfma(TileArgs a) {
    __shared__ __attribute__((aligned(16))) float tbuf[4][64 * kTStride];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int c16 = lane & 15;
    const int qblk = blockIdx.x;
    const int split = blockIdx.y;
    const int slot0 = qblk * kTileQ + wave * kWave;
    float* tb = tbuf[wave];

    // Query fragments: qf[qb][s] = -2 * Q[slot0 + 16 qb + c16][16 s + 4 g .. + 3].
    f4 qf[4][KS];
#pragma unroll
    for (int qb = 0; qb < 4; ++qb) {
        const int slot = slot0 + 16 * qb + c16;
        const int qs = slot < a.m ? slot : a.m - 1;
        const int qrow = a.qmap ? a.qmap[qs] : qs;
        const float* qp = a.Q + (int64_t)qrow * a.ldq;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int f = 16 * s + 4 * g;
            f4 v = {0.f, 0.f, 0.f, 0.f};
            if (f < a.d) v = *(const f4*)(qp + f);
            qf[qb][s] = v * -2.0f;
        }
    }

    const int myslot = slot0 + lane;
    const bool qvalid = myslot < a.m;
    int myrow = 0;
    if (GROUPED && qvalid) myrow = a.qmap ? a.qmap[myslot] : myslot;

    TopC<C> top;
    top.init();
    int64_t pairs = 0;

    for_each_segment(a, qblk, split, [&](int32_t r0, int32_t r1, int32_t rep) {
        bool act = qvalid;
        if (GROUPED) act = act && a.keep[(int64_t)myrow * a.n_r + rep] != 0;
        const uint64_t any = __ballot(act);
        if (any == 0) return;  // no query of this wavefront kept the list
        if (GROUPED && lane == 0) pairs += (int64_t)__popcll(any) * (r1 - r0);

        for (int32_t base = r0; base < r1; base += kRowsMfma) {
            f4 xa[2][KS];
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) {
                int row = base + 16 * rb + c16;
                row = row < a.n ? row : a.n - 1;
                const float* xp = a.X + (int64_t)row * a.ldx;
#pragma unroll
                for (int s = 0; s < KS; ++s) {
                    const int f = 16 * s + 4 * g;
                    f4 v = {0.f, 0.f, 0.f, 0.f};
                    if (f < a.d) v = *(const f4*)(xp + f);
                    xa[rb][s] = v;
                }
            }
            f4 acc[2][4];
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) {
                f4 nv;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = base + 16 * rb + 4 * g + i;
                    nv[i] = row < r1 ? a.xn[row] : RBC_INF;
                }
#pragma unroll
                for (int qb = 0; qb < 4; ++qb) acc[rb][qb] = nv;
            }
#pragma unroll
            for (int s = 0; s < KS; ++s) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
#pragma unroll
                    for (int rb = 0; rb < 2; ++rb) {
#pragma unroll
                        for (int qb = 0; qb < 4; ++qb) {
                            acc[rb][qb] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                                xa[rb][s][j], qf[qb][s][j], acc[rb][qb], 0, 0, 0);
                        }
                    }
                }
            }
            // transpose: element (query 16 qb + c16, row 16 rb + 4 g + i)
            wave_lds_sync();
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int qb = 0; qb < 4; ++qb)
                    *(f4*)(tb + (16 * qb + c16) * kTStride + 16 * rb + 4 * g) = acc[rb][qb];
            wave_lds_sync();
            f4 vals[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) vals[t] = *(const f4*)(tb + lane * kTStride + 4 * t);
            if (act) {
#pragma unroll
                for (int t = 0; t < 8; ++t)
#pragma unroll
                    for (int i = 0; i < 4; ++i) top.push(vals[t][i], base + 4 * t + i);
            }
        }
    });

    if (qvalid) {
        const int64_t off = ((int64_t)split * a.m + myslot) * C;
        top.store(a.pval + off, a.pidx + off);
    }
    if (GROUPED && a.stats && lane == 0 && pairs) atomicAdd((unsigned long long*)&a.stats[2], (unsigned long long)pairs);
}

template <int KS, int C>
static hipError_t launch_c(bool grouped, dim3 grid, const TileArgs& a, hipStream_t st) {
    if (grouped)
        hipLaunchKernelGGL((tile_l2_mfma<KS, C, true>), grid, dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((tile_l2_mfma<KS, C, false>), grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

// This file is compiled once per slab count RBC_KS (1..8); each object holds
// that slab count's kernels for every shortlist length.
hipError_t RBC_CAT(launch_tile_mfma_ks, RBC_KS)(int c, bool grouped, dim3 grid,
                                                const TileArgs& a, hipStream_t st) {
    switch (c) {
        case 4: return launch_c<RBC_KS, 4>(grouped, grid, a, st);
        case 8: return launch_c<RBC_KS, 8>(grouped, grid, a, st);
        case 16: return launch_c<RBC_KS, 16>(grouped, grid, a, st);
        case 32: return launch_c<RBC_KS, 32>(grouped, grid, a, st);
        case 64: return launch_c<RBC_KS, 64>(grouped, grid, a, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace rbc
