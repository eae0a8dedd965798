// k_tile_mfma.hip -- L2 distance tile on the gfx950 matrix cores.
//
// Sec. 3 observes that the distance step of BF(Q, X) is shaped like a
// matrix product.  For the Euclidean metric the ranking of database rows for
// a fixed query q only needs  val(x) = ||x||^2 - 2 q.x  (||q||^2 is common to
// all rows), a dense contraction over the d features.
//
// Layout of one wavefront's tile (v_mfma_f32_16x16x4f32, fp32 in / fp32
// accumulate): rows of the MFMA output are 32 database rows (two 16-row
// blocks), columns are the wavefront's 64 queries (four 16-query blocks).  The
// accumulators start at ||x||^2 and the query fragments are pre-scaled by -2
// (exact), so the MFMA result is val directly.  Which feature feeds which
// k-slot of an MFMA is free as long as both operands agree: lane l loads the
// float4 at features 16s + 4(l/16) of its row (one 64-byte segment per row per
// slab) and uses its four components in four consecutive MFMAs.  The database
// fragments of the next 32 rows are loaded while the current ones are used.
//
// The comparison step (per-query top-c) needs one query per lane, so each
// 32x64 block of results goes through a wavefront-private LDS tile (written as
// [query][row], read back one query per lane), then every lane pushes its 32
// values into a sorted register shortlist (TopC).
//
// Three launch forms share the row scan:
//   BF mode    -- grid (query blocks, database splits); a workgroup's 256
//                 queries scan one split of the rows.
//   item mode  -- RBC stage 2, persistent wavefronts pulling work items
//                 (representative r, 64 of the queries that search L_r) from
//                 a queue; the queries scan the rows of L_r, their shortlists
//                 start at a per-query threshold known from stage 1 (exact
//                 mode).
//   all mode   -- every value written out (one-shot build).
#include "rbc_device.h"

#ifndef RBC_KS
#error "compile with -DRBC_KS=<1..8>"
#endif

namespace rbc {

constexpr int kTStride = 36;  // floats per query row of the transpose tile

// Two workgroups per CU while the register footprint allows it.
template <int KS, int C>
struct MfmaOcc {
    static constexpr int value = (32 * KS + 2 * C + 64 <= 232) ? 2 : 1;
};

// Query fragments: qf[qb][s] = -2 * Q[qrow[qb]][16 s + 4 g .. + 3].
template <int KS>
__device__ __forceinline__ void load_qfrag(f4 (&qf)[4][KS], const float* Q, int64_t ldq, int d,
                                           const int (&qrow)[4], int g) {
#pragma unroll
    for (int qb = 0; qb < 4; ++qb) {
        const float* qp = Q + (int64_t)qrow[qb] * ldq;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int f = 16 * s + 4 * g;
            f4 v = {0.f, 0.f, 0.f, 0.f};
            if (f < d) v = *(const f4*)(qp + f);
            qf[qb][s] = v * -2.0f;
        }
    }
}

template <int KS>
__device__ __forceinline__ void load_xfrag(f4 (&xa)[2][KS], const float* X, int64_t ldx, int n,
                                           int d, int base, int c16, int g) {
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
        int row = base + 16 * rb + c16;
        row = row < n ? row : n - 1;
        const float* xp = X + (int64_t)row * ldx;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int f = 16 * s + 4 * g;
            f4 v = {0.f, 0.f, 0.f, 0.f};
            if (f < d) v = *(const f4*)(xp + f);
            xa[rb][s] = v;
        }
    }
}

// Scan database rows [r0, r1) for the wavefront's 64 queries; lanes with act
// push their values into top.
template <int KS, int C>
__device__ __forceinline__ void scan_rows(const f4 (&qf)[4][KS], const float* X, int64_t ldx,
                                          const float* xn, int n, int d, int r0, int r1, bool act,
                                          TopC<C>& top, float* tb, int lane) {
    const int g = lane >> 4;
    const int c16 = lane & 15;
    f4 xa[2][KS];
    load_xfrag<KS>(xa, X, ldx, n, d, r0, c16, g);
    for (int base = r0; base < r1; base += kRowsMfma) {
        f4 acc[2][4];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            f4 nv;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = base + 16 * rb + 4 * g + i;
                nv[i] = row < r1 ? xn[row] : RBC_INF;
            }
#pragma unroll
            for (int qb = 0; qb < 4; ++qb) acc[rb][qb] = nv;
        }
        f4 xb[2][KS];
        const int next = base + kRowsMfma;
        load_xfrag<KS>(xb, X, ldx, n, d, next < r1 ? next : base, c16, g);
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
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int s = 0; s < KS; ++s) xa[rb][s] = xb[rb][s];
    }
}

template <int KS, int C>
__global__ __launch_bounds__(256, (MfmaOcc<KS, C>::value)) void tile_l2_mfma(TileArgs a) {
    __shared__ __attribute__((aligned(16))) float tbuf[4][64 * kTStride];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int c16 = lane & 15;
    const int slot0 = blockIdx.x * kTileQ + wave * kWave;

    f4 qf[4][KS];
    int qrow[4];
#pragma unroll
    for (int qb = 0; qb < 4; ++qb) {
        const int slot = slot0 + 16 * qb + c16;
        qrow[qb] = slot < a.m ? slot : a.m - 1;
    }
    load_qfrag<KS>(qf, a.Q, a.ldq, a.d, qrow, g);

    const int myslot = slot0 + lane;
    TopC<C> top;
    top.init();
    const int64_t r0 = (int64_t)blockIdx.y * a.rps;
    const int64_t r1 = r0 + a.rps < a.n ? r0 + a.rps : a.n;
    if (r0 < r1)
        scan_rows<KS, C>(qf, a.X, a.ldx, a.xn, a.n, a.d, (int)r0, (int)r1, myslot < a.m, top,
                         tbuf[wave], lane);
    if (myslot < a.m) {
        const int64_t off = ((int64_t)blockIdx.y * a.m + myslot) * C;
        top.store(a.pval + off, a.pidx + off);
    }
}

// RBC stage 2: persistent wavefronts, each taking (representative, 64-query
// chunk) items from the queue until it is empty.  Wavefronts work
// independently (no workgroup barrier); consecutive items usually belong to
// the same representative, so co-resident wavefronts share its list rows in
// the caches.
template <int KS, int C>
__global__ __launch_bounds__(256, (MfmaOcc<KS, C>::value)) void tile_l2_mfma_items(TileArgs a) {
    __shared__ __attribute__((aligned(16))) float tbuf[4][64 * kTStride];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int c16 = lane & 15;
    const int total = *a.item_total;

    for (;;) {
        int item = 0;
        if (lane == 0) item = atomicAdd(a.item_queue, 1);
        item = __shfl(item, 0);
        if (item >= total) break;
        const int r = item_rep(a, item);
        const int q_begin = a.roff[r] + (item - a.ioff[r]) * kWave;
        const int q_end = a.roff[r + 1];

        f4 qf[4][KS];
        int qrow[4];
#pragma unroll
        for (int qb = 0; qb < 4; ++qb) {
            const int p = q_begin + 16 * qb + c16;
            qrow[qb] = a.qlist[p < q_end ? p : q_end - 1];
        }
        load_qfrag<KS>(qf, a.Q, a.ldq, a.d, qrow, g);

        const int p = q_begin + lane;
        const bool valid = p < q_end;
        const int q = a.qlist[valid ? p : q_end - 1];
        TopC<C> top;
        if (a.tau) top.seed(a.tau[q]); else top.init();
        scan_rows<KS, C>(qf, a.X, a.ldx, a.xn, a.n, a.d, a.list_off[r], a.list_off[r + 1], valid,
                         top, tbuf[wave], lane);
        if (valid) {
            const int64_t pair =
                a.lrank ? (int64_t)a.qoff[q] + a.lrank[(int64_t)q * a.n_r + r] : (int64_t)q;
            top.store(a.pval + pair * C, a.pidx + pair * C);
        }
        if (a.stats && lane == 0) {
            const int nq = q_end - q_begin < kWave ? q_end - q_begin : kWave;
            atomicAdd((unsigned long long*)&a.stats[2],
                      (unsigned long long)nq * (a.list_off[r + 1] - a.list_off[r]));
        }
    }
}

// Every value of the tile written out (one-shot build): out[q * ldo + row] =
// ||x||^2 - 2 q.x for the rows [blockIdx.y * rps, ...) of the split.
template <int KS>
__global__ __launch_bounds__(256, 2) void tile_l2_mfma_all(TileArgs a) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int c16 = lane & 15;
    const int slot0 = blockIdx.x * kTileQ + wave * kWave;
    f4 qf[4][KS];
    int qrow[4];
#pragma unroll
    for (int qb = 0; qb < 4; ++qb) {
        const int slot = slot0 + 16 * qb + c16;
        qrow[qb] = slot < a.m ? slot : a.m - 1;
    }
    load_qfrag<KS>(qf, a.Q, a.ldq, a.d, qrow, g);
    const int r0 = (int)((int64_t)blockIdx.y * a.rps);
    const int r1 = (int)(r0 + (int64_t)a.rps < a.n ? r0 + a.rps : a.n);
    if (r0 >= r1) return;
    f4 xa[2][KS];
    load_xfrag<KS>(xa, a.X, a.ldx, a.n, a.d, r0, c16, g);
    for (int base = r0; base < r1; base += kRowsMfma) {
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
        f4 xb[2][KS];
        const int next = base + kRowsMfma;
        load_xfrag<KS>(xb, a.X, a.ldx, a.n, a.d, next < r1 ? next : base, c16, g);
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                    for (int qb = 0; qb < 4; ++qb)
                        acc[rb][qb] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                            xa[rb][s][j], qf[qb][s][j], acc[rb][qb], 0, 0, 0);
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            const int row = base + 16 * rb + 4 * g;
#pragma unroll
            for (int qb = 0; qb < 4; ++qb) {
                const int slot = slot0 + 16 * qb + c16;
                if (slot >= a.m) continue;
                float* op = a.pval + (int64_t)slot * a.ldo + row;
                if (row + 3 < r1) {
                    *(f4*)op = acc[rb][qb];
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (row + i < r1) op[i] = acc[rb][qb][i];
                }
            }
        }
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int s = 0; s < KS; ++s) xa[rb][s] = xb[rb][s];
    }
}

template <int KS, int C>
static hipError_t launch_c(int mode, dim3 grid, const TileArgs& a, hipStream_t st) {
    if (mode == kTileItems)
        hipLaunchKernelGGL((tile_l2_mfma_items<KS, C>), grid, dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((tile_l2_mfma<KS, C>), grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

// This file is compiled once per slab count RBC_KS (1..8); each object holds
// that slab count's kernels for every shortlist length.
hipError_t RBC_CAT(launch_tile_mfma_ks, RBC_KS)(int c, int mode, dim3 grid,
                                                const TileArgs& a, hipStream_t st) {
    if (mode == kTileAll) {
        hipLaunchKernelGGL((tile_l2_mfma_all<RBC_KS>), grid, dim3(256), 0, st, a);
        return hipGetLastError();
    }
    switch (c) {
        case 4: return launch_c<RBC_KS, 4>(mode, grid, a, st);
        case 8: return launch_c<RBC_KS, 8>(mode, grid, a, st);
        case 16: return launch_c<RBC_KS, 16>(mode, grid, a, st);
        case 32: return launch_c<RBC_KS, 32>(mode, grid, a, st);
        case 64: return launch_c<RBC_KS, 64>(mode, grid, a, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace rbc
