// tile_mfma32.h -- the fp32 matrix-core distance tile in the 32x32x2 shape
// (v_mfma_f32_32x32x2f32), for the Euclidean metric: val(x) = ||x||^2 - 2 q.x
// per (query, database row), the quantity whose per-query order is that of
// the distance (Sec. 3: the distance step of BF(Q, X) is a matrix product).
//
// Layout of one wavefront's tile: 32 database rows per block (the M side of
// the MFMA) by 64 queries (two 32-query blocks, the N side).  Lane l works in
// half h = l / 32 of the feature range: at k-step s it feeds feature
// 8 KS h + s of row (l mod 32) of the block, and of query 32 qb + (l mod 32),
// so each lane loads contiguous float4 runs of its own row and query.  The
// MFMA result gives lane l the values of query 32 qb + (l mod 32) for the
// rows 8 i + 4 h + j (i, j < 4) of the block: every lane already holds one
// query, so the comparison step needs no transpose.  Each lane keeps one
// shortlist per query block over its half of the rows; at the end the two
// halves of each query are merged with one cross-half shuffle, lane l ending
// with the list of query l.
//
// Per block and wavefront: 2 x 8 KS MFMAs of 64 cycles (the same work as the
// 16x16x4 tile in half the instructions), 2 KS float4 loads of database rows
// issued one block ahead and 16 row-norm loads issued at the block's start.
#pragma once

#include "rbc_device.h"

namespace rbc {

typedef float f16v __attribute__((ext_vector_type(16)));

// Features [8 KS h, 8 KS (h + 1)) of one row: 2 KS float4 runs; runs at or
// past d read the row's first run and are zeroed by a select, so every load
// is issued unconditionally (rows are zero-padded to whole float4 runs).
template <int KS>
__device__ __forceinline__ void load_half_row(f4 (&fr)[2 * KS], const float* base, int d, int h,
                                              float scale) {
#pragma unroll
    for (int j = 0; j < 2 * KS; ++j) {
        const int f = 8 * KS * h + 4 * j;
        const bool in = f < d;
        const f4 v = *(const f4*)(base + (in ? f : 0));
        const f4 z = {0.f, 0.f, 0.f, 0.f};
        fr[j] = (in ? v : z) * scale;
    }
}

// Norms of rows base + 8 i + 4 h + j (v = 4 i + j), clamped to r1 - 1.
__device__ __forceinline__ void load_norms32(float (&nv)[16], const float* xn, int base, int r1,
                                             int h) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int row = base + 8 * (v >> 2) + 4 * h + (v & 3);
        nv[v] = xn[row < r1 ? row : r1 - 1];
    }
}

template <int KS>
__device__ __forceinline__ void load_x32(f4 (&xf)[2 * KS], const TileArgs& a, int base, int c32,
                                         int h) {
    int row = base + c32;
    row = row < a.n ? row : a.n - 1;
    load_half_row<KS>(xf, a.X + (int64_t)row * a.ldx, a.d, h, 1.0f);
}

// Lane l holds, per query block qb, the shortlist of query 32 qb + (l mod 32)
// over its half of the rows.  Lane l ends with the merged list of query l:
// its own list of block h and the list of the same query kept by lane l ^ 32.
template <int C>
__device__ __forceinline__ TopC<C> merge_halves(const TopC<C> (&top)[2], int h) {
    TopC<C> own, mine;
#pragma unroll
    for (int j = 0; j < C; ++j) {
        own.v[j] = h ? top[1].v[j] : top[0].v[j];
        own.i[j] = h ? top[1].i[j] : top[0].i[j];
        // the partner (half 1 - h) needs block 1 - h of this lane
        mine.v[j] = __shfl_xor(h ? top[0].v[j] : top[1].v[j], 32);
        mine.i[j] = __shfl_xor(h ? top[0].i[j] : top[1].i[j], 32);
    }
#pragma unroll
    for (int j = 0; j < C; ++j) insert_lex<C>(own, mine.v[j], mine.i[j]);
    return own;
}

// One block: the values of rows [base, base + 32) for both query blocks,
// then the pushes.  The MFMAs accumulate -2 q.x from zero and the row norms
// (loaded at the start of the block, ahead of the MFMAs) are added after
// them, which keeps a single norm buffer.  A block whose values all lie at or
// above their list's bound is skipped after a per-lane minimum.
template <int KS, int C>
__device__ __forceinline__ void scan_block32(const f4 (&qf)[2][2 * KS], const f4 (&xf)[2 * KS],
                                             const float (&nr)[16], int base, int r1,
                                             const bool (&act)[2], TopC<C> (&top)[2], int h) {
    f16v acc[2];
#pragma unroll
    for (int qb = 0; qb < 2; ++qb)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[qb][v] = 0.f;
#pragma unroll
    for (int j = 0; j < 2 * KS; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int qb = 0; qb < 2; ++qb)
                acc[qb] = __builtin_amdgcn_mfma_f32_32x32x2f32(xf[j][e], qf[qb][j][e], acc[qb], 0,
                                                               0, 0);
    bool need = false;
#pragma unroll
    for (int qb = 0; qb < 2; ++qb) {
        float mn = RBC_INF;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int row = base + 8 * (v >> 2) + 4 * h + (v & 3);
            acc[qb][v] = row < r1 ? acc[qb][v] + nr[v] : RBC_INF;
            mn = fminf(mn, acc[qb][v]);
        }
        need |= act[qb] && mn < top[qb].worst();
    }
    if (__ballot(need) == 0ull) return;
#pragma unroll
    for (int qb = 0; qb < 2; ++qb) {
        if (!act[qb]) continue;
#pragma unroll
        for (int v = 0; v < 16; ++v)
            top[qb].push(acc[qb][v], base + 8 * (v >> 2) + 4 * h + (v & 3));
    }
}

// Scan rows [r0, r1) for the wavefront's 64 queries.  Per block: the block's
// norms are loaded first, then the next block's rows into the other buffer
// (so waiting for the norms never waits for those rows), then the MFMAs.
template <int KS, int C>
__device__ __forceinline__ void scan_rows32(const f4 (&qf)[2][2 * KS], const TileArgs& a, int r0,
                                            int r1, const bool (&act)[2], TopC<C> (&top)[2],
                                            int lane) {
    const int h = lane >> 5;
    const int c32 = lane & 31;
    f4 xa[2 * KS], xb[2 * KS];
    float nr[16];
    load_x32<KS>(xa, a, r0, c32, h);
    int base = r0;
    for (;;) {
        int next = base + kRowsMfma;
        int nbase = next < r1 ? next : base;
        load_norms32(nr, a.xn, base, r1, h);
        load_x32<KS>(xb, a, nbase, c32, h);
        __builtin_amdgcn_sched_barrier(0);
        scan_block32<KS, C>(qf, xa, nr, base, r1, act, top, h);
        base = next;
        if (base >= r1) break;
        next = base + kRowsMfma;
        nbase = next < r1 ? next : base;
        load_norms32(nr, a.xn, base, r1, h);
        load_x32<KS>(xa, a, nbase, c32, h);
        __builtin_amdgcn_sched_barrier(0);
        scan_block32<KS, C>(qf, xb, nr, base, r1, act, top, h);
        base = next;
        if (base >= r1) break;
    }
}

// Query fragments (-2 q) of the wavefront's two 32-query blocks.
template <int KS>
__device__ __forceinline__ void load_q32(f4 (&qf)[2][2 * KS], const TileArgs& a,
                                         const int (&qrow)[2], int h) {
#pragma unroll
    for (int qb = 0; qb < 2; ++qb)
        load_half_row<KS>(qf[qb], a.Q + (int64_t)qrow[qb] * a.ldq, a.d, h, -2.0f);
}

// BF mode, as tile_bf_body: grid (query blocks of 256, database splits), or a
// 1-D grid laid out by dev_split for a device-side query count.
template <int KS, int C>
__device__ __forceinline__ void tile32_bf_body(const TileArgs& a) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int h = lane >> 5;
    const int c32 = lane & 31;
    int m = a.m, qblk = blockIdx.x, split = blockIdx.y, stride = a.m;
    int64_t rps = a.rps;
    if (a.m_dev) {
        m = *a.m_dev;
        const DevSplit ds = dev_split(m, a.dev_blocks, a.n);
        qblk = blockIdx.x / ds.S;
        split = blockIdx.x % ds.S;
        if (qblk >= ds.A) return;
        stride = ds.M;
        rps = ds.rps;
    }
    const int slot0 = qblk * kTileQ + wave * kWave;
    if (slot0 >= m) return;  // uniform per wavefront
    f4 qf[2][2 * KS];
    int qrow[2];
    bool act[2];
#pragma unroll
    for (int qb = 0; qb < 2; ++qb) {
        const int slot = slot0 + 32 * qb + c32;
        act[qb] = slot < m;
        qrow[qb] = act[qb] ? slot : m - 1;
    }
    load_q32<KS>(qf, a, qrow, h);
    TopC<C> top[2];
    top[0].init();
    top[1].init();
    const int64_t r0 = (int64_t)split * rps;
    const int64_t r1 = r0 + rps < a.n ? r0 + rps : a.n;
    if (r0 < r1) scan_rows32<KS, C>(qf, a, (int)r0, (int)r1, act, top, lane);
    const TopC<C> mine = merge_halves<C>(top, h);
    const int myslot = slot0 + lane;
    if (myslot < m) {
        const int64_t off = ((int64_t)split * stride + myslot) * C;
        mine.store(a.pval + off, a.pidx + off);
    }
}

// An item record (8 int32, uniform across the wavefront) through the
// scalar unit: constant address space, so it lands in scalar registers.
struct ItemRec32 {
    int r, q_begin, q_end, r0, r1;
};

__device__ __forceinline__ ItemRec32 load_rec(const int32_t* irec, int pos) {
    typedef const __attribute__((address_space(4))) int32_t cint;
    cint* p = (cint*)(irec + (int64_t)kItemRec * pos);
    return ItemRec32{p[0], p[1], p[2], p[3], p[4]};
}

// Item mode over records in longest-first order (see tile_recs_body): the
// item's queries, bounds and output slots, the next record and ticket loaded
// during the scan.
template <int KS, int C>
__device__ __forceinline__ void tile32_recs_body(const TileArgs& a) {
    const int lane = threadIdx.x & 63;
    const int h = lane >> 5;
    const int c32 = lane & 31;
    const int total = *a.item_total;
    int ticket = 0;
    if (lane == 0) ticket = atomicAdd(a.item_queue, 1);
    const int first = __builtin_amdgcn_readfirstlane(__shfl(ticket, 0));
    if (first >= total) return;
    ItemRec32 rc = load_rec(a.irec, first);
    if (lane == 0) ticket = atomicAdd(a.item_queue, 1);
    for (;;) {
        const int r = rc.r, q_begin = rc.q_begin, q_end = rc.q_end, r0 = rc.r0, r1 = rc.r1;
        int qrow[2];
        bool act[2];
#pragma unroll
        for (int qb = 0; qb < 2; ++qb) {
            const int p = q_begin + 32 * qb + c32;
            act[qb] = p < q_end;
            qrow[qb] = a.qlist[act[qb] ? p : q_end - 1];
        }
        const int p = q_begin + lane;
        const bool valid = p < q_end;
        const int q = a.qlist[valid ? p : q_end - 1];
        const int nxt = __builtin_amdgcn_readfirstlane(__shfl(ticket, 0));
        const bool more = nxt < total;
        const ItemRec32 nrc = load_rec(a.irec, more ? nxt : first);
        if (lane == 0 && more) ticket = atomicAdd(a.item_queue, 1);
        f4 qf[2][2 * KS];
        load_q32<KS>(qf, a, qrow, h);
        // shortlist seeds: the bound of query 32 qb + c32, on both halves
        TopC<C> top[2];
#pragma unroll
        for (int qb = 0; qb < 2; ++qb) {
            if (a.tau) top[qb].seed(a.tau[qrow[qb]]); else top[qb].init();
        }
        const int64_t pair = (int64_t)a.qoff[q] + a.lrank[(int64_t)q * a.n_r + r];
        if (r0 < r1) scan_rows32<KS, C>(qf, a, r0, r1, act, top, lane);
        const TopC<C> mine = merge_halves<C>(top, h);
        if (valid) mine.store(a.pval + pair * C, a.pidx + pair * C);
        if (a.stats && lane == 0) {
            const int nq = q_end - q_begin < kWave ? q_end - q_begin : kWave;
            const int nrow = r1 > r0 ? r1 - r0 : 0;
            atomicAdd((unsigned long long*)&a.stats[2], (unsigned long long)nq * nrow);
            atomicAdd((unsigned long long*)&a.stats[6], 1ull);
            atomicAdd((unsigned long long*)&a.stats[7],
                      (unsigned long long)kWave * ((nrow + kRowsMfma - 1) / kRowsMfma * kRowsMfma));
        }
        if (!more) break;
        rc = nrc;
    }
}

}  // namespace rbc
