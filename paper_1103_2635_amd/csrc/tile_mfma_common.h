// tile_mfma_common.h -- the matrix-core distance tile, generic over the
// arithmetic of the contraction (fp32, bf16, fp8), shared by k_tile_mfma.hip
// (fp32), k_tile_bf16.hip and k_tile_fp8.hip.
//
// Sec. 3 observes that the distance step of BF(Q, X) is shaped like a
// matrix product.  For the Euclidean metric the ranking of database rows for
// a fixed query q only needs  val(x) = ||x||^2 - 2 q.x  (||q||^2 is common to
// all rows), a dense contraction over the d features.
//
// Layout of one wavefront's tile: rows of the 16x16 MFMA output are 32
// database rows (two 16-row blocks), columns are the wavefront's 64 queries
// (four 16-query blocks).  The first MFMA of each accumulator takes ||x||^2 as
// its C operand and the query fragments carry the factor -2 (exact in every
// format), so the MFMA result is val directly.  Which feature feeds which
// k-slot of an MFMA is free as long as both operands agree: every lane loads
// one contiguous run of features of its row per MFMA.  The database fragments
// of the next 32 rows are loaded while the current ones are used.
//
// The comparison step (per-query top-c) needs one query per lane, so each
// 32x64 block of results goes through a wavefront-private LDS tile (written as
// [query][row], read back one query per lane), then every lane pushes its 32
// values into a sorted register shortlist (TopC).
//
// A Policy provides
//   QFrag / XFrag          fragment types of one lane,
//   kBlocks                MFMAs per 16x16 output block (feature blocks),
//   load_q(frag, base, f)  the query run for feature block f (already -2 q),
//   load_x(frag, base, f)  the database run,
//   mma(xf, qf, c)         one MFMA step.
#pragma once

#include "rbc_device.h"

namespace rbc {

constexpr int kTStride = 36;  // floats per query row of the transpose tile

template <class P>
__device__ __forceinline__ void load_xfrags(typename P::XFrag (&xa)[2][P::kBlocks],
                                            const TileArgs& a, int base, int c16, int g) {
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
        int row = base + 16 * rb + c16;
        row = row < a.n ? row : a.n - 1;
#pragma unroll
        for (int f = 0; f < P::kBlocks; ++f) P::load_x(xa[rb][f], a, row, f, g);
    }
}

template <class P, int QB>
__device__ __forceinline__ void load_qfrags(typename P::QFrag (&qf)[QB][P::kBlocks],
                                            const TileArgs& a, const int (&qrow)[QB], int g) {
#pragma unroll
    for (int qb = 0; qb < QB; ++qb)
#pragma unroll
        for (int f = 0; f < P::kBlocks; ++f) P::load_q(qf[qb][f], a, qrow[qb], f, g);
}

// Squared norms of the rows base + 16 rb + 4 g + i (clamped to r1 - 1, so the
// loads need no branch); tile_step puts +inf at rows >= r1.
__device__ __forceinline__ void load_norms(f4 (&nr)[2], const float* xn, int base, int r1, int g) {
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = base + 16 * rb + 4 * g + i;
            nr[rb][i] = xn[row < r1 ? row : r1 - 1];
        }
}

// The 32 x 16 QB values of rows [base, base + 32): acc[rb][qb][i] is row
// base + 16 rb + 4 g + i, query 16 qb + c16 (+inf beyond r1).
template <class P, int QB>
__device__ __forceinline__ void tile_step(f4 (&acc)[2][QB], const typename P::QFrag (&qf)[QB][P::kBlocks],
                                          const typename P::XFrag (&xa)[2][P::kBlocks],
                                          const f4 (&nr)[2], int base, int r1, int g) {
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
        f4 nv;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = base + 16 * rb + 4 * g + i;
            nv[i] = row < r1 ? nr[rb][i] : RBC_INF;
        }
#pragma unroll
        for (int qb = 0; qb < QB; ++qb) acc[rb][qb] = P::mma(xa[rb][0], qf[qb][0], nv);
    }
#pragma unroll
    for (int f = 1; f < P::kBlocks; ++f)
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int qb = 0; qb < QB; ++qb) acc[rb][qb] = P::mma(xa[rb][f], qf[qb][f], acc[rb][qb]);
}

// Each lane keeps, for the four queries whose values it holds in the MFMA
// layout (16 qb + c16), a copy of their shortlist bound (-inf for lanes
// without a query, which never insert).
template <int C, int QB>
__device__ __forceinline__ void refresh_bounds(float (&wq)[QB], const TopC<C>& top, bool act,
                                               int c16) {
    const float w = act ? top.worst() : -RBC_INF;
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) wq[qb] = __shfl(w, 16 * qb + c16);
}

// One 32-row block: the values, the min-filter, and (only when some lane
// may insert) the transpose and the pushes.
template <class P, int C, int QB>
__device__ __forceinline__ void scan_block(const typename P::QFrag (&qf)[QB][P::kBlocks],
                                           const typename P::XFrag (&x)[2][P::kBlocks],
                                           const f4 (&nr)[2], int base, int r1, bool act,
                                           TopC<C>& top, float (&wq)[QB], float* tb, int lane) {
    const int g = lane >> 4;
    const int c16 = lane & 15;
    f4 acc[2][QB];
    tile_step<P, QB>(acc, qf, x, nr, base, r1, g);
    bool need = false;
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) {
        const float m0 = fminf(fminf(acc[0][qb][0], acc[0][qb][1]), fminf(acc[0][qb][2], acc[0][qb][3]));
        const float m1 = fminf(fminf(acc[1][qb][0], acc[1][qb][1]), fminf(acc[1][qb][2], acc[1][qb][3]));
        need |= fminf(m0, m1) < wq[qb];
    }
    if (__ballot(need) != 0ull) {
        // transpose: element (query 16 qb + c16, row 16 rb + 4 g + i)
        wave_lds_sync();
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int qb = 0; qb < QB; ++qb)
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
        refresh_bounds<C, QB>(wq, top, act, c16);
    }
}

// Scan database rows [r0, r1) for the wavefront's 64 queries; lanes with act
// push their values into top.  A 32-row block whose values all lie at or
// above their query's bound cannot change any shortlist, so it is skipped
// after a min-reduction in the MFMA layout; otherwise the block goes through
// the LDS transpose and every value is pushed (the pushes, and so the
// shortlists, are those of the plain scan).  Two fragment buffers alternate:
// while one block is scored, the next block's fragments and norms load into
// the other, issued before the block's MFMAs, with no register copies.
template <class P, int C, int QB = 4>
__device__ __forceinline__ void scan_rows(const typename P::QFrag (&qf)[QB][P::kBlocks],
                                          const TileArgs& a, int r0, int r1, bool act,
                                          TopC<C>& top, float* tb, int lane) {
    const int g = lane >> 4;
    const int c16 = lane & 15;
    float wq[QB];
    refresh_bounds<C, QB>(wq, top, act, c16);
    typename P::XFrag xa[2][P::kBlocks], xb[2][P::kBlocks];
    f4 na[2], nb[2];
    load_xfrags<P>(xa, a, r0, c16, g);
    load_norms(na, a.xn, r0, r1, g);
    int base = r0;
    for (;;) {
        int next = base + kRowsMfma;
        int nbase = next < r1 ? next : base;
        load_xfrags<P>(xb, a, nbase, c16, g);
        load_norms(nb, a.xn, nbase, r1, g);
        __builtin_amdgcn_sched_barrier(0);
        scan_block<P, C, QB>(qf, xa, na, base, r1, act, top, wq, tb, lane);
        base = next;
        if (base >= r1) break;
        next = base + kRowsMfma;
        nbase = next < r1 ? next : base;
        load_xfrags<P>(xa, a, nbase, c16, g);
        load_norms(na, a.xn, nbase, r1, g);
        __builtin_amdgcn_sched_barrier(0);
        scan_block<P, C, QB>(qf, xb, nb, base, r1, act, top, wq, tb, lane);
        base = next;
        if (base >= r1) break;
    }
}

// One query block per wavefront (QB = 1): lane (g, c16) holds the values of
// rows base + 16 rb + 4 g + i for query c16, and pushes them into its own
// shortlist, one of four per query (one per g), with no transpose: all 64
// lanes insert, 8 values each.  merge_groups joins the four at the end.
template <class P, int C>
__device__ __forceinline__ void scan_block_direct(const typename P::QFrag (&qf)[1][P::kBlocks],
                                                  const typename P::XFrag (&x)[2][P::kBlocks],
                                                  const f4 (&nr)[2], int base, int r1,
                                                  TopC<C>& top, int g) {
    f4 acc[2][1];
    tile_step<P, 1>(acc, qf, x, nr, base, r1, g);
    const float m0 = fminf(fminf(acc[0][0][0], acc[0][0][1]), fminf(acc[0][0][2], acc[0][0][3]));
    const float m1 = fminf(fminf(acc[1][0][0], acc[1][0][1]), fminf(acc[1][0][2], acc[1][0][3]));
    if (fminf(m0, m1) < top.worst()) {
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) top.push(acc[rb][0][i], base + 16 * rb + 4 * g + i);
    }
}

template <class P, int C>
__device__ __forceinline__ void scan_rows_direct(const typename P::QFrag (&qf)[1][P::kBlocks],
                                                 const TileArgs& a, int r0, int r1, TopC<C>& top,
                                                 int lane) {
    const int g = lane >> 4;
    const int c16 = lane & 15;
    typename P::XFrag xa[2][P::kBlocks], xb[2][P::kBlocks];
    f4 na[2], nb[2];
    load_xfrags<P>(xa, a, r0, c16, g);
    load_norms(na, a.xn, r0, r1, g);
    int base = r0;
    for (;;) {
        int next = base + kRowsMfma;
        int nbase = next < r1 ? next : base;
        load_xfrags<P>(xb, a, nbase, c16, g);
        load_norms(nb, a.xn, nbase, r1, g);
        __builtin_amdgcn_sched_barrier(0);
        scan_block_direct<P, C>(qf, xa, na, base, r1, top, g);
        base = next;
        if (base >= r1) break;
        next = base + kRowsMfma;
        nbase = next < r1 ? next : base;
        load_xfrags<P>(xa, a, nbase, c16, g);
        load_norms(na, a.xn, nbase, r1, g);
        __builtin_amdgcn_sched_barrier(0);
        scan_block_direct<P, C>(qf, xb, nb, base, r1, top, g);
        base = next;
        if (base >= r1) break;
    }
}

// The four shortlists of query c16 (lanes c16, c16 + 16, c16 + 32, c16 + 48)
// merged; lanes 0 .. 15 end with the merged list of their query.
template <int C>
__device__ __forceinline__ void merge_groups(TopC<C>& top) {
#pragma unroll
    for (int mask = 16; mask <= 32; mask <<= 1) {
        TopC<C> o;
#pragma unroll
        for (int j = 0; j < C; ++j) {
            o.v[j] = __shfl_xor(top.v[j], mask);
            o.i[j] = __shfl_xor(top.i[j], mask);
        }
#pragma unroll
        for (int j = 0; j < C; ++j) insert_lex<C>(top, o.v[j], o.i[j]);
    }
}

// BF mode: grid (query blocks of 256, database splits), or, with a device-side
// query count, a 1-D grid laid out by dev_split.
template <class P, int C>
__device__ __forceinline__ void tile_bf_body(const TileArgs& a, float* tbuf_wave) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int c16 = lane & 15;
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
    if (slot0 >= m) return;  // uniform per wavefront; no workgroup barrier follows
    typename P::QFrag qf[4][P::kBlocks];
    int qrow[4];
#pragma unroll
    for (int qb = 0; qb < 4; ++qb) {
        const int slot = slot0 + 16 * qb + c16;
        qrow[qb] = slot < m ? slot : m - 1;
    }
    load_qfrags<P, 4>(qf, a, qrow, g);
    const int myslot = slot0 + lane;
    TopC<C> top;
    top.init();
    const int64_t r0 = (int64_t)split * rps;
    const int64_t r1 = r0 + rps < a.n ? r0 + rps : a.n;
    if (r0 < r1) scan_rows<P, C>(qf, a, (int)r0, (int)r1, myslot < m, top, tbuf_wave, lane);
    if (myslot < m) {
        const int64_t off = ((int64_t)split * stride + myslot) * C;
        top.store(a.pval + off, a.pidx + off);
    }
}

// Item mode: persistent wavefronts, each taking (representative, 16 QB-query
// chunk) items from the queue until it is empty.  Wavefronts work
// independently (no workgroup barrier); consecutive items usually belong to
// the same representative, so co-resident wavefronts share its list rows in
// the caches.
template <class P, int C, int QB = 4>
__device__ __forceinline__ void tile_items_body(const TileArgs& a, float* tbuf_wave) {
    constexpr int kQ = 16 * QB;  // queries per item
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4;
    const int c16 = lane & 15;
    const int total = *a.item_total;
    // The next item's ticket is taken while the current item is scanned, so
    // the queue's latency is off the critical path.  The ticket is made
    // wave-uniform (readfirstlane) so the loop control is scalar.
    int ticket = 0;
    if (lane == 0) ticket = atomicAdd(a.item_queue, 1);
    for (;;) {
        const int item = __builtin_amdgcn_readfirstlane(__shfl(ticket, 0));
        if (item >= total) break;
        const int r = a.irep ? __builtin_amdgcn_readfirstlane(a.irep[item]) : item_rep(a, item);
        int chunk = item - a.ioff[r], split = 0;
        if (a.isplit > 1) {
            split = chunk % a.isplit;
            chunk /= a.isplit;
        }
        const int q_begin = a.roff[r] + chunk * kQ;
        const int q_end = a.roff[r + 1];
        typename P::QFrag qf[QB][P::kBlocks];
        int qrow[QB];
#pragma unroll
        for (int qb = 0; qb < QB; ++qb) {
            const int p = q_begin + 16 * qb + c16;
            qrow[qb] = a.qlist[p < q_end ? p : q_end - 1];
        }
        load_qfrags<P, QB>(qf, a, qrow, g);
        const int p = q_begin + lane;
        const bool valid = lane < kQ && p < q_end;
        const int q = a.qlist[valid ? p : q_end - 1];
        TopC<C> top;
        if constexpr (QB == 1) {
            // every lane keeps a shortlist of query c16 (see scan_block_direct);
            // lanes of empty query slots never insert
            if (q_begin + c16 >= q_end) top.seed(-RBC_INF);
            else if (a.tau) top.seed(a.tau[qrow[0]]);
            else top.init();
        } else if (a.tau) {
            top.seed(a.tau[q]);
        } else {
            top.init();
        }
        int r0 = a.list_off[r], r1 = a.list_off[r + 1];
        if (a.irows) {
            r0 = __builtin_amdgcn_readfirstlane(a.irows[2 * (int64_t)item]);
            r1 = __builtin_amdgcn_readfirstlane(a.irows[2 * (int64_t)item + 1]);
        } else if (a.isplit > 1) {
            const int64_t len = r1 - r0;
            r1 = r0 + (int)(len * (split + 1) / a.isplit);
            r0 = r0 + (int)(len * split / a.isplit);
        }
        // next ticket: issued after this item's metadata loads (memory
        // counters retire in issue order), consumed at the next iteration
        if (lane == 0) ticket = atomicAdd(a.item_queue, 1);
        if constexpr (QB == 1) {
            if (r0 < r1) scan_rows_direct<P, C>(qf, a, r0, r1, top, lane);
            merge_groups<C>(top);
        } else if (r0 < r1) {
            scan_rows<P, C, QB>(qf, a, r0, r1, valid, top, tbuf_wave, lane);
        }
        if (valid) {
            const int64_t pair = a.lrank ? (int64_t)a.qoff[q] + a.lrank[(int64_t)q * a.n_r + r]
                                         : (int64_t)q * (a.isplit > 1 ? a.isplit : 1) + split;
            top.store(a.pval + pair * C, a.pidx + pair * C);
        }
        if (a.stats && lane == 0) {
            const int nq = q_end - q_begin < kQ ? q_end - q_begin : kQ;
            const int nrow = r1 > r0 ? r1 - r0 : 0;
            atomicAdd((unsigned long long*)&a.stats[2], (unsigned long long)nq * nrow);
            atomicAdd((unsigned long long*)&a.stats[6], 1ull);
            atomicAdd((unsigned long long*)&a.stats[7],
                      (unsigned long long)kQ * ((nrow + kRowsMfma - 1) / kRowsMfma * kRowsMfma));
        }
    }
}

// Item mode over records (irec non-null, exact search pairs): the queue hands
// out positions of irec, which holds the items longest first, so the last
// items of the launch are short and the wavefronts finish together.  A record
// carries the item's representative, query range and row run, so an item
// starts with the loads of its query ids; the next record and the next ticket
// are loaded while the current item is scanned, and the output slot of each
// query is looked up before the scan.
template <class P, int C, int QB = 4>
__device__ __forceinline__ void tile_recs_body(const TileArgs& a, float* tbuf_wave) {
    constexpr int kQ = 16 * QB;  // queries per item
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4;
    const int c16 = lane & 15;
    const int total = *a.item_total;
    int ticket = 0;
    if (lane == 0) ticket = atomicAdd(a.item_queue, 1);
    const int first = __builtin_amdgcn_readfirstlane(__shfl(ticket, 0));
    if (first >= total) return;
    int4 rc0 = *(const int4*)(a.irec + (int64_t)kItemRec * first);
    int4 rc1 = *(const int4*)(a.irec + (int64_t)kItemRec * first + 4);
    if (lane == 0) ticket = atomicAdd(a.item_queue, 1);
    for (;;) {
        const int r = __builtin_amdgcn_readfirstlane(rc0.x);
        const int q_begin = __builtin_amdgcn_readfirstlane(rc0.y);
        const int q_end = __builtin_amdgcn_readfirstlane(rc0.z);
        const int r0 = __builtin_amdgcn_readfirstlane(rc0.w);
        const int r1 = __builtin_amdgcn_readfirstlane(rc1.x);
        int qrow[QB];
#pragma unroll
        for (int qb = 0; qb < QB; ++qb) {
            const int p = q_begin + 16 * qb + c16;
            qrow[qb] = a.qlist[p < q_end ? p : q_end - 1];
        }
        const int p = q_begin + lane;
        const bool valid = lane < kQ && p < q_end;
        const int q = a.qlist[valid ? p : q_end - 1];
        // the ticket taken during the previous item names the next record
        const int nxt = __builtin_amdgcn_readfirstlane(__shfl(ticket, 0));
        const bool more = nxt < total;
        const int nrec = more ? nxt : first;
        const int4 nr0 = *(const int4*)(a.irec + (int64_t)kItemRec * nrec);
        const int4 nr1 = *(const int4*)(a.irec + (int64_t)kItemRec * nrec + 4);
        if (lane == 0 && more) ticket = atomicAdd(a.item_queue, 1);
        typename P::QFrag qf[QB][P::kBlocks];
        load_qfrags<P, QB>(qf, a, qrow, g);
        TopC<C> top;
        if (a.tau) top.seed(a.tau[q]); else top.init();
        const int64_t pair = (int64_t)a.qoff[q] + a.lrank[(int64_t)q * a.n_r + r];
        if (r0 < r1) scan_rows<P, C, QB>(qf, a, r0, r1, valid, top, tbuf_wave, lane);
        if (valid) top.store(a.pval + pair * C, a.pidx + pair * C);
        if (a.stats && lane == 0) {
            const int nq = q_end - q_begin < kQ ? q_end - q_begin : kQ;
            const int nrow = r1 > r0 ? r1 - r0 : 0;
            atomicAdd((unsigned long long*)&a.stats[2], (unsigned long long)nq * nrow);
            atomicAdd((unsigned long long*)&a.stats[6], 1ull);
            atomicAdd((unsigned long long*)&a.stats[7],
                      (unsigned long long)kQ * ((nrow + kRowsMfma - 1) / kRowsMfma * kRowsMfma));
        }
        if (!more) break;
        rc0 = nr0;
        rc1 = nr1;
    }
}

// All mode: every value written out, out[q * ldo + row] (one-shot build).
template <class P>
__device__ __forceinline__ void tile_all_body(const TileArgs& a) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int c16 = lane & 15;
    const int slot0 = blockIdx.x * kTileQ + wave * kWave;
    typename P::QFrag qf[4][P::kBlocks];
    int qrow[4];
#pragma unroll
    for (int qb = 0; qb < 4; ++qb) {
        const int slot = slot0 + 16 * qb + c16;
        qrow[qb] = slot < a.m ? slot : a.m - 1;
    }
    load_qfrags<P, 4>(qf, a, qrow, g);
    const int r0 = (int)((int64_t)blockIdx.y * a.rps);
    const int r1 = (int)(r0 + (int64_t)a.rps < a.n ? r0 + a.rps : a.n);
    if (r0 >= r1) return;
    typename P::XFrag xa[2][P::kBlocks];
    f4 na[2];
    load_xfrags<P>(xa, a, r0, c16, g);
    load_norms(na, a.xn, r0, r1, g);
    for (int base = r0; base < r1; base += kRowsMfma) {
        typename P::XFrag xb[2][P::kBlocks];
        f4 nb[2];
        const int next = base + kRowsMfma;
        const int nbase = next < r1 ? next : base;
        load_xfrags<P>(xb, a, nbase, c16, g);
        load_norms(nb, a.xn, nbase, r1, g);
        f4 acc[2][4];
        tile_step<P, 4>(acc, qf, xa, na, base, r1, g);
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
        for (int rb = 0; rb < 2; ++rb) {
            na[rb] = nb[rb];
#pragma unroll
            for (int f = 0; f < P::kBlocks; ++f) xa[rb][f] = xb[rb][f];
        }
    }
}

}  // namespace rbc
