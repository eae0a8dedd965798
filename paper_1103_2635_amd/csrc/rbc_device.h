// rbc_device.h -- device helpers shared by the tile kernels: the per-query
// shortlist (the comparison step of BF, Sec. 3, kept as a sorted top-c list in
// registers) and the walk over the rows a workgroup has to scan.
#pragma once

#include "rbc_common.h"

namespace rbc {

#define RBC_INF __builtin_huge_valf()
#define RBC_INF_D __builtin_huge_val()

// Float64 distance in a fixed order: differences of the exactly converted
// inputs, summed from the first feature to the last, no fused multiply-add.
static __device__ __noinline__ double rho_fp64(const float* a, const float* b, int d, int metric) {
#pragma clang fp contract(off)
    double s = 0.0;
    if (metric == 1) {
        for (int i = 0; i < d; ++i) s += __builtin_fabs((double)a[i] - (double)b[i]);
        return s;
    }
    for (int i = 0; i < d; ++i) {
        const double t = (double)a[i] - (double)b[i];
        s += t * t;
    }
    return __builtin_sqrt(s);
}

// True when the matrix-core tile value ||x||^2 - 2 q.x is computed without
// rounding: every input is an integer and every product and partial sum is
// an integer of magnitude below 2^24 (exactly representable in fp32), in any
// summation order.  With non-negative inputs all partial sums lie between
// -d M^2 and d M^2 (M = the largest magnitude), otherwise within 3 d M^2.
// fa / fb are value flags: [0] bit 1 = computed, bit 0 = non-integer seen,
// [1] max |v| bits, [2] negative seen.
__device__ __forceinline__ bool tile_exact(const uint32_t* fa, const uint32_t* fb, int d) {
    if (!fa || !fb) return false;
    if (fa[0] != 2u || fb[0] != 2u) return false;  // not computed, or a non-integer value
    const double ma = (double)__uint_as_float(fa[1]);
    const double mb = (double)__uint_as_float(fb[1]);
    const double m = ma > mb ? ma : mb;
    const bool neg = (fa[2] | fb[2]) != 0;
    return neg ? 3.0 * d * m * m <= 16777216.0 : d * m * m <= 8388608.0;
}

// Layout of a BF-mode search whose query count is known on the device only:
// a fixed 1-D grid of `blocks` workgroups (256 queries each) is spread over
// the A = ceil(cnt / 256) active query blocks, S = blocks / A database splits
// each (at most one per 32 rows), rps rows per split; the partial list of
// split s for query q sits at (s * M + q) * C with M = 256 A.
struct DevSplit {
    int A, S, rps, M;
};

__device__ __forceinline__ DevSplit dev_split(int cnt, int blocks, int n) {
    DevSplit r;
    r.A = (cnt + 255) >> 8;
    r.M = r.A << 8;
    int s = r.A > 0 ? blocks / r.A : 1;
    const int smax = (n + 31) >> 5;
    s = s < 1 ? 1 : (s > smax ? smax : s);
    r.S = s;
    r.rps = (((n + s - 1) / s) + 31) & ~31;
    return r;
}

// (distance, id) lexicographic order.
__device__ __forceinline__ bool before(double va, int64_t ia, double vb, int64_t ib) {
    return va < vb || (va == vb && ia < ib);
}

// Sorted ascending top-C list held by one lane.  Values arrive in increasing
// row order, so the strict comparison keeps the earlier (lower) row on a tie.
template <int C>
struct TopC {
    float v[C];
    int32_t i[C];

    __device__ __forceinline__ void init() {
#pragma unroll
        for (int j = 0; j < C; ++j) {
            v[j] = RBC_INF;
            i[j] = -1;
        }
    }

    // Start from a known bound: only values below t can enter.
    __device__ __forceinline__ void seed(float t) {
#pragma unroll
        for (int j = 0; j < C; ++j) {
            v[j] = t;
            i[j] = -1;
        }
    }

    __device__ __forceinline__ float worst() const { return v[C - 1]; }

    // Insert (x, id) given x < v[C - 1]; the last entry drops out.
    __device__ __forceinline__ void insert(float x, int32_t id) {
        bool lt[C];
#pragma unroll
        for (int j = 0; j < C; ++j) lt[j] = x < v[j];
#pragma unroll
        for (int j = C - 1; j > 0; --j) {
            const float nv = lt[j - 1] ? v[j - 1] : (lt[j] ? x : v[j]);
            const int32_t ni = lt[j - 1] ? i[j - 1] : (lt[j] ? id : i[j]);
            v[j] = nv;
            i[j] = ni;
        }
        v[0] = lt[0] ? x : v[0];
        i[0] = lt[0] ? id : i[0];
    }

    __device__ __forceinline__ void push(float x, int32_t id) {
        if (x < v[C - 1]) insert(x, id);
    }

    __device__ __forceinline__ void store(float* pv, int32_t* pi) const {
#pragma unroll
        for (int j = 0; j < C; ++j) {
            pv[j] = v[j];
            pi[j] = i[j];
        }
    }
};

// Insert (x, id) into a sorted shortlist in (value, row) order; merging two
// shortlists this way keeps the c smallest values of their union.
template <int C>
__device__ __forceinline__ void insert_lex(TopC<C>& t, float x, int32_t id) {
    bool lt[C];
#pragma unroll
    for (int j = 0; j < C; ++j) lt[j] = x < t.v[j] || (x == t.v[j] && id < t.i[j]);
    if (!lt[C - 1]) return;
#pragma unroll
    for (int j = C - 1; j > 0; --j) {
        const float nv = lt[j - 1] ? t.v[j - 1] : (lt[j] ? x : t.v[j]);
        const int32_t ni = lt[j - 1] ? t.i[j - 1] : (lt[j] ? id : t.i[j]);
        t.v[j] = nv;
        t.i[j] = ni;
    }
    t.v[0] = lt[0] ? x : t.v[0];
    t.i[0] = lt[0] ? id : t.i[0];
}


// Representative of work item `item` (item mode): the last r with
// ioff[r] <= item (representatives without items have ioff[r] == ioff[r + 1]).
__device__ __forceinline__ int item_rep(const TileArgs& a, int item) {
    int lo = 0, hi = a.n_r - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.ioff[mid] <= item) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Makes this wavefront's LDS writes visible to its own later LDS reads (and
// keeps the compiler from moving LDS accesses across the point).  LDS
// operations of one wavefront are executed in issue order.
// The smallest float not below x (x >= 0, finite).
__device__ __forceinline__ float round_up_f(double x) {
    float f = (float)x;
    if ((double)f < x) f = __uint_as_float(__float_as_uint(f) + 1u);
    return f;
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace rbc
