// k_tile_mfma.hip -- fp32 matrix-core distance tile (v_mfma_f32_16x16x4f32).
//
// Fragment of one lane for slab s (16 features): the float4 at features
// 16 s + 4 (l / 16) of its row; its four components feed four consecutive
// MFMAs (k-slot l / 16 each).  Query fragments are -2 q (exact).  The scan,
// transpose and shortlist are in tile_mfma_common.h.
#include "tile_mfma_common.h"
#include "tile_mfma32.h"

#ifndef RBC_KS
#error "compile with -DRBC_KS=<1..8>"
#endif

namespace rbc {

template <int KS>
struct Fp32Policy {
    typedef f4 QFrag;
    typedef f4 XFrag;
    static constexpr int kBlocks = KS;
    // Runs past the last feature read the row's first run and are zeroed by a
    // select: every load is issued unconditionally, so the compiler can count
    // the outstanding loads exactly and the prefetch stays one block ahead.
    static __device__ __forceinline__ void load_q(f4& q, const TileArgs& a, int row, int s, int g) {
        const int f = 16 * s + 4 * g;
        const bool in = f < a.d;
        const f4 v = *(const f4*)(a.Q + (int64_t)row * a.ldq + (in ? f : 0));
        const f4 z = {0.f, 0.f, 0.f, 0.f};
        q = (in ? v : z) * -2.0f;
    }
    static __device__ __forceinline__ void load_x(f4& x, const TileArgs& a, int row, int s, int g) {
        const int f = 16 * s + 4 * g;
        const bool in = f < a.d;
        const f4 v = *(const f4*)(a.X + (int64_t)row * a.ldx + (in ? f : 0));
        const f4 z = {0.f, 0.f, 0.f, 0.f};
        x = in ? v : z;
    }
    static __device__ __forceinline__ f4 mma(const f4& x, const f4& q, f4 c) {
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(x[0], q[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(x[1], q[1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(x[2], q[2], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(x[3], q[3], c, 0, 0, 0);
        return c;
    }
};

// Two workgroups per CU while the register footprint allows it.
template <int KS, int C>
struct MfmaOcc {
    static constexpr int value = (32 * KS + 2 * C + 64 <= 232) ? 2 : 1;
};

template <int KS, int C>
__global__ __launch_bounds__(256, (MfmaOcc<KS, C>::value)) void tile_l2_mfma(TileArgs a) {
    __shared__ __attribute__((aligned(16))) float tbuf[4][64 * kTStride];
    tile_bf_body<Fp32Policy<KS>, C>(a, tbuf[threadIdx.x >> 6]);
}

template <int KS, int C>
__global__ __launch_bounds__(256, (MfmaOcc<KS, C>::value)) void tile_l2_mfma_items(TileArgs a) {
    __shared__ __attribute__((aligned(16))) float tbuf[4][64 * kTStride];
    if (a.irec)
        tile_recs_body<Fp32Policy<KS>, C>(a, tbuf[threadIdx.x >> 6]);
    else
        tile_items_body<Fp32Policy<KS>, C>(a, tbuf[threadIdx.x >> 6]);
}

// Stage 2 on 32-query items (two query blocks per wavefront): narrower row
// runs per item and about 170 VGPRs, so three wavefronts per SIMD.
template <int KS, int C>
struct Mfma32qOcc {
    static constexpr int value = (16 * KS + 2 * C + 96 <= 168) ? 3 : (MfmaOcc<KS, C>::value);
};

template <int KS, int C>
__global__ __launch_bounds__(256, (Mfma32qOcc<KS, C>::value)) void tile_l2_mfma_items32q(TileArgs a) {
    __shared__ __attribute__((aligned(16))) float tbuf[4][64 * kTStride];
    tile_recs_body<Fp32Policy<KS>, C, 2>(a, tbuf[threadIdx.x >> 6]);
}

// Pass 1 of the two-pass search: the item body over the nearest lists, with
// 16-query items (one query block per wavefront): a nearest list holds few
// queries (about m / n_r), so wider items would mostly score empty slots.
// Each lane inserts its own MFMA outputs into one of four shortlists per
// query (scan_rows_direct), so the kernel needs no LDS.
template <int KS, int C>
__global__ __launch_bounds__(256, (MfmaOcc<KS, C>::value)) void tile_l2_mfma_home(TileArgs a) {
    tile_items_body<Fp32Policy<KS>, C, 1>(a, nullptr);  // no transpose, no LDS
}

// The 32x32x2 shape (tile_mfma32.h): no LDS, two shortlists per lane.
template <int KS, int C>
struct Mfma32Occ {
    static constexpr int value = (32 * KS + 4 * C + 96 <= 256) ? 2 : 1;
};

template <int KS, int C>
__global__ __launch_bounds__(256, (Mfma32Occ<KS, C>::value)) void tile_l2_mfma32(TileArgs a) {
    tile32_bf_body<KS, C>(a);
}

template <int KS, int C>
__global__ __launch_bounds__(256, (Mfma32Occ<KS, C>::value)) void tile_l2_mfma32_items(TileArgs a) {
    tile32_recs_body<KS, C>(a);
}

template <int KS>
__global__ __launch_bounds__(256, 2) void tile_l2_mfma_all(TileArgs a) {
    tile_all_body<Fp32Policy<KS>>(a);
}

template <int KS, int C>
static hipError_t launch_c(int mode, dim3 grid, const TileArgs& a, hipStream_t st) {
    if (a.shape == kShape32 && mode == kTileBF)
        hipLaunchKernelGGL((tile_l2_mfma32<KS, C>), grid, dim3(256), 0, st, a);
    else if (a.shape == kShape32 && mode == kTileItems && a.irec)
        hipLaunchKernelGGL((tile_l2_mfma32_items<KS, C>), grid, dim3(256), 0, st, a);
    else if (a.qb == 2 && mode == kTileItems && a.irec)
        hipLaunchKernelGGL((tile_l2_mfma_items32q<KS, C>), grid, dim3(256), 0, st, a);
    else if (mode == kTileItems)
        hipLaunchKernelGGL((tile_l2_mfma_items<KS, C>), grid, dim3(256), 0, st, a);
    else if (mode == kTileHome)
        hipLaunchKernelGGL((tile_l2_mfma_home<KS, C>), grid, dim3(256), 0, st, a);
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
