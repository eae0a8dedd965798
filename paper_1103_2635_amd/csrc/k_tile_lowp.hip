// k_tile_lowp.hip -- low-precision matrix-core distance tiles, fp32 accumulate:
//   bf16: v_mfma_f32_16x16x32_bf16; a lane's fragment for feature block f is
//         the 8 consecutive bf16 at features 32 f + 8 (l / 16) of its row;
//   fp8:  v_mfma_scale_f32_16x16x128_f8f6f4 with OCP e4m3 operands; a lane's
//         fragment for block f is the 32 bytes at features 128 f + 32 (l / 16)
//         and the row's power-of-two scale (E8M0 byte), which the instruction
//         applies to the products.
// Q and X of TileArgs point at the quantised rows (queries hold -2 q~), with
// row strides in elements; xn holds ||x~||^2.  The scan, transpose and
// shortlist are in tile_mfma_common.h.  Compiled once per feature-block count
// RBC_KB (1..4, i.e. d <= 32 RBC_KB for bf16; fp8 uses one 128-feature block).
#include "tile_mfma_common.h"

#ifndef RBC_KB
#error "compile with -DRBC_KB=<1..4>"
#endif

namespace rbc {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

template <int KB>
struct Bf16Policy {
    typedef bf16x8 QFrag;
    typedef bf16x8 XFrag;
    static constexpr int kBlocks = KB;
    static __device__ __forceinline__ void load_q(bf16x8& q, const TileArgs& a, int row, int f, int g) {
        q = *(const bf16x8*)((const uint16_t*)a.Q + (int64_t)row * a.ldq + 32 * f + 8 * g);
    }
    static __device__ __forceinline__ void load_x(bf16x8& x, const TileArgs& a, int row, int f, int g) {
        x = *(const bf16x8*)((const uint16_t*)a.X + (int64_t)row * a.ldx + 32 * f + 8 * g);
    }
    static __device__ __forceinline__ f4 mma(const bf16x8& x, const bf16x8& q, f4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, q, c, 0, 0, 0);
    }
};

struct Fp8Frag {
    i32x8 v;
    int scale;
};

struct Fp8Policy {
    typedef Fp8Frag QFrag;
    typedef Fp8Frag XFrag;
    static constexpr int kBlocks = 1;
    static __device__ __forceinline__ void load_q(Fp8Frag& q, const TileArgs& a, int row, int f, int g) {
        q.v = *(const i32x8*)((const uint8_t*)a.Q + (int64_t)row * a.ldq + 128 * f + 32 * g);
        q.scale = a.qscale[row];
    }
    static __device__ __forceinline__ void load_x(Fp8Frag& x, const TileArgs& a, int row, int f, int g) {
        x.v = *(const i32x8*)((const uint8_t*)a.X + (int64_t)row * a.ldx + 128 * f + 32 * g);
        x.scale = a.xscale[row];
    }
    static __device__ __forceinline__ f4 mma(const Fp8Frag& x, const Fp8Frag& q, f4 c) {
        // formats 0/0: e4m3 x e4m3; scale bytes selected at byte 0
        return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(x.v, q.v, c, 0, 0, 0, x.scale, 0,
                                                                q.scale);
    }
};

template <int KB, int C>
__global__ __launch_bounds__(256, 2) void tile_bf16(TileArgs a) {
    __shared__ __attribute__((aligned(16))) float tbuf[4][64 * kTStride];
    tile_bf_body<Bf16Policy<KB>, C>(a, tbuf[threadIdx.x >> 6]);
}

template <int C>
__global__ __launch_bounds__(256, 2) void tile_fp8(TileArgs a) {
    __shared__ __attribute__((aligned(16))) float tbuf[4][64 * kTStride];
    tile_bf_body<Fp8Policy, C>(a, tbuf[threadIdx.x >> 6]);
}

template <int KB, int C>
__global__ __launch_bounds__(256, 2) void tile_bf16_items(TileArgs a) {
    __shared__ __attribute__((aligned(16))) float tbuf[4][64 * kTStride];
    tile_items_body<Bf16Policy<KB>, C>(a, tbuf[threadIdx.x >> 6]);
}

template <int C>
__global__ __launch_bounds__(256, 2) void tile_fp8_items(TileArgs a) {
    __shared__ __attribute__((aligned(16))) float tbuf[4][64 * kTStride];
    tile_items_body<Fp8Policy, C>(a, tbuf[threadIdx.x >> 6]);
}

template <int C>
static hipError_t launch_c(int fmt, int mode, dim3 grid, const TileArgs& a, hipStream_t st) {
    if (fmt == 0) {
        if (mode == kTileItems)
            hipLaunchKernelGGL((tile_bf16_items<RBC_KB, C>), grid, dim3(256), 0, st, a);
        else
            hipLaunchKernelGGL((tile_bf16<RBC_KB, C>), grid, dim3(256), 0, st, a);
    } else {
        if (mode == kTileItems)
            hipLaunchKernelGGL((tile_fp8_items<C>), grid, dim3(256), 0, st, a);
        else
            hipLaunchKernelGGL((tile_fp8<C>), grid, dim3(256), 0, st, a);
    }
    return hipGetLastError();
}

hipError_t RBC_CAT(launch_tile_lowp_kb, RBC_KB)(int fmt, int c, int mode, dim3 grid,
                                                const TileArgs& a, hipStream_t st) {
    if (fmt == 1 && RBC_KB != 1) return hipErrorInvalidValue;  // fp8 kernels live in the KB = 1 object
    switch (c) {
        case 4: return launch_c<4>(fmt, mode, grid, a, st);
        case 8: return launch_c<8>(fmt, mode, grid, a, st);
        case 16: return launch_c<16>(fmt, mode, grid, a, st);
        case 32: return launch_c<32>(fmt, mode, grid, a, st);
        case 64: return launch_c<64>(fmt, mode, grid, a, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace rbc
