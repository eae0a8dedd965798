// k_quant.hip -- quantisation of query / database rows for the low-precision
// distance tiles (bf16 and fp8 e4m3 with a per-row power-of-two scale).
//
// Per row the kernel writes the quantised values (times `mult`, -2 for
// queries, which is exact in both formats), the squared norm of the
// quantised row ||x~||^2 (fp32), and an upper bound on the quantisation
// error ||x - x~|| (its fp32 sum widened by the sum's relative error).
// Optionally (norm32, flags32) also the fp32 squared norm of the row itself
// and the value flags of the row-norm kernel, from the same read.  The
// largest row norm and the largest error go to stat words through integer
// atomic maxima on non-negative float bits.
//   stat[0] = max ||x~||, stat[1] = max ||x - x~||.
#include <cmath>

#include "rbc_device.h"
#include "rbc_kernels.h"

namespace rbc {

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float v) {
    const uint32_t u = __float_as_uint(v);
    const uint32_t r = ((u >> 16) & 1u) + 0x7fffu;
    return (uint16_t)((u + r) >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// OCP fp8 e4m3 (bias 7, no infinities, largest finite 448), round to nearest
// even, saturating.  Inputs are finite and |v| <= 448 after scaling.
__device__ __forceinline__ uint8_t f32_to_e4m3(float v) {
    const uint32_t u = __float_as_uint(v);
    const uint8_t sign = (uint8_t)((u >> 24) & 0x80u);
    float a = __builtin_fabsf(v);
    if (a >= 448.f) return sign | 0x7eu;
    if (a < 0.0009765625f) {  // below half the smallest subnormal 2^-9
        return sign;
    }
    int e;
    frexpf(a, &e);             // a = f * 2^e, f in [0.5, 1)
    int ue = e - 1;            // unbiased exponent of a
    if (ue < -6) ue = -6;      // subnormal range: fixed exponent -6
    const float step = ldexpf(1.f, ue - 3);   // spacing of representable values
    float qv = __builtin_rintf(a / step) * step;  // round to nearest even multiple
    if (qv >= 448.f) qv = 448.f;
    // encode
    int qe;
    const float qf = frexpf(qv, &qe);
    int be = qe - 1 + 7;       // biased exponent
    uint32_t mant;
    if (qv == 0.f) return sign;
    if (be <= 0) {             // subnormal: value = m * 2^-9
        mant = (uint32_t)__builtin_rintf(qv * 512.f);
        return sign | (uint8_t)mant;
    }
    mant = (uint32_t)__builtin_rintf((qf * 2.f - 1.f) * 8.f);
    if (mant == 8) {
        mant = 0;
        ++be;
    }
    return sign | (uint8_t)(be << 3) | (uint8_t)mant;
}

__device__ __forceinline__ float e4m3_to_f32(uint8_t b) {
    const float sign = (b & 0x80) ? -1.f : 1.f;
    const int be = (b >> 3) & 0xf;
    const int mant = b & 7;
    if (be == 0) return sign * ldexpf((float)mant, -9);
    return sign * ldexpf(1.f + mant / 8.f, be - 7);
}

// 16 lanes per row.  FMT 0: bf16, out row stride ldo elements (uint16);
// FMT 1: e4m3 bytes, out row stride ldo bytes, scale byte (E8M0, applied by
// the MFMA) in scale_out[row]; the scale applied to mult * row is a power of
// two 2^e with max |mult * x| / 2^e <= 448.
template <int FMT>
__global__ __launch_bounds__(256) void quantize_kernel(const float* A, int64_t rows, int64_t lda,
                                                       int32_t d, float mult, void* out,
                                                       int64_t ldo, int32_t dpad, float* norm2,
                                                       float* err, uint8_t* scale_out,
                                                       uint32_t* stat, bool vec4, float inv,
                                                       float* norm32, uint32_t* flags32) {
    __shared__ float wmax[4][2];
    __shared__ uint32_t wflag[4][3];
    uint32_t nonint = 0, neg = 0;
    float amax32 = 0.f;
    const int sub = threadIdx.x & 15;
    float nmax = 0.f, emax = 0.f;
    for (int64_t r = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 4; r < rows;
         r += ((int64_t)gridDim.x * blockDim.x) >> 4) {
        const float* p = A + r * lda;
        int sexp = 0;
        if (FMT == 1) {
            float amax = 0.f;
            for (int f = sub; f < d; f += 16) amax = fmaxf(amax, __builtin_fabsf(mult * p[f]));
#pragma unroll
            for (int off = 8; off >= 1; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off, 16));
            // smallest power of two 2^e with amax / 2^e <= 448
            int e = -126;
            if (amax > 0.f) {
                int fe;
                frexpf(amax / 448.f, &fe);   // amax/448 = f * 2^fe, f in [0.5, 1)
                e = fe;
                if (ldexpf(1.f, e - 1) >= amax / 448.f) e -= 1;
            }
            if (e < -126) e = -126;
            if (e > 127) e = 127;
            sexp = e;
            if (sub == 0) scale_out[r] = (uint8_t)(e + 127);
        }
        float s2 = 0.f, e2 = 0.f, s32 = 0.f;
        if (FMT == 0 && vec4) {
            // float4 runs 4 sub + 64 j, four bf16 stored together; mult is
            // a power of two, so dividing by it is the exact product inv
            for (int f = 4 * sub; f < dpad; f += 64) {
                f4 v = {0.f, 0.f, 0.f, 0.f};
                if (f < d) v = *(const f4*)(p + f);
                uint16_t b[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if (norm32) {
                        s32 = __builtin_fmaf(v[e], v[e], s32);
                        nonint |= (__builtin_rintf(v[e]) != v[e]) ? 1u : 0u;
                        neg |= v[e] < 0.f ? 1u : 0u;
                        amax32 = fmaxf(amax32, __builtin_fabsf(v[e]));
                    }
                    b[e] = f32_to_bf16_rne(mult * v[e]);
                    const float deq = bf16_to_f32(b[e]) * inv;
                    s2 = __builtin_fmaf(deq, deq, s2);
                    const float t = v[e] - deq;
                    e2 = __builtin_fmaf(t, t, e2);
                }
                uint2 w;
                w.x = (uint32_t)b[0] | ((uint32_t)b[1] << 16);
                w.y = (uint32_t)b[2] | ((uint32_t)b[3] << 16);
                *(uint2*)((uint16_t*)out + r * ldo + f) = w;
            }
        } else
        for (int f = sub; f < dpad; f += 16) {
            const float v = f < d ? p[f] : 0.f;
            if (norm32) {
                s32 = __builtin_fmaf(v, v, s32);
                nonint |= (__builtin_rintf(v) != v) ? 1u : 0u;
                neg |= v < 0.f ? 1u : 0u;
                amax32 = fmaxf(amax32, __builtin_fabsf(v));
            }
            float deq;  // the quantised value of v (without mult)
            if (FMT == 0) {
                const uint16_t b = f32_to_bf16_rne(mult * v);
                ((uint16_t*)out)[r * ldo + f] = b;
                deq = bf16_to_f32(b) / mult;
            } else {
                const float sc = ldexpf(1.f, sexp);
                const uint8_t b = f32_to_e4m3(mult * v / sc);
                ((uint8_t*)out)[r * ldo + f] = b;
                deq = e4m3_to_f32(b) * sc / mult;
            }
            s2 = __builtin_fmaf(deq, deq, s2);
            const float t = v - deq;
            e2 = __builtin_fmaf(t, t, e2);
        }
#pragma unroll
        for (int off = 8; off >= 1; off >>= 1) {
            s2 += __shfl_xor(s2, off, 16);
            e2 += __shfl_xor(e2, off, 16);
            if (norm32) s32 += __shfl_xor(s32, off, 16);
        }
        if (norm32 && sub == 0) norm32[r] = s32;
        // widen the error bound by the relative error of its fp32 sum
        const float eb = __builtin_sqrtf(e2 * (1.f + 4.f * (d + 2) * 5.9604645e-8f)) * (1.f + 1e-6f);
        if (sub == 0) {
            norm2[r] = s2;
            if (err) err[r] = eb;
        }
        nmax = fmaxf(nmax, __builtin_sqrtf(s2));
        emax = fmaxf(emax, eb);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        nmax = fmaxf(nmax, __shfl_xor(nmax, off));
        emax = fmaxf(emax, __shfl_xor(emax, off));
    }
    if ((threadIdx.x & 63) == 0) {
        wmax[threadIdx.x >> 6][0] = nmax;
        wmax[threadIdx.x >> 6][1] = emax;
    }
    __syncthreads();
    if (flags32) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            nonint |= __shfl_xor(nonint, off);
            neg |= __shfl_xor(neg, off);
            amax32 = fmaxf(amax32, __shfl_xor(amax32, off));
        }
        if ((threadIdx.x & 63) == 0) {
            wflag[threadIdx.x >> 6][0] = nonint;
            wflag[threadIdx.x >> 6][1] = __float_as_uint(amax32);
            wflag[threadIdx.x >> 6][2] = neg;
        }
    }
    __syncthreads();
    if (flags32 && threadIdx.x == 0) {
        uint32_t f0 = 0, f1 = 0, f2 = 0;
        for (int w = 0; w < 4; ++w) {
            f0 |= wflag[w][0];
            f1 = f1 > wflag[w][1] ? f1 : wflag[w][1];
            f2 |= wflag[w][2];
        }
        // the same words and skip-if-present rule as the row-norm kernel
        if ((__atomic_load_n(flags32, __ATOMIC_RELAXED) | f0 | 2u) !=
            __atomic_load_n(flags32, __ATOMIC_RELAXED))
            atomicOr(flags32, f0 | 2u);
        if (__atomic_load_n(flags32 + 1, __ATOMIC_RELAXED) < f1) atomicMax(flags32 + 1, f1);
        if (f2 && !(__atomic_load_n(flags32 + 2, __ATOMIC_RELAXED) & f2)) atomicOr(flags32 + 2, f2);
    }
    if (threadIdx.x == 0) {
        float a0 = 0.f, a1 = 0.f;
        for (int w = 0; w < 4; ++w) {
            a0 = fmaxf(a0, wmax[w][0]);
            a1 = fmaxf(a1, wmax[w][1]);
        }
        // maxima only grow: skip the atomic when the word already holds more
        if (__atomic_load_n(stat, __ATOMIC_RELAXED) < __float_as_uint(a0))
            atomicMax(stat, __float_as_uint(a0));
        if (__atomic_load_n(stat + 1, __ATOMIC_RELAXED) < __float_as_uint(a1))
            atomicMax(stat + 1, __float_as_uint(a1));
    }
}

hipError_t launch_quantize(int fmt, const float* A, int64_t rows, int64_t lda, int32_t d,
                           float mult, void* out, int64_t ldo, int32_t dpad, float* norm2,
                           float* err, uint8_t* scale_out, uint32_t* stat, hipStream_t st) {
    return launch_quantize_norms(fmt, A, rows, lda, d, mult, out, ldo, dpad, norm2, err,
                                 scale_out, stat, nullptr, nullptr, st);
}

hipError_t launch_quantize_norms(int fmt, const float* A, int64_t rows, int64_t lda, int32_t d,
                                 float mult, void* out, int64_t ldo, int32_t dpad, float* norm2,
                                 float* err, uint8_t* scale_out, uint32_t* stat, float* norm32,
                                 uint32_t* flags32, hipStream_t st) {
    if (rows <= 0) return hipSuccess;
    int64_t blocks = (rows * 16 + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    // bf16 float4 path: aligned runs and a power-of-two multiplier
    int mexp = 0;
    const bool pow2 = mult != 0.f && std::fabs(std::frexp(mult, &mexp)) == 0.5f;
    const bool vec4 = fmt == 0 && pow2 && (d % 4) == 0 && (lda % 4) == 0 && (dpad % 4) == 0 &&
                      (ldo % 4) == 0 && ((uintptr_t)A & 15) == 0 && ((uintptr_t)out & 7) == 0;
    const float inv = pow2 ? 1.0f / mult : 0.f;
    if (fmt == 0)
        hipLaunchKernelGGL(quantize_kernel<0>, dim3((unsigned)blocks), dim3(256), 0, st, A, rows,
                           lda, d, mult, out, ldo, dpad, norm2, err, scale_out, stat, vec4, inv,
                           norm32, flags32);
    else
        hipLaunchKernelGGL(quantize_kernel<1>, dim3((unsigned)blocks), dim3(256), 0, st, A, rows,
                           lda, d, mult, out, ldo, dpad, norm2, err, scale_out, stat, false, inv,
                           norm32, flags32);
    return hipGetLastError();
}

}  // namespace rbc
