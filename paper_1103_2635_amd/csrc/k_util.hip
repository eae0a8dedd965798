// k_util.hip -- small kernels: fills, row repacking, row norms.
#include "rbc_device.h"

namespace rbc {

__global__ void fill_i32_kernel(int32_t* p, int64_t count, int32_t value) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

hipError_t launch_fill_i32(int32_t* p, int64_t count, int32_t value, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, count, value);
    return hipGetLastError();
}

__global__ void iota_i32_kernel(int32_t* p, int32_t count) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = i;
}

hipError_t launch_iota_i32(int32_t* p, int32_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(iota_i32_kernel, dim3((count + 255) / 256), dim3(256), 0, st, p, count);
    return hipGetLastError();
}

__global__ void set_count_kernel(int32_t* p, int32_t value) { *p = value; }

hipError_t launch_set_count(int32_t* p, int32_t value, hipStream_t st) {
    hipLaunchKernelGGL(set_count_kernel, dim3(1), dim3(1), 0, st, p, value);
    return hipGetLastError();
}

// out[r][0 .. ldo) = A[r][0 .. d) followed by zeros.
__global__ void repack_kernel(const float* A, int64_t rows, int64_t lda, int32_t d, float* out,
                              int64_t ldo) {
    const int64_t total = rows * ldo;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / ldo;
        const int64_t c = e - r * ldo;
        out[e] = c < d ? A[r * lda + c] : 0.f;
    }
}

hipError_t launch_repack(const float* A, int64_t rows, int64_t lda, int32_t d, float* out,
                         int64_t ldo, hipStream_t st) {
    if (rows <= 0) return hipSuccess;
    int64_t blocks = (rows * ldo + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(repack_kernel, dim3((unsigned)blocks), dim3(256), 0, st, A, rows, lda, d,
                       out, ldo);
    return hipGetLastError();
}

// Squared norm of every row (16 lanes per row, fp32), and the largest row
// norm as float bits through an integer atomic max (valid for non-negative
// floats).  A bounded grid strides over the rows so that each workgroup
// issues one atomic; 4,096 workgroups keep enough rows in flight for the
// loop to stream at HBM rates.  rowmap (optional) gives the source row of
// output row i.
constexpr int kNormBlocks = 4096;

// flags (optional, 3 words): [0] |= 2 (flags computed) and |= 1 if a value
// is not an integer, [1] = max |value| as float bits, [2] |= 1 if a value is
// negative.
__global__ __launch_bounds__(256) void row_norms_kernel(const float* A, int64_t rows, int64_t lda,
                                                        int32_t d, const int32_t* rowmap,
                                                        float* out, uint32_t* maxbits,
                                                        uint32_t* flags, const int32_t* gate,
                                                        bool vec4) {
    if (gate && *gate == 0) return;  // uniform per launch
    __shared__ float wmax[4];
    __shared__ uint32_t wflag[4][3];
    const int sub = threadIdx.x & 15;
    float nmax = 0.f;
    uint32_t nonint = 0, neg = 0;
    float amax = 0.f;
    for (int64_t r = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 4; r < rows;
         r += ((int64_t)gridDim.x * blockDim.x) >> 4) {
        const int64_t src = rowmap ? rowmap[r] : r;
        const float* p = A + src * lda;
        float s = 0.f;
        if (vec4) {
            // float4 runs 4 sub + 64 j (d, lda multiples of 4, rows 16-byte aligned)
            for (int f = 4 * sub; f < d; f += 64) {
                const f4 v = *(const f4*)(p + f);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    s = __builtin_fmaf(v[e], v[e], s);
                    if (flags) {
                        nonint |= (__builtin_rintf(v[e]) != v[e]) ? 1u : 0u;
                        neg |= v[e] < 0.f ? 1u : 0u;
                        amax = fmaxf(amax, __builtin_fabsf(v[e]));
                    }
                }
            }
        } else {
            for (int f = sub; f < d; f += 16) {
                const float v = p[f];
                s = __builtin_fmaf(v, v, s);
                if (flags) {
                    nonint |= (__builtin_rintf(v) != v) ? 1u : 0u;
                    neg |= v < 0.f ? 1u : 0u;
                    amax = fmaxf(amax, __builtin_fabsf(v));
                }
            }
        }
#pragma unroll
        for (int off = 8; off >= 1; off >>= 1) s += __shfl_xor(s, off, 16);
        if (sub == 0) out[r] = s;
        nmax = fmaxf(nmax, __builtin_sqrtf(s));
    }
    if (flags) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            nonint |= __shfl_xor(nonint, off);
            neg |= __shfl_xor(neg, off);
            amax = fmaxf(amax, __shfl_xor(amax, off));
        }
        if ((threadIdx.x & 63) == 0) {
            wflag[threadIdx.x >> 6][0] = nonint;
            wflag[threadIdx.x >> 6][1] = __float_as_uint(amax);
            wflag[threadIdx.x >> 6][2] = neg;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t f0 = 0, f1 = 0, f2 = 0;
            for (int w = 0; w < 4; ++w) {
                f0 |= wflag[w][0];
                f1 = f1 > wflag[w][1] ? f1 : wflag[w][1];
                f2 |= wflag[w][2];
            }
            // the words only grow, so a workgroup whose bits or maximum are
            // already there skips its atomic (thousands of workgroups would
            // otherwise serialise on the same three words)
            if ((__atomic_load_n(flags, __ATOMIC_RELAXED) | f0 | 2u) !=
                __atomic_load_n(flags, __ATOMIC_RELAXED))
                atomicOr(flags, f0 | 2u);
            if (__atomic_load_n(flags + 1, __ATOMIC_RELAXED) < f1) atomicMax(flags + 1, f1);
            if (f2 && !(__atomic_load_n(flags + 2, __ATOMIC_RELAXED) & f2)) atomicOr(flags + 2, f2);
        }
    }
    if (maxbits) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) nmax = fmaxf(nmax, __shfl_xor(nmax, off));
        if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = nmax;
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint32_t v = __float_as_uint(fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3])));
            if (__atomic_load_n(maxbits, __ATOMIC_RELAXED) < v) atomicMax(maxbits, v);
        }
    }
}

hipError_t launch_row_norms(const float* A, int64_t rows, int64_t lda, int32_t d,
                            const int32_t* rowmap, float* out, uint32_t* maxbits,
                            hipStream_t st, uint32_t* flags, const int32_t* gate) {
    if (rows <= 0) return hipSuccess;
    int64_t blocks = (rows * 16 + 255) / 256;
    if (blocks > kNormBlocks) blocks = kNormBlocks;
    const bool vec4 = (d % 4) == 0 && (lda % 4) == 0 && ((uintptr_t)A & 15) == 0;
    hipLaunchKernelGGL(row_norms_kernel, dim3((unsigned)blocks), dim3(256), 0, st, A, rows, lda,
                       d, rowmap, out, maxbits, flags, gate, vec4);
    return hipGetLastError();
}

// Compaction of the queries listed in list[0 .. *count) (at most m): row i
// of Qc (ldc floats, zero beyond d) is query list[i], qn[i] its squared norm
// (fp32, a wavefront sum), qmap[i] = list[i]; *count_out = *count.  One
// wavefront per row.
__device__ __forceinline__ void gather_one(const float* Q, int64_t ldq, int32_t d,
                                           const int32_t* list, float* Qc, int64_t ldc, float* qn,
                                           int32_t* qmap, int64_t i, int lane) {
    const int32_t q = list[i];
    const float* src = Q + (int64_t)q * ldq;
    float* dst = Qc + i * ldc;
    float s = 0.f;
    for (int f = lane; f < ldc; f += 64) {
        const float v = f < d ? src[f] : 0.f;
        dst[f] = v;
        s = __builtin_fmaf(v, v, s);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) {
        qn[i] = s;
        qmap[i] = q;
    }
}

__global__ __launch_bounds__(256) void cascade_gather_kernel(const float* Q, int64_t ldq,
                                                             int32_t d, const int32_t* list,
                                                             const int32_t* count, float* Qc,
                                                             int64_t ldc, float* qn,
                                                             int32_t* qmap, int32_t* count_out) {
    const int cnt = *count;
    if (blockIdx.x == 0 && threadIdx.x == 0) *count_out = cnt;
    const int lane = threadIdx.x & 63;
    for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < cnt;
         i += (int64_t)gridDim.x * 4)
        gather_one(Q, ldq, d, list, Qc, ldc, qn, qmap, i, lane);
}

hipError_t launch_cascade_gather(const float* Q, int64_t ldq, int32_t d, int64_t m,
                                 const int32_t* list, const int32_t* count, float* Qc,
                                 int64_t ldc, float* qn, int32_t* qmap, int32_t* count_out,
                                 hipStream_t st) {
    if (m <= 0) return hipSuccess;
    const int64_t waves = m > 8192 ? 8192 : m;  // grid-stride over the device-side count
    hipLaunchKernelGGL(cascade_gather_kernel, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, Q,
                       ldq, d, list, count, Qc, ldc, qn, qmap, count_out);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void item_rep_kernel(const int32_t* ioff, int32_t nr,
                                                       int32_t* irep) {
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= nr) return;
    const int e = ioff[r + 1];
    for (int i = ioff[r] + (threadIdx.x & 63); i < e; i += 64) irep[i] = r;
}

// a[i] = min(a[i], b[i]) (two upper bounds on the same distance).
__global__ __launch_bounds__(256) void min_f32_kernel(float* a, const float* b, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) a[i] = fminf(a[i], b[i]);
}

hipError_t launch_min_f32(float* a, const float* b, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(min_f32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, b,
                       n);
    return hipGetLastError();
}

hipError_t launch_item_reps(const int32_t* ioff, int32_t nr, int32_t* irep, hipStream_t st) {
    if (nr <= 0) return hipSuccess;
    hipLaunchKernelGGL(item_rep_kernel, dim3((nr + 3) / 4), dim3(256), 0, st, ioff, nr, irep);
    return hipGetLastError();
}

}  // namespace rbc
