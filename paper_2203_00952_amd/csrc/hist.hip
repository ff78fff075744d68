// Histogram sketch, eq. (2) with unit bins then eq. (3):  S = H . F,  n = row sums of H,  z = S / n.
//
// H [P x T] uint16 counts, F [T x 2m] with columns (cos, sin)(w_l t), l = 1..m (interleaved so
// that S is already in the [P][m][2] sketch layout).  This is a dense contraction, so it runs on
// the matrix cores:
//  * FP32:   v_mfma_f32_16x16x4_f32 on FP32 counts (exact) and FP32-rounded F.
//  * FP16X2: counts split exactly into hi + lo (s = 11, both exact in FP16), F = F1 + F2 with
//            F1 = fp16(F), F2 = fp16(F - F1); v_mfma_f32_16x16x32_f16, FP32 accumulation.
//  * BF16X3: counts split into hi + lo (s = 8, exact in BF16), F = F1 + F2 + F3 in BF16;
//            v_mfma_f32_16x16x32_bf16.
//  The hi products run only for k-chunks where some reduced count in the wave's rows reaches 2^s
//  in magnitude.
// Before the product every count of a row is reduced by a constant c of that row (the rounded
// mean of its first 32 bins, at most 2^15): sum_t exp(i w_l t) over all T bins is zero for
// 0 < l < T, so S is unchanged in exact arithmetic, while the FP32 partial sums of a row with a
// high common level (a constant row sketches to exactly zero) stay at the scale of the
// deviations.  The reduced counts d lie in [-2^15, 2^16) and split exactly: d itself when
// |d| < 2^s, else a multiple of 2^s plus a remainder in [0, 2^s).
// A operands come straight from HBM into registers (each lane loads 8 consecutive counts of one
// row, 16 B, which is exactly its slice of a 16x32 A tile); F is small and stays in L2.  The
// 16-bit A tile for FP32 uses the same 8 counts over 8 MFMAs with K = 4 (k order is immaterial
// to the sum as long as A and B agree).
#include "common.hpp"

namespace srt3d {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

template <int PREC> struct Prec;
template <> struct Prec<SRT3D_PREC_FP32> { static constexpr int splits = 1, shift = 0, elem = 4; };
template <> struct Prec<SRT3D_PREC_FP16X2> { static constexpr int splits = 2, shift = 11, elem = 2; };
template <> struct Prec<SRT3D_PREC_BF16X3> { static constexpr int splits = 3, shift = 8, elem = 2; };

__host__ __device__ static inline int n_tiles(int m) { return (2 * m + 15) / 16; }

size_t hist_ws_bytes(int T, int m, int precision) {
    int splits = precision == SRT3D_PREC_FP32 ? 1 : (precision == SRT3D_PREC_FP16X2 ? 2 : 3);
    int elem = precision == SRT3D_PREC_FP32 ? 4 : 2;
    size_t b = (size_t)splits * n_tiles(m) * 16 * (size_t)T * elem;
    return (b + 255) & ~(size_t)255;
}

__device__ __forceinline__ uint16_t bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// FT[s][r][t] = split s of F[t][r], rows r >= 2m are zero.  F is evaluated in FP64 with the
// exact integer phase (l t) mod T.
template <int PREC>
__global__ void build_dft_kernel(int T, int m, void* __restrict__ ws) {
    const int rows = n_tiles(m) * 16;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)rows * T) return;
    const int r = (int)(idx / T), t = (int)(idx % T);
    double f = 0.0;
    if (r < 2 * m) {
        const int l = r / 2 + 1;
        const int k = (int)(((int64_t)l * t) % T);
        double s, c;
        sincospi(2.0 * (double)k / (double)T, &s, &c);
        f = (r & 1) ? s : c;
    }
    const int64_t plane = (int64_t)rows * T;
    if constexpr (PREC == SRT3D_PREC_FP32) {
        reinterpret_cast<float*>(ws)[idx] = (float)f;
    } else if constexpr (PREC == SRT3D_PREC_FP16X2) {
        _Float16* o = reinterpret_cast<_Float16*>(ws);
        const _Float16 f1 = (_Float16)f;
        const _Float16 f2 = (_Float16)(f - (double)f1);
        o[idx] = f1;
        o[plane + idx] = f2;
    } else {
        uint16_t* o = reinterpret_cast<uint16_t*>(ws);
        const uint16_t b1 = bf16_rne((float)f);
        const double r1 = f - (double)bf16_to_f(b1);
        const uint16_t b2 = bf16_rne((float)r1);
        const double r2 = r1 - (double)bf16_to_f(b2);
        const uint16_t b3 = bf16_rne((float)r2);
        o[idx] = b1;
        o[plane + idx] = b2;
        o[2 * plane + idx] = b3;
    }
}

// Wave tile: MT x 16 rows, NT x 16 columns.  lane: row/col = lane & 15, k-group = lane >> 4.
template <int PREC, int NT, int MT>
__global__ __launch_bounds__(256) void hist_mfma_kernel(const uint16_t* __restrict__ H, int P, int T, int m,
                                                        const void* __restrict__ ws, float* __restrict__ z,
                                                        int32_t* __restrict__ nout) {
    constexpr int S = Prec<PREC>::splits;
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t r0 = (int64_t)wave * MT * 16;
    if (r0 >= P) return;
    const int li = lane & 15, kg = lane >> 4;
    const int rowsF = NT * 16;
    const int64_t plane = (int64_t)rowsF * T;

    v4f acc[MT][NT];
    uint32_t rsum[MT];
#pragma unroll
    for (int a = 0; a < MT; ++a) {
        rsum[a] = 0;
#pragma unroll
        for (int b = 0; b < NT; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
    }

    // The counts of the next 32-bin step are loaded while this one is contracted (one step of
    // prefetch doubles the loads each wave keeps in flight).
    uint4 qn[MT];
#pragma unroll
    for (int a = 0; a < MT; ++a) {
        const int64_t row = r0 + a * 16 + li;
        qn[a] = row < P ? *reinterpret_cast<const uint4*>(H + row * T + 8 * kg) : make_uint4(0, 0, 0, 0);
    }
    uint4 fbn[NT][S];                                  // 16-bit forms: the next step's F fragments
    if constexpr (PREC != SRT3D_PREC_FP32) {
        const uint16_t* F = reinterpret_cast<const uint16_t*>(ws);
#pragma unroll
        for (int b = 0; b < NT; ++b)
#pragma unroll
            for (int s = 0; s < S; ++s)
                fbn[b][s] = *reinterpret_cast<const uint4*>(F + s * plane + (int64_t)(b * 16 + li) * T + 8 * kg);
    }
    float4 fn0[NT], fn1[NT];                           // FP32 form: the next step's F fragments
    if constexpr (PREC == SRT3D_PREC_FP32) {
        const float* F = reinterpret_cast<const float*>(ws);
#pragma unroll
        for (int b = 0; b < NT; ++b) {
            const float4* fp = reinterpret_cast<const float4*>(F + (int64_t)(b * 16 + li) * T + 8 * kg);
            fn0[b] = fp[0];
            fn1[b] = fp[1];
        }
    }
    // Per-row level c: rounded mean of the row's first 32 bins (the four lanes of a row hold
    // eight bins each), capped at 2^15 so that every reduced count splits exactly.
    int32_t lvl[MT];
#pragma unroll
    for (int a = 0; a < MT; ++a) {
        const uint4 q = qn[a];
        const uint32_t w[4] = {q.x, q.y, q.z, q.w};
        uint32_t s8 = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) s8 += (w[j] & 0xffffu) + (w[j] >> 16);
        s8 += __shfl_xor(s8, 16, 64);
        s8 += __shfl_xor(s8, 32, 64);
        const uint32_t c = (s8 + 16u) >> 5;
        lvl[a] = (int32_t)(c < 32768u ? c : 32768u);
    }
    for (int k0 = 0; k0 < T; k0 += 32) {
        const int kk = k0 + 8 * kg;
        int32_t cnt[MT][8];
        bool anyhi = false;
        uint4 qc[MT];
#pragma unroll
        for (int a = 0; a < MT; ++a) qc[a] = qn[a];
        if (k0 + 32 < T) {
#pragma unroll
            for (int a = 0; a < MT; ++a) {
                const int64_t row = r0 + a * 16 + li;
                if (row < P) qn[a] = *reinterpret_cast<const uint4*>(H + row * T + kk + 32);
            }
        }
#pragma unroll
        for (int a = 0; a < MT; ++a) {
            const uint4 q = qc[a];
            const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                rsum[a] += (w[j] & 0xffffu) + (w[j] >> 16);
                cnt[a][2 * j] = (int32_t)(w[j] & 0xffffu) - lvl[a];
                cnt[a][2 * j + 1] = (int32_t)(w[j] >> 16) - lvl[a];
            }
            if constexpr (PREC != SRT3D_PREC_FP32) {
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int32_t d = cnt[a][j];
                    anyhi |= (d < 0 ? -d : d) >= (1 << Prec<PREC>::shift);
                }
            }
        }
        if constexpr (PREC == SRT3D_PREC_FP32) {
            const float* F = reinterpret_cast<const float*>(ws);
            float4 fc0[NT], fc1[NT];
#pragma unroll
            for (int b = 0; b < NT; ++b) {
                fc0[b] = fn0[b];
                fc1[b] = fn1[b];
            }
            if (k0 + 32 < T) {
#pragma unroll
                for (int b = 0; b < NT; ++b) {
                    const float4* fp = reinterpret_cast<const float4*>(F + (int64_t)(b * 16 + li) * T + kk + 32);
                    fn0[b] = fp[0];
                    fn1[b] = fp[1];
                }
            }
#pragma unroll
            for (int b = 0; b < NT; ++b) {
                const float4 f0 = fc0[b], f1 = fc1[b];
                const float fv[8] = {f0.x, f0.y, f0.z, f0.w, f1.x, f1.y, f1.z, f1.w};
#pragma unroll
                for (int a = 0; a < MT; ++a)
#pragma unroll
                    for (int j = 0; j < 8; ++j)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32((float)cnt[a][j], fv[j], acc[a][b], 0, 0, 0);
            }
        } else {
            constexpr int SH = Prec<PREC>::shift;
            const uint16_t* F = reinterpret_cast<const uint16_t*>(ws);
            const bool hi_wave = __any(anyhi);
            typedef typename std::conditional<PREC == SRT3D_PREC_FP16X2, v8h, v8bf>::type v8;
            v8 alo[MT], ahi[MT];
#pragma unroll
            for (int a = 0; a < MT; ++a) {
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    // d = hi + lo, both exact in the 16-bit format: hi = 0 when |d| < 2^SH,
                    // else hi = d rounded down to a multiple of 2^SH (in [-2^15, 2^16)) and
                    // lo in [0, 2^SH)
                    const int32_t d = cnt[a][j];
                    const int32_t hi = (d < 0 ? -d : d) < (1 << SH) ? 0 : (d & ~((1 << SH) - 1));
                    const int32_t lo = d - hi;
                    if constexpr (PREC == SRT3D_PREC_FP16X2) {
                        alo[a][j] = (_Float16)(float)lo;
                        ahi[a][j] = (_Float16)(float)hi;
                    } else {
                        alo[a][j] = (__bf16)(float)lo;
                        ahi[a][j] = (__bf16)(float)hi;
                    }
                }
            }
            uint4 fc[NT][S];
#pragma unroll
            for (int b = 0; b < NT; ++b)
#pragma unroll
                for (int s = 0; s < S; ++s) fc[b][s] = fbn[b][s];
            if (k0 + 32 < T) {
#pragma unroll
                for (int b = 0; b < NT; ++b)
#pragma unroll
                    for (int s = 0; s < S; ++s)
                        fbn[b][s] = *reinterpret_cast<const uint4*>(F + s * plane + (int64_t)(b * 16 + li) * T + kk + 32);
            }
#pragma unroll
            for (int b = 0; b < NT; ++b) {
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    const v8 fb = __builtin_bit_cast(v8, fc[b][s]);
#pragma unroll
                    for (int a = 0; a < MT; ++a) {
                        if constexpr (PREC == SRT3D_PREC_FP16X2)
                            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(alo[a], fb, acc[a][b], 0, 0, 0);
                        else
                            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[a], fb, acc[a][b], 0, 0, 0);
                    }
                    if (hi_wave) {
#pragma unroll
                        for (int a = 0; a < MT; ++a) {
                            if constexpr (PREC == SRT3D_PREC_FP16X2)
                                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ahi[a], fb, acc[a][b], 0, 0, 0);
                            else
                                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[a], fb, acc[a][b], 0, 0, 0);
                        }
                    }
                }
            }
        }
    }

    // Row sums: the 4 lanes with the same (lane & 15) hold partial sums of one row.
#pragma unroll
    for (int a = 0; a < MT; ++a) {
        uint32_t v = rsum[a];
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        rsum[a] = v;
    }
    const int twom = 2 * m;
#pragma unroll
    for (int a = 0; a < MT; ++a) {
        if (kg == 0 && r0 + a * 16 + li < P) nout[r0 + a * 16 + li] = (int32_t)rsum[a];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int rl = 4 * kg + i;                       // row of acc[..][i] within the tile
            const uint32_t n = __shfl(rsum[a], rl, 64);
            const int64_t row = r0 + a * 16 + rl;
#pragma unroll
            for (int b = 0; b < NT; ++b) {
                const int col = b * 16 + li;
                if (row < P && col < twom)
                    z[row * twom + col] = n > 0 ? (float)((double)acc[a][b][i] / (double)n) : 0.f;
            }
        }
    }
}

template <int PREC, int NT>
static hipError_t launch_hist_nt(const uint16_t* H, int P, int T, int m, const void* ws, float* z, int32_t* n,
                                 hipStream_t s) {
    // two 16-row tiles per wave: 2048 waves at 256^2, which keeps more loads in flight than four
    // tiles (FP16x2 77 -> 59 us, BF16x3 90 -> 80 us) and more MFMA work per load than one (FP32
    // 65 -> 81 us)
    constexpr int MT = 2;
    const int64_t waves = ((int64_t)P + MT * 16 - 1) / (MT * 16);
    const unsigned blocks = (unsigned)((waves + 3) / 4);
    hipLaunchKernelGGL((hist_mfma_kernel<PREC, NT, MT>), dim3(blocks), dim3(256), 0, s, H, P, T, m, ws, z, n);
    return hipGetLastError();
}

template <int PREC>
static hipError_t launch_hist_p(const uint16_t* H, int P, int T, int m, const void* ws, float* z, int32_t* n,
                                hipStream_t s) {
    switch (n_tiles(m)) {
        case 1: return launch_hist_nt<PREC, 1>(H, P, T, m, ws, z, n, s);
        case 2: return launch_hist_nt<PREC, 2>(H, P, T, m, ws, z, n, s);
        case 3: return launch_hist_nt<PREC, 3>(H, P, T, m, ws, z, n, s);
        default: return launch_hist_nt<PREC, 4>(H, P, T, m, ws, z, n, s);
    }
}

hipError_t launch_hist_prepare(int T, int m, int precision, void* ws, hipStream_t s) {
    const int64_t total = (int64_t)n_tiles(m) * 16 * T;
    const dim3 grid((unsigned)((total + 255) / 256));
    switch (precision) {
        case SRT3D_PREC_FP32: hipLaunchKernelGGL(build_dft_kernel<SRT3D_PREC_FP32>, grid, dim3(256), 0, s, T, m, ws); break;
        case SRT3D_PREC_FP16X2: hipLaunchKernelGGL(build_dft_kernel<SRT3D_PREC_FP16X2>, grid, dim3(256), 0, s, T, m, ws); break;
        default: hipLaunchKernelGGL(build_dft_kernel<SRT3D_PREC_BF16X3>, grid, dim3(256), 0, s, T, m, ws); break;
    }
    return hipGetLastError();
}

hipError_t launch_sketch_hist(const uint16_t* hist, int P, int T, int m, int precision, const void* ws, float* z,
                              int32_t* n, hipStream_t s) {
    switch (precision) {
        case SRT3D_PREC_FP32: return launch_hist_p<SRT3D_PREC_FP32>(hist, P, T, m, ws, z, n, s);
        case SRT3D_PREC_FP16X2: return launch_hist_p<SRT3D_PREC_FP16X2>(hist, P, T, m, ws, z, n, s);
        default: return launch_hist_p<SRT3D_PREC_BF16X3>(hist, P, T, m, ws, z, n, s);
    }
}

}  // namespace srt3d
