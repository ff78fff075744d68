// Histogram sketch, eq. (2) with unit bins then eq. (3):  S = H . F,  n = row sums of H,  z = S / n.
//
// H [P x T] uint16 counts, F [T x 2m] with columns (cos, sin)(w_l t), l = 1..m (interleaved so
// that S is already in the [P][m][2] sketch layout).  This is a dense contraction, so it runs on
// the matrix cores.  The T bins are taken in chunks of 32.  Within chunk k every count of a row
// is reduced by the chunk's level c_k (its rounded mean count), and
//     S = sum_t (H_t - c_k(t)) F_t  +  sum_k c_k G_k,      G_k = sum_{t in chunk k} F_t,
// which is the same number in exact arithmetic.  The first product sees only deviations from a
// local level, so its FP32 partial sums stay at the scale of the deviations (a row that is
// constant on each chunk contributes exactly zero there); the second is a product of exact
// integers with G evaluated in FP64 from exact integer phases, on the FP64 matrix cores.
//  * FP32:   v_mfma_f32_16x16x4_f32 on the deviations (exact in FP32) and FP32-rounded F.
//  * FP16X2: deviations d split exactly as d = 2^11 q + r, |r| <= 2^10, |q| <= 31 (both exact in
//            FP16), F = F1 + F2 with F1 = fp16(F), F2 = fp16(F - F1); v_mfma_f32_16x16x32_f16,
//            FP32 accumulation.
//  * BF16X3: d = 2^8 q + r, |r| <= 2^7, |q| <= 248 (exact in BF16), F = F1 + F2 + F3 in BF16;
//            v_mfma_f32_16x16x32_bf16.
//  The q products run only for chunks where some deviation in the wave's rows needs them.
//  Level part: v_mfma_f64_16x16x4_f64 over the chunk levels, which each wave keeps in LDS.
// A operands come straight from HBM into registers (each lane loads 8 consecutive counts of one
// row, 16 B, which is exactly its slice of a 16x32 A tile); F and G are small and stay in L2.
// The 16-bit A tile for FP32 uses the same 8 counts over 8 MFMAs with K = 4 (k order is
// immaterial to the sum as long as A and B agree).
#include "common.hpp"

namespace srt3d {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

template <int PREC> struct Prec;
template <> struct Prec<SRT3D_PREC_FP32> { static constexpr int splits = 1, shift = 0, elem = 4; };
template <> struct Prec<SRT3D_PREC_FP16X2> { static constexpr int splits = 2, shift = 11, elem = 2; };
template <> struct Prec<SRT3D_PREC_BF16X3> { static constexpr int splits = 3, shift = 8, elem = 2; };

constexpr int kChunk = 32;                 // bins per chunk (one k-step of the 16-bit products)
constexpr int kWavesPerBlock = 4;
constexpr int kMT = 2;                     // 16-row tiles per wave

__host__ __device__ static inline int n_tiles(int m) { return (2 * m + 15) / 16; }
// chunks per row rounded up to the K of the FP64 product (4)
__host__ __device__ static inline int n_chunks4(int T) { return ((T / kChunk + 3) / 4) * 4; }

__host__ __device__ static inline size_t dft_bytes(int T, int m, int precision) {
    const int splits = precision == SRT3D_PREC_FP32 ? 1 : (precision == SRT3D_PREC_FP16X2 ? 2 : 3);
    const int elem = precision == SRT3D_PREC_FP32 ? 4 : 2;
    const size_t b = (size_t)splits * n_tiles(m) * 16 * (size_t)T * elem;
    return (b + 255) & ~(size_t)255;
}

// workspace: the split F planes, then G [n_chunks4][16 n_tiles] FP64 (padding chunks and
// columns zero)
size_t hist_ws_bytes(int T, int m, int precision) {
    const size_t g = (size_t)n_chunks4(T) * n_tiles(m) * 16 * sizeof(double);
    return dft_bytes(T, m, precision) + ((g + 255) & ~(size_t)255);
}

__device__ __forceinline__ uint16_t bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// (cos, sin)(2 pi k / T) for an exact integer phase k in [0, T), FP64.
__device__ __forceinline__ void phase_cs(int k, int T, double* c, double* s) {
    sincospi(2.0 * (double)k / (double)T, s, c);
}

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
        double s, c;
        phase_cs((int)(((int64_t)l * t) % T), T, &c, &s);
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

// G[k][r] = sum over the 32 bins t of chunk k of column r of F, in FP64 with exact phases;
// zero for padding chunks (k >= T / 32) and padding columns (r >= 2m).
__global__ void build_chunk_dft_kernel(int T, int m, double* __restrict__ G) {
    const int cols = n_tiles(m) * 16;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_chunks4(T) * cols) return;
    const int k = idx / cols, r = idx % cols;
    double acc = 0.0;
    if (r < 2 * m && k < T / kChunk) {
        const int l = r / 2 + 1;
        for (int i = 0; i < kChunk; ++i) {
            const int t = k * kChunk + i;
            double s, c;
            phase_cs((int)(((int64_t)l * t) % T), T, &c, &s);
            acc += (r & 1) ? s : c;
        }
    }
    G[idx] = acc;
}

// Wave tile: kMT x 16 rows, NT x 16 columns.  lane: row/col = lane & 15, k-group = lane >> 4.
// Dynamic LDS: per wave, the chunk levels lv[k][32 rows] (uint16), k < n_chunks4(T).
template <int PREC, int NT>
__global__ __launch_bounds__(256) void hist_mfma_kernel(const uint16_t* __restrict__ H, int P, int T, int m,
                                                        const void* __restrict__ ws, float* __restrict__ z,
                                                        int32_t* __restrict__ nout) {
    constexpr int S = Prec<PREC>::splits;
    constexpr int MT = kMT;
    extern __shared__ uint16_t lds_levels[];
    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;
    const int wave = blockIdx.x * kWavesPerBlock + wib;
    const int64_t r0 = (int64_t)wave * MT * 16;
    if (r0 >= P) return;
    const int li = lane & 15, kg = lane >> 4;
    const int rowsF = NT * 16;
    const int64_t plane = (int64_t)rowsF * T;
    const int nk = T / kChunk, nk4 = n_chunks4(T);
    uint16_t* lv = lds_levels + (size_t)wib * nk4 * (MT * 16);
    // padding chunks have level 0 (their G rows are zero too)
    for (int i = nk * MT * 16 + lane; i < nk4 * MT * 16; i += 64) lv[i] = 0;

    v4f acc[MT][NT];
    uint32_t rsum[MT];
#pragma unroll
    for (int a = 0; a < MT; ++a) {
        rsum[a] = 0;
#pragma unroll
        for (int b = 0; b < NT; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
    }

    // The counts of the next chunk are loaded while this one is contracted (one step of
    // prefetch doubles the loads each wave keeps in flight).
    uint4 qn[MT];
#pragma unroll
    for (int a = 0; a < MT; ++a) {
        const int64_t row = r0 + a * 16 + li;
        qn[a] = row < P ? *reinterpret_cast<const uint4*>(H + row * T + 8 * kg) : make_uint4(0, 0, 0, 0);
    }
    uint4 fbn[NT][S];                                  // 16-bit forms: the next chunk's F fragments
    if constexpr (PREC != SRT3D_PREC_FP32) {
        const uint16_t* F = reinterpret_cast<const uint16_t*>(ws);
#pragma unroll
        for (int b = 0; b < NT; ++b)
#pragma unroll
            for (int s = 0; s < S; ++s)
                fbn[b][s] = *reinterpret_cast<const uint4*>(F + s * plane + (int64_t)(b * 16 + li) * T + 8 * kg);
    }
    float4 fn0[NT], fn1[NT];                           // FP32 form: the next chunk's F fragments
    if constexpr (PREC == SRT3D_PREC_FP32) {
        const float* F = reinterpret_cast<const float*>(ws);
#pragma unroll
        for (int b = 0; b < NT; ++b) {
            const float4* fp = reinterpret_cast<const float4*>(F + (int64_t)(b * 16 + li) * T + 8 * kg);
            fn0[b] = fp[0];
            fn1[b] = fp[1];
        }
    }
    for (int k0 = 0, kc = 0; k0 < T; k0 += kChunk, ++kc) {
        const int kk = k0 + 8 * kg;
        int32_t cnt[MT][8];
        bool anyhi = false;
        uint4 qc[MT];
#pragma unroll
        for (int a = 0; a < MT; ++a) qc[a] = qn[a];
        if (k0 + kChunk < T) {
#pragma unroll
            for (int a = 0; a < MT; ++a) {
                const int64_t row = r0 + a * 16 + li;
                if (row < P) qn[a] = *reinterpret_cast<const uint4*>(H + row * T + kk + kChunk);
            }
        }
#pragma unroll
        for (int a = 0; a < MT; ++a) {
            const uint4 q = qc[a];
            const uint32_t w[4] = {q.x, q.y, q.z, q.w};
            uint32_t s8 = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) s8 += (w[j] & 0xffffu) + (w[j] >> 16);
            rsum[a] += s8;
            // the chunk's level: its rounded mean (the four lanes of a row hold eight bins each)
            s8 += __shfl_xor(s8, 16, 64);
            s8 += __shfl_xor(s8, 32, 64);
            const int32_t c = (int32_t)((s8 + 16u) >> 5);
            if (kg == 0) lv[kc * (MT * 16) + a * 16 + li] = (uint16_t)c;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                cnt[a][2 * j] = (int32_t)(w[j] & 0xffffu) - c;
                cnt[a][2 * j + 1] = (int32_t)(w[j] >> 16) - c;
            }
            if constexpr (PREC != SRT3D_PREC_FP32) {
                constexpr int HALF = 1 << (Prec<PREC>::shift - 1);
#pragma unroll
                for (int j = 0; j < 8; ++j) anyhi |= (uint32_t)(cnt[a][j] + HALF) >= (uint32_t)(2 * HALF);
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
            if (k0 + kChunk < T) {
#pragma unroll
                for (int b = 0; b < NT; ++b) {
                    const float4* fp = reinterpret_cast<const float4*>(F + (int64_t)(b * 16 + li) * T + kk + kChunk);
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
                    // d = 2^SH q + r with q = round(d / 2^SH) (ties up) and |r| <= 2^(SH-1):
                    // both exact in the 16-bit format for |d| <= 63487 (see the file comment)
                    const int32_t d = cnt[a][j];
                    const int32_t q = (d + (1 << (SH - 1))) >> SH;
                    const int32_t r = d - (q << SH);
                    if constexpr (PREC == SRT3D_PREC_FP16X2) {
                        alo[a][j] = (_Float16)(float)r;
                        ahi[a][j] = (_Float16)(float)(q << SH);
                    } else {
                        alo[a][j] = (__bf16)(float)r;
                        ahi[a][j] = (__bf16)(float)(q << SH);
                    }
                }
            }
            uint4 fc[NT][S];
#pragma unroll
            for (int b = 0; b < NT; ++b)
#pragma unroll
                for (int s = 0; s < S; ++s) fc[b][s] = fbn[b][s];
            if (k0 + kChunk < T) {
#pragma unroll
                for (int b = 0; b < NT; ++b)
#pragma unroll
                    for (int s = 0; s < S; ++s)
                        fbn[b][s] = *reinterpret_cast<const uint4*>(F + s * plane + (int64_t)(b * 16 + li) * T + kk + kChunk);
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
    // The wave's own LDS writes (the levels) are complete before it reads them back.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");

    // Level part L = C . G on the FP64 matrix cores: A = levels (chunk 4 g + kg), B = G (chunk
    // 4 g + kg, column li).  The FP64 product leaves result row 4 i + kg in register i (the FP32
    // products leave row 4 kg + i there), so A's row li carries the levels of row
    // 4 (li & 3) + (li >> 2): then register i holds row 4 kg + i, as in the FP32 accumulators.
    const double* G = reinterpret_cast<const double*>(reinterpret_cast<const char*>(ws) +
                                                      dft_bytes(T, m, PREC));
    const int twom = 2 * m;
    const int prow = 4 * (li & 3) + (li >> 2);
#pragma unroll
    for (int b = 0; b < NT; ++b) {
        v4d lacc[MT];
#pragma unroll
        for (int a = 0; a < MT; ++a) lacc[a] = v4d{0.0, 0.0, 0.0, 0.0};
        for (int g = 0; g < nk4; g += 4) {
            const double gb = G[(size_t)(g + kg) * rowsF + b * 16 + li];
#pragma unroll
            for (int a = 0; a < MT; ++a) {
                const double ca = (double)lv[(g + kg) * (MT * 16) + a * 16 + prow];
                lacc[a] = __builtin_amdgcn_mfma_f64_16x16x4f64(ca, gb, lacc[a], 0, 0, 0);
            }
        }
#pragma unroll
        for (int a = 0; a < MT; ++a) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int rl = 4 * kg + i;                       // row of acc[..][i] within the tile
                const uint32_t n = __shfl(rsum[a], rl, 64);
                const int64_t row = r0 + a * 16 + rl;
                const int col = b * 16 + li;
                if (row < P && col < twom)
                    z[row * twom + col] =
                        n > 0 ? (float)(((double)acc[a][b][i] + lacc[a][i]) / (double)n) : 0.f;
            }
        }
    }
#pragma unroll
    for (int a = 0; a < MT; ++a)
        if (kg == 0 && r0 + a * 16 + li < P) nout[r0 + a * 16 + li] = (int32_t)rsum[a];
}

static size_t hist_lds_bytes(int T) { return (size_t)kWavesPerBlock * n_chunks4(T) * kMT * 16 * sizeof(uint16_t); }

template <int PREC, int NT>
static hipError_t launch_hist_nt(const uint16_t* H, int P, int T, int m, const void* ws, float* z, int32_t* n,
                                 hipStream_t s) {
    // two 16-row tiles per wave: 2048 waves at 256^2, which keeps more loads in flight than four
    // tiles and more matrix work per load than one
    const int64_t waves = ((int64_t)P + kMT * 16 - 1) / (kMT * 16);
    const unsigned blocks = (unsigned)((waves + kWavesPerBlock - 1) / kWavesPerBlock);
    hipLaunchKernelGGL((hist_mfma_kernel<PREC, NT>), dim3(blocks), dim3(64 * kWavesPerBlock), hist_lds_bytes(T), s,
                       H, P, T, m, ws, z, n);
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
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    double* G = reinterpret_cast<double*>(static_cast<char*>(ws) + dft_bytes(T, m, precision));
    const int gtotal = n_chunks4(T) * n_tiles(m) * 16;
    hipLaunchKernelGGL(build_chunk_dft_kernel, dim3((gtotal + 255) / 256), dim3(256), 0, s, T, m, G);
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
