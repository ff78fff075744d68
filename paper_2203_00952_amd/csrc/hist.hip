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
//  The split and the q products run only for chunks where some deviation in the wave's rows
//  needs them; elsewhere (most chunks) the deviations are formed two at a time with packed
//  16-bit integer adds and turned into FP16 or BF16 exactly by a few bit operations.
//  Level part: v_mfma_f64_16x16x4_f64 over the chunk levels, which each wave keeps in LDS, one
//  product per group of 4 chunks inside the chunk loop.
// A operands come straight from HBM into registers (each lane loads 8 consecutive counts of one
// row, 16 B, which is exactly its slice of a 16x32 A tile), two chunks ahead of their use.  Each
// 32-bin chunk of F is staged in LDS once per workgroup and read there by its four waves (F is
// read from L2 once per workgroup rather than once per wave); G stays in L2.
// The 16-bit A tile for FP32 uses the same 8 counts over 8 MFMAs with K = 4 (k order is
// immaterial to the sum as long as A and B agree).
#include "common.hpp"

namespace srt3d {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 h16x2 __attribute__((ext_vector_type(2)));

template <int PREC> struct Prec;
template <> struct Prec<SRT3D_PREC_FP32> { static constexpr int splits = 1, shift = 0, elem = 4; };
template <> struct Prec<SRT3D_PREC_FP16X2> { static constexpr int splits = 2, shift = 11, elem = 2; };
template <> struct Prec<SRT3D_PREC_BF16X3> { static constexpr int splits = 3, shift = 8, elem = 2; };

constexpr int kChunk = 32;                 // bins per chunk (one k-step of the 16-bit products)
constexpr int kWavesPerBlock = 4;
constexpr int kThreads = 64 * kWavesPerBlock;
constexpr int kMT = 1;                     // 16-row tiles per wave
constexpr int kDepth = 2;                  // chunks of counts in flight ahead of the one contracted (1, 2 or 4)

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

// A chunk of F (32 bins of every column, every split) is staged in LDS once per workgroup and
// read there by its four waves: row (s, b, c) of the chunk holds the 32 bins of column 16 b + c of
// split s, padded by 16 bytes so that the 16-byte fragment reads of 16 consecutive columns fall on
// distinct banks.  Two buffers: the next chunk is fetched from L2 into registers while this one is
// contracted and stored after it, one barrier per chunk.
template <int PREC> __host__ __device__ constexpr int f_pitch() { return kChunk * Prec<PREC>::elem + 16; }
template <int PREC, int NT> __host__ __device__ constexpr int f_chunk_bytes() {
    return Prec<PREC>::splits * NT * 16 * f_pitch<PREC>();
}

// Wave tile: kMT x 16 rows, NT x 16 columns.  lane: row/col = lane & 15, k-group = lane >> 4.
// Dynamic LDS: two staged chunks of F, then per wave the chunk levels lv[k][32 rows] (uint16),
// k < n_chunks4(T).
template <int PREC, int NT>
__global__ __launch_bounds__(kThreads) void hist_mfma_kernel(const uint16_t* __restrict__ H, int P, int T, int m,
                                                        const void* __restrict__ ws, float* __restrict__ z,
                                                        int32_t* __restrict__ nout) {
    constexpr int S = Prec<PREC>::splits;
    constexpr int E = Prec<PREC>::elem;
    constexpr int MT = kMT;
    constexpr int FP = f_pitch<PREC>(), FCB = f_chunk_bytes<PREC, NT>();
    constexpr int ROW_U4 = kChunk * E / 16;                 // 16-byte pieces of a column's chunk
    constexpr int FU4 = S * NT * 16 * ROW_U4;               // of the whole chunk
    constexpr int FPT = (FU4 + kThreads - 1) / kThreads;    // per thread
    extern __shared__ __align__(16) uint8_t lds_dyn[];
    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;
    const int wave = blockIdx.x * kWavesPerBlock + wib;
    // a wave past the last row still takes part in staging F and in the barriers; its rows are
    // zero counts and nothing of it is stored
    const int64_t r0 = (int64_t)wave * MT * 16;
    const int li = lane & 15, kg = lane >> 4;
    const int rowsF = NT * 16;
    const int64_t plane = (int64_t)rowsF * T;
    const int nk = T / kChunk, nk4 = n_chunks4(T);
    uint8_t* fbuf = lds_dyn;
    uint16_t* lv = reinterpret_cast<uint16_t*>(lds_dyn + 2 * FCB) + (size_t)wib * nk4 * (MT * 16);
    // padding chunks have level 0 (their G rows are zero too)
    for (int i = nk * MT * 16 + lane; i < nk4 * MT * 16; i += 64) lv[i] = 0;

    // Staging of F: thread x moves the 16-byte pieces x, x + kThreads, ... of a chunk (clamped
    // to the chunk's last piece, which some threads then move more than once).  Named registers,
    // not an array: an array carried across the loop stays in private memory.
    static_assert(FPT <= 3, "at most three 16-byte pieces of a staged chunk per thread");
    const uint8_t* Fb = reinterpret_cast<const uint8_t*>(ws);
    auto f_src = [&](int u) {
        const int idx = min((int)threadIdx.x + u * kThreads, FU4 - 1);
        const int part = idx % ROW_U4, rowi = idx / ROW_U4;            // rowi = (s NT + b) 16 + c
        return Fb + ((int64_t)(rowi / rowsF) * plane + (int64_t)(rowi % rowsF) * T) * E + part * 16;
    };
    auto f_dst = [&](int u) {
        const int idx = min((int)threadIdx.x + u * kThreads, FU4 - 1);
        return (idx / ROW_U4) * FP + (idx % ROW_U4) * 16;
    };
    const uint8_t* fs0 = f_src(0);
    const uint8_t* fs1 = f_src(FPT > 1 ? 1 : 0);
    const uint8_t* fs2 = f_src(FPT > 2 ? 2 : 0);
    const int fd0 = f_dst(0), fd1 = f_dst(FPT > 1 ? 1 : 0), fd2 = f_dst(FPT > 2 ? 2 : 0);
    uint4 fp0, fp1, fp2;
#define SRT3D_F_FETCH(kc_)                                                                  \
    {                                                                                       \
        const int64_t o_ = (int64_t)(kc_) * (kChunk * E);                                   \
        fp0 = *reinterpret_cast<const uint4*>(fs0 + o_);                                    \
        if constexpr (FPT > 1) fp1 = *reinterpret_cast<const uint4*>(fs1 + o_);             \
        if constexpr (FPT > 2) fp2 = *reinterpret_cast<const uint4*>(fs2 + o_);             \
    }
#define SRT3D_F_STORE(buf_)                                                                 \
    {                                                                                       \
        uint8_t* d_ = fbuf + (buf_) * FCB;                                                  \
        *reinterpret_cast<uint4*>(d_ + fd0) = fp0;                                          \
        if constexpr (FPT > 1) *reinterpret_cast<uint4*>(d_ + fd1) = fp1;                  \
        if constexpr (FPT > 2) *reinterpret_cast<uint4*>(d_ + fd2) = fp2;                  \
    }

    v4f acc[MT][NT];
    uint32_t rsum[MT];
#pragma unroll
    for (int a = 0; a < MT; ++a) {
        rsum[a] = 0;
#pragma unroll
        for (int b = 0; b < NT; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
    }

    // The counts of the next kDepth chunks are in flight while one is contracted: a ring of
    // registers, slot d holding chunk kb + d of the group of kDepth chunks at kb.
    // Every load of the loop is unconditional (rows past the last one read the last row, chunks
    // past the last one read the last chunk, and both are discarded), so that the wait before a
    // use covers only the loads that use needs and the prefetches stay in flight.
    // (The results of rows past the last one are never stored, so they may hold anything.)
    const uint16_t* hrow[MT];
#pragma unroll
    for (int a = 0; a < MT; ++a) {
        const int64_t row = r0 + a * 16 + li;
        hrow[a] = H + (row < P ? row : (int64_t)P - 1) * T + 8 * kg;
    }
    static_assert(4 % kDepth == 0, "the ring's slots follow the chunk's place in its group of 4");
    uint4 qr[kDepth][MT];
#pragma unroll
    for (int d = 0; d < kDepth; ++d)
#pragma unroll
        for (int a = 0; a < MT; ++a)
            qr[d][a] = *reinterpret_cast<const uint4*>(hrow[a] + min(d, nk - 1) * kChunk);
    // Level part L = C . G on the FP64 matrix cores, one product per group of 4 chunks (its K),
    // run as the group's last chunk is done: A = levels (chunk g + kg), B = G (chunk g + kg,
    // column li).  The FP64 product leaves result row 4 i + kg in register i (the FP32 products
    // leave row 4 kg + i there), so A's row li carries the levels of row 4 (li & 3) + (li >> 2):
    // then register i holds row 4 kg + i, as in the FP32 accumulators.  Each lane loads its G
    // value of a group as the group starts.
    const double* G = reinterpret_cast<const double*>(reinterpret_cast<const char*>(ws) +
                                                      dft_bytes(T, m, PREC));
    const int prow = 4 * (li & 3) + (li >> 2);
    v4d lacc[MT][NT];
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b) lacc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
    double gcur[NT];

    SRT3D_F_FETCH(0)
    SRT3D_F_STORE(0)
    lds_barrier();
    for (int kb = 0; kb < nk; kb += 4)
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const int kc = kb + d;
        if (kc >= nk) break;
        if (d == 0) {
#pragma unroll
            for (int b = 0; b < NT; ++b) gcur[b] = G[(size_t)(kb + kg) * rowsF + b * 16 + li];
        }
        SRT3D_F_FETCH(min(kc + 1, nk - 1))               // in flight during the contraction
        const uint8_t* fb = fbuf + (kc & 1) * FCB;
        uint32_t w[MT][4];                       // 8 counts of the lane's row, two per word
        int32_t c[MT];                           // the chunk's level of that row
        bool anyhi = false;
#pragma unroll
        for (int a = 0; a < MT; ++a) {
            const uint4 q = qr[d % kDepth][a];      // (a row past the last one: the last row again)
            w[a][0] = q.x, w[a][1] = q.y, w[a][2] = q.z, w[a][3] = q.w;
            // slot d, consumed, now takes chunk kc + kDepth
            qr[d % kDepth][a] = *reinterpret_cast<const uint4*>(hrow[a] + min(kc + kDepth, nk - 1) * kChunk);
            uint32_t s8 = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) s8 = __builtin_amdgcn_udot2(__builtin_bit_cast(u16x2, w[a][j]), u16x2{1, 1}, s8, false);
            rsum[a] += s8;
            // the chunk's level: its rounded mean.  The four lanes of a row (lane, lane ^ 16,
            // lane ^ 32, lane ^ 48) hold eight bins each: swapping 16-lane rows, then 32-lane
            // halves, and adding gives each of them the sum of all four.
            const auto p16 = __builtin_amdgcn_permlane16_swap(s8, s8, false, false);
            const uint32_t s16 = p16[0] + p16[1];
            const auto p32 = __builtin_amdgcn_permlane32_swap(s16, s16, false, false);
            c[a] = (int32_t)((p32[0] + p32[1] + 16u) >> 5);
            if (kg == 0) lv[kc * (MT * 16) + a * 16 + li] = (uint16_t)c[a];
        }
        if constexpr (PREC == SRT3D_PREC_FP32) {
#pragma unroll
            for (int b = 0; b < NT; ++b) {
                const float4* fp = reinterpret_cast<const float4*>(fb + (b * 16 + li) * FP + kg * 32);
                const float4 f0 = fp[0], f1 = fp[1];
                const float fv[8] = {f0.x, f0.y, f0.z, f0.w, f1.x, f1.y, f1.z, f1.w};
#pragma unroll
                for (int a = 0; a < MT; ++a)
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const int32_t cnt = (int32_t)((j & 1) ? w[a][j >> 1] >> 16 : w[a][j >> 1] & 0xffffu) - c[a];
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32((float)cnt, fv[j], acc[a][b], 0, 0, 0);
                    }
            }
        } else {
            // Fast form: x = count - level + LIM in each 16-bit half (packed, modulo 2^16).  When
            // every x of the wave is below 2 LIM, every d = x - LIM is exact in the 16-bit format
            // and the split is not needed (LIM = 512 for FP16: the value 1024 + x read from the
            // bits 0x6400 | x, minus 1536; LIM = 128 for BF16: x from its low byte, minus 128).
            // For |d| < LIM no x wraps: levels are chunk means, so |d| <= 63487.
            constexpr bool H16 = PREC == SRT3D_PREC_FP16X2;
            constexpr uint32_t LIM = H16 ? 512u : 128u;
            constexpr uint32_t HIGH = H16 ? 0xFC00FC00u : 0xFF00FF00u;      // bits at or above 2 LIM
            uint32_t x[MT][4];
#pragma unroll
            for (int a = 0; a < MT; ++a) {
                const uint32_t bc = ((LIM - (uint32_t)c[a]) & 0xffffu) * 0x10001u;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    x[a][j] = __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, w[a][j]) + __builtin_bit_cast(u16x2, bc));
                anyhi |= ((x[a][0] | x[a][1] | x[a][2] | x[a][3]) & HIGH) != 0;
            }
            const bool hi_wave = __any(anyhi);
            typedef typename std::conditional<H16, v8h, v8bf>::type v8;
            v8 alo[MT], ahi[MT];
            if (!hi_wave) {
#pragma unroll
                for (int a = 0; a < MT; ++a) {
                    uint32_t o[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        if constexpr (H16) {
                            const h16x2 v = __builtin_bit_cast(h16x2, x[a][j] | 0x64006400u) -
                                            h16x2{(_Float16)1536.f, (_Float16)1536.f};
                            o[j] = __builtin_bit_cast(uint32_t, v);
                        } else {
                            // |d| < 128 has at most 8 significant bits: the high half of its FP32
                            // form is its BF16 form
                            const float lo = (float)(x[a][j] & 0xffu) - 128.f;
                            const float hi = (float)((x[a][j] >> 16) & 0xffu) - 128.f;
                            o[j] = (__builtin_bit_cast(uint32_t, lo) >> 16) | (__builtin_bit_cast(uint32_t, hi) & 0xffff0000u);
                        }
                    }
                    alo[a] = __builtin_bit_cast(v8, make_uint4(o[0], o[1], o[2], o[3]));
                }
            } else {
                constexpr int SH = Prec<PREC>::shift;
#pragma unroll
                for (int a = 0; a < MT; ++a) {
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        // d = 2^SH q + r with q = round(d / 2^SH) (ties up) and |r| <= 2^(SH-1):
                        // both exact in the 16-bit format for |d| <= 63487 (see the file comment)
                        const int32_t dd = (int32_t)((j & 1) ? w[a][j >> 1] >> 16 : w[a][j >> 1] & 0xffffu) - c[a];
                        const int32_t q = (dd + (1 << (SH - 1))) >> SH;
                        const int32_t r = dd - (q << SH);
                        if constexpr (H16) {
                            alo[a][j] = (_Float16)(float)r;
                            ahi[a][j] = (_Float16)(float)(q << SH);
                        } else {
                            alo[a][j] = (__bf16)(float)r;
                            ahi[a][j] = (__bf16)(float)(q << SH);
                        }
                    }
                }
            }
#pragma unroll
            for (int b = 0; b < NT; ++b) {
#pragma unroll
                for (int sp = 0; sp < S; ++sp) {
                    const v8 fbv = __builtin_bit_cast(
                        v8, *reinterpret_cast<const uint4*>(fb + ((sp * NT + b) * 16 + li) * FP + kg * 16));
#pragma unroll
                    for (int a = 0; a < MT; ++a) {
                        if constexpr (H16)
                            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(alo[a], fbv, acc[a][b], 0, 0, 0);
                        else
                            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[a], fbv, acc[a][b], 0, 0, 0);
                    }
                    if (hi_wave) {
#pragma unroll
                        for (int a = 0; a < MT; ++a) {
                            if constexpr (H16)
                                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ahi[a], fbv, acc[a][b], 0, 0, 0);
                            else
                                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[a], fbv, acc[a][b], 0, 0, 0);
                        }
                    }
                }
            }
        }
        if (d == 3 || kc == nk - 1) {
            // the group's levels, this wave's own LDS writes (padding chunks hold level 0)
#pragma unroll
            for (int a = 0; a < MT; ++a) {
                const double ca = (double)lv[(kb + kg) * (MT * 16) + a * 16 + prow];
#pragma unroll
                for (int b = 0; b < NT; ++b)
                    lacc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ca, gcur[b], lacc[a][b], 0, 0, 0);
            }
        }
        SRT3D_F_STORE((kc + 1) & 1)                      // (the last chunk again after the last one)
        lds_barrier();                                          // staged chunk kc + 1 complete, kc free
    }

    // Row sums: the 4 lanes with the same (lane & 15) hold partial sums of one row.
#pragma unroll
    for (int a = 0; a < MT; ++a) {
        uint32_t v = rsum[a];
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        rsum[a] = v;
    }
    if (r0 >= P) return;                                        // (no barrier follows)

    const int twom = 2 * m;
#pragma unroll
    for (int b = 0; b < NT; ++b) {
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
                        n > 0 ? (float)(((double)acc[a][b][i] + lacc[a][b][i]) / (double)n) : 0.f;
            }
        }
    }
#pragma unroll
    for (int a = 0; a < MT; ++a)
        if (kg == 0 && r0 + a * 16 + li < P) nout[r0 + a * 16 + li] = (int32_t)rsum[a];
}
#undef SRT3D_F_FETCH
#undef SRT3D_F_STORE

template <int PREC, int NT>
static size_t hist_lds_bytes(int T) {
    return 2 * (size_t)f_chunk_bytes<PREC, NT>() + (size_t)kWavesPerBlock * n_chunks4(T) * kMT * 16 * sizeof(uint16_t);
}

template <int PREC, int NT>
static hipError_t launch_hist_nt(const uint16_t* H, int P, int T, int m, const void* ws, float* z, int32_t* n,
                                 hipStream_t s) {
    // one 16-row tile per wave: 4096 waves at 256^2, four per SIMD (two tiles per wave measured
    // slower: fewer waves to hide the loads and the barriers behind)
    const int64_t waves = ((int64_t)P + kMT * 16 - 1) / (kMT * 16);
    const unsigned blocks = (unsigned)((waves + kWavesPerBlock - 1) / kWavesPerBlock);
    const size_t lds = hist_lds_bytes<PREC, NT>(T);
    if (lds > 65536) {
        // T = 8192 with wide column tiles needs more than the default dynamic LDS limit
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&hist_mfma_kernel<PREC, NT>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((hist_mfma_kernel<PREC, NT>), dim3(blocks), dim3(kThreads), lds, s,
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
