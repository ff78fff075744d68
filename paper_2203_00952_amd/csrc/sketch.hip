// Photon sketch, Section 2, eq. (3):  z_l = (1/n) sum_p exp(i w_l x_p),  w_l = 2 pi l / T.
//
// Design (gfx950):
//  * The phase w_l x_p is reduced exactly: k_l = (l x_p) mod T is advanced by integer adds and
//    a wrap, and (cos, sin)(2 pi k / T) is read from a T-entry float2 table held in LDS (loaded
//    once per persistent workgroup).  Odd harmonics are table reads; each even harmonic is the
//    preceding entry times exp(i w_1 x) (one complex multiply), halving the LDS reads.  No
//    transcendental runs per photon.
//  * A group of G lanes owns one pixel; its lanes stride through the pixel's stamps, so each
//    wave load is G contiguous int32 per pixel (coalesced).  Each lane keeps 2*MC FP32 partial
//    sums (MC harmonics per pass; m is split into power-of-two passes <= 32).
//  * The G partial sums are combined by a reduce-scatter butterfly across the group (each step
//    halves the values a lane keeps), so the reduction costs O(values) instead of
//    O(values * log G), and the surviving lanes hold distinct outputs for a coalesced store.
//  * Normalisation z = S / n is done in FP64; optional FP64 long-exposure accumulators take
//    S and n across calls (the sketch is updated online, Section 2).
#include "common.hpp"

namespace srt3d {

__global__ void phase_table_kernel(int T, float2* __restrict__ table) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= T) return;
    double s, c;
    sincospi(2.0 * (double)k / (double)T, &s, &c);
    table[k] = make_float2((float)c, (float)s);
}

hipError_t launch_phase_table(int T, float2* table, hipStream_t s) {
    hipLaunchKernelGGL(phase_table_kernel, dim3((T + 255) / 256), dim3(256), 0, s, T, table);
    return hipGetLastError();
}

__global__ void phase_indices_kernel(const int32_t* __restrict__ x, int64_t N, int T, int m,
                                     int32_t* __restrict__ kout) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const uint32_t T8 = (uint32_t)T << 3;
    const uint32_t x8 = (uint32_t)fold_stamp(x[p], T) << 3;
    const bool pow2 = (T & (T - 1)) == 0;
    uint32_t k8 = 0;
    for (int l = 0; l < m; ++l) {
        k8 = pow2 ? phase_advance<true>(k8, x8, T8) : phase_advance<false>(k8, x8, T8);
        kout[(int64_t)l * N + p] = (int32_t)(k8 >> 3);
    }
}

hipError_t launch_phase_indices(const int32_t* x, int64_t N, int T, int m, int32_t* k, hipStream_t s) {
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(phase_indices_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, x, N, T, m, k);
    return hipGetLastError();
}

// Reduce-scatter across the G lanes of a group.  On entry each lane holds V values; at each
// step with xor distance O the lane keeps one half (upper half if lane & O) and adds the
// partner's copy of that half.  Once a lane holds one value the remaining steps are plain
// butterflies.  `base` returns the index (into the original V) of the first value kept.
template <int V, int O>
__device__ __forceinline__ void reduce_scatter(float* v, int lane, int& base) {
    if constexpr (O >= 1) {
        if constexpr (V > 1) {
            const bool upper = (lane & O) != 0;
#pragma unroll
            for (int i = 0; i < V / 2; ++i) {
                const float send = upper ? v[i] : v[i + V / 2];
                const float keep = upper ? v[i + V / 2] : v[i];
                v[i] = keep + shfl_xor_f(send, O);
            }
            if (upper) base += V / 2;
            reduce_scatter<V / 2, O / 2>(v, lane, base);
        } else {
            v[0] += shfl_xor_f(v[0], O);
            reduce_scatter<1, O / 2>(v, lane, base);
        }
    }
}

// Add photon x's harmonics l0+1 .. l0+MC into v (odd ones from the table, even ones as the
// preceding entry times exp(i w_1 x)).  EXPORT (inspection only): also write the table index of
// every harmonic read from the table, kexp[(l - 1) N + pidx]; the others are left as they are.
template <int MC, bool POW2, bool EXPORT>
__device__ __forceinline__ void add_photon(float* v, int32_t x, int l0, int T, uint32_t T8, const char* tab,
                                           int32_t* kexp, int64_t N, int64_t pidx) {
    const uint32_t x8 = (uint32_t)x << 3;
    if constexpr (MC == 1) {
        uint32_t k8 = x8;
        if (l0 != 0) {
            const uint32_t lx = (uint32_t)(l0 + 1) * (uint32_t)x;
            k8 = (POW2 ? (lx & (uint32_t)(T - 1)) : (lx % (uint32_t)T)) << 3;
        }
        const float2 c = *reinterpret_cast<const float2*>(tab + k8);
        if constexpr (EXPORT) kexp[(int64_t)l0 * N + pidx] = (int32_t)(k8 >> 3);
        v[0] += c.x;
        v[1] += c.y;
    } else {
        const float2 u1 = *reinterpret_cast<const float2*>(tab + x8);   // exp(i w_1 x)
        const uint32_t x8x2 = phase_advance<POW2>(x8, x8, T8);            // 2x mod T
        uint32_t k8 = x8;                                                  // phase of l0 + 1
        if (l0 != 0) {
            const uint32_t lx = (uint32_t)(l0 + 1) * (uint32_t)x;
            k8 = (POW2 ? (lx & (uint32_t)(T - 1)) : (lx % (uint32_t)T)) << 3;
        }
#pragma unroll
        for (int j = 0; j < MC; j += 2) {
            const float2 c = (j == 0 && l0 == 0) ? u1 : *reinterpret_cast<const float2*>(tab + k8);
            if constexpr (EXPORT) kexp[(int64_t)(l0 + j) * N + pidx] = (int32_t)(((j == 0 && l0 == 0) ? x8 : k8) >> 3);
            v[2 * j] += c.x;
            v[2 * j + 1] += c.y;
            // next harmonic: += c * u1, as four fused multiply-adds
            v[2 * j + 2] = fmaf(c.x, u1.x, v[2 * j + 2]);
            v[2 * j + 2] = fmaf(-c.y, u1.y, v[2 * j + 2]);
            v[2 * j + 3] = fmaf(c.x, u1.y, v[2 * j + 3]);
            v[2 * j + 3] = fmaf(c.y, u1.x, v[2 * j + 3]);
            k8 = phase_advance<POW2>(k8, x8x2, T8);
        }
    }
}

// One pass over a pixel's photons for harmonics l0+1 .. l0+MC.  Harmonics come in pairs: the
// first of each pair is read from the table at its exact phase k = (l x) mod T (advanced by 2x
// per pair), the second is that entry times exp(i w_1 x), the table entry at k = x, so each
// photon costs MC/2 table reads (LDS bandwidth, with its data-dependent bank conflicts, is a
// binding resource) and two extra multiply-adds per pair.  Stamps are loaded kU per lane at a
// time, the next group while the current one is summed, to keep loads in flight.
//
// Summation is two-level so that FP32 rounding stays bounded for any photon count: a lane's
// run of at most kSeg * kU photons goes into v, the group's runs are combined by the
// reduce-scatter, and the segments are added into f (KEEP values per lane).  A run of k equal
// terms rounds to within about k 2^-25 relative; k <= 128 keeps that near 4e-6.
constexpr int kU = 4;
constexpr int kSeg = 32;

template <int MC, int G, bool POW2, bool EXPORT>
__device__ __forceinline__ void sketch_pass(const int32_t* __restrict__ stamps, int64_t b, int64_t e, int lane,
                                            int l0, int T, uint32_t T8, const float2* s_table, int64_t count,
                                            int64_t count_total, float* __restrict__ zrow,
                                            double* __restrict__ accrow, int& bad, int32_t* kexp, int64_t N) {
    constexpr int V = 2 * MC;
    constexpr int KEEP = V >= G ? V / G : 1;
    constexpr int DUP = V >= G ? 1 : G / V;       // lanes holding identical sums
    const char* tab = reinterpret_cast<const char*>(s_table);
    float v[V], f[KEEP];
#pragma unroll
    for (int i = 0; i < V; ++i) v[i] = 0.f;
#pragma unroll
    for (int i = 0; i < KEEP; ++i) f[i] = 0.f;
    const int sub = lane & (G - 1);
    int32_t cur[kU], nxt[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) cur[u] = (b + sub + u * G < e) ? stamps[b + sub + u * G] : 0;
    int base = 0, run = 0;
    // q0 is the same for every lane of the group, so a segment flush (which shuffles within the
    // group) is taken by all of its lanes together.
    for (int64_t q0 = b; q0 < e; q0 += kU * G) {
        const int64_t p = q0 + sub, pn = p + kU * G;
#pragma unroll
        for (int u = 0; u < kU; ++u) nxt[u] = (pn + u * G < e) ? stamps[pn + u * G] : 0;
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            if (p + u * G < e) {
                int32_t x = cur[u];
                if ((uint32_t)x >= (uint32_t)T) {
                    x = fold_stamp(x, T);
                    if (l0 == 0) ++bad;
                }
                add_photon<MC, POW2, EXPORT>(v, x, l0, T, T8, tab, kexp, N, p + u * G);
            }
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) cur[u] = nxt[u];
        if (++run == kSeg && q0 + kU * G < e) {
            base = 0;
            reduce_scatter<V, G / 2>(v, lane, base);
#pragma unroll
            for (int i = 0; i < KEEP; ++i) f[i] += v[i];
#pragma unroll
            for (int i = 0; i < V; ++i) v[i] = 0.f;
            run = 0;
        }
    }
    base = 0;
    reduce_scatter<V, G / 2>(v, lane, base);
#pragma unroll
    for (int i = 0; i < KEEP; ++i) f[i] += v[i];
    if ((sub & (DUP - 1)) != 0) return;
    const int o = 2 * l0 + base;
    if (accrow) {
#pragma unroll
        for (int i = 0; i < KEEP; ++i) {
            const double a = accrow[o + i] + (double)f[i];
            accrow[o + i] = a;
            zrow[o + i] = count_total > 0 ? (float)(a / (double)count_total) : 0.f;
        }
    } else {
#pragma unroll
        for (int i = 0; i < KEEP; ++i)
            zrow[o + i] = count > 0 ? (float)((double)f[i] / (double)count) : 0.f;
    }
}

// TB is the LDS capacity of the table (a power of two >= T): a static array whose LDS offset is
// known at compile time, so the byte phase k8 is the ds_read address with no base add.
// MCMAX bounds the harmonics per pass (16 or 32): the register budget, and with it occupancy,
// follows the largest pass the kernel contains, so m <= 16 uses a kernel without the 32 pass.
template <int G, bool POW2, int TB, int MCMAX, bool EXPORT>
__global__ __launch_bounds__(256) void sketch_photons_kernel(
    const int32_t* __restrict__ stamps, int64_t N, const int64_t* __restrict__ offsets, int P, int T, int m,
    const float2* __restrict__ table, float* __restrict__ z, int32_t* __restrict__ nout,
    double* __restrict__ acc, int64_t* __restrict__ nacc, int32_t* __restrict__ err, int32_t* __restrict__ kexp) {
    __shared__ float2 s_table[TB];
    for (int i = threadIdx.x; i < T; i += blockDim.x) s_table[i] = table[i];
    __syncthreads();

    const int lane = threadIdx.x & (kWave - 1);
    const int sub = lane & (G - 1);
    const int groups_per_block = blockDim.x / G;
    const int64_t total_groups = (int64_t)gridDim.x * groups_per_block;
    const uint32_t T8 = (uint32_t)T << 3;
    int bad_stamps = 0, bad_offsets = 0;

    for (int64_t pix = (int64_t)blockIdx.x * groups_per_block + threadIdx.x / G; pix < P; pix += total_groups) {
        int64_t b = offsets[pix], e = offsets[pix + 1];
        const bool clipped = b < 0 || b > N || e < 0 || e > N;
        b = b < 0 ? 0 : (b > N ? N : b);
        e = e < 0 ? 0 : (e > N ? N : e);
        if (e < b || clipped) {
            if (sub == 0) ++bad_offsets;
            if (e < b) e = b;
        }
        const int64_t count = e - b;
        int64_t count_total = count;
        float* zrow = z + (int64_t)pix * m * 2;
        double* accrow = nullptr;
        if (acc) {
            accrow = acc + (int64_t)pix * m * 2;
            count_total = nacc[pix] + count;
        }
        for (int l0 = 0; l0 < m;) {
            const int rem = m - l0;
            const int mc = rem >= MCMAX ? MCMAX : (1 << (31 - __builtin_clz((unsigned)rem)));
            switch (mc) {
                case 32:
                    if constexpr (MCMAX >= 32)
                        sketch_pass<32, G, POW2, EXPORT>(stamps, b, e, lane, l0, T, T8, s_table, count, count_total, zrow, accrow, bad_stamps, kexp, N);
                    break;
                case 16: sketch_pass<16, G, POW2, EXPORT>(stamps, b, e, lane, l0, T, T8, s_table, count, count_total, zrow, accrow, bad_stamps, kexp, N); break;
                case 8: sketch_pass<8, G, POW2, EXPORT>(stamps, b, e, lane, l0, T, T8, s_table, count, count_total, zrow, accrow, bad_stamps, kexp, N); break;
                case 4: sketch_pass<4, G, POW2, EXPORT>(stamps, b, e, lane, l0, T, T8, s_table, count, count_total, zrow, accrow, bad_stamps, kexp, N); break;
                case 2: sketch_pass<2, G, POW2, EXPORT>(stamps, b, e, lane, l0, T, T8, s_table, count, count_total, zrow, accrow, bad_stamps, kexp, N); break;
                default: sketch_pass<1, G, POW2, EXPORT>(stamps, b, e, lane, l0, T, T8, s_table, count, count_total, zrow, accrow, bad_stamps, kexp, N); break;
            }
            l0 += mc;
        }
        if (sub == 0) {
            if (acc) nacc[pix] = count_total;
            nout[pix] = (int32_t)(count_total > 0x7fffffff ? 0x7fffffff : count_total);
        }
    }
    if (err) {
        if (bad_stamps) atomicAdd(&err[0], bad_stamps);
        if (bad_offsets) atomicAdd(&err[1], bad_offsets);
    }
}

template <int G, bool POW2, int TB, int MCMAX, bool EXPORT = false>
static hipError_t launch_sketch_g(const int32_t* stamps, int64_t N, const int64_t* offsets, int P, int T, int m,
                                  const float2* table, float* z, int32_t* n, double* acc, int64_t* nacc,
                                  int32_t* err, hipStream_t s, int32_t* kexp = nullptr) {
    constexpr int threads = 256;
    int cus = 0, per_cu = 0;
    hipError_t st = current_device_cus(&cus);
    if (st != hipSuccess) return st;
    st = cached_occupancy<sketch_photons_kernel<G, POW2, TB, MCMAX, EXPORT>, threads>(&per_cu);
    if (st != hipSuccess) return st;
    const int64_t groups_per_block = threads / G;
    const int64_t need = ((int64_t)P + groups_per_block - 1) / groups_per_block;
    const int64_t cap = (int64_t)cus * per_cu;
    const unsigned blocks = (unsigned)(need < cap ? need : cap);
    hipLaunchKernelGGL((sketch_photons_kernel<G, POW2, TB, MCMAX, EXPORT>), dim3(blocks), dim3(threads), 0, s, stamps, N,
                       offsets, P, T, m, table, z, n, acc, nacc, err, kexp);
    return hipGetLastError();
}

template <int G, bool POW2>
static hipError_t launch_sketch_tb(const int32_t* stamps, int64_t N, const int64_t* offsets, int P, int T, int m,
                                   const float2* table, float* z, int32_t* n, double* acc, int64_t* nacc,
                                   int32_t* err, hipStream_t s) {
#define SRT3D_TB(TBV)                                                                                            \
    return m <= 16 ? launch_sketch_g<G, POW2, TBV, 16>(stamps, N, offsets, P, T, m, table, z, n, acc, nacc, err, s) \
                   : launch_sketch_g<G, POW2, TBV, 32>(stamps, N, offsets, P, T, m, table, z, n, acc, nacc, err, s)
    if (T <= 1024) SRT3D_TB(1024);
    if (T <= 2048) SRT3D_TB(2048);
    if (T <= 4096) SRT3D_TB(4096);
    SRT3D_TB(8192);
#undef SRT3D_TB
}

// The photon pass with its table indices written out (inspection): four lanes per pixel (the
// lane count decides which lane takes a photon, not how its phases are formed), otherwise the
// kernel and pass structure of launch_sketch_photons for this T and m.
template <bool POW2>
static hipError_t launch_sketch_export_tb(const int32_t* stamps, int64_t N, const int64_t* offsets, int P, int T, int m,
                                          const float2* table, float* z, int32_t* n, int32_t* kexp, hipStream_t s) {
#define SRT3D_TBX(TBV)                                                                                                    \
    return m <= 16 ? launch_sketch_g<4, POW2, TBV, 16, true>(stamps, N, offsets, P, T, m, table, z, n, nullptr, nullptr, \
                                                             nullptr, s, kexp)                                          \
                   : launch_sketch_g<4, POW2, TBV, 32, true>(stamps, N, offsets, P, T, m, table, z, n, nullptr, nullptr, \
                                                             nullptr, s, kexp)
    if (T <= 1024) SRT3D_TBX(1024);
    if (T <= 2048) SRT3D_TBX(2048);
    if (T <= 4096) SRT3D_TBX(4096);
    SRT3D_TBX(8192);
#undef SRT3D_TBX
}

hipError_t launch_sketch_photons_export(const int32_t* stamps, int64_t N, const int64_t* offsets, int P, int T, int m,
                                        const float2* table, float* z, int32_t* n, int32_t* kexp, hipStream_t s) {
    return (T & (T - 1)) == 0 ? launch_sketch_export_tb<true>(stamps, N, offsets, P, T, m, table, z, n, kexp, s)
                              : launch_sketch_export_tb<false>(stamps, N, offsets, P, T, m, table, z, n, kexp, s);
}

// Lanes per pixel from the mean photon count: enough lanes to keep the stride loop busy, few
// enough that the per-pixel reduction and the idle tail stay small.
static int lanes_per_pixel(int64_t N, int P) {
    const double mean = P > 0 ? (double)N / (double)P : 0.0;
    if (mean < 24) return 4;
    if (mean < 96) return 8;
    if (mean < 384) return 16;
    if (mean < 1536) return 32;
    return 64;
}

hipError_t launch_sketch_photons(const int32_t* stamps, int64_t N, const int64_t* offsets, int P, int T, int m,
                                 const float2* table, float* z, int32_t* n, double* acc, int64_t* nacc,
                                 int32_t* err, hipStream_t s, int lanes) {
    const bool pow2 = (T & (T - 1)) == 0;
    const int G = lanes > 0 ? lanes : lanes_per_pixel(N, P);
#define SRT3D_SK(GG)                                                                                              \
    return pow2 ? launch_sketch_tb<GG, true>(stamps, N, offsets, P, T, m, table, z, n, acc, nacc, err, s)         \
                : launch_sketch_tb<GG, false>(stamps, N, offsets, P, T, m, table, z, n, acc, nacc, err, s)
    switch (G) {
        case 4: SRT3D_SK(4);
        case 8: SRT3D_SK(8);
        case 16: SRT3D_SK(16);
        case 32: SRT3D_SK(32);
        default: SRT3D_SK(64);
    }
#undef SRT3D_SK
}

}  // namespace srt3d
