// Photon sketch through a per-pixel histogram on the matrix cores (Section 2, eq. 2 with unit
// bins, then eq. 3).  Same result as the photon-parallel pass, by a different route.
//
// Stamps are integers in [0, T), so the sketch of the photons equals the sketch of their unit-bin
// histogram H.  Write a stamp as x = 64 j + r (j < J = ceil(T / 64), r < 64); then
//     S_l = sum_j W_l[j] G_l[j],   G_l[j] = sum_r H[j][r] V_l[r],
//     V_l[r] = exp(i w_l r),       W_l[j] = exp(i w_l 64 j),
// with both phases reduced exactly mod T and read from the FP32 phase table.  Per pixel:
//  * H is built in LDS by integer atomics, four 8-bit bins to a 32-bit word (one ds_add per
//    photon, no per-photon harmonic work).  A bin that passes 255 carries into its neighbour (or
//    out of the word); then the bins no longer sum to n.  A pixel with more than 255 photons sums
//    its bins (exactly, on the matrix cores) and, if the sum is off, is redone in chunks of at
//    most 255 photons, which cannot overflow.
//  * G = H[J x 64] . V[64 x 2m] runs as v_mfma_f32_16x16x32_f16.  Counts <= 255 are exact in
//    FP16; V is split as V = V1 + V2 with V1 = fp16(V), V2 = fp16(V - V1), both products
//    accumulated in FP32 in one chain, so G carries V to about 2^-22 (2^-25 absolute).
//  * The twiddle sum over j is FP32 FMAs in the MFMA output layout, then a fixed-order sum over the
//    lanes' row groups; z = S / n in FP64 as in the photon pass.
// The per-photon cost is one LDS atomic and five integer instructions; the per-pixel cost is
// T * 2m * 2 MFMA multiply-adds and the conversion of T bytes to FP16.
//
// Work layout: every wave owns a contiguous range of pixels (so one contiguous range of stamps)
// and its own histogram in LDS, and works through its pixels without any workgroup barrier, so
// the latencies of one wave's steps (loads, LDS round trips, MFMA chains) overlap the work of
// the others.  Stamps stream in runs of U per lane through bounds-checked buffer loads (one
// descriptor per run, no per-load address arithmetic); two register sets alternate so the next
// run is always in flight, across pixel boundaries.  The twiddles W are shared by the
// workgroup's four waves in LDS; the V fragments (B operands) stay in registers.
#include "common.hpp"

namespace srt3d {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef _Float16 v2h __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) uint32_t lds_u32;

constexpr int kBinThreads = 256;
constexpr int kBinWaves = kBinThreads / kWave;
constexpr int kRowBins = 64;            // r range: bins per histogram row
// A row is 64 8-bit bins (64 bytes) and 16 bytes of padding, so consecutive rows start 20 banks
// apart and the lanes that read 8 bytes at the same place of 16 consecutive rows (an A-operand
// load) touch different banks.
constexpr int kRowPitch = 80;
constexpr int kTilePitch = 16 * kRowPitch;
constexpr int kSafeChunk = 255;         // photons per chunk that cannot overflow an 8-bit bin
constexpr int kRsrcFlags = 0x00020000;  // buffer descriptor word 3: raw 32-bit dwords

__device__ __forceinline__ uint32_t lds_address(const void* p) {
    return (uint32_t)(size_t)(__attribute__((address_space(3))) const uint8_t*)p;
}

// Byte layout of a 64-bin histogram row: bin r is byte r, so bin x (0 <= x < 64 J) sits in byte
// x & 3 of the row's word (x & 63) >> 2.  Both the word address and the one-hot increment then take
// two instructions each: the shift amount 8 (x & 3) is (x << 3) mod 32, which is what a 32-bit shift
// uses of its amount.  (Spreading a surface's ~20 consecutive bins over more words, bin r in word
// r & 15 and byte r >> 4, avoids some same-word atomics in one instruction but costs three more
// instructions per photon, which measured slower.)  The V fragments follow the same order.
__device__ __forceinline__ int row_bin(int p) { return p; }

// Byte address of the 32-bit word that holds bin x in the histogram at hbase (a multiple of 64):
// row x >> 6 starts at byte 80 (x >> 6).
__device__ __forceinline__ uint32_t bin_word(uint32_t hbase, uint32_t x) {
    return __builtin_amdgcn_ubfe(x, 6, 16) * (uint32_t)kRowPitch + ((x & 60u) | hbase);
}

// 1 in the byte of its word that holds bin x.
__device__ __forceinline__ uint32_t bin_one(uint32_t x) { return 1u << ((x << 3) & 31u); }

__device__ __forceinline__ void bin_add(uint32_t hbase, uint32_t x, uint32_t one) {
    __hip_atomic_fetch_add((lds_u32*)(size_t)bin_word(hbase, x), one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Eight 8-bit counts (two words) as eight FP16 values b - c: each byte b becomes the FP16 bit
// pattern 0x6400 | b, which is 1024 + b, and bias = -(1024 + c) is then added exactly.
__device__ __forceinline__ v8h bytes_to_h8(uint32_t w0, uint32_t w1, v2h bias) {
    const uint32_t k64 = 0x64646464u;
    uint32_t u[4];
    u[0] = __builtin_amdgcn_perm(k64, w0, 0x04010400u);
    u[1] = __builtin_amdgcn_perm(k64, w0, 0x04030402u);
    u[2] = __builtin_amdgcn_perm(k64, w1, 0x04010400u);
    u[3] = __builtin_amdgcn_perm(k64, w1, 0x04030402u);
    v8h out;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        v2h h = __builtin_bit_cast(v2h, u[i]);
        h = h + bias;
        out[2 * i] = h[0];
        out[2 * i + 1] = h[1];
    }
    return out;
}

// Eight histogram bytes, replaced by zeros (ds_wrxchg_rtn_b64).
__device__ __forceinline__ uint2 take8(uint8_t* p) {
    const uint64_t v = __hip_atomic_exchange(reinterpret_cast<uint64_t*>(p), (uint64_t)0, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_WORKGROUP);
    return make_uint2((uint32_t)v, (uint32_t)(v >> 32));
}

__device__ __forceinline__ _Float16 split_hi(float v) { return (_Float16)v; }
__device__ __forceinline__ _Float16 split_lo(float v) { return (_Float16)(v - (float)(_Float16)v); }

// Sum over the 64 lanes: inclusive scans within each row of 16 lanes (DPP row shifts, no LDS),
// then the four row totals.
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);   // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);   // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);   // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);   // row_shr:8
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 15) + (uint32_t)__builtin_amdgcn_readlane((int)v, 31) +
           (uint32_t)__builtin_amdgcn_readlane((int)v, 47) + (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ __forceinline__ int64_t uniform64(int64_t x) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// B operands: lane c = lane & 15 is column (harmonic l = 16 q + c + 1), g = lane >> 4 its
// k group (bins r = 32 ks + 8 g .. + 7).
template <int Q>
struct VFrags {
    v8h hi[2][Q][2], lo[2][Q][2];     // [k-step][q][re/im]
    float2 wl[4][Q];                  // W_l[4 g + i]: the lane's row twiddles within a tile
};

template <int Q>
__device__ __forceinline__ void load_vfrags(VFrags<Q>& V, const float2* __restrict__ table, int T, int m, int lane) {
    const int c = lane & 15, g = lane >> 4;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int l = 16 * q + c + 1;
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int r = row_bin(32 * ks + 8 * g + e);
                float cv = 0.f, sv = 0.f;
                if (l <= m) {
                    int ph = l * r;                         // < 32 * 64: a few subtractions at most for T >= 1024
                    while (ph >= T) ph -= T;
                    const float2 t = table[ph];
                    cv = t.x;
                    sv = t.y;
                }
                V.hi[ks][q][0][e] = split_hi(cv);
                V.lo[ks][q][0][e] = split_lo(cv);
                V.hi[ks][q][1][e] = split_hi(sv);
                V.lo[ks][q][1][e] = split_lo(sv);
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
            V.wl[i][q] = l <= m ? table[(int)(((int64_t)l * kRowBins * (4 * g + i)) % T)] : make_float2(0.f, 0.f);
    }
}

// One M-tile (rows j = 16 mt .. 16 mt + 15) of the product, added into sre/sim.  Both terms of
// the split V = V1 + V2 multiply the same A in one accumulator (V2 = fp16(V - V1) is stored
// unscaled: where it is subnormal its absolute error stays below 2^-25).  The twiddle of row
// j = 16 mt + 4 g + i factors exactly as W_l[16 mt] * W_l[4 g + i]: the lane's four row twiddles
// W_l[4 g + i] stay in registers, the tile's common factor W_l[16 mt] is one LDS read per lane
// and tile.  The counts enter as count - dc (see mfma_tiles); their raw byte sum is added to bsum.
template <int Q>
__device__ __forceinline__ void mfma_tile(uint8_t* hist, const float2* s_wm, const VFrags<Q>& V, int mt,
                                          int lane, v2h bias, float* sre, float* sim, uint32_t& bsum) {
    const int c = lane & 15, g = lane >> 4;
    // row c of the tile, bytes 8 g .. 8 g + 7 (k-step 0) and 32 + 8 g .. (k-step 1); each byte is
    // read by exactly one lane of one tile: read it and leave zero behind in one LDS exchange, so
    // the histogram is clear for the next pixel without a separate pass
    uint8_t* row = hist + mt * kTilePitch + c * kRowPitch + 8 * g;
    const uint2 w0 = take8(row), w1 = take8(row + 32);
    float2 wm[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) wm[q] = s_wm[mt * (16 * Q) + 16 * q + c];
    bsum = __builtin_amdgcn_sad_u8(w0.x, 0u, bsum);
    bsum = __builtin_amdgcn_sad_u8(w0.y, 0u, bsum);
    bsum = __builtin_amdgcn_sad_u8(w1.x, 0u, bsum);
    bsum = __builtin_amdgcn_sad_u8(w1.y, 0u, bsum);
    const v8h A0 = bytes_to_h8(w0.x, w0.y, bias), A1 = bytes_to_h8(w1.x, w1.y, bias);
    v4f acc[Q][2];
    const v4f zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            acc[q][p] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A0, V.hi[0][q][p], zero, 0, 0, 0);
            acc[q][p] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A0, V.lo[0][q][p], acc[q][p], 0, 0, 0);
            acc[q][p] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A1, V.hi[1][q][p], acc[q][p], 0, 0, 0);
            acc[q][p] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A1, V.lo[1][q][p], acc[q][p], 0, 0, 0);
        }
    // output element i of a tile: row 4 g + i, column c
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        float ur = 0.f, ui = 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float gr = acc[q][0][i], gi = acc[q][1][i];
            const float wr = V.wl[i][q].x, wi = V.wl[i][q].y;
            ur = fmaf(wr, gr, fmaf(-wi, gi, ur));
            ui = fmaf(wr, gi, fmaf(wi, gr, ui));
        }
        sre[q] = fmaf(wm[q].x, ur, fmaf(-wm[q].y, ui, sre[q]));
        sim[q] = fmaf(wm[q].x, ui, fmaf(wm[q].y, ur, sim[q]));
    }
}

// Add the contribution of the histogram minus a constant `dc` in every bin to the lane's partial
// sums sre/sim (harmonic 16 q + c + 1, summed over the lane's rows 16 mt + 4 g + i) and the
// lane's raw byte sum to bsum, and leave the histogram zero.
//
// The constant changes nothing exactly: the sum of exp(i w_l t) over all T bins is zero for
// 0 < l < T.  With dc near the mean count it removes the common level of the bins, which would
// otherwise make every row sum G_l[j] of a low harmonic large (a row spans 64/T of a period)
// and the sum over j a cancellation whose FP32 rounding grows like n instead of sqrt(n).  It
// needs every A element to be a real bin (T a multiple of 1024, no padding rows); otherwise
// the caller passes dc = 0.
template <int Q, int MTT>
__device__ __forceinline__ void mfma_tiles(uint8_t* hist, const float2* s_wm, const VFrags<Q>& V, int MT,
                                           int lane, int dc, float* sre, float* sim, uint32_t& bsum) {
    const _Float16 bh = (_Float16)(float)(-1024 - dc);
    const v2h bias = {bh, bh};
    if (MT == MTT) {
        // every tile (the usual case): one straight block, so that one tile's loads and
        // conversions are scheduled among another's matrix products
#pragma unroll
        for (int mt = 0; mt < MTT; ++mt) mfma_tile<Q>(hist, s_wm, V, mt, lane, bias, sre, sim, bsum);
    } else {
#pragma unroll
        for (int mt = 0; mt < MTT; ++mt)
            if (mt < MT) mfma_tile<Q>(hist, s_wm, V, mt, lane, bias, sre, sim, bsum);
    }
}

__device__ __forceinline__ void zero_hist_wave(uint8_t* hist, int bytes, int lane) {
    for (int o = lane * 16; o < bytes; o += kWave * 16)
        *reinterpret_cast<uint4*>(hist + o) = make_uint4(0, 0, 0, 0);
}

// A run of stamps a wave streams: stamps [c0, c1) of pixel pix, whose clamped range is [pb, pe)
// (raw_e: its unclamped end offset, the next pixel's start).  `last` marks the pixel's final
// run; an empty pixel is one empty run.  Every field is wave-uniform.
struct Run {
    int64_t pix, c0, c1, pb, pe, raw_e;
    bool last, valid;
};

template <int Q, int MTT, int U>
__global__ __launch_bounds__(kBinThreads) __attribute__((amdgpu_waves_per_eu(Q == 1 && MTT == 4 && U <= 8 ? 4 : 1))) void sketch_binned_kernel(
    const int32_t* __restrict__ stamps, int64_t N, const int64_t* __restrict__ offsets, int P, int T, int m,
    const float2* __restrict__ table, float* __restrict__ z, int32_t* __restrict__ nout, double* __restrict__ acc,
    int64_t* __restrict__ nacc, int32_t* __restrict__ err) {
    constexpr int HB = MTT * kTilePitch;                      // histogram bytes per wave
    constexpr int C = U * kWave;                              // stamps per run
    __shared__ __align__(64) uint8_t s_hist[kBinWaves][HB];
    __shared__ float2 s_wm[MTT * 16 * Q];

    // the wave index is uniform across the wave: say so, so that everything derived from it (the
    // pixel range, each run, the offsets loads) stays in scalar registers and scalar loads
    const int lane = threadIdx.x & (kWave - 1), wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int J = (T + kRowBins - 1) / kRowBins;
    const int MT = (J + 15) / 16;
    uint8_t* hist = s_hist[wave];
    const uint32_t hbase = lds_address(hist);

    // tile twiddle factors W_l[16 mt] (zero for l > m), shared by the waves
    for (int idx = threadIdx.x; idx < MT * 16 * Q; idx += kBinThreads) {
        const int mt = idx / (16 * Q), l = idx % (16 * Q) + 1;
        s_wm[idx] = l <= m ? table[(int)(((int64_t)l * 16 * kRowBins * mt) % T)] : make_float2(0.f, 0.f);
    }
    zero_hist_wave(hist, HB, lane);
    VFrags<Q> V;
    load_vfrags<Q>(V, table, T, m, lane);
    __syncthreads();                                          // s_wm complete; the only barrier

    const int64_t gw = (int64_t)blockIdx.x * kBinWaves + wave, nw = (int64_t)gridDim.x * kBinWaves;
    const int64_t p0 = (int64_t)P * gw / nw, p1 = (int64_t)P * (gw + 1) / nw;
    if (p0 >= p1) return;                                     // whole wave
    int bad_stamps = 0, bad_offsets = 0;

    auto pixel_run = [&](int64_t pix, int64_t raw_b, int64_t raw_e) {
        int64_t b = raw_b < 0 ? 0 : (raw_b > N ? N : raw_b);
        int64_t e = raw_e < 0 ? 0 : (raw_e > N ? N : raw_e);
        if (e < b || b != raw_b || e != raw_e) {              // clamped or decreasing (as the photon pass)
            ++bad_offsets;
            if (e < b) e = b;
        }
        const int64_t c1 = b + C < e ? b + C : e;
        return Run{pix, b, c1, b, e, raw_e, c1 == e, true};
    };
    auto next = [&](const Run& d) {
        if (!d.valid) return d;
        if (!d.last) {
            const int64_t c1 = d.c1 + C < d.pe ? d.c1 + C : d.pe;
            return Run{d.pix, d.c1, c1, d.pb, d.pe, d.raw_e, c1 == d.pe, true};
        }
        if (d.pix + 1 >= p1) {
            Run r = d;
            r.valid = false;
            return r;
        }
        return pixel_run(d.pix + 1, d.raw_e, uniform64(offsets[d.pix + 2]));
    };
    // Every run issues its U loads, valid or not, through a buffer descriptor that covers exactly
    // the run's stamps: loads past its end (a short or invalid run) return 0 without touching
    // memory, and the compiler knows exactly which loads are younger than a run's data, so it
    // waits for that run alone.
    auto issue = [&](int32_t* v, const Run& d) {
        const int bytes = d.valid ? (int)(d.c1 - d.c0) * 4 : 0;
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<int32_t*>(stamps) + d.c0, (short)0, bytes, kRsrcFlags);
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = __builtin_amdgcn_raw_buffer_load_b32(rs, (lane + u * kWave) * 4, 0, 0);
    };

    // All of pixel d.pix is in the histogram: contract, check, emit, clear.
    auto complete = [&](const Run& d) {
        const int64_t pix = d.pix, count = d.pe - d.pb;
        int64_t count_total = count;
        if (acc) count_total = nacc[pix] + count;
        float sre[Q], sim[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) sre[q] = sim[q] = 0.f;
        if (count > 0) {
            // about the mean count per bin (any integer is exact; this one keeps the bins small)
            int dc = T % 1024 == 0 ? (int)((float)count * (1.0f / (float)T) + 0.5f) : 0;
            if (dc > kSafeChunk) dc = kSafeChunk;
            uint32_t bsum = 0;
            mfma_tiles<Q, MTT>(hist, s_wm, V, MT, lane, dc, sre, sim, bsum);   // leaves the histogram zero
            if (count > kSafeChunk && (int64_t)wave_sum_u32(bsum) != count) {
                // Some bin passed 255: redo the pixel in chunks that cannot (rare).
#pragma unroll
                for (int q = 0; q < Q; ++q) sre[q] = sim[q] = 0.f;
                for (int64_t c0 = d.pb; c0 < d.pe; c0 += kSafeChunk) {
                    const int64_t ce = c0 + kSafeChunk < d.pe ? c0 + kSafeChunk : d.pe;
                    for (int64_t i = c0 + lane; i < ce; i += kWave) {
                        int32_t x = stamps[i];
                        if ((uint32_t)x >= (uint32_t)T) x = fold_stamp(x, T);   // counted in the first pass
                        bin_add(hbase, (uint32_t)x, bin_one((uint32_t)x));
                    }
                    uint32_t unused = 0;
                    mfma_tiles<Q, MTT>(hist, s_wm, V, MT, lane, 0, sre, sim, unused);
                }
            }
        }
        // Sum over the four row groups g in the fixed order (g0 + g1) + (g2 + g3).  Swapping the
        // odd 16-lane rows of the real sums with the even rows of the imaginary sums and adding
        // leaves row 0 with re(g0 + g1), row 1 with im(g0 + g1), rows 2 and 3 with the same for
        // g2 + g3; swapping 32-lane halves and adding then gives rows 0 and 2 the real total and
        // rows 1 and 3 the imaginary one.  Lane (row, c) stores component row & 1 of harmonic
        // 16 q + c + 1, q = row >> 1 (with one set of harmonics, rows 2 and 3 store nothing).
        float v[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const auto p16 = __builtin_amdgcn_permlane16_swap(__float_as_uint(sre[q]), __float_as_uint(sim[q]), false,
                                                              false);
            const float u = __uint_as_float(p16[0]) + __uint_as_float(p16[1]);
            const auto p32 = __builtin_amdgcn_permlane32_swap(__float_as_uint(u), __float_as_uint(u), false, false);
            v[q] = __uint_as_float(p32[0]) + __uint_as_float(p32[1]);
        }
        const int c = lane & 15, comp = (lane >> 4) & 1, qs = lane >> 5;
        if (qs < Q) {
            const int l = 16 * qs + c + 1;
            const float val = Q == 1 ? v[0] : (qs == 0 ? v[0] : v[Q - 1]);
            if (l <= m) {
                const int64_t o = pix * m * 2 + 2 * (l - 1) + comp;
                // 1 / n in FP64: the reciprocal estimate and two Newton steps (n >= 1 is an
                // integer, so no special case arises)
                double inv = 0.0;
                if (count_total > 0) {
                    const double nd = (double)count_total;
                    double r = __builtin_amdgcn_rcp(nd);
                    r = fma(r, fma(-nd, r, 1.0), r);
                    r = fma(r, fma(-nd, r, 1.0), r);
                    inv = r;
                }
                if (acc) {
                    const double a = acc[o] + (double)val;
                    acc[o] = a;
                    z[o] = (float)(a * inv);
                } else {
                    z[o] = (float)((double)val * inv);
                }
            }
        }
        if (lane == 0) {
            if (acc) nacc[pix] = count_total;
            nout[pix] = (int32_t)(count_total > 0x7fffffff ? 0x7fffffff : count_total);
        }
    };
    auto consume = [&](const int32_t* v, const Run& d) {
        const int len = (int)(d.c1 - d.c0);                   // <= C
        // loads past the run's end read 0, which is in range: the largest stamp (as unsigned, so
        // negative ones count as large) decides whether this run needs the folding path
        uint32_t mx = 0;
#pragma unroll
        for (int u = 0; u < U; ++u) mx = max(mx, (uint32_t)v[u]);
        if (__builtin_amdgcn_ballot_w64(mx >= (uint32_t)T) == 0) {
            if (len == C) {                                   // full run: no guards, no branches
#pragma unroll
                for (int u = 0; u < U; ++u) bin_add(hbase, (uint32_t)v[u], bin_one((uint32_t)v[u]));
            } else {                                          // only the lanes inside the run add
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (lane + u * kWave < len) bin_add(hbase, (uint32_t)v[u], bin_one((uint32_t)v[u]));
            }
        } else {                                              // rare: stamps outside [0, T) are counted and folded
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (lane + u * kWave < len) {
                    int32_t x = v[u];
                    if ((uint32_t)x >= (uint32_t)T) {
                        ++bad_stamps;
                        x = fold_stamp(x, T);
                    }
                    bin_add(hbase, (uint32_t)x, bin_one((uint32_t)x));
                }
            }
        }
        if (d.last) complete(d);
    };

    Run dx = pixel_run(p0, uniform64(offsets[p0]), uniform64(offsets[p0 + 1]));
    Run dy = next(dx);
    int32_t X[U], Y[U];
    issue(X, dx);
    issue(Y, dy);
    // One exit, after both issues: every path into the loop head then has X's loads older than
    // Y's, so consuming X waits for X alone.
    while (true) {
        consume(X, dx);
        const Run dz = next(dy);
        issue(X, dz);
        if (dy.valid) consume(Y, dy);
        const Run dw = next(dz);
        issue(Y, dw);
        if (!dz.valid) break;
        dx = dz;
        dy = dw;
    }
    if (err) {
        bad_stamps = (int)wave_sum_u32((uint32_t)bad_stamps);
        if (lane == 0 && bad_stamps) atomicAdd(&err[0], bad_stamps);
        if (lane == 0 && bad_offsets) atomicAdd(&err[1], bad_offsets);
    }
}

template <int Q, int MTT, int U>
hipError_t launch_binned(const int32_t* stamps, int64_t N, const int64_t* offsets, int P, int T, int m,
                         const float2* table, float* z, int32_t* n, double* acc, int64_t* nacc, int32_t* err,
                         hipStream_t s) {
    int cus = 0, per_cu = 0;
    hipError_t st = current_device_cus(&cus);
    if (st != hipSuccess) return st;
    st = cached_occupancy<sketch_binned_kernel<Q, MTT, U>, kBinThreads>(&per_cu);
    if (st != hipSuccess) return st;
    const int64_t cap = (int64_t)cus * per_cu;
    const int64_t need = ((int64_t)P + kBinWaves - 1) / kBinWaves;
    const unsigned blocks = (unsigned)(need < cap ? need : cap);
    hipLaunchKernelGGL((sketch_binned_kernel<Q, MTT, U>), dim3(blocks), dim3(kBinThreads), 0, s, stamps, N, offsets,
                       P, T, m, table, z, n, acc, nacc, err);
    return hipGetLastError();
}

template <int Q, int MTT>
hipError_t launch_binned_u(const int32_t* stamps, int64_t N, const int64_t* offsets, int P, int T, int m,
                           const float2* table, float* z, int32_t* n, double* acc, int64_t* nacc, int32_t* err,
                           hipStream_t s) {
    // longer runs (more bytes in flight per wave) when pixels hold many photons
    if ((double)N >= 2048.0 * (double)P)
        return launch_binned<Q, MTT, 16>(stamps, N, offsets, P, T, m, table, z, n, acc, nacc, err, s);
    return launch_binned<Q, MTT, 8>(stamps, N, offsets, P, T, m, table, z, n, acc, nacc, err, s);
}

}  // namespace

hipError_t launch_sketch_binned(const int32_t* stamps, int64_t N, const int64_t* offsets, int P, int T, int m,
                                const float2* table, float* z, int32_t* n, double* acc, int64_t* nacc, int32_t* err,
                                hipStream_t s) {
    const bool q1 = m <= 16, t1 = T <= 4 * 16 * kRowBins;
    if (q1 && t1) return launch_binned_u<1, 4>(stamps, N, offsets, P, T, m, table, z, n, acc, nacc, err, s);
    if (q1) return launch_binned_u<1, 8>(stamps, N, offsets, P, T, m, table, z, n, acc, nacc, err, s);
    if (t1) return launch_binned_u<2, 4>(stamps, N, offsets, P, T, m, table, z, n, acc, nacc, err, s);
    return launch_binned_u<2, 8>(stamps, N, offsets, P, T, m, table, z, n, acc, nacc, err, s);
}

}  // namespace srt3d
