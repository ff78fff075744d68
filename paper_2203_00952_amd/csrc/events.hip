// Sketch of an arrival-order event stream (Section 2: the sketch is updated online as each
// photon arrives).  Events (pixel, stamp) come in any order; the sketch of a pixel is the sum
// over its events, so the stream is first grouped by pixel on the device and then sketched by
// the binned pass.  The binned pass sums exact integer histograms, so the order in which a
// pixel's stamps are placed does not change the result (a pixel whose bin passes 255 is
// recomputed in chunks of the stored order; its rounding then follows that order, within the
// same error bound).
//
// The grouping is a two-level counting sort whose counters all live in LDS and whose stores
// land in a small, moving window of cache lines, so that partial lines merge in L2 instead of
// travelling to memory one stamp at a time:
//   1. bucket counts: pixels are cut into NB buckets of W (a power of two) consecutive pixels;
//      each of G workgroups counts the events of its contiguous chunk of the stream per bucket;
//   2. per bucket, an exclusive scan over the chunks (the chunk's first slot in the bucket),
//      then one exclusive scan over the bucket totals (the bucket's first slot);
//   3. bucket scatter: every workgroup rereads its chunk and writes each event, packed as
//      (pixel within the bucket << 16 | stamp folded into [0, T)), at its bucket's next slot;
//   4. per bucket, one workgroup counts its events per pixel, writes the pixels' CSR offsets,
//      and places each stamp at its pixel's next slot.
// W is about sqrt(P), or P / 512 when that is smaller (two step-4 workgroups per CU), so that
// the keys of a step's tiles -- buckets in step 3, pixels in step 4 -- stay few enough for long
// runs per key.
#include <algorithm>

#include "common.hpp"

namespace srt3d {

namespace {

constexpr int kGrpThreads = 1024;                  // threads of the stream and bucket workgroups
constexpr int kGrpWaves = kGrpThreads / kWave;
constexpr int kUnroll = 4;                         // loads in flight per thread
constexpr int kMaxGroups = 512;                    // chunks of the stream
constexpr int kMaxBuckets = 32768;                 // LDS counters of steps 1 and 3 (128 KB)
constexpr int kMaxWidth = 32768;                   // LDS counters of step 4 (128 KB)
constexpr int kSmallTable = 1024;                  // the 4 KB variants

struct Plan {
    int64_t G;        // stream chunks (workgroups of steps 1 and 3)
    int64_t chunk;    // events per chunk
    int64_t NB;       // buckets
    int wbits;        // W = 1 << wbits pixels per bucket
};

int ceil_log2(int64_t v) {
    int b = 0;
    while (((int64_t)1 << b) < v) ++b;
    return b;
}

Plan make_plan(int64_t N, int P) {
    Plan q;
    q.G = std::max<int64_t>(1, std::min<int64_t>((N + 8191) / 8192, kMaxGroups));
    q.chunk = (N + q.G - 1) / q.G;
    const int root = (ceil_log2(P) + 1) / 2;                   // W ~ sqrt(P)
    const int spread = ceil_log2(((int64_t)P + 511) / 512);    // NB >= 512 where P allows
    q.wbits = std::min(root, spread);
    q.NB = ((int64_t)P + ((int64_t)1 << q.wbits) - 1) >> q.wbits;
    return q;
}

// Exclusive scan of one value per thread over a workgroup of THREADS threads; `s` holds
// THREADS / 64 + 1 entries.  `total` receives the workgroup's sum.
template <int THREADS>
__device__ int64_t group_exclusive(int64_t v, int64_t* s, int64_t& total) {
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    int64_t incl = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int64_t t = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += t;
    }
    if (lane == kWave - 1) s[wave] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int w = 0; w < THREADS / kWave; ++w) {
            const int64_t t = s[w];
            s[w] = run;
            run += t;
        }
        s[THREADS / kWave] = run;
    }
    __syncthreads();
    const int64_t ex = s[wave] + incl - v;
    total = s[THREADS / kWave];
    __syncthreads();
    return ex;
}

// Step 1.  cnt[b][g] = events of chunk g in bucket b; events outside [0, P) are counted in
// err[1].
template <int MAXNB>
__global__ __launch_bounds__(kGrpThreads) void bucket_count_kernel(const int32_t* __restrict__ pix, int64_t N, int P,
                                                                   Plan q, int32_t* __restrict__ cnt,
                                                                   int32_t* __restrict__ err) {
    __shared__ uint32_t s_cnt[MAXNB];
    const int g = blockIdx.x;
    const int64_t e0 = (int64_t)g * q.chunk, e1 = std::min<int64_t>(e0 + q.chunk, N);
    for (int b = threadIdx.x; b < q.NB; b += kGrpThreads) s_cnt[b] = 0;
    __syncthreads();
    int bad = 0;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kUnroll * kGrpThreads) {
        int32_t p[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t eu = e + (int64_t)u * kGrpThreads;
            p[u] = eu < e1 ? pix[eu] : 0;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if (e + (int64_t)u * kGrpThreads >= e1) continue;
            if ((uint32_t)p[u] < (uint32_t)P) atomicAdd(&s_cnt[p[u] >> q.wbits], 1u);
            else ++bad;
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < q.NB; b += kGrpThreads) cnt[(int64_t)b * q.G + g] = (int32_t)s_cnt[b];
    if (err) {
        for (int o = 32; o > 0; o >>= 1) bad += __shfl_xor(bad, o, kWave);
        if ((threadIdx.x & (kWave - 1)) == 0 && bad) atomicAdd(&err[1], bad);
    }
}

// Step 2a.  Row b of cnt becomes each chunk's first slot within bucket b; tot[b] = the
// bucket's events.  One workgroup of kMaxGroups threads per bucket.
__global__ __launch_bounds__(kMaxGroups) void bucket_chunk_scan_kernel(int32_t* __restrict__ cnt, Plan q,
                                                                       int64_t* __restrict__ tot) {
    __shared__ int64_t s[kMaxGroups / kWave + 1];
    const int64_t b = blockIdx.x;
    const int g = threadIdx.x;
    const int32_t c = g < q.G ? cnt[b * q.G + g] : 0;
    int64_t total;
    const int64_t ex = group_exclusive<kMaxGroups>(c, s, total);
    if (g < q.G) cnt[b * q.G + g] = (int32_t)ex;
    if (g == 0) tot[b] = total;
}

// Step 2b.  tot[0 .. NB) becomes each bucket's first slot and tot[NB] the events kept (an
// exclusive scan, one workgroup, kGrpThreads buckets at a time); offsets[0] = 0.
__global__ __launch_bounds__(kGrpThreads) void bucket_base_scan_kernel(int64_t* __restrict__ tot, int64_t NB,
                                                                       int64_t* __restrict__ offsets) {
    __shared__ int64_t s[kGrpWaves + 1];
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 <= NB; b0 += kGrpThreads) {
        const int64_t b = b0 + threadIdx.x;
        const int64_t v = b < NB ? tot[b] : 0;
        int64_t total;
        const int64_t ex = group_exclusive<kGrpThreads>(v, s, total);
        if (b <= NB) tot[b] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) offsets[0] = 0;
}

// Step 3.  Each event of chunk g at its bucket's next slot of tmp, packed as (pixel within the
// bucket << 16 | folded stamp); stamps outside [0, T) are counted in err[0].
template <int MAXNB>
__global__ __launch_bounds__(kGrpThreads) void bucket_scatter_kernel(const int32_t* __restrict__ pix,
                                                                     const int32_t* __restrict__ stamps, int64_t N,
                                                                     int P, int T, Plan q,
                                                                     const int32_t* __restrict__ first,
                                                                     const int64_t* __restrict__ base,
                                                                     uint32_t* __restrict__ tmp,
                                                                     int32_t* __restrict__ err) {
    __shared__ int32_t s_next[MAXNB];
    const int g = blockIdx.x;
    const int64_t e0 = (int64_t)g * q.chunk, e1 = std::min<int64_t>(e0 + q.chunk, N);
    for (int b = threadIdx.x; b < q.NB; b += kGrpThreads)
        s_next[b] = (int32_t)(base[b] + first[(int64_t)b * q.G + g]);
    __syncthreads();
    const uint32_t wmask = (1u << q.wbits) - 1u;
    int folded = 0;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kUnroll * kGrpThreads) {
        int32_t p[kUnroll], x[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t eu = e + (int64_t)u * kGrpThreads;
            p[u] = eu < e1 ? pix[eu] : -1;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
            if ((uint32_t)p[u] < (uint32_t)P) x[u] = stamps[e + (int64_t)u * kGrpThreads];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if ((uint32_t)p[u] >= (uint32_t)P) continue;           // past the chunk, or outside the frame
            int32_t xs = x[u];
            if ((uint32_t)xs >= (uint32_t)T) {
                xs = fold_stamp(xs, T);
                ++folded;
            }
            const int32_t pos = atomicAdd(&s_next[p[u] >> q.wbits], 1);
            if (pos >= 0 && (int64_t)pos < N) tmp[pos] = (((uint32_t)p[u] & wmask) << 16) | (uint32_t)xs;
        }
    }
    if (err) {
        for (int o = 32; o > 0; o >>= 1) folded += __shfl_xor(folded, o, kWave);
        if ((threadIdx.x & (kWave - 1)) == 0 && folded) atomicAdd(&err[0], folded);
    }
}

// Step 4.  Workgroup b takes bucket b's events tmp[base[b] .. base[b + 1]), counts them per
// pixel, writes offsets[p + 1] for the bucket's pixels, and places every stamp at its pixel's
// next slot of `sorted`.
template <int MAXW>
__global__ __launch_bounds__(kGrpThreads) void bucket_place_kernel(const uint32_t* __restrict__ tmp, int P, Plan q,
                                                                   const int64_t* __restrict__ base,
                                                                   int64_t* __restrict__ offsets,
                                                                   int32_t* __restrict__ sorted) {
    __shared__ int32_t s_pix[MAXW];
    __shared__ int64_t s_scan[kGrpWaves + 1];
    const int64_t b = blockIdx.x;
    const int64_t p0 = b << q.wbits;
    const int W = (int)std::min<int64_t>((int64_t)1 << q.wbits, (int64_t)P - p0);
    const int64_t a0 = base[b], a1 = base[b + 1];
    for (int i = threadIdx.x; i < W; i += kGrpThreads) s_pix[i] = 0;
    __syncthreads();
    for (int64_t e = a0 + threadIdx.x; e < a1; e += kUnroll * kGrpThreads) {
        uint32_t v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t eu = e + (int64_t)u * kGrpThreads;
            v[u] = eu < a1 ? tmp[eu] : 0xffffffffu;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const uint32_t i = v[u] >> 16;
            if (i < (uint32_t)W) atomicAdd(&s_pix[i], 1);
        }
    }
    __syncthreads();
    // pixel counts -> first slots (each thread a contiguous run of `per` pixels)
    const int per = (W + kGrpThreads - 1) / kGrpThreads;
    const int i0 = threadIdx.x * per, i1 = std::min(i0 + per, W);
    int64_t run = 0;
    for (int i = i0; i < i1; ++i) run += s_pix[i];
    int64_t total;
    int64_t slot = a0 + group_exclusive<kGrpThreads>(run, s_scan, total);
    for (int i = i0; i < i1; ++i) {
        const int32_t c = s_pix[i];
        s_pix[i] = (int32_t)slot;
        slot += c;
        offsets[p0 + i + 1] = slot;
    }
    __syncthreads();
    for (int64_t e = a0 + threadIdx.x; e < a1; e += kUnroll * kGrpThreads) {
        uint32_t v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t eu = e + (int64_t)u * kGrpThreads;
            v[u] = eu < a1 ? tmp[eu] : 0xffffffffu;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const uint32_t i = v[u] >> 16;
            if (i < (uint32_t)W) {
                const int32_t pos = atomicAdd(&s_pix[i], 1);
                if (pos >= a0 && pos < a1) sorted[pos] = (int32_t)(v[u] & 0xffffu);
            }
        }
    }
}

// Tiled forms of steps 3 and 4 for key ranges of at most kSmallTable (buckets, or pixels of a
// bucket).  A tile of kTile events is first grouped by key in LDS (ranks from LDS atomics, an
// exclusive scan of the tile's key counts), each key's run of the tile is given its next slots
// at once, and the grouped tile is then written with consecutive lanes on consecutive slots:
// a wave stores a few cache lines instead of one line per event.
constexpr int kTilePer = 8;                                   // events per thread and tile
constexpr int kTile = kGrpThreads * kTilePer;
constexpr bool kScatterPrefetch = false, kPlacePrefetch = true;
constexpr int kRsrcFlags = 0x00020000;                       // buffer descriptor word 3: raw dwords

struct TileLds {
    int32_t hist[kSmallTable];     // the tile's events per key, then their ranks' base
    int32_t off[kSmallTable];      // first index of each key's run within the grouped tile
    int32_t slot[kSmallTable];     // first output slot of each key's run
    int32_t next[kSmallTable];     // next output slot per key (this workgroup's cursors)
    uint32_t val[kTile];           // the grouped tile
    uint16_t key[kTile];
    int64_t scan[kGrpWaves + 1];
};

// Writes every event e of [e0, e1) whose decode(a[e], b[e], key, val) returns true at
// out[next[key]++], tile by tile (b is read only when NSRC == 2).  The tile's words come in by
// buffer loads (past the end they read 0 and are not decoded); with PREFETCH the next tile's
// loads are issued before this tile is grouped.  `next` (in t.next, nkeys <= kGrpThreads
// entries) must be set and visible before the call.
template <bool PREFETCH, int NSRC, class Decode>
__device__ void tiled_scatter(const uint32_t* a, const uint32_t* b, int64_t e0, int64_t e1, int nkeys, Decode decode,
                              uint32_t* __restrict__ out, int64_t out_end, TileLds& t) {
    const int k = threadIdx.x;                     // thread k owns key k
    const int vo = threadIdx.x * 4;
    uint32_t ra[kTilePer], rb[kTilePer];
    auto fetch = [&](int64_t t0) {
        const int n = (int)std::max<int64_t>(0, std::min<int64_t>(kTile, e1 - t0));
        const __amdgpu_buffer_rsrc_t sa =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t*>(a) + t0, (short)0, n * 4, kRsrcFlags);
#pragma unroll
        for (int u = 0; u < kTilePer; ++u) ra[u] = __builtin_amdgcn_raw_buffer_load_b32(sa, vo, u * kGrpThreads * 4, 0);
        if (NSRC == 2) {
            const __amdgpu_buffer_rsrc_t sb =
                __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t*>(b) + t0, (short)0, n * 4, kRsrcFlags);
#pragma unroll
            for (int u = 0; u < kTilePer; ++u)
                rb[u] = __builtin_amdgcn_raw_buffer_load_b32(sb, vo, u * kGrpThreads * 4, 0);
        }
    };
    if (k < nkeys) t.hist[k] = 0;
    if (PREFETCH) fetch(e0);
    __syncthreads();
    for (int64_t t0 = e0; t0 < e1; t0 += kTile) {
        if (!PREFETCH) fetch(t0);
        const int live = (int)std::min<int64_t>(e1 - t0, kTile);
        uint32_t key[kTilePer], val[kTilePer];
#pragma unroll
        for (int u = 0; u < kTilePer; ++u) {
            key[u] = 0xffffffffu;
            if (u * kGrpThreads + k < live && !decode(ra[u], rb[u], key[u], val[u])) key[u] = 0xffffffffu;
        }
        if (PREFETCH) fetch(t0 + kTile);
        int32_t rank[kTilePer];
#pragma unroll
        for (int u = 0; u < kTilePer; ++u)
            if (key[u] < (uint32_t)nkeys) rank[u] = atomicAdd(&t.hist[key[u]], 1);
        __syncthreads();
        const int32_t h = k < nkeys ? t.hist[k] : 0;
        if (k < nkeys) t.hist[k] = 0;              // for the next tile (its adds follow two barriers)
        int64_t total;
        const int32_t ex = (int32_t)group_exclusive<kGrpThreads>(h, t.scan, total);
        if (k < nkeys) {
            t.off[k] = ex;
            t.slot[k] = t.next[k];
            t.next[k] += h;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kTilePer; ++u)
            if (key[u] < (uint32_t)nkeys) {
                const int j = t.off[key[u]] + rank[u];
                t.val[j] = val[u];
                t.key[j] = (uint16_t)key[u];
            }
        __syncthreads();
        for (int j = threadIdx.x; j < (int)total; j += kGrpThreads) {
            const int kk = t.key[j];
            const int32_t pos = t.slot[kk] + (j - t.off[kk]);
            if (pos >= 0 && (int64_t)pos < out_end) out[pos] = t.val[j];
        }
    }
}

// Step 3, tiled (NB <= kSmallTable); two workgroups share a CU (64 KB of LDS each, at most 64
// registers).
__global__ __launch_bounds__(kGrpThreads) __attribute__((amdgpu_waves_per_eu(8))) void bucket_scatter_tiled_kernel(const int32_t* __restrict__ pix,
                                                                           const int32_t* __restrict__ stamps,
                                                                           int64_t N, int P, int T, Plan q,
                                                                           const int32_t* __restrict__ first,
                                                                           const int64_t* __restrict__ base,
                                                                           uint32_t* __restrict__ tmp,
                                                                           int32_t* __restrict__ err) {
    __shared__ TileLds t;
    const int g = blockIdx.x;
    const int64_t e0 = (int64_t)g * q.chunk, e1 = std::min<int64_t>(e0 + q.chunk, N);
    for (int b = threadIdx.x; b < q.NB; b += kGrpThreads) t.next[b] = (int32_t)(base[b] + first[(int64_t)b * q.G + g]);
    __syncthreads();
    const uint32_t wmask = (1u << q.wbits) - 1u;
    const int wbits = q.wbits;
    int folded = 0;
    auto decode = [&](uint32_t p, uint32_t x, uint32_t& key, uint32_t& val) {
        if (p >= (uint32_t)P) return false;
        if (x >= (uint32_t)T) {
            x = (uint32_t)fold_stamp((int32_t)x, T);
            ++folded;
        }
        key = p >> wbits;
        val = ((p & wmask) << 16) | x;
        return true;
    };
    tiled_scatter<kScatterPrefetch, 2>(reinterpret_cast<const uint32_t*>(pix), reinterpret_cast<const uint32_t*>(stamps),
                                       e0, e1, (int)q.NB, decode, tmp, N, t);
    if (err) {
        for (int o = 32; o > 0; o >>= 1) folded += __shfl_xor(folded, o, kWave);
        if ((threadIdx.x & (kWave - 1)) == 0 && folded) atomicAdd(&err[0], folded);
    }
}

// Step 4, tiled (W <= kSmallTable); two workgroups share a CU.
__global__ __launch_bounds__(kGrpThreads) __attribute__((amdgpu_waves_per_eu(8))) void bucket_place_tiled_kernel(const uint32_t* __restrict__ tmp, int P,
                                                                         Plan q, const int64_t* __restrict__ base,
                                                                         int64_t* __restrict__ offsets,
                                                                         int32_t* __restrict__ sorted) {
    __shared__ TileLds t;
    const int64_t b = blockIdx.x;
    const int64_t p0 = b << q.wbits;
    const int W = (int)std::min<int64_t>((int64_t)1 << q.wbits, (int64_t)P - p0);
    const int64_t a0 = base[b], a1 = base[b + 1];
    for (int i = threadIdx.x; i < W; i += kGrpThreads) t.hist[i] = 0;
    __syncthreads();
    for (int64_t e = a0 + threadIdx.x; e < a1; e += kUnroll * kGrpThreads) {
        uint32_t v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t eu = e + (int64_t)u * kGrpThreads;
            v[u] = eu < a1 ? tmp[eu] : 0xffffffffu;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const uint32_t i = v[u] >> 16;
            if (i < (uint32_t)W) atomicAdd(&t.hist[i], 1);
        }
    }
    __syncthreads();
    // W <= kGrpThreads: pixel i's count is thread i's
    const int i = threadIdx.x;
    const int32_t c = i < W ? t.hist[i] : 0;
    int64_t total;
    const int64_t ex = group_exclusive<kGrpThreads>(c, t.scan, total);
    if (i < W) {
        t.next[i] = (int32_t)(a0 + ex);
        offsets[p0 + i + 1] = a0 + ex + c;
    }
    __syncthreads();
    auto decode = [&](uint32_t v, uint32_t, uint32_t& key, uint32_t& val) {
        key = v >> 16;
        val = v & 0xffffu;
        return key < (uint32_t)W;
    };
    tiled_scatter<kPlacePrefetch, 1>(tmp, nullptr, a0, a1, W, decode, reinterpret_cast<uint32_t*>(sorted), a1, t);
}

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct Layout {
    int32_t* first;     // [NB][G] chunk counts, then first slots
    int64_t* base;      // [NB + 1] bucket totals, then first slots; base[NB] = events kept
    int64_t* offsets;   // [P + 1]
    uint32_t* tmp;      // [N] bucket-grouped packed events
    int32_t* sorted;    // [N] pixel-grouped stamps
    size_t bytes;
};

Layout layout(void* ws, int64_t N, int P, const Plan& q) {
    Layout L{};
    char* w = reinterpret_cast<char*>(ws);
    size_t o = 0;
    L.first = reinterpret_cast<int32_t*>(w + o);
    o += align256((size_t)q.NB * q.G * 4);
    L.base = reinterpret_cast<int64_t*>(w + o);
    o += align256((size_t)(q.NB + 1) * 8);
    L.offsets = reinterpret_cast<int64_t*>(w + o);
    o += align256((size_t)(P + 1) * 8);
    const size_t nN = (size_t)(N > 0 ? N : 1) * 4;
    L.tmp = reinterpret_cast<uint32_t*>(w + o);
    o += align256(nN);
    L.sorted = reinterpret_cast<int32_t*>(w + o);
    o += align256(nN);
    L.bytes = o;
    return L;
}

}  // namespace

size_t events_ws_bytes(int64_t N, int P) { return layout(nullptr, N, P, make_plan(N, P)).bytes; }

hipError_t launch_sketch_events(const int32_t* pix, const int32_t* stamps, int64_t N, int P, int T, int m,
                                const float2* table, float* z, int32_t* n, double* acc, int64_t* nacc, int32_t* err,
                                void* ws, hipStream_t s) {
    const Plan q = make_plan(N, P);
    const Layout L = layout(ws, N, P, q);
    const bool small_nb = q.NB <= kSmallTable, small_w = (1 << q.wbits) <= kSmallTable;
    hipError_t e;
    if (small_nb)
        hipLaunchKernelGGL(bucket_count_kernel<kSmallTable>, dim3((unsigned)q.G), dim3(kGrpThreads), 0, s, pix, N, P, q,
                           L.first, err);
    else
        hipLaunchKernelGGL(bucket_count_kernel<kMaxBuckets>, dim3((unsigned)q.G), dim3(kGrpThreads), 0, s, pix, N, P, q,
                           L.first, err);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(bucket_chunk_scan_kernel, dim3((unsigned)q.NB), dim3(kMaxGroups), 0, s, L.first, q, L.base);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(bucket_base_scan_kernel, dim3(1), dim3(kGrpThreads), 0, s, L.base, q.NB, L.offsets);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (small_nb)
        hipLaunchKernelGGL(bucket_scatter_tiled_kernel, dim3((unsigned)q.G), dim3(kGrpThreads), 0, s, pix, stamps, N, P,
                           T, q, L.first, L.base, L.tmp, err);
    else
        hipLaunchKernelGGL(bucket_scatter_kernel<kMaxBuckets>, dim3((unsigned)q.G), dim3(kGrpThreads), 0, s, pix, stamps,
                           N, P, T, q, L.first, L.base, L.tmp, err);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (small_w)
        hipLaunchKernelGGL(bucket_place_tiled_kernel, dim3((unsigned)q.NB), dim3(kGrpThreads), 0, s, L.tmp, P, q, L.base,
                           L.offsets, L.sorted);
    else
        hipLaunchKernelGGL(bucket_place_kernel<kMaxWidth>, dim3((unsigned)q.NB), dim3(kGrpThreads), 0, s, L.tmp, P, q,
                           L.base, L.offsets, L.sorted);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // the grouped stream is an ordinary CSR frame of at most N stamps, already folded into [0, T)
    if (m <= 32) return launch_sketch_binned(L.sorted, N, L.offsets, P, T, m, table, z, n, acc, nacc, err, s);
    return launch_sketch_photons(L.sorted, N, L.offsets, P, T, m, table, z, n, acc, nacc, err, s);
}

}  // namespace srt3d
