// Sketched RT3D iteration, Section 3: eq. (8) with W = I, alternated with point-cloud and
// intensity denoising (RT3D's plug-and-play scheme).
//
//   frame_constants   hhat_l = sum_i h_i exp(i w_l (i - o)) / sum h (eq. 4) in FP64, the sums
//                     sum |hhat|^2 and sum w^2 |hhat|^2, the impulse-response spread and the
//                     depth gate; one workgroup, one wave per harmonic subset
//   init              greedy sketched matched filter on the grid tau = 0, s, 2s, ...: the filter
//                     over all pixels and grid points is a real matrix product on the FP32 matrix
//                     cores (16 pixels per wave) with the argmax in its epilogue; also the
//                     per-workgroup maximum photon count
//   step_sizes        frame maximum photon count and the two step sizes
//   data_step         per pixel: residual e = Phi - z, depth step, residual at the new depths,
//                     intensity step, projection onto {alpha >= 0, sum alpha <= 1} (eq. 1);
//                     the workgroup's sketches are staged in LDS by coalesced loads
//   depth_denoise     per point: weighted least-squares height-field fit over a gated
//                     (2R+1)^2 window (4x4 Cholesky, plane and mean fallbacks); 16x16 pixel
//                     tiles with an R-pixel halo in LDS
//   intensity_denoise per point: gated weighted mean of n * alpha, removal below r_min
//   finalize          background n * max(0, 1 - sum alpha) / T with a box filter, output
//                     points sorted by depth
// Every kernel writes only its own pixels; denoisers read one buffer and write the other.
#include "common.hpp"

namespace srt3d {

constexpr float kCholEps = 1e-5f;    // pivot <= kCholEps * trace counts as singular
constexpr int kTile = 16;            // denoiser tile edge (pixels)
constexpr int kInitBlocksMax = 4096; // init workgroups at most; also the number of photon-count partials

struct IterArgs {
    int rows, cols, P, T, m, K, R, Rb;
    float lambda_z, r_min;
    float invT, twoinvT;    // 1 / T and 2 / T, correctly rounded (host division)
};

// ----------------------------------------------------------------------------- helpers
// Map t onto [0, T).  Steps move t by much less than T, so one add or subtract is the usual
// path; FP32 rounding of t + T onto T is mapped to 0.
__device__ __forceinline__ float wrap_t(float t, float Tf) {
    if (t < 0.f) t += Tf;
    else if (t >= Tf) t -= Tf;
    if (!(t >= 0.f && t < Tf)) {
        t = t - Tf * floorf(t / Tf);
        if (!(t >= 0.f && t < Tf)) t = 0.f;
    }
    return t;
}

// Signed circular difference of d = a - b, a and b in [0, T): d - T * round(d / T), which is d
// reduced to [-T/2, T/2] (the two ends of that range only differ at |d| = T/2, far outside
// every depth gate).
__device__ __forceinline__ float circ_diff(float d, float Tf, float invT) {
    return fmaf(-Tf, rintf(d * invT), d);
}

// a mod T for 0 <= a < 2^24 (exact: the float quotient is off by at most one).
__device__ __forceinline__ int mod_small(int a, int T, float invT) {
    const int q = (int)((float)a * invT);
    int r = a - q * T;
    if (r < 0) r += T;
    else if (r >= T) r -= T;
    return r;
}

// exp(i 2 pi k / T) for an integer phase k in [0, T).
__device__ __forceinline__ float2 phasor_int(int k, float twoinvT) {
    float s, c;
    sincospif((float)k * twoinvT, &s, &c);
    return make_float2(c, s);
}

// exp(i w_l t), t in [0, T): the phase (l t) mod T is reduced through the integer part of t,
// so the angle reaches the hardware sine and cosine (v_sin_f32 / v_cos_f32, argument in turns)
// as a fraction of a turn in [0, 1 + l / T).  Measured against FP64 on this device over 5e5 such
// phases: at most 1.2e-7 absolute error (about 2 ulp of 1), the size of the FP32 rounding of the
// turn itself.
__device__ __forceinline__ float2 phasor(int l, float t, int T, float invT, float twoinvT) {
    const float ft = floorf(t);
    const int k = mod_small(l * (int)ft, T, invT);
    const float ph = (float)k + (float)l * (t - ft);
    const float turn = ph * (0.5f * twoinvT);
    return make_float2(__builtin_amdgcn_cosf(turn), __builtin_amdgcn_sinf(turn));
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Euclidean projection of the active entries onto {a >= 0, sum a <= 1} (eq. 1 constraint).
template <int K>
__device__ __forceinline__ void project_capped_simplex(float* a, const bool* act) {
    float w[K], sum = 0.f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        w[k] = act[k] ? fmaxf(a[k], 0.f) : 0.f;
        sum += w[k];
    }
    if (!(sum > 1.f)) {
#pragma unroll
        for (int k = 0; k < K; ++k) a[k] = w[k];
        return;
    }
    float u[K];
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (act[k]) u[cnt++] = a[k];
    for (int i = 1; i < cnt; ++i)                // descending insertion sort, cnt <= 3
        for (int j = i; j > 0 && u[j] > u[j - 1]; --j) {
            const float tmp = u[j];
            u[j] = u[j - 1];
            u[j - 1] = tmp;
        }
    float cs = 0.f, theta = 0.f;
    for (int j = 0; j < cnt; ++j) {
        cs += u[j];
        const float th = (cs - 1.f) / (float)(j + 1);
        if (u[j] - th > 0.f) theta = th;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) a[k] = act[k] ? fmaxf(a[k] - theta, 0.f) : 0.f;
}

__device__ __forceinline__ double wave_sum_d(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ----------------------------------------------------------------------------- frame constants
// scal: [0] n_max, [1] gamma_t, [2] gamma_alpha, [3] tau_z, [4] sum |hhat|^2, [5] sum w^2 |hhat|^2
// One workgroup; the harmonics are spread over its waves (one or two each at 16 waves).
__device__ void frame_constants_block(const double* __restrict__ irf, int irf_len, int origin, int T, int m,
                                      float tau_z_param, float* __restrict__ hhat_out, float* __restrict__ scal) {
    __shared__ double s_e2[SRT3D_MAX_M_RECON], s_et[SRT3D_MAX_M_RECON];
    __shared__ double s_mom[3];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // moments of the impulse response (wave 0): sum h, sum h lag, sum h lag^2
    if (wv == 0) {
        double h0 = 0, h1 = 0, h2 = 0;
        for (int i = lane; i < irf_len; i += 64) {
            const double lag = (double)(i - origin);
            h0 += irf[i];
            h1 += irf[i] * lag;
            h2 += irf[i] * lag * lag;
        }
        h0 = wave_sum_d(h0);
        h1 = wave_sum_d(h1);
        h2 = wave_sum_d(h2);
        if (lane == 0) {
            s_mom[0] = h0;
            s_mom[1] = h1;
            s_mom[2] = h2;
        }
    }
    __syncthreads();
    const double H = s_mom[0];
    // hhat_l, harmonics distributed over the waves, lags over the lanes
    for (int l = 1 + wv; l <= m; l += blockDim.x >> 6) {
        double re = 0, im = 0;
        for (int i = lane; i < irf_len; i += 64) {
            int k = (int)(((int64_t)l * (i - origin)) % T);
            if (k < 0) k += T;
            double s, c;
            sincospi(2.0 * (double)k / (double)T, &s, &c);
            re += irf[i] * c;
            im += irf[i] * s;
        }
        re = wave_sum_d(re) / H;
        im = wave_sum_d(im) / H;
        if (lane == 0) {
            hhat_out[2 * (l - 1)] = (float)re;
            hhat_out[2 * (l - 1) + 1] = (float)im;
            const double w = 2.0 * M_PI * (double)l / (double)T;
            s_e2[l - 1] = re * re + im * im;
            s_et[l - 1] = w * w * (re * re + im * im);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double e2 = 0, et = 0;
        for (int l = 0; l < m; ++l) {
            e2 += s_e2[l];
            et += s_et[l];
        }
        const double mu = s_mom[1] / H;
        const double var = s_mom[2] / H - mu * mu;
        const double sigma = sqrt(var > 0 ? var : 0.0);
        scal[3] = tau_z_param > 0 ? tau_z_param : (float)(3.0 * sigma);
        scal[4] = (float)e2;
        scal[5] = (float)et;
        scal[6] = 0.f;
        scal[7] = 0.f;
    }
}

// ----------------------------------------------------------------------------- init
// c(tau_g) = Re sum_l conj(hhat_l) w_l exp(-i w_l tau_g) over all pixels and grid points is the
// real product C = Y E: Y[p][k] holds the real (k even) and imaginary (k odd) parts of
// conj(hhat_l) w_l for k = 2(l-1) + {0, 1}, and E[k][g] = cos / sin(w_l tau_g) at the exact phase
// (l tau_g) mod T.  One wave takes 16 pixels: its Y rows stay in registers as the A operand of
// v_mfma_f32_16x16x4_f32, E is read as prebuilt B-operand fragments, and the argmax of every row
// is folded into the epilogue of each 16-column tile (larger c, then smaller tau).  Each greedy
// pick removes its atom: either from the working sketch w, after which the product is redone, or
// (RHO) from the kept correlation directly, by the atom's autocorrelation.
typedef float v4f __attribute__((ext_vector_type(4)));

// EB[(nt * KS + ks) * 64 + lane] = E[4 ks + lane / 16][16 nt + lane % 16], zero outside 2m x G.
__device__ __forceinline__ void grid_table_entry(int idx, int T, int m, int stride, int G, int KS, int NT,
                                                 float* __restrict__ EB) {
    if (idx >= NT * KS * 64) return;
    const int lane = idx & 63, ks = (idx >> 6) % KS, nt = (idx >> 6) / KS;
    const int k = 4 * ks + (lane >> 4), g = 16 * nt + (lane & 15);
    double v = 0.0;
    if (k < 2 * m && g < G) {
        const int64_t ph = ((int64_t)(k / 2 + 1) * ((int64_t)g * stride)) % T;
        double sn, cs;
        sincospi(2.0 * (double)ph / (double)T, &sn, &cs);
        v = (k & 1) ? sn : cs;
    }
    EB[idx] = (float)v;
}

// Correlation of the atom with itself at grid lag d (d = 0 .. G - 1, lag d * stride):
// rho[d] = Re sum_l conj(hhat_l) hhat_l e^{-i w_l d stride} = sum_l |hhat_l|^2 cos(w_l d stride), even
// in d.  Removing the atom a hhat_l e^{i w_l tau_k} from the working sketch lowers the grid
// correlation at tau by exactly a rho(tau - tau_k), so the greedy picks after the first update
// the correlation instead of recomputing it.  Exact integer phase, FP64 sum of the FP32 hhat
// the correlation itself uses, stored as FP32; lags past the grid are 0 (read only with a zero
// amplitude).  cos(w_l lag) follows from the first harmonic's phasor by an FP64 complex
// recurrence (m - 1 products: rounding near 1e-15, far below the FP32 result).
__device__ __forceinline__ float rho_entry(const float* __restrict__ hhat, int d, int T, int m, int stride, int G) {
    double acc = 0.0;
    if (d < G) {
        const int64_t lag = ((int64_t)d * stride) % T;
        double s1, c1;
        sincospi(2.0 * (double)lag / (double)T, &s1, &c1);
        double c = c1, s = s1;
        for (int l = 1; l <= m; ++l) {
            const double hr = hhat[2 * (l - 1)], hi = hhat[2 * (l - 1) + 1];
            acc += (hr * hr + hi * hi) * c;
            const double cn = c * c1 - s * s1;
            s = c * s1 + s * c1;
            c = cn;
        }
    }
    return (float)acc;
}

// Everything a frame needs before init, in one launch: workgroup 0 computes the frame constants
// and (GP > 0) tabulates rho on GP lags; the next `tb` workgroups build the grid table for init's
// matrix product; the rest each write the largest photon count of one stretch of 1024 cpt pixels.
constexpr int kSetupThreads = 1024;
__global__ __launch_bounds__(kSetupThreads) void frame_setup_kernel(
    const double* __restrict__ irf, int irf_len, int origin, int T, int m, float tau_z_param, int stride, int G,
    int KS, int NT, int GP, int tb, const int32_t* __restrict__ n, int P, int cpt, float* __restrict__ hhat,
    float* __restrict__ scal, float* __restrict__ EB, float* __restrict__ rho, int* __restrict__ nmax_part) {
    if (blockIdx.x > tb) {
        __shared__ int s_w[kSetupThreads / 64];
        const int b = blockIdx.x - tb - 1;
        const int64_t base = (int64_t)b * kSetupThreads * cpt + threadIdx.x;
        int v = 0;
        // 16 counts per round, all loaded (clamped into the frame) before the first is used
        constexpr int U = 16;
        for (int i0 = 0; i0 < cpt; i0 += U) {
            int c[U];
#pragma unroll
            for (int u = 0; u < U; ++u) c[u] = n[min(base + (int64_t)(i0 + u) * kSetupThreads, (int64_t)P - 1)];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (i0 + u < cpt && base + (int64_t)(i0 + u) * kSetupThreads < P) v = max(v, c[u]);
        }
        for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
        if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int i = 1; i < kSetupThreads / 64; ++i) v = max(v, s_w[i]);
            nmax_part[b] = v;
        }
        return;
    }
    if (blockIdx.x > 0) {
        grid_table_entry((blockIdx.x - 1) * kSetupThreads + threadIdx.x, T, m, stride, G, KS, NT, EB);
        return;
    }
    frame_constants_block(irf, irf_len, origin, T, m, tau_z_param, hhat, scal);
    if (GP > 0) {
        __syncthreads();                    // hhat written by this workgroup
        for (int d = threadIdx.x; d < GP; d += kSetupThreads) rho[d] = rho_entry(hhat, d, T, m, stride, G);
    }
}

// n_max and the step sizes of eq. (8).
__device__ __forceinline__ void step_sizes(int nmax_i, int K, float eta_t, float eta_a, const float* __restrict__ scal,
                                           float& gam_t, float& gam_a) {
    const double nmax = (double)nmax_i;
    const double e2 = (double)scal[4], et = (double)scal[5];
    gam_t = nmax > 0 ? (float)((double)eta_t / (2.0 * nmax * et)) : 0.f;
    gam_a = nmax > 0 ? (float)((double)eta_a / (2.0 * nmax * K * e2)) : 0.f;
}
__device__ __forceinline__ void step_sizes_store(int nmax_i, int K, float eta_t, float eta_a, float* __restrict__ scal) {
    float gam_t, gam_a;
    step_sizes(nmax_i, K, eta_t, eta_a, scal, gam_t, gam_a);
    scal[0] = (float)(double)nmax_i;
    scal[1] = gam_t;
    scal[2] = gam_a;
}

// The first data step of an iteration, fused into init (defined with the data step below).
template <int K>
__device__ void init_data_step(const IterArgs& A, const float* __restrict__ z, const float* __restrict__ hhat,
                               int grp, int lane, int np, const float (&t_r)[K], const float (&a_r)[K],
                               const int (&on_r)[K], float gam_t, float gam_a, float* __restrict__ t_out,
                               float* __restrict__ a_out, uint8_t* __restrict__ act_out);

// RHO: the first pick's correlation stays in LDS (NT <= KSMAX column tiles, 16 bytes per lane and
// tile) and the later picks update it with rho; otherwise every pick recomputes it from the
// updated working sketch.
// Argmax step across lanes: take the partner's entry if its value is larger, or equal with a
// smaller grid index (a total order, so any pairing sequence gives the same winner).
template <int CTRL>
__device__ __forceinline__ void argmax_dpp(float& best, int& bestg) {
    const float ob = __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, best), CTRL, 0xf, 0xf,
                                                                       false));
    const int og = __builtin_amdgcn_mov_dpp(bestg, CTRL, 0xf, 0xf, false);
    if (ob > best || (ob == best && og < bestg)) {
        best = ob;
        bestg = og;
    }
}

// EBL: the grid table is first copied to LDS (dynamic shared memory of NT KS 64 floats), so
// the B operands of every column tile are LDS reads instead of L2 round trips.
// Workgroup size: 1024 threads when the grid table is copied to LDS without the per-wave
// correlation tiles (one copy per 16 waves instead of per 4, so fewer workgroups read the same
// table lines from L2 at the same moment), else 256.
// With the fused data step (DS) and several points, 1024 threads would leave too few registers.
template <bool EBL, bool RHO, int KSMAX, int K, bool DS>
constexpr int kInitThreads = (EBL && !RHO && KSMAX <= 8 && (!DS || K == 1)) ? 1024 : 256;

// DS: the iteration's first data step follows in the same launch (srt3d_reconstruct), on the
// state the plain form writes, with the step sizes every wave derives as init's first workgroup
// stores them; the result is that of init followed by the stand-alone data step, bit for bit.
template <int K, int KSMAX, bool RHO, bool EBL, bool DS>
__global__ __launch_bounds__((kInitThreads<EBL, RHO, KSMAX, K, DS>)) void init_kernel(const float* __restrict__ z, const int32_t* __restrict__ n,
                                                   const float* __restrict__ hhat, float* __restrict__ scal,
                                                   const float* __restrict__ EB, const float* __restrict__ rho, int P,
                                                   int T, int m, int stride, int G, int KS, int NT, float r_min,
                                                   float* __restrict__ t_out, float* __restrict__ a_out,
                                                   uint8_t* __restrict__ act_out,
                                                   const int* __restrict__ nmax_part, int nparts, float eta_t,
                                                   float eta_a, const IterArgs A) {
    __shared__ float s_rho[RHO ? 16 * KSMAX : 1];
    __shared__ v4f s_C[RHO ? 4 * KSMAX * 64 : 1];     // [wave][column tile][lane]
    extern __shared__ float4 s_eb4[];                 // EBL: the grid table
    const float* s_eb = reinterpret_cast<const float*>(s_eb4);
    if constexpr (RHO) {
        for (int i = threadIdx.x; i < 16 * KSMAX; i += blockDim.x) s_rho[i] = i < 16 * NT ? rho[i] : 0.f;
        __syncthreads();
    }
    if constexpr (EBL) {
        // 16-byte pieces (the table starts 16-byte aligned and holds a multiple of 64 floats),
        // eight rounds of loads in flight per thread before the first store
        const float4* eb4 = reinterpret_cast<const float4*>(EB);
        const int n4 = NT * KS * 16;
        constexpr int U = 8;
        for (int b = threadIdx.x; b < n4; b += U * blockDim.x) {
            float4 v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = eb4[min(b + u * (int)blockDim.x, n4 - 1)];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (b + u * (int)blockDim.x < n4) s_eb4[b + u * blockDim.x] = v[u];
        }
        __syncthreads();
    }
    // B fragment ks of column tile nt for this lane
    auto ebv = [&](int nt, int ks, int lane_) -> float {
        if constexpr (EBL) return s_eb[(nt * KS + ks) * 64 + lane_];
        else return EB[(int64_t)(nt * KS + ks) * 64 + lane_];
    };
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r = lane & 15, kq = lane >> 4;          // A row (pixel) / k quarter of this lane
    const float e2 = scal[4], invT = 1.0f / (float)T, twoinvT = 2.0f / (float)T;
    const int groups = (P + 15) / 16;
    const int waves_total = gridDim.x * (blockDim.x >> 6);
    const int l_first = kq / 2 + 1;                    // harmonic of ks = 0; +2 per ks
    // Loads are unconditional (clamped indices, unused entries zeroed afterwards), so that all of
    // a group's are in flight together rather than each waited for under its own branch.
    float gam_t = 0.f, gam_a = 0.f;                    // DS: the step sizes of eq. (8)
    if constexpr (DS) {
        int v = 0;
        for (int i = lane; i < nparts; i += 64) v = max(v, nmax_part[i]);
        for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
        step_sizes(v, K, eta_t, eta_a, scal, gam_t, gam_a);
    }
    float2 hl[KSMAX];
#pragma unroll
    for (int ks = 0; ks < KSMAX; ++ks) {
        const int k = 4 * ks + kq;
        const float2 h = reinterpret_cast<const float2*>(hhat)[min(k / 2, m - 1)];
        hl[ks] = (ks < KS && k < 2 * m) ? h : make_float2(0.f, 0.f);
    }
    for (int grp = blockIdx.x * (blockDim.x >> 6) + wv; grp < groups; grp += waves_total) {
        const int prow = grp * 16 + r;
        const bool rv = prow < P;
        const float2* zrow = reinterpret_cast<const float2*>(z + (int64_t)(rv ? prow : P - 1) * 2 * m);
        float2 w[KSMAX];
#pragma unroll
        for (int ks = 0; ks < KSMAX; ++ks) {
            const int k = 4 * ks + kq;
            const float2 v = zrow[min(k / 2, m - 1)];
            w[ks] = (rv && ks < KS && k < 2 * m) ? v : make_float2(0.f, 0.f);
        }
        const int np_raw = n[rv ? prow : P - 1];
        const int np = rv ? np_raw : 0;
        int tau_row[K][4];                              // picks of C rows 4 kq + i
        int tau_mine[K];                                // picks of A row r
        float amp_mine[K];
        v4f* Cw = s_C + (RHO ? wv * KSMAX * 64 + lane : 0);   // RHO: this lane's correlation, tile nt at Cw[64 nt]
        float amp_row[4] = {0.f, 0.f, 0.f, 0.f};       // RHO: the previous pick's amplitude per C row
#pragma unroll
        for (int k = 0; k < K; ++k) {
            float ya[KSMAX];
#pragma unroll
            for (int ks = 0; ks < KSMAX; ++ks) {        // conj(hhat) w, real part for even k
                const float re = hl[ks].x * w[ks].x + hl[ks].y * w[ks].y;
                const float im = hl[ks].x * w[ks].y - hl[ks].y * w[ks].x;
                ya[ks] = (kq & 1) ? im : re;
            }
            float best[4];
            int bestg[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                best[i] = -INFINITY;
                bestg[i] = 0x7fffffff;
            }
            // two column tiles per pass: two independent accumulation chains
            auto scan = [&](const v4f& acc, int nt) {
                const int g = 16 * nt + r;              // column of this lane's C entries
                const int tg = g * stride;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    bool excl = g >= G;
#pragma unroll
                    for (int j = 0; j < k; ++j) {
                        int d = tg - tau_row[j][i];
                        d = d < 0 ? -d : d;
                        d = min(d, T - d);
                        excl |= (int64_t)d * m < (int64_t)T;
                    }
                    if (!excl && acc[i] > best[i]) {     // g grows with nt: ties keep the smaller
                        best[i] = acc[i];
                        bestg[i] = g;
                    }
                }
            };
            if (RHO && k > 0) {
                // remove the previous pick of each row: c(g) -= a rho(|g - g_prev|)
                for (int nt = 0; nt < NT; ++nt) {
                    v4f c = Cw[64 * nt];
                    const int g = 16 * nt + r;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int d = g - tau_row[k - 1][i] / stride;
                        c[i] -= amp_row[i] * s_rho[d < 0 ? -d : d];
                    }
                    Cw[64 * nt] = c;
                    scan(c, nt);
                }
            } else {
                for (int nt = 0; nt < NT; nt += 2) {
                    v4f acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
                    if (nt + 1 < NT) {
#pragma unroll
                        for (int ks = 0; ks < KSMAX; ++ks)
                            if (ks < KS) {
                                acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(ya[ks], ebv(nt, ks, lane), acc0, 0, 0, 0);
                                acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(ya[ks], ebv(nt + 1, ks, lane), acc1, 0, 0,
                                                                            0);
                            }
                        scan(acc0, nt);
                        scan(acc1, nt + 1);
                        if (RHO) {
                            Cw[64 * nt] = acc0;
                            Cw[64 * (nt + 1)] = acc1;
                        }
                    } else {
#pragma unroll
                        for (int ks = 0; ks < KSMAX; ++ks)
                            if (ks < KS) acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(ya[ks], ebv(nt, ks, lane), acc0, 0, 0, 0);
                        scan(acc0, nt);
                        if (RHO) Cw[64 * nt] = acc0;
                    }
                }
            }
            // argmax over the 16 lanes of each row (DPP: pairs within quads, then the two quads of
            // each half row, then the two half rows)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                argmax_dpp<0xB1>(best[i], bestg[i]);    // quad_perm 1, 0, 3, 2
                argmax_dpp<0x4E>(best[i], bestg[i]);    // quad_perm 2, 3, 0, 1
                argmax_dpp<0x141>(best[i], bestg[i]);   // row_half_mirror
                argmax_dpp<0x140>(best[i], bestg[i]);   // row_mirror
            }
            float arow[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const bool none = bestg[i] == 0x7fffffff;
                arow[i] = none ? 0.f : fmaxf(0.f, best[i] / e2);
                tau_row[k][i] = none ? 0 : bestg[i] * stride;
                amp_row[i] = arow[i];
            }
            // this lane's A row r: its pick sits in lanes 16 (r / 4) .. + 15, element r % 4
            const int src = (r >> 2) * 16;
            float a_sel = 0.f;
            int t_sel = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float av = __shfl(arow[i], src, 64);
                const int tv = __shfl(tau_row[k][i], src, 64);
                if ((r & 3) == i) {
                    a_sel = av;
                    t_sel = tv;
                }
            }
            amp_mine[k] = a_sel;
            tau_mine[k] = t_sel;
            if (!RHO && k + 1 < K) {                    // w_l -= a hhat_l exp(i w_l tau)
                float2 u = phasor_int(mod_small(l_first * t_sel, T, invT), twoinvT);
                const float2 step = phasor_int(mod_small(2 * t_sel, T, invT), twoinvT);
#pragma unroll
                for (int ks = 0; ks < KSMAX; ++ks) {
                    const float2 gv = cmul(hl[ks], u);
                    w[ks].x -= a_sel * gv.x;
                    w[ks].y -= a_sel * gv.y;
                    u = cmul(u, step);
                }
            }
        }
        if constexpr (!DS) {
            if (kq == 0 && rv) {
                bool all[K];
#pragma unroll
                for (int k = 0; k < K; ++k) all[k] = true;
                project_capped_simplex<K>(amp_mine, all);
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const bool on = np > 0 && (float)np * amp_mine[k] >= r_min;
                    t_out[(int64_t)prow * K + k] = (float)tau_mine[k];
                    a_out[(int64_t)prow * K + k] = on ? amp_mine[k] : 0.f;
                    act_out[(int64_t)prow * K + k] = on ? 1 : 0;
                }
            }
        } else {
            // every lane forms its row's state (the four lanes of a row hold the same picks)
            bool all[K];
#pragma unroll
            for (int k = 0; k < K; ++k) all[k] = true;
            project_capped_simplex<K>(amp_mine, all);
            float t_r[K], a_r[K];
            int on_r[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const bool on = np > 0 && (float)np * amp_mine[k] >= r_min;
                t_r[k] = (float)tau_mine[k];
                a_r[k] = on ? amp_mine[k] : 0.f;
                on_r[k] = on ? 1 : 0;
            }
            init_data_step<K>(A, z, hhat, grp, lane, np, t_r, a_r, on_r, gam_t, gam_a, t_out, a_out, act_out);
        }
    }
    if (blockIdx.x == 0 && wv == 0) {                  // n_max and the step sizes (eq. 8)
        int v = 0;
        for (int i = lane; i < nparts; i += 64) v = max(v, nmax_part[i]);
        for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
        if (lane == 0) step_sizes_store(v, K, eta_t, eta_a, scal);
    }
}


// ----------------------------------------------------------------------------- data step
// Moves between the four lanes of a pixel (an aligned quad, always active together): DPP quad
// permutes, one VALU instruction each instead of an LDS round trip, the same values.
template <int CTRL>
__device__ __forceinline__ float quad_dpp(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}
__device__ __forceinline__ float quad_xor1(float v) { return quad_dpp<0xB1>(v); }    // lanes 1, 0, 3, 2
__device__ __forceinline__ float quad_xor2(float v) { return quad_dpp<0x4E>(v); }    // lanes 2, 3, 0, 1
__device__ __forceinline__ float quad_first(float v) { return quad_dpp<0x00>(v); }   // lane 0 of the quad

// Four lanes per pixel: lane `sub` takes harmonics l in (lo, hi], a contiguous quarter of 1..m,
// reads its slice of the pixel's sketch directly (the four lanes cover the row contiguously)
// and keeps a phasor recurrence re-anchored at the start of its slice and every 8 harmonics.
// Partial gradient sums are combined over the four lanes, which then apply identical updates.
constexpr int kLanesPerPixel = 4;
constexpr int kMaxSlice = (SRT3D_MAX_M_RECON + kLanesPerPixel - 1) / kLanesPerPixel;   // harmonics per lane
constexpr int kPrefetchSlice = 8;   // slices of up to 8 harmonics (m <= 32) are prefetched into registers

// Where a lane's sketch values come from: the pixel's row in global memory, or registers filled
// earlier (the fused iteration prefetches them at its start).  Same values either way.
struct GlobalSketch {
    const float2* zp;    // the pixel's sketch row
    const float2* hp;    // the IRF spectrum
    __device__ __forceinline__ float2 z(int l0, int) const { return zp[l0]; }
    __device__ __forceinline__ float2 h(int l0, int) const { return hp[l0]; }
};
template <int MS>
struct RegSketch {
    const float2* zr;    // zr[j] = z_{lo + j + 1}, j < hi - lo <= MS (registers after inlining)
    const float2* hs;    // the IRF spectrum in LDS
    __device__ __forceinline__ float2 z(int, int j) const { return zr[j]; }
    __device__ __forceinline__ float2 h(int l0, int) const { return hs[l0]; }
};
template <int MS>
struct RegSketchH {
    const float2* zr;    // zr[j] = z_{lo + j + 1} and hr[j] = hhat_{lo + j + 1}, j < hi - lo <= MS
    const float2* hr;
    __device__ __forceinline__ float2 z(int, int j) const { return zr[j]; }
    __device__ __forceinline__ float2 h(int, int j) const { return hr[j]; }
};

template <int K, int MS, class Src>
__device__ __forceinline__ void residual_pass(const Src& src, int lo, int hi, int T, float invT, float twoinvT,
                                              const float* tk, const float* ak, const bool* on, float* gsum,
                                              bool depth) {
    // each lane anchors at the first harmonic of its slice; lane 0 of the pixel's group holds
    // harmonic 1, whose phasor drives everyone's recurrence
    float2 u[K], u1[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        u[k] = on[k] ? phasor(lo + 1, tk[k], T, invT, twoinvT) : make_float2(1.f, 0.f);
        u1[k].x = quad_first(u[k].x);
        u1[k].y = quad_first(u[k].y);
    }
    const float w1 = 6.283185307179586f * invT;
    // harmonic l = l0 + 1, l0 = lo + j; MS bounds the slice at compile time so that a register
    // source is indexed by constants
#pragma unroll
    for (int j = 0; j < MS; ++j) {
        const int l0 = lo + j;
        if (l0 >= hi) break;
        const int l = l0 + 1;
        const float2 h = src.h(l0, j);
        const float2 zl = src.z(l0, j);
        float2 g[K];
        float2 e = make_float2(-zl.x, -zl.y);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (!on[k]) continue;
            if (l0 > lo) u[k] = ((l0 - lo) & 7) == 0 ? phasor(l, tk[k], T, invT, twoinvT) : cmul(u[k], u1[k]);
            g[k] = cmul(h, u[k]);
            e.x += ak[k] * g[k].x;
            e.y += ak[k] * g[k].y;
        }
        if (depth) {
            const float wl = w1 * (float)l;
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (on[k]) gsum[k] += wl * (e.x * g[k].y - e.y * g[k].x);
        } else {
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (on[k]) gsum[k] += e.x * g[k].x + e.y * g[k].y;
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        gsum[k] += quad_xor1(gsum[k]);
        gsum[k] += quad_xor2(gsum[k]);
    }
}

// One data step for the K points of a pixel, by the four lanes `sub` = 0..3 of the pixel; each
// lane's slice of harmonics has at most MS entries.
template <int K, int MS, class Src>
__device__ __forceinline__ void data_point(const Src& src, int sub, int m, int T, float invT, float twoinvT, float nn,
                                           float gam_t, float gam_a, float* tk, float* ak, const bool* on) {
    const int lo = (sub * m) / kLanesPerPixel, hi = ((sub + 1) * m) / kLanesPerPixel;
    const float Tf = (float)T;
    // sums start at -0 (x + -0 = x exactly, so the first add is dropped)
    float gt[K];
#pragma unroll
    for (int k = 0; k < K; ++k) gt[k] = -0.f;
    residual_pass<K, MS>(src, lo, hi, T, invT, twoinvT, tk, ak, on, gt, true);
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (on[k]) tk[k] = wrap_t(tk[k] - gam_t * (-2.f * nn * ak[k] * gt[k]), Tf);
    float ga[K];
#pragma unroll
    for (int k = 0; k < K; ++k) ga[k] = -0.f;
    residual_pass<K, MS>(src, lo, hi, T, invT, twoinvT, tk, ak, on, ga, false);
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (on[k]) ak[k] = ak[k] - gam_a * (2.f * nn * ga[k]);
    project_capped_simplex<K>(ak, on);
}

template <int K>
__global__ __launch_bounds__(256) void data_step_kernel(IterArgs A, const float* __restrict__ z,
                                                        const int32_t* __restrict__ n,
                                                        const float* __restrict__ hhat,
                                                        const float* __restrict__ scal, float* __restrict__ t,
                                                        float* __restrict__ alpha,
                                                        const uint8_t* __restrict__ active) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int pix = gid / kLanesPerPixel, sub = gid % kLanesPerPixel;
    if (pix >= A.P) return;                      // the four lanes of a pixel leave together
    float tk[K], ak[K];
    bool on[K];
    bool any = false;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        tk[k] = t[(int64_t)pix * K + k];
        ak[k] = alpha[(int64_t)pix * K + k];
        on[k] = active[(int64_t)pix * K + k] != 0;
        any |= on[k];
    }
    const float nq = (float)n[pix];
    const float2* zrow = reinterpret_cast<const float2*>(z + (int64_t)pix * 2 * A.m);
    const float2* hh = reinterpret_cast<const float2*>(hhat);
    if (A.m <= kLanesPerPixel * kPrefetchSlice) {
        // the lane's slice of the sketch and of the spectrum, loaded with the state above (clamped
        // to the row, entries past the slice unused), so that every load is in flight at once
        const int lo = (sub * A.m) / kLanesPerPixel;
        float2 zr[kPrefetchSlice], hr[kPrefetchSlice];
#pragma unroll
        for (int j = 0; j < kPrefetchSlice; ++j) {
            zr[j] = zrow[min(lo + j, A.m - 1)];
            hr[j] = hh[min(lo + j, A.m - 1)];
        }
        if (!any) return;
        const RegSketchH<kPrefetchSlice> src{zr, hr};
        data_point<K, kPrefetchSlice>(src, sub, A.m, A.T, A.invT, A.twoinvT, nq, scal[1], scal[2], tk, ak, on);
    } else {
        if (!any) return;
        const GlobalSketch src{zrow, hh};
        data_point<K, kMaxSlice>(src, sub, A.m, A.T, A.invT, A.twoinvT, nq, scal[1], scal[2], tk, ak, on);
    }
    if (sub != 0) return;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        t[(int64_t)pix * K + k] = tk[k];
        alpha[(int64_t)pix * K + k] = ak[k];
    }
}

// The group's 16 pixels move from init's layout (row r of the product in lanes r, r + 16, r + 32,
// r + 48) to the data step's (pixel q in the aligned quad 4q .. 4q + 3), then take the same data
// step as data_step_kernel on the same values: the state as init stores it and the count, sketch
// and spectrum slices from memory.
template <int K>
__device__ void init_data_step(const IterArgs& A, const float* __restrict__ z, const float* __restrict__ hhat,
                               int grp, int lane, int np, const float (&t_r)[K], const float (&a_r)[K],
                               const int (&on_r)[K], float gam_t, float gam_a, float* __restrict__ t_out,
                               float* __restrict__ a_out, uint8_t* __restrict__ act_out) {
    const int q = lane >> 2, sub = lane & 3;           // lane q (its product row q) holds pixel q's state
    float tk[K], ak[K];
    bool on[K];
    bool any = false;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        tk[k] = __shfl(t_r[k], q, 64);
        ak[k] = __shfl(a_r[k], q, 64);
        on[k] = __shfl(on_r[k], q, 64) != 0;
        any |= on[k];
    }
    const float nq = (float)__shfl(np, q, 64);
    const int pix = grp * 16 + q;
    const bool pv = pix < A.P;                          // the same for the four lanes of a quad
    const float2* zrow = reinterpret_cast<const float2*>(z + (int64_t)(pv ? pix : A.P - 1) * 2 * A.m);
    const float2* hh = reinterpret_cast<const float2*>(hhat);
    if (any && pv) {                                    // slices read where used: fewer live registers
        const GlobalSketch src{zrow, hh};
        data_point<K, kMaxSlice>(src, sub, A.m, A.T, A.invT, A.twoinvT, nq, gam_t, gam_a, tk, ak, on);
    }
    if (sub == 0 && pv) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int64_t o = (int64_t)pix * K + k;
            t_out[o] = tk[k];
            a_out[o] = ak[k];
            act_out[o] = on[k] ? 1 : 0;
        }
    }
}

// ----------------------------------------------------------------------------- pixelwise estimator
// The comparison estimator of Sections 1 and 4 (SMLE): each pixel's sketched loss minimised on
// its own -- the data steps above with no denoisers -- from `starts` starting points, keeping
// the lowest loss.  Start 0 is the SRT3D initialisation; start s >= 1 puts point k at
// (s T / S + k T / K) mod T with its single-atom least-squares amplitude, all points active
// where n > 0, and alpha projected onto the constraint set.  Steps are per pixel: the pixel
// takes the frame's step sizes as if it had n_max photons.  Points are never removed.

// Sum over the four lanes of a pixel's quad (identical on all four).
__device__ __forceinline__ float quad_sum(float v) {
    v += quad_xor1(v);
    v += quad_xor2(v);
    return v;
}

template <int K, int MS, class Src>
__device__ __forceinline__ void smle_start(const Src& src, int lo, int hi, int s, int S, int T, float e2, bool has,
                                           float* tk, float* ak, bool* on) {
    const float Tf = (float)T, invT = 1.0f / Tf, twoinvT = 2.0f / Tf;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double t = fmod((double)s * T / S + (double)k * T / K, (double)T);
        tk[k] = wrap_t((float)t, Tf);
        float c = 0.f;
#pragma unroll
        for (int j = 0; j < MS; ++j) {
            const int l0 = lo + j;
            if (l0 >= hi) break;
            const float2 g = cmul(src.h(l0, j), phasor(l0 + 1, tk[k], T, invT, twoinvT));
            const float2 zl = src.z(l0, j);
            c += g.x * zl.x + g.y * zl.y;
        }
        c = quad_sum(c);
        ak[k] = e2 > 0.f ? fmaxf(0.f, c / e2) : 0.f;
        on[k] = has;
    }
    project_capped_simplex<K>(ak, on);
}

// Sum over the pixel's harmonics of |Phi_l - z_l|^2 (active points only).
template <int K, int MS, class Src>
__device__ __forceinline__ float smle_residual(const Src& src, int lo, int hi, int T, const float* tk, const float* ak,
                                               const bool* on) {
    const float Tf = (float)T, invT = 1.0f / Tf, twoinvT = 2.0f / Tf;
    float acc = 0.f;
#pragma unroll
    for (int j = 0; j < MS; ++j) {
        const int l0 = lo + j;
        if (l0 >= hi) break;
        const float2 h = src.h(l0, j);
        const float2 zl = src.z(l0, j);
        float2 e = make_float2(-zl.x, -zl.y);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (!on[k]) continue;
            const float2 g = cmul(h, phasor(l0 + 1, tk[k], T, invT, twoinvT));
            e.x += ak[k] * g.x;
            e.y += ak[k] * g.y;
        }
        acc += e.x * e.x + e.y * e.y;
    }
    return quad_sum(acc);
}

template <int K, int MS, class Src>
__device__ __forceinline__ void smle_pixel(const Src& src, int pix, int sub, const IterArgs& A, int starts, int iters,
                                           const int32_t* __restrict__ n, const float* __restrict__ scal,
                                           const float* __restrict__ t0, const float* __restrict__ a0,
                                           const uint8_t* __restrict__ act0, float* __restrict__ t_out,
                                           float* __restrict__ a_out, uint8_t* __restrict__ act_out,
                                           float* __restrict__ loss_out) {
    const int lo = (sub * A.m) / kLanesPerPixel, hi = ((sub + 1) * A.m) / kLanesPerPixel;
    const int np = n[pix];
    const float nq = (float)np, nstep = np > 0 ? scal[0] : 0.f;
    float tb[K], ab[K], best = 0.f;
    bool ob[K];
    for (int s = 0; s < starts; ++s) {
        float tk[K], ak[K];
        bool on[K];
        if (s == 0) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int64_t q = (int64_t)pix * K + k;
                tk[k] = t0[q];
                ak[k] = a0[q];
                on[k] = act0[q] != 0;
            }
        } else {
            smle_start<K, MS>(src, lo, hi, s, starts, A.T, scal[4], np > 0, tk, ak, on);
        }
        bool any = false;
#pragma unroll
        for (int k = 0; k < K; ++k) any |= on[k];
        if (any)
            for (int it = 0; it < iters; ++it)
                data_point<K, MS>(src, sub, A.m, A.T, A.invT, A.twoinvT, nstep, scal[1], scal[2], tk, ak, on);
        const float L = nq * smle_residual<K, MS>(src, lo, hi, A.T, tk, ak, on);
        if (s == 0 || L < best) {
            best = L;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                tb[k] = tk[k];
                ab[k] = ak[k];
                ob[k] = on[k];
            }
        }
    }
    if (sub != 0) return;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t q = (int64_t)pix * K + k;
        t_out[q] = tb[k];
        a_out[q] = ab[k];
        act_out[q] = ob[k] ? 1 : 0;
    }
    loss_out[pix] = best;
}

// One launch for all starts and steps: four lanes per pixel, the pixel's sketch slice in
// registers when m <= 32.
template <int K, bool PREFETCH>
__global__ __launch_bounds__(256) void smle_kernel(IterArgs A, int starts, int iters, const float* __restrict__ z,
                                                   const int32_t* __restrict__ n, const float* __restrict__ hhat,
                                                   const float* __restrict__ scal, const float* __restrict__ t0,
                                                   const float* __restrict__ a0, const uint8_t* __restrict__ act0,
                                                   float* __restrict__ t_out, float* __restrict__ a_out,
                                                   uint8_t* __restrict__ act_out, float* __restrict__ loss_out) {
    __shared__ float2 s_h[SRT3D_MAX_M_RECON];
    for (int l = threadIdx.x; l < A.m; l += blockDim.x) s_h[l] = reinterpret_cast<const float2*>(hhat)[l];
    __syncthreads();
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int pix = gid / kLanesPerPixel, sub = gid % kLanesPerPixel;
    if (pix >= A.P) return;                      // the four lanes of a pixel leave together
    const float2* zp = reinterpret_cast<const float2*>(z + (int64_t)pix * 2 * A.m);
    if constexpr (PREFETCH) {
        const int lo = (sub * A.m) / kLanesPerPixel, hi = ((sub + 1) * A.m) / kLanesPerPixel;
        float2 zr[kPrefetchSlice];
#pragma unroll
        for (int j = 0; j < kPrefetchSlice; ++j) zr[j] = zp[lo + j < hi ? lo + j : lo];
        const RegSketch<kPrefetchSlice> src{zr, s_h};
        smle_pixel<K, kPrefetchSlice>(src, pix, sub, A, starts, iters, n, scal, t0, a0, act0, t_out, a_out, act_out,
                                      loss_out);
    } else {
        const GlobalSketch src{zp, s_h};
        smle_pixel<K, kMaxSlice>(src, pix, sub, A, starts, iters, n, scal, t0, a0, act0, t_out, a_out, act_out,
                                 loss_out);
    }
}

// ----------------------------------------------------------------------------- merge and birth
// Optional stage between iterations (RT3D's split and merge of points; the paper cites RT3D for
// scenes with several surfaces per pixel but does not describe the moves): active points of a
// pixel closer than T/(2m) merge, in slot order, into the lower slot (alpha-weighted circular
// mean depth, summed alpha); then a pixel with a free slot and photons runs the sketched matched
// filter of the initialisation on its residual z - Phi(theta), over the grid 0, s, 2s, ... at
// circular distance >= T/m from every active point, and the peak (lowest tau on ties), with
// amplitude max(0, c / sum |hhat|^2), fills the first free slot when it carries >= r_min
// photons; alpha is then projected.  One thread per pixel, the residual kept in LDS.
constexpr int kBirthThreads = 64;

template <int K>
__global__ __launch_bounds__(kBirthThreads) void birth_kernel(IterArgs A, int stride, int G,
                                                              const float* __restrict__ z,
                                                              const int32_t* __restrict__ n,
                                                              const float* __restrict__ hhat,
                                                              const float* __restrict__ scal, float* __restrict__ t_io,
                                                              float* __restrict__ a_io, uint8_t* __restrict__ act_io) {
    __shared__ float2 s_w[kBirthThreads][SRT3D_MAX_M_RECON];
    __shared__ float2 s_h[SRT3D_MAX_M_RECON];
    for (int l = threadIdx.x; l < A.m; l += kBirthThreads) s_h[l] = reinterpret_cast<const float2*>(hhat)[l];
    __syncthreads();
    const int pix = blockIdx.x * kBirthThreads + threadIdx.x;
    if (pix >= A.P) return;
    const int T = A.T, m = A.m;
    const float Tf = (float)T, invT = 1.0f / Tf, twoinvT = 2.0f / Tf;
    float tk[K], ak[K];
    bool on[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t q = (int64_t)pix * K + k;
        tk[k] = t_io[q];
        ak[k] = a_io[q];
        on[k] = act_io[q] != 0;
    }
    // merge
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int q = k + 1; q < K; ++q) {
            if (!(on[k] && on[q])) continue;
            const float d = circ_diff(tk[q] - tk[k], Tf, invT);
            if (!(fabsf(d) * (float)(2 * m) < Tf)) continue;
            const float sum = ak[k] + ak[q];
            const float w = sum > 0.f ? ak[q] / sum : 0.5f;
            tk[k] = wrap_t(tk[k] + w * d, Tf);
            ak[k] = sum;
            ak[q] = 0.f;
            on[q] = false;
        }
    int slot = -1;
#pragma unroll
    for (int k = K - 1; k >= 0; --k)
        if (!on[k]) slot = k;
    const int np = n[pix];
    if (slot >= 0 && np > 0) {
        const float2* zp = reinterpret_cast<const float2*>(z + (int64_t)pix * 2 * m);
        float2* w = s_w[threadIdx.x];
        for (int l = 0; l < m; ++l) {
            const float2 h = s_h[l];
            float2 e = zp[l];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (!on[k]) continue;
                const float2 g = cmul(h, phasor(l + 1, tk[k], T, invT, twoinvT));
                e.x -= ak[k] * g.x;
                e.y -= ak[k] * g.y;
            }
            w[l] = e;
        }
        float best = 0.f;
        int bg = -1;
        for (int g = 0; g < G; ++g) {
            const int tau = g * stride;
            bool excluded = false;
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (on[k] && fabsf(circ_diff((float)tau - tk[k], Tf, invT)) * (float)m < Tf) excluded = true;
            if (excluded) continue;
            // c = Re sum_l conj(hhat_l e^{i w_l tau}) w_l, the phase (l tau) mod T kept exactly
            float c = 0.f;
            int kph = 0;
            for (int l = 0; l < m; ++l) {
                kph += tau;
                if (kph >= T) kph -= T;
                const float2 q = cmul(s_h[l], phasor_int(kph, twoinvT));
                const float2 wl = w[l];
                c += q.x * wl.x + q.y * wl.y;
            }
            if (bg < 0 || c > best) {
                best = c;
                bg = g;
            }
        }
        const float e2 = scal[4];
        const float a = (bg >= 0 && e2 > 0.f) ? fmaxf(0.f, best / e2) : 0.f;
        if (bg >= 0 && (float)np * a >= A.r_min) {
            tk[slot] = (float)(bg * stride);
            ak[slot] = a;
            on[slot] = true;
        }
    }
    project_capped_simplex<K>(ak, on);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t q = (int64_t)pix * K + k;
        t_io[q] = tk[k];
        a_io[q] = ak[k];
        act_io[q] = on[k] ? 1 : 0;
    }
}

// ----------------------------------------------------------------------------- precision weighting
// Eq. (6) with W = Sigma^{-1}, pixel by pixel, as the second step after the pixelwise W = I
// estimate theta_1.  Sigma is the covariance of the sketch's 2m real coordinates
// [cos w_l x, sin w_l x] under pi_theta_1 (eq. 1), built from the characteristic function at
// sums and differences of frequencies (eq. 4 at w_a +- w_b), ridged by 1e-5 tr(Sigma) / (2m),
// factored once (L L^T) and held fixed; then Levenberg-Marquardt on the whitened residual
// L^{-1} [Re(z - Phi), Im(z - Phi)] over the active points' (t_k, alpha_k), a step kept iff it
// lowers n ||L^{-1} r||^2 (mu from 1e-3, / 10 on success down to 1e-7, * 10 on failure up to
// 1e7), alpha projected onto the constraint set, t wrapped.
//
// One segment of M2 >= 2m lanes per pixel (a wave holds 64 / M2 pixels); lane i of a segment
// owns row i of Sigma, then of L (row-oriented Cholesky with the pivot column broadcast across
// the segment), and entry i of every whitened vector.  Rows 2m..M2-1 are identity.

// hhat_l for l = 1..J (J <= 2 SRT3D_MAX_M_RECON), one harmonic per wave, the FP64 sums of the
// frame setup.
__global__ __launch_bounds__(1024) void spectrum_kernel(const double* __restrict__ irf, int irf_len, int origin,
                                                        int T, int J, float2* __restrict__ out) {
    __shared__ double s_H;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (wv == 0) {
        double h0 = 0;
        for (int i = lane; i < irf_len; i += 64) h0 += irf[i];
        h0 = wave_sum_d(h0);
        if (lane == 0) s_H = h0;
    }
    __syncthreads();
    const double H = s_H;
    for (int l = 1 + wv; l <= J; l += blockDim.x >> 6) {
        double re = 0, im = 0;
        for (int i = lane; i < irf_len; i += 64) {
            int k = (int)(((int64_t)l * (i - origin)) % T);
            if (k < 0) k += T;
            double sn, cs;
            sincospi(2.0 * (double)k / (double)T, &sn, &cs);
            re += irf[i] * cs;
            im += irf[i] * sn;
        }
        re = wave_sum_d(re) / H;
        im = wave_sum_d(im) / H;
        if (lane == 0) out[l - 1] = make_float2((float)re, (float)im);
    }
}

// A wave holds 64 / M2 pixels, one per segment of M2 lanes (M2 = 64: one pixel).  Broadcast of
// lane `base + j` of the caller's segment: readlane when the segment is the wave; with two
// segments, one readlane per segment and a select (scalar reads, no LDS traffic: the broadcasts
// of the factorisation and the whitening outnumber the arithmetic); with more segments a
// cross-lane permute through the LDS crossbar (one instruction for every segment).
template <int M2>
__device__ __forceinline__ float sbcast(float v, int base, int j) {
    if constexpr (M2 == 64) {
        return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), j));
    } else if constexpr (M2 == 32) {
        const float lo = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), j));
        const float hi = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 32 + j));
        return base == 0 ? lo : hi;
    } else {
        return __shfl(v, base + j, 64);
    }
}

// Sum over the caller's segment of M2 lanes (identical in all of them).
template <int M2>
__device__ __forceinline__ float seg_sum(float v) {
#pragma unroll
    for (int o = M2 / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Entry i of the real residual and Jacobian at (tk, ak, on): lane i < 2m takes harmonic
// l = i mod m + 1, its real part for i < m and imaginary part otherwise.  Columns t_1..t_K,
// alpha_1..alpha_K; zero for inactive points and for lanes >= 2m.
template <int K>
__device__ __forceinline__ void w_residual(const float2* __restrict__ zp, const float2* __restrict__ h2, int i, int m,
                                           int T, const float* tk, const float* ak, const bool* on, float& r,
                                           float* jc);

// The same with this lane's spectrum and sketch entries (h = hhat_l, zl = z_l, l the lane's
// harmonic) already in registers.
template <int K>
__device__ __forceinline__ void w_residual_v(float2 h, float2 zl, int i, int m, int T, const float* tk,
                                             const float* ak, const bool* on, float& r, float* jc) {
    const float Tf = (float)T, invT = 1.0f / Tf, twoinvT = 2.0f / Tf;
    r = 0.f;
#pragma unroll
    for (int c = 0; c < 2 * K; ++c) jc[c] = 0.f;
    if (i >= 2 * m) return;
    const bool re = i < m;
    const int l = (re ? i : i - m) + 1;
    const float w = 6.283185307179586f * (float)l * invT;
    float2 phi = make_float2(0.f, 0.f);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (!on[k]) continue;
        const float2 g = cmul(h, phasor(l, tk[k], T, invT, twoinvT));
        phi.x += ak[k] * g.x;
        phi.y += ak[k] * g.y;
        // dPhi/dt_k = a_k i w g, dPhi/dalpha_k = g
        jc[k] = re ? -ak[k] * w * g.y : ak[k] * w * g.x;
        jc[K + k] = re ? g.x : g.y;
    }
    r = re ? zl.x - phi.x : zl.y - phi.y;
}

template <int K>
__device__ __forceinline__ void w_residual(const float2* __restrict__ zp, const float2* __restrict__ h2, int i, int m,
                                           int T, const float* tk, const float* ak, const bool* on, float& r,
                                           float* jc) {
    const int l = i < 2 * m ? (i < m ? i : i - m) + 1 : 1;
    w_residual_v<K>(h2[l - 1], zp[l - 1], i, m, T, tk, ak, on, r, jc);
}

// Row pitch (floats) of a segment's M2 x M2 LDS matrix: unpadded, so that four waves of two
// 32-lane segments fit four workgroups per CU; rows start on 16-byte boundaries and the lanes of
// a segment writing one column hit consecutive words.
template <int M2> constexpr int kLdsPitch = M2;
// A segment's LDS matrix with 32 words of padding after it, so that the two segments of a wave
// (M2 = 32) sit 32 banks apart and their simultaneous accesses do not collide.
template <int M2> constexpr int kLdsSegment = M2 * kLdsPitch<M2> + 32;

// Rows of L^{-1} (lower triangular) for the segment: lane i gets row i in linv.  Lane i solves
// L x = e_i, i.e. column i of L^{-1}, by forward substitution with the rows of L read from LDS
// (the lanes of a segment read the same entries, four at a time: broadcast reads, no cross-lane
// permutes), then the columns are transposed through the same LDS.  sl: the segment's
// M2 x kLdsPitch<M2> floats, 16-byte aligned, private to the wave.
template <int M2>
__device__ __forceinline__ void w_inverse_rows(const float (&row)[M2], const float (&invd)[M2], float (&linv)[M2],
                                               int i, float* sl) {
    constexpr int LP = kLdsPitch<M2>;
#pragma unroll
    for (int c = 0; c < M2; c += 4)       // row i of L (its entries c < i are read)
        *reinterpret_cast<float4*>(sl + i * LP + c) = make_float4(row[c], row[c + 1], row[c + 2], row[c + 3]);
    float x[M2];
#pragma unroll
    for (int c = 0; c < M2; ++c) {
        float acc = c == i ? 1.f : 0.f;
#pragma unroll
        for (int k = 0; k < c; k += 4) {
            const float4 q = *reinterpret_cast<const float4*>(sl + c * LP + k);
            acc -= q.x * x[k];
            if (k + 1 < c) acc -= q.y * x[k + 1];
            if (k + 2 < c) acc -= q.z * x[k + 2];
            if (k + 3 < c) acc -= q.w * x[k + 3];
        }
        x[c] = acc * invd[c];
    }
    // x[c] = (L^{-1})_{c i}; the reads above precede these writes in the wave's LDS order
#pragma unroll
    for (int c = 0; c < M2; ++c) sl[c * LP + i] = x[c];
#pragma unroll
    for (int c = 0; c < M2; c += 4) {
        const float4 q = *reinterpret_cast<const float4*>(sl + i * LP + c);
        linv[c] = q.x;
        linv[c + 1] = q.y;
        linv[c + 2] = q.z;
        linv[c + 3] = q.w;
    }
}

// In place: b <- Linv b for V vectors, lane i holding row i of Linv: each vector is written to
// LDS once and read back whole by every lane of the segment (broadcast reads, four at a time),
// one FMA per column.  sb: the segment's V x M2 floats, 16-byte aligned, private to the wave.
template <int M2, int V>
__device__ __forceinline__ void w_apply_inverse(const float (&linv)[M2], float (&b)[V], int i, float* sb) {
#pragma unroll
    for (int v = 0; v < V; ++v) sb[v * M2 + i] = b[v];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        float y = 0.f;
#pragma unroll
        for (int c = 0; c < M2; c += 4) {
            const float4 q = *reinterpret_cast<const float4*>(sb + v * M2 + c);
            y = fmaf(linv[c], q.x, y);
            y = fmaf(linv[c + 1], q.y, y);
            y = fmaf(linv[c + 2], q.z, y);
            y = fmaf(linv[c + 3], q.w, y);
        }
        b[v] = y;
    }
}

// Whitening b <- L^{-1} b through the explicit inverse, formed once per pixel (lane i holds row i
// of L^{-1}).  With 64-entry rows it takes most of the registers and spills a little while it is
// formed, and still beats forward substitution in every whitening (weights 7.8x, fit 2.3x faster
// at m = 32).  lds: the segment's M2 x kLdsPitch<M2> floats.
template <int M2>
struct Whitener {
    float row[M2], invd[M2];      // the Cholesky factor (w_factor)
    float linv[M2];               // row i of L^{-1} (w_inverse_rows)
    template <int V>
    __device__ __forceinline__ void apply(float (&b)[V], int i, float* lds) const {
        static_assert(V <= M2 + 4, "the vectors fit the segment's LDS matrix");
        w_apply_inverse<M2, V>(linv, b, i, lds);
    }
};

// Sigma(theta) of the pixel of this segment, ridged, and its Cholesky factor: lane i builds row i
// of Sigma from Psi_0..Psi_2m (eq. 4 at the sums and differences of the frequencies), then the
// row-oriented factorisation leaves L_ij (j <= i) in wh.row[j] and 1 / L_jj in wh.invd[j].  Rows and
// columns 2m..M2-1 are identity.  psi: the segment's 2m + 1 LDS slots.  Every thread of the block
// must call it (one workgroup barrier).
template <int K, int M2>
__device__ __forceinline__ void w_factor(const float2* __restrict__ h2, int i, int base, int m, int T, const float* tk,
                                         const float* ak, const bool* on, float2* psi, Whitener<M2>& wh) {
    const float invT = 1.0f / (float)T, twoinvT = 2.0f / (float)T;
    // characteristic function Psi_j, j = 0..2m, at theta
    for (int j = i; j <= 2 * m; j += M2) {
        float2 v = make_float2(j == 0 ? 1.f : 0.f, 0.f);
        if (j > 0) {
            const float2 h = h2[j - 1];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (!on[k]) continue;
                const float2 g = cmul(h, phasor(j, tk[k], T, invT, twoinvT));
                v.x += ak[k] * g.x;
                v.y += ak[k] * g.y;
            }
        }
        psi[j] = v;
    }
    __syncthreads();
    // row i of Sigma
    float (&row)[M2] = wh.row;
    float (&invd)[M2] = wh.invd;
    {
        const float2* ps = psi;
        const bool ri = i < m;
        const int a = (ri ? i : i - m) + 1;
        const float2 pa = i < 2 * m ? ps[a] : make_float2(0.f, 0.f);
        const float mui = ri ? pa.x : pa.y;
        float dg = 0.f;
#pragma unroll
        for (int c = 0; c < M2; ++c) {
            float v;
            if (i >= 2 * m || c >= 2 * m) {
                v = c == i ? 1.f : 0.f;
            } else {
                const bool rc = c < m;
                const int b = (rc ? c : c - m) + 1;
                const float2 pb = ps[b];
                const float2 s = ps[a + b];
                const int d = a - b;
                float2 df = ps[d >= 0 ? d : -d];
                if (d < 0) df.y = -df.y;
                if (ri && rc) v = 0.5f * (s.x + df.x);
                else if (!ri && !rc) v = 0.5f * (df.x - s.x);
                else if (ri) v = 0.5f * (s.y - df.y);           // E[cos_a sin_b]
                else v = 0.5f * (s.y + df.y);                   // E[sin_a cos_b]
                v -= mui * (rc ? pb.x : pb.y);
            }
            row[c] = v;
            if (c == i) dg = v;
        }
        const float tr = seg_sum<M2>(i < 2 * m ? dg : 0.f);
        const float ridge = 1e-5f * tr / (float)(2 * m);
#pragma unroll
        for (int c = 0; c < M2; ++c)
            if (c == i && i < 2 * m) row[c] += ridge;
    }
    // Cholesky, row-oriented: after step j lane i >= j holds L_ij in row[j]
#pragma unroll
    for (int j = 0; j < M2; ++j) {
        const float d = sbcast<M2>(row[j], base, j);
        const float piv = sqrtf(fmaxf(d, 1e-30f));
        const float inv = 1.0f / piv;
        invd[j] = inv;
        const float lj = row[j] * inv;
        row[j] = lj;
#pragma unroll
        for (int c = j + 1; c < M2; ++c) row[c] -= lj * sbcast<M2>(lj, base, c);
    }
}

template <int K, int M2>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(M2 == 32 ? 4 : (M2 == 64 ? 2 : 1)))) void wsmle_kernel(IterArgs A, int witers, const float* __restrict__ z,
                                                    const int32_t* __restrict__ n, const float2* __restrict__ h2,
                                                    float* __restrict__ t_io, float* __restrict__ a_io,
                                                    const uint8_t* __restrict__ act, float* __restrict__ loss_out) {
    constexpr int kWaves = 256 / 64;
    constexpr int kPPW = 64 / M2;                      // pixels per wave, one per segment
    __shared__ float2 s_psi[kWaves][kPPW][2 * M2 + 1];
    __shared__ __align__(16) float s_lw[kWaves][kPPW][kLdsSegment<M2>];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int seg = lane / M2, i = lane % M2, base = seg * M2;
    const int pix_raw = (blockIdx.x * kWaves + wv) * kPPW + seg;
    const bool valid = pix_raw < A.P;
    const int pix = valid ? pix_raw : A.P - 1;
    const int m = A.m, T = A.T;
    const float Tf = (float)T, invT = 1.0f / Tf, twoinvT = 2.0f / Tf;
    float* lw = s_lw[wv][seg];
    float tk[K], ak[K];
    bool on[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t q = (int64_t)pix * K + k;
        tk[k] = t_io[q];
        ak[k] = a_io[q];
        on[k] = act[q] != 0;
    }
    Whitener<M2> wh;
    w_factor<K, M2>(h2, i, base, m, T, tk, ak, on, s_psi[wv][seg], wh);
    w_inverse_rows<M2>(wh.row, wh.invd, wh.linv, i, lw);         // lane i: row i
    const float2* zp = reinterpret_cast<const float2*>(z + (int64_t)pix * 2 * m);
    const float nq = (float)n[pix];
    auto loss_at = [&](const float* tt, const float* aa) {
        float b[1];
        float jc[2 * K];
        w_residual<K>(zp, h2, i, m, T, tt, aa, on, b[0], jc);
        wh.apply(b, i, lw);
        return nq * seg_sum<M2>(b[0] * b[0]);
    };
    float loss = loss_at(tk, ak);
    float mu = 1e-3f;
    {
        // every segment runs all steps (a pixel without active points has a zero Jacobian: its
        // step is zero and never kept)
        for (int it = 0; it < witers; ++it) {
            float b[1 + 2 * K];
            float jc[2 * K];
            w_residual<K>(zp, h2, i, m, T, tk, ak, on, b[0], jc);
#pragma unroll
            for (int c = 0; c < 2 * K; ++c) b[1 + c] = jc[c];
            wh.apply(b, i, lw);
            // normal equations (identical in every lane of the segment)
            float Am[2 * K][2 * K], g[2 * K];
#pragma unroll
            for (int p = 0; p < 2 * K; ++p) {
                g[p] = seg_sum<M2>(b[1 + p] * b[0]);
#pragma unroll
                for (int q = 0; q <= p; ++q) {
                    Am[p][q] = seg_sum<M2>(b[1 + p] * b[1 + q]);
                    Am[q][p] = Am[p][q];
                }
            }
#pragma unroll
            for (int p = 0; p < 2 * K; ++p) Am[p][p] += mu * (Am[p][p] + 1e-12f);
            // Cholesky solve of the small system
            float Lm[2 * K][2 * K], y[2 * K], dlt[2 * K];
#pragma unroll
            for (int p = 0; p < 2 * K; ++p) {
#pragma unroll
                for (int q = 0; q <= p; ++q) {
                    float sacc = Am[p][q];
#pragma unroll
                    for (int r2 = 0; r2 < q; ++r2) sacc -= Lm[p][r2] * Lm[q][r2];
                    Lm[p][q] = p == q ? sqrtf(fmaxf(sacc, 1e-38f)) : sacc / Lm[q][q];
                }
            }
#pragma unroll
            for (int p = 0; p < 2 * K; ++p) {
                float sacc = g[p];
#pragma unroll
                for (int q = 0; q < p; ++q) sacc -= Lm[p][q] * y[q];
                y[p] = sacc / Lm[p][p];
            }
#pragma unroll
            for (int p = 2 * K - 1; p >= 0; --p) {
                float sacc = y[p];
#pragma unroll
                for (int q = p + 1; q < 2 * K; ++q) sacc -= Lm[q][p] * dlt[q];
                dlt[p] = sacc / Lm[p][p];
            }
            float tn[K], an[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                tn[k] = on[k] ? wrap_t(tk[k] + dlt[k], Tf) : tk[k];
                an[k] = on[k] ? ak[k] + dlt[K + k] : 0.f;
            }
            project_capped_simplex<K>(an, on);
            const float ln = loss_at(tn, an);
            if (ln < loss) {
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    tk[k] = tn[k];
                    ak[k] = an[k];
                }
                loss = ln;
                mu = fmaxf(mu * 0.1f, 1e-7f);
            } else {
                mu = fminf(mu * 10.f, 1e7f);
            }
        }
    }
    if (!valid || i != 0) return;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t q = (int64_t)pix * K + k;
        t_io[q] = tk[k];
        a_io[q] = ak[k];
    }
    loss_out[pix] = loss;
}

// ----------------------------------------------------------------------------- weighted SRT3D
// W_p is stored as its lower triangle by columns: column c holds W_ic for i = c .. d - 1
// (d = 2m), at offset c d - c (c - 1) / 2 of the pixel's block; blocks of d (d + 1) / 2 floats
// rounded up to a multiple of four (16-byte aligned).  Half of the full matrix's bytes, and the
// entries of one column are consecutive.
__host__ __device__ constexpr int w_tri(int d) { return ((d * (d + 1) / 2) + 3) & ~3; }
__host__ __device__ constexpr int w_col(int d, int c) { return c * d - c * (c - 1) / 2; }

// Eq. (8) with a per-pixel W inside SRT3D's data step: W_p = Sigma(theta_0)^{-1}, the inverse of
// the ridged covariance of the sketch's 2m real coordinates at the pixel's points theta_0 (the
// state when prepared, normally the initialisation), held fixed.  The data step is SRT3D's with
// the loss n e^T W e, e = [Re(Phi - z), Im(Phi - z)]: gradient 2 n J^T W e, steps the W = I ones
// with n_max replaced by n_w = max_p n_p max_i sum_j |W_p,ij| (a Gershgorin bound of the largest
// eigenvalue of W_p, exact for W_p = c I).
//
// wprep_kernel: one segment of M2 >= 2m lanes per pixel; Sigma and its Cholesky factor as in the
// weighted pixelwise fit, L^{-1} by the column solves of w_inverse_rows (left in LDS), then
// W_ij = sum_k (L^{-1})_ki (L^{-1})_kj through LDS (the same bits for W_ji: same products, same
// order), and the frame's n_w is an atomic maximum of the (non-negative) float bits.  Lane i
// writes the entries W_ij, j <= i, of its row: the lanes of one store (one j) write consecutive
// words of column j of the packed lower triangle.
template <int K, int M2>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(M2 == 32 ? 4 : (M2 == 64 ? 2 : 1)))) void wprep_kernel(IterArgs A, const int32_t* __restrict__ n,
                                                    const float2* __restrict__ h2, const float* __restrict__ t_in,
                                                    const float* __restrict__ a_in, const uint8_t* __restrict__ act,
                                                    float* __restrict__ W, unsigned int* __restrict__ nw_bits) {
    constexpr int kWaves = 256 / 64;
    constexpr int kPPW = 64 / M2;
    __shared__ float2 s_psi[kWaves][kPPW][2 * M2 + 1];
    constexpr int LP = kLdsPitch<M2>;
    __shared__ __align__(16) float s_li[kWaves][kPPW][kLdsSegment<M2>];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int seg = lane / M2, i = lane % M2, base = seg * M2;
    const int pix_raw = (blockIdx.x * kWaves + wv) * kPPW + seg;
    const bool valid = pix_raw < A.P;
    const int pix = valid ? pix_raw : A.P - 1;
    const int m = A.m, twom = 2 * A.m;
    float tk[K], ak[K];
    bool on[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t q = (int64_t)pix * K + k;
        tk[k] = t_in[q];
        ak[k] = a_in[q];
        on[k] = act[q] != 0;
    }
    Whitener<M2> wh;
    w_factor<K, M2>(h2, i, base, m, A.T, tk, ak, on, s_psi[wv][seg], wh);
    float li[M2];
    float (*sl)[LP] = reinterpret_cast<float (*)[LP]>(s_li[wv][seg]);
    w_inverse_rows<M2>(wh.row, wh.invd, li, i, &sl[0][0]);          // leaves L^{-1} in sl, row-major
    __syncthreads();
    float gsum = 0.f;
    float* wtri = W + (int64_t)pix * w_tri(twom);
    {
        // All of row i at once: for each k, entry (k, i) of L^{-1} and row k read four entries
        // at a time by the whole segment (broadcast reads).  The products with k < max(i, j) or
        // k >= 2m are exact zeros (L^{-1} is lower triangular with identity rows past 2m), so each
        // sum is the one over k = max(i, j) .. 2m - 1 in the same order, and W_ij and W_ji the
        // same bits.  (The k loop stays rolled: unrolled, the reads of every row are hoisted.)
        float acc[M2];
#pragma unroll
        for (int j = 0; j < M2; ++j) acc[j] = 0.f;
#pragma unroll 1
        for (int k = 0; k < M2; ++k) {
            const float xk = sl[k][i];
#pragma unroll
            for (int j = 0; j < M2; j += 4) {
                const float4 q = *reinterpret_cast<const float4*>(&sl[k][j]);
                acc[j] = fmaf(xk, q.x, acc[j]);
                acc[j + 1] = fmaf(xk, q.y, acc[j + 1]);
                acc[j + 2] = fmaf(xk, q.z, acc[j + 2]);
                acc[j + 3] = fmaf(xk, q.w, acc[j + 3]);
            }
        }
        if (i < twom) {
#pragma unroll
            for (int j = 0; j < M2; ++j) {
                if (j < twom) {
                    if (valid && j <= i) wtri[w_col(twom, j) + (i - j)] = acc[j];
                    gsum += fabsf(acc[j]);
                }
            }
        }
    }
#pragma unroll
    for (int o = M2 / 2; o > 0; o >>= 1) gsum = fmaxf(gsum, __shfl_xor(gsum, o, 64));
    if (valid && i == 0) atomicMax(nw_bits, __float_as_uint(gsum * (float)n[pix]));
}

// One weighted data step of every pixel, in place on the current half: the wave's packed
// triangles (consecutive pixels, so one contiguous range) are copied to LDS by 16-byte loads,
// then lane i < 2m of the pixel's segment reads row i of W_p from there (W_ic from column c for
// c <= i, from column i for c > i); v = W e through one broadcast and one FMA per column.
template <int K, int M2>
__global__ __launch_bounds__(256) void wdata_kernel(IterArgs A, const float* __restrict__ z,
                                                    const int32_t* __restrict__ n, const float2* __restrict__ hhat,
                                                    const float* __restrict__ scal, const float* __restrict__ W,
                                                    const unsigned int* __restrict__ nw_bits, float* __restrict__ t_io,
                                                    float* __restrict__ a_io, const uint8_t* __restrict__ act) {
    constexpr int kWaves = 256 / 64;
    constexpr int kPPW = 64 / M2;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int seg = lane / M2, i = lane % M2, base = seg * M2;
    const int pix_raw = (blockIdx.x * kWaves + wv) * kPPW + seg;
    const bool valid = pix_raw < A.P;
    const int pix = valid ? pix_raw : A.P - 1;
    const int m = A.m, twom = 2 * A.m, T = A.T;
    const float Tf = (float)T;
    float tk[K], ak[K];
    bool on[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t q = (int64_t)pix * K + k;
        tk[k] = t_io[q];
        ak[k] = a_io[q];
        on[k] = act[q] != 0;
    }
    // the lane's spectrum and sketch entries, the counts and the weight bound, loaded with the state
    const int lh = i < twom ? (i < m ? i : i - m) : 0;     // harmonic - 1 of this lane's component
    const float2 h_own = hhat[lh];
    const float2 z_own = reinterpret_cast<const float2*>(z + (int64_t)pix * 2 * m)[lh];
    const int32_t n_own = n[pix];
    const unsigned int nw_raw = *nw_bits;
    float wrow[M2];
    {
        constexpr int kMaxTri = w_tri(M2);
        __shared__ __align__(16) float s_w[kWaves][kPPW * kMaxTri];
        const int tri = w_tri(twom);                         // floats per pixel, a multiple of 4
        const int p0 = (blockIdx.x * kWaves + wv) * kPPW;    // the wave's first pixel
        const int np = A.P - p0 < kPPW ? A.P - p0 : kPPW;     // its pixels in the frame (>= 1)
        const float4* src = reinterpret_cast<const float4*>(W + (int64_t)p0 * tri);
        float4* dst = reinterpret_cast<float4*>(s_w[wv]);
        // every round's 16-byte load in flight before the first store (clamped to the last
        // piece, which is then copied again)
        constexpr int kRounds = (kPPW * kMaxTri / 4 + 63) / 64;
        const int nq4 = np * tri / 4;
        float4 wv4[kRounds];
#pragma unroll
        for (int u = 0; u < kRounds; ++u) wv4[u] = src[min(lane + 64 * u, nq4 - 1)];
#pragma unroll
        for (int u = 0; u < kRounds; ++u)
            if (lane + 64 * u < nq4) dst[lane + 64 * u] = wv4[u];
        const float* tw = s_w[wv] + (valid ? seg : 0) * tri;  // (same wave: LDS order suffices)
#pragma unroll
        for (int c = 0; c < M2; ++c) {
            float v = 0.f;
            if (i < twom && c < twom) v = c <= i ? tw[w_col(twom, c) + (i - c)] : tw[w_col(twom, i) + (c - i)];
            wrow[c] = v;
        }
    }
    // the W = I steps with n_max replaced by n_w
    const float nw = __uint_as_float(nw_raw);
    const float gam_t = nw > 0.f ? scal[1] * (scal[0] / nw) : 0.f;
    const float gam_a = nw > 0.f ? scal[2] * (scal[0] / nw) : 0.f;
    const float nq = (float)n_own;
    // g = 2 n J^T W e at (tt, ak); e goes to LDS once and every lane of the segment reads it
    // whole, four entries at a time (broadcast reads)
    __shared__ __align__(16) float s_e[kWaves][64];
    float* se = s_e[wv] + base;
    auto grad = [&](const float* tt, float* g) {
        float r, jc[2 * K];
        w_residual_v<K>(h_own, z_own, i, m, T, tt, ak, on, r, jc);    // r = z - Phi
        se[i] = -r;                                                    // e
        float v = 0.f;
#pragma unroll
        for (int c = 0; c < M2; c += 4) {
            const float4 q = *reinterpret_cast<const float4*>(se + c);
            v = fmaf(wrow[c], q.x, v);
            v = fmaf(wrow[c + 1], q.y, v);
            v = fmaf(wrow[c + 2], q.z, v);
            v = fmaf(wrow[c + 3], q.w, v);
        }
#pragma unroll
        for (int c = 0; c < 2 * K; ++c) g[c] = 2.f * nq * seg_sum<M2>(jc[c] * v);
    };
    float g[2 * K];
    grad(tk, g);
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (on[k]) tk[k] = wrap_t(tk[k] - gam_t * g[k], Tf);
    grad(tk, g);
    float an[K];
#pragma unroll
    for (int k = 0; k < K; ++k) an[k] = on[k] ? ak[k] - gam_a * g[K + k] : ak[k];
    project_capped_simplex<K>(an, on);
    if (!valid || i != 0) return;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t q = (int64_t)pix * K + k;
        t_io[q] = tk[k];
        a_io[q] = an[k];
    }
}

__global__ void fill_u32_kernel(unsigned int* __restrict__ p, unsigned int v) { *p = v; }

// ----------------------------------------------------------------------------- denoisers
// Solve the leading D x D block of M x = b by M = L diag(d) L^T (unit lower L), with
// reciprocals of the pivots.  The pivot d_j = M_jj - sum_k L_jk^2 d_k is the square of the
// Cholesky diagonal, so "d_j <= kCholEps * trace" is the Cholesky singularity rule.  Only x[0]
// is needed.
template <int D>
__device__ __forceinline__ bool ldl_x0(const float (&M)[4][4], const float (&b)[4], float& x0) {
    float L[D][D], d[D], inv[D];
    float tr = 0.f;
#pragma unroll
    for (int i = 0; i < D; ++i) tr += M[i][i];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        float v[D];
        float s = M[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) {
            v[k] = L[j][k] * d[k];
            s -= L[j][k] * v[k];
        }
        if (!(s > kCholEps * tr)) return false;
        d[j] = s;
        inv[j] = __builtin_amdgcn_rcpf(s);
#pragma unroll
        for (int i = j + 1; i < D; ++i) {
            float w = M[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) w -= L[i][k] * v[k];
            L[i][j] = w * inv[j];
        }
    }
    float y[D], x[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        float w = b[j];
#pragma unroll
        for (int k = 0; k < j; ++k) w -= L[j][k] * y[k];
        y[j] = w;
    }
#pragma unroll
    for (int j = D - 1; j >= 0; --j) {
        float w = y[j] * inv[j];
#pragma unroll
        for (int k = j + 1; k < D; ++k) w -= L[k][j] * x[k];
        x[j] = w;
    }
    x0 = x[0];
    return true;
}

// Integer window weight q = ((R+1)^2 - di^2 - dj^2)^4 = (R+1)^8 w.  The constant factor cancels
// in the least-squares solution, the pivot rule and the weighted mean, and with integer weights
// every normal-matrix entry is an integer: exact in FP32 for R <= 2 (largest entry < 2^18).
template <int R>
__device__ constexpr float win_q(int di, int dj) {
    const int64_t u = (int64_t)(R + 1) * (R + 1) - di * di - dj * dj;
    return (float)(u * u * u * u);
}

template <int R>
__device__ constexpr float full_moment(int r, int c) {
    int64_t acc = 0;
    for (int di = -R; di <= R; ++di)
        for (int dj = -R; dj <= R; ++dj) {
            const int64_t u = (int64_t)(R + 1) * (R + 1) - di * di - dj * dj;
            const int64_t phi[4] = {1, di, dj, di * di + dj * dj};
            acc += u * u * u * u * phi[r] * phi[c];
        }
    return (float)acc;
}

// Depth denoiser for point k of the pixel at LDS cell (ci, cj); t and act are (E x E cells) x K
// arrays whose window cells lie within the array.  With one point per pixel and R <= 2 the
// normal matrix is the full-window sum minus the (few) neighbours that fail the gate -- exact,
// since all entries are integers below 2^24.  With several points per pixel the K candidates of
// a window cell share the cell's offsets, so each cell contributes (gated count) x (its weighted
// monomials) to the matrix and q x (sum of its gated offsets) x (monomials) to the right-hand
// side: one set of updates per cell instead of per candidate.  Entries whose factor is zero for
// a given offset are skipped at compile time.
//
// The window is summed in two parts, rows -R..0 and rows 1..R (each in window order), added as
// part 0 + part 1: the fused iteration gives the parts to different waves, the stand-alone
// kernel sums both in one thread, and both get the same bits.
template <int K, int R>
__device__ __forceinline__ void dd_start(float (&M)[4][4], float (&b)[4], bool first) {
    constexpr bool SUB = (K == 1) && (R <= 2);
    // zero sums start at -0, the identity of addition, so the first update is a plain product
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        b[r] = -0.f;
#pragma unroll
        for (int c = 0; c < 4; ++c) M[r][c] = (SUB && first) ? full_moment<R>(r, c) : -0.f;
    }
}

template <int K, int R, int DI0, int DI1>
__device__ __forceinline__ void dd_rows(const float* st, const uint8_t* sa, int E, int ci, int cj, float tq, float Tf,
                                        float invT, float tau_z, float (&M)[4][4], float (&b)[4]) {
    constexpr bool SUB = (K == 1) && (R <= 2);
#pragma unroll
    for (int di = DI0; di <= DI1; ++di) {
#pragma unroll
        for (int dj = -R; dj <= R; ++dj) {
            const float q = win_q<R>(di, dj);
            const int r2 = di * di + dj * dj;
            // the cell's gated offsets: their sum and how many pass (or, with SUB, fail) the gate
            float dsum = -0.f, cnt = -0.f;
#pragma unroll
            for (int kk = 0; kk < K; ++kk) {
                const int cn = ((ci + di) * E + (cj + dj)) * K + kk;
                const float d = circ_diff(st[cn] - tq, Tf, invT);
                const bool gate = sa[cn] && fabsf(d) <= tau_z;
                dsum += gate ? d : 0.f;
                cnt += (SUB ? !gate : gate) ? 1.f : 0.f;
            }
            // q phi_r is an integer below 2^24 for R <= 2, so each update is one fused multiply-add
            b[0] = fmaf(q, dsum, b[0]);
            if (di != 0) b[1] = fmaf(q * (float)di, dsum, b[1]);
            if (dj != 0) b[2] = fmaf(q * (float)dj, dsum, b[2]);
            if (r2 != 0) b[3] = fmaf(q * (float)r2, dsum, b[3]);
            const float sq = SUB ? -q : q;
            M[0][0] = fmaf(sq, cnt, M[0][0]);
            if (di != 0) { M[0][1] = fmaf(sq * di, cnt, M[0][1]); M[1][1] = fmaf(sq * (di * di), cnt, M[1][1]); }
            if (dj != 0) { M[0][2] = fmaf(sq * dj, cnt, M[0][2]); M[2][2] = fmaf(sq * (dj * dj), cnt, M[2][2]); }
            if (di != 0 && dj != 0) M[1][2] = fmaf(sq * (di * dj), cnt, M[1][2]);
            if (r2 != 0) { M[0][3] = fmaf(sq * r2, cnt, M[0][3]); M[3][3] = fmaf(sq * (r2 * r2), cnt, M[3][3]); }
            if (di != 0 && r2 != 0) M[1][3] = fmaf(sq * (di * r2), cnt, M[1][3]);
            if (dj != 0 && r2 != 0) M[2][3] = fmaf(sq * (dj * r2), cnt, M[2][3]);
        }
    }
}

// The ten distinct matrix entries and the right-hand side of a part, for passing it on.
constexpr int kDDPart = 14;
__device__ __forceinline__ void dd_pack(const float (&M)[4][4], const float (&b)[4], float* o) {
    int i = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = r; c < 4; ++c) o[i++] = M[r][c];
#pragma unroll
    for (int r = 0; r < 4; ++r) o[i++] = b[r];
}
__device__ __forceinline__ void dd_add_part(float (&M)[4][4], float (&b)[4], const float* o) {
    int i = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = r; c < 4; ++c) M[r][c] += o[i++];
#pragma unroll
    for (int r = 0; r < 4; ++r) b[r] += o[i++];
}

// Solve the combined equations (upper triangle of M) and return the new depth.
__device__ __forceinline__ float dd_solve(float (&M)[4][4], float (&b)[4], float tq, float Tf, float lambda_z) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < r; ++c) M[r][c] = M[c][r];
    float a;
    if (!ldl_x0<4>(M, b, a)) {
        if (!ldl_x0<3>(M, b, a)) a = b[0] * __builtin_amdgcn_rcpf(M[0][0] > 0.f ? M[0][0] : 1.f);
    }
    return wrap_t(tq + lambda_z * a, Tf);
}

template <int K, int R>
__device__ __forceinline__ float dd_point(const float* st, const uint8_t* sa, int E, int ci, int cj, int k, float Tf,
                                          float invT, float tau_z, float lambda_z) {
    const float tq = st[(ci * E + cj) * K + k];
    float M[4][4], b[4], M1[4][4], b1[4], o[kDDPart];
    dd_start<K, R>(M, b, true);
    dd_rows<K, R, -R, 0>(st, sa, E, ci, cj, tq, Tf, invT, tau_z, M, b);
    dd_start<K, R>(M1, b1, false);
    dd_rows<K, R, 1, R>(st, sa, E, ci, cj, tq, Tf, invT, tau_z, M1, b1);
    dd_pack(M1, b1, o);
    dd_add_part(M, b, o);
    return dd_solve(M, b, tq, Tf, lambda_z);
}

// Intensity denoiser: gated weighted mean of r = n * alpha around point k of cell (ci, cj).
// The window's cells w = (di + R)(2R + 1) + (dj + R) are split into kIdParts interleaved parts
// (w = s, s + 4, ...): part s is summed in window order, and the mean is
// ((num_0 + num_1) + (num_2 + num_3)) / ((den_0 + den_1) + (den_2 + den_3)).  The fused iteration
// gives each part to one of a pixel's four lanes and adds them with two butterfly shuffles (which
// produce exactly that grouping in every lane); the stand-alone kernel adds the same parts in
// one thread, so both compute the same bits.
constexpr int kIdParts = 4;

template <int K, int R>
__device__ __forceinline__ void id_part(const float* st, const uint8_t* sa, const float* sr, int E, int ci, int cj,
                                        int k, float Tf, float invT, float tau_z, int s, float& num, float& den) {
    constexpr int W = 2 * R + 1;
    const float tq = st[(ci * E + cj) * K + k];
    num = -0.f;
    den = -0.f;
#pragma unroll
    for (int jj = 0; jj < (W * W + kIdParts - 1) / kIdParts; ++jj) {
        const int w = s + kIdParts * jj;
        if (w < W * W) {
            const int di = w / W - R, dj = w % W - R;
            const int u = (R + 1) * (R + 1) - di * di - dj * dj;
            const float q = (float)(u * u * u * u);          // the integer window weight (exact)
#pragma unroll
            for (int kk = 0; kk < K; ++kk) {
                const int cn = ((ci + di) * E + (cj + dj)) * K + kk;
                const float d = circ_diff(st[cn] - tq, Tf, invT);
                const float gw = (sa[cn] && fabsf(d) <= tau_z) ? q : 0.f;
                num = fmaf(gw, sr[cn], num);
                den += gw;
            }
        }
    }
}

__device__ __forceinline__ float id_ratio(float num, float den) {
    return num * __builtin_amdgcn_rcpf(den > 0.f ? den : 1.f);
}

// The whole mean in one thread (the four parts, added in the grouping above).
template <int K, int R>
__device__ __forceinline__ float id_mean(const float* st, const uint8_t* sa, const float* sr, int E, int ci, int cj,
                                         int k, float Tf, float invT, float tau_z) {
    float nm[kIdParts], dn[kIdParts];
#pragma unroll
    for (int s = 0; s < kIdParts; ++s) id_part<K, R>(st, sa, sr, E, ci, cj, k, Tf, invT, tau_z, s, nm[s], dn[s]);
    return id_ratio((nm[0] + nm[1]) + (nm[2] + nm[3]), (dn[0] + dn[1]) + (dn[2] + dn[3]));
}

// New alpha and activity of a pixel's K points from their gated means rt (eq. 1 projection).
template <int K>
__device__ __forceinline__ void id_update(const float* rt, const bool* was_on, float nq, float r_min, float* an,
                                          bool* keep) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
        keep[k] = was_on[k] && rt[k] >= r_min;
        an[k] = keep[k] ? rt[k] / (nq > 0.f ? nq : 1.f) : 0.f;
    }
    project_capped_simplex<K>(an, keep);
}

// Tile of this workgroup, XCD-aware: workgroups go to the eight XCDs in turn (linear id mod 8), and
// each XCD has its own L2.  XCD x takes a contiguous band of the row-major tile order, so a tile's
// ring of neighbouring pixels (written by the previous launch) mostly comes from tiles that ran on
// the same XCD.  A bijection of the linear ids for any tile count.
constexpr int kXcds = 8;
__device__ __forceinline__ int2 xcd_tile() {
    const int nx = gridDim.x, total = gridDim.x * gridDim.y;
    const int id = blockIdx.x + nx * blockIdx.y;
    const int per = (total + kXcds - 1) / kXcds, rem = total % kXcds;
    const int x = id % kXcds, k = id / kXcds;
    const int start = rem == 0 ? x * per : x * (per - 1) + (x < rem ? x : rem);
    const int t = start + k;
    return make_int2(t % nx, t / nx);
}

// An (EY x E cells) x K region with origin (gi0, gj0), read into LDS (row stride E cells; cells
// outside the frame inactive with depth 0) in two halves, so that every load of a kernel's start
// can be issued before the first of them is waited for: region_fetch issues this thread's NR
// rounds of loads into registers, region_store writes them to LDS once they are needed.  The loads are unconditional
// (cells outside the frame or past the region read the nearest frame cell, and region_store
// writes zeros for them): a load under a branch would be waited for inside the branch, and
// after the join the wait counter could no longer tell which loads are still in flight.
// TA: depth and activity; WR: n * alpha.
template <int K, int NR, bool TA, bool WR>
struct RegionRegs {
    float t[NR], a[NR];
    int32_t n[NR];
    uint32_t act[NR];
    bool in[NR];
};

template <int K, int NR, bool TA, bool WR>
__device__ __forceinline__ void region_fetch(RegionRegs<K, NR, TA, WR>& g, int EY, int E, int gi0, int gj0,
                                             const IterArgs& A, const float* __restrict__ t_in,
                                             const float* __restrict__ a_in, const uint8_t* __restrict__ act_in,
                                             const int32_t* __restrict__ n) {
#pragma unroll
    for (int u = 0; u < NR; ++u) {
        const int idx = threadIdx.x + u * blockDim.x;
        const int k = idx % K, cell = idx / K;
        const int gi = gi0 + cell / E, gj = gj0 + cell % E;
        g.in[u] = idx < EY * E * K && gi >= 0 && gi < A.rows && gj >= 0 && gj < A.cols;
        const int gic = min(max(gi, 0), A.rows - 1), gjc = min(max(gj, 0), A.cols - 1);
        const int64_t pc = (int64_t)gic * A.cols + gjc, q = pc * K + k;
        if constexpr (TA) {
            g.t[u] = t_in[q];
            g.act[u] = act_in[q];
        }
        if constexpr (WR) {
            g.a[u] = a_in[q];
            g.n[u] = n[pc];
        }
    }
}

template <int K, int NR, bool TA, bool WR>
__device__ __forceinline__ void region_store(const RegionRegs<K, NR, TA, WR>& g, float* st, uint8_t* sa, float* sr,
                                             int EY, int E) {
#pragma unroll
    for (int u = 0; u < NR; ++u) {
        const int idx = threadIdx.x + u * blockDim.x;
        if (idx < EY * E * K) {
            if constexpr (TA) {
                st[idx] = g.in[u] ? g.t[u] : 0.f;
                sa[idx] = g.in[u] ? (uint8_t)g.act[u] : (uint8_t)0;
            }
            if constexpr (WR) sr[idx] = g.in[u] ? (float)g.n[u] * g.a[u] : 0.f;
        }
    }
}

template <int K, int R>
__global__ __launch_bounds__(kTile * kTile) void depth_denoise_kernel(
    IterArgs A, const float* __restrict__ scal, const float* __restrict__ t_in, const float* __restrict__ a_in,
    const uint8_t* __restrict__ act_in, float* __restrict__ t_out, float* __restrict__ a_out,
    uint8_t* __restrict__ act_out) {
    constexpr int E = kTile + 2 * R;
    __shared__ float s_t[E * E * K];
    __shared__ uint8_t s_a[E * E * K];
    const int2 tile = xcd_tile();
    const int i0 = tile.y * kTile, j0 = tile.x * kTile;
    {
        RegionRegs<K, (E * E * K + kTile * kTile - 1) / (kTile * kTile), true, false> g;
        region_fetch(g, E, E, i0 - R, j0 - R, A, t_in, a_in, act_in, nullptr);
        region_store(g, s_t, s_a, nullptr, E, E);
    }
    __syncthreads();
    const int ti = threadIdx.x / kTile, tj = threadIdx.x % kTile;
    const int i = i0 + ti, j = j0 + tj;
    if (i >= A.rows || j >= A.cols) return;
    const float Tf = (float)A.T, tau_z = scal[3];
    const int pix = i * A.cols + j;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t q = (int64_t)pix * K + k;
        const int c = ((ti + R) * E + (tj + R)) * K + k;
        a_out[q] = a_in[q];
        act_out[q] = s_a[c];
        t_out[q] = s_a[c] ? dd_point<K, R>(s_t, s_a, E, ti + R, tj + R, k, Tf, A.invT, tau_z, A.lambda_z) : s_t[c];
    }
}

template <int K, int R>
__global__ __launch_bounds__(kTile * kTile) void intensity_denoise_kernel(
    IterArgs A, const int32_t* __restrict__ n, const float* __restrict__ scal, const float* __restrict__ t_in,
    const float* __restrict__ a_in, const uint8_t* __restrict__ act_in, float* __restrict__ t_out,
    float* __restrict__ a_out, uint8_t* __restrict__ act_out) {
    constexpr int E = kTile + 2 * R;
    __shared__ float s_t[E * E * K], s_r[E * E * K];
    __shared__ uint8_t s_a[E * E * K];
    const int2 tile = xcd_tile();
    const int i0 = tile.y * kTile, j0 = tile.x * kTile;
    {
        RegionRegs<K, (E * E * K + kTile * kTile - 1) / (kTile * kTile), true, true> g;
        region_fetch(g, E, E, i0 - R, j0 - R, A, t_in, a_in, act_in, n);
        region_store(g, s_t, s_a, s_r, E, E);
    }
    __syncthreads();
    const int ti = threadIdx.x / kTile, tj = threadIdx.x % kTile;
    const int i = i0 + ti, j = j0 + tj;
    if (i >= A.rows || j >= A.cols) return;
    const float Tf = (float)A.T, tau_z = scal[3];
    const int pix = i * A.cols + j;
    float rt[K], an[K];
    bool was[K], keep[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int c = ((ti + R) * E + (tj + R)) * K + k;
        was[k] = s_a[c] != 0;
        rt[k] = was[k] ? id_mean<K, R>(s_t, s_a, s_r, E, ti + R, tj + R, k, Tf, A.invT, tau_z) : 0.f;
        t_out[(int64_t)pix * K + k] = s_t[c];
    }
    id_update<K>(rt, was, (float)n[pix], A.r_min, an, keep);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        a_out[(int64_t)pix * K + k] = an[k];
        act_out[(int64_t)pix * K + k] = keep[k] ? 1 : 0;
    }
}

// One whole iteration for a kIterTY x kIterTX tile: depth denoiser on the tile and an R-pixel ring
// (the ring is recomputed by each neighbouring tile), intensity denoiser on the tile, then
// (DS_NEXT) the next iteration's data step.  Input: the state after a data step; output: the
// state after the next data step (or after the intensity denoiser).  One launch per iteration
// instead of three; four threads per tile pixel so that the data step runs four lanes per pixel
// in one round.  Tiles of 8 x 16 (512 threads) let two or more blocks share a CU, so one block's
// load and barrier waits overlap another's denoiser arithmetic.
//
// DD_DONE: the input is the state after the depth denoiser (depth_denoise_kernel ran first), so
// the tile skips its own depth fits.  With several points per pixel the fit dominates the
// iteration and the ring makes each tile fit 1.9 times its own pixels; the separate launch fits
// each pixel once.  dd_point sees the same inputs either way, so both forms give the same bits.
constexpr int kIterTY = 8, kIterTX = 16;
constexpr int kRsrcFlags = 0x00020000;   // buffer descriptor word 3: raw 32-bit dwords

constexpr int kIterPix = kIterTY * kIterTX;
constexpr int kIterThreads = kIterPix * kLanesPerPixel;


template <int K, int R, bool DS_NEXT, bool DD_DONE>
__global__ __launch_bounds__(kIterThreads) void iteration_kernel(
    IterArgs A, const float* __restrict__ z, const int32_t* __restrict__ n, const float* __restrict__ hhat,
    const float* __restrict__ scal, const float* __restrict__ t_in, const float* __restrict__ a_in,
    const uint8_t* __restrict__ act_in, float* __restrict__ t_out, float* __restrict__ a_out,
    uint8_t* __restrict__ act_out) {
    constexpr int E2 = kIterTX + 4 * R, E1 = kIterTX + 2 * R;        // region widths (row strides)
    constexpr int E2Y = kIterTY + 4 * R, E1Y = kIterTY + 2 * R;      // region heights
    __shared__ float s_t2[E2Y * E2 * K];         // depths after the data step, tile + 2R ring
    __shared__ uint8_t s_a2[E2Y * E2 * K];
    __shared__ float s_td[E1Y * E1 * K];         // depths after the depth denoiser, tile + R ring
    __shared__ float s_r1[E1Y * E1 * K];         // n * alpha after the data step
    __shared__ uint8_t s_a1[E1Y * E1 * K];
    __shared__ float2 s_h[SRT3D_MAX_M_RECON];
    __shared__ float s_ddp[(K == 1 && !DD_DONE && E1Y * E1 <= kIterThreads / 2) ? E1Y * E1 * kDDPart : 1];
    const int2 tile = xcd_tile();
    const int i0 = tile.y * kIterTY, j0 = tile.x * kIterTX;
    // The data step's sketch slice (this thread's pixel and harmonics) is loaded first, into
    // registers, and stays in flight through the denoisers: the barriers below order LDS only.
    const int sub = threadIdx.x % kLanesPerPixel, pl = threadIdx.x / kLanesPerPixel;   // pl < kIterPix
    const int dti = pl / kIterTX, dtj = pl % kIterTX;
    const int dpi = i0 + dti, dpj = j0 + dtj;
    const bool dpix_in = dpi < A.rows && dpj < A.cols;
    const int dpix = dpix_in ? dpi * A.cols + dpj : 0;
    const bool prefetch = DS_NEXT && A.m <= kLanesPerPixel * kPrefetchSlice;
    // Every load of the start goes out before the first wait: the state of the two regions, the
    // IRF spectrum and this pixel's photon count first, the sketch prefetch last, so that the
    // wait before the LDS stores covers the state and the prefetch stays in flight through the
    // denoisers.  Without the stand-alone depth launch before (DD_DONE false) the tile + R
    // region needs only n and alpha: its depths are the depth denoiser's output, and its
    // activity flags are those of the wider region (copied in LDS during the depth phase).
    constexpr int NR2 = (E2Y * E2 * K + kIterThreads - 1) / kIterThreads;
    constexpr int NR1 = (E1Y * E1 * K + kIterThreads - 1) / kIterThreads;
    RegionRegs<K, NR2, true, false> g2;
    RegionRegs<K, NR1, DD_DONE, true> g1;
    if constexpr (!DD_DONE) region_fetch(g2, E2Y, E2, i0 - 2 * R, j0 - 2 * R, A, t_in, a_in, act_in, n);
    region_fetch(g1, E1Y, E1, i0 - R, j0 - R, A, t_in, a_in, act_in, n);
    static_assert(SRT3D_MAX_M_RECON <= kIterThreads, "one harmonic of the spectrum per thread");
    const float2 hreg = reinterpret_cast<const float2*>(hhat)[min((int)threadIdx.x, A.m - 1)];
    const int32_t n_own = n[dpix];                   // (pixel 0 for threads outside the frame: unused)
    float2 zr[kPrefetchSlice];
    if constexpr (DS_NEXT) {
        {   // issued whether or not it is used (m > 32 reads nothing: an empty descriptor)
            // A wave is one tile row of 16 pixels (kIterTX * kLanesPerPixel = 64 lanes).  Its
            // sketch rows are read through a buffer descriptor that starts at the wave's first
            // pixel and ends at the end of z: each lane reads kPrefetchSlice entries from the
            // start of its slice at constant offsets, and reads past the end of z (pixels right
            // of the frame, the frame's last slice) return 0.  Entries beyond the slice are not used.
            static_assert(kIterTX * kLanesPerPixel == kWave, "one tile row per wave");
            const int lo = (sub * A.m) / kLanesPerPixel;
            const int64_t p0 = (int64_t)__builtin_amdgcn_readfirstlane(dpi) * A.cols + j0;
            const int64_t left = (prefetch && p0 < A.P) ? ((int64_t)A.P - p0) * A.m * 8 : 0;
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<float*>(z) + (p0 < A.P ? p0 : 0) * 2 * A.m, (short)0,
                (int)(left < 0x7fffffff ? left : 0x7fffffff), kRsrcFlags);
            const int voff = (dtj * A.m + lo) * 8;
#pragma unroll
            for (int j = 0; j < kPrefetchSlice; ++j)
                zr[j] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, voff + j * 8, 0, 0));
        }
    }
    // the frame constants (depth gate, step sizes) are read before the barrier, so that their
    // scalar loads are not waited for behind it
    const float tau_z = scal[3], gam_t = scal[1], gam_a = scal[2];
    if (DS_NEXT && (int)threadIdx.x < A.m) s_h[threadIdx.x] = hreg;
    if constexpr (!DD_DONE) region_store(g2, s_t2, s_a2, nullptr, E2Y, E2);
    region_store(g1, s_td, s_a1, s_r1, E1Y, E1);
    lds_barrier();
    const float Tf = (float)A.T, invT = A.invT;
    constexpr bool SPLIT_DD = !DD_DONE && K == 1 && E1Y * E1 <= kIterThreads / 2;
    if constexpr (SPLIT_DD) {
        // depth denoiser on the tile + R ring, one cell per thread of each half of the block:
        // waves 0-3 sum window rows -R..0 and pass theirs on through LDS, waves 4-7 sum rows
        // 1..R, add part 0 (the sum is the same either way round) and solve -- the larger part
        // on one side, the solve on the other
        const bool second = threadIdx.x >= kIterThreads / 2;            // uniform per wave
        const int idx = threadIdx.x - (second ? kIterThreads / 2 : 0);
        float M[4][4], b[4];
        bool fit = false;
        float tq = 0.f;
        if (idx < E1Y * E1) {
            const int ci = idx / E1 + R, cj = idx % E1 + R;                // cell in the E2 region
            const int c2 = ci * E2 + cj;
            tq = s_t2[c2];
            fit = s_a2[c2] != 0;
            if (!second) s_a1[idx] = s_a2[c2];                             // read after the barriers
            if (fit) {
                dd_start<K, R>(M, b, !second);
                if (second) {
                    dd_rows<K, R, 1, R>(s_t2, s_a2, E2, ci, cj, tq, Tf, invT, tau_z, M, b);
                } else {
                    dd_rows<K, R, -R, 0>(s_t2, s_a2, E2, ci, cj, tq, Tf, invT, tau_z, M, b);
                    dd_pack(M, b, s_ddp + idx * kDDPart);
                }
            }
        }
        lds_barrier();
        if (second && idx < E1Y * E1) {
            if (fit) {
                dd_add_part(M, b, s_ddp + idx * kDDPart);
                s_td[idx] = dd_solve(M, b, tq, Tf, A.lambda_z);
            } else {
                s_td[idx] = tq;
            }
        }
        lds_barrier();
    } else if constexpr (!DD_DONE) {
        // depth denoiser on the tile + R ring
        for (int idx = threadIdx.x; idx < E1Y * E1 * K; idx += blockDim.x) {
            const int k = idx % K, cell = idx / K;
            const int ci = cell / E1 + R, cj = cell % E1 + R;          // cell in the E2 region
            const int c2 = (ci * E2 + cj) * K + k;
            s_a1[idx] = s_a2[c2];
            if (s_a2[c2]) s_td[idx] = dd_point<K, R>(s_t2, s_a2, E2, ci, cj, k, Tf, invT, tau_z, A.lambda_z);
            else s_td[idx] = s_t2[c2];
        }
        lds_barrier();
    }
    // intensity denoiser, four lanes per pixel (the data step's lanes): each lane sums one part
    // of the window, two shuffles combine them, and every lane holds the pixel's new state
    if (dpix_in) {                                   // the same for the four lanes of a pixel
        const int ti = dti, tj = dtj;
        const int pix = dpix;
        float rt[K], ak[K], tk[K];
        bool was[K], on[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int c = ((ti + R) * E1 + (tj + R)) * K + k;
            was[k] = s_a1[c] != 0;
            tk[k] = s_td[c];
            float nm, dn;
            id_part<K, R>(s_td, s_a1, s_r1, E1, ti + R, tj + R, k, Tf, invT, tau_z, sub, nm, dn);
            nm += quad_xor1(nm);
            dn += quad_xor1(dn);
            nm += quad_xor2(nm);
            dn += quad_xor2(dn);
            rt[k] = was[k] ? id_ratio(nm, dn) : 0.f;
        }
        const float nq = (float)n_own;
        id_update<K>(rt, was, nq, A.r_min, ak, on);
        if constexpr (DS_NEXT) {
            // next data step
            bool any = false;
#pragma unroll
            for (int k = 0; k < K; ++k) any |= on[k];
            if (any) {
                if (prefetch) {
                    const RegSketch<kPrefetchSlice> src{zr, s_h};
                    data_point<K, kPrefetchSlice>(src, sub, A.m, A.T, A.invT, A.twoinvT, nq, gam_t, gam_a, tk, ak,
                                                  on);
                } else {
                    const GlobalSketch src{reinterpret_cast<const float2*>(z + (int64_t)pix * 2 * A.m), s_h};
                    data_point<K, kMaxSlice>(src, sub, A.m, A.T, A.invT, A.twoinvT, nq, gam_t, gam_a, tk, ak, on);
                }
            }
        }
        if (sub == 0) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int64_t q = (int64_t)pix * K + k;
                t_out[q] = tk[k];
                a_out[q] = ak[k];
                act_out[q] = on[k] ? 1 : 0;
            }
        }
    }
}

// ----------------------------------------------------------------------------- finalize
// RB >= 0: the background radius fixed at compile time, the window unrolled and every load
// unconditional (clamped into the frame, outside cells masked out of the sums: adding +0 changes
// nothing), so they are all in flight together; RB < 0: the radius A.Rb at run time.  Both sum
// the same terms in the same order.
template <int K, int RB>
__global__ __launch_bounds__(256) void finalize_kernel(IterArgs A, const int32_t* __restrict__ n,
                                                       const float* __restrict__ t_in,
                                                       const float* __restrict__ a_in,
                                                       const uint8_t* __restrict__ act_in,
                                                       float* __restrict__ depth, float* __restrict__ inten,
                                                       uint8_t* __restrict__ act_out, float* __restrict__ bg) {
    const int pix = blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= A.P) return;
    const int i = pix / A.cols, j = pix - (pix / A.cols) * A.cols;
    // the pixel's own state, loaded with the window's below
    float t_own[K], a_own[K];
    uint32_t act_own[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t q = (int64_t)pix * K + k;
        t_own[k] = t_in[q];
        a_own[k] = a_in[q];
        act_own[k] = act_in[q];
    }
    const int32_t n_own = n[pix];
    if (RB >= 0 && bg) {
        constexpr int W = 2 * (RB > 0 ? RB : 0) + 1;
        float nb[W * W], sa[W * W];
        bool in[W * W];
#pragma unroll
        for (int w = 0; w < W * W; ++w) {
            const int ii = i + w / W - (W / 2), jj = j + w % W - (W / 2);
            in[w] = ii >= 0 && ii < A.rows && jj >= 0 && jj < A.cols;
            const int64_t nbp = (int64_t)min(max(ii, 0), A.rows - 1) * A.cols + min(max(jj, 0), A.cols - 1);
            nb[w] = (float)n[nbp];
            sa[w] = 0.f;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const float av = a_in[nbp * K + k];
                sa[w] += act_in[nbp * K + k] ? av : 0.f;
            }
        }
        float s = 0.f;
        int c = 0;
#pragma unroll
        for (int w = 0; w < W * W; ++w) {
            s += in[w] ? nb[w] * fmaxf(0.f, 1.f - sa[w]) / (float)A.T : 0.f;
            c += in[w] ? 1 : 0;
        }
        bg[pix] = s / (float)c;
    } else if (bg) {
        float s = 0.f;
        int c = 0;
        for (int di = -A.Rb; di <= A.Rb; ++di) {
            const int ii = i + di;
            if (ii < 0 || ii >= A.rows) continue;
            for (int dj = -A.Rb; dj <= A.Rb; ++dj) {
                const int jj = j + dj;
                if (jj < 0 || jj >= A.cols) continue;
                const int64_t nbp = (int64_t)ii * A.cols + jj;
                float sa = 0.f;
#pragma unroll
                for (int k = 0; k < K; ++k)
                    if (act_in[nbp * K + k]) sa += a_in[nbp * K + k];
                s += (float)n[nbp] * fmaxf(0.f, 1.f - sa) / (float)A.T;
                ++c;
            }
        }
        bg[pix] = s / (float)c;
    }
    // slots sorted by depth, inactive last (stable)
    float tk[K], rk[K];
    bool on[K];
    const float nq = (float)n_own;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        on[k] = act_own[k] != 0;
        tk[k] = on[k] ? t_own[k] : 0.f;
        rk[k] = on[k] ? nq * a_own[k] : 0.f;
    }
    for (int a = 1; a < K; ++a)
        for (int b = a; b > 0; --b) {
            const bool swap = (on[b] && !on[b - 1]) || (on[b] && on[b - 1] && tk[b] < tk[b - 1]);
            if (!swap) break;
            const float t0 = tk[b]; tk[b] = tk[b - 1]; tk[b - 1] = t0;
            const float r0 = rk[b]; rk[b] = rk[b - 1]; rk[b - 1] = r0;
            const bool o0 = on[b]; on[b] = on[b - 1]; on[b - 1] = o0;
        }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t q = (int64_t)pix * K + k;
        if (depth) depth[q] = tk[k];
        if (inten) inten[q] = rk[k];
        if (act_out) act_out[q] = on[k] ? 1 : 0;
    }
}

// ----------------------------------------------------------------------------- launchers
static IterArgs make_args(const srt3d_params& p) {
    IterArgs A;
    A.rows = p.rows;
    A.cols = p.cols;
    A.P = p.rows * p.cols;
    A.T = p.T;
    A.m = p.m;
    A.K = p.K_max;
    A.R = p.R;
    A.Rb = p.Rb;
    A.lambda_z = p.lambda_z;
    A.r_min = p.r_min;
    A.invT = 1.0f / (float)p.T;
    A.twoinvT = 2.0f / (float)p.T;
    return A;
}

static inline dim3 pixel_grid(int P, int threads) { return dim3((unsigned)((P + threads - 1) / threads)); }
static inline dim3 tile_grid(const srt3d_params& p) {
    return dim3((unsigned)((p.cols + kTile - 1) / kTile), (unsigned)((p.rows + kTile - 1) / kTile));
}
static inline dim3 iter_grid(const srt3d_params& p) {
    return dim3((unsigned)((p.cols + kIterTX - 1) / kIterTX), (unsigned)((p.rows + kIterTY - 1) / kIterTY));
}

struct InitGrid {
    int stride, G, KS, NT;
};
static InitGrid init_grid(const srt3d_params& p) {
    InitGrid g;
    g.stride = p.init_stride > 0 ? p.init_stride : (p.T / (8 * p.m) > 1 ? p.T / (8 * p.m) : 1);
    g.G = (p.T + g.stride - 1) / g.stride;
    g.KS = (2 * p.m + 3) / 4;
    g.NT = (g.G + 15) / 16;
    return g;
}

// Greedy picks after the first update the correlation kept in LDS (see rho_entry)
// when there are several and it fits: at most 16 column tiles.
static bool init_keeps_correlation(const srt3d_params& p, const InitGrid& g) {
    return p.K_max >= 2 && g.NT <= 16 && g.KS <= 16;
}

// workspace: photon-count maxima of stretches of pixels (kInitWsHead bytes), the grid table
// (B-operand fragments), then the atom's autocorrelation on 16 NT grid lags
constexpr size_t kInitWsHead = (size_t)kInitBlocksMax * sizeof(int) + 256;
constexpr size_t kInitTableLds = 32768;     // largest grid table the init kernel stages in LDS
size_t init_ws_bytes(const srt3d_params& p) {
    const InitGrid g = init_grid(p);
    return kInitWsHead + (size_t)g.NT * g.KS * 64 * sizeof(float) + (size_t)16 * g.NT * sizeof(float);
}

#define SRT3D_BY_K(K_, CALL)                            \
    switch (K_) {                                       \
        case 1: { constexpr int KK = 1; CALL; } break;  \
        case 2: { constexpr int KK = 2; CALL; } break;  \
        default: { constexpr int KK = 3; CALL; } break; \
    }

#define SRT3D_BY_KR(K_, R_, CALL)                                              \
    switch ((K_) * 4 + (R_)) {                                                 \
        case 4: { constexpr int KK = 1, RR = 0; CALL; } break;                 \
        case 5: { constexpr int KK = 1, RR = 1; CALL; } break;                 \
        case 6: { constexpr int KK = 1, RR = 2; CALL; } break;                 \
        case 7: { constexpr int KK = 1, RR = 3; CALL; } break;                 \
        case 8: { constexpr int KK = 2, RR = 0; CALL; } break;                 \
        case 9: { constexpr int KK = 2, RR = 1; CALL; } break;                 \
        case 10: { constexpr int KK = 2, RR = 2; CALL; } break;                \
        case 11: { constexpr int KK = 2, RR = 3; CALL; } break;                \
        case 12: { constexpr int KK = 3, RR = 0; CALL; } break;                \
        case 13: { constexpr int KK = 3, RR = 1; CALL; } break;                \
        case 14: { constexpr int KK = 3, RR = 2; CALL; } break;                \
        default: { constexpr int KK = 3, RR = 3; CALL; } break;                \
    }

hipError_t launch_init(const float* z, const int32_t* n, const double* irf, int irf_len, int irf_origin,
                       const srt3d_params& p, const srt3d_state& st, void* ws, hipStream_t s, bool ds) {
    const int P = p.rows * p.cols;
    const InitGrid g = init_grid(p);
    int* part = reinterpret_cast<int*>(ws);
    float* EB = reinterpret_cast<float*>(reinterpret_cast<char*>(ws) + kInitWsHead);
    const int tab = g.NT * g.KS * 64;
    float* rho = EB + tab;
    const bool keep = init_keeps_correlation(p, g);
    const int tb = (tab + kSetupThreads - 1) / kSetupThreads;
    // counts per thread: at least 16, and few enough stretches for the kInitBlocksMax partials
    const int64_t per_part = (int64_t)kSetupThreads * kInitBlocksMax;
    const int cpt = (int)std::max<int64_t>(16, ((int64_t)P + per_part - 1) / per_part);
    const int nparts = (int)(((int64_t)P + (int64_t)kSetupThreads * cpt - 1) / ((int64_t)kSetupThreads * cpt));
    hipLaunchKernelGGL(frame_setup_kernel, dim3(1 + tb + nparts), dim3(kSetupThreads), 0, s, irf, irf_len, irf_origin,
                       p.T, p.m, p.tau_z, g.stride, g.G, g.KS, g.NT, keep ? 16 * g.NT : 0, tb, n, P, cpt, st.hhat, st.scal,
                       EB, rho, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int cus = 0;
    if ((e = current_device_cus(&cus)) != hipSuccess) return e;
    const int64_t groups = ((int64_t)P + 15) / 16;            // 16 pixels per wave
    const IterArgs A = make_args(p);                           // 1 / T and 2 / T for the fused data step
// one launch of init_kernel<KK, ...> (KK from SRT3D_BY_K): its workgroup size, then the grid
#define SRT3D_INIT_LAUNCH(KSM, RH, EBL, DS)                                                                       \
    {                                                                                                             \
        constexpr int TH = kInitThreads<EBL, RH, KSM, KK, DS>;                                                    \
        int64_t blocks = (groups + TH / 64 - 1) / (TH / 64);                                                      \
        const int64_t cap = std::min<int64_t>((int64_t)cus * (8 * 256 / TH), kInitBlocksMax);                      \
        if (blocks > cap) blocks = cap;                                                                           \
        hipLaunchKernelGGL((init_kernel<KK, KSM, RH, EBL, DS>), dim3((unsigned)blocks), dim3(TH),                  \
                           EBL ? (size_t)tab * sizeof(float) : 0, s, z, n, st.hhat, st.scal, EB, rho, P, p.T, p.m,  \
                           g.stride, g.G, g.KS, g.NT, p.r_min, st.t[0], st.alpha[0], st.active[0], part, nparts,     \
                           p.eta_t, p.eta_a, A);                                                                  \
    }
// The data step runs inside init only for one point per pixel with the grid table in LDS (the
// 1024-thread forms): there it saves a launch; the other forms hold too many registers already
// (fewer waves, and the step's sketch reads then wait in turn), so they are followed by the
// stand-alone data step instead -- the same state either way.
#define SRT3D_INIT(KSM, RH, EBL)                                                                                  \
    SRT3D_BY_K(p.K_max, {                                                                                         \
        if constexpr (KK == 1 && EBL && !RH && KSM <= 8) {                                                        \
            if (ds) SRT3D_INIT_LAUNCH(KSM, RH, EBL, true)                                                         \
            else SRT3D_INIT_LAUNCH(KSM, RH, EBL, false)                                                           \
        } else {                                                                                                  \
            SRT3D_INIT_LAUNCH(KSM, RH, EBL, false)                                                                \
            separate = ds;                                                                                        \
        }                                                                                                         \
    })
    bool separate = false;                          // ds, not fused: the stand-alone data step follows
    const int ksn = g.KS > g.NT ? g.KS : g.NT;     // with the correlation kept, tiles index registers too
    // without the kept correlation, a grid table of up to 32 KB is read from LDS
    const bool ebl = (size_t)tab * sizeof(float) <= kInitTableLds;
    if (keep && ksn <= 4) { SRT3D_INIT(4, true, false); }
    else if (keep && ksn <= 8) { SRT3D_INIT(8, true, false); }
    else if (keep) { SRT3D_INIT(16, true, false); }
    else if (g.KS <= 4) { if (ebl) { SRT3D_INIT(4, false, true); } else { SRT3D_INIT(4, false, false); } }
    else if (g.KS <= 8) { if (ebl) { SRT3D_INIT(8, false, true); } else { SRT3D_INIT(8, false, false); } }
    else if (g.KS <= 16) { if (ebl) { SRT3D_INIT(16, false, true); } else { SRT3D_INIT(16, false, false); } }
    else { SRT3D_INIT(32, false, false); }
#undef SRT3D_INIT
#undef SRT3D_INIT_LAUNCH
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return separate ? launch_data_step(p, z, n, st, 0, s) : hipSuccess;
}

hipError_t launch_data_step(const srt3d_params& p, const float* z, const int32_t* n, const srt3d_state& st,
                            int cur, hipStream_t s) {
    const IterArgs A = make_args(p);
    const dim3 grid((unsigned)(((int64_t)A.P * kLanesPerPixel + 255) / 256));
    SRT3D_BY_K(p.K_max, hipLaunchKernelGGL((data_step_kernel<KK>), grid, dim3(256), 0, s, A, z, n, st.hhat, st.scal, st.t[cur], st.alpha[cur],
                                           st.active[cur]));
    return hipGetLastError();
}

hipError_t launch_smle(const srt3d_params& p, const float* z, const int32_t* n, const srt3d_state& st, int starts,
                       int src, int dst, float* loss, hipStream_t s) {
    const IterArgs A = make_args(p);
    const dim3 grid((unsigned)(((int64_t)A.P * kLanesPerPixel + 255) / 256));
    const bool pref = p.m <= kLanesPerPixel * kPrefetchSlice;
    if (pref) {
        SRT3D_BY_K(p.K_max, hipLaunchKernelGGL((smle_kernel<KK, true>), grid, dim3(256), 0, s, A, starts, p.iters, z, n,
                                               st.hhat, st.scal, st.t[src], st.alpha[src], st.active[src], st.t[dst],
                                               st.alpha[dst], st.active[dst], loss));
    } else {
        SRT3D_BY_K(p.K_max, hipLaunchKernelGGL((smle_kernel<KK, false>), grid, dim3(256), 0, s, A, starts, p.iters, z, n,
                                               st.hhat, st.scal, st.t[src], st.alpha[src], st.active[src], st.t[dst],
                                               st.alpha[dst], st.active[dst], loss));
    }
    return hipGetLastError();
}

hipError_t launch_birth(const srt3d_params& p, const float* z, const int32_t* n, const srt3d_state& st, int cur,
                        hipStream_t s) {
    const IterArgs A = make_args(p);
    const InitGrid g = init_grid(p);
    const dim3 grid((unsigned)((A.P + kBirthThreads - 1) / kBirthThreads));
    SRT3D_BY_K(p.K_max, hipLaunchKernelGGL((birth_kernel<KK>), grid, dim3(kBirthThreads), 0, s, A, g.stride, g.G, z, n,
                                           st.hhat, st.scal, st.t[cur], st.alpha[cur], st.active[cur]));
    return hipGetLastError();
}

hipError_t launch_wsmle(const srt3d_params& p, const double* irf, int irf_len, int irf_origin, const float* z,
                        const int32_t* n, const srt3d_state& st, int half, int witers, float* loss, void* spec,
                        hipStream_t s) {
    const IterArgs A = make_args(p);
    float2* h2 = reinterpret_cast<float2*>(spec);
    hipLaunchKernelGGL(spectrum_kernel, dim3(1), dim3(1024), 0, s, irf, irf_len, irf_origin, p.T, 2 * p.m, h2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
#define SRT3D_WSMLE(M2_)                                                                                            \
    SRT3D_BY_K(p.K_max, hipLaunchKernelGGL((wsmle_kernel<KK, M2_>), dim3((unsigned)((A.P + 4 * (64 / M2_) - 1) /    \
                                           (4 * (64 / M2_)))), dim3(256), 0, s, A, witers, z, n, h2,              \
                                           st.t[half], st.alpha[half], st.active[half], loss))
    if (2 * p.m <= 16) { SRT3D_WSMLE(16); }
    else if (2 * p.m <= 32) { SRT3D_WSMLE(32); }
    else { SRT3D_WSMLE(64); }
#undef SRT3D_WSMLE
    return hipGetLastError();
}

// weighted-SRT3D workspace: n_w (256 bytes), the spectrum to harmonic 2m, then W's packed lower
// triangles [P][w_tri(2m)]
static size_t wsrt_spec_offset() { return 256; }
static size_t wsrt_w_offset(const srt3d_params& p) {
    return wsrt_spec_offset() + (((size_t)2 * p.m * sizeof(float2) + 255) & ~(size_t)255);
}
size_t wsrt_ws_bytes(const srt3d_params& p) {
    return wsrt_w_offset(p) + (size_t)p.rows * p.cols * w_tri(2 * p.m) * sizeof(float);
}

hipError_t launch_wsrt_prepare(const srt3d_params& p, const double* irf, int irf_len, int irf_origin,
                               const int32_t* n, const srt3d_state& st, int half, void* ws, hipStream_t s) {
    const IterArgs A = make_args(p);
    char* w = static_cast<char*>(ws);
    unsigned int* nw = reinterpret_cast<unsigned int*>(w);
    float2* h2 = reinterpret_cast<float2*>(w + wsrt_spec_offset());
    float* Wm = reinterpret_cast<float*>(w + wsrt_w_offset(p));
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(1), 0, s, nw, 0u);
    hipLaunchKernelGGL(spectrum_kernel, dim3(1), dim3(1024), 0, s, irf, irf_len, irf_origin, p.T, 2 * p.m, h2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
#define SRT3D_WPREP(M2_)                                                                                            \
    SRT3D_BY_K(p.K_max, hipLaunchKernelGGL((wprep_kernel<KK, M2_>), dim3((unsigned)((A.P + 4 * (64 / M2_) - 1) /    \
                                           (4 * (64 / M2_)))), dim3(256), 0, s, A, n, h2, st.t[half],             \
                                           st.alpha[half], st.active[half], Wm, nw))
    if (2 * p.m <= 16) { SRT3D_WPREP(16); }
    else if (2 * p.m <= 32) { SRT3D_WPREP(32); }
    else { SRT3D_WPREP(64); }
#undef SRT3D_WPREP
    return hipGetLastError();
}

hipError_t launch_wsrt_data_step(const srt3d_params& p, const float* z, const int32_t* n, const srt3d_state& st,
                                 int half, const void* ws, hipStream_t s) {
    const IterArgs A = make_args(p);
    const char* w = static_cast<const char*>(ws);
    const unsigned int* nw = reinterpret_cast<const unsigned int*>(w);
    const float* Wm = reinterpret_cast<const float*>(w + wsrt_w_offset(p));
    const float2* hh = reinterpret_cast<const float2*>(st.hhat);
#define SRT3D_WDATA(M2_)                                                                                            \
    SRT3D_BY_K(p.K_max, hipLaunchKernelGGL((wdata_kernel<KK, M2_>), dim3((unsigned)((A.P + 4 * (64 / M2_) - 1) /    \
                                           (4 * (64 / M2_)))), dim3(256), 0, s, A, z, n, hh, st.scal, Wm, nw,     \
                                           st.t[half], st.alpha[half], st.active[half]))
    if (2 * p.m <= 16) { SRT3D_WDATA(16); }
    else if (2 * p.m <= 32) { SRT3D_WDATA(32); }
    else { SRT3D_WDATA(64); }
#undef SRT3D_WDATA
    return hipGetLastError();
}

hipError_t launch_depth_denoise(const srt3d_params& p, const srt3d_state& st, int src, int dst, hipStream_t s) {
    const IterArgs A = make_args(p);
    SRT3D_BY_KR(p.K_max, p.R, hipLaunchKernelGGL((depth_denoise_kernel<KK, RR>), tile_grid(p), dim3(kTile * kTile), 0,
                                                 s, A, st.scal, st.t[src], st.alpha[src], st.active[src], st.t[dst],
                                                 st.alpha[dst], st.active[dst]));
    return hipGetLastError();
}

hipError_t launch_intensity_denoise(const srt3d_params& p, const int32_t* n, const srt3d_state& st, int src,
                                    int dst, hipStream_t s) {
    const IterArgs A = make_args(p);
    SRT3D_BY_KR(p.K_max, p.R, hipLaunchKernelGGL((intensity_denoise_kernel<KK, RR>), tile_grid(p),
                                                 dim3(kTile * kTile), 0, s, A, n, st.scal, st.t[src], st.alpha[src],
                                                 st.active[src], st.t[dst], st.alpha[dst], st.active[dst]));
    return hipGetLastError();
}

// Whether an iteration runs as a depth-denoiser launch plus the fused rest or as one launch.
// With several points per pixel the fits dominate and the fused kernel's ring repeats them
// (1.9x at 8x16 tiles, R = 2), which costs more than the second launch on large frames; on
// smaller ones the launches are latency bound and one launch wins.  Measured per 50 iterations
// (fused / split): K = 3, m = 32: 128^2 0.96 / 1.46 ms, 256^2 1.38 / 1.78, 384^2 2.86 / 2.52,
// 512^2 4.44 / 3.67; K = 2, m = 10: 32^2 0.53 / 0.70, 256^2 0.82 / 0.93, 512^2 2.43 / 2.07.
static bool split_iteration(const srt3d_params& p) {
    return p.K_max >= 2 && (int64_t)p.rows * p.cols >= (1 << 17);
}

hipError_t launch_iteration(const srt3d_params& p, const float* z, const int32_t* n, const srt3d_state& st, int src,
                            bool ds_next, hipStream_t s, int* out) {
    const IterArgs A = make_args(p);
    const int dst = 1 - src;
    int in = src, to = dst;
    if (split_iteration(p)) {
        hipError_t e = launch_depth_denoise(p, st, src, dst, s);      // src -> dst, each pixel fitted once
        if (e != hipSuccess) return e;
        in = dst;
        to = src;
    }
#define SRT3D_ITER(DS, DD)                                                                                          \
    SRT3D_BY_KR(p.K_max, p.R, hipLaunchKernelGGL((iteration_kernel<KK, RR, DS, DD>), iter_grid(p), dim3(kIterThreads), \
                                                 0, s, A, z, n, st.hhat, st.scal, st.t[in], st.alpha[in],            \
                                                 st.active[in], st.t[to], st.alpha[to], st.active[to]))
    const bool dd_done = in != src;
    if (ds_next && dd_done) { SRT3D_ITER(true, true); }
    else if (ds_next) { SRT3D_ITER(true, false); }
    else if (dd_done) { SRT3D_ITER(false, true); }
    else { SRT3D_ITER(false, false); }
#undef SRT3D_ITER
    *out = to;
    return hipGetLastError();
}

hipError_t launch_finalize(const srt3d_params& p, const int32_t* n, const srt3d_state& st, float* depth,
                           float* intensity, uint8_t* active, float* bg, hipStream_t s) {
    const IterArgs A = make_args(p);
    const int c = st.cur;
    if (p.Rb == 1)
        SRT3D_BY_K(p.K_max, hipLaunchKernelGGL((finalize_kernel<KK, 1>), pixel_grid(A.P, 256), dim3(256), 0, s, A, n,
                                               st.t[c], st.alpha[c], st.active[c], depth, intensity, active, bg))
    else
    SRT3D_BY_K(p.K_max, hipLaunchKernelGGL((finalize_kernel<KK, -1>), pixel_grid(A.P, 256), dim3(256), 0, s, A, n,
                                           st.t[c], st.alpha[c], st.active[c], depth, intensity, active, bg));
    return hipGetLastError();
}

}  // namespace srt3d
