// Sketched RT3D iteration, Section 3: eq. (8) with W = I, alternated with point-cloud and
// intensity denoising (RT3D's plug-and-play scheme).
//
//   frame_constants  hhat_l = sum_i h_i exp(i w_l (i - o)) / sum h (eq. 4), n_max, step sizes,
//                    depth gate (one workgroup, FP64)
//   init             greedy sketched matched filter on the grid tau = 0, s, 2s, ...: one wave
//                    per pixel, lanes over grid points, exact phases (l tau) mod T from an LDS
//                    table
//   data_step        per pixel: residual e = Phi - z, depth step, residual at the new depths,
//                    intensity step, projection onto {alpha >= 0, sum alpha <= 1} (eq. 1);
//                    streams over harmonics so no per-harmonic arrays are kept
//   depth_denoise    per point: weighted least-squares height-field fit over a gated
//                    (2R+1)^2 window (4x4 Cholesky, plane and mean fallbacks)
//   intensity_denoise per point: gated weighted mean of n * alpha, removal below r_min
//   finalize         background n * max(0, 1 - sum alpha) / T with a box filter, output
//                    points sorted by depth
// Every kernel writes only its own pixels; denoisers read one buffer and write the other.
#include "common.hpp"

namespace srt3d {

constexpr int kMaxW = (2 * SRT3D_MAX_R + 1) * (2 * SRT3D_MAX_R + 1);
constexpr float kCholEps = 1e-5f;   // pivot <= kCholEps * trace counts as singular

struct IterArgs {
    int rows, cols, P, T, m, K, R, Rb;
    float lambda_z, r_min;
    float wgt[kMaxW];   // window weights (1 - (di^2 + dj^2) / (R+1)^2)^4, row-major over (di, dj)
};

// ----------------------------------------------------------------------------- helpers
__device__ __forceinline__ float wrap_t(float t, float Tf) {
    float r = t - Tf * floorf(t / Tf);
    if (r >= Tf) r -= Tf;
    if (r < 0.f) r += Tf;
    if (r >= Tf) r = 0.f;
    return r;
}

__device__ __forceinline__ float circ_diff(float d, float Tf) {
    float r = wrap_t(d, Tf);
    return r > 0.5f * Tf ? r - Tf : r;
}

// exp(i w_l t) with the phase (l t) mod T reduced through the integer part of t.
__device__ __forceinline__ float2 phasor(int l, float t, int T) {
    const float ft = floorf(t);
    const int it = (int)ft;
    const float fr = t - ft;
    const int k = (int)(((int64_t)l * it) % T);
    const float ph = (float)k + (float)l * fr;
    const float x = (2.0f * ph) / (float)T;
    float s, c;
    sincospif(x, &s, &c);
    return make_float2(c, s);
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

// ----------------------------------------------------------------------------- frame constants
// scal: [0] n_max, [1] gamma_t, [2] gamma_alpha, [3] tau_z, [4] sum |hhat|^2
__global__ __launch_bounds__(256) void frame_constants_kernel(const int32_t* __restrict__ n, int P,
                                                              const double* __restrict__ irf, int irf_len,
                                                              int origin, int T, int m, int K, float eta_t,
                                                              float eta_a, float tau_z_param,
                                                              float* __restrict__ hhat_out,
                                                              float* __restrict__ scal) {
    __shared__ int s_max[256];
    __shared__ double s_e2[256], s_et[256];
    __shared__ double s_h[3][256];
    const int tid = threadIdx.x;
    int mx = 0;
    for (int p = tid; p < P; p += blockDim.x) mx = max(mx, n[p]);
    s_max[tid] = mx;
    // impulse response moments: sum h, sum h*lag, sum h*lag^2
    double h0 = 0, h1 = 0, h2 = 0;
    for (int i = tid; i < irf_len; i += blockDim.x) {
        const double lag = (double)(i - origin);
        h0 += irf[i];
        h1 += irf[i] * lag;
        h2 += irf[i] * lag * lag;
    }
    s_h[0][tid] = h0;
    s_h[1][tid] = h1;
    s_h[2][tid] = h2;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) {
            s_max[tid] = max(s_max[tid], s_max[tid + o]);
            s_h[0][tid] += s_h[0][tid + o];
            s_h[1][tid] += s_h[1][tid + o];
            s_h[2][tid] += s_h[2][tid + o];
        }
        __syncthreads();
    }
    const double H = s_h[0][0];
    double e2 = 0, et = 0;
    if (tid < m) {
        const int l = tid + 1;
        double re = 0, im = 0;
        for (int i = 0; i < irf_len; ++i) {
            int64_t k = ((int64_t)l * (i - origin)) % T;
            if (k < 0) k += T;
            double s, c;
            sincospi(2.0 * (double)k / (double)T, &s, &c);
            re += irf[i] * c;
            im += irf[i] * s;
        }
        re /= H;
        im /= H;
        hhat_out[2 * tid] = (float)re;
        hhat_out[2 * tid + 1] = (float)im;
        const double w = 2.0 * M_PI * (double)l / (double)T;
        e2 = re * re + im * im;
        et = w * w * e2;
    }
    s_e2[tid] = e2;
    s_et[tid] = et;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) {
            s_e2[tid] += s_e2[tid + o];
            s_et[tid] += s_et[tid + o];
        }
        __syncthreads();
    }
    if (tid == 0) {
        const double nmax = (double)s_max[0];
        const double mu = s_h[1][0] / H;
        const double var = s_h[2][0] / H - mu * mu;
        const double sigma = sqrt(var > 0 ? var : 0.0);
        scal[0] = (float)nmax;
        scal[1] = nmax > 0 ? (float)(eta_t / (2.0 * nmax * s_et[0])) : 0.f;
        scal[2] = nmax > 0 ? (float)(eta_a / (2.0 * nmax * K * s_e2[0])) : 0.f;
        scal[3] = tau_z_param > 0 ? tau_z_param : (float)(3.0 * sigma);
        scal[4] = (float)s_e2[0];
        for (int i = 5; i < SRT3D_NSCAL; ++i) scal[i] = 0.f;
    }
}

// ----------------------------------------------------------------------------- init
// One wave per pixel.  c(tau_g) = Re sum_l conj(hhat_l) w_l exp(-i w_l tau_g).
template <int K>
__global__ __launch_bounds__(256) void init_kernel(const float* __restrict__ z, const int32_t* __restrict__ n,
                                                   const float2* __restrict__ table, const float* __restrict__ hhat,
                                                   const float* __restrict__ scal, int P, int T, int m, int stride,
                                                   float r_min, float* __restrict__ t_out,
                                                   float* __restrict__ a_out, uint8_t* __restrict__ act_out) {
    extern __shared__ float2 s_mem[];
    float2* s_table = s_mem;                       // T entries
    float2* s_y = s_mem + T;                       // 4 waves x SRT3D_MAX_M_RECON
    for (int i = threadIdx.x; i < T; i += blockDim.x) s_table[i] = table[i];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    float2* y = s_y + wv * SRT3D_MAX_M_RECON;
    const int G = (T + stride - 1) / stride;
    const float e2 = scal[4];
    const uint32_t T8 = (uint32_t)T << 3;
    const bool pow2 = (T & (T - 1)) == 0;
    const int waves_total = gridDim.x * (blockDim.x >> 6);

    for (int pix = blockIdx.x * (blockDim.x >> 6) + wv; pix < P; pix += waves_total) {
        // working sketch w_l, one harmonic per lane (m <= 64)
        float2 wl = make_float2(0.f, 0.f), hl = make_float2(0.f, 0.f);
        if (lane < m) {
            wl = reinterpret_cast<const float2*>(z + (int64_t)pix * 2 * m)[lane];
            hl = reinterpret_cast<const float2*>(hhat)[lane];
        }
        const int np = n[pix];
        int tau[K];
        float amp[K];
        for (int k = 0; k < K; ++k) {
            // y_l = conj(hhat_l) * w_l
            if (lane < m) y[lane] = make_float2(hl.x * wl.x + hl.y * wl.y, hl.x * wl.y - hl.y * wl.x);
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            float best = -INFINITY;
            int bestg = 0x7fffffff;
            for (int g = lane; g < G; g += 64) {
                const int tg = g * stride;
                bool excl = false;
                for (int j = 0; j < k; ++j) {
                    int d = tg - tau[j];
                    d = d < 0 ? -d : d;
                    d = min(d, T - d);
                    excl |= (int64_t)d * m < (int64_t)T;
                }
                if (excl) continue;
                const uint32_t x8 = (uint32_t)tg << 3;
                uint32_t k8 = 0;
                float c = 0.f;
                for (int l = 0; l < m; ++l) {
                    k8 = pow2 ? phase_advance<true>(k8, x8, T8) : phase_advance<false>(k8, x8, T8);
                    const float2 cs = *reinterpret_cast<const float2*>(reinterpret_cast<const char*>(s_table) + k8);
                    const float2 yl = y[l];
                    c += yl.x * cs.x + yl.y * cs.y;   // Re(y e^{-i theta})
                }
                if (c > best) {               // g increases per lane, so ties keep the smaller g
                    best = c;
                    bestg = g;
                }
            }
            // wave argmax: larger c, then smaller g
            for (int o = 32; o > 0; o >>= 1) {
                const float ob = __shfl_xor(best, o, 64);
                const int og = __shfl_xor(bestg, o, 64);
                if (ob > best || (ob == best && og < bestg)) {
                    best = ob;
                    bestg = og;
                }
            }
            const float a = (bestg == 0x7fffffff) ? 0.f : fmaxf(0.f, best / e2);
            const int tk = (bestg == 0x7fffffff) ? 0 : bestg * stride;
            tau[k] = tk;
            amp[k] = a;
            // w_l -= a * hhat_l * exp(i w_l tau)
            if (lane < m) {
                const uint32_t kk = (uint32_t)(((int64_t)(lane + 1) * tk) % T);
                const float2 cs = s_table[kk];
                const float2 g = cmul(hl, cs);
                wl.x -= a * g.x;
                wl.y -= a * g.y;
            }
            __builtin_amdgcn_wave_barrier();
        }
        if (lane == 0) {
            bool all[K];
#pragma unroll
            for (int k = 0; k < K; ++k) all[k] = true;
            project_capped_simplex<K>(amp, all);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const bool on = np > 0 && (float)np * amp[k] >= r_min;
                t_out[(int64_t)pix * K + k] = (float)tau[k];
                a_out[(int64_t)pix * K + k] = on ? amp[k] : 0.f;
                act_out[(int64_t)pix * K + k] = on ? 1 : 0;
            }
        }
    }
}

// ----------------------------------------------------------------------------- data step
template <int K>
__global__ __launch_bounds__(256) void data_step_kernel(IterArgs A, const float* __restrict__ z,
                                                        const int32_t* __restrict__ n,
                                                        const float* __restrict__ hhat,
                                                        const float* __restrict__ scal, float* __restrict__ t,
                                                        float* __restrict__ alpha,
                                                        const uint8_t* __restrict__ active) {
    const int pix = blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= A.P) return;
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
    if (!any) return;
    const float nn = (float)n[pix];
    const float gam_t = scal[1], gam_a = scal[2];
    const float Tf = (float)A.T;
    const float w1 = 6.283185307179586f / Tf;
    const float2* zp = reinterpret_cast<const float2*>(z + (int64_t)pix * 2 * A.m);
    const float2* hp = reinterpret_cast<const float2*>(hhat);

    // pass 1: depth gradient at (t, alpha)
    float gt[K];
    float2 u[K], u1[K];
#pragma unroll
    for (int k = 0; k < K; ++k) gt[k] = 0.f;
    for (int l = 1; l <= A.m; ++l) {
        const float2 h = hp[l - 1];
        const float2 zl = zp[l - 1];
        float2 g[K];
        float2 e = make_float2(-zl.x, -zl.y);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (!on[k]) continue;
            if (l == 1) {
                u1[k] = phasor(1, tk[k], A.T);
                u[k] = u1[k];
            } else if ((l & 7) == 1) {
                u[k] = phasor(l, tk[k], A.T);
            } else {
                u[k] = cmul(u[k], u1[k]);
            }
            g[k] = cmul(h, u[k]);
            e.x += ak[k] * g[k].x;
            e.y += ak[k] * g[k].y;
        }
        const float wl = w1 * (float)l;
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (on[k]) gt[k] += wl * (e.x * g[k].y - e.y * g[k].x);
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (on[k]) tk[k] = wrap_t(tk[k] - gam_t * (-2.f * nn * ak[k] * gt[k]), Tf);

    // pass 2: intensity gradient at (t_new, alpha)
    float ga[K];
#pragma unroll
    for (int k = 0; k < K; ++k) ga[k] = 0.f;
    for (int l = 1; l <= A.m; ++l) {
        const float2 h = hp[l - 1];
        const float2 zl = zp[l - 1];
        float2 g[K];
        float2 e = make_float2(-zl.x, -zl.y);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (!on[k]) continue;
            if (l == 1) {
                u1[k] = phasor(1, tk[k], A.T);
                u[k] = u1[k];
            } else if ((l & 7) == 1) {
                u[k] = phasor(l, tk[k], A.T);
            } else {
                u[k] = cmul(u[k], u1[k]);
            }
            g[k] = cmul(h, u[k]);
            e.x += ak[k] * g[k].x;
            e.y += ak[k] * g[k].y;
        }
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (on[k]) ga[k] += e.x * g[k].x + e.y * g[k].y;
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (on[k]) ak[k] = ak[k] - gam_a * (2.f * nn * ga[k]);
    project_capped_simplex<K>(ak, on);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        t[(int64_t)pix * K + k] = tk[k];
        alpha[(int64_t)pix * K + k] = ak[k];
    }
}

// ----------------------------------------------------------------------------- denoisers
// Solve the d x d system (d = 4 or 3) packed as Ms (upper triangle row-major) by Cholesky with
// the pivot rule; returns false if singular.  Only x[0] is needed.
template <int D>
__device__ __forceinline__ bool chol_x0(const float (&M)[4][4], const float (&b)[4], float& x0) {
    float L[D][D];
    float tr = 0.f;
#pragma unroll
    for (int i = 0; i < D; ++i) tr += M[i][i];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        float s = M[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) s -= L[j][k] * L[j][k];
        if (!(s > kCholEps * tr)) return false;
        L[j][j] = sqrtf(s);
#pragma unroll
        for (int i = j + 1; i < D; ++i) {
            float v = M[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
            L[i][j] = v / L[j][j];
        }
    }
    float y[D], x[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        float v = b[j];
#pragma unroll
        for (int k = 0; k < j; ++k) v -= L[j][k] * y[k];
        y[j] = v / L[j][j];
    }
#pragma unroll
    for (int j = D - 1; j >= 0; --j) {
        float v = y[j];
#pragma unroll
        for (int k = j + 1; k < D; ++k) v -= L[k][j] * x[k];
        x[j] = v / L[j][j];
    }
    x0 = x[0];
    return true;
}

template <int K>
__global__ __launch_bounds__(256) void depth_denoise_kernel(IterArgs A, const float* __restrict__ scal,
                                                            const float* __restrict__ t_in,
                                                            const float* __restrict__ a_in,
                                                            const uint8_t* __restrict__ act_in,
                                                            float* __restrict__ t_out, float* __restrict__ a_out,
                                                            uint8_t* __restrict__ act_out) {
    const int pix = blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= A.P) return;
    const int i = pix / A.cols, j = pix - (pix / A.cols) * A.cols;
    const float Tf = (float)A.T;
    const float tau_z = scal[3];
    const int R = A.R, W = 2 * R + 1;
    for (int k = 0; k < K; ++k) {
        const int64_t q = (int64_t)pix * K + k;
        const float tq = t_in[q];
        const bool on = act_in[q] != 0;
        a_out[q] = a_in[q];
        act_out[q] = act_in[q];
        if (!on) {
            t_out[q] = tq;
            continue;
        }
        float M[4][4] = {}, b[4] = {};
        for (int di = -R; di <= R; ++di) {
            const int ii = i + di;
            if (ii < 0 || ii >= A.rows) continue;
            for (int dj = -R; dj <= R; ++dj) {
                const int jj = j + dj;
                if (jj < 0 || jj >= A.cols) continue;
                const float w = A.wgt[(di + R) * W + (dj + R)];
                const int64_t nb = ((int64_t)ii * A.cols + jj) * K;
                for (int kk = 0; kk < K; ++kk) {
                    if (!act_in[nb + kk]) continue;
                    const float d = circ_diff(t_in[nb + kk] - tq, Tf);
                    if (!(fabsf(d) <= tau_z)) continue;
                    const float phi[4] = {1.f, (float)di, (float)dj, (float)(di * di + dj * dj)};
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        b[r] += w * phi[r] * d;
#pragma unroll
                        for (int c = 0; c < 4; ++c) M[r][c] += w * phi[r] * phi[c];
                    }
                }
            }
        }
        float a;
        if (!chol_x0<4>(M, b, a)) {
            if (!chol_x0<3>(M, b, a)) a = b[0] / (M[0][0] > 0.f ? M[0][0] : 1.f);
        }
        t_out[q] = wrap_t(tq + A.lambda_z * a, Tf);
    }
}

template <int K>
__global__ __launch_bounds__(256) void intensity_denoise_kernel(IterArgs A, const int32_t* __restrict__ n,
                                                                const float* __restrict__ scal,
                                                                const float* __restrict__ t_in,
                                                                const float* __restrict__ a_in,
                                                                const uint8_t* __restrict__ act_in,
                                                                float* __restrict__ t_out,
                                                                float* __restrict__ a_out,
                                                                uint8_t* __restrict__ act_out) {
    const int pix = blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= A.P) return;
    const int i = pix / A.cols, j = pix - (pix / A.cols) * A.cols;
    const float Tf = (float)A.T;
    const float tau_z = scal[3];
    const int R = A.R, W = 2 * R + 1;
    const float nq = (float)n[pix];
    float an[K];
    bool keep[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t q = (int64_t)pix * K + k;
        const float tq = t_in[q];
        t_out[q] = tq;
        keep[k] = false;
        an[k] = 0.f;
        if (!act_in[q]) continue;
        float num = 0.f, den = 0.f;
        for (int di = -R; di <= R; ++di) {
            const int ii = i + di;
            if (ii < 0 || ii >= A.rows) continue;
            for (int dj = -R; dj <= R; ++dj) {
                const int jj = j + dj;
                if (jj < 0 || jj >= A.cols) continue;
                const float w = A.wgt[(di + R) * W + (dj + R)];
                const int64_t nbp = (int64_t)ii * A.cols + jj;
                const float nnb = (float)n[nbp];
                for (int kk = 0; kk < K; ++kk) {
                    const int64_t nb = nbp * K + kk;
                    if (!act_in[nb]) continue;
                    const float d = circ_diff(t_in[nb] - tq, Tf);
                    if (!(fabsf(d) <= tau_z)) continue;
                    num += w * (nnb * a_in[nb]);
                    den += w;
                }
            }
        }
        const float rt = num / (den > 0.f ? den : 1.f);
        if (rt >= A.r_min) {
            keep[k] = true;
            an[k] = rt / (nq > 0.f ? nq : 1.f);
        }
    }
    project_capped_simplex<K>(an, keep);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t q = (int64_t)pix * K + k;
        a_out[q] = an[k];
        act_out[q] = keep[k] ? 1 : 0;
    }
}

// ----------------------------------------------------------------------------- finalize
template <int K>
__global__ __launch_bounds__(256) void finalize_kernel(IterArgs A, const int32_t* __restrict__ n,
                                                       const float* __restrict__ t_in,
                                                       const float* __restrict__ a_in,
                                                       const uint8_t* __restrict__ act_in,
                                                       float* __restrict__ depth, float* __restrict__ inten,
                                                       uint8_t* __restrict__ act_out, float* __restrict__ bg) {
    const int pix = blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= A.P) return;
    const int i = pix / A.cols, j = pix - (pix / A.cols) * A.cols;
    if (bg) {
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
    const float nq = (float)n[pix];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t q = (int64_t)pix * K + k;
        on[k] = act_in[q] != 0;
        tk[k] = on[k] ? t_in[q] : 0.f;
        rk[k] = on[k] ? nq * a_in[q] : 0.f;
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
    const int W = 2 * p.R + 1;
    for (int i = 0; i < kMaxW; ++i) A.wgt[i] = 0.f;
    for (int di = -p.R; di <= p.R; ++di)
        for (int dj = -p.R; dj <= p.R; ++dj) {
            const double r = 1.0 - (double)(di * di + dj * dj) / (double)((p.R + 1) * (p.R + 1));
            A.wgt[(di + p.R) * W + (dj + p.R)] = (float)(r * r * r * r);
        }
    return A;
}

static inline dim3 pixel_grid(int P) { return dim3((unsigned)((P + 255) / 256)); }

size_t init_ws_bytes(const srt3d_params& p) { return table_bytes(p.T); }

#define SRT3D_BY_K(K_, CALL)            \
    switch (K_) {                       \
        case 1: { constexpr int KK = 1; CALL; } break; \
        case 2: { constexpr int KK = 2; CALL; } break; \
        default: { constexpr int KK = 3; CALL; } break; \
    }

hipError_t launch_init(const float* z, const int32_t* n, const double* irf, int irf_len, int irf_origin,
                       const srt3d_params& p, const srt3d_state& st, void* ws, hipStream_t s) {
    const int P = p.rows * p.cols;
    hipLaunchKernelGGL(frame_constants_kernel, dim3(1), dim3(256), 0, s, n, P, irf, irf_len, irf_origin, p.T, p.m,
                       p.K_max, p.eta_t, p.eta_a, p.tau_z, st.hhat, st.scal);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    float2* table = reinterpret_cast<float2*>(ws);
    e = launch_phase_table(p.T, table, s);
    if (e != hipSuccess) return e;
    const int stride = p.init_stride > 0 ? p.init_stride : (p.T / (8 * p.m) > 1 ? p.T / (8 * p.m) : 1);
    const size_t lds = (size_t)p.T * sizeof(float2) + 4 * SRT3D_MAX_M_RECON * sizeof(float2);
    int dev = 0, cus = 0;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const int64_t need = ((int64_t)P + 3) / 4;
    const int64_t cap = (int64_t)cus * 8;
    const unsigned blocks = (unsigned)(need < cap ? need : cap);
    SRT3D_BY_K(p.K_max, hipLaunchKernelGGL((init_kernel<KK>), dim3(blocks), dim3(256), lds, s, z, n, table, st.hhat,
                                           st.scal, P, p.T, p.m, stride, p.r_min, st.t[0], st.alpha[0],
                                           st.active[0]));
    return hipGetLastError();
}

hipError_t launch_data_step(const srt3d_params& p, const float* z, const int32_t* n, const srt3d_state& st,
                            int cur, hipStream_t s) {
    const IterArgs A = make_args(p);
    SRT3D_BY_K(p.K_max, hipLaunchKernelGGL((data_step_kernel<KK>), pixel_grid(A.P), dim3(256), 0, s, A, z, n,
                                           st.hhat, st.scal, st.t[cur], st.alpha[cur], st.active[cur]));
    return hipGetLastError();
}

hipError_t launch_depth_denoise(const srt3d_params& p, const srt3d_state& st, int src, int dst, hipStream_t s) {
    const IterArgs A = make_args(p);
    SRT3D_BY_K(p.K_max, hipLaunchKernelGGL((depth_denoise_kernel<KK>), pixel_grid(A.P), dim3(256), 0, s, A, st.scal,
                                           st.t[src], st.alpha[src], st.active[src], st.t[dst], st.alpha[dst],
                                           st.active[dst]));
    return hipGetLastError();
}

hipError_t launch_intensity_denoise(const srt3d_params& p, const int32_t* n, const srt3d_state& st, int src,
                                    int dst, hipStream_t s) {
    const IterArgs A = make_args(p);
    SRT3D_BY_K(p.K_max, hipLaunchKernelGGL((intensity_denoise_kernel<KK>), pixel_grid(A.P), dim3(256), 0, s, A, n,
                                           st.scal, st.t[src], st.alpha[src], st.active[src], st.t[dst],
                                           st.alpha[dst], st.active[dst]));
    return hipGetLastError();
}

hipError_t launch_finalize(const srt3d_params& p, const int32_t* n, const srt3d_state& st, float* depth,
                           float* intensity, uint8_t* active, float* bg, hipStream_t s) {
    const IterArgs A = make_args(p);
    const int c = st.cur;
    SRT3D_BY_K(p.K_max, hipLaunchKernelGGL((finalize_kernel<KK>), pixel_grid(A.P), dim3(256), 0, s, A, n, st.t[c],
                                           st.alpha[c], st.active[c], depth, intensity, active, bg));
    return hipGetLastError();
}

}  // namespace srt3d
