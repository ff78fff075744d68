/*
 * srt3d.h -- C ABI of the sketched RT3D (SRT3D) library for AMD Instinct MI355X (gfx950).
 *
 * Paper: J. Tachella, M. P. Sheehan, M. E. Davies, "Sketched RT3D: How to reconstruct
 * billions of photons per second", ICASSP 2022 (arXiv 2203.00952).
 *
 * Conventions shared by every entry point
 *  - A pointer named d_* is a device pointer owned by the caller.  The library never
 *    allocates device memory; scratch space comes from a caller-provided workspace whose
 *    size is returned by the matching *_workspace_bytes query.  A pointer named h_* is a
 *    host pointer.
 *  - Every call is asynchronous on the HIP stream passed as `stream` (a hipStream_t cast to
 *    void*, NULL = the null stream).  Argument errors are detected on the host and returned
 *    before anything is enqueued.  A HIP launch failure returns SRT3D_EDEVICE.
 *  - Data-dependent problems are counted on the device into an optional int32 d_err[2]
 *    (may be NULL) that the caller zeroes and reads after synchronising:
 *      d_err[0] += number of stamps outside [0, T) (folded by the mathematical modulus),
 *      d_err[1] += number of pixels whose offsets decrease (treated as empty).
 *  - The library keeps no global mutable state apart from write-once caches of device
 *    properties (compute-unit counts, kernel occupancies); concurrent calls on different streams
 *    with disjoint outputs and workspaces are safe.
 *  - Layouts: a sketch is float32 [P][m][2] (real, imaginary interleaved, harmonic l = 1..m
 *    at index l-1), i.e. complex64 [P][m]; pixels are row-major (p = i * cols + j).
 */
#ifndef SRT3D_H
#define SRT3D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SRT3D_VERSION 1

enum srt3d_status {
    SRT3D_OK = 0,
    SRT3D_EINVAL = -1,   /* invalid argument (sizes, NULL pointers, parameters) */
    SRT3D_ENOMEM = -2,   /* workspace smaller than the matching *_workspace_bytes */
    SRT3D_EDEVICE = -3,  /* a HIP call failed */
    SRT3D_ESCRATCH = -4  /* the problem needs more scratch than srt3d_reconstruct_noalloc's
                            static array holds (SRT3D_STATIC_SCRATCH_BYTES) */
};

/* Arithmetic of the histogram sketch (srt3d_sketch_from_hist). */
enum srt3d_precision {
    SRT3D_PREC_FP32 = 0,   /* FP32 counts x FP32 DFT matrix, FP32 accumulation */
    SRT3D_PREC_FP16X2 = 1, /* counts split exactly into FP16 hi/lo, DFT matrix as a sum of 2 FP16 */
    SRT3D_PREC_BF16X3 = 2  /* counts split exactly into BF16 hi/lo, DFT matrix as a sum of 3 BF16 */
};

/* One stage of an SRT3D iteration (srt3d_step). */
enum srt3d_stage {
    SRT3D_STAGE_DATA = 0,      /* gradient step on depth then intensity, projection */
    SRT3D_STAGE_DEPTH = 1,     /* point-cloud (depth) denoiser */
    SRT3D_STAGE_INTENSITY = 2, /* intensity denoiser and point removal */
    SRT3D_STAGE_BIRTH = 3      /* merge of close points, birth of a point from the residual */
};

/* Limits of the reconstruction kernels. */
#define SRT3D_MAX_M_RECON 64   /* harmonics usable by init/iterate */
#define SRT3D_MAX_K 3          /* surfaces per pixel */
#define SRT3D_MAX_R 3          /* denoiser window radius */
#define SRT3D_MAX_STARTS 64    /* starting points of srt3d_smle */
#define SRT3D_MAX_M_WEIGHTED 32 /* harmonics usable by srt3d_smle_weighted */
#define SRT3D_MAX_WITERS 1000  /* weighted-fit iterations of srt3d_smle_weighted */
#define SRT3D_NSCAL 8          /* floats in srt3d_state.scal */

/*
 * Reconstruction parameters.  Section 3 fixes the data term (eq. 8 with W = I); the
 * initialisation, step sizes, denoisers and thresholds are left open by the paper and are
 * exposed here.  Fill with srt3d_params_default and override fields as needed.
 */
typedef struct srt3d_params {
    int32_t rows, cols;   /* frame size in pixels; P = rows * cols */
    int32_t T;            /* number of time bins; stamps live in [0, T) */
    int32_t m;            /* harmonics l = 1..m, w_l = 2 pi l / T */
    int32_t K_max;        /* surfaces per pixel, 1..SRT3D_MAX_K */
    int32_t iters;        /* iterations run by srt3d_reconstruct */
    int32_t R;            /* denoiser window radius (default 2) */
    int32_t Rb;           /* background box-filter radius (default 1) */
    int32_t init_stride;  /* grid step of the initial search; 0 = max(1, T / (8 m)) */
    float eta_t;          /* depth step scale (default 1) */
    float eta_a;          /* intensity step scale (default 1) */
    float lambda_z;       /* depth-denoiser relaxation (default 1) */
    float tau_z;          /* depth gate in bins; <= 0 = 3 x std of the impulse response */
    float r_min;          /* photons below which a point is removed (default 1) */
    int32_t birth_every;  /* iterations between merge/birth stages in srt3d_iterate; 0 = none
                             (default) */
} srt3d_params;

/*
 * Reconstruction state, all arrays caller-allocated on the device.
 *   t[b], alpha[b], active[b] : b = 0, 1 ping-pong halves, each [P][K_max] (point p*K_max + k)
 *   hhat  : float32 [m][2], spectrum of the impulse response (written by srt3d_init)
 *   scal  : float32 [SRT3D_NSCAL]: [0] max photon count n_max, [1] gamma_t, [2] gamma_alpha,
 *           [3] depth gate tau_z (all written by srt3d_init)
 *   cur   : index of the half that holds the current state; every call that advances the
 *           state updates it on the host (the value is known at enqueue time).
 * t is in bins on [0, T), alpha is the probability of each surface (eq. 1), active is 0/1.
 */
typedef struct srt3d_state {
    float* t[2];
    float* alpha[2];
    uint8_t* active[2];
    float* hhat;
    float* scal;
    int32_t cur;
} srt3d_state;

/* Defaults for the fields the paper leaves open (see srt3d_params). */
void srt3d_params_default(srt3d_params* p, int32_t rows, int32_t cols, int32_t T, int32_t m,
                          int32_t K_max);

/* Calls whose workspace size srt3d_workspace_bytes reports. */
enum srt3d_call {
    SRT3D_CALL_SKETCH = 0,         /* srt3d_sketch, srt3d_sketch_binned: no workspace (0 bytes) */
    SRT3D_CALL_RECONSTRUCT = 1,    /* srt3d_init, srt3d_reconstruct, srt3d_smle */
    SRT3D_CALL_SMLE_WEIGHTED = 2,  /* srt3d_smle_weighted, srt3d_weighted_fit */
    SRT3D_CALL_HIST_FP32 = 3,      /* srt3d_hist_prepare / srt3d_sketch_from_hist, by precision */
    SRT3D_CALL_HIST_FP16X2 = 4,
    SRT3D_CALL_HIST_BF16X3 = 5,
    SRT3D_CALL_WEIGHTED_ITERATE = 6 /* srt3d_weighted_prepare, _step, _iterate */
};

/* ---------------------------------------------------------------------------------------
 * Sizes of the caller-owned device memory.
 * srt3d_workspace_bytes: the workspace of call `which` (srt3d_call) for the frame of p (p->T,
 *   p->m and, for the reconstruction calls, the whole of p) with P pixels.  P must equal
 *   p->rows * p->cols for SRT3D_CALL_RECONSTRUCT and SRT3D_CALL_SMLE_WEIGHTED; the sketch and
 *   histogram calls read only p->T and p->m.  Returns 0 for invalid arguments (also for
 *   SRT3D_CALL_SKETCH, which needs none).  The event-stream sketch's workspace depends on the
 *   number of events: srt3d_sketch_events_workspace_bytes.
 * srt3d_state_bytes: one device allocation that holds every array of srt3d_state for p (with
 *   P = p->rows * p->cols pixels), each array starting on a 256-byte boundary; 0 when invalid.
 * srt3d_state_carve: points st's arrays into such an allocation d_base of `bytes` bytes
 *   (256-byte aligned) and sets st->cur = 0.  Host arithmetic only: nothing is enqueued.
 *   Layout, in order: t[0], t[1], alpha[0], alpha[1] (float32 [P * K_max] each), active[0],
 *   active[1] (uint8 [P * K_max] each), hhat (float32 [m][2]), scal (float32 [SRT3D_NSCAL]).
 * ------------------------------------------------------------------------------------- */
size_t srt3d_workspace_bytes(const srt3d_params* p, int32_t P, int32_t which);
size_t srt3d_state_bytes(const srt3d_params* p, int32_t P);
int srt3d_state_carve(srt3d_state* st, const srt3d_params* p, void* d_base, size_t bytes);

/* ---------------------------------------------------------------------------------------
 * Phase table -- the frequencies of Section 2, w_l = 2 pi l / T, evaluated at integer phases:
 *     d_table[k] = (cos, sin)(2 pi k / T), k = 0..T-1, FP64 values rounded to FP32.
 * Build it once per T and pass it to every srt3d_sketch call with that T.
 *   d_table float32 [T][2], 8-byte aligned.  Constraints: 2 <= T, T * 8 <= 65536.
 * ------------------------------------------------------------------------------------- */
int srt3d_phase_table(int32_t T, float* d_table, void* stream);

/* ---------------------------------------------------------------------------------------
 * Sketch of photon time stamps -- Section 2, eq. (3):
 *     z_l = (1/n) sum_p exp(i w_l x_p),  w_l = 2 pi l / T,  l = 1..m.
 * The phase w_l x_p is reduced exactly as the integer k = (l x_p) mod T and looked up in the
 * phase table; partial sums are FP32 and the division by n is FP64.  One kernel launch.
 *   d_stamps  int32 [N] time stamps, pixel-major (CSR); stamps outside [0, T) are folded
 *             mod T and counted in d_err[0]
 *   N         number of stamps in d_stamps; offsets are clamped to [0, N] before use
 *             (a clamped pixel is counted in d_err[1])
 *   d_offsets int64 [P + 1] pixel p owns stamps [offsets[p], offsets[p+1]); a decreasing pair
 *             makes the pixel empty and is counted in d_err[1]
 *   d_table   float32 [T][2] built by srt3d_phase_table(T)
 *   d_z       float32 [P][m][2] output sketch (8-byte aligned); z = 0 for a pixel with n = 0
 *   d_n       int32 [P] output photon count (of this call, or the accumulated count)
 *   d_acc, d_nacc  optional long-exposure accumulators (both NULL or both set):
 *             double [P][m][2] running sums S_l and int64 [P] running counts; the call adds
 *             this batch (the sketch is updated online with each photon, Section 2) and
 *             writes z = acc / nacc (FP64 division rounded to FP32) and n = min(nacc, INT32_MAX).
 *             The caller zeroes them at the start of an exposure.
 * Constraints: P >= 1, N >= 0, 2 <= T, 1 <= m, m <= T/2 (higher harmonics are conjugates of
 * lower ones), (int64) m * T < 2^31, T * 8 <= 65536 (the table lives in LDS).
 * ------------------------------------------------------------------------------------- */
int srt3d_sketch(const int32_t* d_stamps, int64_t N, const int64_t* d_offsets, int32_t P,
                 int32_t T, int32_t m, const float* d_table, float* d_z, int32_t* d_n,
                 double* d_acc, int64_t* d_nacc, int32_t* d_err, void* stream);

/* ---------------------------------------------------------------------------------------
 * Sketch of photon time stamps through each pixel's unit-bin histogram -- Section 2: the
 * stamps are integer bins, so eq. (3) over the photons equals eq. (3) over the histogram of
 * eq. (2).  Same arguments, outputs, long-exposure accumulators, error counters and
 * constraints as srt3d_sketch, plus m <= 32.  One kernel launch.
 * Each pixel's histogram is built in on-chip memory (8-bit bins; a bin that would pass 255 is
 * detected and its pixel recomputed in chunks of at most 255 photons) and contracted with the
 * DFT columns on the FP16 matrix cores: with x = 64 j + r, the product over r uses an exact
 * two-term FP16 split of exp(i w_l r) and FP32 accumulation, and the sum over j multiplies
 * by exp(i w_l 64 j) from the phase table in FP32.  The per-photon cost is one on-chip
 * integer add, independent of m.  The result differs from srt3d_sketch by rounding only
 * (about 2^-22 of sum |counts| in S before the division by n).
 * ------------------------------------------------------------------------------------- */
int srt3d_sketch_binned(const int32_t* d_stamps, int64_t N, const int64_t* d_offsets, int32_t P,
                        int32_t T, int32_t m, const float* d_table, float* d_z, int32_t* d_n,
                        double* d_acc, int64_t* d_nacc, int32_t* d_err, void* stream);

/* ---------------------------------------------------------------------------------------
 * Sketch of an arrival-order event stream -- Section 2 (the sketch is updated online as each
 * photon arrives) and eq. (3): event e = (d_pix[e], d_stamps[e]) adds exp(i w_l x_e) to its
 * pixel.  The stream is grouped by pixel on the device (a two-level counting sort, by
 * buckets of consecutive pixels and then by pixel, into d_ws) and sketched as by
 * srt3d_sketch_binned (m <= 32) or srt3d_sketch (m > 32); with the binned pass the result does
 * not depend on the order of the events (integer histograms).  Six kernel launches.
 *   d_pix     int32 [N] pixel index of each event; events with an index outside [0, P) are
 *             dropped and counted in d_err[1]
 *   d_stamps  int32 [N] time stamps; stamps outside [0, T) of kept events are folded mod T
 *             and counted in d_err[0]
 *   d_ws      workspace of srt3d_sketch_events_workspace_bytes(N, P) bytes, 256-byte aligned
 *             (bucket tables, CSR offsets, the bucket-grouped and the pixel-grouped stream, about
 *             8 N + 8 P bytes); overwritten by each call
 *   d_table, d_z, d_n, d_acc, d_nacc, d_err: as srt3d_sketch
 * Constraints: as srt3d_sketch, and 0 <= N <= 2^31 - 1, 1 <= P <= 2^30 (longer streams are
 * given in parts with d_acc / d_nacc).  srt3d_sketch_events_workspace_bytes returns 0 outside
 * these; a smaller workspace gives SRT3D_ENOMEM.
 * ------------------------------------------------------------------------------------- */
size_t srt3d_sketch_events_workspace_bytes(int64_t N, int32_t P);
int srt3d_sketch_events(const int32_t* d_pix, const int32_t* d_stamps, int64_t N, int32_t P,
                        int32_t T, int32_t m, const float* d_table, float* d_z, int32_t* d_n,
                        double* d_acc, int64_t* d_nacc, int32_t* d_err, void* d_ws,
                        size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------------------
 * Sketch of per-pixel ToA histograms -- eq. (2) with unit bins [t, t+1), then eq. (3):
 *     S_l = sum_t H[p][t] exp(i w_l t),  n = sum_t H[p][t],  z = S / n,
 * computed as the product H [P x T] . F [T x 2m] with F the cos/sin DFT columns.  Each row is
 * taken in chunks of 32 bins; the chunk's rounded mean count c_k is removed from its counts
 * before the product and added back as sum_k c_k G_k with G_k the sum of F over the chunk (exact
 * integers times FP64 G on the FP64 matrix cores), so the FP32 accumulation only sees
 * deviations from a local level.
 * srt3d_hist_prepare writes F (split for the chosen precision) and G (FP64) into d_ws, of
 * srt3d_hist_workspace_bytes(T, m, precision) bytes; build it once per (T, m, precision).
 * srt3d_sketch_from_hist is then one kernel launch:
 *   d_hist    uint16 [P][T] row-major counts, 16-byte aligned
 *   precision srt3d_precision: FP32 (FP32 matrix cores), FP16X2 or BF16X3 (16-bit matrix
 *             cores on exact hi/lo splits of the counts and a 2- or 3-term split of F,
 *             FP32 accumulation)
 *   d_ws      the prepared F
 *   d_z, d_n  as in srt3d_sketch (n is exact)
 * Constraints: P >= 1, 2 <= T, 1 <= m <= 32, m <= T/2, T % 32 == 0, d_ws 16-byte aligned.
 * ------------------------------------------------------------------------------------- */
size_t srt3d_hist_workspace_bytes(int32_t T, int32_t m, int32_t precision);
int srt3d_hist_prepare(int32_t T, int32_t m, int32_t precision, void* d_ws, size_t ws_bytes,
                       void* stream);
int srt3d_sketch_from_hist(const uint16_t* d_hist, int32_t P, int32_t T, int32_t m,
                           int32_t precision, const void* d_ws, size_t ws_bytes, float* d_z,
                           int32_t* d_n, void* stream);

/* ---------------------------------------------------------------------------------------
 * SRT3D reconstruction -- Section 3, eq. (8) with W = I (the sketched loss
 * n ||z - Phi(theta)||^2, Phi_l = hhat_l sum_k alpha_k exp(i w_l t_k), eq. 4), alternated
 * with point-cloud and intensity denoising as in RT3D.
 *
 * srt3d_init: computes hhat from the impulse response, the frame's n_max and step sizes,
 * and the initial points (greedy sketched matched filter on the grid 0, s, 2s, ...).
 *   d_z, d_n   sketch and counts of the frame ([P][m][2], [P]); P = rows * cols
 *   d_irf      double [irf_len] impulse response h on lags i - irf_origin (device memory)
 *   st         state whose arrays are allocated for p->rows, p->cols, p->m, p->K_max;
 *              st->cur is set to 0
 *   d_ws       workspace of srt3d_init_workspace_bytes(p) bytes
 * srt3d_step:    runs one stage (srt3d_stage) on the current state.
 * srt3d_iterate: runs `iters` full iterations (data, depth, intensity); with
 *   p->birth_every = B > 0, after iteration i (counted from 1 in this call) with i % B == 0 and
 *   i < iters, the merge/birth stage runs before the next data step.
 * Merge/birth stage (RT3D's split and merge of points, cited by Section 3 for scenes with
 *   several surfaces, not described in the paper; in place): active points of a pixel closer
 *   than T/(2m) merge into the lower slot (alpha-weighted circular mean depth, summed alpha);
 *   then a pixel with a free slot and n > 0 takes the peak of the initialisation's matched
 *   filter on its residual z - Phi(theta), over grid points at circular distance >= T/m from
 *   every active point (amplitude max(0, c / sum |hhat|^2)), into its first free slot when
 *   n * amplitude >= r_min; alpha is then projected.
 * srt3d_finalize: background b = n max(0, 1 - sum alpha) / T (box filtered) and the output
 *   points per pixel sorted by depth with inactive slots last:
 *   d_depth, d_intensity float32 [P][K_max] (bins; photons n alpha), d_active uint8 [P][K_max],
 *   d_bg float32 [P] (photons per bin).  Any output pointer may be NULL to skip it.
 * srt3d_reconstruct: init + iterate(p->iters) + finalize, with the same result bit for bit; the
 *   iterations' first data step runs inside the initialisation's launch.
 * Constraints: rows, cols >= 1, 1 <= m <= SRT3D_MAX_M_RECON, m <= T/2, T * 8 <= 65536,
 * 1 <= K_max <= SRT3D_MAX_K, 0 <= R <= SRT3D_MAX_R, 0 <= Rb <= 8, irf_len >= 1,
 * 0 <= irf_origin < irf_len, iters >= 0, eta_t, eta_a >= 0, birth_every >= 0.
 * ------------------------------------------------------------------------------------- */
size_t srt3d_init_workspace_bytes(const srt3d_params* p);
int srt3d_init(const float* d_z, const int32_t* d_n, const double* d_irf, int32_t irf_len,
               int32_t irf_origin, const srt3d_params* p, srt3d_state* st, void* d_ws,
               size_t ws_bytes, void* stream);
int srt3d_step(srt3d_state* st, const float* d_z, const int32_t* d_n, const srt3d_params* p,
               int32_t stage, void* stream);
int srt3d_iterate(srt3d_state* st, const float* d_z, const int32_t* d_n,
                  const srt3d_params* p, int32_t iters, void* stream);
int srt3d_finalize(const srt3d_state* st, const int32_t* d_n, const srt3d_params* p,
                   float* d_depth, float* d_intensity, uint8_t* d_active, float* d_bg,
                   void* stream);
int srt3d_reconstruct(const float* d_z, const int32_t* d_n, const double* d_irf,
                      int32_t irf_len, int32_t irf_origin, const srt3d_params* p,
                      srt3d_state* st, float* d_depth, float* d_intensity, uint8_t* d_active,
                      float* d_bg, void* d_ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------------------
 * srt3d_reconstruct without a workspace argument, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments (less d_ws, ws_bytes), computation and outputs as srt3d_reconstruct; the
 * initialisation's scratch lives in a static device array of SRT3D_STATIC_SCRATCH_BYTES bytes
 * that the library holds on each device it runs on until the process ends.  The call allocates
 * nothing.  It returns SRT3D_ESCRATCH, before enqueueing anything, when
 * srt3d_init_workspace_bytes(p) exceeds that size (every configuration with the default
 * init_stride and T * 8 <= 65536 fits; a small explicit init_stride may not).  Every call on
 * one device shares that device's array: calls that overlap in time on one device (other
 * streams, other host threads) race and must be serialised by the caller.
 * ------------------------------------------------------------------------------------- */
#define SRT3D_STATIC_SCRATCH_BYTES (1u << 20)
int srt3d_reconstruct_noalloc(const float* d_z, const int32_t* d_n, const double* d_irf,
                              int32_t irf_len, int32_t irf_origin, const srt3d_params* p,
                              srt3d_state* st, float* d_depth, float* d_intensity,
                              uint8_t* d_active, float* d_bg, void* stream);

/* ---------------------------------------------------------------------------------------
 * Pixelwise sketched estimator -- the comparison system of Sections 1 and 4 (SMLE): each
 * pixel's loss n ||z - Phi(theta)||^2 (eq. 6 with W = I) minimised on its own, with no
 * spatial prior, from `starts` starting points, keeping the lowest loss.  srt3d_smle runs
 * srt3d_init (its points are start 0), then for start s = 1..starts-1 puts point k at
 * (s T / starts + k T / K_max) mod T with the single-atom least-squares amplitude
 * max(0, Re sum_l conj(hhat_l e^{i w_l t_k}) z_l / sum_l |hhat_l|^2), every point active where
 * n > 0 and alpha projected onto {alpha >= 0, sum alpha <= 1}; each start takes p->iters data
 * steps (srt3d_stage DATA with per-pixel step sizes: the frame's steps scaled by n_max / n;
 * no point is removed).  All starts run in one kernel launch after the initialisation.
 *   d_z, d_n, d_irf, irf_len, irf_origin, p, st, d_ws, ws_bytes: as srt3d_init (workspace of
 *              srt3d_init_workspace_bytes(p) bytes)
 *   starts     1 <= starts <= SRT3D_MAX_STARTS
 *   d_loss     float32 [P]: the chosen start's loss (the earliest start on ties)
 * On return st->cur = 1 holds the chosen points; srt3d_finalize gives the outputs.
 * ------------------------------------------------------------------------------------- */
int srt3d_smle(const float* d_z, const int32_t* d_n, const double* d_irf, int32_t irf_len,
               int32_t irf_origin, const srt3d_params* p, int32_t starts, srt3d_state* st,
               float* d_loss, void* d_ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------------------
 * Eq. (6) with the precision-matrix weighting W = Sigma^{-1} (Section 2, with eq. (5): the
 * sketch is asymptotically normal with covariance Sigma / n), pixel by pixel, as a two-step
 * estimator.  srt3d_smle_weighted runs srt3d_smle (starts, p->iters steps: theta_1), then for
 * each pixel builds Sigma(theta_1), the covariance of the sketch's 2m real coordinates
 * [cos w_l x, sin w_l x] under eq. (1)'s pmf, from the characteristic function at sums and
 * differences of frequencies (eq. 4 at w_a +- w_b, so the impulse response's spectrum up to
 * harmonic 2m), adds 1e-5 tr(Sigma) / (2m) to its diagonal, factors it (L L^T) and runs
 * `witers` Levenberg-Marquardt steps on n ||L^{-1} [Re(z - Phi), Im(z - Phi)]||^2 over the
 * active points (a step kept iff it lowers that loss; mu from 1e-3, / 10 on success down to
 * 1e-7, * 10 on failure up to 1e7; alpha projected, t wrapped).  Points are neither added nor
 * removed.  One segment of 16, 32 or 64 lanes (>= 2m) per pixel.
 *   arguments as srt3d_smle, plus witers (0 <= witers <= SRT3D_MAX_WITERS); the workspace is
 *   srt3d_smle_weighted_workspace_bytes(p) bytes, 16-byte aligned
 *   d_loss     float32 [P]: the weighted loss at the returned points
 * Constraints: as srt3d_smle, and m <= SRT3D_MAX_M_WEIGHTED, 2 m < T.  On return
 * st->cur = 1 holds the points.
 * srt3d_weighted_fit: the second step alone, from the points of the current half (taken as
 *   theta_1), in place; same workspace; st->cur is unchanged.
 * ------------------------------------------------------------------------------------- */
size_t srt3d_smle_weighted_workspace_bytes(const srt3d_params* p);
int srt3d_weighted_fit(srt3d_state* st, const float* d_z, const int32_t* d_n, const double* d_irf,
                       int32_t irf_len, int32_t irf_origin, const srt3d_params* p, int32_t witers,
                       float* d_loss, void* d_ws, size_t ws_bytes, void* stream);
int srt3d_smle_weighted(const float* d_z, const int32_t* d_n, const double* d_irf, int32_t irf_len,
                        int32_t irf_origin, const srt3d_params* p, int32_t starts, int32_t witers,
                        srt3d_state* st, float* d_loss, void* d_ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------------------
 * SRT3D with the precision weighting inside its data step -- eq. (8) with a per-pixel W
 * (Section 2 allows any positive definite W in eq. (6) and names W = Sigma^{-1}, eq. (5), the
 * efficient one; Section 3's SRT3D uses W = I).  W_p = Sigma(theta_0)^{-1} is the inverse of the
 * ridged covariance of the sketch's 2m real coordinates (as in srt3d_smle_weighted) at the
 * pixel's points theta_0, held fixed.  The data step is SRT3D's with the loss n e^T W e,
 * e = [Re(Phi - z), Im(Phi - z)]: t <- t - gamma_t 2 n (J^T W e)_t, then alpha at the new t, then
 * the projection; gamma are the W = I steps of srt3d_init with the frame's n_max replaced by
 * n_w = max_p n_p max_i sum_j |W_p,ij| (a bound of the largest eigenvalue of n_p W_p, equal to
 * c n_max when every W_p = c I, so that case is exactly SRT3D).  The denoisers are SRT3D's.
 * srt3d_weighted_prepare: W_p from the current half of st (normally right after srt3d_init,
 *   whose hhat and scal it needs) and n_w, into d_ws (srt3d_workspace_bytes(p, P,
 *   SRT3D_CALL_WEIGHTED_ITERATE) bytes, 256-byte aligned: per pixel the lower triangle of the
 *   symmetric 2m x 2m W_p by columns, d (d + 1) / 2 floats (d = 2m) rounded up to a multiple of
 *   4); the impulse response as for srt3d_init.
 * srt3d_weighted_step: one weighted data step, in place (st->cur unchanged).
 * srt3d_weighted_iterate: `iters` x (weighted data step, depth denoiser, intensity denoiser);
 *   st->cur is unchanged after each iteration.
 * Constraints: as srt3d_init, and m <= SRT3D_MAX_M_WEIGHTED, 2 m < T.
 * ------------------------------------------------------------------------------------- */
int srt3d_weighted_prepare(srt3d_state* st, const int32_t* d_n, const double* d_irf, int32_t irf_len,
                           int32_t irf_origin, const srt3d_params* p, void* d_ws, size_t ws_bytes,
                           void* stream);
int srt3d_weighted_step(srt3d_state* st, const float* d_z, const int32_t* d_n, const srt3d_params* p,
                        const void* d_ws, size_t ws_bytes, void* stream);
int srt3d_weighted_iterate(srt3d_state* st, const float* d_z, const int32_t* d_n, const srt3d_params* p,
                           int32_t iters, const void* d_ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------------------
 * Inspection entry points used to check the exact part of the sketch and every launch form.
 * srt3d_phase_indices: d_k[(l-1) * N + p] = (l * x_p) mod T (mathematical modulus) for
 *   l = 1..m, the integer phase the sketch kernels use; d_x int32 [N], d_k int32 [m * N].
 * srt3d_sketch_lanes: srt3d_sketch (eq. 3) with the number of lanes that share a pixel fixed
 *   to `lanes` (4, 8, 16, 32 or 64; anything else is SRT3D_EINVAL) instead of chosen from the
 *   mean photon count.  Same arguments, outputs and constraints as srt3d_sketch.
 * srt3d_sketch_phases: the photon pass of srt3d_sketch (eq. 3) at 4 lanes per pixel (the
 *   kernel srt3d_sketch_lanes runs with lanes = 4, so d_z and d_n come out identical to it),
 *   which also writes the integer phase of every table entry it reads: for each photon p inside
 *   some pixel's [offsets[i], offsets[i+1]) and each odd l <= m, d_k[(l-1) * N + p] =
 *   (l * x) mod T, x being the stamp after folding into [0, T).  Even-l entries are not
 *   written: that harmonic is the product of the l-1 entry and the l = 1 entry, so its phase
 *   is their sum.  Entries of photons outside every pixel range are not written either.
 *   d_k: int32 [m * N], device, caller-owned (null only when N = 0); other arguments as
 *   srt3d_sketch without the accumulators and the error counters.
 * ------------------------------------------------------------------------------------- */
int srt3d_phase_indices(const int32_t* d_x, int64_t N, int32_t T, int32_t m, int32_t* d_k,
                        void* stream);
int srt3d_sketch_lanes(const int32_t* d_stamps, int64_t N, const int64_t* d_offsets, int32_t P,
                       int32_t T, int32_t m, const float* d_table, float* d_z, int32_t* d_n,
                       double* d_acc, int64_t* d_nacc, int32_t* d_err, int32_t lanes, void* stream);
int srt3d_sketch_phases(const int32_t* d_stamps, int64_t N, const int64_t* d_offsets, int32_t P,
                        int32_t T, int32_t m, const float* d_table, float* d_z, int32_t* d_n,
                        int32_t* d_k, void* stream);

const char* srt3d_strerror(int status);
int srt3d_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SRT3D_H */
