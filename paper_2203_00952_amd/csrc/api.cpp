// C ABI of libsrt3d: argument validation, workspace carving and launch order.
#include <climits>
#include <cstring>

#include "common.hpp"

using namespace srt3d;

namespace {

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }
inline int dev_status(hipError_t e) { return e == hipSuccess ? SRT3D_OK : SRT3D_EDEVICE; }
inline bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

bool sketch_dims_ok(int32_t T, int32_t m) {
    return T >= 2 && m >= 1 && m <= T / 2 && (int64_t)m * T < (1LL << 31) && (int64_t)T * 8 <= 65536;
}

int check_params(const srt3d_params* p) {
    if (!p) return SRT3D_EINVAL;
    if (p->rows < 1 || p->cols < 1 || (int64_t)p->rows * p->cols > INT_MAX) return SRT3D_EINVAL;
    if (!sketch_dims_ok(p->T, p->m) || p->m > SRT3D_MAX_M_RECON) return SRT3D_EINVAL;
    if (p->K_max < 1 || p->K_max > SRT3D_MAX_K) return SRT3D_EINVAL;
    if (p->R < 0 || p->R > SRT3D_MAX_R || p->Rb < 0 || p->Rb > 8) return SRT3D_EINVAL;
    if (p->iters < 0 || p->init_stride < 0 || p->init_stride >= p->T) return SRT3D_EINVAL;
    if (!(p->eta_t >= 0.f) || !(p->eta_a >= 0.f) || !(p->lambda_z >= 0.f) || !(p->r_min >= 0.f))
        return SRT3D_EINVAL;
    if (p->tau_z != p->tau_z) return SRT3D_EINVAL;   // NaN
    if (p->birth_every < 0) return SRT3D_EINVAL;
    return SRT3D_OK;
}

int check_state(const srt3d_state* st) {
    if (!st) return SRT3D_EINVAL;
    for (int b = 0; b < 2; ++b)
        if (!st->t[b] || !st->alpha[b] || !st->active[b]) return SRT3D_EINVAL;
    if (!st->hhat || !st->scal) return SRT3D_EINVAL;
    if (st->cur != 0 && st->cur != 1) return SRT3D_EINVAL;
    return SRT3D_OK;
}

// Scratch of srt3d_reconstruct_noalloc (the initialisation's workspace), one copy per device.
// Host code never uses the array's name as an address: each device's copy is looked up once with
// hipGetSymbolAddress, with that device current, and kept in scratch_addr.
static __device__ __align__(256) unsigned char scratch[SRT3D_STATIC_SCRATCH_BYTES];
std::atomic<void*> scratch_addr[kMaxDevices];

// Device address of the current device's scratch (write-once cache: concurrent first calls on a
// device store the same address).
hipError_t device_scratch(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    void* ptr = scratch_addr[dev].load(std::memory_order_acquire);
    if (ptr == nullptr) {
        if ((e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch))) != hipSuccess) return e;
        if (ptr == nullptr) return hipErrorInvalidSymbol;
        scratch_addr[dev].store(ptr, std::memory_order_release);
    }
    *out = ptr;
    return hipSuccess;
}

}  // namespace

namespace srt3d {

hipError_t current_device_cus(int* cus) {
    static std::atomic<int> cache[kMaxDevices];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev >= 0 && dev < kMaxDevices) {
        const int v = cache[dev].load(std::memory_order_relaxed);
        if (v > 0) {
            *cus = v;
            return hipSuccess;
        }
    }
    int v = 0;
    if ((e = hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    if (v < 1) v = 1;
    if (dev >= 0 && dev < kMaxDevices) cache[dev].store(v, std::memory_order_relaxed);
    *cus = v;
    return hipSuccess;
}

}  // namespace srt3d

extern "C" {

void srt3d_params_default(srt3d_params* p, int32_t rows, int32_t cols, int32_t T, int32_t m, int32_t K_max) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->rows = rows;
    p->cols = cols;
    p->T = T;
    p->m = m;
    p->K_max = K_max;
    p->iters = 50;
    p->R = 2;
    p->Rb = 1;
    p->init_stride = 0;
    p->eta_t = 1.f;
    p->eta_a = 1.f;
    p->lambda_z = 1.f;
    p->tau_z = 0.f;
    p->r_min = 1.f;
    p->birth_every = 0;
}

namespace {
inline size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }
// the state's arrays in carving order, with their sizes
void state_parts(const srt3d_params& p, size_t (&bytes)[8]) {
    const size_t PK = (size_t)p.rows * p.cols * p.K_max;
    for (int b = 0; b < 4; ++b) bytes[b] = up256(PK * sizeof(float));     // t[0], t[1], alpha[0], alpha[1]
    for (int b = 4; b < 6; ++b) bytes[b] = up256(PK);                      // active[0], active[1]
    bytes[6] = up256((size_t)p.m * 2 * sizeof(float));                    // hhat
    bytes[7] = up256((size_t)SRT3D_NSCAL * sizeof(float));                // scal
}
}  // namespace

size_t srt3d_workspace_bytes(const srt3d_params* p, int32_t P, int32_t which) {
    if (!p || P < 1) return 0;
    switch (which) {
        case SRT3D_CALL_RECONSTRUCT:
            if (check_params(p) != SRT3D_OK || (int64_t)p->rows * p->cols != P) return 0;
            return init_ws_bytes(*p);
        case SRT3D_CALL_SMLE_WEIGHTED:
            if ((int64_t)p->rows * p->cols != P) return 0;
            return srt3d_smle_weighted_workspace_bytes(p);
        case SRT3D_CALL_HIST_FP32:
        case SRT3D_CALL_HIST_FP16X2:
        case SRT3D_CALL_HIST_BF16X3:
            return srt3d_hist_workspace_bytes(p->T, p->m, which - SRT3D_CALL_HIST_FP32);
        case SRT3D_CALL_WEIGHTED_ITERATE:
            if (check_params(p) != SRT3D_OK || (int64_t)p->rows * p->cols != P) return 0;
            if (p->m > SRT3D_MAX_M_WEIGHTED || 2 * p->m >= p->T) return 0;
            return wsrt_ws_bytes(*p);
        default: return 0;   // SRT3D_CALL_SKETCH needs none; anything else is invalid
    }
}

size_t srt3d_state_bytes(const srt3d_params* p, int32_t P) {
    if (check_params(p) != SRT3D_OK || (int64_t)p->rows * p->cols != P) return 0;
    size_t parts[8], total = 0;
    state_parts(*p, parts);
    for (size_t b : parts) total += b;
    return total;
}

int srt3d_state_carve(srt3d_state* st, const srt3d_params* p, void* d_base, size_t bytes) {
    if (!st || check_params(p) != SRT3D_OK || !d_base || !aligned(d_base, 256)) return SRT3D_EINVAL;
    size_t parts[8], total = 0;
    state_parts(*p, parts);
    for (size_t b : parts) total += b;
    if (bytes < total) return SRT3D_ENOMEM;
    char* c = static_cast<char*>(d_base);
    void* ptr[8];
    for (int i = 0; i < 8; ++i) {
        ptr[i] = c;
        c += parts[i];
    }
    st->t[0] = static_cast<float*>(ptr[0]);
    st->t[1] = static_cast<float*>(ptr[1]);
    st->alpha[0] = static_cast<float*>(ptr[2]);
    st->alpha[1] = static_cast<float*>(ptr[3]);
    st->active[0] = static_cast<uint8_t*>(ptr[4]);
    st->active[1] = static_cast<uint8_t*>(ptr[5]);
    st->hhat = static_cast<float*>(ptr[6]);
    st->scal = static_cast<float*>(ptr[7]);
    st->cur = 0;
    return SRT3D_OK;
}

int srt3d_sketch(const int32_t* d_stamps, int64_t N, const int64_t* d_offsets, int32_t P, int32_t T, int32_t m,
                 const float* d_table, float* d_z, int32_t* d_n, double* d_acc, int64_t* d_nacc, int32_t* d_err,
                 void* stream) {
    if (P < 1 || N < 0 || !sketch_dims_ok(T, m)) return SRT3D_EINVAL;
    if ((!d_stamps && N > 0) || !d_offsets || !d_table || !d_z || !d_n) return SRT3D_EINVAL;
    if ((d_acc == nullptr) != (d_nacc == nullptr)) return SRT3D_EINVAL;
    if (!aligned(d_table, 8) || !aligned(d_z, 8)) return SRT3D_EINVAL;
    return dev_status(launch_sketch_photons(d_stamps, N, d_offsets, P, T, m, reinterpret_cast<const float2*>(d_table),
                                            d_z, d_n, d_acc, d_nacc, d_err, as_stream(stream)));
}

int srt3d_sketch_lanes(const int32_t* d_stamps, int64_t N, const int64_t* d_offsets, int32_t P, int32_t T, int32_t m,
                       const float* d_table, float* d_z, int32_t* d_n, double* d_acc, int64_t* d_nacc, int32_t* d_err,
                       int32_t lanes, void* stream) {
    if (lanes != 4 && lanes != 8 && lanes != 16 && lanes != 32 && lanes != 64) return SRT3D_EINVAL;
    if (P < 1 || N < 0 || !sketch_dims_ok(T, m)) return SRT3D_EINVAL;
    if ((!d_stamps && N > 0) || !d_offsets || !d_table || !d_z || !d_n) return SRT3D_EINVAL;
    if ((d_acc == nullptr) != (d_nacc == nullptr)) return SRT3D_EINVAL;
    if (!aligned(d_table, 8) || !aligned(d_z, 8)) return SRT3D_EINVAL;
    return dev_status(launch_sketch_photons(d_stamps, N, d_offsets, P, T, m, reinterpret_cast<const float2*>(d_table),
                                            d_z, d_n, d_acc, d_nacc, d_err, as_stream(stream), lanes));
}

int srt3d_sketch_binned(const int32_t* d_stamps, int64_t N, const int64_t* d_offsets, int32_t P, int32_t T,
                        int32_t m, const float* d_table, float* d_z, int32_t* d_n, double* d_acc, int64_t* d_nacc,
                        int32_t* d_err, void* stream) {
    if (P < 1 || N < 0 || !sketch_dims_ok(T, m) || m > 32) return SRT3D_EINVAL;
    if ((!d_stamps && N > 0) || !d_offsets || !d_table || !d_z || !d_n) return SRT3D_EINVAL;
    if ((d_acc == nullptr) != (d_nacc == nullptr)) return SRT3D_EINVAL;
    if (!aligned(d_table, 8) || !aligned(d_z, 8)) return SRT3D_EINVAL;
    return dev_status(launch_sketch_binned(d_stamps, N, d_offsets, P, T, m, reinterpret_cast<const float2*>(d_table),
                                           d_z, d_n, d_acc, d_nacc, d_err, as_stream(stream)));
}

namespace {
bool events_dims_ok(int64_t N, int32_t P) { return N >= 0 && N <= INT32_MAX && P >= 1 && P <= (1 << 30); }
}  // namespace

size_t srt3d_sketch_events_workspace_bytes(int64_t N, int32_t P) {
    if (!events_dims_ok(N, P)) return 0;
    return events_ws_bytes(N, P);
}

int srt3d_sketch_events(const int32_t* d_pix, const int32_t* d_stamps, int64_t N, int32_t P, int32_t T, int32_t m,
                        const float* d_table, float* d_z, int32_t* d_n, double* d_acc, int64_t* d_nacc,
                        int32_t* d_err, void* d_ws, size_t ws_bytes, void* stream) {
    if (!events_dims_ok(N, P) || !sketch_dims_ok(T, m)) return SRT3D_EINVAL;
    if (((!d_pix || !d_stamps) && N > 0) || !d_table || !d_z || !d_n || !d_ws) return SRT3D_EINVAL;
    if ((d_acc == nullptr) != (d_nacc == nullptr)) return SRT3D_EINVAL;
    if (!aligned(d_table, 8) || !aligned(d_z, 8) || !aligned(d_ws, 256)) return SRT3D_EINVAL;
    if (ws_bytes < events_ws_bytes(N, P)) return SRT3D_ENOMEM;
    return dev_status(launch_sketch_events(d_pix, d_stamps, N, P, T, m, reinterpret_cast<const float2*>(d_table), d_z,
                                           d_n, d_acc, d_nacc, d_err, d_ws, as_stream(stream)));
}

size_t srt3d_hist_workspace_bytes(int32_t T, int32_t m, int32_t precision) {
    if (!sketch_dims_ok(T, m) || m > 32 || precision < 0 || precision > 2) return 0;
    return hist_ws_bytes(T, m, precision);
}

int srt3d_hist_prepare(int32_t T, int32_t m, int32_t precision, void* d_ws, size_t ws_bytes, void* stream) {
    if (!sketch_dims_ok(T, m) || m > 32 || T % 32 != 0) return SRT3D_EINVAL;
    if (precision < SRT3D_PREC_FP32 || precision > SRT3D_PREC_BF16X3) return SRT3D_EINVAL;
    if (!d_ws || !aligned(d_ws, 16)) return SRT3D_EINVAL;
    if (ws_bytes < hist_ws_bytes(T, m, precision)) return SRT3D_ENOMEM;
    return dev_status(launch_hist_prepare(T, m, precision, d_ws, as_stream(stream)));
}

int srt3d_sketch_from_hist(const uint16_t* d_hist, int32_t P, int32_t T, int32_t m, int32_t precision,
                           const void* d_ws, size_t ws_bytes, float* d_z, int32_t* d_n, void* stream) {
    if (P < 1 || !sketch_dims_ok(T, m) || m > 32 || T % 32 != 0) return SRT3D_EINVAL;
    if (precision < SRT3D_PREC_FP32 || precision > SRT3D_PREC_BF16X3) return SRT3D_EINVAL;
    if (!d_hist || !d_z || !d_n || !d_ws) return SRT3D_EINVAL;
    if (!aligned(d_hist, 16) || !aligned(d_ws, 16)) return SRT3D_EINVAL;
    if (ws_bytes < hist_ws_bytes(T, m, precision)) return SRT3D_ENOMEM;
    return dev_status(launch_sketch_hist(d_hist, P, T, m, precision, d_ws, d_z, d_n, as_stream(stream)));
}

size_t srt3d_init_workspace_bytes(const srt3d_params* p) {
    if (check_params(p) != SRT3D_OK) return 0;
    return init_ws_bytes(*p);
}

namespace {
// ds: the first data step of the iterations that follow runs inside the init launch
int init_impl(const float* d_z, const int32_t* d_n, const double* d_irf, int32_t irf_len, int32_t irf_origin,
              const srt3d_params* p, srt3d_state* st, void* d_ws, size_t ws_bytes, void* stream, bool ds) {
    int rc = check_params(p);
    if (rc != SRT3D_OK) return rc;
    if ((rc = check_state(st)) != SRT3D_OK) return rc;
    if (!d_z || !d_n || !d_irf || !d_ws || irf_len < 1 || irf_origin < 0 || irf_origin >= irf_len)
        return SRT3D_EINVAL;
    if (!aligned(d_ws, 16) || !aligned(d_z, 8) || !aligned(st->hhat, 8)) return SRT3D_EINVAL;
    if (ws_bytes < init_ws_bytes(*p)) return SRT3D_ENOMEM;
    st->cur = 0;
    return dev_status(launch_init(d_z, d_n, d_irf, irf_len, irf_origin, *p, *st, d_ws, as_stream(stream), ds));
}
}  // namespace

int srt3d_init(const float* d_z, const int32_t* d_n, const double* d_irf, int32_t irf_len, int32_t irf_origin,
               const srt3d_params* p, srt3d_state* st, void* d_ws, size_t ws_bytes, void* stream) {
    return init_impl(d_z, d_n, d_irf, irf_len, irf_origin, p, st, d_ws, ws_bytes, stream, false);
}

int srt3d_smle(const float* d_z, const int32_t* d_n, const double* d_irf, int32_t irf_len, int32_t irf_origin,
               const srt3d_params* p, int32_t starts, srt3d_state* st, float* d_loss, void* d_ws, size_t ws_bytes,
               void* stream) {
    int rc = check_params(p);
    if (rc != SRT3D_OK) return rc;
    if ((rc = check_state(st)) != SRT3D_OK) return rc;
    if (starts < 1 || starts > SRT3D_MAX_STARTS || !d_loss) return SRT3D_EINVAL;
    if (!d_z || !d_n || !d_irf || !d_ws || irf_len < 1 || irf_origin < 0 || irf_origin >= irf_len)
        return SRT3D_EINVAL;
    if (!aligned(d_ws, 16) || !aligned(d_z, 8) || !aligned(st->hhat, 8) || !aligned(d_loss, 4)) return SRT3D_EINVAL;
    if (ws_bytes < init_ws_bytes(*p)) return SRT3D_ENOMEM;
    const hipStream_t s = as_stream(stream);
    st->cur = 0;
    if (launch_init(d_z, d_n, d_irf, irf_len, irf_origin, *p, *st, d_ws, s) != hipSuccess) return SRT3D_EDEVICE;
    if (launch_smle(*p, d_z, d_n, *st, starts, 0, 1, d_loss, s) != hipSuccess) return SRT3D_EDEVICE;
    st->cur = 1;
    return SRT3D_OK;
}

namespace {
size_t smle_weighted_ws(const srt3d_params& p) {
    return ((init_ws_bytes(p) + 255) & ~(size_t)255) + (size_t)2 * p.m * sizeof(float) * 2;
}
bool weighted_dims_ok(const srt3d_params* p) { return p->m <= SRT3D_MAX_M_WEIGHTED && 2 * p->m < p->T; }
}  // namespace

size_t srt3d_smle_weighted_workspace_bytes(const srt3d_params* p) {
    if (check_params(p) != SRT3D_OK || !weighted_dims_ok(p)) return 0;
    return smle_weighted_ws(*p);
}

int srt3d_weighted_fit(srt3d_state* st, const float* d_z, const int32_t* d_n, const double* d_irf, int32_t irf_len,
                       int32_t irf_origin, const srt3d_params* p, int32_t witers, float* d_loss, void* d_ws,
                       size_t ws_bytes, void* stream) {
    int rc = check_params(p);
    if (rc != SRT3D_OK) return rc;
    if ((rc = check_state(st)) != SRT3D_OK) return rc;
    if (!weighted_dims_ok(p) || witers < 0 || witers > SRT3D_MAX_WITERS || !d_loss) return SRT3D_EINVAL;
    if (!d_z || !d_n || !d_irf || !d_ws || irf_len < 1 || irf_origin < 0 || irf_origin >= irf_len)
        return SRT3D_EINVAL;
    if (!aligned(d_ws, 16) || !aligned(d_z, 8) || !aligned(d_loss, 4)) return SRT3D_EINVAL;
    if (ws_bytes < smle_weighted_ws(*p)) return SRT3D_ENOMEM;
    void* spec = static_cast<char*>(d_ws) + ((init_ws_bytes(*p) + 255) & ~(size_t)255);
    return dev_status(launch_wsmle(*p, d_irf, irf_len, irf_origin, d_z, d_n, *st, st->cur, witers, d_loss, spec,
                                   as_stream(stream)));
}

int srt3d_smle_weighted(const float* d_z, const int32_t* d_n, const double* d_irf, int32_t irf_len,
                        int32_t irf_origin, const srt3d_params* p, int32_t starts, int32_t witers, srt3d_state* st,
                        float* d_loss, void* d_ws, size_t ws_bytes, void* stream) {
    int rc = check_params(p);
    if (rc != SRT3D_OK) return rc;
    if ((rc = check_state(st)) != SRT3D_OK) return rc;
    if (!weighted_dims_ok(p) || witers < 0 || witers > SRT3D_MAX_WITERS) return SRT3D_EINVAL;
    if (starts < 1 || starts > SRT3D_MAX_STARTS || !d_loss) return SRT3D_EINVAL;
    if (!d_z || !d_n || !d_irf || !d_ws || irf_len < 1 || irf_origin < 0 || irf_origin >= irf_len)
        return SRT3D_EINVAL;
    if (!aligned(d_ws, 16) || !aligned(d_z, 8) || !aligned(st->hhat, 8) || !aligned(d_loss, 4)) return SRT3D_EINVAL;
    if (ws_bytes < smle_weighted_ws(*p)) return SRT3D_ENOMEM;
    const hipStream_t s = as_stream(stream);
    void* spec = static_cast<char*>(d_ws) + ((init_ws_bytes(*p) + 255) & ~(size_t)255);
    st->cur = 0;
    if (launch_init(d_z, d_n, d_irf, irf_len, irf_origin, *p, *st, d_ws, s) != hipSuccess) return SRT3D_EDEVICE;
    if (launch_smle(*p, d_z, d_n, *st, starts, 0, 1, d_loss, s) != hipSuccess) return SRT3D_EDEVICE;
    st->cur = 1;
    if (launch_wsmle(*p, d_irf, irf_len, irf_origin, d_z, d_n, *st, 1, witers, d_loss, spec, s) != hipSuccess)
        return SRT3D_EDEVICE;
    return SRT3D_OK;
}

int srt3d_step(srt3d_state* st, const float* d_z, const int32_t* d_n, const srt3d_params* p, int32_t stage,
               void* stream) {
    int rc = check_params(p);
    if (rc != SRT3D_OK) return rc;
    if ((rc = check_state(st)) != SRT3D_OK) return rc;
    if (!d_n || ((stage == SRT3D_STAGE_DATA || stage == SRT3D_STAGE_BIRTH) && !d_z)) return SRT3D_EINVAL;
    hipStream_t s = as_stream(stream);
    const int c = st->cur;
    hipError_t e;
    switch (stage) {
        case SRT3D_STAGE_DATA: e = launch_data_step(*p, d_z, d_n, *st, c, s); break;
        case SRT3D_STAGE_DEPTH: e = launch_depth_denoise(*p, *st, c, 1 - c, s); break;
        case SRT3D_STAGE_INTENSITY: e = launch_intensity_denoise(*p, d_n, *st, c, 1 - c, s); break;
        case SRT3D_STAGE_BIRTH: e = launch_birth(*p, d_z, d_n, *st, c, s); break;
        default: return SRT3D_EINVAL;
    }
    if (e != hipSuccess) return SRT3D_EDEVICE;
    if (stage == SRT3D_STAGE_DEPTH || stage == SRT3D_STAGE_INTENSITY) st->cur = 1 - c;
    return SRT3D_OK;
}

namespace {
// first_done: the first data step already ran (inside the init launch)
int iterate_impl(srt3d_state* st, const float* d_z, const int32_t* d_n, const srt3d_params* p, int32_t iters,
                 void* stream, bool first_done) {
    int rc = check_params(p);
    if (rc != SRT3D_OK) return rc;
    if ((rc = check_state(st)) != SRT3D_OK) return rc;
    if (!d_z || !d_n || iters < 0) return SRT3D_EINVAL;
    if (iters == 0) return SRT3D_OK;
    // data step, then per iteration the depth and intensity denoisers of iteration it and the data
    // step of iteration it + 1 (none after the last): one fused launch, or with several points per
    // pixel a depth-denoiser launch and the fused rest.  With merge/birth stages, an iteration
    // followed by one ends without the data step, which then follows the stage.
    hipStream_t s = as_stream(stream);
    if (!first_done && launch_data_step(*p, d_z, d_n, *st, st->cur, s) != hipSuccess) return SRT3D_EDEVICE;
    for (int it = 0; it < iters; ++it) {
        const bool birth = p->birth_every > 0 && (it + 1) % p->birth_every == 0 && it + 1 < iters;
        int next = st->cur;
        if (launch_iteration(*p, d_z, d_n, *st, st->cur, it + 1 < iters && !birth, s, &next) != hipSuccess)
            return SRT3D_EDEVICE;
        st->cur = next;
        if (birth) {
            if (launch_birth(*p, d_z, d_n, *st, st->cur, s) != hipSuccess) return SRT3D_EDEVICE;
            if (launch_data_step(*p, d_z, d_n, *st, st->cur, s) != hipSuccess) return SRT3D_EDEVICE;
        }
    }
    return SRT3D_OK;
}
}  // namespace

int srt3d_iterate(srt3d_state* st, const float* d_z, const int32_t* d_n, const srt3d_params* p, int32_t iters,
                  void* stream) {
    return iterate_impl(st, d_z, d_n, p, iters, stream, false);
}

namespace {
int check_weighted(const srt3d_params* p, const srt3d_state* st, const void* d_ws, size_t ws_bytes) {
    int rc = check_params(p);
    if (rc != SRT3D_OK) return rc;
    if ((rc = check_state(st)) != SRT3D_OK) return rc;
    if (p->m > SRT3D_MAX_M_WEIGHTED || 2 * p->m >= p->T) return SRT3D_EINVAL;
    if (!d_ws || !aligned(d_ws, 256) || !aligned(st->hhat, 8)) return SRT3D_EINVAL;
    if (ws_bytes < wsrt_ws_bytes(*p)) return SRT3D_ENOMEM;
    return SRT3D_OK;
}
}  // namespace

int srt3d_weighted_prepare(srt3d_state* st, const int32_t* d_n, const double* d_irf, int32_t irf_len,
                           int32_t irf_origin, const srt3d_params* p, void* d_ws, size_t ws_bytes, void* stream) {
    const int rc = check_weighted(p, st, d_ws, ws_bytes);
    if (rc != SRT3D_OK) return rc;
    if (!d_n || !d_irf || irf_len < 1 || irf_origin < 0 || irf_origin >= irf_len) return SRT3D_EINVAL;
    return dev_status(launch_wsrt_prepare(*p, d_irf, irf_len, irf_origin, d_n, *st, st->cur, d_ws, as_stream(stream)));
}

int srt3d_weighted_step(srt3d_state* st, const float* d_z, const int32_t* d_n, const srt3d_params* p,
                        const void* d_ws, size_t ws_bytes, void* stream) {
    const int rc = check_weighted(p, st, d_ws, ws_bytes);
    if (rc != SRT3D_OK) return rc;
    if (!d_z || !d_n || !aligned(d_z, 8)) return SRT3D_EINVAL;
    return dev_status(launch_wsrt_data_step(*p, d_z, d_n, *st, st->cur, d_ws, as_stream(stream)));
}

int srt3d_weighted_iterate(srt3d_state* st, const float* d_z, const int32_t* d_n, const srt3d_params* p,
                           int32_t iters, const void* d_ws, size_t ws_bytes, void* stream) {
    const int rc = check_weighted(p, st, d_ws, ws_bytes);
    if (rc != SRT3D_OK) return rc;
    if (!d_z || !d_n || !aligned(d_z, 8) || iters < 0) return SRT3D_EINVAL;
    hipStream_t s = as_stream(stream);
    const int c = st->cur;
    for (int it = 0; it < iters; ++it) {
        if (launch_wsrt_data_step(*p, d_z, d_n, *st, c, d_ws, s) != hipSuccess) return SRT3D_EDEVICE;
        if (launch_depth_denoise(*p, *st, c, 1 - c, s) != hipSuccess) return SRT3D_EDEVICE;
        if (launch_intensity_denoise(*p, d_n, *st, 1 - c, c, s) != hipSuccess) return SRT3D_EDEVICE;
    }
    return SRT3D_OK;
}

int srt3d_finalize(const srt3d_state* st, const int32_t* d_n, const srt3d_params* p, float* d_depth,
                   float* d_intensity, uint8_t* d_active, float* d_bg, void* stream) {
    int rc = check_params(p);
    if (rc != SRT3D_OK) return rc;
    if ((rc = check_state(st)) != SRT3D_OK) return rc;
    if (!d_n) return SRT3D_EINVAL;
    return dev_status(launch_finalize(*p, d_n, *st, d_depth, d_intensity, d_active, d_bg, as_stream(stream)));
}

int srt3d_reconstruct(const float* d_z, const int32_t* d_n, const double* d_irf, int32_t irf_len,
                      int32_t irf_origin, const srt3d_params* p, srt3d_state* st, float* d_depth,
                      float* d_intensity, uint8_t* d_active, float* d_bg, void* d_ws, size_t ws_bytes,
                      void* stream) {
    // the iterations' first data step runs inside the init launch (one launch fewer; the same state
    // as srt3d_init followed by srt3d_iterate)
    if (!p) return SRT3D_EINVAL;
    const bool fuse = p->iters > 0;
    int rc = init_impl(d_z, d_n, d_irf, irf_len, irf_origin, p, st, d_ws, ws_bytes, stream, fuse);
    if (rc != SRT3D_OK) return rc;
    if ((rc = iterate_impl(st, d_z, d_n, p, p->iters, stream, fuse)) != SRT3D_OK) return rc;
    return srt3d_finalize(st, d_n, p, d_depth, d_intensity, d_active, d_bg, stream);
}

int srt3d_reconstruct_noalloc(const float* d_z, const int32_t* d_n, const double* d_irf, int32_t irf_len,
                              int32_t irf_origin, const srt3d_params* p, srt3d_state* st, float* d_depth,
                              float* d_intensity, uint8_t* d_active, float* d_bg, void* stream) {
    // host-side checks first: a problem too large for the static scratch is refused before any
    // HIP call
    int rc = check_params(p);
    if (rc != SRT3D_OK) return rc;
    if (init_ws_bytes(*p) > (size_t)SRT3D_STATIC_SCRATCH_BYTES) return SRT3D_ESCRATCH;
    if ((rc = check_state(st)) != SRT3D_OK) return rc;
    if (!d_z || !d_n || !d_irf || irf_len < 1 || irf_origin < 0 || irf_origin >= irf_len) return SRT3D_EINVAL;
    void* ws = nullptr;
    if (device_scratch(&ws) != hipSuccess) return SRT3D_EDEVICE;
    return srt3d_reconstruct(d_z, d_n, d_irf, irf_len, irf_origin, p, st, d_depth, d_intensity, d_active, d_bg, ws,
                             (size_t)SRT3D_STATIC_SCRATCH_BYTES, stream);
}

int srt3d_phase_indices(const int32_t* d_x, int64_t N, int32_t T, int32_t m, int32_t* d_k, void* stream) {
    if (N < 0 || !sketch_dims_ok(T, m) || (N > 0 && (!d_x || !d_k))) return SRT3D_EINVAL;
    return dev_status(launch_phase_indices(d_x, N, T, m, d_k, as_stream(stream)));
}

int srt3d_sketch_phases(const int32_t* d_stamps, int64_t N, const int64_t* d_offsets, int32_t P, int32_t T, int32_t m,
                        const float* d_table, float* d_z, int32_t* d_n, int32_t* d_k, void* stream) {
    if (P < 1 || N < 0 || !sketch_dims_ok(T, m)) return SRT3D_EINVAL;
    if ((!d_stamps && N > 0) || (!d_k && N > 0) || !d_offsets || !d_table || !d_z || !d_n) return SRT3D_EINVAL;
    if (!aligned(d_table, 8) || !aligned(d_z, 8)) return SRT3D_EINVAL;
    return dev_status(launch_sketch_photons_export(d_stamps, N, d_offsets, P, T, m,
                                                   reinterpret_cast<const float2*>(d_table), d_z, d_n, d_k,
                                                   as_stream(stream)));
}

int srt3d_phase_table(int32_t T, float* d_table, void* stream) {
    if (T < 2 || (int64_t)T * 8 > 65536 || !d_table || !aligned(d_table, 8)) return SRT3D_EINVAL;
    return dev_status(launch_phase_table(T, reinterpret_cast<float2*>(d_table), as_stream(stream)));
}

const char* srt3d_strerror(int status) {
    switch (status) {
        case SRT3D_OK: return "ok";
        case SRT3D_EINVAL: return "invalid argument";
        case SRT3D_ENOMEM: return "workspace too small";
        case SRT3D_EDEVICE: return "HIP device error";
        case SRT3D_ESCRATCH: return "problem needs more scratch than the static array of srt3d_reconstruct_noalloc";
        default: return "unknown status";
    }
}

int srt3d_version(void) { return SRT3D_VERSION; }

}  // extern "C"
