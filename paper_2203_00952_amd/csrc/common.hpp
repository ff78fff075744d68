// Shared device helpers and the internal launch interface of libsrt3d.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include "srt3d.h"

namespace srt3d {

constexpr int kWave = 64;

// Bytes of the workspace given to the phase table (T float2 entries), 256-byte aligned.
inline size_t table_bytes(int T) { return ((size_t)T * 8 + 255) & ~(size_t)255; }

// Exact phase advance: k <- (k + x) mod T for k, x in [0, T).  The power-of-two form keeps
// a byte offset (k * 8) so the result addresses the float2 table directly.
template <bool POW2>
__device__ __forceinline__ uint32_t phase_advance(uint32_t k8, uint32_t x8, uint32_t T8) {
    if constexpr (POW2) {
        return (k8 + x8) & (T8 - 1u);
    } else {
        uint32_t a = k8 + x8;
        return a >= T8 ? a - T8 : a;
    }
}

// Mathematical modulus of a signed stamp into [0, T).
__device__ __forceinline__ int32_t fold_stamp(int32_t x, int32_t T) {
    int32_t r = x % T;
    return r < 0 ? r + T : r;
}

__device__ __forceinline__ float shfl_xor_f(float v, int mask) { return __shfl_xor(v, mask, kWave); }

// Workgroup barrier ordering on-chip memory only: LDS traffic is complete and visible across it,
// while global loads issued earlier stay in flight.  For kernels whose threads share data only
// through LDS (global inputs read-only, each global output written by one thread).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Device properties the launch shapes depend on, queried once per device and kept for the life of
// the process (write-once caches: concurrent first calls store the same value).
constexpr int kMaxDevices = 64;

// Compute units of the current device.
hipError_t current_device_cus(int* cus);

// Resident workgroups per compute unit of `Kernel` launched with `Threads` threads and no dynamic
// LDS, on the current device (at least 1).
template <auto Kernel, int Threads>
hipError_t cached_occupancy(int* per_cu) {
    static std::atomic<int> cache[kMaxDevices];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev >= 0 && dev < kMaxDevices) {
        const int v = cache[dev].load(std::memory_order_relaxed);
        if (v > 0) {
            *per_cu = v;
            return hipSuccess;
        }
    }
    int v = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, Kernel, Threads, 0);
    if (e != hipSuccess) return e;
    if (v < 1) v = 1;
    if (dev >= 0 && dev < kMaxDevices) cache[dev].store(v, std::memory_order_relaxed);
    *per_cu = v;
    return hipSuccess;
}

// Launch wrappers (defined in the .hip files).  All return hipSuccess or the launch error.
hipError_t launch_phase_table(int T, float2* table, hipStream_t s);
hipError_t launch_phase_indices(const int32_t* x, int64_t N, int T, int m, int32_t* k, hipStream_t s);
// lanes: lanes per pixel (4, 8, 16, 32 or 64), 0 = chosen from the mean photon count
hipError_t launch_sketch_photons(const int32_t* stamps, int64_t N, const int64_t* offsets, int P, int T,
                                 int m, const float2* table, float* z, int32_t* n, double* acc,
                                 int64_t* nacc, int32_t* err, hipStream_t s, int lanes = 0);
// the photon pass (four lanes per pixel) also writing the table index of every harmonic it reads
// from the table: kexp[(l - 1) N + p]
hipError_t launch_sketch_photons_export(const int32_t* stamps, int64_t N, const int64_t* offsets, int P, int T, int m,
                                        const float2* table, float* z, int32_t* n, int32_t* kexp, hipStream_t s);
hipError_t launch_sketch_binned(const int32_t* stamps, int64_t N, const int64_t* offsets, int P, int T,
                                int m, const float2* table, float* z, int32_t* n, double* acc,
                                int64_t* nacc, int32_t* err, hipStream_t s);
size_t events_ws_bytes(int64_t N, int P);
hipError_t launch_sketch_events(const int32_t* pix, const int32_t* stamps, int64_t N, int P, int T, int m,
                                const float2* table, float* z, int32_t* n, double* acc, int64_t* nacc, int32_t* err,
                                void* ws, hipStream_t s);
hipError_t launch_hist_prepare(int T, int m, int precision, void* ws, hipStream_t s);
hipError_t launch_sketch_hist(const uint16_t* hist, int P, int T, int m, int precision, const void* ws,
                              float* z, int32_t* n, hipStream_t s);
size_t hist_ws_bytes(int T, int m, int precision);

// ds: the iteration's first data step runs in the same launch (the state it leaves is that of
// init followed by launch_data_step)
hipError_t launch_init(const float* z, const int32_t* n, const double* irf, int irf_len, int irf_origin,
                       const srt3d_params& p, const srt3d_state& st, void* ws, hipStream_t s, bool ds = false);
hipError_t launch_data_step(const srt3d_params& p, const float* z, const int32_t* n, const srt3d_state& st,
                            int cur, hipStream_t s);
hipError_t launch_smle(const srt3d_params& p, const float* z, const int32_t* n, const srt3d_state& st, int starts,
                       int src, int dst, float* loss, hipStream_t s);
hipError_t launch_wsmle(const srt3d_params& p, const double* irf, int irf_len, int irf_origin, const float* z,
                        const int32_t* n, const srt3d_state& st, int half, int witers, float* loss, void* spec,
                        hipStream_t s);
hipError_t launch_birth(const srt3d_params& p, const float* z, const int32_t* n, const srt3d_state& st, int cur,
                        hipStream_t s);
hipError_t launch_depth_denoise(const srt3d_params& p, const srt3d_state& st, int src, int dst, hipStream_t s);
hipError_t launch_intensity_denoise(const srt3d_params& p, const int32_t* n, const srt3d_state& st, int src,
                                    int dst, hipStream_t s);
hipError_t launch_iteration(const srt3d_params& p, const float* z, const int32_t* n, const srt3d_state& st, int src,
                            bool ds_next, hipStream_t s, int* out);   // *out: the buffer now holding the state
hipError_t launch_finalize(const srt3d_params& p, const int32_t* n, const srt3d_state& st, float* depth,
                           float* intensity, uint8_t* active, float* bg, hipStream_t s);
size_t init_ws_bytes(const srt3d_params& p);
// SRT3D with W_p = Sigma(theta_0)^{-1} in the data step: workspace size, preparation (W_p and the
// frame bound from the current state of half `half`), one weighted data step in place
size_t wsrt_ws_bytes(const srt3d_params& p);
hipError_t launch_wsrt_prepare(const srt3d_params& p, const double* irf, int irf_len, int irf_origin,
                               const int32_t* n, const srt3d_state& st, int half, void* ws, hipStream_t s);
hipError_t launch_wsrt_data_step(const srt3d_params& p, const float* z, const int32_t* n, const srt3d_state& st,
                                 int half, const void* ws, hipStream_t s);

}  // namespace srt3d
