// HBM bandwidth probes for the benchmark: the achievable ceiling of plain
// streams on this device, next to which the sweeps' achieved bandwidth is
// read.  Three hand-written kernels over one large buffer: a copy, a
// read-only stream and a write-only stream, each with 8- or 16-byte loads per
// lane and non-temporal 8-byte stores (the library writes at most 8 bytes per
// lane and store instruction).  Grid-stride loops over whole elements; the
// byte count must be a multiple of 16.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kThreads = 256;

template <int W>
struct Lane;
template <>
struct Lane<8> {
    typedef uint64_t type;
};
template <>
struct Lane<16> {
    typedef uint4 type;
};

__device__ __forceinline__ void store_nt(uint64_t *p, uint64_t v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void store_nt(uint4 *p, uint4 v) {
    uint64_t *q = reinterpret_cast<uint64_t *>(p);
    __builtin_nontemporal_store((uint64_t(v.y) << 32) | v.x, q);
    __builtin_nontemporal_store((uint64_t(v.w) << 32) | v.z, q + 1);
}
__device__ __forceinline__ uint64_t fold(uint64_t v) { return v; }
__device__ __forceinline__ uint64_t fold(uint4 v) { return (uint64_t(v.x ^ v.z) << 32) | (v.y ^ v.w); }

template <int W>
__global__ void __launch_bounds__(kThreads) k_copy(const typename Lane<W>::type *__restrict__ src,
                                                   typename Lane<W>::type *__restrict__ dst, int64_t n) {
    const int64_t stride = int64_t(gridDim.x) * kThreads;
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += stride) store_nt(dst + i, src[i]);
}

// The fold of everything read is written only if it equals a value the data
// never holds, so the loads stay live without a store per lane.
template <int W>
__global__ void __launch_bounds__(kThreads) k_read(const typename Lane<W>::type *__restrict__ src, int64_t n,
                                                   uint64_t *__restrict__ sink) {
    const int64_t stride = int64_t(gridDim.x) * kThreads;
    uint64_t acc = 0;
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += stride) acc ^= fold(src[i]);
    if (acc == 0x9e3779b97f4a7c15ull) sink[0] = acc;
}

__global__ void __launch_bounds__(kThreads) k_write(uint64_t *__restrict__ dst, int64_t n, uint64_t v) {
    const int64_t stride = int64_t(gridDim.x) * kThreads;
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += stride) store_nt(dst + i, v);
}

int blocks_for(int64_t n, int per_cu) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t want = int64_t(cus) * per_cu, need = (n + kThreads - 1) / kThreads;
    return int(want < need ? want : need);
}

}  // namespace

extern "C" {

// lane: 8 or 16 bytes per load; per_cu: blocks per compute unit.
int hbm_probe_copy(void *dst, const void *src, size_t bytes, int lane, int per_cu, void *stream) {
    if (!dst || !src || bytes % 16 || (lane != 8 && lane != 16) || per_cu < 1) return -1;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (lane == 8) {
        const int64_t n = int64_t(bytes / 8);
        hipLaunchKernelGGL(k_copy<8>, dim3(blocks_for(n, per_cu)), dim3(kThreads), 0, s,
                           static_cast<const uint64_t *>(src), static_cast<uint64_t *>(dst), n);
    } else {
        const int64_t n = int64_t(bytes / 16);
        hipLaunchKernelGGL(k_copy<16>, dim3(blocks_for(n, per_cu)), dim3(kThreads), 0, s,
                           static_cast<const uint4 *>(src), static_cast<uint4 *>(dst), n);
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

// sink: 8 bytes of device memory.
int hbm_probe_read(const void *src, size_t bytes, void *sink, int lane, int per_cu, void *stream) {
    if (!src || !sink || bytes % 16 || (lane != 8 && lane != 16) || per_cu < 1) return -1;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (lane == 8) {
        const int64_t n = int64_t(bytes / 8);
        hipLaunchKernelGGL(k_read<8>, dim3(blocks_for(n, per_cu)), dim3(kThreads), 0, s,
                           static_cast<const uint64_t *>(src), n, static_cast<uint64_t *>(sink));
    } else {
        const int64_t n = int64_t(bytes / 16);
        hipLaunchKernelGGL(k_read<16>, dim3(blocks_for(n, per_cu)), dim3(kThreads), 0, s,
                           static_cast<const uint4 *>(src), n, static_cast<uint64_t *>(sink));
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int hbm_probe_write(void *dst, size_t bytes, int per_cu, void *stream) {
    if (!dst || bytes % 16 || per_cu < 1) return -1;
    const int64_t n = int64_t(bytes / 8);
    hipLaunchKernelGGL(k_write, dim3(blocks_for(n, per_cu)), dim3(kThreads), 0, static_cast<hipStream_t>(stream),
                       static_cast<uint64_t *>(dst), n, 0x0123456789abcdefull);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // extern "C"
