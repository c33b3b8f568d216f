// The compact-state D3Q19 step on one lattice (k_step_compact; its first
// step after an initialisation or a restore reads a pair state) and the
// conversion of a compact state to a pair state (k_expand).  The sweep
// itself, its layout and the reasons for it are in lbcg_compact_sweep.h.
#include "lbcg_compact_sweep.h"

namespace lbcg {

namespace {

// Work items (tile, z chunk), tile-major, dealt to the 8 XCDs in contiguous
// bands (blocks go to XCDs round-robin), so each XCD sweeps a compact band of
// tiles and the ring re-reads mostly hit its L2.  Tiles TX x 8: TX = 64
// (512 threads, one block per CU) or 32 (256 threads, several blocks per CU,
// each with its own barrier).  S: storage of the state (float or _Float16).
template <bool PAIR_IN, int TX, typename S>
__global__ void __launch_bounds__(TX * kCR) k_step_compact(CompactArgs a, Model<float> mo) {
    extern __shared__ float lds[];
    const int total = a.ntx * a.nty * a.zchunks;
    const int xcd = blockIdx.x % kCXCD, l = blockIdx.x / kCXCD;
    const int item = xcd * (total / kCXCD) + min(xcd, total % kCXCD) + l;
    if (item == 0 && threadIdx.x == 0) *a.ctr_out = *a.ctr_in + 1u;
    if (PAIR_IN)
        sweep_pairs<TX, S>(a, mo, item / a.zchunks, item % a.zchunks, lds);
    else
        sweep_compact<true, TX, S>(a, mo, item / a.zchunks, item % a.zchunks, lds);
}

// Pair state of nodes [0, N) from a compact state: each population's
// minority colour part M f_i + (c_i . V_c) / 36 (the split the receiver
// makes), as a share of f_i, with the flag of the colour it belongs to.
template <typename S>
__global__ void k_expand(const uint8_t *__restrict__ cin, typename PairOf<S>::type *__restrict__ pout, int64_t N,
                         int64_t pitch) {
    using L = D3Q19;
    typedef CStore<S> St;
    const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const uint8_t *rec = cin + int64_t(L::Q) * pitch * St::E;
    const typename St::RawB rb = *reinterpret_cast<const typename St::RawB *>(rec + St::kRecA * pitch + St::kRecB * n);
    const f4 e = St::entry(*reinterpret_cast<const typename St::RawA *>(rec + St::kRecA * n), rb);
    const float Rd = St::ratio(rb);
    bool fl;
    const float M = Codec<float>::col<float>(e[0], fl);
    const float Va[3] = {e[1], e[2], e[3]};
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const float d = St::df(*reinterpret_cast<const typename St::Raw *>(cin + (int64_t(i) * pitch + n) * St::E), i);
        const int n2 = csq<L>(i);
        // the receiver's expression: c_i . V_axis, times R_d for a diagonal
        const float cva = float(L::cx[i]) * Va[0] + float(L::cy[i]) * Va[1] + float(L::cz[i]) * Va[2];
        const float vd = n2 == 0 ? 0.0f : (n2 == 1 ? cva : Rd * cva);
        const float f = float(wgt<L>(i)) + d;
        const float mu36 = M * (float(w36<L>(i)) + 36.0f * d) + vd;
        const float q = f != 0.0f ? mu36 / (36.0f * f) : 0.0f;
        const bool keep = q <= 0.5f;
        pout[int64_t(i) * pitch + n] = encode_pair<L, S, float>(d, keep ? q : 1.0f - q, keep ? fl : !fl, i);
    }
}

template <bool PAIR_IN, typename S>
const void *compact_kernel(int tx) {
    return tx == 32 ? reinterpret_cast<const void *>(&k_step_compact<PAIR_IN, 32, S>)
                    : reinterpret_cast<const void *>(&k_step_compact<PAIR_IN, 64, S>);
}

// The kernel (tile width tx, storage S) and its LDS, allowed beyond 64 KiB.
template <bool PAIR_IN, typename S>
const void *compact_fn(int tx, size_t &lds) {
    lds = PAIR_IN ? (tx == 32 ? CTile<32>::lds_pair : CTile<64>::lds_pair) : (tx == 32 ? CTile<32>::lds : CTile<64>::lds);
    if (!PAIR_IN) allow_lds(compact_kernel<false, S>(tx), (tx == 32 ? 1 : 0) + (sizeof(S) == 2 ? 3 : 0), lds);
    return compact_kernel<PAIR_IN, S>(tx);
}

}  // namespace


// The first step reads the pair state, so both layouts must stay within
// 32-bit byte offsets.  The D3Q19 sweep stores FP32 or FP16, the D2Q9 one
// FP32.
bool compact_supported(int lattice, int prec, const Geo &g) {
    // with geometry: D3Q19, on the split step
    if (g.mask != nullptr)
        return lattice == 1 && (prec == 1 || prec == 2) &&
               uint64_t(2 * D3Q19::Q) * uint64_t(g.pitch) * (prec == 1 ? 4u : 2u) < (uint64_t(1) << 32);
    if (lattice == 0) return prec == 1 && g.nz == 1 && uint64_t(2 * D2Q9::Q) * uint64_t(g.pitch) * 4u < (uint64_t(1) << 32);
    const uint64_t elem = prec == 1 ? 4 : 2;
    return lattice == 1 && (prec == 1 || prec == 2) &&
           uint64_t(2 * D3Q19::Q) * uint64_t(g.pitch) * elem < (uint64_t(1) << 32);
}

int compact_resident_blocks(int tx, int prec) {
    int per_cu = 0;
    size_t lds = 0;
    const void *fn = prec == 2 ? compact_fn<false, _Float16>(tx, lds) : compact_fn<false, float>(tx, lds);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, tx * kCR, lds) != hipSuccess) {
        (void)hipGetLastError();
        per_cu = 1;
    }
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return (per_cu > 0 ? per_cu : 1) * cus;
}

hipError_t launch_step_compact(int prec, const Geo &g, const ModelD &md, const void *in, bool pair_in, void *out,
                               const uint32_t *ctr_in, uint32_t *ctr_out, FusedShape sh, hipStream_t s) {
    if (sh.rows != kCR || (sh.tx != 64 && sh.tx != 32)) return hipErrorInvalidValue;
    if (g.mask || md.bgk || (prec != 1 && prec != 2)) return hipErrorInvalidValue;
    if (uint64_t(2 * D3Q19::Q) * uint64_t(g.pitch) * (prec == 1 ? 4u : 2u) >= (uint64_t(1) << 32))
        return hipErrorInvalidValue;
    CompactArgs a;
    a.in = in;
    a.out = out;
    a.nx = g.nx;
    a.ny = g.ny;
    a.nz = g.nz;
    a.pitch = g.pitch;
    a.ctr_in = ctr_in;
    a.ctr_out = ctr_out;
    a.ntx = (g.nx + sh.tx - 1) / sh.tx;
    a.nty = (g.ny + kCR - 1) / kCR;
    a.zchunks = sh.zchunks < 1 ? 1 : (sh.zchunks > g.nz ? g.nz : sh.zchunks);
    const int64_t nblocks = int64_t(a.ntx) * a.nty * a.zchunks;
    if (nblocks > 0x7fffffff) return hipErrorInvalidValue;
    const Model<float> mo = to_model<float>(md);
    size_t lds = 0;
    const void *fn = prec == 2 ? (pair_in ? compact_fn<true, _Float16>(sh.tx, lds) : compact_fn<false, _Float16>(sh.tx, lds))
                               : (pair_in ? compact_fn<true, float>(sh.tx, lds) : compact_fn<false, float>(sh.tx, lds));
    void *args[] = {&a, const_cast<Model<float> *>(&mo)};
    return hipLaunchKernel(fn, dim3(unsigned(nblocks)), dim3(unsigned(sh.tx * kCR)), args, lds, s);
}

hipError_t launch_expand(int prec, const Geo &g, const void *cin, void *pout, hipStream_t s) {
    if (g.N <= 0) return hipSuccess;
    const int64_t blocks = (g.N + 255) / 256;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    if (prec == 2)
        hipLaunchKernelGGL(k_expand<_Float16>, dim3(unsigned(blocks)), dim3(256), 0, s, static_cast<const uint8_t *>(cin),
                           static_cast<typename PairOf<_Float16>::type *>(pout), g.N, g.pitch);
    else
        hipLaunchKernelGGL(k_expand<float>, dim3(unsigned(blocks)), dim3(256), 0, s, static_cast<const uint8_t *>(cin),
                           static_cast<typename PairOf<float>::type *>(pout), g.N, g.pitch);
    return hipGetLastError();
}

}  // namespace lbcg
