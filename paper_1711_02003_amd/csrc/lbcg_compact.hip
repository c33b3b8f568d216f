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
// each with its own barrier).
template <bool PAIR_IN, int TX>
__global__ void __launch_bounds__(TX * kCR) k_step_compact(CompactArgs a, Model<float> mo) {
    extern __shared__ float lds[];
    const int total = a.ntx * a.nty * a.zchunks;
    const int xcd = blockIdx.x % kCXCD, l = blockIdx.x / kCXCD;
    const int item = xcd * (total / kCXCD) + min(xcd, total % kCXCD) + l;
    if (item == 0 && threadIdx.x == 0) *a.ctr_out = *a.ctr_in + 1u;
    if (PAIR_IN)
        sweep_pairs<TX>(a, mo, item / a.zchunks, item % a.zchunks, lds);
    else
        sweep_compact<true, TX>(a, mo, item / a.zchunks, item % a.zchunks, lds);
}

// Pair state of nodes [0, N) from a compact state: each population's
// minority colour part M f_i + (c_i . V_c) / 36 (the split the receiver
// makes), as a share of f_i, with the flag of the colour it belongs to.
__global__ void k_expand(const float *__restrict__ cin, typename PairOf<float>::type *__restrict__ pout, int64_t N,
                         int64_t pitch) {
    using L = D3Q19;
    const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const float *ra = cin + int64_t(L::Q) * pitch + 4 * n, *rb = cin + int64_t(L::Q + 4) * pitch + n;
    bool fl;
    const float M = Codec<float>::col<float>(ra[0], fl);
    const float Va[3] = {ra[1], ra[2], ra[3]}, Rd = rb[0];
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const float d = cin[int64_t(i) * pitch + n];
        const int n2 = csq<L>(i);
        // the receiver's expression: c_i . V_axis, times R_d for a diagonal
        const float cva = float(L::cx[i]) * Va[0] + float(L::cy[i]) * Va[1] + float(L::cz[i]) * Va[2];
        const float vd = n2 == 0 ? 0.0f : (n2 == 1 ? cva : Rd * cva);
        const float f = float(wgt<L>(i)) + d;
        const float mu36 = M * (float(w36<L>(i)) + 36.0f * d) + vd;
        const float q = f != 0.0f ? mu36 / (36.0f * f) : 0.0f;
        const bool keep = q <= 0.5f;
        pout[int64_t(i) * pitch + n] = encode_pair<L, float, float>(d, keep ? q : 1.0f - q, keep ? fl : !fl, i);
    }
}

}  // namespace


// The first step reads the pair state, so both layouts must stay within
// 32-bit byte offsets.
bool compact_supported(int lattice, int prec, const Geo &g) {
    if (prec != 1 || g.mask != nullptr) return false;
    if (lattice == 0) return g.nz == 1 && uint64_t(2 * D2Q9::Q) * uint64_t(g.pitch) * 4u < (uint64_t(1) << 32);
    return lattice == 1 && uint64_t(2 * D3Q19::Q) * uint64_t(g.pitch) * 4u < (uint64_t(1) << 32);
}

int compact_resident_blocks(int tx) {
    int per_cu = 0;
    const void *fn = tx == 32 ? reinterpret_cast<const void *>(&k_step_compact<false, 32>)
                              : reinterpret_cast<const void *>(&k_step_compact<false, 64>);
    if (tx == 32) allow_lds(fn, 1, CTile<32>::lds);
    else allow_lds(fn, 0, CTile<64>::lds);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, tx * kCR,
                                                     tx == 32 ? CTile<32>::lds : CTile<64>::lds) != hipSuccess) {
        (void)hipGetLastError();
        per_cu = 1;
    }
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return (per_cu > 0 ? per_cu : 1) * cus;
}

hipError_t launch_step_compact(const Geo &g, const ModelD &md, const void *in, bool pair_in, void *out,
                               const uint32_t *ctr_in, uint32_t *ctr_out, FusedShape sh, hipStream_t s) {
    if (sh.rows != kCR || (sh.tx != 64 && sh.tx != 32)) return hipErrorInvalidValue;
    if (g.mask || md.bgk) return hipErrorInvalidValue;
    if (uint64_t(2 * D3Q19::Q) * uint64_t(g.pitch) * 4u >= (uint64_t(1) << 32)) return hipErrorInvalidValue;
    CompactArgs a;
    a.in = static_cast<const float *>(in);
    a.out = static_cast<float *>(out);
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
    const dim3 grid = dim3(unsigned(nblocks)), block = dim3(unsigned(sh.tx * kCR));
    if (sh.tx == 32) {
        allow_lds(reinterpret_cast<const void *>(&k_step_compact<false, 32>), 1, CTile<32>::lds);
        if (pair_in)
            hipLaunchKernelGGL((k_step_compact<true, 32>), grid, block, CTile<32>::lds_pair, s, a, mo);
        else
            hipLaunchKernelGGL((k_step_compact<false, 32>), grid, block, CTile<32>::lds, s, a, mo);
    } else {
        allow_lds(reinterpret_cast<const void *>(&k_step_compact<false, 64>), 0, CTile<64>::lds);
        if (pair_in)
            hipLaunchKernelGGL((k_step_compact<true, 64>), grid, block, CTile<64>::lds_pair, s, a, mo);
        else
            hipLaunchKernelGGL((k_step_compact<false, 64>), grid, block, CTile<64>::lds, s, a, mo);
    }
    return hipGetLastError();
}

hipError_t launch_expand(const Geo &g, const void *cin, void *pout, hipStream_t s) {
    if (g.N <= 0) return hipSuccess;
    const int64_t blocks = (g.N + 255) / 256;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_expand, dim3(unsigned(blocks)), dim3(256), 0, s, static_cast<const float *>(cin),
                       static_cast<typename PairOf<float>::type *>(pout), g.N, g.pitch);
    return hipGetLastError();
}

}  // namespace lbcg
