// The compact-state D3Q19 sweep over many lattices in one launch (batched
// form).  Built apart from the single-lattice kernels so that each object
// gets the code-generation options measured best for it.
#include "lbcg_compact_sweep.h"

namespace lbcg {

namespace {

// Many lattices in one launch (batched form): entry k of the block table is
// work item bitem[k] of lattice blat[k]; entries are dealt to the 8 XCDs in
// contiguous bands (blocks go to XCDs round-robin), as the single-lattice
// kernel deals its work items.  Every lattice is compact and periodic with
// 8-row tiles and storage S (float or _Float16).
template <typename S>
__global__ void __launch_bounds__(kCTX * kCR)
    k_step_compact_batch(const BatchDesc<float> *__restrict__ desc, const int *__restrict__ blat,
                         const int *__restrict__ bitem) {
    extern __shared__ float lds[];
    const int total = int(gridDim.x);
    const int xcd = blockIdx.x % kCXCD, l = blockIdx.x / kCXCD;
    const int k = xcd * (total / kCXCD) + min(xcd, total % kCXCD) + l;
    const int item = bitem[k];
    const BatchDesc<float> d = desc[blat[k]];
    CompactArgs a;
    a.in = d.a.in;
    a.out = d.a.out;
    a.nx = d.a.nx;
    a.ny = d.a.ny;
    a.nz = d.a.nz;
    a.pitch = d.a.pitch;
    a.ctr_in = d.a.ctr_in;
    a.ctr_out = d.a.ctr_out;
    a.ntx = d.a.ntx;
    a.nty = d.a.nty;
    a.zchunks = d.a.zchunks;
    if (item == 0 && threadIdx.x == 0) *a.ctr_out = *a.ctr_in + 1u;
    sweep_compact<false, kCTX, S>(a, d.mo, item / a.zchunks, item % a.zchunks, lds);
}

}  // namespace

hipError_t launch_step_compact_batch(int prec, const void *desc, const int *blat, const int *bitem, int nblocks,
                                     hipStream_t s) {
    if (prec != 1 && prec != 2) return hipErrorInvalidValue;
    if (nblocks <= 0) return hipSuccess;
    const BatchDesc<float> *d = static_cast<const BatchDesc<float> *>(desc);
    const dim3 grid{unsigned(nblocks)}, block{unsigned(kCTX * kCR)};
    if (prec == 1) {
        allow_lds(reinterpret_cast<const void *>(&k_step_compact_batch<float>), 0, kCompactLds);
        hipLaunchKernelGGL(k_step_compact_batch<float>, grid, block, kCompactLds, s, d, blat, bitem);
    } else {
        allow_lds(reinterpret_cast<const void *>(&k_step_compact_batch<_Float16>), 1, kCompactLds);
        hipLaunchKernelGGL(k_step_compact_batch<_Float16>, grid, block, kCompactLds, s, d, blat, bitem);
    }
    return hipGetLastError();
}

}  // namespace lbcg
