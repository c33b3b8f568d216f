// Internal interface between the C-ABI runtime and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbcg_device.h"

namespace lbcg {

// Model parameters in double; launchers convert to the compute type.
struct ModelD {
    double ivR, ivB, Abar, beta, aR, aB, eps_F;  // ivR, ivB: 1/nu_k
    double w0;  // rest weight of the lattice
    double omR, omB;  // 1/tau_k
    int bgk;    // 0 regularized, 1 BGK at the node's rate, 2 BGK per colour
};

template <typename T>
inline Model<T> to_model(const ModelD &m) {
    Model<T> r;
    r.ivR = T(m.ivR);
    r.ivB = T(m.ivB);
    r.Abar = T(m.Abar);
    r.beta = T(m.beta);
    r.aR = T(m.aR);
    r.aB = T(m.aB);
    r.dR0 = T(m.aR - m.w0);
    r.dB0 = T(m.aB - m.w0);
    r.kR = T((m.w0 - m.aR) / (1.0 - m.w0));
    r.kB = T((m.w0 - m.aB) / (1.0 - m.w0));
    r.eps_F = T(m.eps_F);
    r.omR = T(m.omR);
    r.omB = T(m.omB);
    r.bgk = m.bgk;
    return r;
}

// Number of doubles per block in the diagnostics partials.
constexpr int kDiagVals = 13;
// Blocks of the diagnostics reduction (partials = kDiagBlocks * kDiagVals).
constexpr int kDiagBlocks = 1024;

// lattice: 0 = D2Q9, 1 = D3Q19; prec: 0 = F64, 1 = F32, 2 = F16.
// Equilibrium state (Eq. (6)) of nodes [n0, n0 + cnt) from chunk-local fields
// rhoR, rhoB (cnt each) and u (3 * cnt, component-major, nullable).
hipError_t launch_init(int lattice, int prec, const Geo &g, const ModelD &md, int64_t n0, int64_t cnt,
                       const double *rhoR, const double *rhoB, const double *u, void *st, hipStream_t s);
hipError_t launch_psi(int lattice, int prec, const Geo &g, const ModelD &md, const void *st,
                      bool pulled, void *psi, hipStream_t s);
// ctr_in / ctr_out: the time-step counter read by this step and the slot
// that receives its successor (device memory, one uint32 each).
hipError_t launch_step_generic(int lattice, int prec, const Geo &g, const ModelD &md,
                               const void *in, bool pulled, const void *psi, void *out,
                               const uint32_t *ctr_in, uint32_t *ctr_out, hipStream_t s);
// Fields of nodes [n0, n0 + cnt): out = rhoR | rhoB | ux | uy | uz | psi (cnt each).
hipError_t launch_fields(int lattice, int prec, const Geo &g, const ModelD &md, const void *st,
                         bool pulled, int64_t n0, int64_t cnt, double *out, hipStream_t s);
// Populations of nodes [n0, n0 + cnt): out[(k * Q + i) * cnt + (n - n0)].
hipError_t launch_pops(int lattice, int prec, const Geo &g, const ModelD &md, const void *st,
                       bool pulled, int64_t n0, int64_t cnt, double *out, hipStream_t s);
// Populations of cnt listed nodes: out[(j * 2 + k) * Q + i].
hipError_t launch_pops_at(int lattice, int prec, const Geo &g, const ModelD &md, const void *st,
                          bool pulled, const int64_t *nodes, int64_t cnt, double *out, hipStream_t s);
// Deterministic two-stage FP64 reduction into res[kDiagVals].
hipError_t launch_diag(int lattice, int prec, const Geo &g, const ModelD &md, const void *st,
                       bool pulled, double *partials, double *res, hipStream_t s);

// Fused single-pass D3Q19 step; F32 or F16 storage, with or without geometry;
// the regularized collision, or plain BGK (md.bgk: 8-row tiles only).
struct FusedShape {
    int rows;     // rows of the x-y tile (one wave of 64 nodes per row)
    int zchunks;  // z range split per column of tiles
    int tx = 64;  // tile width (the compact D3Q19 sweep: 64 or 32)
};

// Kernel view of one lattice for the fused sweep.
template <typename S>
struct FusedArgs {
    const S *in;
    S *out;
    int nx, ny, nz;
    int64_t pitch;
    const uint8_t *mask;  // nullptr = every node fluid
    const DevInlet *inlets;
    const DevOutlet *outlets;
    const DevWall *walls;
    const uint32_t *links;   // link words (with a mask)
    const uint32_t *ctr_in;  // time-step counter of this step
    uint32_t *ctr_out;       // receives ctr_in + 1
    int ntx, nty, zchunks;
};
template <typename S>
FusedArgs<S> fused_args(const Geo &g, const void *in, void *out, const uint32_t *ctr_in, uint32_t *ctr_out,
                        FusedShape sh);

hipError_t launch_step_fused(int prec, const Geo &g, const ModelD &md, const void *in, void *out,
                             const uint32_t *ctr_in, uint32_t *ctr_out, FusedShape shape, hipStream_t s);
bool fused_supported(int lattice, int prec, const Geo &g);
// Blocks of the fused kernel that fit on the device at once (pops: its plain
// BGK form).
int fused_resident_blocks(int prec, int rows, bool masked, bool pops = false);

// Split D3Q19 step for lattices with geometry (F32 or F16 storage,
// regularized): a moments kernel writes psi (`psi`, pitch floats) and the
// kSplitMoments collision moments of every fluid node, a collision kernel
// takes the gradient, collides and stores, and a boundary kernel stores the
// inlet and outlet values.  Bitwise the column sweep's results; chosen by
// FusedShape rows 0.  The moments and collision kernels run blocks of
// kSplitGX x kSplitGY nodes of one z plane, only those with fluid, from a
// block list; the boundary kernel runs one thread per node with links from
// inlets or outlets, from a node list.  split_prepare builds the lists on the
// device once per lattice in `scratch` (split_scratch_bytes: the moments,
// then the lists).
constexpr int kSplitMoments = 12;
constexpr int kSplitGX = 64, kSplitGY = 4;
int64_t split_blocks(int nx, int ny, int nz);
size_t split_scratch_bytes(int64_t pitch, int nx, int ny, int nz);
struct SplitPlan {
    int64_t active = 0, io = 0;  // blocks with fluid, blocks with inlet or outlet links
    int64_t ionodes = 0;         // nodes with inlet or outlet links
};
// Builds the block lists and returns their lengths (waits for the stream).
hipError_t split_prepare(const Geo &g, void *scratch, SplitPlan &sp, hipStream_t s);
// The split step on the compact state (D3Q19 F32 or F16 with geometry): reads the
// compact state `in` (or, with pair_in, the pair state `in`, on the first
// step after an initialisation or a restore), the inlet and outlet values in
// the pair buffer gin, writes the compact state `cout` and the new inlet and
// outlet values into the pair buffer gout.
hipError_t launch_step_cgeo(int prec, const Geo &g, const ModelD &md, bool pair_in, const void *in, const void *gin,
                            void *cout, void *gout, void *psi, void *scratch, const SplitPlan &sp,
                            const uint32_t *ctr_in, uint32_t *ctr_out, hipStream_t s);
// Its compact state as pairs (fluid nodes and wall values) into pout, which
// already holds the inlet and outlet values.
hipError_t launch_expand_cgeo(int prec, const Geo &g, const void *cin, void *pout, void *scratch, const SplitPlan &sp,
                              hipStream_t s);
hipError_t launch_step_split(int prec, const Geo &g, const ModelD &md, const void *in, void *out, void *psi,
                             void *scratch, const SplitPlan &sp, const uint32_t *ctr_in, uint32_t *ctr_out,
                             hipStream_t s);

// Fused single-pass D2Q9 step on periodic lattices, F32 or F16 storage:
// strips of 64 columns, each row range split into ychunks.
hipError_t launch_step_fused2d(int prec, const Geo &g, const ModelD &md, const void *in, void *out,
                               const uint32_t *ctr_in, uint32_t *ctr_out, int ychunks, hipStream_t s);
bool fused2d_supported(int prec, const Geo &g);

// Fused D3Q19 step on the compact state (periodic, regularized, tiles of 8
// rows, FP32 or FP16 storage): 19 arrays of pitch totals and 5 colour
// scalars per node in two record arrays, kCompactBytes (FP32) or
// kCompactBytes16 (FP16) per pitch node.  pair_in: `in` is a pair state of
// the same precision (the first step after an initialisation or a restore);
// `out` is always compact.
constexpr int kCompactBytes = 19 * 4 + 20;    // D3Q19, FP32: 19 totals, 5 scalars
constexpr int kCompactBytes16 = 19 * 2 + 12;  // D3Q19, FP16 (M kept FP32)
constexpr int kCompactBytes2d = 9 * 4 + 16;   // D2Q9: 9 totals, 4 scalars
hipError_t launch_step_compact(int prec, const Geo &g, const ModelD &md, const void *in, bool pair_in, void *out,
                               const uint32_t *ctr_in, uint32_t *ctr_out, FusedShape shape, hipStream_t s);
bool compact_supported(int lattice, int prec, const Geo &g);
int compact_resident_blocks(int tile_width, int prec);
// Pair state (post-collision, as the pair kernels store it) of a compact state.
hipError_t launch_expand(int prec, const Geo &g, const void *cin, void *pout, hipStream_t s);
// The D2Q9 strip sweep on the compact state (periodic, FP32, regularized):
// 9 arrays of pitch floats and 4 colour scalars per node in one record
// array, kCompactBytes2d per pitch node; rows split into ychunks.
hipError_t launch_step_compact2d(const Geo &g, const ModelD &md, const void *in, bool pair_in, void *out,
                                 const uint32_t *ctr_in, uint32_t *ctr_out, int ychunks, hipStream_t s);
hipError_t launch_expand2d(const Geo &g, const void *cin, void *pout, hipStream_t s);

// Batched fused step: one launch steps many lattices by one time level.
// Block b sweeps work item bitem[b] (tile-major (tile, z chunk) index) of
// lattice blat[b], described by desc[blat[b]].
template <typename S>
struct BatchDesc {
    FusedArgs<S> a;
    Model<float> mo;
};
hipError_t launch_step_fused_batch(int prec, const void *desc, const int *blat, const int *bitem, int nblocks,
                                   int rows, bool masked, hipStream_t s);
// Batched compact step: desc are BatchDesc<float> of compact lattices (in,
// out: compact buffers of storage prec, 1 = F32 or 2 = F16; shapes of 8
// rows).
hipError_t launch_step_compact_batch(int prec, const void *desc, const int *blat, const int *bitem, int nblocks,
                                     hipStream_t s);

}  // namespace lbcg
