// Split D3Q19 step for lattices with geometry (arXiv:1711.02003, Sec. II,
// Eqs. (1)-(11)): the fused step in two kernels, one thread per node.
//
// The column sweep (lbcg_fused.hip) keeps a tile's phase field in LDS and
// recomputes a one-node ring of neighbour psi from their pulled populations;
// a z chunk re-pulls the two planes around it.  On a channel geometry the
// fluid fills few tiles, so filling the device takes short chunks, and the
// ring and the chunk halo then cost as much as the nodes themselves.  Here:
//   k_geo_moments: each fluid node pulls its 19 pairs (Eq. (1)), takes the
//     moments the collision needs (drho, 36 rho^R, 36 rho^B, j, trace-adjusted
//     flux S: 12 values) and psi (Eq. (4) input), and writes them;
//   k_geo_collide: each fluid node forms the colour gradient from its
//     neighbours' psi (neutral walls and outlets: its own psi; inlets and
//     wetting walls: their phase value), collides (Eqs. (9)-(11)) and
//     stores its 19 new pairs and, for links from walls, their bounce-back
//     values;
//   k_geo_boundary: each fluid node with links from inlets or outlets
//     stores their values (from its new pairs, read back).
// Every value is computed by the expressions and in the order of the column
// sweep, so the results are bitwise those of the sweep.  Traffic per fluid
// node: pairs read and written once (2 x 38 x E bytes), plus 12 moments and
// psi written and read once (2 x 52 bytes), the neighbours' psi from cache,
// and at nodes next to a boundary their new pairs read back.
#include "lbcg_buffer.h"
#include "lbcg_internal.h"

namespace lbcg {

namespace {

// Blocks of 64 x 4 nodes of one z plane (a wave per x row), numbered plane
// first, then y range, then x range; the kernels run only the blocks in
// their list (in that order).  Blocks go to the 8 XCDs round-robin, so
// every XCD gets an even share of each tile's planes whatever the channel
// layout.  Numbered x range first, a lattice 512 wide (8 x ranges) gives
// each XCD one x range, and a channel that crosses the lattice in y then
// runs on one XCD; numbered y range first, the junction's kernels measured
// 1.5 to 1.8 x slower than plane first.  Launching every block of the
// lattice, solid ones included, cost each kernel about 15 us on the
// junction (16384 blocks, 70 % of them solid).
constexpr int kGX = kSplitGX, kGY = kSplitGY, kGeoBlock = kGX * kGY;
constexpr int kNM = kSplitMoments;  // moments per node

template <typename S>
struct SplitArgs {
    FusedArgs<S> a;
    float *psi;                 // psi of every fluid node
    float *mom;                 // kNM arrays of pitch floats
    const uint32_t *blocks;     // the kernel's block list
};

// Scratch layout: the moments, then the per-block flags, the list of blocks
// with fluid, the list of blocks with inlet or outlet links and the two
// lengths.
struct ScratchMap {
    float *mom;
    uint8_t *flags;
    uint32_t *act, *io, *counts;
};
__host__ __device__ inline size_t align256(size_t v) { return (v + 255) / 256 * 256; }
inline ScratchMap scratch_map(void *scratch, int64_t pitch, int64_t nb) {
    char *p = static_cast<char *>(scratch);
    ScratchMap m;
    m.mom = reinterpret_cast<float *>(p);
    p += align256(sizeof(float) * kNM * size_t(pitch));
    m.flags = reinterpret_cast<uint8_t *>(p);
    p += align256(size_t(nb));
    m.act = reinterpret_cast<uint32_t *>(p);
    p += align256(sizeof(uint32_t) * size_t(nb));
    m.io = reinterpret_cast<uint32_t *>(p);
    p += align256(sizeof(uint32_t) * size_t(nb));
    m.counts = reinterpret_cast<uint32_t *>(p);
    return m;
}

// The node of this thread in block b (false outside the lattice), and the
// node index x' + nx (y' + ny z') of its neighbour x + (dx, dy, dz)
// (periodic).  Node indices fit 32 bits: the state buffers are below 4 GiB.
struct Here {
    int x, y, z;
    uint32_t n;
};
__device__ __forceinline__ bool here(int nx, int ny, int nz, uint32_t b, Here &h) {
    const uint32_t nby = uint32_t(uniform((ny + kGY - 1) / kGY)), nzu = uint32_t(uniform(nz));
    const uint32_t t = b / nzu, u = t / nby;
    h.z = int(b - t * nzu);
    h.y = int(t - u * nby) * kGY + int(threadIdx.x / kGX);
    h.x = int(u) * kGX + int(threadIdx.x % kGX);
    h.n = uint32_t(h.x) + uint32_t(nx) * (uint32_t(h.y) + uint32_t(ny) * uint32_t(h.z));
    return h.x < nx && h.y < ny;
}
__device__ __forceinline__ uint32_t nbr(int nx, int ny, int nz, const Here &h, int dx, int dy, int dz) {
    const uint32_t xs = uint32_t(wrap_m1(h.x + dx, nx)), ys = uint32_t(wrap_m1(h.y + dy, ny)),
                   zs = uint32_t(wrap_m1(h.z + dz, nz));
    return xs + uint32_t(nx) * (ys + uint32_t(ny) * zs);
}

// A node whose link from a non-fluid neighbour is not a wall's: the
// boundary kernel stores that link's value.
__device__ __forceinline__ bool has_io_link(uint32_t lk) {
    return (lk & kLinkFluid) && (lk & kLinkBits) && ((lk & kLinkMixed) || !is_wall(link_code(lk)));
}

// Flags of block b: 1 = some node fluid, 2 = some node with an inlet or
// outlet link (mixed codes count: the boundary kernel checks each link).
__global__ void __launch_bounds__(kGeoBlock) k_geo_flags(const uint32_t *__restrict__ links, int nx, int ny, int nz,
                                                        uint8_t *__restrict__ flags) {
    Here h;
    const bool in = here(nx, ny, nz, blockIdx.x, h);
    const uint32_t lk = in ? links[h.n] : 0u;
    const int f = __syncthreads_or((lk & kLinkFluid) != 0u), io = __syncthreads_or(has_io_link(lk));
    if (threadIdx.x == 0) flags[blockIdx.x] = uint8_t((f ? 1 : 0) | (io ? 2 : 0));
}

// The two block lists in ascending block order, by one block: thread t
// takes the flags of a contiguous range, counts, and writes its ids after
// the counts of the threads before it.
constexpr int kListThreads = 1024;
__global__ void __launch_bounds__(kListThreads) k_geo_lists(const uint8_t *__restrict__ flags, uint32_t nb,
                                                           uint32_t *__restrict__ act, uint32_t *__restrict__ io,
                                                           uint32_t *__restrict__ counts) {
    __shared__ uint32_t ca[kListThreads], ci[kListThreads];
    const uint32_t per = (nb + kListThreads - 1) / kListThreads;
    const uint32_t b0 = min(nb, threadIdx.x * per), b1 = min(nb, b0 + per);
    uint32_t na = 0, ni = 0;
    for (uint32_t b = b0; b < b1; ++b) {
        na += flags[b] & 1u;
        ni += (flags[b] >> 1) & 1u;
    }
    ca[threadIdx.x] = na;
    ci[threadIdx.x] = ni;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t sa = 0, si = 0;
        for (int t = 0; t < kListThreads; ++t) {
            const uint32_t va = ca[t], vi = ci[t];
            ca[t] = sa;
            ci[t] = si;
            sa += va;
            si += vi;
        }
        counts[0] = sa;
        counts[1] = si;
    }
    __syncthreads();
    uint32_t oa = ca[threadIdx.x], oi = ci[threadIdx.x];
    for (uint32_t b = b0; b < b1; ++b) {
        if (flags[b] & 1u) act[oa++] = b;
        if (flags[b] & 2u) io[oi++] = b;
    }
}

// psi that a non-fluid node shows the gradient of a fluid neighbour: the
// inlet's or the wetting wall's phase value; neutral walls and outlets show
// the fluid node's own psi (pc)
template <typename S>
__device__ __forceinline__ float solid_psi(const FusedArgs<S> &a, uint8_t c, float pc) {
    if (is_inlet(c)) {
        const DevInlet in = a.inlets[c - kInlet0];
        return float((in.rhoR - in.rhoB) / (in.rhoR + in.rhoB));
    }
    if (c >= kWall0 && c < kOutlet0) return float(a.walls[c - kWall0].psi);
    return pc;
}

template <typename S>
__global__ void __launch_bounds__(kGeoBlock) k_geo_moments(SplitArgs<S> sa) {
    using L = D3Q19;
    typedef float T;
    typedef typename PairOf<S>::type P2;
    constexpr uint32_t E = sizeof(P2);
    const FusedArgs<S> &a = sa.a;
    Here h;
    if (!here(a.nx, a.ny, a.nz, sa.blocks[blockIdx.x], h)) return;
    const uint32_t n = h.n;
    if (!(a.links[n] & kLinkFluid)) return;
    const uint32_t cstride = uint32_t(a.pitch) * E;
    const __amdgpu_buffer_rsrc_t rin = state_rsrc(a.in, uint32_t(L::Q) * cstride);
    P2 v[L::Q];
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const uint32_t m = nbr(a.nx, a.ny, a.nz, h, -L::cx[i], -L::cy[i], -L::cz[i]);
        v[i] = load_pair<P2>(rin, m * E, uint32_t(i) * cstride);
    }
    Pops<L, T> q;
    q.red = 0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) decode_pair<L, S, T>(v[i], i, q);
    Mom<T> mm;
    moments<L, T>(q, mm);
    sa.psi[n] = float(psi_of<T>(mm.drho, mm.r36R, mm.r36B));
    const float vals[kNM] = {mm.drho, mm.r36R, mm.r36B, mm.j[0], mm.j[1], mm.j[2],
                             mm.S[0], mm.S[1], mm.S[2], mm.S[3], mm.S[4], mm.S[5]};
#pragma unroll
    for (int k = 0; k < kNM; ++k) sa.mom[int64_t(k) * a.pitch + n] = vals[k];
}

// Collision kernel, the moments kernel's blocks, one plane per block (a
// block stepping its tile column up a chunk of 4 or 8 planes with the next
// plane's loads in flight measured slower on the junction: 104 and 147
// against 92 us, with more registers and fewer blocks).
template <typename S>
__global__ void __launch_bounds__(kGeoBlock) k_geo_collide(SplitArgs<S> sa, Model<float> mo) {
    using L = D3Q19;
    typedef float T;
    typedef typename PairOf<S>::type P2;
    constexpr uint32_t E = sizeof(P2);
    const FusedArgs<S> &a = sa.a;
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.ctr_out = *a.ctr_in + 1u;
    if (!sa.blocks) return;  // no fluid node
    Here h;
    if (!here(a.nx, a.ny, a.nz, sa.blocks[blockIdx.x], h)) return;
    const uint32_t n = h.n;
    const uint32_t clk = a.links[n];
    if (!(clk & kLinkFluid)) return;
    const uint32_t step = *a.ctr_in;  // seeds the stochastic rounding of 16-bit shares

    // colour gradient from the neighbours' psi, in the column sweep's order
    const float pc = sa.psi[n];
    T fx = 0, fy = 0, fz = 0;
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        const uint32_t m = nbr(a.nx, a.ny, a.nz, h, L::cx[i], L::cy[i], L::cz[i]);
        // x + c_i is the upstream node of the opposite link
        const float pv = ((clk >> L::opp[i]) & 1u) ? solid_psi(a, a.mask[m], pc) : sa.psi[m];
        const T wp = T(3.0 * wgt<L>(i)) * T(pv);
        if (L::cx[i]) fx += L::cx[i] > 0 ? wp : -wp;
        if (L::cy[i]) fy += L::cy[i] > 0 ? wp : -wp;
        if (L::cz[i]) fz += L::cz[i] > 0 ? wp : -wp;
    }
    const T F[3] = {fx, fy, fz};
    T mv[kNM];
#pragma unroll
    for (int k = 0; k < kNM; ++k) mv[k] = sa.mom[int64_t(k) * a.pitch + n];
    const T cj[3] = {mv[3], mv[4], mv[5]}, cS[6] = {mv[6], mv[7], mv[8], mv[9], mv[10], mv[11]};
    PostOut<L, T> o;
    collide<L, T>(mo, mv[0], mv[1], mv[2], cj, cS, F, nullptr, o);
    Dither dz(step, n);
    const uint32_t cstride = uint32_t(a.pitch) * E;
    const __amdgpu_buffer_rsrc_t rout = state_rsrc(a.out, uint32_t(L::Q) * cstride);
    // Each new pair is stored as soon as it is encoded; where the link of the
    // opposite direction comes from a wall, the same pair is also its
    // half-way bounce-back value, stored in the wall node's slot.
#pragma unroll
    for (int j = 0; j < L::Q; ++j) {
        const P2 v = encode_step<L, S, T>(o.df[j], o.mm[j], (o.red >> j) & 1u, j, dz);
        store_pair<P2>(rout, n * E, uint32_t(j) * cstride, v);
        const int i = L::opp[j];
        if (j != 0 && ((clk >> i) & 1u)) {
            const uint32_t m = nbr(a.nx, a.ny, a.nz, h, -L::cx[i], -L::cy[i], -L::cz[i]);
            if (is_wall((clk & kLinkMixed) ? a.mask[m] : link_code(clk)))
                store_pair<P2>(rout, m * E, uint32_t(i) * cstride, v);
        }
    }
}

// Inlet and outlet values: every fluid node with a link from an inlet or an
// outlet reads back the new pairs it stored and writes, for each such link,
// the value it will pull through it at the next step into the upstream
// node's slot (the rules of the column sweep, from the same stored pairs).
// Kept out of the collision kernel, whose registers they would take from 59
// to 137.
template <typename S>
__global__ void __launch_bounds__(kGeoBlock) k_geo_boundary(SplitArgs<S> sa, Model<float> mo) {
    using L = D3Q19;
    typedef float T;
    typedef typename PairOf<S>::type P2;
    constexpr uint32_t E = sizeof(P2);
    const FusedArgs<S> &a = sa.a;
    Here h;
    if (!here(a.nx, a.ny, a.nz, sa.blocks[blockIdx.x], h)) return;
    const uint32_t n = h.n;
    const uint32_t clk = a.links[n];
    if (!has_io_link(clk)) return;
    const uint32_t cstride = uint32_t(a.pitch) * E;
    const __amdgpu_buffer_rsrc_t rout = state_rsrc(a.out, uint32_t(L::Q) * cstride);
    P2 ov[L::Q];
#pragma unroll
    for (int i = 0; i < L::Q; ++i) ov[i] = load_pair<P2>(rout, n * E, uint32_t(i) * cstride);
    Geo g;
    g.nx = a.nx;
    g.ny = a.ny;
    g.nz = a.nz;
    g.N = int64_t(a.nx) * a.ny * a.nz;
    g.pitch = a.pitch;
    g.mask = a.mask;
    g.inlets = a.inlets;
    g.outlets = a.outlets;
    g.walls = a.walls;
    g.links = a.links;
    OwnMom<T> om{};
    if (clk & kLinkOutlet) om = own_moments<L, S, T>(ov);
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        if (!((clk >> i) & 1u)) continue;
        const uint32_t m = nbr(a.nx, a.ny, a.nz, h, -L::cx[i], -L::cy[i], -L::cz[i]);
        const uint8_t c = (clk & kLinkMixed) ? a.mask[m] : link_code(clk);
        if (!is_wall(c))
            store_pair<P2>(rout, m * E, uint32_t(i) * cstride, boundary_pair<L, S, T>(g, mo, i, c, ov[L::opp[i]], om));
    }
}

template <typename S>
hipError_t run_split(const Geo &g, const ModelD &md, const void *in, void *out, float *psi, void *scratch,
                     const SplitPlan &sp, const uint32_t *ctr_in, uint32_t *ctr_out, hipStream_t s) {
    typedef typename PairOf<S>::type P2;
    if (!g.mask || !g.links || !psi || !scratch) return hipErrorInvalidValue;
    if (uint64_t(D3Q19::Q) * uint64_t(g.pitch) * sizeof(P2) >= (uint64_t(1) << 32)) return hipErrorInvalidValue;
    const int64_t nb = split_blocks(g.nx, g.ny, g.nz);
    if (nb <= 0 || nb > 0x7fffffff || sp.active > nb || sp.io > nb || sp.active < 0 || sp.io < 0)
        return hipErrorInvalidValue;
    const ScratchMap m = scratch_map(scratch, g.pitch, nb);
    SplitArgs<S> sa;
    sa.a = fused_args<S>(g, in, out, ctr_in, ctr_out, FusedShape{8, 1});
    sa.psi = psi;
    sa.mom = m.mom;
    const Model<float> mo = to_model<float>(md);
    sa.blocks = m.act;
    if (sp.active > 0) hipLaunchKernelGGL(k_geo_moments<S>, dim3(unsigned(sp.active)), dim3(kGeoBlock), 0, s, sa);
    // one block at least: it advances the step counter
    if (sp.active == 0) sa.blocks = nullptr;
    hipLaunchKernelGGL(k_geo_collide<S>, dim3(unsigned(sp.active > 0 ? sp.active : 1)), dim3(kGeoBlock), 0, s, sa,
                       mo);
    sa.blocks = m.io;
    if (sp.io > 0) hipLaunchKernelGGL(k_geo_boundary<S>, dim3(unsigned(sp.io)), dim3(kGeoBlock), 0, s, sa, mo);
    return hipGetLastError();
}

}  // namespace

int64_t split_blocks(int nx, int ny, int nz) {
    return int64_t((nx + kGX - 1) / kGX) * ((ny + kGY - 1) / kGY) * nz;
}

size_t split_scratch_bytes(int64_t pitch, int nx, int ny, int nz) {
    const int64_t nb = split_blocks(nx, ny, nz);
    return align256(sizeof(float) * kNM * size_t(pitch)) + align256(size_t(nb)) +
           2 * align256(sizeof(uint32_t) * size_t(nb)) + align256(2 * sizeof(uint32_t));
}

hipError_t split_prepare(const Geo &g, void *scratch, SplitPlan &sp, hipStream_t s) {
    sp = SplitPlan{};
    if (!g.links || !scratch) return hipErrorInvalidValue;
    const int64_t nb = split_blocks(g.nx, g.ny, g.nz);
    if (nb <= 0 || nb > 0x7fffffff) return hipErrorInvalidValue;
    const ScratchMap m = scratch_map(scratch, g.pitch, nb);
    hipLaunchKernelGGL(k_geo_flags, dim3(unsigned(nb)), dim3(kGeoBlock), 0, s, g.links, g.nx, g.ny, g.nz, m.flags);
    hipLaunchKernelGGL(k_geo_lists, dim3(1), dim3(kListThreads), 0, s, m.flags, uint32_t(nb), m.act, m.io, m.counts);
    hipError_t e = hipGetLastError();
    uint32_t c[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(c, m.counts, sizeof(c), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    if (int64_t(c[0]) > nb || int64_t(c[1]) > nb) return hipErrorUnknown;
    sp.active = c[0];
    sp.io = c[1];
    return hipSuccess;
}

hipError_t launch_step_split(int prec, const Geo &g, const ModelD &md, const void *in, void *out, void *psi,
                             void *scratch, const SplitPlan &sp, const uint32_t *ctr_in, uint32_t *ctr_out,
                             hipStream_t s) {
    if (md.bgk) return hipErrorInvalidValue;
    float *p = static_cast<float *>(psi);
    if (prec == 1) return run_split<float>(g, md, in, out, p, scratch, sp, ctr_in, ctr_out, s);
    if (prec == 2) return run_split<_Float16>(g, md, in, out, p, scratch, sp, ctr_in, ctr_out, s);
    return hipErrorInvalidValue;
}

}  // namespace lbcg
