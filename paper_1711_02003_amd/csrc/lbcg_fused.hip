// Fused single-pass D3Q19 RCG step (arXiv:1711.02003, Sec. II, Eqs. (1)-(11)).
//
// The colour gradient at x needs psi at the 18 neighbours at the same time
// level, and psi there needs the populations pulled from two hops away, so
// the step cannot be one independent pass per node.  Instead each block owns
// a column tile of 64 x R nodes (one wave per row) and sweeps a chunk of z
// planes.  For plane z+1 it pulls the 19 populations of its nodes (Eq. (1);
// each one a (total deviation, colour share) pair), keeps only the 12
// scalars the collision needs (drho, 36 rho^R, 36 rho^B, j, trace-adjusted
// momentum flux S), and writes psi of the tile plus a one-node ring (the ring
// recomputes the neighbours' densities from cache) into a 5-slot LDS ring
// buffer.  After one barrier it collides plane z with the gradient taken from
// the LDS planes z-1, z, z+1 and stores the 19 new pairs coalesced, with
// non-temporal stores (the new state is not read again in this step).  The
// populations of a plane (interior and ring) are loaded one iteration ahead
// of their use, so their latency overlaps the moments, the barrier, the
// collision and the stores; the barrier orders only LDS traffic and leaves
// those loads in flight.
//
// Every stored population is read from HBM once and written once: the
// algorithmic traffic is 2 x 38 x sizeof(storage) bytes per node.
//
// With a geometry mask (compile-time switch) the pull applies the boundary
// rules of the generic path (walls, velocity inlets, pressure outlets), psi
// of an inlet node is the inlet's phase value, psi of a wetting wall its
// own phase value, and a neutral wall or outlet neighbour contributes the
// centre node's psi to the gradient.
//
// Block -> work mapping (single lattice): work items (tile, z chunk) are
// numbered tile-major.  Periodic lattices deal them to the 8 XCDs in
// contiguous bands matching the round-robin dispatch of blocks to XCDs, so
// each XCD sweeps a compact band of tiles and the ring re-reads mostly hit
// that XCD's L2.  With geometry the fluid is usually concentrated in a few
// bands (a channel), so consecutive items go to consecutive XCDs instead:
// XCD k gets the z chunks k, k + 8, ... of every tile, which spreads the
// fluid evenly and still keeps each chunk's x-y neighbours on one XCD.  The
// batched form steps many lattices in one launch from a block -> (lattice,
// item) table, dealt the same two ways.
#include <type_traits>

#include "lbcg_buffer.h"
#include "lbcg_internal.h"

namespace lbcg {

constexpr int kTX = 64;
constexpr int kXCD = 8;
constexpr float kSentinel = 1e30f;  // LDS psi of a neutral wall or outlet node

// Barrier that orders LDS accesses only; global loads stay in flight.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Byte offsets (x' + nx y') * sizeof(pair) of the 9 source columns
// x' = x - c_x, y' = y - c_y of node (x, y), periodic; entry (1 - c_x) +
// 3 (1 - c_y).
template <typename S>
__device__ __forceinline__ void column_offsets(const FusedArgs<S> &a, int x, int y, uint32_t t[9]) {
    constexpr uint32_t E = sizeof(typename PairOf<S>::type);
    const uint32_t xs[3] = {uint32_t(x == 0 ? a.nx - 1 : x - 1), uint32_t(x), uint32_t(x == a.nx - 1 ? 0 : x + 1)};
    const uint32_t ys[3] = {uint32_t(y == 0 ? a.ny - 1 : y - 1), uint32_t(y), uint32_t(y == a.ny - 1 ? 0 : y + 1)};
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) t[c + 3 * b] = (xs[c] + uint32_t(a.nx) * ys[b]) * E;
}

// Populations requested but not yet used: the loaded pairs, decoded only
// where they are consumed so that nothing waits on a load before then, and
// (with geometry) the node's link word.
template <typename S, typename T>
struct Pending {
    typename PairOf<S>::type v[D3Q19::Q];
    uint32_t lk;
    __device__ __forceinline__ void take(Pops<D3Q19, T> &p) const {
        p.red = 0;
#pragma unroll
        for (int i = 0; i < D3Q19::Q; ++i) decode_pair<D3Q19, S, T>(v[i], i, p);
    }
};

// Request the 19 population pairs of a node at plane z from its column
// offsets t.  With geometry, a link whose upstream node is not fluid reads
// the boundary value that the node itself stored in that node's slot at the
// previous step, so every link is a plain load.
template <typename S, typename T>
__device__ __forceinline__ void pull_plane(const FusedArgs<S> &a, __amdgpu_buffer_rsrc_t r, const uint32_t t[9],
                                           int z, Pending<S, T> &pend) {
    using L = D3Q19;
    typedef typename PairOf<S>::type P2;
    constexpr uint32_t E = sizeof(P2);
    const uint32_t plane = uniform(int(uint32_t(a.nx) * uint32_t(a.ny) * E));
    const uint32_t cstride = uniform(int(uint32_t(a.pitch) * E));
    const uint32_t zo[3] = {uint32_t(uniform(z == 0 ? a.nz - 1 : z - 1)) * plane, uint32_t(uniform(z)) * plane,
                            uint32_t(uniform(z == a.nz - 1 ? 0 : z + 1)) * plane};
#pragma unroll
    for (int i = 0; i < L::Q; ++i)
        pend.v[i] = load_pair<P2>(r, t[(1 - L::cx[i]) + 3 * (1 - L::cy[i])], uint32_t(i) * cstride + zo[1 - L::cz[i]]);
}

__device__ __forceinline__ int wrapz(int z, int nz) { return z < 0 ? z + nz : (z >= nz ? z - nz : z); }

template <typename S>
__device__ __forceinline__ Geo geo_of(const FusedArgs<S> &a) {
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
    return g;
}

// One work item: column tile `tile`, z chunk `chunk` of one lattice.  POPS:
// the collision needs the node's populations, not only its moments (plain
// BGK, Eq. (5)): the decoded populations of the plane being collided are
// kept beside the moments until its collision.
template <typename S, typename T, int R, bool MASKED, bool POPS = false>
__device__ __forceinline__ void sweep(const FusedArgs<S> &a, const Model<T> &mo, int tile, int chunk,
                                      float *lds) {
    using L = D3Q19;
    constexpr int W = kTX + 2, H = R + 2, PL = W * H;  // LDS plane: (R+2) x 66
    const int lane = threadIdx.x % kTX, row = threadIdx.x / kTX;
    const int tx = tile % a.ntx, ty = tile / a.ntx;
    const int x0 = tx * kTX, y0 = ty * R;
    const int tw = min(kTX, a.nx - x0), th = min(R, a.ny - y0);
    const int z0 = int((int64_t(chunk) * a.nz) / a.zchunks);
    const int z1 = int((int64_t(chunk + 1) * a.nz) / a.zchunks);
    if (z1 <= z0) return;  // uniform over the block

    const bool intile = lane < tw && row < th;
    const int x = x0 + lane, y = y0 + row;
    const uint32_t step = *a.ctr_in;  // seeds the stochastic rounding of 16-bit shares

    // With geometry, a chunk whose own nodes are all non-fluid has nothing to
    // do: a non-fluid node's slots hold only the boundary values that its
    // fluid neighbours store there themselves, and the ring only feeds the
    // gradients of the chunk's own fluid nodes.
    if (MASKED) {
        bool any = false;
        if (intile)
            for (int zz = z0; zz < z1 && !any; ++zz)
                any = (a.links[int64_t(x) + int64_t(a.nx) * (int64_t(y) + int64_t(a.ny) * zz)] & kLinkFluid) != 0u;
        if (!__syncthreads_or(any)) return;  // uniform over the block
    }

    // ring node of this thread (at most one): rows -1 and th over x in [-1, tw],
    // then columns -1 and tw over y in [0, th)
    const int nring = 2 * (tw + 2) + 2 * th;
    int rx = 0, ry = 0;
    const bool has_ring = threadIdx.x < nring;
    if (has_ring) {
        const int r = threadIdx.x;
        if (r < tw + 2) {
            rx = r - 1;
            ry = -1;
        } else if (r < 2 * (tw + 2)) {
            rx = r - (tw + 2) - 1;
            ry = th;
        } else {
            const int q = r - 2 * (tw + 2);
            rx = q < th ? -1 : tw;
            ry = q < th ? q : q - th;
        }
    }
    const int gx = wrap_m1(x0 + rx, a.nx), gy = wrap_m1(y0 + ry, a.ny);

    typedef typename PairOf<S>::type P2;
    constexpr uint32_t E = sizeof(P2);
    const uint32_t cstride = uniform(int(uint32_t(a.pitch) * E));
    const uint32_t plane = uniform(int(uint32_t(a.nx) * uint32_t(a.ny) * E));
    const __amdgpu_buffer_rsrc_t rin = state_rsrc(a.in, uint32_t(L::Q) * cstride);
    const __amdgpu_buffer_rsrc_t rout = state_rsrc(a.out, uint32_t(L::Q) * cstride);
    // column offsets of the interior node and of the ring node (unused
    // entries of threads outside the tile stay in range)
    uint32_t ixy[9], rxy[9];
    column_offsets(a, intile ? x : 0, intile ? y : 0, ixy);
    column_offsets(a, gx, gy, rxy);

    auto node = [&](int xx, int yy, int zz) {
        return int64_t(xx) + int64_t(a.nx) * (int64_t(yy) + int64_t(a.ny) * zz);
    };
    // LDS psi of a non-fluid node: the inlet's or the wetting wall's phase
    // value, or the sentinel that the gradient replaces by the centre node's
    // own psi
    auto solid_psi = [&](uint8_t c) -> float {
        if (is_inlet(c)) {
            const DevInlet in = a.inlets[c - kInlet0];
            return float((in.rhoR - in.rhoB) / (in.rhoR + in.rhoB));
        }
        if (c >= kWall0 && c < kOutlet0) return float(a.walls[c - kWall0].psi);
        return kSentinel;
    };
    auto fluid = [&](uint32_t lk) { return !MASKED || (lk & kLinkFluid) != 0u; };
    // psi planes live in a 5-slot LDS ring: iteration z writes plane z+1
    // (interior and ring) and then collides plane z from planes z-1..z+1; the
    // barrier keeps the waves within one iteration of each other, so a slot
    // is rewritten only after every wave has passed its last read.
    auto slot_of = [&](int zp) { return lds + ((zp - z0 + 1) % 5) * PL; };

    // Ring nodes: psi of the one-node ring around the tile.  Ring and
    // interior populations of a plane are requested one iteration before
    // they are used, ring first: the neighbour tiles' rows are then requested
    // while those tiles load them too, and waiting for the ring (loads retire
    // in order) leaves the interior loads in flight.  With geometry, a node's
    // link word for a plane is read one request earlier.
    Pending<S, T> rp;
    rp.lk = kLinkFluid;
    uint32_t rlk = 0;  // link word of the next ring request
    if (MASKED && has_ring) rlk = a.links[node(gx, gy, wrapz(z0 - 1, a.nz))];
    auto ring_issue = [&](int zp) {
        if (has_ring) {
            const int zz = wrapz(zp, a.nz);
            rp.lk = MASKED ? rlk : kLinkFluid;
            if (fluid(rp.lk)) pull_plane<S, T>(a, rin, rxy, zz, rp);
            if (MASKED) rlk = a.links[node(gx, gy, wrapz(zp + 1, a.nz))];
        }
    };
    auto ring_finish = [&](int zp) {
        if (has_ring) {
            float v;
            if (fluid(rp.lk)) {
                Pops<L, T> q;
                rp.take(q);
                T dr, rR, rB;
                densities<L, T>(q, dr, rR, rB);
                v = float(psi_of<T>(dr, rR, rB));
            } else {
                v = solid_psi(link_code(rp.lk));
            }
            slot_of(zp)[(ry + 1) * W + rx + 1] = v;
        }
    };

    // Interior: moments of plane z are carried in registers, the populations
    // of plane z+1 are in flight.
    T cd = 0, cR = 0, cB = 0, cj[3] = {0, 0, 0}, cS[6] = {0, 0, 0, 0, 0, 0};
    bool cfl = false;
    // plain BGK: populations of the plane being collided (cq) and of the
    // plane whose moments were just taken (nq); nothing otherwise
    struct NoPops {};
    using Kept = typename std::conditional<POPS, Pops<L, T>, NoPops>::type;
    Kept cq{}, nq{};
    uint32_t clk = 0;  // link word of the plane being collided
    Pending<S, T> pp;
    pp.lk = kLinkFluid;
    uint32_t ilk = 0;  // link word of the next interior request
    if (MASKED && intile) ilk = a.links[node(x, y, wrapz(z0 - 1, a.nz))];
    int pz = 0;  // plane of the pending interior request
    auto interior_issue = [&](int zp) {
        if (intile) {
            pz = wrapz(zp, a.nz);
            pp.lk = MASKED ? ilk : kLinkFluid;
            if (fluid(pp.lk)) pull_plane<S, T>(a, rin, ixy, pz, pp);
            if (MASKED) ilk = a.links[node(x, y, wrapz(zp + 1, a.nz))];
        }
    };
    auto interior_take = [&](Pops<L, T> &q) { pp.take(q); };
    // moments of the pulled interior plane into (d, r36R, r36B, j, flux); returns psi
    auto interior_moments = [&](T &d, T &r36R, T &r36B, T j[3], T flux[6], bool &fl) -> float {
        fl = fluid(pp.lk);
        if (!fl) return solid_psi(link_code(pp.lk));
        Pops<L, T> q;
        interior_take(q);
        Mom<T> m;
        moments<L, T>(q, m);
        if constexpr (POPS) nq = q;
        d = m.drho;
        r36R = m.r36R;
        r36B = m.r36B;
        j[0] = m.j[0];
        j[1] = m.j[1];
        j[2] = m.j[2];
#pragma unroll
        for (int q = 0; q < 6; ++q) flux[q] = m.S[q];
        return float(psi_of<T>(m.drho, m.r36R, m.r36B));
    };

    // prologue: psi of planes z0-1 and z0, moments of z0, ring of z0+1 and
    // the interior loads of z0+1
    ring_issue(z0 - 1);
    interior_issue(z0 - 1);
    if (intile) {
        float v;
        if (fluid(pp.lk)) {
            Pops<L, T> q;
            interior_take(q);
            T dr, rR, rB;
            densities<L, T>(q, dr, rR, rB);
            v = float(psi_of<T>(dr, rR, rB));
        } else {
            v = solid_psi(link_code(pp.lk));
        }
        slot_of(z0 - 1)[(row + 1) * W + lane + 1] = v;
    }
    ring_finish(z0 - 1);
    ring_issue(z0);
    interior_issue(z0);
    if (intile) slot_of(z0)[(row + 1) * W + lane + 1] = interior_moments(cd, cR, cB, cj, cS, cfl);
    if constexpr (POPS) cq = nq;
    clk = pp.lk;
    ring_finish(z0);
    ring_issue(z0 + 1);
    interior_issue(z0 + 1);

    // Output pairs of the last collided plane.  Loads and stores share one
    // completion counter that the compiler cannot treat as ordered while both
    // are pending, so every use of a requested value waits for all
    // outstanding memory operations (the explicit wait at the top of the
    // sweep makes that wait one, on every path).  With 16-bit storage the
    // sweep is bound by arithmetic, and the stores are held one iteration
    // and issued right after the next plane is requested, so that wait finds
    // them complete; with 32-bit storage the sweep is bound by memory
    // traffic, and storing at once (measured faster) keeps more writes in
    // flight.
    constexpr bool kDelayStores = !MASKED && sizeof(P2) == 4;
    P2 ov[L::Q];
    bool ovalid = false;
    uint32_t ozoff = 0;
    auto flush = [&]() {
        if (ovalid) {
            const uint32_t zoff = uint32_t(uniform(int(ozoff)));
#pragma unroll
            for (int i = 0; i < L::Q; ++i) store_pair<P2>(rout, ixy[4], uint32_t(i) * cstride + zoff, ov[i]);
        }
    };

    for (int z = z0; z < z1; ++z) {
        const bool more = z + 2 <= z1;  // uniform over the block
        T nd = 0, nR = 0, nB = 0, nj[3] = {0, 0, 0}, nS[6] = {0, 0, 0, 0, 0, 0};
        bool nfl = false;
        // plane z+1: its ring and interior populations were requested one
        // iteration ago.  Wait for everything outstanding here, on every
        // path, so that no later use waits for the loads issued below.
        wait_memory();
        ring_finish(z + 1);
        if (intile) slot_of(z + 1)[(row + 1) * W + lane + 1] = interior_moments(nd, nR, nB, nj, nS, nfl);
        const uint32_t nlk = pp.lk;
        if (more) {
            ring_issue(z + 2);
            interior_issue(z + 2);
        }
        if (kDelayStores) flush();
        lds_barrier();
        ovalid = intile && (!MASKED || cfl);
        if (ovalid) {
            const float *sm = slot_of(z - 1), *s0 = slot_of(z), *sp = slot_of(z + 1);
            const int c = (row + 1) * W + lane + 1;
            const float pc = s0[c];
            T fx = 0, fy = 0, fz = 0;
#pragma unroll
            for (int i = 1; i < L::Q; ++i) {
                const float *sl = L::cz[i] > 0 ? sp : (L::cz[i] < 0 ? sm : s0);
                float pv = sl[c + L::cy[i] * W + L::cx[i]];
                if (MASKED) pv = pv == kSentinel ? pc : pv;
                const T wp = T(3.0 * wgt<L>(i)) * T(pv);
                if (L::cx[i]) fx += L::cx[i] > 0 ? wp : -wp;
                if (L::cy[i]) fy += L::cy[i] > 0 ? wp : -wp;
                if (L::cz[i]) fz += L::cz[i] > 0 ? wp : -wp;
            }
            const T F[3] = {fx, fy, fz};
            PostOut<L, T> o;
            const Pops<L, T> *pin = nullptr;
            if constexpr (POPS) pin = &cq;
            collide<L, T>(mo, cd, cR, cB, cj, cS, F, pin, o);
            Dither dz(step, uint32_t(x) + uint32_t(a.nx) * (uint32_t(y) + uint32_t(a.ny) * uint32_t(z)));
#pragma unroll
            for (int i = 0; i < L::Q; ++i) ov[i] = encode_step<L, S, T>(o.df[i], o.mm[i], (o.red >> i) & 1u, i, dz);
            // boundary values of the node's non-fluid links, stored in the
            // upstream nodes' slots (the addresses it pulls them from)
            if (MASKED && (clk & kLinkBits)) {
                const Geo g = geo_of(a);
                const uint32_t zg[3] = {uint32_t(uniform(z == 0 ? a.nz - 1 : z - 1)) * plane,
                                        uint32_t(uniform(z)) * plane,
                                        uint32_t(uniform(z == a.nz - 1 ? 0 : z + 1)) * plane};
                OwnMom<T> om{};
                if (clk & kLinkOutlet) om = own_moments<L, S, T>(ov);
#pragma unroll
                for (int i = 1; i < L::Q; ++i) {
                    if (!((clk >> i) & 1u)) continue;
                    uint8_t c = link_code(clk);
                    if (clk & kLinkMixed)
                        c = a.mask[node(wrap_m1(x - L::cx[i], a.nx), wrap_m1(y - L::cy[i], a.ny),
                                        wrap_m1(z - L::cz[i], a.nz))];
                    store_pair<P2>(rout, ixy[(1 - L::cx[i]) + 3 * (1 - L::cy[i])],
                                   uint32_t(i) * cstride + zg[1 - L::cz[i]],
                                   boundary_pair<L, S, T>(g, mo, i, c, ov[L::opp[i]], om));
                }
            }
        }
        ozoff = uint32_t(uniform(z)) * plane;
        if (!kDelayStores) flush();
        cfl = nfl;
        clk = nlk;
        if constexpr (POPS) cq = nq;
        cd = nd;
        cR = nR;
        cB = nB;
#pragma unroll
        for (int q = 0; q < 3; ++q) cj[q] = nj[q];
#pragma unroll
        for (int q = 0; q < 6; ++q) cS[q] = nS[q];
    }
    if (kDelayStores) flush();
}

// Block -> table or item index: XCD bands for periodic lattices, plain
// order (consecutive indices on consecutive XCDs) with geometry.
template <bool MASKED>
__device__ __forceinline__ int work_index(int total) {
    if (MASKED) return int(blockIdx.x);
    const int xcd = blockIdx.x % kXCD, l = blockIdx.x / kXCD;
    return xcd * (total / kXCD) + min(xcd, total % kXCD) + l;
}

// Single lattice (see the file comment for the work mapping).
template <typename S, typename T, int R, bool MASKED, bool POPS>
__global__ void __launch_bounds__(kTX * R) k_step_fused(FusedArgs<S> a, Model<T> mo) {
    extern __shared__ float lds[];
    const int item = work_index<MASKED>(a.ntx * a.nty * a.zchunks);
    if (item == 0 && threadIdx.x == 0) *a.ctr_out = *a.ctr_in + 1u;
    sweep<S, T, R, MASKED, POPS>(a, mo, item / a.zchunks, item % a.zchunks, lds);
}

// Many lattices in one launch: the grid covers table entries [0, gridDim.x),
// dealt to the XCDs as above; entry k is work item bitem[k] of lattice
// blat[k].
template <typename S, typename T, int R, bool MASKED>
__global__ void __launch_bounds__(kTX * R)
    k_step_fused_batch(const BatchDesc<S> *__restrict__ desc, const int *__restrict__ blat,
                       const int *__restrict__ bitem) {
    extern __shared__ float lds[];
    const int k = work_index<MASKED>(int(gridDim.x));
    const int item = bitem[k];
    const BatchDesc<S> d = desc[blat[k]];
    if (item == 0 && threadIdx.x == 0) *d.a.ctr_out = *d.a.ctr_in + 1u;
    sweep<S, T, R, MASKED>(d.a, d.mo, item / d.a.zchunks, item % d.a.zchunks, lds);
}

bool fused_supported(int lattice, int prec, const Geo &g) {
    const uint64_t elem = prec == 1 ? 4 : 2;
    return lattice == 1 && (prec == 1 || prec == 2) &&
           uint64_t(2 * D3Q19::Q) * uint64_t(g.pitch) * elem < (uint64_t(1) << 32);
}

static size_t fused_lds(int R) { return size_t(5) * (R + 2) * (kTX + 2) * sizeof(float); }

template <typename S, int R>
static const void *fused_fn(bool masked) {
    return masked ? reinterpret_cast<const void *>(&k_step_fused<S, float, R, true, false>)
                  : reinterpret_cast<const void *>(&k_step_fused<S, float, R, false, false>);
}
template <typename S>
static const void *fused_fn_pops(bool masked) {
    return masked ? reinterpret_cast<const void *>(&k_step_fused<S, float, 8, true, true>)
                  : reinterpret_cast<const void *>(&k_step_fused<S, float, 8, false, true>);
}

int fused_resident_blocks(int prec, int rows, bool masked, bool pops) {
    int per_cu = 0;
    const void *fn = pops ? (prec == 2 ? fused_fn_pops<_Float16>(masked) : fused_fn_pops<float>(masked))
                     : prec == 2 ? (rows == 4 ? fused_fn<_Float16, 4>(masked) : fused_fn<_Float16, 8>(masked))
                                 : (rows == 4 ? fused_fn<float, 4>(masked) : fused_fn<float, 8>(masked));
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kTX * rows, fused_lds(rows)) != hipSuccess) {
        (void)hipGetLastError();
        per_cu = 1;
    }
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return (per_cu > 0 ? per_cu : 1) * cus;
}

template <typename S>
FusedArgs<S> fused_args(const Geo &g, const void *in, void *out, const uint32_t *ctr_in, uint32_t *ctr_out,
                        FusedShape sh) {
    FusedArgs<S> a;
    a.in = static_cast<const S *>(in);
    a.out = static_cast<S *>(out);
    a.ctr_in = ctr_in;
    a.ctr_out = ctr_out;
    a.nx = g.nx;
    a.ny = g.ny;
    a.nz = g.nz;
    a.pitch = g.pitch;
    a.mask = g.mask;
    a.inlets = g.inlets;
    a.outlets = g.outlets;
    a.walls = g.walls;
    a.links = g.links;
    a.ntx = (g.nx + kTX - 1) / kTX;
    a.nty = (g.ny + sh.rows - 1) / sh.rows;
    a.zchunks = sh.zchunks < 1 ? 1 : (sh.zchunks > g.nz ? g.nz : sh.zchunks);
    return a;
}
template FusedArgs<float> fused_args<float>(const Geo &, const void *, void *, const uint32_t *, uint32_t *,
                                            FusedShape);
template FusedArgs<_Float16> fused_args<_Float16>(const Geo &, const void *, void *, const uint32_t *, uint32_t *,
                                                  FusedShape);

template <typename S, int R, bool MASKED, bool POPS = false>
static void launch_one(const FusedArgs<S> &a, const Model<float> &mo, unsigned nblocks, hipStream_t s) {
    hipLaunchKernelGGL((k_step_fused<S, float, R, MASKED, POPS>), dim3(nblocks), dim3(kTX * R), fused_lds(R), s, a,
                       mo);
}

template <typename S>
static hipError_t run_fused(const Geo &g, const ModelD &md, const void *in, void *out, const uint32_t *ctr_in,
                            uint32_t *ctr_out, FusedShape sh, hipStream_t s) {
    const int R = sh.rows;
    // Rows 4 and 8 only: a 1024-thread block (16 rows) caps the kernel at 128
    // VGPRs, where it spills.
    if (R != 4 && R != 8) return hipErrorInvalidValue;
    typedef typename PairOf<S>::type P2;
    // 32-bit byte offsets must cover a state buffer
    if (uint64_t(D3Q19::Q) * uint64_t(g.pitch) * sizeof(P2) >= (uint64_t(1) << 32)) return hipErrorInvalidValue;
    const FusedArgs<S> a = fused_args<S>(g, in, out, ctr_in, ctr_out, sh);
    const int64_t nblocks = int64_t(a.ntx) * a.nty * a.zchunks;
    if (nblocks > 0x7fffffff) return hipErrorInvalidValue;
    const Model<float> mo = to_model<float>(md);
    const bool masked = g.mask != nullptr;
    const unsigned nb = unsigned(nblocks);
    if (md.bgk) {
        // plain BGK keeps a plane of populations per thread: 8-row tiles only
        if (R != 8) return hipErrorInvalidValue;
        masked ? launch_one<S, 8, true, true>(a, mo, nb, s) : launch_one<S, 8, false, true>(a, mo, nb, s);
        return hipGetLastError();
    }
    if (R == 4)
        masked ? launch_one<S, 4, true>(a, mo, nb, s) : launch_one<S, 4, false>(a, mo, nb, s);
    else
        masked ? launch_one<S, 8, true>(a, mo, nb, s) : launch_one<S, 8, false>(a, mo, nb, s);
    return hipGetLastError();
}

hipError_t launch_step_fused(int prec, const Geo &g, const ModelD &md, const void *in, void *out,
                             const uint32_t *ctr_in, uint32_t *ctr_out, FusedShape shape, hipStream_t s) {
    if (prec == 1) return run_fused<float>(g, md, in, out, ctr_in, ctr_out, shape, s);
    if (prec == 2) return run_fused<_Float16>(g, md, in, out, ctr_in, ctr_out, shape, s);
    return hipErrorInvalidValue;
}

template <typename S, int R, bool MASKED>
static void launch_batch(const void *desc, const int *blat, const int *bitem, unsigned nblocks, hipStream_t s) {
    hipLaunchKernelGGL((k_step_fused_batch<S, float, R, MASKED>), dim3(nblocks), dim3(kTX * R), fused_lds(R), s,
                       static_cast<const BatchDesc<S> *>(desc), blat, bitem);
}

template <typename S>
static hipError_t run_batch(const void *desc, const int *blat, const int *bitem, int nblocks, int rows,
                            bool masked, hipStream_t s) {
    const unsigned nb = unsigned(nblocks);
    if (rows == 4)
        masked ? launch_batch<S, 4, true>(desc, blat, bitem, nb, s)
               : launch_batch<S, 4, false>(desc, blat, bitem, nb, s);
    else if (rows == 8)
        masked ? launch_batch<S, 8, true>(desc, blat, bitem, nb, s)
               : launch_batch<S, 8, false>(desc, blat, bitem, nb, s);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_step_fused_batch(int prec, const void *desc, const int *blat, const int *bitem, int nblocks,
                                   int rows, bool masked, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    if (prec == 1) return run_batch<float>(desc, blat, bitem, nblocks, rows, masked, s);
    if (prec == 2) return run_batch<_Float16>(desc, blat, bitem, nblocks, rows, masked, s);
    return hipErrorInvalidValue;
}

}  // namespace lbcg
