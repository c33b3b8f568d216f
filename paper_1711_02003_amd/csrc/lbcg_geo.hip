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
//     stores their values (from its new pairs, read back); one thread per
//     such node and direction, from a list of the nodes.
// Every value is computed by the expressions and in the order of the column
// sweep, so the results are bitwise those of the sweep.  Traffic per fluid
// node: pairs read and written once (2 x 38 x E bytes), plus 12 moments and
// psi written and read once (2 x 52 bytes), the neighbours' psi from cache,
// and at nodes next to a boundary their new pairs read back.  The same three
// kernels also run on the compact state (below): 2 x 96 (FP32) or 2 x 50
// (FP16) bytes of state per fluid node instead of 2 x 152 or 2 x 76.
#include "lbcg_buffer.h"
#include "lbcg_compact_sweep.h"  // CStore: the compact state's storage
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
    const uint32_t *blocks;     // the kernel's block list (the boundary kernel's: its node list)
};

// Scratch layout: the moments, then the per-block flags, the per-block
// counts of nodes with inlet or outlet links, the list of blocks with fluid,
// the list of blocks with inlet or outlet links, the offsets of their nodes
// in the node list, the node list and the three lengths.
struct ScratchMap {
    float *mom;
    uint8_t *flags;
    uint16_t *ioc;
    uint32_t *act, *io, *ioofs, *ionodes, *counts;
};
__host__ __device__ inline size_t align256(size_t v) { return (v + 255) / 256 * 256; }
inline ScratchMap scratch_map(void *scratch, int64_t pitch, int64_t nb) {
    char *p = static_cast<char *>(scratch);
    ScratchMap m;
    m.mom = reinterpret_cast<float *>(p);
    p += align256(sizeof(float) * kNM * size_t(pitch));
    m.flags = reinterpret_cast<uint8_t *>(p);
    p += align256(size_t(nb));
    m.ioc = reinterpret_cast<uint16_t *>(p);
    p += align256(sizeof(uint16_t) * size_t(nb));
    m.act = reinterpret_cast<uint32_t *>(p);
    p += align256(sizeof(uint32_t) * size_t(nb));
    m.io = reinterpret_cast<uint32_t *>(p);
    p += align256(sizeof(uint32_t) * size_t(nb));
    m.ioofs = reinterpret_cast<uint32_t *>(p);
    p += align256(sizeof(uint32_t) * size_t(nb));
    m.ionodes = reinterpret_cast<uint32_t *>(p);
    p += align256(sizeof(uint32_t) * size_t(pitch));
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

// Rank of this thread's node among the block's nodes with `pred` (in
// thread order) and, through `total`, their count.
__device__ __forceinline__ uint32_t block_rank(bool pred, uint32_t &total) {
    __shared__ uint32_t wc[kGeoBlock / 64];
    const uint64_t bal = __builtin_amdgcn_ballot_w64(pred);
    const uint32_t lane = __builtin_amdgcn_mbcnt_hi(uint32_t(bal >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(bal), 0u));
    const int w = int(threadIdx.x / 64);
    if (threadIdx.x % 64 == 0) wc[w] = uint32_t(__builtin_popcountll(bal));
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int k = 0; k < kGeoBlock / 64; ++k) {
        before += k < w ? wc[k] : 0u;
        all += wc[k];
    }
    total = all;
    return before + lane;
}

// Flags of block b: 1 = some node fluid, 2 = some node with an inlet or
// outlet link (mixed codes count: the boundary kernel checks each link);
// and the number of such nodes.
__global__ void __launch_bounds__(kGeoBlock) k_geo_flags(const uint32_t *__restrict__ links, int nx, int ny, int nz,
                                                        uint8_t *__restrict__ flags, uint16_t *__restrict__ ioc) {
    Here h;
    const bool in = here(nx, ny, nz, blockIdx.x, h);
    const uint32_t lk = in ? links[h.n] : 0u;
    const int f = __syncthreads_or((lk & kLinkFluid) != 0u);
    uint32_t nio = 0;
    block_rank(has_io_link(lk), nio);
    if (threadIdx.x == 0) {
        flags[blockIdx.x] = uint8_t((f ? 1 : 0) | (nio ? 2 : 0));
        ioc[blockIdx.x] = uint16_t(nio);
    }
}

// The two block lists in ascending block order, and for each listed io
// block the offset of its nodes in the io node list, by one block: thread t
// takes the flags of a contiguous range, counts, and writes its entries
// after the counts of the threads before it.
constexpr int kListThreads = 1024;
__global__ void __launch_bounds__(kListThreads) k_geo_lists(const uint8_t *__restrict__ flags,
                                                           const uint16_t *__restrict__ ioc, uint32_t nb,
                                                           uint32_t *__restrict__ act, uint32_t *__restrict__ io,
                                                           uint32_t *__restrict__ ioofs,
                                                           uint32_t *__restrict__ counts) {
    __shared__ uint32_t ca[kListThreads], ci[kListThreads], cn[kListThreads], tot[3];
    const uint32_t per = (nb + kListThreads - 1) / kListThreads;
    const uint32_t b0 = min(nb, threadIdx.x * per), b1 = min(nb, b0 + per);
    uint32_t na = 0, ni = 0, nn = 0;
    for (uint32_t b = b0; b < b1; ++b) {
        na += flags[b] & 1u;
        ni += (flags[b] >> 1) & 1u;
        nn += ioc[b];
    }
    ca[threadIdx.x] = na;
    ci[threadIdx.x] = ni;
    cn[threadIdx.x] = nn;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t sa = 0, si = 0, sn = 0;
        for (int t = 0; t < kListThreads; ++t) {
            const uint32_t va = ca[t], vi = ci[t], vn = cn[t];
            ca[t] = sa;
            ci[t] = si;
            cn[t] = sn;
            sa += va;
            si += vi;
            sn += vn;
        }
        tot[0] = sa;
        tot[1] = si;
        tot[2] = sn;
    }
    __syncthreads();
    if (threadIdx.x < 3) counts[threadIdx.x] = tot[threadIdx.x];  // a lane each: no wide store
    uint32_t oa = ca[threadIdx.x], oi = ci[threadIdx.x], on = cn[threadIdx.x];
    for (uint32_t b = b0; b < b1; ++b) {
        if (flags[b] & 1u) act[oa++] = b;
        if (flags[b] & 2u) {
            ioofs[oi] = on;
            io[oi++] = b;
            on += ioc[b];
        }
    }
}

// The io node list: block k of the io block list writes its nodes with
// inlet or outlet links, in thread order, from offset ioofs[k].
__global__ void __launch_bounds__(kGeoBlock) k_geo_ionodes(const uint32_t *__restrict__ links, int nx, int ny, int nz,
                                                          const uint32_t *__restrict__ io,
                                                          const uint32_t *__restrict__ ioofs,
                                                          uint32_t *__restrict__ ionodes) {
    Here h;
    const bool in = here(nx, ny, nz, io[blockIdx.x], h);
    const bool mine = in && has_io_link(links[h.n]);
    uint32_t total = 0;
    const uint32_t r = block_rank(mine, total);
    if (mine) ionodes[ioofs[blockIdx.x] + r] = h.n;
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
// to 137.  A wave takes one direction i (uniform over the wave) for 64 nodes
// of the io node list; lanes whose node has no inlet or outlet link i leave
// at once.  One thread per node looping over its 18 links took 12-13 us on
// the 512 x 128 x 64 junction (7 936 such nodes, one wave per CU, each wave
// running the 18 links' code one after another); one thread per block node
// over the io blocks, 13 us.
constexpr int kIoBlock = 64;

// Opposite of D3Q19 direction i from the numbering (rest; +x -x +y -y +z -z;
// then per plane (+,+) (+,-) (-,+) (-,-)), for a direction known only at run
// time; checked against the lattice table at compile time.
__host__ __device__ constexpr int opp19(int i) {
    return i == 0 ? 0 : i <= 6 ? ((i & 1) ? i + 1 : i - 1) : i - 2 * ((i - 7) % 4) + 3;
}
constexpr bool opp19_matches() {
    for (int i = 0; i < D3Q19::Q; ++i)
        if (opp19(i) != D3Q19::opp[i]) return false;
    return true;
}
static_assert(opp19_matches(), "D3Q19 opposite directions");

// Link I of node n; so_i and so_o are the byte offsets of the arrays of
// directions I and opp(I), passed in from before any branch that lanes take
// differently, so that they stay in scalar registers.
template <int I, typename S>
__device__ __forceinline__ void io_link(const FusedArgs<S> &a, const Model<float> &mo, uint32_t n, uint32_t so_i,
                                        uint32_t so_o) {
    using L = D3Q19;
    typedef float T;
    typedef typename PairOf<S>::type P2;
    constexpr uint32_t E = sizeof(P2);
    const uint32_t clk = a.links[n];
    if (!((clk >> I) & 1u)) return;
    Here h;
    const uint32_t t = n / uint32_t(a.nx);
    h.n = n;
    h.x = int(n - t * uint32_t(a.nx));
    h.z = int(t / uint32_t(a.ny));
    h.y = int(t - uint32_t(h.z) * uint32_t(a.ny));
    const uint32_t m = nbr(a.nx, a.ny, a.nz, h, -L::cx[I], -L::cy[I], -L::cz[I]);
    const uint8_t c = (clk & kLinkMixed) ? a.mask[m] : link_code(clk);
    if (is_wall(c)) return;
    const uint32_t cstride = uint32_t(a.pitch) * E;
    const __amdgpu_buffer_rsrc_t rout = state_rsrc(a.out, uint32_t(L::Q) * cstride);
    Geo g{};
    g.inlets = a.inlets;
    g.outlets = a.outlets;
    OwnMom<T> om{};
    P2 own;
    if (c >= kOutlet0) {
        // outlet values need the node's own moments, from all its new pairs
        P2 ov[L::Q];
#pragma unroll
        for (int i = 0; i < L::Q; ++i) ov[i] = load_pair<P2>(rout, n * E, uint32_t(i) * cstride);
        om = own_moments<L, S, T>(ov);
        own = ov[L::opp[I]];
    } else {
        own = load_pair<P2>(rout, n * E, uint32_t(uniform(int(so_o))));
    }
    store_pair<P2>(rout, m * E, uint32_t(uniform(int(so_i))),
                   boundary_pair_v<L, S, T>(mo, I, c, io_vals<T>(g, c), own, om));
}

template <typename S>
__global__ void __launch_bounds__(kIoBlock) k_geo_boundary(SplitArgs<S> sa, Model<float> mo, uint32_t count) {
    // block b: direction 1 + b % 18 of list entries 64 (b / 18) .. + 63
    typedef typename PairOf<S>::type P2;
    const uint32_t b = blockIdx.x, chunk = b / 18u, dir = 1u + (b - chunk * 18u);
    const uint32_t cstride = uint32_t(sa.a.pitch) * uint32_t(sizeof(P2));
    const uint32_t so_i = dir * cstride, so_o = uint32_t(opp19(int(dir))) * cstride;
    const uint32_t k = chunk * kIoBlock + threadIdx.x;
    if (k >= count) return;
    const uint32_t n = sa.blocks[k];
    switch (dir) {
        case 1: io_link<1, S>(sa.a, mo, n, so_i, so_o); break;
        case 2: io_link<2, S>(sa.a, mo, n, so_i, so_o); break;
        case 3: io_link<3, S>(sa.a, mo, n, so_i, so_o); break;
        case 4: io_link<4, S>(sa.a, mo, n, so_i, so_o); break;
        case 5: io_link<5, S>(sa.a, mo, n, so_i, so_o); break;
        case 6: io_link<6, S>(sa.a, mo, n, so_i, so_o); break;
        case 7: io_link<7, S>(sa.a, mo, n, so_i, so_o); break;
        case 8: io_link<8, S>(sa.a, mo, n, so_i, so_o); break;
        case 9: io_link<9, S>(sa.a, mo, n, so_i, so_o); break;
        case 10: io_link<10, S>(sa.a, mo, n, so_i, so_o); break;
        case 11: io_link<11, S>(sa.a, mo, n, so_i, so_o); break;
        case 12: io_link<12, S>(sa.a, mo, n, so_i, so_o); break;
        case 13: io_link<13, S>(sa.a, mo, n, so_i, so_o); break;
        case 14: io_link<14, S>(sa.a, mo, n, so_i, so_o); break;
        case 15: io_link<15, S>(sa.a, mo, n, so_i, so_o); break;
        case 16: io_link<16, S>(sa.a, mo, n, so_i, so_o); break;
        case 17: io_link<17, S>(sa.a, mo, n, so_i, so_o); break;
        default: io_link<18, S>(sa.a, mo, n, so_i, so_o); break;
    }
}

// ------------------------------------------------------------ compact state
// The same split step on the compact state, FP32 or FP16 storage (the
// layout and rounding of the periodic compact sweep, CStore: 19 arrays of
// totals, then records {M with the majority flag, V_axis} and R_d; 96 or 50
// B per node).  A receiver splits each pulled total with its sender's record
// (the recolouring of Eq. (10) done at the receiver).  A link from a wall
// brings back the node's own new total of the opposite direction, split with
// its own record for that direction, so walls need no stored values.  A link
// from an inlet or an outlet reads the pair (total deviation, minority share)
// that the boundary kernel stored in that node's slot of a pair buffer (the
// values of the pair-state step, formed from the node's own new
// populations).
template <typename S>
struct CGeoArgs {
    SplitArgs<S> s;      // s.a.in: pair buffer read (inlet and outlet values), s.a.out: pair buffer written
    const uint8_t *cin;  // compact state read
    uint8_t *cout;       // compact state written
};
template <typename S>
constexpr uint32_t c_bytes() {  // bytes per node of the compact state
    return uint32_t(D3Q19::Q) * CStore<S>::E + CStore<S>::kRecA + CStore<S>::kRecB;
}

// Record of node u: minority share M and majority flag, V_axis, R_d.
struct CRec {
    float M, Va[3], Rd;
    bool fl;
};
template <typename S>
__device__ __forceinline__ CRec c_record(__amdgpu_buffer_rsrc_t rc, uint32_t u, uint32_t pitch) {
    typedef CStore<S> St;
    const uint32_t base = uint32_t(D3Q19::Q) * pitch * St::E;
    const typename St::RawB rb = St::load_b(rc, u * St::kRecB, base + pitch * St::kRecA);
    const f4 e = St::entry(St::load_a(rc, u * St::kRecA, base), rb);
    CRec c;
    c.M = Codec<float>::col<float>(e[0], c.fl);
    c.Va[0] = e[1];
    c.Va[1] = e[2];
    c.Va[2] = e[3];
    c.Rd = St::ratio(rb);
    return c;
}
// Total deviation f_i - w_i stored at element `at` of the totals (i * pitch
// + node; a direction of the speed class of i).
template <typename S>
__device__ __forceinline__ float c_total(__amdgpu_buffer_rsrc_t rc, uint32_t at, int i) {
    return CStore<S>::df(CStore<S>::load(rc, at * CStore<S>::E, 0u), i);
}
// 36 x the recolouring term of a population the record's node sends along
// c_i: c_i . V_axis, times R_d on a diagonal (the periodic sweep's split)
__device__ __forceinline__ float c_vd(int i, const CRec &r) {
    using L = D3Q19;
    const float cva = float(L::cx[i]) * r.Va[0] + float(L::cy[i]) * r.Va[1] + float(L::cz[i]) * r.Va[2];
    const int n2 = csq<L>(i);
    return n2 == 0 ? 0.0f : (n2 == 1 ? cva : r.Rd * cva);
}
// Pair (total deviation, minority share with flag) of the population the
// record's node sends along c_i with total deviation d: the conversion the
// periodic compact state's export uses.
template <typename S>
__device__ __forceinline__ typename PairOf<S>::type c_pair(float d, int i, const CRec &r) {
    using L = D3Q19;
    const float f = float(wgt<L>(i)) + d;
    const float mu36 = r.M * (float(w36<L>(i)) + 36.0f * d) + c_vd(i, r);
    const float q = f != 0.0f ? mu36 / (36.0f * f) : 0.0f;
    const bool keep = q <= 0.5f;
    return encode_pair<L, S, float>(d, keep ? q : 1.0f - q, keep ? r.fl : !r.fl, i);
}

// The node's own moments (density, red density, velocity) from its new
// totals and record: own_moments of its populations, each split as a
// receiver splits it (no division per population).
template <typename S>
__device__ __forceinline__ OwnMom<float> c_own_moments(__amdgpu_buffer_rsrc_t rc, uint32_t n, uint32_t pitch,
                                                       const CRec &r) {
    using L = D3Q19;
    float drho = 0, Ra = 0, jx = 0, jy = 0, jz = 0;
    int K = 0;
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
        const float d = c_total<S>(rc, uint32_t(k) * pitch + n, k);
        const float mu = r.M * (float(w36<L>(k)) + 36.0f * d) + c_vd(k, r);
        const float t = 36.0f * d - mu;
        drho += d;
        Ra += r.fl ? t : mu;
        K += r.fl ? w36<L>(k) : 0;
        jx += float(L::cx[k]) * d;
        jy += float(L::cy[k]) * d;
        jz += float(L::cz[k]) * d;
    }
    OwnMom<float> om;
    om.rho = 1.0f + drho;
    om.rR = (float(K) + Ra) / 36.0f;
    om.u[0] = jx / om.rho;
    om.u[1] = jy / om.rho;
    om.u[2] = jz / om.rho;
    return om;
}

// Each link is one load of a total and one of a record (from the cache: a
// record serves up to 19 receivers).  Staging the block's records with a
// one-node halo in LDS first (66 x 6 x 3 per block) measured slower on the
// 512 x 128 x 64 junction: 0.129 against 0.119 ms per step.
template <typename S>
__global__ void __launch_bounds__(kGeoBlock) k_cgeo_moments(CGeoArgs<S> ca) {
    using L = D3Q19;
    typedef float T;
    typedef typename PairOf<S>::type P2;
    constexpr uint32_t E = sizeof(P2);
    const FusedArgs<S> &a = ca.s.a;
    Here h;
    if (!here(a.nx, a.ny, a.nz, ca.s.blocks[blockIdx.x], h)) return;
    const uint32_t pitch = uint32_t(a.pitch);
    const __amdgpu_buffer_rsrc_t rc = state_rsrc(ca.cin, c_bytes<S>() * pitch);
    const uint32_t n = h.n;
    const uint32_t clk = a.links[n];
    if (!(clk & kLinkFluid)) return;
    // links from walls and from inlets or outlets (a node whose non-fluid
    // neighbours mix codes reads them from the mask)
    uint32_t wall = 0;
    if (clk & kLinkMixed) {
#pragma unroll
        for (int i = 1; i < L::Q; ++i)
            if ((clk >> i) & 1u)
                wall |= is_wall(a.mask[nbr(a.nx, a.ny, a.nz, h, -L::cx[i], -L::cy[i], -L::cz[i])]) ? (1u << i) : 0u;
    } else if (is_wall(link_code(clk))) {
        wall = clk & kLinkBits;
    }
    const uint32_t io = clk & kLinkBits & ~wall;
    // Every link as a plain load with a per-lane address: from a fluid node
    // its total of direction i and its record; from a wall the node's own
    // total of the opposite direction and its own record, the recolouring
    // term with the opposite sign.  Links from inlets and outlets are
    // replaced below.
    CPops<L, T> q;
    q.red = 0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const bool wl = (wall >> i) & 1u;
        const uint32_t u = nbr(a.nx, a.ny, a.nz, h, -L::cx[i], -L::cy[i], -L::cz[i]);
        const uint32_t src = wl ? uint32_t(L::opp[i]) * pitch + n : uint32_t(i) * pitch + u;
        const float d = c_total<S>(rc, src, i);
        const CRec r = c_record<S>(rc, wl ? n : u, pitch);
        const float vd = c_vd(i, r);
        q.df[i] = d;
        q.mm[i] = r.M;
        q.vd[i] = wl ? -vd : vd;
        q.red |= r.fl ? (1u << i) : 0u;
    }
    if (io) {
        const __amdgpu_buffer_rsrc_t rg = state_rsrc(a.in, uint32_t(L::Q) * pitch * E);
#pragma unroll
        for (int i = 1; i < L::Q; ++i) {
            if (!((io >> i) & 1u)) continue;
            const uint32_t u = nbr(a.nx, a.ny, a.nz, h, -L::cx[i], -L::cy[i], -L::cz[i]);
            const P2 v = load_pair<P2>(rg, u * E, uniform(int(uint32_t(i) * pitch * E)));
            bool fl;
            q.df[i] = Codec<S>::template df<L, T>(v.x, i);
            q.mm[i] = Codec<S>::template col<T>(v.y, fl);
            q.vd[i] = 0.0f;
            q.red = fl ? (q.red | (1u << i)) : (q.red & ~(1u << i));
        }
    }
    Mom<T> mm;
    moments<L, T>(q, mm);
    ca.s.psi[n] = float(psi_of<T>(mm.drho, mm.r36R, mm.r36B));
    const float vals[kNM] = {mm.drho, mm.r36R, mm.r36B, mm.j[0], mm.j[1], mm.j[2],
                             mm.S[0], mm.S[1], mm.S[2], mm.S[3], mm.S[4], mm.S[5]};
#pragma unroll
    for (int k = 0; k < kNM; ++k) ca.s.mom[int64_t(k) * a.pitch + n] = vals[k];
}

template <typename S>
__global__ void __launch_bounds__(kGeoBlock) k_cgeo_collide(CGeoArgs<S> ca, Model<float> mo) {
    using L = D3Q19;
    typedef float T;
    const FusedArgs<S> &a = ca.s.a;
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.ctr_out = *a.ctr_in + 1u;
    if (!ca.s.blocks) return;  // no fluid node
    Here h;
    if (!here(a.nx, a.ny, a.nz, ca.s.blocks[blockIdx.x], h)) return;
    const uint32_t n = h.n;
    const uint32_t clk = a.links[n];
    if (!(clk & kLinkFluid)) return;
    const uint32_t step = *a.ctr_in;  // seeds the stochastic rounding of FP16 storage
    const float pc = ca.s.psi[n];
    T fx = 0, fy = 0, fz = 0;
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        const uint32_t m = nbr(a.nx, a.ny, a.nz, h, L::cx[i], L::cy[i], L::cz[i]);
        const float pv = ((clk >> L::opp[i]) & 1u) ? solid_psi(a, a.mask[m], pc) : ca.s.psi[m];
        const T wp = T(3.0 * wgt<L>(i)) * T(pv);
        if (L::cx[i]) fx += L::cx[i] > 0 ? wp : -wp;
        if (L::cy[i]) fy += L::cy[i] > 0 ? wp : -wp;
        if (L::cz[i]) fz += L::cz[i] > 0 ? wp : -wp;
    }
    const T F[3] = {fx, fy, fz};
    T mv[kNM];
#pragma unroll
    for (int k = 0; k < kNM; ++k) mv[k] = ca.s.mom[int64_t(k) * a.pitch + n];
    const T cj[3] = {mv[3], mv[4], mv[5]}, cS[6] = {mv[6], mv[7], mv[8], mv[9], mv[10], mv[11]};
    CompactOut<L, T> o;
    collide<L, T>(mo, mv[0], mv[1], mv[2], cj, cS, F, nullptr, o);
    const uint32_t pitch = uint32_t(a.pitch);
    const __amdgpu_buffer_rsrc_t rout = state_rsrc(ca.cout, c_bytes<S>() * pitch);
    // the node's totals at byte n E of each array, its records at n kRecA
    // and n kRecB (the periodic sweep's store, with the plane offset 0)
    CStore<S>::store(rout, n * CStore<S>::E, 0u, pitch, o, step);
}

// Inlet and outlet values on the compact state: as k_geo_boundary (a wave
// per direction and 64 listed nodes), from the node's new totals and record.
template <int I, typename S>
__device__ __forceinline__ void cio_link(const CGeoArgs<S> &ca, const Model<float> &mo, uint32_t n, uint32_t so_i) {
    using L = D3Q19;
    typedef float T;
    typedef typename PairOf<S>::type P2;
    constexpr uint32_t E = sizeof(P2);
    const FusedArgs<S> &a = ca.s.a;
    const uint32_t clk = a.links[n];
    if (!((clk >> I) & 1u)) return;
    Here h;
    const uint32_t t = n / uint32_t(a.nx);
    h.n = n;
    h.x = int(n - t * uint32_t(a.nx));
    h.z = int(t / uint32_t(a.ny));
    h.y = int(t - uint32_t(h.z) * uint32_t(a.ny));
    const uint32_t m = nbr(a.nx, a.ny, a.nz, h, -L::cx[I], -L::cy[I], -L::cz[I]);
    const uint8_t c = (clk & kLinkMixed) ? a.mask[m] : link_code(clk);
    if (is_wall(c)) return;
    const uint32_t pitch = uint32_t(a.pitch);
    const __amdgpu_buffer_rsrc_t rc = state_rsrc(ca.cout, c_bytes<S>() * pitch);
    const __amdgpu_buffer_rsrc_t rg = state_rsrc(a.out, uint32_t(L::Q) * pitch * E);
    const CRec own = c_record<S>(rc, n, pitch);
    Geo g{};
    g.inlets = a.inlets;
    g.outlets = a.outlets;
    OwnMom<T> om{};
    if (c >= kOutlet0) om = c_own_moments<S>(rc, n, pitch, own);
    const P2 ov = c_pair<S>(c_total<S>(rc, uint32_t(L::opp[I]) * pitch + n, L::opp[I]), L::opp[I], own);
    store_pair<P2>(rg, m * E, uint32_t(uniform(int(so_i))),
                   boundary_pair_v<L, S, T>(mo, I, c, io_vals<T>(g, c), ov, om));
}

template <typename S>
__global__ void __launch_bounds__(kIoBlock) k_cgeo_boundary(CGeoArgs<S> ca, Model<float> mo, uint32_t count) {
    constexpr uint32_t E = sizeof(typename PairOf<S>::type);
    const uint32_t b = blockIdx.x, chunk = b / 18u, dir = 1u + (b - chunk * 18u);
    const uint32_t so_i = dir * uint32_t(ca.s.a.pitch) * E;
    const uint32_t k = chunk * kIoBlock + threadIdx.x;
    if (k >= count) return;
    const uint32_t n = ca.s.blocks[k];
    switch (dir) {
        case 1: cio_link<1, S>(ca, mo, n, so_i); break;
        case 2: cio_link<2, S>(ca, mo, n, so_i); break;
        case 3: cio_link<3, S>(ca, mo, n, so_i); break;
        case 4: cio_link<4, S>(ca, mo, n, so_i); break;
        case 5: cio_link<5, S>(ca, mo, n, so_i); break;
        case 6: cio_link<6, S>(ca, mo, n, so_i); break;
        case 7: cio_link<7, S>(ca, mo, n, so_i); break;
        case 8: cio_link<8, S>(ca, mo, n, so_i); break;
        case 9: cio_link<9, S>(ca, mo, n, so_i); break;
        case 10: cio_link<10, S>(ca, mo, n, so_i); break;
        case 11: cio_link<11, S>(ca, mo, n, so_i); break;
        case 12: cio_link<12, S>(ca, mo, n, so_i); break;
        case 13: cio_link<13, S>(ca, mo, n, so_i); break;
        case 14: cio_link<14, S>(ca, mo, n, so_i); break;
        case 15: cio_link<15, S>(ca, mo, n, so_i); break;
        case 16: cio_link<16, S>(ca, mo, n, so_i); break;
        case 17: cio_link<17, S>(ca, mo, n, so_i); break;
        default: cio_link<18, S>(ca, mo, n, so_i); break;
    }
}

// The compact state of the fluid nodes as pairs, for reads of the state:
// each fluid node's 19 pairs in its own slots and, for links from walls, its
// bounce-back values in the wall nodes' slots; the inlet and outlet values
// are already in the pair buffer.
template <typename S>
__global__ void __launch_bounds__(kGeoBlock) k_cgeo_expand(CGeoArgs<S> ca) {
    using L = D3Q19;
    typedef typename PairOf<S>::type P2;
    constexpr uint32_t E = sizeof(P2);
    const FusedArgs<S> &a = ca.s.a;
    Here h;
    if (!here(a.nx, a.ny, a.nz, ca.s.blocks[blockIdx.x], h)) return;
    const uint32_t n = h.n;
    const uint32_t clk = a.links[n];
    if (!(clk & kLinkFluid)) return;
    const uint32_t pitch = uint32_t(a.pitch);
    const __amdgpu_buffer_rsrc_t rc = state_rsrc(ca.cin, c_bytes<S>() * pitch);
    const __amdgpu_buffer_rsrc_t rg = state_rsrc(a.out, uint32_t(L::Q) * pitch * E);
    const CRec own = c_record<S>(rc, n, pitch);
    P2 ov[L::Q];
#pragma unroll
    for (int j = 0; j < L::Q; ++j) {
        ov[j] = c_pair<S>(c_total<S>(rc, uint32_t(j) * pitch + n, j), j, own);
        store_pair<P2>(rg, n * E, uint32_t(uniform(int(uint32_t(j) * pitch * E))), ov[j]);
    }
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        if (!((clk >> i) & 1u)) continue;
        const uint32_t m = nbr(a.nx, a.ny, a.nz, h, -L::cx[i], -L::cy[i], -L::cz[i]);
        if (is_wall((clk & kLinkMixed) ? a.mask[m] : link_code(clk)))
            store_pair<P2>(rg, m * E, uint32_t(uniform(int(uint32_t(i) * pitch * E))), ov[L::opp[i]]);
    }
}

template <typename S>
hipError_t run_cgeo(const Geo &g, const ModelD &md, bool pair_in, const void *in, const void *gin, void *cout,
                    void *gout, void *psi, void *scratch, const SplitPlan &sp, const uint32_t *ctr_in,
                    uint32_t *ctr_out, hipStream_t s) {
    typedef typename PairOf<S>::type P2;
    if (md.bgk || !g.mask || !g.links || !psi || !scratch) return hipErrorInvalidValue;
    if (uint64_t(D3Q19::Q) * uint64_t(g.pitch) * sizeof(P2) >= (uint64_t(1) << 32)) return hipErrorInvalidValue;
    const int64_t nb = split_blocks(g.nx, g.ny, g.nz);
    if (nb <= 0 || nb > 0x7fffffff || sp.active > nb || sp.io > nb || sp.active < 0 || sp.io < 0 ||
        sp.ionodes < 0 || sp.ionodes > g.pitch || (sp.ionodes > 0) != (sp.io > 0))
        return hipErrorInvalidValue;
    const ScratchMap m = scratch_map(scratch, g.pitch, nb);
    CGeoArgs<S> ca;
    // the pair buffer read: the pair state on a first step (pulled as pairs)
    // or the inlet and outlet values; the pair buffer written: those values
    ca.s.a = fused_args<S>(g, pair_in ? in : gin, gout, ctr_in, ctr_out, FusedShape{8, 1});
    ca.s.psi = static_cast<float *>(psi);
    ca.s.mom = m.mom;
    ca.s.blocks = m.act;
    ca.cin = static_cast<const uint8_t *>(in);
    ca.cout = static_cast<uint8_t *>(cout);
    const Model<float> mo = to_model<float>(md);
    if (sp.active > 0) {
        if (pair_in)
            hipLaunchKernelGGL(k_geo_moments<S>, dim3(unsigned(sp.active)), dim3(kGeoBlock), 0, s, ca.s);
        else
            hipLaunchKernelGGL(k_cgeo_moments<S>, dim3(unsigned(sp.active)), dim3(kGeoBlock), 0, s, ca);
    }
    if (sp.active == 0) ca.s.blocks = nullptr;
    hipLaunchKernelGGL(k_cgeo_collide<S>, dim3(unsigned(sp.active > 0 ? sp.active : 1)), dim3(kGeoBlock), 0, s, ca,
                       mo);
    ca.s.blocks = m.ionodes;
    if (sp.ionodes > 0)
        hipLaunchKernelGGL(k_cgeo_boundary<S>, dim3(unsigned(18 * ((sp.ionodes + kIoBlock - 1) / kIoBlock))),
                           dim3(kIoBlock), 0, s, ca, mo, uint32_t(sp.ionodes));
    return hipGetLastError();
}

template <typename S>
hipError_t run_expand_cgeo(const Geo &g, const void *cin, void *pout, void *scratch, const SplitPlan &sp,
                           hipStream_t s) {
    if (!g.mask || !g.links || !scratch) return hipErrorInvalidValue;
    const int64_t nb = split_blocks(g.nx, g.ny, g.nz);
    if (nb <= 0 || nb > 0x7fffffff || sp.active > nb || sp.active < 0) return hipErrorInvalidValue;
    if (sp.active == 0) return hipSuccess;
    const ScratchMap m = scratch_map(scratch, g.pitch, nb);
    CGeoArgs<S> ca;
    ca.s.a = fused_args<S>(g, nullptr, pout, nullptr, nullptr, FusedShape{8, 1});
    ca.s.psi = nullptr;
    ca.s.mom = nullptr;
    ca.s.blocks = m.act;
    ca.cin = static_cast<const uint8_t *>(cin);
    ca.cout = nullptr;
    hipLaunchKernelGGL(k_cgeo_expand<S>, dim3(unsigned(sp.active)), dim3(kGeoBlock), 0, s, ca);
    return hipGetLastError();
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
    if (sp.ionodes < 0 || sp.ionodes > g.pitch || (sp.ionodes > 0) != (sp.io > 0)) return hipErrorInvalidValue;
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
    sa.blocks = m.ionodes;
    if (sp.ionodes > 0)
        hipLaunchKernelGGL(k_geo_boundary<S>, dim3(unsigned(18 * ((sp.ionodes + kIoBlock - 1) / kIoBlock))),
                           dim3(kIoBlock), 0, s, sa, mo, uint32_t(sp.ionodes));
    return hipGetLastError();
}

}  // namespace

int64_t split_blocks(int nx, int ny, int nz) {
    return int64_t((nx + kGX - 1) / kGX) * ((ny + kGY - 1) / kGY) * nz;
}

size_t split_scratch_bytes(int64_t pitch, int nx, int ny, int nz) {
    const int64_t nb = split_blocks(nx, ny, nz);
    return align256(sizeof(float) * kNM * size_t(pitch)) + align256(size_t(nb)) + align256(sizeof(uint16_t) * size_t(nb)) +
           3 * align256(sizeof(uint32_t) * size_t(nb)) + align256(sizeof(uint32_t) * size_t(pitch)) +
           align256(3 * sizeof(uint32_t));
}

hipError_t split_prepare(const Geo &g, void *scratch, SplitPlan &sp, hipStream_t s) {
    sp = SplitPlan{};
    if (!g.links || !scratch) return hipErrorInvalidValue;
    const int64_t nb = split_blocks(g.nx, g.ny, g.nz);
    if (nb <= 0 || nb > 0x7fffffff) return hipErrorInvalidValue;
    const ScratchMap m = scratch_map(scratch, g.pitch, nb);
    hipLaunchKernelGGL(k_geo_flags, dim3(unsigned(nb)), dim3(kGeoBlock), 0, s, g.links, g.nx, g.ny, g.nz, m.flags,
                       m.ioc);
    hipLaunchKernelGGL(k_geo_lists, dim3(1), dim3(kListThreads), 0, s, m.flags, m.ioc, uint32_t(nb), m.act, m.io,
                       m.ioofs, m.counts);
    hipError_t e = hipGetLastError();
    uint32_t c[3] = {0, 0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(c, m.counts, sizeof(c), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    if (int64_t(c[0]) > nb || int64_t(c[1]) > nb || int64_t(c[2]) > g.pitch || (c[1] > 0) != (c[2] > 0))
        return hipErrorUnknown;
    if (c[1] > 0) {
        hipLaunchKernelGGL(k_geo_ionodes, dim3(c[1]), dim3(kGeoBlock), 0, s, g.links, g.nx, g.ny, g.nz, m.io, m.ioofs,
                           m.ionodes);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
    }
    sp.active = c[0];
    sp.io = c[1];
    sp.ionodes = c[2];
    return hipSuccess;
}

hipError_t launch_step_cgeo(int prec, const Geo &g, const ModelD &md, bool pair_in, const void *in, const void *gin,
                            void *cout, void *gout, void *psi, void *scratch, const SplitPlan &sp,
                            const uint32_t *ctr_in, uint32_t *ctr_out, hipStream_t s) {
    if (prec == 1)
        return run_cgeo<float>(g, md, pair_in, in, gin, cout, gout, psi, scratch, sp, ctr_in, ctr_out, s);
    if (prec == 2)
        return run_cgeo<_Float16>(g, md, pair_in, in, gin, cout, gout, psi, scratch, sp, ctr_in, ctr_out, s);
    return hipErrorInvalidValue;
}

hipError_t launch_expand_cgeo(int prec, const Geo &g, const void *cin, void *pout, void *scratch, const SplitPlan &sp,
                              hipStream_t s) {
    if (prec == 1) return run_expand_cgeo<float>(g, cin, pout, scratch, sp, s);
    if (prec == 2) return run_expand_cgeo<_Float16>(g, cin, pout, scratch, sp, s);
    return hipErrorInvalidValue;
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
