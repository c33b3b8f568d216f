// Fused single-pass D2Q9 step (arXiv:1711.02003, Sec. II, Eqs. (1)-(11)), FP32
// or FP16 storage, with or without geometry.
//
// The 2-D counterpart of the D3Q19 sweep: each wave owns a strip of 64
// columns and sweeps a chunk of rows.  For row y+1 it pulls the 9 population
// pairs of its nodes (Eq. (1)) and, on two lanes, of the two nodes left and
// right of the strip, and writes psi of the 66 nodes into a 3-row LDS ring of
// its own; it then collides row y with the gradient read from the LDS rows
// y-1, y, y+1 and stores the 9 new pairs coalesced and non-temporal.  The
// populations of a row are requested one row ahead of their use.  A wave's
// LDS rows are its own, so no barrier is needed: a wave's LDS accesses
// complete in program order.
//
// With geometry (compile-time switch) a node's link word tells whether it is
// fluid; non-fluid nodes pull nothing and put the inlet's phase value (or a
// sentinel that the gradient replaces by the centre node's psi) into the
// LDS ring; a fluid node with non-fluid links stores its boundary values in
// the upstream nodes' slots after its collision, as in the D3Q19 sweep.
//
// Every stored population is read from HBM once and written once: 2 x 18 x
// sizeof(storage) bytes per node (144 B FP32), against ~224 B for the
// two-pass step (psi pass plus step pass).
//
// POPS (plain BGK, Eq. (5), at the node's rate or per colour): every
// population relaxes from its own pulled value, so the sweep keeps the
// decoded populations of the row being collided beside its moments.
#include <type_traits>

#include "lbcg_buffer.h"
#include "lbcg_internal.h"

namespace lbcg {

constexpr int kStrip = 64;        // columns of a strip (one wave)
constexpr int kStripWaves = 4;    // strips (work items) per block
constexpr int kRing = kStrip + 2; // LDS row: the strip and one node each side

template <typename S>
struct Fused2dArgs {
    const S *in;
    S *out;
    int nx, ny;
    int64_t pitch;
    const uint8_t *mask;       // nullptr = every node fluid
    const DevInlet *inlets;
    const DevOutlet *outlets;
    const DevWall *walls;
    const uint32_t *links;     // link words (with a mask)
    const uint32_t *ctr_in;
    uint32_t *ctr_out;
    int nstrips, ychunks;
};

template <typename S>
struct Pending2d {
    typename PairOf<S>::type v[D2Q9::Q];
};

// Request the 9 pairs of the node whose source columns are t (entry 1 - c_x)
// at row y.
template <typename S>
__device__ __forceinline__ void pull_row(const Fused2dArgs<S> &a, __amdgpu_buffer_rsrc_t r, const uint32_t t[3],
                                         int y, Pending2d<S> &p) {
    using L = D2Q9;
    typedef typename PairOf<S>::type P2;
    constexpr uint32_t E = sizeof(P2);
    const uint32_t row = uniform(int(uint32_t(a.nx) * E));
    const uint32_t cstride = uniform(int(uint32_t(a.pitch) * E));
    const uint32_t yo[3] = {uint32_t(uniform(y == 0 ? a.ny - 1 : y - 1)) * row, uint32_t(uniform(y)) * row,
                            uint32_t(uniform(y == a.ny - 1 ? 0 : y + 1)) * row};
#pragma unroll
    for (int i = 0; i < L::Q; ++i) p.v[i] = load_pair<P2>(r, t[1 - L::cx[i]], uint32_t(i) * cstride + yo[1 - L::cy[i]]);
}

template <typename S>
__device__ __forceinline__ void take2d(const Pending2d<S> &p, Pops<D2Q9, float> &q) {
    q.red = 0;
#pragma unroll
    for (int i = 0; i < D2Q9::Q; ++i) decode_pair<D2Q9, S, float>(p.v[i], i, q);
}

constexpr float kSentinel2d = 1e30f;  // LDS psi of a wall or outlet node

struct NoPops2d {};

template <typename S, bool MASKED, bool POPS>
__device__ __forceinline__ void sweep2d(const Fused2dArgs<S> &a, const Model<float> &mo, int strip, int chunk,
                                        float *lds) {
    using L = D2Q9;
    using T = float;
    // the decoded populations of the row being collided (POPS) and of the
    // row after it
    typedef typename std::conditional<POPS, Pops<L, T>, NoPops2d>::type Kept;
    typedef typename PairOf<S>::type P2;
    constexpr uint32_t E = sizeof(P2);
    const int lane = threadIdx.x % kStrip;
    const int x0 = strip * kStrip, tw = min(kStrip, a.nx - x0);
    const int y0 = int((int64_t(chunk) * a.ny) / a.ychunks);
    const int y1 = int((int64_t(chunk + 1) * a.ny) / a.ychunks);
    if (y1 <= y0) return;  // uniform over the wave
    const bool intile = lane < tw;
    const int x = x0 + (intile ? lane : 0);
    const uint32_t step = *a.ctr_in;  // seeds the stochastic rounding of 16-bit shares

    // lanes 0 and 1 also pull the node left and right of the strip
    const bool has_ring = lane < 2;
    const int gx = lane == 0 ? wrap_m1(x0 - 1, a.nx) : wrap_m1(x0 + tw, a.nx);
    const int rslot = lane == 0 ? 0 : tw + 1;
    auto cols = [&](int xx, uint32_t t[3]) {
        t[0] = uint32_t(wrap_m1(xx - 1, a.nx)) * E;
        t[1] = uint32_t(xx) * E;
        t[2] = uint32_t(wrap_m1(xx + 1, a.nx)) * E;
    };
    uint32_t it[3], rt[3];
    cols(x, it);
    cols(gx, rt);
    const uint32_t cstride = uniform(int(uint32_t(a.pitch) * E));
    const uint32_t row = uniform(int(uint32_t(a.nx) * E));
    const __amdgpu_buffer_rsrc_t rin = state_rsrc(a.in, uint32_t(L::Q) * cstride);
    const __amdgpu_buffer_rsrc_t rout = state_rsrc(a.out, uint32_t(L::Q) * cstride);
    // the 3-row psi ring of this wave: row yy lives in slot (yy - y0 + 1) % 3
    auto slot = [&](int yy) { return lds + ((yy - y0 + 1) % 3) * kRing; };
    auto wrapy = [&](int yy) { return yy < 0 ? yy + a.ny : (yy >= a.ny ? yy - a.ny : yy); };
    auto link = [&](int xx, int yy) { return MASKED ? a.links[int64_t(xx) + int64_t(a.nx) * wrapy(yy)] : kLinkFluid; };
    auto fluid = [&](uint32_t lk) { return !MASKED || (lk & kLinkFluid) != 0u; };
    // LDS psi of a non-fluid node: the inlet's or the wetting wall's phase
    // value, or the sentinel that the gradient replaces by the centre node's
    // own psi
    auto solid_psi = [&](uint8_t c) -> float {
        if (is_inlet(c)) {
            const DevInlet in = a.inlets[c - kInlet0];
            return float((in.rhoR - in.rhoB) / (in.rhoR + in.rhoB));
        }
        if (c >= kWall0 && c < kOutlet0) return float(a.walls[c - kWall0].psi);
        return kSentinel2d;
    };

    Pending2d<S> pp, rp;
    // link words of the pending rows, and of the next request (read one
    // request ahead, so that a pull never waits for its own link word)
    uint32_t plk = kLinkFluid, rlk = kLinkFluid, ilk = kLinkFluid, glk = kLinkFluid;
    if (MASKED && intile) ilk = link(x, y0 - 1);
    if (MASKED && has_ring) glk = link(gx, y0 - 1);
    auto issue = [&](int yy) {
        const int yw = wrapy(yy);
        if (has_ring) {
            rlk = glk;
            if (fluid(rlk)) pull_row<S>(a, rin, rt, yw, rp);
            if (MASKED) glk = link(gx, yy + 1);
        }
        if (intile) {
            plk = ilk;
            if (fluid(plk)) pull_row<S>(a, rin, it, yw, pp);
            if (MASKED) ilk = link(x, yy + 1);
        }
    };
    auto ring_psi = [&](int yy) {
        if (has_ring) {
            float v;
            if (fluid(rlk)) {
                Pops<L, T> q;
                take2d<S>(rp, q);
                T dr, rR, rB;
                densities<L, T>(q, dr, rR, rB);
                v = float(psi_of<T>(dr, rR, rB));
            } else {
                v = solid_psi(link_code(rlk));
            }
            slot(yy)[rslot] = v;
        }
    };
    T cd = 0, cR = 0, cB = 0, cj[3] = {0, 0, 0}, cS[6] = {0, 0, 0, 0, 0, 0};
    Kept cq{}, nq{};
    auto interior = [&](int yy, T &d, T &r36R, T &r36B, T j[3], T flux[6]) {
        if (intile && !fluid(plk)) slot(yy)[lane + 1] = solid_psi(link_code(plk));
        if (intile && fluid(plk)) {
            Pops<L, T> q;
            take2d<S>(pp, q);
            if constexpr (POPS) nq = q;
            Mom<T> m;
            moments<L, T>(q, m);
            d = m.drho;
            r36R = m.r36R;
            r36B = m.r36B;
#pragma unroll
            for (int k = 0; k < 3; ++k) j[k] = m.j[k];
#pragma unroll
            for (int k = 0; k < 6; ++k) flux[k] = m.S[k];
            slot(yy)[lane + 1] = float(psi_of<T>(m.drho, m.r36R, m.r36B));
        }
    };

    // With geometry, a chunk with no fluid node of its own has nothing to do
    // (a non-fluid node's slots hold only what its fluid neighbours store).
    // The link words are read 8 at a time, so that the loads of a batch are in
    // flight together (a chunk of non-fluid nodes is then dismissed in a few
    // load latencies, not one per row).
    if (MASKED) {
        bool any = false;
        if (intile)
            for (int yb = y0; yb < y1 && !any; yb += 8) {
                uint32_t w[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) w[k] = link(x, min(yb + k, y1 - 1));
                uint32_t acc = 0;
#pragma unroll
                for (int k = 0; k < 8; ++k) acc |= w[k];
                any = (acc & kLinkFluid) != 0u;
            }
        if (!__builtin_amdgcn_ballot_w64(any)) return;  // uniform over the wave
    }

    // prologue: psi of rows y0-1 and y0, moments of y0, requests of y0+1
    {
        T d, r, b, j[3], f[6];
        issue(y0 - 1);
        wait_memory();
        ring_psi(y0 - 1);
        interior(y0 - 1, d, r, b, j, f);
    }
    issue(y0);
    wait_memory();
    ring_psi(y0);
    interior(y0, cd, cR, cB, cj, cS);
    cq = nq;
    uint32_t clk = plk;  // link word of the row being collided
    issue(y0 + 1);

    for (int y = y0; y < y1; ++y) {
        T nd = 0, nR = 0, nB = 0, nj[3] = {0, 0, 0}, nS[6] = {0, 0, 0, 0, 0, 0};
        // row y+1 was requested one iteration ago; the compiler waits for
        // each loaded register before its use, which does not wait for the
        // stores of the row before (a wait for everything outstanding here
        // made the junction sweep 1 % slower)
        ring_psi(y + 1);
        interior(y + 1, nd, nR, nB, nj, nS);
        const uint32_t nlk = plk;
        if (y + 2 <= y1) issue(y + 2);
        __builtin_amdgcn_wave_barrier();
        if (intile && fluid(clk)) {
            const float *sm = slot(y - 1), *s0 = slot(y), *sp = slot(y + 1);
            const int c = lane + 1;
            const float pc = s0[c];
            T fx = 0, fy = 0;
#pragma unroll
            for (int i = 1; i < L::Q; ++i) {
                const float *sl = L::cy[i] > 0 ? sp : (L::cy[i] < 0 ? sm : s0);
                float pv = sl[c + L::cx[i]];
                if (MASKED) pv = pv == kSentinel2d ? pc : pv;
                const T wp = T(3.0 * wgt<L>(i)) * T(pv);
                if (L::cx[i]) fx += L::cx[i] > 0 ? wp : -wp;
                if (L::cy[i]) fy += L::cy[i] > 0 ? wp : -wp;
            }
            const T F[3] = {fx, fy, T(0)};
            PostOut<L, T> o;
            const Pops<L, T> *pin = nullptr;
            if constexpr (POPS) pin = &cq;
            collide<L, T>(mo, cd, cR, cB, cj, cS, F, pin, o);
            P2 enc[L::Q];
            encode_out<L, S, T>(o, step, uint32_t(x) + uint32_t(a.nx) * uint32_t(y), enc);
            const uint32_t yo = uint32_t(uniform(y)) * row;
#pragma unroll
            for (int i = 0; i < L::Q; ++i) store_pair<P2>(rout, it[1], uint32_t(i) * cstride + yo, enc[i]);
            // boundary values of the node's non-fluid links, stored in the
            // upstream nodes' slots (the addresses it pulls them from)
            if (MASKED && (clk & kLinkBits)) {
                Geo g;
                g.nx = a.nx;
                g.ny = a.ny;
                g.nz = 1;
                g.N = int64_t(a.nx) * a.ny;
                g.pitch = a.pitch;
                g.mask = a.mask;
                g.inlets = a.inlets;
                g.outlets = a.outlets;
                g.walls = a.walls;
                g.links = a.links;
                const uint32_t yg[3] = {uint32_t(uniform(y == 0 ? a.ny - 1 : y - 1)) * row, yo,
                                        uint32_t(uniform(y == a.ny - 1 ? 0 : y + 1)) * row};
                OwnMom<T> om{};
                if (clk & kLinkOutlet) om = own_moments<L, S, T>(enc);
#pragma unroll
                for (int i = 1; i < L::Q; ++i) {
                    if (!((clk >> i) & 1u)) continue;
                    uint8_t cd8 = link_code(clk);
                    if (clk & kLinkMixed)
                        cd8 = a.mask[int64_t(wrap_m1(x - L::cx[i], a.nx)) +
                                     int64_t(a.nx) * wrap_m1(y - L::cy[i], a.ny)];
                    store_pair<P2>(rout, it[1 - L::cx[i]], uint32_t(i) * cstride + yg[1 - L::cy[i]],
                                   boundary_pair<L, S, T>(g, mo, i, cd8, enc[L::opp[i]], om));
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        clk = nlk;
        cq = nq;
        cd = nd;
        cR = nR;
        cB = nB;
#pragma unroll
        for (int k = 0; k < 3; ++k) cj[k] = nj[k];
#pragma unroll
        for (int k = 0; k < 6; ++k) cS[k] = nS[k];
    }
}

// kStripWaves work items per block.  Periodic lattices number the items
// chunk-major (neighbouring strips of one chunk share a block and an L2).
// With geometry they are numbered strip-major, so that the busy items of a
// channel form runs of consecutive blocks (busy blocks interleaved with
// blocks that return at once were measured to crowd onto fewer CUs), and the
// tuner picks short chunks that spread a channel over the device.
template <typename S, bool MASKED, bool POPS>
__global__ void __launch_bounds__(kStrip * kStripWaves) k_step_fused2d(Fused2dArgs<S> a, Model<float> mo) {
    __shared__ float lds[kStripWaves * 3 * kRing];
    const int wave = threadIdx.x / kStrip;
    const int item = blockIdx.x * kStripWaves + wave;
    if (item == 0 && threadIdx.x == 0) *a.ctr_out = *a.ctr_in + 1u;
    if (item >= a.nstrips * a.ychunks) return;  // uniform over the wave
    const int strip = MASKED ? item / a.ychunks : item % a.nstrips;
    const int chunk = MASKED ? item % a.ychunks : item / a.nstrips;
    sweep2d<S, MASKED, POPS>(a, mo, strip, chunk, lds + wave * 3 * kRing);
}

bool fused2d_supported(int prec, const Geo &g) {
    const uint64_t elem = prec == 1 ? 4 : 2;
    return (prec == 1 || prec == 2) && g.nz == 1 && (g.mask == nullptr || g.links != nullptr) &&
           uint64_t(2 * D2Q9::Q) * uint64_t(g.pitch) * elem < (uint64_t(1) << 32);
}

template <typename S>
static hipError_t launch2d(const Geo &g, const ModelD &md, const void *in, void *out, const uint32_t *ctr_in,
                           uint32_t *ctr_out, int ychunks, hipStream_t s) {
    Fused2dArgs<S> a;
    a.in = static_cast<const S *>(in);
    a.out = static_cast<S *>(out);
    a.nx = g.nx;
    a.ny = g.ny;
    a.pitch = g.pitch;
    a.mask = g.mask;
    a.inlets = g.inlets;
    a.outlets = g.outlets;
    a.walls = g.walls;
    a.links = g.links;
    a.ctr_in = ctr_in;
    a.ctr_out = ctr_out;
    a.nstrips = (g.nx + kStrip - 1) / kStrip;
    a.ychunks = ychunks < 1 ? 1 : (ychunks > g.ny ? g.ny : ychunks);
    const int items = a.nstrips * a.ychunks;
    const dim3 grid{unsigned((items + kStripWaves - 1) / kStripWaves)}, block{unsigned(kStrip * kStripWaves)};
    const Model<float> mo = to_model<float>(md);
    if (md.bgk) {
        if (g.mask)
            hipLaunchKernelGGL((k_step_fused2d<S, true, true>), grid, block, 0, s, a, mo);
        else
            hipLaunchKernelGGL((k_step_fused2d<S, false, true>), grid, block, 0, s, a, mo);
    } else {
        if (g.mask)
            hipLaunchKernelGGL((k_step_fused2d<S, true, false>), grid, block, 0, s, a, mo);
        else
            hipLaunchKernelGGL((k_step_fused2d<S, false, false>), grid, block, 0, s, a, mo);
    }
    return hipGetLastError();
}

hipError_t launch_step_fused2d(int prec, const Geo &g, const ModelD &md, const void *in, void *out,
                               const uint32_t *ctr_in, uint32_t *ctr_out, int ychunks, hipStream_t s) {
    if (!fused2d_supported(prec, g)) return hipErrorInvalidValue;
    return prec == 1 ? launch2d<float>(g, md, in, out, ctr_in, ctr_out, ychunks, s)
                     : launch2d<_Float16>(g, md, in, out, ctr_in, ctr_out, ychunks, s);
}

}  // namespace lbcg
