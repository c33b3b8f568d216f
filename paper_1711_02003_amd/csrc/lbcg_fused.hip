// Fused single-pass D3Q19 RCG step (arXiv:1711.02003, Sec. II, Eqs. (1)-(11)).
//
// The colour gradient at x needs psi at the 18 neighbours at the same time
// level, and psi there needs the populations pulled from two hops away, so
// the step cannot be one independent pass per node.  Instead each block owns
// a column tile of 64 x R nodes (one wave per row) and sweeps a chunk of z
// planes.  For plane z+1 it pulls the 19 populations of its nodes (Eq. (1);
// each one a (total deviation, colour share) pair), keeps only the 12
// scalars the collision needs (drho, 36 rho^R, 36 rho^B, j, folded momentum
// flux G), and writes psi of the tile plus a one-node ring (the ring
// recomputes the neighbours' densities from cache) into a 5-slot LDS ring
// buffer.  After one barrier it collides plane z with the gradient taken from
// the LDS planes z-1, z, z+1 and stores the 19 new pairs coalesced, with
// non-temporal stores (the new state is not read again in this step).  The
// populations of plane z+2 (interior and ring) are loaded one iteration
// ahead, so their latency overlaps the barrier, the collision and the stores;
// the barrier orders only LDS traffic and leaves those loads in flight.
//
// Every stored population is read from HBM once and written once: the
// algorithmic traffic is 2 x 38 x sizeof(storage) bytes per node.
//
// With a geometry mask (compile-time switch) the pull applies the boundary
// rules of the generic path (walls, velocity inlets, pressure outlets), psi
// of an inlet node is the inlet's phase value, and a wall or outlet
// neighbour contributes the centre node's psi to the gradient.
//
// Block -> work mapping (single lattice): work items (tile, z chunk) are
// numbered tile-major and dealt to the 8 XCDs in contiguous bands matching the
// round-robin dispatch of blocks to XCDs, so each XCD sweeps a compact band
// of tiles and the ring re-reads mostly hit that XCD's L2.  The batched form
// steps many lattices in one launch from a block -> (lattice, item) table.
#include "lbcg_internal.h"

namespace lbcg {

constexpr int kTX = 64;
constexpr int kXCD = 8;
constexpr float kSentinel = 1e30f;  // LDS psi of a wall or outlet node

#ifndef LBCG_NT_STORE
#define LBCG_NT_STORE 1
#endif

template <typename V>
__device__ __forceinline__ void put(V *p, V v) {
#if LBCG_NT_STORE
    __builtin_nontemporal_store(v, p);
#else
    *p = v;
#endif
}

// Barrier that orders LDS accesses only; global loads stay in flight.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Pull the 19 population pairs of node (x, y, z) of a lattice without
// geometry.  Addresses are 32-bit byte offsets from the uniform state base
// (the host checks that a state buffer is below 4 GiB), which keeps one VGPR
// per load instead of two.
template <typename S, typename T>
__device__ __forceinline__ void pull_periodic(const FusedArgs<S> &a, int x, int y, int z, Pops<D3Q19, T> &p) {
    using L = D3Q19;
    typedef typename PairOf<S>::type P2;
    const int xm = x == 0 ? a.nx - 1 : x - 1, xp = x == a.nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? a.ny - 1 : y - 1, yp = y == a.ny - 1 ? 0 : y + 1;
    const int zm = z == 0 ? a.nz - 1 : z - 1, zp = z == a.nz - 1 ? 0 : z + 1;
    const char *base = reinterpret_cast<const char *>(a.in);
    const uint32_t cstride = uint32_t(a.pitch) * uint32_t(sizeof(P2));
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        // source = x - c_i
        const int xs = L::cx[i] > 0 ? xm : (L::cx[i] < 0 ? xp : x);
        const int ys = L::cy[i] > 0 ? ym : (L::cy[i] < 0 ? yp : y);
        const int zs = L::cz[i] > 0 ? zm : (L::cz[i] < 0 ? zp : z);
        const uint32_t nd = uint32_t(xs) + uint32_t(a.nx) * (uint32_t(ys) + uint32_t(a.ny) * uint32_t(zs));
        const uint32_t off = uint32_t(i) * cstride + nd * uint32_t(sizeof(P2));
        decode_pair<L, S, T>(*reinterpret_cast<const P2 *>(base + off), i, p);
    }
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
    return g;
}

// One work item: column tile `tile`, z chunk `chunk` of one lattice.
template <typename S, typename T, int R, bool MASKED>
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

    auto node = [&](int xx, int yy, int zz) {
        return int64_t(xx) + int64_t(a.nx) * (int64_t(yy) + int64_t(a.ny) * zz);
    };
    auto code = [&](int xx, int yy, int zz) -> uint8_t {
        if (!MASKED) return kFluid;
        return a.mask ? a.mask[node(xx, yy, zz)] : kFluid;
    };
    // LDS psi of a non-fluid node: the inlet's phase value, or the sentinel
    // that the gradient replaces by the centre node's own psi
    auto solid_psi = [&](uint8_t c) -> float {
        if (c >= kInlet0 && c < kOutlet0) {
            const DevInlet in = a.inlets[c - kInlet0];
            return float((in.rhoR - in.rhoB) / (in.rhoR + in.rhoB));
        }
        return kSentinel;
    };
    auto pull = [&](int xx, int yy, int zz, Pops<L, T> &p) {
        if (MASKED) {
            const Geo g = geo_of(a);
            pull_node<L, S, T>(g, mo, a.in, xx, yy, zz, node(xx, yy, zz), true, p);
        } else {
            pull_periodic<S, T>(a, xx, yy, zz, p);
        }
    };

    // psi planes live in a 5-slot LDS ring: iteration z writes the interior of
    // plane z+1 and the ring of plane z+2 while the collision reads planes
    // z-1..z+1, so a slot is rewritten only after every wave has passed the
    // barrier that follows its last read.
    auto slot_of = [&](int zp) { return lds + ((zp - z0 + 1) % 5) * PL; };

    // Ring nodes: psi of the one-node ring around the tile.  Their loads are
    // issued one plane ahead, together with the interior prefetch, so the
    // neighbour tiles' rows are requested while those tiles load them too,
    // and before the interior prefetch so that waiting for them (loads retire
    // in order) leaves the prefetch in flight.
    Pops<L, T> rp;
    rp.red = 0;
    uint8_t rcode = kFluid;
    auto ring_issue = [&](int zp) {
        if (has_ring) {
            const int zz = wrapz(zp, a.nz);
            rcode = code(gx, gy, zz);
            if (rcode == kFluid) pull(gx, gy, zz, rp);
        }
    };
    auto ring_finish = [&](int zp) {
        if (has_ring) {
            float v;
            if (rcode == kFluid) {
                T dr, rR, rB;
                densities<L, T>(rp, dr, rR, rB);
                v = float(psi_of<T>(dr, rR, rB));
            } else {
                v = solid_psi(rcode);
            }
            slot_of(zp)[(ry + 1) * W + rx + 1] = v;
        }
    };

    // Interior: moments of plane z are carried in registers, the populations
    // of plane z+1 are in flight.
    T cd = 0, cR = 0, cB = 0, cj[3] = {0, 0, 0}, cG[6] = {0, 0, 0, 0, 0, 0};
    bool cfl = false;
    Pops<L, T> pp;
    pp.red = 0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) pp.df[i] = pp.mm[i] = T(0);
    uint8_t pcode = kFluid;
    auto interior_issue = [&](int zp) {
        if (intile) {
            const int zz = wrapz(zp, a.nz);
            pcode = code(x, y, zz);
            if (pcode == kFluid) pull(x, y, zz, pp);
        }
    };
    // moments of the pulled interior plane into (d, r36R, r36B, j, G); returns psi
    auto interior_moments = [&](T &d, T &r36R, T &r36B, T j[3], T G[6], bool &fl) -> float {
        fl = pcode == kFluid;
        if (!fl) return solid_psi(pcode);
        Mom<T> m;
        moments<L, T>(pp, m);
        d = m.drho;
        r36R = m.r36R;
        r36B = m.r36B;
        j[0] = m.j[0];
        j[1] = m.j[1];
        j[2] = m.j[2];
        fold_flux<T>(mo, m, G);
        return float(psi_of<T>(m.drho, m.r36R, m.r36B));
    };

    // prologue: psi of planes z0-1 and z0, moments of z0, ring of z0+1 and
    // the interior loads of z0+1
    ring_issue(z0 - 1);
    interior_issue(z0 - 1);
    if (intile) {
        float v;
        if (pcode == kFluid) {
            T dr, rR, rB;
            densities<L, T>(pp, dr, rR, rB);
            v = float(psi_of<T>(dr, rR, rB));
        } else {
            v = solid_psi(pcode);
        }
        slot_of(z0 - 1)[(row + 1) * W + lane + 1] = v;
    }
    ring_finish(z0 - 1);
    ring_issue(z0);
    interior_issue(z0);
    if (intile) slot_of(z0)[(row + 1) * W + lane + 1] = interior_moments(cd, cR, cB, cj, cG, cfl);
    ring_finish(z0);
    ring_issue(z0 + 1);
    interior_issue(z0 + 1);
    ring_finish(z0 + 1);

    for (int z = z0; z < z1; ++z) {
        const bool more = z + 2 <= z1;  // uniform over the block
        T nd = 0, nR = 0, nB = 0, nj[3] = {0, 0, 0}, nG[6] = {0, 0, 0, 0, 0, 0};
        bool nfl = false;
        if (more) ring_issue(z + 2);
        if (intile) slot_of(z + 1)[(row + 1) * W + lane + 1] = interior_moments(nd, nR, nB, nj, nG, nfl);
        if (more) interior_issue(z + 2);
        if (more) ring_finish(z + 2);
        lds_barrier();
        if (intile && (!MASKED || cfl)) {
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
            collide<L, T>(mo, cd, cR, cB, cj, cG, F, nullptr, o);
            typedef typename PairOf<S>::type P2;
            const uint32_t n = uint32_t(x) + uint32_t(a.nx) * (uint32_t(y) + uint32_t(a.ny) * uint32_t(z));
            char *ob = reinterpret_cast<char *>(a.out);
            const uint32_t cstride = uint32_t(a.pitch) * uint32_t(sizeof(P2));
#pragma unroll
            for (int i = 0; i < L::Q; ++i) {
                const uint32_t off = uint32_t(i) * cstride + n * uint32_t(sizeof(P2));
                put(reinterpret_cast<P2 *>(ob + off), encode_pair<L, S, T>(o.df[i], o.mm[i], (o.red >> i) & 1u, i));
            }
        }
        cfl = nfl;
        cd = nd;
        cR = nR;
        cB = nB;
#pragma unroll
        for (int q = 0; q < 3; ++q) cj[q] = nj[q];
#pragma unroll
        for (int q = 0; q < 6; ++q) cG[q] = nG[q];
    }
}

// Single lattice, XCD-banded work mapping (see the file comment).
template <typename S, typename T, int R, bool MASKED>
__global__ void __launch_bounds__(kTX * R) k_step_fused(FusedArgs<S> a, Model<T> mo) {
    extern __shared__ float lds[];
    const int total = a.ntx * a.nty * a.zchunks;
    const int xcd = blockIdx.x % kXCD, l = blockIdx.x / kXCD;
    const int item = xcd * (total / kXCD) + min(xcd, total % kXCD) + l;
    sweep<S, T, R, MASKED>(a, mo, item / a.zchunks, item % a.zchunks, lds);
}

// Many lattices in one launch: the grid covers table entries [0, gridDim.x),
// dealt to the XCDs in contiguous bands as above; entry k is work item
// bitem[k] of lattice blat[k].
template <typename S, typename T, int R, bool MASKED>
__global__ void __launch_bounds__(kTX * R)
    k_step_fused_batch(const BatchDesc<S> *__restrict__ desc, const int *__restrict__ blat,
                       const int *__restrict__ bitem) {
    extern __shared__ float lds[];
    const int total = gridDim.x;
    const int xcd = blockIdx.x % kXCD, l = blockIdx.x / kXCD;
    const int k = xcd * (total / kXCD) + min(xcd, total % kXCD) + l;
    const int item = bitem[k];
    const BatchDesc<S> d = desc[blat[k]];
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
    return masked ? reinterpret_cast<const void *>(&k_step_fused<S, float, R, true>)
                  : reinterpret_cast<const void *>(&k_step_fused<S, float, R, false>);
}

int fused_resident_blocks(int prec, int rows, bool masked) {
    int per_cu = 0;
    const void *fn = prec == 2 ? (rows == 4 ? fused_fn<_Float16, 4>(masked) : fused_fn<_Float16, 8>(masked))
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
FusedArgs<S> fused_args(const Geo &g, const void *in, void *out, FusedShape sh) {
    FusedArgs<S> a;
    a.in = static_cast<const S *>(in);
    a.out = static_cast<S *>(out);
    a.nx = g.nx;
    a.ny = g.ny;
    a.nz = g.nz;
    a.pitch = g.pitch;
    a.mask = g.mask;
    a.inlets = g.inlets;
    a.outlets = g.outlets;
    a.ntx = (g.nx + kTX - 1) / kTX;
    a.nty = (g.ny + sh.rows - 1) / sh.rows;
    a.zchunks = sh.zchunks < 1 ? 1 : (sh.zchunks > g.nz ? g.nz : sh.zchunks);
    return a;
}
template FusedArgs<float> fused_args<float>(const Geo &, const void *, void *, FusedShape);
template FusedArgs<_Float16> fused_args<_Float16>(const Geo &, const void *, void *, FusedShape);

template <typename S, int R, bool MASKED>
static void launch_one(const FusedArgs<S> &a, const Model<float> &mo, unsigned nblocks, hipStream_t s) {
    hipLaunchKernelGGL((k_step_fused<S, float, R, MASKED>), dim3(nblocks), dim3(kTX * R), fused_lds(R), s, a, mo);
}

template <typename S>
static hipError_t run_fused(const Geo &g, const ModelD &md, const void *in, void *out, FusedShape sh,
                            hipStream_t s) {
    const int R = sh.rows;
    // Rows 4 and 8 only: a 1024-thread block (16 rows) caps the kernel at 128
    // VGPRs, where it spills.
    if (R != 4 && R != 8) return hipErrorInvalidValue;
    typedef typename PairOf<S>::type P2;
    // 32-bit byte offsets must cover a state buffer
    if (uint64_t(D3Q19::Q) * uint64_t(g.pitch) * sizeof(P2) >= (uint64_t(1) << 32)) return hipErrorInvalidValue;
    const FusedArgs<S> a = fused_args<S>(g, in, out, sh);
    const int64_t nblocks = int64_t(a.ntx) * a.nty * a.zchunks;
    if (nblocks > 0x7fffffff) return hipErrorInvalidValue;
    const Model<float> mo = to_model<float>(md);
    const bool masked = g.mask != nullptr;
    const unsigned nb = unsigned(nblocks);
    if (R == 4)
        masked ? launch_one<S, 4, true>(a, mo, nb, s) : launch_one<S, 4, false>(a, mo, nb, s);
    else
        masked ? launch_one<S, 8, true>(a, mo, nb, s) : launch_one<S, 8, false>(a, mo, nb, s);
    return hipGetLastError();
}

hipError_t launch_step_fused(int prec, const Geo &g, const ModelD &md, const void *in, void *out,
                             FusedShape shape, hipStream_t s) {
    if (prec == 1) return run_fused<float>(g, md, in, out, shape, s);
    if (prec == 2) return run_fused<_Float16>(g, md, in, out, shape, s);
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
