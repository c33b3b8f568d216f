// Fused single-pass D3Q19 RCG step (arXiv:1711.02003, Sec. II, Eqs. (1)-(11))
// for periodic lattices without geometry.
//
// The colour gradient at x needs psi at the 18 neighbours at the same time
// level, and psi there needs the populations pulled from two hops away, so
// the step cannot be one independent pass per node.  Instead each block owns
// a column tile of 64 x R nodes (one wave per row) and sweeps a chunk of z
// planes.  For plane z+1 it pulls the 38 populations of its nodes (Eq. (1)),
// keeps only the 11 scalars the collision needs (drho, rho^R, j, folded
// momentum flux G), and writes psi of the tile plus a one-node ring (the
// ring recomputes the neighbours' densities from cache) into a 5-slot LDS
// ring buffer.  After one barrier it collides plane z with the gradient taken
// from the LDS planes z-1, z, z+1 and stores the 38 new values coalesced,
// with non-temporal stores (the new state is not read again in this step).
// The populations of plane z+2 are loaded one iteration ahead, so their HBM
// latency overlaps the barrier, the collision and the stores; the barrier
// orders only LDS traffic and leaves those loads in flight.
//
// Every stored population is read from HBM once and written once: the
// algorithmic traffic is 2 x 38 x sizeof(storage) bytes per node.
//
// Block -> work mapping: work items (tile, z chunk) are numbered tile-major
// and dealt to the 8 XCDs in contiguous bands matching the round-robin
// dispatch of blocks to XCDs, so each XCD sweeps a compact band of tiles and
// the ring re-reads mostly hit that XCD's L2.
#include "lbcg_internal.h"

namespace lbcg {

constexpr int kTX = 64;
constexpr int kXCD = 8;

#ifndef LBCG_NT_STORE
#define LBCG_NT_STORE 1
#endif

template <typename S>
struct FusedArgs {
    const S *in;
    S *out;
    int nx, ny, nz;
    int64_t pitch;
    int ntx, nty, zchunks;
};

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

// Pull the 38 values of node (x, y, z) (periodic).  Addresses are 32-bit
// byte offsets from the uniform state base (the host checks that a state
// buffer is below 4 GiB), which keeps one VGPR per load instead of two.
template <typename S, typename T>
__device__ __forceinline__ void pull_periodic(const FusedArgs<S> &a, int x, int y, int z, Pops<D3Q19, T> &p) {
    using L = D3Q19;
    const int xm = x == 0 ? a.nx - 1 : x - 1, xp = x == a.nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? a.ny - 1 : y - 1, yp = y == a.ny - 1 ? 0 : y + 1;
    const int zm = z == 0 ? a.nz - 1 : z - 1, zp = z == a.nz - 1 ? 0 : z + 1;
    typedef typename PairOf<S>::type P2;
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

template <typename S, typename T, int R>
__global__ void __launch_bounds__(kTX * R) k_step_fused(FusedArgs<S> a, Model<T> mo) {
    using L = D3Q19;
    extern __shared__ float lds[];
    constexpr int W = kTX + 2, H = R + 2, PL = W * H;  // LDS plane: (R+2) x 66
    const int lane = threadIdx.x % kTX, row = threadIdx.x / kTX;

    // work item of this block (see the file comment)
    const int total = a.ntx * a.nty * a.zchunks;
    const int xcd = blockIdx.x % kXCD, l = blockIdx.x / kXCD;
    const int item = xcd * (total / kXCD) + min(xcd, total % kXCD) + l;
    const int chunk = item % a.zchunks;
    const int tile = item / a.zchunks;
    const int tx = tile % a.ntx, ty = tile / a.ntx;
    const int x0 = tx * kTX, y0 = ty * R;
    const int tw = min(kTX, a.nx - x0), th = min(R, a.ny - y0);
    const int z0 = int((int64_t(chunk) * a.nz) / a.zchunks);
    const int z1 = int((int64_t(chunk + 1) * a.nz) / a.zchunks);
    if (z1 <= z0) return;  // uniform over the block

    const bool active = lane < tw && row < th;
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
    // psi planes live in a 5-slot LDS ring: iteration z writes the interior of
    // plane z+1 and the ring of plane z+2 while the collision reads planes
    // z-1..z+1, so a slot is rewritten only after every wave has passed the
    // barrier that follows its last read.
    auto slot_of = [&](int zp) { return lds + ((zp - z0 + 1) % 5) * PL; };

    // Ring nodes: psi of the one-node ring around the tile.  Their loads are
    // issued one plane ahead, together with the interior prefetch, so the
    // neighbour tiles' rows are requested while those tiles load them too
    // (L2 hits), and before the interior prefetch so that waiting for them
    // (loads retire in order) leaves the prefetch in flight.
    Pops<L, T> rp;
    rp.red = 0;
    auto ring_issue = [&](int zp) {
        if (has_ring) pull_periodic<S, T>(a, gx, gy, wrapz(zp, a.nz), rp);
    };
    auto ring_finish = [&](int zp) {
        if (has_ring) {
            T dr, rR, rB;
            densities<L, T>(rp, dr, rR, rB);
            slot_of(zp)[(ry + 1) * W + rx + 1] = float(psi_of<T>(dr, rR, rB));
        }
    };

    T cd = 0, cR = 0, cB = 0, cj[3] = {0, 0, 0}, cG[6] = {0, 0, 0, 0, 0, 0};
    Pops<L, T> pp;  // populations of the next interior plane
    pp.red = 0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) pp.df[i] = pp.mm[i] = T(0);

    // prologue: psi of planes z0-1 and z0, moments of z0, ring of z0+1 and
    // the interior loads of z0+1
    ring_issue(z0 - 1);
    if (active) {
        pull_periodic<S, T>(a, x, y, wrapz(z0 - 1, a.nz), pp);
        T dr, rR, rB;
        densities<L, T>(pp, dr, rR, rB);
        slot_of(z0 - 1)[(row + 1) * W + lane + 1] = float(psi_of<T>(dr, rR, rB));
    }
    ring_finish(z0 - 1);
    ring_issue(z0);
    if (active) {
        pull_periodic<S, T>(a, x, y, z0, pp);
        Mom<T> m;
        moments<L, T>(pp, m);
        cd = m.drho;
        cR = m.r36R;
        cB = m.r36B;
        cj[0] = m.j[0];
        cj[1] = m.j[1];
        cj[2] = m.j[2];
        fold_flux<T>(mo, m, cG);
        slot_of(z0)[(row + 1) * W + lane + 1] = float(psi_of<T>(m.drho, m.r36R, m.r36B));
    }
    ring_finish(z0);
    ring_issue(z0 + 1);
    if (active) pull_periodic<S, T>(a, x, y, wrapz(z0 + 1, a.nz), pp);
    ring_finish(z0 + 1);

    for (int z = z0; z < z1; ++z) {
        const bool more = z + 2 <= z1;  // uniform over the block
        T nd = 0, nR = 0, nB = 0, nj[3] = {0, 0, 0}, nG[6] = {0, 0, 0, 0, 0, 0};
        if (more) ring_issue(z + 2);
        if (active) {
            Mom<T> m;
            moments<L, T>(pp, m);
            nd = m.drho;
            nR = m.r36R;
            nB = m.r36B;
            nj[0] = m.j[0];
            nj[1] = m.j[1];
            nj[2] = m.j[2];
            fold_flux<T>(mo, m, nG);
            slot_of(z + 1)[(row + 1) * W + lane + 1] = float(psi_of<T>(m.drho, m.r36R, m.r36B));
        }
        if (more && active) pull_periodic<S, T>(a, x, y, wrapz(z + 2, a.nz), pp);
        if (more) ring_finish(z + 2);
        lds_barrier();
        if (active) {
            const float *sm = slot_of(z - 1), *s0 = slot_of(z), *sp = slot_of(z + 1);
            const int c = (row + 1) * W + lane + 1;
            T fx = 0, fy = 0, fz = 0;
#pragma unroll
            for (int i = 1; i < L::Q; ++i) {
                const float *sl = L::cz[i] > 0 ? sp : (L::cz[i] < 0 ? sm : s0);
                const T p = T(sl[c + L::cy[i] * W + L::cx[i]]);
                const T wp = T(3.0 * wgt<L>(i)) * p;
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
        cd = nd;
        cR = nR;
        cB = nB;
#pragma unroll
        for (int q = 0; q < 3; ++q) cj[q] = nj[q];
#pragma unroll
        for (int q = 0; q < 6; ++q) cG[q] = nG[q];
    }
}

bool fused_supported(int lattice, int prec, const Geo &g) {
    const uint64_t elem = prec == 1 ? 4 : 2;
    return lattice == 1 && (prec == 1 || prec == 2) && g.mask == nullptr &&
           uint64_t(2 * D3Q19::Q) * uint64_t(g.pitch) * elem < (uint64_t(1) << 32);
}

template <typename S>
static const void *fused_fn(int R) {
    return R == 4 ? reinterpret_cast<const void *>(&k_step_fused<S, float, 4>)
                  : reinterpret_cast<const void *>(&k_step_fused<S, float, 8>);
}

static size_t fused_lds(int R) { return size_t(5) * (R + 2) * (kTX + 2) * sizeof(float); }

int fused_resident_blocks(int prec, int rows) {
    int per_cu = 0;
    const void *fn = prec == 2 ? fused_fn<_Float16>(rows) : fused_fn<float>(rows);
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
static hipError_t run_fused(const Geo &g, const ModelD &md, const void *in, void *out, FusedShape sh,
                            hipStream_t s) {
    FusedArgs<S> a;
    a.in = static_cast<const S *>(in);
    a.out = static_cast<S *>(out);
    a.nx = g.nx;
    a.ny = g.ny;
    a.nz = g.nz;
    a.pitch = g.pitch;
    const int R = sh.rows;
    // Rows 4 and 8 only: a 1024-thread block (16 rows) caps the kernel at 128
    // VGPRs, where it spills and the compiler fuses multiplies differently,
    // which breaks bitwise agreement between tile shapes.
    if (R != 4 && R != 8) return hipErrorInvalidValue;
    // 32-bit byte offsets must cover both component halves of a state buffer
    if (uint64_t(2 * D3Q19::Q) * uint64_t(g.pitch) * sizeof(S) >= (uint64_t(1) << 32)) return hipErrorInvalidValue;
    a.ntx = (g.nx + kTX - 1) / kTX;
    a.nty = (g.ny + R - 1) / R;
    a.zchunks = sh.zchunks < 1 ? 1 : (sh.zchunks > g.nz ? g.nz : sh.zchunks);
    const int64_t nblocks = int64_t(a.ntx) * a.nty * a.zchunks;
    if (nblocks > 0x7fffffff) return hipErrorInvalidValue;
    const Model<float> mo = to_model<float>(md);
    if (R == 4)
        hipLaunchKernelGGL((k_step_fused<S, float, 4>), dim3(unsigned(nblocks)), dim3(kTX * 4), fused_lds(4), s,
                           a, mo);
    else
        hipLaunchKernelGGL((k_step_fused<S, float, 8>), dim3(unsigned(nblocks)), dim3(kTX * 8), fused_lds(8), s,
                           a, mo);
    return hipGetLastError();
}

hipError_t launch_step_fused(int prec, const Geo &g, const ModelD &md, const void *in, void *out,
                             FusedShape shape, hipStream_t s) {
    if (prec == 1) return run_fused<float>(g, md, in, out, shape, s);
    if (prec == 2) return run_fused<_Float16>(g, md, in, out, shape, s);
    return hipErrorInvalidValue;
}

}  // namespace lbcg
