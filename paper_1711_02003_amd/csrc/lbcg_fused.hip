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
// ring recomputes the neighbours' densities from cache) into a 4-slot LDS
// ring buffer.  After one barrier it collides plane z with the gradient taken
// from the LDS planes z-1, z, z+1 and stores the 38 new values coalesced.
// Every stored population is read from HBM once and written once: the
// algorithmic traffic is 2 x 38 x sizeof(storage) bytes per node.
//
// Block -> tile mapping: block b takes z chunk b % zchunks and column tile
// b / zchunks, so with zchunks a multiple of 8 all tiles of one chunk land on
// the same XCD (blocks are dealt round-robin over the 8 XCDs) and the ring
// re-reads hit that XCD's L2.
#include "lbcg_internal.h"

namespace lbcg {

constexpr int kTX = 64;

template <typename S>
struct FusedArgs {
    const S *in;
    S *out;
    int nx, ny, nz;
    int64_t pitch;
    int ntx, nty, zchunks;
};

// Pull the 38 values of node (x, y, z) (periodic).  Addresses are 32-bit
// byte offsets from the uniform state base (the host checks that a state
// buffer is below 4 GiB), which keeps one VGPR per load instead of two.
template <typename S, typename T>
__device__ __forceinline__ void pull_periodic(const FusedArgs<S> &a, int x, int y, int z, T *df, T *chi) {
    using L = D3Q19;
    const int xm = x == 0 ? a.nx - 1 : x - 1, xp = x == a.nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? a.ny - 1 : y - 1, yp = y == a.ny - 1 ? 0 : y + 1;
    const int zm = z == 0 ? a.nz - 1 : z - 1, zp = z == a.nz - 1 ? 0 : z + 1;
    const char *base = reinterpret_cast<const char *>(a.in);
    const uint32_t cstride = uint32_t(a.pitch) * uint32_t(sizeof(S));
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        // source = x - c_i
        const int xs = L::cx[i] > 0 ? xm : (L::cx[i] < 0 ? xp : x);
        const int ys = L::cy[i] > 0 ? ym : (L::cy[i] < 0 ? yp : y);
        const int zs = L::cz[i] > 0 ? zm : (L::cz[i] < 0 ? zp : z);
        const uint32_t m = uint32_t(xs) + uint32_t(a.nx) * (uint32_t(ys) + uint32_t(a.ny) * uint32_t(zs));
        const uint32_t o1 = uint32_t(i) * cstride + m * uint32_t(sizeof(S));
        const uint32_t o2 = o1 + uint32_t(L::Q) * cstride;
        df[i] = Codec<S>::template df<L, T>(*reinterpret_cast<const S *>(base + o1), i);
        chi[i] = T(*reinterpret_cast<const S *>(base + o2));
    }
}

template <typename S, typename T, int R>
__global__ void __launch_bounds__(kTX * R) k_step_fused(FusedArgs<S> a, Model<T> mo) {
    using L = D3Q19;
    extern __shared__ float lds[];
    const int W = kTX + 2, H = R + 2;  // LDS plane: (R+2) x 66
    const int lane = threadIdx.x % kTX, row = threadIdx.x / kTX;

    const int b = blockIdx.x;
    const int chunk = b % a.zchunks;
    const int tile = b / a.zchunks;
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

    // psi of plane zp into LDS slot; interior nodes also return their moments
    auto plane = [&](int zp, bool carry, T &drho, T &rR, T *j, T *G) {
        const int zz = zp < 0 ? zp + a.nz : (zp >= a.nz ? zp - a.nz : zp);
        float *slot = lds + ((zp - z0 + 1) & 3) * (W * H);
        if (active) {
            T df[L::Q], chi[L::Q];
            pull_periodic<S, T>(a, x, y, zz, df, chi);
            T ps;
            if (carry) {
                Mom<T> m;
                moments<L, T>(df, chi, m);
                drho = m.drho;
                rR = m.rhoR;
                j[0] = m.j[0];
                j[1] = m.j[1];
                j[2] = m.j[2];
                fold_flux<T>(mo, m, G);
                ps = psi_of<T>(m.drho, m.rhoR);
            } else {
                T dr, rhoR;
                densities<L, T>(df, chi, dr, rhoR);
                ps = psi_of<T>(dr, rhoR);
            }
            slot[(row + 1) * W + lane + 1] = float(ps);
        }
        if (has_ring) {
            T df[L::Q], chi[L::Q];
            pull_periodic<S, T>(a, gx, gy, zz, df, chi);
            T dr, rhoR;
            densities<L, T>(df, chi, dr, rhoR);
            slot[(ry + 1) * W + rx + 1] = float(psi_of<T>(dr, rhoR));
        }
    };

    T cd = 0, cR = 0, cj[3] = {0, 0, 0}, cG[6] = {0, 0, 0, 0, 0, 0};
    T nd = 0, nR = 0, nj[3] = {0, 0, 0}, nG[6] = {0, 0, 0, 0, 0, 0};
    plane(z0 - 1, false, nd, nR, nj, nG);
    plane(z0, true, cd, cR, cj, cG);

    for (int z = z0; z < z1; ++z) {
        plane(z + 1, true, nd, nR, nj, nG);
        __syncthreads();
        if (active) {
            const float *sm = lds + ((z - 1 - z0 + 1) & 3) * (W * H);
            const float *s0 = lds + ((z - z0 + 1) & 3) * (W * H);
            const float *sp = lds + ((z + 1 - z0 + 1) & 3) * (W * H);
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
            collide<L, T>(mo, cd, cR, cj, cG, F, nullptr, nullptr, o);
            const uint32_t n = uint32_t(x) + uint32_t(a.nx) * (uint32_t(y) + uint32_t(a.ny) * uint32_t(z));
            char *ob = reinterpret_cast<char *>(a.out);
            const uint32_t cstride = uint32_t(a.pitch) * uint32_t(sizeof(S));
#pragma unroll
            for (int i = 0; i < L::Q; ++i) {
                const uint32_t o1 = uint32_t(i) * cstride + n * uint32_t(sizeof(S));
                *reinterpret_cast<S *>(ob + o1) = Codec<S>::template enc_df<L, T>(o.df[i], i);
                *reinterpret_cast<S *>(ob + o1 + uint32_t(L::Q) * cstride) = S(o.chi[i]);
            }
        }
        cd = nd;
        cR = nR;
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
    const size_t shmem = size_t(4) * (R + 2) * (kTX + 2) * sizeof(float);
    const Model<float> mo = to_model<float>(md);
    if (R == 4)
        hipLaunchKernelGGL((k_step_fused<S, float, 4>), dim3(unsigned(nblocks)), dim3(kTX * 4), shmem, s, a, mo);
    else
        hipLaunchKernelGGL((k_step_fused<S, float, 8>), dim3(unsigned(nblocks)), dim3(kTX * 8), shmem, s, a, mo);
    return hipGetLastError();
}

hipError_t launch_step_fused(int prec, const Geo &g, const ModelD &md, const void *in, void *out,
                             FusedShape shape, hipStream_t s) {
    if (prec == 1) return run_fused<float>(g, md, in, out, shape, s);
    if (prec == 2) return run_fused<_Float16>(g, md, in, out, shape, s);
    return hipErrorInvalidValue;
}

}  // namespace lbcg
