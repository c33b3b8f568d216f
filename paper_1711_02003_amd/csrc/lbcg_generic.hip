// Generic kernels of the RCG step: every lattice, storage precision,
// collision form and boundary rule.  The step is two passes: the phase field
// psi of the pulled state (Eq. (2)), then pull + moments + colour gradient +
// collide/perturb/recolour + store (Eqs. (3)-(11), (1)).  Also: the
// equilibrium initialisation (Eq. (6)), field and population export and the
// FP64 diagnostics.
#include "lbcg_internal.h"

namespace lbcg {

constexpr int kBlock = 256;

__device__ __forceinline__ void node_xyz(const Geo &g, int64_t n, int &x, int &y, int &z) {
    x = int(n % g.nx);
    const int64_t r = n / g.nx;
    y = int(r % g.ny);
    z = int(r / g.ny);
}

__device__ __forceinline__ uint8_t code_at(const Geo &g, int64_t n) {
    return g.mask ? g.mask[n] : kFluid;
}

template <class L, typename S, typename T>
__global__ void __launch_bounds__(kBlock) k_init(Geo g, Model<T> mo, int64_t n0, int64_t cnt,
                                                 const double *__restrict__ rR,
                                                 const double *__restrict__ rB,
                                                 const double *__restrict__ u, S *__restrict__ st) {
    const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (k >= cnt) return;
    const int64_t n = n0 + k;
    const double r0 = rR[k], r1 = rB[k];
    double ux = 0, uy = 0, uz = 0;
    if (u) {
        ux = u[k];
        uy = u[cnt + k];
        uz = u[2 * cnt + k];
    }
    const double usq = ux * ux + uy * uy + uz * uz;
    const double aR = double(mo.aR), aB = double(mo.aB);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const double w = wgt<L>(i);
        const double cu = L::cx[i] * ux + L::cy[i] * uy + L::cz[i] * uz;
        const double U = w * (3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
        const double phR = i == 0 ? aR : (1.0 - aR) * w / (1.0 - wgt<L>(0));
        const double phB = i == 0 ? aB : (1.0 - aB) * w / (1.0 - wgt<L>(0));
        const double fR = r0 * (phR + U), fB = r1 * (phB + U);  // Eq. (6)
        const double f = fR + fB;
        double m;
        bool redmaj;
        split_shares<double>(f != 0.0 ? fR / f : 0.0, f != 0.0 ? fB / f : 0.0, m, redmaj);
        put_pair(reinterpret_cast<typename PairOf<S>::type *>(st) + int64_t(i) * g.pitch + n,
                 encode_pair<L, S, double>(f - w, m, redmaj, i));
    }
}

template <class L, typename S, typename T>
__global__ void __launch_bounds__(kBlock) k_psi(Geo g, Model<T> mo, const S *__restrict__ st, bool pulled,
                                                T *__restrict__ psi) {
    const int64_t n = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (n >= g.N) return;
    if (code_at(g, n) != kFluid) {
        psi[n] = T(0);
        return;
    }
    int x, y, z;
    node_xyz(g, n, x, y, z);
    Pops<L, T> p;
    pull_node<L, S, T>(g, mo, st, x, y, z, n, pulled, p);
    T drho, rR, rB;
    densities<L, T>(p, drho, rR, rB);
    psi[n] = psi_of<T>(drho, rR, rB);
}

// Colour gradient F = (1/c_s^2) sum_i w_i c_i psi~(x + c_i), psi~ = psi at fluid
// neighbours, the inlet's phase value at inlets, the wall's phase value at
// wetting walls, psi(x) at neutral walls and outlets.
template <class L, typename T>
__device__ __forceinline__ void gradient(const Geo &g, const T *__restrict__ psi, int x, int y, int z,
                                         int64_t n, T F[3]) {
    const T pc = psi[n];
    T fx = 0, fy = 0, fz = 0;
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        const int xs = wrap_m1(x + L::cx[i], g.nx);
        const int ys = wrap_m1(y + L::cy[i], g.ny);
        const int zs = wrap_m1(z + L::cz[i], g.nz);
        const int64_t m = xs + int64_t(g.nx) * (ys + int64_t(g.ny) * zs);
        const uint8_t code = code_at(g, m);
        T p;
        if (code == kFluid)
            p = psi[m];
        else if (is_inlet(code)) {
            const DevInlet in = g.inlets[code - kInlet0];
            p = T((in.rhoR - in.rhoB) / (in.rhoR + in.rhoB));
        } else if (code >= kWall0 && code < kOutlet0)
            p = T(g.walls[code - kWall0].psi);
        else
            p = pc;
        const T wp = T(3.0 * wgt<L>(i)) * p;
        if (L::cx[i]) fx += L::cx[i] > 0 ? wp : -wp;
        if (L::cy[i]) fy += L::cy[i] > 0 ? wp : -wp;
        if (L::cz[i]) fz += L::cz[i] > 0 ? wp : -wp;
    }
    F[0] = fx;
    F[1] = fy;
    F[2] = fz;
}

template <class L, typename S, typename T>
__global__ void __launch_bounds__(kBlock) k_step_generic(Geo g, Model<T> mo, const S *__restrict__ in,
                                                         bool pulled, const T *__restrict__ psi,
                                                         S *__restrict__ out, const uint32_t *__restrict__ ctr_in,
                                                         uint32_t *__restrict__ ctr_out) {
    const int64_t n = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    // time-step counter (seeds the stochastic rounding of 16-bit shares)
    const uint32_t step = *ctr_in;
    if (n == 0) *ctr_out = step + 1u;
    if (n >= g.N) return;
    if (code_at(g, n) != kFluid) return;
    int x, y, z;
    node_xyz(g, n, x, y, z);
    Pops<L, T> p;
    pull_node<L, S, T>(g, mo, in, x, y, z, n, pulled, p);
    Mom<T> m;
    moments<L, T>(p, m);
    T F[3];
    gradient<L, T>(g, psi, x, y, z, n, F);
    PostOut<L, T> o;
    collide<L, T>(mo, m.drho, m.r36R, m.r36B, m.j, m.S, F, &p, o);
    typename PairOf<S>::type enc[L::Q];
    encode_out<L, S, T>(o, step, uint32_t(n), enc);
    store_node<L, S, T>(g, mo, out, x, y, z, n, enc);
}

template <class L, typename S, typename T>
__global__ void __launch_bounds__(kBlock) k_fields(Geo g, Model<T> mo, const S *__restrict__ st, bool pulled,
                                                   int64_t n0, int64_t cnt, double *__restrict__ out) {
    const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (k >= cnt) return;
    const int64_t n = n0 + k;
    double v[6] = {0, 0, 0, 0, 0, 0};
    if (code_at(g, n) == kFluid) {
        int x, y, z;
        node_xyz(g, n, x, y, z);
        Pops<L, T> p;
        pull_node<L, S, T>(g, mo, st, x, y, z, n, pulled, p);
        Mom<T> m;
        moments<L, T>(p, m);
        const T rho = T(1) + m.drho;
        v[0] = double(m.r36R / T(36));
        v[1] = double(m.r36B / T(36));
        v[2] = double(m.j[0] / rho);
        v[3] = double(m.j[1] / rho);
        v[4] = double(m.j[2] / rho);
        v[5] = double(psi_of<T>(m.drho, m.r36R, m.r36B));
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) out[q * cnt + k] = v[q];
}

template <class L, typename S, typename T>
__global__ void __launch_bounds__(kBlock) k_pops(Geo g, Model<T> mo, const S *__restrict__ st, bool pulled,
                                                 int64_t n0, int64_t cnt, double *__restrict__ out) {
    const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (k >= cnt) return;
    const int64_t n = n0 + k;
    Pops<L, T> p;
    const bool fl = code_at(g, n) == kFluid;
    if (fl) {
        int x, y, z;
        node_xyz(g, n, x, y, z);
        pull_node<L, S, T>(g, mo, st, x, y, z, n, pulled, p);
    }
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        double fR = 0, fB = 0;
        if (fl) {
            const T f = T(wgt<L>(i)) + p.df[i];
            const T r = p.fred(i);
            fR = double(r);
            fB = double(f - r);
        }
        out[int64_t(i) * cnt + k] = fR;
        out[int64_t(L::Q + i) * cnt + k] = fB;
    }
}

template <class L, typename S, typename T>
__global__ void __launch_bounds__(kBlock) k_pops_at(Geo g, Model<T> mo, const S *__restrict__ st, bool pulled,
                                                    const int64_t *__restrict__ nodes, int64_t cnt,
                                                    double *__restrict__ out) {
    const int64_t j = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (j >= cnt) return;
    const int64_t n = nodes[j];
    double *o = out + j * 2 * L::Q;
    if (n < 0 || n >= g.N || code_at(g, n) != kFluid) {
#pragma unroll
        for (int i = 0; i < 2 * L::Q; ++i) {
            o[i] = 0.0;
            asm volatile("" ::: "memory");  // 8-byte stores only (see put_pair)
        }
        return;
    }
    int x, y, z;
    node_xyz(g, n, x, y, z);
    Pops<L, T> p;
    pull_node<L, S, T>(g, mo, st, x, y, z, n, pulled, p);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const T f = T(wgt<L>(i)) + p.df[i];
        const T r = p.fred(i);
        o[i] = double(r);
        o[L::Q + i] = double(f - r);
        asm volatile("" ::: "memory");  // 8-byte stores only (see put_pair)
    }
}

// Diagnostics.  Each fluid node's colour populations are decoded exactly as
// the population export decodes them (each colour part formed in the compute
// type, then widened to FP64), and its moments are summed in FP64 in
// direction order without fused multiply-adds: rho^k = sum_i f_i^k (Eq. (2)),
// rho u = sum_i (f_i^R + f_i^B) c_i (Eq. (3)), psi, |u| and the Eq. (8)
// pressure sum_k phat_k rho^k.  A node whose densities or momentum are not
// finite is counted and left out of the other sums.  The reduction is fixed:
// each thread sums its grid-stride nodes in node order, a wave combines its
// 64 lanes by a butterfly of cross-lane exchanges, the block's waves are
// added in wave order, and a second kernel reduces the block partials the
// same way, so a lattice's diagnostics are bitwise reproducible.  Layout of
// the 13 values: mass_R, mass_B, mom x y z, max|u|, sum p (psi > 0.99),
// n_in, sum p (psi < -0.99), n_out, vol_R, nonfinite, fluid nodes.
constexpr int kDiagMax = 5;  // the one value reduced by max (max |u|)

__device__ __forceinline__ double wave_reduce(double v, bool is_max) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(v, off, 64);
        v = is_max ? fmax(v, o) : v + o;
    }
    return v;
}

// pR, pB: phat_k = sum_i phi_i^k c_ix^2 in FP64 (from the FP64 alpha_k, not
// the compute type's).
template <class L, typename S, typename T>
__global__ void __launch_bounds__(kBlock) k_diag(Geo g, Model<T> mo, const S *__restrict__ st, bool pulled,
                                                 double pR, double pB, double *__restrict__ partials) {
#pragma clang fp contract(off)
    __shared__ double red[kBlock / 64][kDiagVals];
    double acc[kDiagVals];
#pragma unroll
    for (int q = 0; q < kDiagVals; ++q) acc[q] = 0.0;
    for (int64_t n = int64_t(blockIdx.x) * kBlock + threadIdx.x; n < g.N; n += int64_t(gridDim.x) * kBlock) {
        if (code_at(g, n) != kFluid) continue;
        int x, y, z;
        node_xyz(g, n, x, y, z);
        Pops<L, T> p;
        pull_node<L, S, T>(g, mo, st, x, y, z, n, pulled, p);
        double r0 = 0.0, r1 = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            const T f = T(wgt<L>(i)) + p.df[i];
            const T r = p.fred(i);
            const double fr = double(r), fb = double(f - r);
            r0 += fr;
            r1 += fb;
            const double ft = fr + fb;
            jx += ft * double(L::cx[i]);
            jy += ft * double(L::cy[i]);
            jz += ft * double(L::cz[i]);
        }
        acc[12] += 1.0;
        if (!(isfinite(r0) && isfinite(r1) && isfinite(jx) && isfinite(jy) && isfinite(jz))) {
            acc[11] += 1.0;
            continue;
        }
        const double rho = r0 + r1;
        const double psi = (r0 - r1) / rho;
        const double speed = sqrt(jx * jx + jy * jy + jz * jz) / rho;
        const double pres = pR * r0 + pB * r1;  // Eq. (8)
        acc[0] += r0;
        acc[1] += r1;
        acc[2] += jx;
        acc[3] += jy;
        acc[4] += jz;
        acc[5] = fmax(acc[5], speed);
        if (psi > 0.99) {
            acc[6] += pres;
            acc[7] += 1.0;
        } else if (psi < -0.99) {
            acc[8] += pres;
            acc[9] += 1.0;
        }
        acc[10] += 0.5 * (1.0 + psi);
    }
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll
    for (int q = 0; q < kDiagVals; ++q) {
        const double v = wave_reduce(acc[q], q == kDiagMax);
        if (lane == 0) red[wave][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < kDiagVals) {
        const int q = threadIdx.x;
        double a = red[0][q];
        for (int w = 1; w < kBlock / 64; ++w) a = q == kDiagMax ? fmax(a, red[w][q]) : a + red[w][q];
        partials[blockIdx.x * kDiagVals + q] = a;
    }
}

// One wave per value: lane l sums partials l, l + 64, ... in order, then the
// butterfly.
__global__ void __launch_bounds__(64 * kDiagVals) k_diag_final(const double *__restrict__ partials, int nblocks,
                                                              double *__restrict__ res) {
    const int q = threadIdx.x / 64, lane = threadIdx.x % 64;
    const bool is_max = q == kDiagMax;
    double a = 0.0;
    for (int b = lane; b < nblocks; b += 64) {
        const double v = partials[b * kDiagVals + q];
        a = is_max ? fmax(a, v) : a + v;
    }
    a = wave_reduce(a, is_max);
    if (lane == 0) res[q] = a;
}

// ---------------------------------------------------------------- dispatch
template <template <class, typename, typename> class F, typename... A>
static hipError_t dispatch(int lattice, int prec, A &&...args) {
    if (lattice == 0) {
        if (prec == 0) return F<D2Q9, double, double>::run(args...);
        if (prec == 1) return F<D2Q9, float, float>::run(args...);
        return F<D2Q9, _Float16, float>::run(args...);
    }
    if (prec == 0) return F<D3Q19, double, double>::run(args...);
    if (prec == 1) return F<D3Q19, float, float>::run(args...);
    return F<D3Q19, _Float16, float>::run(args...);
}

static inline unsigned blocks_for(int64_t n) { return unsigned((n + kBlock - 1) / kBlock); }

template <class L, typename S, typename T>
struct RunInit {
    static hipError_t run(const Geo &g, const ModelD &md, int64_t n0, int64_t cnt, const double *rR,
                          const double *rB, const double *u, void *st, hipStream_t s) {
        hipLaunchKernelGGL((k_init<L, S, T>), dim3(blocks_for(cnt)), dim3(kBlock), 0, s, g, to_model<T>(md), n0,
                           cnt, rR, rB, u, static_cast<S *>(st));
        return hipGetLastError();
    }
};
template <class L, typename S, typename T>
struct RunPsi {
    static hipError_t run(const Geo &g, const ModelD &md, const void *st, bool pulled, void *psi, hipStream_t s) {
        hipLaunchKernelGGL((k_psi<L, S, T>), dim3(blocks_for(g.N)), dim3(kBlock), 0, s, g, to_model<T>(md),
                           static_cast<const S *>(st), pulled, static_cast<T *>(psi));
        return hipGetLastError();
    }
};
template <class L, typename S, typename T>
struct RunStep {
    static hipError_t run(const Geo &g, const ModelD &md, const void *in, bool pulled, const void *psi, void *out,
                          const uint32_t *ctr_in, uint32_t *ctr_out, hipStream_t s) {
        hipLaunchKernelGGL((k_step_generic<L, S, T>), dim3(blocks_for(g.N)), dim3(kBlock), 0, s, g,
                           to_model<T>(md), static_cast<const S *>(in), pulled, static_cast<const T *>(psi),
                           static_cast<S *>(out), ctr_in, ctr_out);
        return hipGetLastError();
    }
};
template <class L, typename S, typename T>
struct RunFields {
    static hipError_t run(const Geo &g, const ModelD &md, const void *st, bool pulled, int64_t n0, int64_t cnt,
                          double *out, hipStream_t s) {
        hipLaunchKernelGGL((k_fields<L, S, T>), dim3(blocks_for(cnt)), dim3(kBlock), 0, s, g, to_model<T>(md),
                           static_cast<const S *>(st), pulled, n0, cnt, out);
        return hipGetLastError();
    }
};
template <class L, typename S, typename T>
struct RunPops {
    static hipError_t run(const Geo &g, const ModelD &md, const void *st, bool pulled, int64_t n0, int64_t cnt,
                          double *out, hipStream_t s) {
        hipLaunchKernelGGL((k_pops<L, S, T>), dim3(blocks_for(cnt)), dim3(kBlock), 0, s, g, to_model<T>(md),
                           static_cast<const S *>(st), pulled, n0, cnt, out);
        return hipGetLastError();
    }
};
template <class L, typename S, typename T>
struct RunPopsAt {
    static hipError_t run(const Geo &g, const ModelD &md, const void *st, bool pulled, const int64_t *nodes,
                          int64_t cnt, double *out, hipStream_t s) {
        hipLaunchKernelGGL((k_pops_at<L, S, T>), dim3(blocks_for(cnt)), dim3(kBlock), 0, s, g, to_model<T>(md),
                           static_cast<const S *>(st), pulled, nodes, cnt, out);
        return hipGetLastError();
    }
};
template <class L, typename S, typename T>
struct RunDiag {
    static hipError_t run(const Geo &g, const ModelD &md, const void *st, bool pulled, double *partials,
                          double *res, hipStream_t s) {
        const double pR = phat<L, double>(md.aR), pB = phat<L, double>(md.aB);
        hipLaunchKernelGGL((k_diag<L, S, T>), dim3(kDiagBlocks), dim3(kBlock), 0, s, g, to_model<T>(md),
                           static_cast<const S *>(st), pulled, pR, pB, partials);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(64 * kDiagVals), 0, s, partials, kDiagBlocks, res);
        return hipGetLastError();
    }
};

hipError_t launch_init(int lattice, int prec, const Geo &g, const ModelD &md, int64_t n0, int64_t cnt,
                       const double *rhoR, const double *rhoB, const double *u, void *st, hipStream_t s) {
    return dispatch<RunInit>(lattice, prec, g, md, n0, cnt, rhoR, rhoB, u, st, s);
}
hipError_t launch_psi(int lattice, int prec, const Geo &g, const ModelD &md, const void *st, bool pulled,
                      void *psi, hipStream_t s) {
    return dispatch<RunPsi>(lattice, prec, g, md, st, pulled, psi, s);
}
hipError_t launch_step_generic(int lattice, int prec, const Geo &g, const ModelD &md, const void *in,
                               bool pulled, const void *psi, void *out, const uint32_t *ctr_in, uint32_t *ctr_out,
                               hipStream_t s) {
    return dispatch<RunStep>(lattice, prec, g, md, in, pulled, psi, out, ctr_in, ctr_out, s);
}
hipError_t launch_fields(int lattice, int prec, const Geo &g, const ModelD &md, const void *st, bool pulled,
                         int64_t n0, int64_t cnt, double *out, hipStream_t s) {
    return dispatch<RunFields>(lattice, prec, g, md, st, pulled, n0, cnt, out, s);
}
hipError_t launch_pops(int lattice, int prec, const Geo &g, const ModelD &md, const void *st, bool pulled,
                       int64_t n0, int64_t cnt, double *out, hipStream_t s) {
    return dispatch<RunPops>(lattice, prec, g, md, st, pulled, n0, cnt, out, s);
}
hipError_t launch_pops_at(int lattice, int prec, const Geo &g, const ModelD &md, const void *st, bool pulled,
                          const int64_t *nodes, int64_t cnt, double *out, hipStream_t s) {
    return dispatch<RunPopsAt>(lattice, prec, g, md, st, pulled, nodes, cnt, out, s);
}
hipError_t launch_diag(int lattice, int prec, const Geo &g, const ModelD &md, const void *st, bool pulled,
                       double *partials, double *res, hipStream_t s) {
    return dispatch<RunDiag>(lattice, prec, g, md, st, pulled, partials, res, s);
}

}  // namespace lbcg
