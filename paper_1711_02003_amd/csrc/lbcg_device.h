// Device-side building blocks of the regularized colour-gradient (RCG) step
// (arXiv:1711.02003, Sec. II): lattice tables, the storage codec, the pull
// with boundary rules, per-node moments, and the collide-perturb-recolour
// update.  Everything here is header-only so the generic and the fused
// kernels inline the same arithmetic.
//
// Storage (per population i of a node): the total deviation
//     df_i = f_i^R + f_i^B - w_i          (rest reference density 1)
// and the red fraction
//     chi_i = f_i^R / (f_i^R + f_i^B).
// The total deviation keeps the small hydrodynamic signal (density and
// velocity perturbations) at full relative precision; chi is exactly 1 or 0
// in the bulk of each colour, so colour bookkeeping adds no round-off there.
// FP16 storage keeps df_i / w_i instead of df_i to stay in the normal range.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbcg {

constexpr uint8_t kFluid = 0, kWall = 1, kInlet0 = 2, kOutlet0 = 128;

// ---------------------------------------------------------------- lattices
// D2Q9: rest, then counter-clockwise from +x alternating axis and diagonal
// (the numbering of Eq. (7), shifted to start at zero).
struct D2Q9 {
    static constexpr int Q = 9, D = 2;
    static constexpr int cx[9] = {0, 1, 1, 0, -1, -1, -1, 0, 1};
    static constexpr int cy[9] = {0, 0, 1, 1, 1, 0, -1, -1, -1};
    static constexpr int cz[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr int opp[9] = {0, 5, 6, 7, 8, 1, 2, 3, 4};
    // weights 4/9, 1/9, 1/36 by squared speed 0, 1, 2
    static constexpr double wc[3] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 36.0};
};

// D3Q19: rest; +x -x +y -y +z -z; the twelve face diagonals grouped by plane
// (xy, xz, yz), each as (+,+) (+,-) (-,+) (-,-).
struct D3Q19 {
    static constexpr int Q = 19, D = 3;
    static constexpr int cx[19] = {0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 0, 0, 0, 0};
    static constexpr int cy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1};
    static constexpr int cz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
    static constexpr int opp[19] = {0, 2, 1, 4, 3, 6, 5, 10, 9, 8, 7, 14, 13, 12, 11, 18, 17, 16, 15};
    static constexpr double wc[3] = {1.0 / 3.0, 1.0 / 18.0, 1.0 / 36.0};
};

template <class L>
__host__ __device__ constexpr int csq(int i) {
    return L::cx[i] * L::cx[i] + L::cy[i] * L::cy[i] + L::cz[i] * L::cz[i];
}
template <class L>
__host__ __device__ constexpr double wgt(int i) {
    return L::wc[csq<L>(i)];
}
// Perturbation constants B_i = w_i (|c_i|^2 - (D - 1) c_s^2): the choice with
// sum_i B_i = c_s^2 (mass kept) and sum_i B_i c_i c_i = 3 c_s^4 I.
template <class L>
__host__ __device__ constexpr double bcoef(int i) {
    return wgt<L>(i) * (double(csq<L>(i)) - double(L::D - 1) / 3.0);
}
template <class L>
__host__ __device__ constexpr double inv_len(int i) {
    return csq<L>(i) == 0 ? 0.0 : (csq<L>(i) == 1 ? 1.0 : 0.70710678118654752440);
}

// ---------------------------------------------------------------- params
struct DevInlet {
    double u[3];
    double rhoR, rhoB;
};
struct DevOutlet {
    double rho;
};

// Scalars of the model in the compute type T, built once per launch.
template <typename T>
struct Model {
    T omR, omB;      // 1/tau_k
    T Abar;          // (A_R + A_B)/2: the perturbations of both colours summed
    T beta;
    T aR, aB;        // alpha_k (Eq. (7)); w_0 for equal densities
    T eps_F;
    int bgk;         // plain BGK relaxation (Eq. (5)) instead of Eq. (11)
};

// Everything a kernel needs about one lattice.
struct Geo {
    int nx, ny, nz;
    int64_t N, pitch;          // node count, elements per component array
    const uint8_t *mask;       // nullptr = all fluid
    const DevInlet *inlets;
    const DevOutlet *outlets;
};

__device__ __forceinline__ int wrap_m1(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// ---------------------------------------------------------------- codec
template <typename S>
struct Codec {
    template <class L, typename T>
    __device__ static __forceinline__ T df(S v, int) { return T(v); }
    template <class L, typename T>
    __device__ static __forceinline__ S enc_df(T v, int) { return S(v); }
};
template <>
struct Codec<_Float16> {
    template <class L, typename T>
    __device__ static __forceinline__ T df(_Float16 v, int i) { return T(float(v)) * T(wgt<L>(i)); }
    template <class L, typename T>
    __device__ static __forceinline__ _Float16 enc_df(T v, int i) {
        return _Float16(float(v * T(1.0 / wgt<L>(i))));
    }
};

template <class L, typename S, typename T>
__device__ __forceinline__ void load_raw(const S *__restrict__ st, int64_t pitch, int64_t node, int i,
                                         T &df, T &chi) {
    df = Codec<S>::template df<L, T>(st[int64_t(i) * pitch + node], i);
    chi = T(st[int64_t(L::Q + i) * pitch + node]);
}

// ---------------------------------------------------------------- moments
// Density and red density (Eq. (2)); also what the phase field needs.  Every
// path computes psi through this one expression sequence, so psi is bitwise
// the same whichever kernel or tile shape produced it.
template <class L, typename T>
__device__ __forceinline__ void densities(const T *df, const T *chi, T &drho_out, T &rhoR) {
    T drho = 0, r1 = 0, r2 = 0;
    const T c0 = chi[0];
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        drho += df[i];
        r1 += (chi[i] - c0) * T(wgt<L>(i));
        r2 += chi[i] * df[i];
    }
    drho_out = drho;
    rhoR = c0 + r1 + r2;
}

// Phase field psi = (rho^R - rho^B) / rho from the density deviation and the
// red density.
template <typename T>
__device__ __forceinline__ T psi_of(T drho, T rhoR) {
    const T rho = T(1) + drho;
    return (rhoR - (rho - rhoR)) / rho;
}

// Moments of one node from its (df, chi) populations: density deviation,
// red density (Eq. (2)), total momentum (Eq. (3)) and the trace-adjusted
// momentum fluxes sum_i f_i Q_i and sum_i f_i^R Q_i with Q_i = c_i c_i - I/3
// (components xx, yy, zz, xy, xz, yz).  sum_i w_i = 1 and sum_i w_i Q_i = 0
// let the rest-state part cancel exactly.
template <typename T>
struct Mom {
    T drho, rhoR;
    T j[3];
    T S[6];
    T PR[6];
};

template <class L, typename T>
__device__ __forceinline__ void moments(const T *df, const T *chi, Mom<T> &m) {
    T drho, rhoR;
    densities<L, T>(df, chi, drho, rhoR);
    T jx = 0, jy = 0, jz = 0;
    T S[6] = {0, 0, 0, 0, 0, 0}, P[6] = {0, 0, 0, 0, 0, 0};
    const T c0 = chi[0];
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const T d = df[i];
        const T g = chi[i] * d + (chi[i] - c0) * T(wgt<L>(i));  // red part minus c0 w_i
        if (L::cx[i]) jx += L::cx[i] > 0 ? d : -d;
        if (L::cy[i]) jy += L::cy[i] > 0 ? d : -d;
        if (L::cz[i]) jz += L::cz[i] > 0 ? d : -d;
        const T qxx = T(L::cx[i] * L::cx[i]) - T(1.0 / 3.0);
        const T qyy = T(L::cy[i] * L::cy[i]) - T(1.0 / 3.0);
        S[0] += qxx * d;
        P[0] += qxx * g;
        S[1] += qyy * d;
        P[1] += qyy * g;
        if (L::D == 3) {
            const T qzz = T(L::cz[i] * L::cz[i]) - T(1.0 / 3.0);
            S[2] += qzz * d;
            P[2] += qzz * g;
        }
        const int xy = L::cx[i] * L::cy[i];
        if (xy) { S[3] += xy > 0 ? d : -d; P[3] += xy > 0 ? g : -g; }
        if (L::D == 3) {
            const int xz = L::cx[i] * L::cz[i], yz = L::cy[i] * L::cz[i];
            if (xz) { S[4] += xz > 0 ? d : -d; P[4] += xz > 0 ? g : -g; }
            if (yz) { S[5] += yz > 0 ? d : -d; P[5] += yz > 0 ? g : -g; }
        }
    }
    m.drho = drho;
    m.rhoR = rhoR;
    m.j[0] = jx;
    m.j[1] = jy;
    m.j[2] = jz;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        m.S[q] = S[q];
        m.PR[q] = P[q];
    }
}

// ---------------------------------------------------------------- pull
// Pre-collision populations of fluid node (x, y, z) = n at the new time level
// from the stored post-collision state (Eq. (1), pull form), with the
// boundary rules for non-fluid upstream nodes: wall -> half-way bounce-back;
// inlet -> moving-wall bounce-back injecting the inlet's colour densities;
// outlet -> anti-bounce-back at the outlet density.  With pulled == false the
// stored state already is pre-collision and is read in place.
template <class L, typename S, typename T>
__device__ __forceinline__ void pull_node(const Geo &g, const Model<T> &mo, const S *__restrict__ st,
                                          int x, int y, int z, int64_t n, bool pulled, T *df,
                                          T *chi) {
    if (!pulled) {
#pragma unroll
        for (int i = 0; i < L::Q; ++i) load_raw<L, S, T>(st, g.pitch, n, i, df[i], chi[i]);
        return;
    }
    bool own = false;
    T oR = 0, oRho = 0, oU[3] = {0, 0, 0};
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const int xs = wrap_m1(x - L::cx[i], g.nx);
        const int ys = wrap_m1(y - L::cy[i], g.ny);
        const int zs = wrap_m1(z - L::cz[i], g.nz);
        const int64_t m = xs + int64_t(g.nx) * (ys + int64_t(g.ny) * zs);
        const uint8_t code = g.mask ? g.mask[m] : kFluid;
        if (code == kFluid) {
            load_raw<L, S, T>(st, g.pitch, m, i, df[i], chi[i]);
            continue;
        }
        const int io = L::opp[i];
        T dfo, chio;
        load_raw<L, S, T>(st, g.pitch, n, io, dfo, chio);
        if (code == kWall) {
            df[i] = dfo;  // w_io == w_i
            chi[i] = chio;
        } else if (code < kOutlet0) {
            const DevInlet in = g.inlets[code - kInlet0];
            const T cu = T(L::cx[io]) * T(in.u[0]) + T(L::cy[io]) * T(in.u[1]) + T(L::cz[io]) * T(in.u[2]);
            const T mom = T(6.0 * wgt<L>(io)) * cu;  // 2 w c.u / c_s^2
            const T tot = T(wgt<L>(io)) + dfo - mom * T(in.rhoR + in.rhoB);
            const T red = chio * (T(wgt<L>(io)) + dfo) - mom * T(in.rhoR);
            df[i] = dfo - mom * T(in.rhoR + in.rhoB);
            chi[i] = tot != T(0) ? red / tot : T(0);
        } else {
            if (!own) {
                // moments of this node's own post-collision populations
                T d[L::Q], c[L::Q];
#pragma unroll
                for (int k = 0; k < L::Q; ++k) load_raw<L, S, T>(st, g.pitch, n, k, d[k], c[k]);
                T odr;
                densities<L, T>(d, c, odr, oR);
                oRho = T(1) + odr;
                T jx = 0, jy = 0, jz = 0;
#pragma unroll
                for (int k = 0; k < L::Q; ++k) {
                    jx += T(L::cx[k]) * d[k];
                    jy += T(L::cy[k]) * d[k];
                    jz += T(L::cz[k]) * d[k];
                }
                oU[0] = jx / oRho;
                oU[1] = jy / oRho;
                oU[2] = jz / oRho;
                own = true;
            }
            const T rout = T(g.outlets[code - kOutlet0].rho);
            const T rwR = rout * oR / oRho, rwB = rout - rwR;
            const T cu = T(L::cx[io]) * oU[0] + T(L::cy[io]) * oU[1] + T(L::cz[io]) * oU[2];
            const T uu = oU[0] * oU[0] + oU[1] * oU[1] + oU[2] * oU[2];
            const T wv = T(wgt<L>(io)) * (T(4.5) * cu * cu - T(1.5) * uu);
            const T phR = io == 0 ? mo.aR : (T(1) - mo.aR) * T(wgt<L>(io) / (1.0 - wgt<L>(0)));
            const T phB = io == 0 ? mo.aB : (T(1) - mo.aB) * T(wgt<L>(io) / (1.0 - wgt<L>(0)));
            const T evR = rwR * (phR + wv), evB = rwB * (phB + wv);
            const T fo = T(wgt<L>(io)) + dfo;
            const T tot = T(2) * (evR + evB) - fo;
            const T red = T(2) * evR - chio * fo;
            df[i] = tot - T(wgt<L>(i));
            chi[i] = tot != T(0) ? red / tot : T(0);
        }
    }
}

// ---------------------------------------------------------------- collide
// phi_i(alpha) of Eq. (7): alpha at rest, the remainder shared among moving
// directions in proportion to w_i.
template <class L, typename T>
__device__ __forceinline__ T phi(int i, T alpha) {
    return i == 0 ? alpha : (T(1) - alpha) * T(wgt<L>(i) / (1.0 - wgt<L>(0)));
}
// sum_i phi_i c_ix^2: (1 - alpha) * sum_{moving} w_i c_ix^2 / (1 - w_0)
template <class L, typename T>
__device__ __forceinline__ T phat(T alpha) {
    return (T(1) - alpha) * T((1.0 / 3.0) / (1.0 - wgt<L>(0)));
}

// Output of one node: the new (df, chi) of every direction.
template <class L, typename T>
struct PostOut {
    T df[L::Q];
    T chi[L::Q];
};

// The part of N = sum_k (1 - omega_k) Pi^{k,neq} that comes straight from
// the populations: G = (1 - omega_B) sum_i f_i Q_i + (omega_B - omega_R)
// sum_i f_i^R Q_i.  A node carries only (drho, rhoR, j, G) into collide.
template <typename T>
__device__ __forceinline__ void fold_flux(const Model<T> &mo, const Mom<T> &m, T G[6]) {
    const T gR = T(1) - mo.omR, gB = T(1) - mo.omB;
#pragma unroll
    for (int q = 0; q < 6; ++q) G[q] = gB * m.S[q] + (gR - gB) * m.PR[q];
}

// Collision (Eq. (11), or Eq. (5) with bgk), perturbation (Eq. (9)) and
// recolouring (Eq. (10)) from the node's density deviation, red density,
// momentum, folded flux G, colour gradient F and - for plain BGK only - its
// populations.
template <class L, typename T>
__device__ __forceinline__ void collide(const Model<T> &mo, T drho, T rR, const T j[3], const T G[6],
                                        const T F[3], const T *dfin, const T *chiin,
                                        PostOut<L, T> &o) {
    const T rho = T(1) + drho;
    const T rB = rho - rR;
    const T inv_rho = T(1) / rho;
    const T ux = j[0] * inv_rho, uy = j[1] * inv_rho, uz = j[2] * inv_rho;
    const T usq = ux * ux + uy * uy + uz * uz;
    const T pR = phat<L, T>(mo.aR), pB = phat<L, T>(mo.aB);
    // N in Q form: Pi^{k,neq} = sum_i f_i^k c c - rho^k (phat_k I + u u)
    //     = sum_i f_i^k Q_i + rho^k (1/3 - phat_k) I - rho^k u u.
    const T gR = T(1) - mo.omR, gB = T(1) - mo.omB;
    const T cw = gR * rR + gB * rB;
    const T iso = gR * rR * (T(1.0 / 3.0) - pR) + gB * rB * (T(1.0 / 3.0) - pB);
    T N[6];
    const T uu[6] = {ux * ux, uy * uy, uz * uz, ux * uy, ux * uz, uy * uz};
#pragma unroll
    for (int q = 0; q < 6; ++q) N[q] = G[q] - cw * uu[q];
    N[0] += iso;
    N[1] += iso;
    if (L::D == 3) N[2] += iso;

    const T Fx = F[0], Fy = F[1], Fz = F[2];
    const T F2 = Fx * Fx + Fy * Fy + Fz * Fz;
    const T Fn = sqrt(F2);
    const bool hasF = Fn > mo.eps_F;
    const T invFn = hasF ? T(1) / Fn : T(0);
    const T seg = mo.beta * rR * rB * inv_rho * inv_rho;
    const T fracR = rR * inv_rho;

#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const T w = T(wgt<L>(i));
        const T cx = T(L::cx[i]), cy = T(L::cy[i]), cz = T(L::cz[i]);
        const T cu = cx * ux + cy * uy + cz * uz;
        const T U = T(3) * cu + T(4.5) * cu * cu - T(1.5) * usq;
        const T phR = phi<L, T>(i, mo.aR), phB = phi<L, T>(i, mo.aB);
        T d;
        if (!mo.bgk) {
            T qn = (cx * cx - T(1.0 / 3.0)) * N[0] + (cy * cy - T(1.0 / 3.0)) * N[1];
            if (L::D == 3) qn += (cz * cz - T(1.0 / 3.0)) * N[2];
            qn += T(2) * cx * cy * N[3];
            if (L::D == 3) qn += T(2) * (cx * cz * N[4] + cy * cz * N[5]);
            // sum_k rho^k phi_i^k - w_i  +  w_i rho U  +  w_i/(2 c_s^4) Q_i : N
            d = w * drho + rR * (phR - w) + rB * (phB - w) + w * rho * U + T(4.5) * w * qn;
        } else {
            // sum_k [(1 - omega_k) f_i^k + omega_k f_i^{k,eq}] - w_i
            const T fi = w + dfin[i];
            const T fRi = chiin[i] * fi;
            d = gB * dfin[i] + (gR - gB) * fRi - mo.omB * w + mo.omR * rR * (phR + w * U) +
                mo.omB * rB * (phB + w * U);
        }
        T cosp = T(0);
        if (hasF) {
            const T Fc = Fx * cx + Fy * cy + Fz * cz;
            const T Fh = Fc * invFn;
            d += mo.Abar * Fn * (w * Fh * Fh - T(bcoef<L>(i)));
            cosp = Fh * T(inv_len<L>(i));
        }
        const T f2 = w + d;
        const T rec = seg * cosp * (rR * phR + rB * phB);
        o.df[i] = d;
        o.chi[i] = f2 != T(0) ? fracR + rec / f2 : fracR;
    }
}

}  // namespace lbcg
