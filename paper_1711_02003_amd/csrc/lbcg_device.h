// Device-side building blocks of the regularized colour-gradient (RCG) step
// (arXiv:1711.02003, Sec. II): lattice tables, the storage codec, the pull
// with boundary rules, per-node moments, and the collide-perturb-recolour
// update.  Everything here is header-only so the generic and the fused
// kernels inline the same arithmetic.
//
// Storage (per population i of a node), two values:
//   df_i = f_i^R + f_i^B - w_i       total deviation from the rest state at
//                                    density 1 (FP16 keeps df_i / w_i);
//   m_i  = the minority colour's share of f_i (f_i^B / f_i when red is the
//          majority of the population, f_i^R / f_i otherwise), rounded to
//          one bit less than the storage format, with the freed lowest bit
//          holding the majority flag (1 = red majority).
// The total deviation keeps the small hydrodynamic signal (density and
// velocity perturbations) at full relative precision.  Storing the minority
// share keeps the thin tails of each colour inside the other one at full
// relative precision too: a plain red fraction would be rounded to exactly 1
// deep inside red drops (the spacing of floating-point numbers just below 1
// is coarse) and so turn a little blue into red every step.  Sums that would
// cancel exactly in the bulk (sum_i w_i = 1, sum_i w_i Q_i = 0) are done with
// integer-scaled weights, so bulk nodes carry no colour round-off at all.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbcg {

// Mask codes: fluid; neutral wall; inlets 2..63; wetting walls 64..127 (a
// wall whose phase value the colour gradient sees); outlets 128..255.
constexpr uint8_t kFluid = 0, kWall = 1, kInlet0 = 2, kWall0 = 64, kOutlet0 = 128;
__host__ __device__ constexpr bool is_wall(uint8_t c) { return c == kWall || (c >= kWall0 && c < kOutlet0); }
__host__ __device__ constexpr bool is_inlet(uint8_t c) { return c >= kInlet0 && c < kWall0; }

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
    // the same weights in units of 1/36
    static constexpr int w36[3] = {16, 4, 1};
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
    static constexpr int w36[3] = {12, 2, 1};
};

template <class L>
__host__ __device__ constexpr int csq(int i) {
    return L::cx[i] * L::cx[i] + L::cy[i] * L::cy[i] + L::cz[i] * L::cz[i];
}
template <class L>
__host__ __device__ constexpr double wgt(int i) {
    return L::wc[csq<L>(i)];
}
// 36 w_i (an integer)
template <class L>
__host__ __device__ constexpr int w36(int i) {
    return L::w36[csq<L>(i)];
}
// Perturbation constants B_i = w_i (|c_i|^2 - (D - 1) c_s^2): the choice with
// sum_i B_i = c_s^2 (mass kept) and sum_i B_i c_i c_i = 3 c_s^4 I.
template <class L>
__host__ __device__ constexpr double bcoef(int i) {
    return wgt<L>(i) * (double(csq<L>(i)) - double(L::D - 1) / 3.0);
}
// 3 w_i in the compute type, for the odd part 3 w_i c_i.j of the new
// populations.  The rounded constants are chosen so that sum_i 3 w_i c_i c_i
// is exactly I in type T: D3Q19 needs 2 a + 8 b = 1 (a axis, b diagonal),
// D2Q9 2 a + 4 b = 1, and one constant is the correctly rounded 1/12 or 1/3
// while the other is derived from it exactly (Sterbenz).  With plain rounded
// constants both round up for FP32, and every node's momentum would grow by
// 3e-8 per step.
template <class L, typename T>
__host__ __device__ constexpr T odd_coef(int i) {
    if (L::D == 3) {
        constexpr T b = T(1) / T(12);
        constexpr T a = (T(1) - T(8) * b) * T(0.5);
        return csq<L>(i) == 1 ? a : b;
    }
    constexpr T a = T(1) / T(3);
    constexpr T b = (T(1) - T(2) * a) * T(0.25);
    return csq<L>(i) == 1 ? a : b;
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
struct DevWall {
    double psi;  // phase value of a wetting wall
};

// Scalars of the model in the compute type T, built once per launch.
template <typename T>
struct Model {
    T ivR, ivB;      // 1/nu_k = 1/(c_s^2 (tau_k - 1/2)), component viscosities
    T Abar;          // (A_R + A_B)/2: the perturbations of both colours summed
    T beta;
    T aR, aB;        // alpha_k (Eq. (7)); w_0 for equal densities
    T dR0, dB0;      // phi_0^k - w_0 = alpha_k - w_0
    T kR, kB;        // (phi_i^k - w_i) / w_i = (w_0 - alpha_k) / (1 - w_0), i > 0
    T eps_F;
    T omR, omB;      // 1/tau_k, the per-colour rates of Eq. (5) (bgk == 2)
    int bgk;         // 0: Eq. (11); 1: Eq. (5) at the node's rate; 2: Eq. (5)
                     // with each colour at its own rate
};

// Everything a kernel needs about one lattice.
struct Geo {
    int nx, ny, nz;
    int64_t N, pitch;          // node count, elements per component array
    const uint8_t *mask;       // nullptr = all fluid
    const DevInlet *inlets;
    const DevOutlet *outlets;
    const DevWall *walls;      // wetting walls (codes kWall0 + j)
    const uint32_t *links;     // link words (below), with a mask only
};

// Link word of a node of a lattice with geometry, built on the host from the
// mask so that the boundary writes need no per-direction mask reads.  Fluid
// node: bit i (i < Q) set when the upstream node x - c_i is not fluid;
// kLinkFluid; kLinkOutlet when some upstream node is an outlet; and the mask
// code shared by all its non-fluid upstream nodes in bits 20..27, or
// kLinkMixed when they differ (walls included).  Non-fluid node: its own
// mask code in bits 20..27, nothing else.
constexpr uint32_t kLinkFluid = 1u << 19;
constexpr uint32_t kLinkMixed = 1u << 28;
constexpr uint32_t kLinkOutlet = 1u << 29;
constexpr uint32_t kLinkBits = (1u << 19) - 2u;  // the per-direction bits 1..18
__host__ __device__ constexpr uint8_t link_code(uint32_t lk) { return uint8_t((lk >> 20) & 0xffu); }

__device__ __forceinline__ int wrap_m1(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// Reciprocal and square root for quantities whose rounding does not feed the
// colour bookkeeping (velocity, 1/|F|).  FP32: the hardware reciprocal refined
// by one Newton step, and the hardware square root.  FP64: exact division and
// square root.
template <typename T>
__device__ __forceinline__ T rcp(T x);
template <>
__device__ __forceinline__ float rcp<float>(float x) {
    const float r = __builtin_amdgcn_rcpf(x);
    const float e = __builtin_fmaf(-x, r, 1.0f);
    return __builtin_fmaf(r, e, r);
}
template <>
__device__ __forceinline__ double rcp<double>(double x) { return 1.0 / x; }
template <typename T>
__device__ __forceinline__ T sqrt_(T x);
template <>
__device__ __forceinline__ float sqrt_<float>(float x) { return __builtin_amdgcn_sqrtf(x); }
template <>
__device__ __forceinline__ double sqrt_<double>(double x) { return sqrt(x); }

// ---------------------------------------------------------------- codec
// Round away the lowest bit (to nearest, ties to even on the next bit) and put
// the flag there.  U is the unsigned integer of the storage width.
template <typename U>
__device__ __forceinline__ U pack_flag(U b, bool flag) {
    const U b0 = b & U(1), b1 = (b >> 1) & U(1);
    b = U(b + (b0 & b1) - (b0 & (b1 ^ U(1))));
    return U((b & U(~U(1))) | U(flag ? 1 : 0));
}

template <typename S>
struct Codec;
template <>
struct Codec<double> {
    template <class L, typename T>
    __device__ static __forceinline__ T df(double v, int) { return T(v); }
    template <class L, typename T>
    __device__ static __forceinline__ double enc_df(T v, int) { return double(v); }
    template <typename T>
    __device__ static __forceinline__ T col(double v, bool &flag) {
        const uint64_t b = uint64_t(__double_as_longlong(v));
        flag = b & 1;
        return T(__longlong_as_double((long long)(b & ~uint64_t(1))));
    }
    template <typename T>
    __device__ static __forceinline__ double enc_col(T m, bool flag) {
        return __longlong_as_double(
            (long long)pack_flag<uint64_t>(uint64_t(__double_as_longlong(double(m))), flag));
    }
};
template <>
struct Codec<float> {
    template <class L, typename T>
    __device__ static __forceinline__ T df(float v, int) { return T(v); }
    template <class L, typename T>
    __device__ static __forceinline__ float enc_df(T v, int) { return float(v); }
    template <typename T>
    __device__ static __forceinline__ T col(float v, bool &flag) {
        const uint32_t b = __float_as_uint(v);
        flag = b & 1u;
        return T(__uint_as_float(b & ~1u));
    }
    template <typename T>
    __device__ static __forceinline__ float enc_col(T m, bool flag) {
        return __uint_as_float(pack_flag<uint32_t>(__float_as_uint(float(m)), flag));
    }
};
template <>
struct Codec<_Float16> {
    template <class L, typename T>
    __device__ static __forceinline__ T df(_Float16 v, int i) { return T(float(v)) * T(wgt<L>(i)); }
    template <class L, typename T>
    __device__ static __forceinline__ _Float16 enc_df(T v, int i) {
        return _Float16(float(v * T(1.0 / wgt<L>(i))));
    }
    // The minority share is stored times 2^14 (exact): the shares in an
    // interface's exponential tail would otherwise fall below FP16's normal
    // range (6.1e-5) and round to zero, which drains the thinner colour a
    // little every step; scaled, they stay representable down to ~1e-11.
    // |m| up to 4 fits.
    template <typename T>
    __device__ static __forceinline__ T col(_Float16 v, bool &flag) {
        const uint16_t b = __builtin_bit_cast(uint16_t, v);
        flag = b & 1u;
        return T(float(__builtin_bit_cast(_Float16, uint16_t(b & ~1u))) * (1.0f / 16384.0f));
    }
    template <typename T>
    __device__ static __forceinline__ _Float16 enc_col(T m, bool flag) {
        const uint16_t b = __builtin_bit_cast(uint16_t, _Float16(float(m) * 16384.0f));
        return __builtin_bit_cast(_Float16, pack_flag<uint16_t>(b, flag));
    }
    // Stochastic rounding of float bits to D fewer mantissa bits with D
    // random bits (the low D bits of r) added to the D discarded ones: they
    // carry into the kept bits with probability exactly equal to the
    // discarded fraction, whatever the values.  Fewer random bits (8, placed
    // on the top of the discarded ones, with a fixed offset for the bits
    // below) leave a bias that depends on how those low bits are
    // distributed; on the pair state the minority colour of the interfaces
    // then gained mass, +2e-5 to +2.6e-5 of the droplets' on average over 24
    // runs of 1000 steps of the 27-droplet recipe at 48^3 (against +6e-7
    // with the full dither).
    template <int D>
    __device__ static __forceinline__ uint32_t sr_bits(uint32_t bits, uint32_t r) {
        return (bits + (r & ((1u << D) - 1u))) & ~((1u << D) - 1u);
    }
    // The scaled share rounded stochastically to the 9 stored mantissa bits
    // (14 discarded, 14 random bits).  Round to nearest would repeat the same error every
    // step in a steady interface and drift the colour mass linearly in time;
    // these errors are independent from step to step.  Values below FP16's
    // normal range (the far tail, shares below ~4e-9) end up rounded to
    // nearest by the conversion.
    template <typename T>
    __device__ static __forceinline__ _Float16 enc_col_sr(T m, bool flag, uint32_t r) {
        const uint32_t t = sr_bits<14>(__float_as_uint(float(m) * 16384.0f), r);
        const uint16_t h = __builtin_bit_cast(uint16_t, _Float16(__uint_as_float(t)));
        return __builtin_bit_cast(_Float16, uint16_t((h & ~1u) | (flag ? 1u : 0u)));
    }
    // The deviation likewise (13 discarded bits, 10 kept; 13 random bits): in
    // a steady flow its round-to-nearest error would also repeat every step.
    template <class L, typename T>
    __device__ static __forceinline__ _Float16 enc_df_sr(T v, int i, uint32_t r) {
        const float x = float(v * T(1.0 / wgt<L>(i)));
        return _Float16(__uint_as_float(sr_bits<13>(__float_as_uint(x), r)));
    }
};

// Random bits for the stochastic rounding of stored colour shares: the PCG
// hash of Jarzynski and Olano (J. Computer Graphics Techniques 9(3), 2020)
// seeds one generator per node and time step, and Marsaglia's xorshift32
// (J. Stat. Software 8(14), 2003) draws one word per population.
__device__ __forceinline__ uint32_t pcg_hash(uint32_t v) {
    const uint32_t state = v * 747796405u + 2891336453u;
    const uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
    return (word >> 22u) ^ word;
}
struct Dither {
    uint32_t x;
    __device__ __forceinline__ Dither(uint32_t step, uint32_t node) : x(pcg_hash(node ^ pcg_hash(step)) | 1u) {}
    __device__ __forceinline__ uint32_t next() {
        x ^= x << 13;
        x ^= x >> 17;
        x ^= x << 5;
        return x;
    }
};

// One node's populations in registers: total deviations, minority shares and
// the majority flags (bit i set = red majority of population i).
template <class L, typename T>
struct Pops {
    T df[L::Q];
    T mm[L::Q];
    uint32_t red;
    __device__ __forceinline__ bool flag(int i) const { return (red >> i) & 1u; }
    __device__ __forceinline__ void set(int i, T d, T m, bool fl) {
        df[i] = d;
        mm[i] = m;
        red = fl ? (red | (1u << i)) : (red & ~(1u << i));
    }
    // red part of population i
    __device__ __forceinline__ T fred(int i) const {
        const T f = T(wgt<L>(i)) + df[i];
        const T mu = mm[i] * f;
        return flag(i) ? f - mu : mu;
    }
};

// Populations pulled from the compact state: population i came from node
// x - c_i with that node's minority share mm[i] and majority flag, and vd[i]
// is 36 x its recolouring term c_i . V (V of the sender's speed class, signed
// for the sender's minority colour), so that 36 x the minority colour part is
// mm[i] (36 w_i + 36 df[i]) + vd[i].
template <class L, typename T>
struct CPops {
    T df[L::Q];
    T mm[L::Q];
    T vd[L::Q];
    uint32_t red;
    __device__ __forceinline__ bool flag(int i) const { return (red >> i) & 1u; }
};

// The two stored values of a population travel together: the state is Q
// arrays (one per direction) of value pairs (df_i, m_i), element n of array i
// at pair index i * pitch + n.  A pull then moves one 2-wide element per
// population, half the memory instructions of separate arrays.
template <typename S>
struct PairOf;
template <>
struct PairOf<double> {
    typedef double type __attribute__((ext_vector_type(2)));
};
template <>
struct PairOf<float> {
    typedef float type __attribute__((ext_vector_type(2)));
};
template <>
struct PairOf<_Float16> {
    typedef _Float16 type __attribute__((ext_vector_type(2)));
};

template <class L, typename S, typename T>
__device__ __forceinline__ void decode_pair(typename PairOf<S>::type v, int i, Pops<L, T> &p) {
    bool fl;
    const T d = Codec<S>::template df<L, T>(v.x, i);
    const T m = Codec<S>::template col<T>(v.y, fl);
    p.set(i, d, m, fl);
}

// Stores of more than 8 bytes per lane may read their data registers after
// the compiler has already reused them (seen on 12-byte stores: data of the
// last lanes of each 16-lane group lost under memory back-pressure from a
// concurrent kernel), so 16-byte (FP64) pairs are written as two 8-byte
// halves, with a compiler barrier between them that keeps them from being
// merged into one store again.
template <typename P2>
__device__ __forceinline__ void put_pair(P2 *p, P2 v) {
    if constexpr (sizeof(P2) > 8) {
        double *d = reinterpret_cast<double *>(p);
        d[0] = double(v.x);
        asm volatile("" ::: "memory");
        d[1] = double(v.y);
    } else {
        *p = v;
    }
}

template <class L, typename S, typename T>
__device__ __forceinline__ typename PairOf<S>::type encode_pair(T df, T m, bool redmaj, int i) {
    typename PairOf<S>::type v;
    v.x = Codec<S>::template enc_df<L, T>(df, i);
    v.y = Codec<S>::template enc_col<T>(m, redmaj);
    return v;
}

// Encoding of a time step's output: 16-bit shares are rounded
// stochastically with the node's generator, wider ones to nearest.
template <class L, typename S, typename T>
__device__ __forceinline__ typename PairOf<S>::type encode_step(T df, T m, bool redmaj, int i, Dither &dz) {
    if constexpr (sizeof(S) == 2) {
        // one 32-bit draw per population: 14 bits for the share, 13 for the
        // deviation
        const uint32_t r = dz.next();
        typename PairOf<S>::type v;
        v.x = Codec<S>::template enc_df_sr<L, T>(df, i, r >> 14);
        v.y = Codec<S>::template enc_col_sr<T>(m, redmaj, r);
        return v;
    } else {
        return encode_pair<L, S, T>(df, m, redmaj, i);
    }
}

template <class L, typename S, typename T>
__device__ __forceinline__ void load_raw(const S *__restrict__ st, int64_t pitch, int64_t node, int i,
                                         Pops<L, T> &p) {
    const typename PairOf<S>::type *a = reinterpret_cast<const typename PairOf<S>::type *>(st);
    decode_pair<L, S, T>(a[int64_t(i) * pitch + node], i, p);
}

// Minority share and majority flag from the red and blue shares of a
// population (each formed directly, so the minority one is precise).
template <typename T>
__device__ __forceinline__ void split_shares(T shareR, T shareB, T &m, bool &redmaj) {
    redmaj = shareR >= shareB;
    m = redmaj ? shareB : shareR;
}

// ---------------------------------------------------------------- moments
// Colour sums are kept in units of 1/36 (the weights are then the integers
// 36 w_i) and rounded once at the end: a rounded weight constant would shift
// every mixed node's colour mass the same way, step after step.  Per
// population, 36 f_i^R and 36 f_i^B are split into an integer weight part
// (counted from the majority flags) and a small floating part:
//   red majority:  36 f^R = 36 w + (36 df - mu),  36 f^B = mu,
//   blue majority: 36 f^R = mu,  36 f^B = 36 w + (36 df - mu),
// with mu = m (36 w + 36 df) the minority colour in units of 1/36.

// Direction masks of a lattice (bit i = direction i), built at compile time.
template <class L>
__host__ __device__ constexpr uint32_t dir_mask(int a, int kind) {
    // kind 0: axis directions along a; 1: diagonals with c_a != 0;
    // 2: diagonals in the plane of pair a with c_p c_q > 0; 3: ... < 0
    uint32_t m = 0;
    for (int i = 1; i < L::Q; ++i) {
        const int c[3] = {L::cx[i], L::cy[i], L::cz[i]};
        const int n2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
        const int pq[3][2] = {{0, 1}, {0, 2}, {1, 2}};
        if (kind == 0 && n2 == 1 && c[a] != 0) m |= 1u << i;
        if (kind == 1 && n2 == 2 && c[a] != 0) m |= 1u << i;
        if (kind >= 2 && n2 == 2) {
            const int pr = c[pq[a][0]] * c[pq[a][1]];
            if ((kind == 2 && pr > 0) || (kind == 3 && pr < 0)) m |= 1u << i;
        }
    }
    return m;
}

__device__ __forceinline__ int popc(uint32_t x) { return __builtin_popcount(x); }

// all diagonal directions
template <class L>
__host__ __device__ constexpr uint32_t dir_mask_diag() {
    uint32_t m = 0;
    for (int i = 1; i < L::Q; ++i)
        if (csq<L>(i) == 2) m |= 1u << i;
    return m;
}

// sum of 36 w_i over the red-majority directions among the given axis and
// diagonal directions (and the rest direction if asked)
template <class L>
__device__ __forceinline__ int w36_sum(uint32_t red, uint32_t axes, uint32_t diags, bool rest) {
    return (rest ? int(red & 1u) * L::w36[0] : 0) + L::w36[1] * popc(red & axes) + L::w36[2] * popc(red & diags);
}

// 36 x red and 36 x blue floating parts of population i
template <class L, typename T>
__device__ __forceinline__ void colour_parts(const Pops<L, T> &p, int i, T &r36, T &b36) {
    const T d = p.df[i];
    const T mu = p.mm[i] * (T(w36<L>(i)) + T(36) * d);
    const T t = T(36) * d - mu;
    const bool fl = p.flag(i);
    r36 = fl ? t : mu;
    b36 = fl ? mu : t;
}
template <class L, typename T>
__device__ __forceinline__ void colour_parts(const CPops<L, T> &p, int i, T &r36, T &b36) {
    const T d = p.df[i];
    const T mu = p.mm[i] * (T(w36<L>(i)) + T(36) * d) + p.vd[i];
    const T t = T(36) * d - mu;
    const bool fl = p.flag(i);
    r36 = fl ? t : mu;
    b36 = fl ? mu : t;
}

// Densities (Eq. (2)): the deviation of the total density and 36 x the red
// and blue densities (each exact in the other colour's bulk).  Every path
// computes psi through this one expression sequence, so psi is bitwise the
// same whichever kernel or tile shape produced it.
template <class L, typename T, class P>
__device__ __forceinline__ void densities(const P &p, T &drho_out, T &r36R, T &r36B) {
    T drho = 0, Ra = 0, Ba = 0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        T r36, b36;
        colour_parts<L, T>(p, i, r36, b36);
        drho += p.df[i];
        Ra += r36;
        Ba += b36;
    }
    const uint32_t all = (1u << L::Q) - 2u;
    const int K = w36_sum<L>(p.red, all & ~dir_mask_diag<L>(), dir_mask_diag<L>(), true);
    drho_out = drho;
    r36R = T(K) + Ra;
    r36B = T(36 - K) + Ba;
}

// 36 x the total density
template <typename T>
__device__ __forceinline__ T rho36(T drho) {
    return T(36) + T(36) * drho;
}

// Phase field psi = (rho^R - rho^B) / rho from 36 x the colour densities,
// with the minority colour's share formed directly so that psi is exactly +1
// or -1 in the bulk of either colour.
template <typename T>
__device__ __forceinline__ T psi_of(T drho, T r36R, T r36B) {
    const T r36 = rho36<T>(drho);
    return r36R >= r36B ? T(1) - T(2) * r36B / r36 : T(2) * r36R / r36 - T(1);
}

// Moments of one node: densities, total momentum (Eq. (3)) and the
// trace-adjusted momentum flux sum_i f_i Q_i with Q_i = c_i c_i - I/3
// (components xx, yy, zz, xy, xz, yz).  The flux sum uses
// sum_i g_i (c_ia^2 - 1/3) = sum_{c_ia != 0} g_i - (1/3) sum_i g_i.
template <typename T>
struct Mom {
    T drho;
    T r36R, r36B;  // 36 x rho^R, 36 x rho^B
    T j[3];
    T S[6];
};

template <class L, typename T, class P>
__device__ __forceinline__ void moments(const P &p, Mom<T> &m) {
    T drho = 0, Ra = 0, Ba = 0;
    T jd[3] = {0, 0, 0}, Sd[3] = {0, 0, 0}, So[3] = {0, 0, 0};
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        T r36, b36;
        colour_parts<L, T>(p, i, r36, b36);
        const T d = p.df[i];
        drho += d;
        Ra += r36;
        Ba += b36;
        const int c[3] = {L::cx[i], L::cy[i], L::cz[i]};
#pragma unroll
        for (int a = 0; a < L::D; ++a) {
            if (c[a]) {
                jd[a] += c[a] > 0 ? d : -d;
                Sd[a] += d;
            }
        }
        const int off[3] = {c[0] * c[1], c[0] * c[2], c[1] * c[2]};
#pragma unroll
        for (int b = 0; b < (L::D == 3 ? 3 : 1); ++b) {
            if (off[b]) So[b] += off[b] > 0 ? d : -d;
        }
    }
    const uint32_t all = (1u << L::Q) - 2u;
    const int K = w36_sum<L>(p.red, all & ~dir_mask_diag<L>(), dir_mask_diag<L>(), true);
    m.drho = drho;
    m.r36R = T(K) + Ra;
    m.r36B = T(36 - K) + Ba;
#pragma unroll
    for (int a = 0; a < 3; ++a) m.j[a] = jd[a];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        m.S[a] = a < L::D ? Sd[a] - drho * T(1.0 / 3.0) : T(0);
    }
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        m.S[3 + b] = (b == 0 || L::D == 3) ? So[b] : T(0);
    }
}

// phi_i(alpha) of Eq. (7): alpha at rest, the remainder shared among moving
// directions in proportion to w_i.  The collision uses phi_i^k - w_i, formed
// from alpha_k - w_0 so that it is exactly zero for equal densities (a
// difference of two rounded constants would add a little mass every step).
template <class L, typename T>
__device__ __forceinline__ T phi(int i, T alpha) {
    return i == 0 ? alpha : (T(1) - alpha) * T(wgt<L>(i) / (1.0 - wgt<L>(0)));
}
template <class L, typename T>
__device__ __forceinline__ T dphi(int i, T d0, T k) {
    return i == 0 ? d0 : T(wgt<L>(i)) * k;
}
// sum_i phi_i c_ix^2: (1 - alpha) * sum_{moving} w_i c_ix^2 / (1 - w_0)
template <class L, typename T>
__host__ __device__ __forceinline__ T phat(T alpha) {
    return (T(1) - alpha) * T((1.0 / 3.0) / (1.0 - wgt<L>(0)));
}

// ---------------------------------------------------------------- pull
// Boundary rules are applied when a fluid node stores its new state: for
// every link i whose upstream node x - c_i is not fluid, the node writes the
// value it will pull through that link at the next step into the upstream
// node's slot of direction i.  Only this node ever reads that slot, so a pull
// is a plain load on every link.  Wall: half-way bounce-back (the node's own
// new pair of the opposite direction, copied as stored).  Inlet: moving-wall
// bounce-back injecting the inlet's colour densities.  Outlet:
// anti-bounce-back at the outlet density with the node's own red fraction
// and velocity, taken from its stored new pairs.

// Density, red density and velocity of a node's stored new pairs (the outlet
// rule's inputs), with the arithmetic and summation order of densities() and
// of the momentum sum.
template <typename T>
struct OwnMom {
    T rho, rR, u[3];
};
template <class L, typename S, typename T>
__device__ __forceinline__ OwnMom<T> own_moments(const typename PairOf<S>::type *enc) {
    T drho = 0, Ra = 0, Ba = 0, jx = 0, jy = 0, jz = 0;
    int K = 0;
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
        bool fl;
        const T d = Codec<S>::template df<L, T>(enc[k].x, k);
        const T m = Codec<S>::template col<T>(enc[k].y, fl);
        const T mu = m * (T(w36<L>(k)) + T(36) * d);
        const T t = T(36) * d - mu;
        drho += d;
        Ra += fl ? t : mu;
        Ba += fl ? mu : t;
        K += fl ? w36<L>(k) : 0;
        jx += T(L::cx[k]) * d;
        jy += T(L::cy[k]) * d;
        jz += T(L::cz[k]) * d;
    }
    OwnMom<T> om;
    om.rho = T(1) + drho;
    om.rR = (T(K) + Ra) / T(36);
    om.u[0] = jx / om.rho;
    om.u[1] = jy / om.rho;
    om.u[2] = jz / om.rho;
    (void)Ba;
    return om;
}

// The scalars of an inlet (velocity and colour densities) or an outlet
// (density) in the compute type; zero for walls.
template <typename T>
struct IoVals {
    T u[3], rhoR, rhoB, rout;
};
template <typename T>
__device__ __forceinline__ IoVals<T> io_vals(const Geo &g, uint8_t code) {
    IoVals<T> v{};
    if (is_inlet(code)) {
        const DevInlet in = g.inlets[code - kInlet0];
        v.u[0] = T(in.u[0]);
        v.u[1] = T(in.u[1]);
        v.u[2] = T(in.u[2]);
        v.rhoR = T(in.rhoR);
        v.rhoB = T(in.rhoB);
    } else if (!is_wall(code)) {
        v.rout = T(g.outlets[code - kOutlet0].rho);
    }
    return v;
}

// Value a fluid node pulls through link i from a non-fluid upstream node of
// mask code `code`, from the node's own stored new pair of the opposite
// direction (own_io) and, for outlets, its own moments.  Walls return own_io
// unchanged; inlet and outlet values are encoded rounded to nearest.  The
// total deviation f_i - w_i is formed from deviations only (the stored dfo,
// the inlet's momentum term, the outlet's density excess, phi - w and the
// velocity terms), never as a difference of two full populations: in FP32
// that difference would lose the ~1e-9 absolute precision that the stored
// deviations keep, and the boundary nodes' velocity with it.
template <class L, typename S, typename T>
__device__ __forceinline__ typename PairOf<S>::type boundary_pair_v(const Model<T> &mo, int i, uint8_t code,
                                                                    const IoVals<T> &iv,
                                                                    typename PairOf<S>::type own_io,
                                                                    const OwnMom<T> &om) {
    if (is_wall(code)) return own_io;
    const int io = L::opp[i];
    bool flo;
    const T dfo = Codec<S>::template df<L, T>(own_io.x, io);
    const T mo_ = Codec<S>::template col<T>(own_io.y, flo);
    const T fo = T(wgt<L>(io)) + dfo;
    const T mu = mo_ * fo;
    const T fRo = flo ? fo - mu : mu, fBo = fo - fRo;
    T fR, fB, dev;  // the colour populations and the total deviation f - w_i
    if (is_inlet(code)) {
        const T cu = T(L::cx[io]) * iv.u[0] + T(L::cy[io]) * iv.u[1] + T(L::cz[io]) * iv.u[2];
        const T mom = T(6.0 * wgt<L>(io)) * cu;  // 2 w c.u / c_s^2
        fR = fRo - mom * iv.rhoR;
        fB = fBo - mom * iv.rhoB;
        dev = dfo - mom * (iv.rhoR + iv.rhoB);
    } else {
        const T rout = iv.rout;
        const T rwR = rout * om.rR / om.rho, rwB = rout - rwR;
        const T cu = T(L::cx[io]) * om.u[0] + T(L::cy[io]) * om.u[1] + T(L::cz[io]) * om.u[2];
        const T uu = om.u[0] * om.u[0] + om.u[1] * om.u[1] + om.u[2] * om.u[2];
        const T wv = T(wgt<L>(io)) * (T(4.5) * cu * cu - T(1.5) * uu);
        const T phR = phi<L, T>(io, mo.aR), phB = phi<L, T>(io, mo.aB);
        fR = T(2) * rwR * (phR + wv) - fRo;
        fB = T(2) * rwB * (phB + wv) - fBo;
        // 2 sum_k rw_k (phi_k + wv) - f_o - w with phi_k = w + (phi_k - w) and
        // f_o = w + dfo
        const T dpR = dphi<L, T>(io, mo.dR0, mo.kR), dpB = dphi<L, T>(io, mo.dB0, mo.kB);
        dev = T(2) * T(wgt<L>(io)) * (rout - T(1)) + T(2) * (rwR * dpR + rwB * dpB) + T(2) * rout * wv - dfo;
    }
    const T f = fR + fB;
    T mm;
    bool fl;
    split_shares<T>(f != T(0) ? fR / f : T(0), f != T(0) ? fB / f : T(0), mm, fl);
    return encode_pair<L, S, T>(dev, mm, fl, i);
}

// The same with the inlet's or outlet's scalars read from the lattice.
template <class L, typename S, typename T>
__device__ __forceinline__ typename PairOf<S>::type boundary_pair(const Geo &g, const Model<T> &mo, int i,
                                                                  uint8_t code,
                                                                  typename PairOf<S>::type own_io,
                                                                  const OwnMom<T> &om) {
    return boundary_pair_v<L, S, T>(mo, i, code, io_vals<T>(g, code), own_io, om);
}

// Pre-collision populations of fluid node (x, y, z) = n at the new time level
// from the stored post-collision state (Eq. (1), pull form).  A link from a
// non-fluid node reads the boundary value its fluid neighbour stored there.
// With pulled == false the stored state already is pre-collision and is read
// in place.
template <class L, typename S, typename T>
__device__ __forceinline__ void pull_node(const Geo &g, const Model<T> &, const S *__restrict__ st,
                                          int x, int y, int z, int64_t n, bool pulled, Pops<L, T> &p) {
    p.red = 0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        int64_t m = n;
        if (pulled) {
            const int xs = wrap_m1(x - L::cx[i], g.nx);
            const int ys = wrap_m1(y - L::cy[i], g.ny);
            const int zs = wrap_m1(z - L::cz[i], g.nz);
            m = xs + int64_t(g.nx) * (ys + int64_t(g.ny) * zs);
        }
        load_raw<L, S, T>(st, g.pitch, m, i, p);
    }
}

// ---------------------------------------------------------------- collide
// Output of one node: new total deviation, minority share and majority flag
// of every direction.
template <class L, typename T>
struct PostOut {
    static constexpr bool kCompact = false;
    T df[L::Q];
    T mm[L::Q];
    uint32_t red;
};

// Output of one node in compact form: the new total deviations and the
// node's colour scalars, from which a receiver recolours each population
// (Eq. (10) is linear in f_i with coefficients that depend only on the
// sending node and on the speed class of c_i).  For a population f_i that
// the node sends, its minority colour part is
//   M f_i + (c_i . V_c) / 36,
// with M the node's minority share, c the speed class of c_i (axis or
// diagonal) and V_c = +-36 beta rho^R rho^B / rho^2 k_c F / |F|, signed for
// the minority colour, k_c = (w_c rho + rho^R (phi_c^R - w_c) +
// rho^B (phi_c^B - w_c)) / |c_c|.
template <class L, typename T>
struct CompactOut {
    static constexpr bool kCompact = true;
    T df[L::Q];
    T M;
    bool redmaj;
    T Va[3], Vd[3];
    T Rd;  // k_diag / k_axis: V_diag = Rd V_axis
};

// First axis and first diagonal direction of a lattice.
template <class L>
__host__ __device__ constexpr int first_dir(int n2) {
    for (int i = 1; i < L::Q; ++i)
        if (csq<L>(i) == n2) return i;
    return 0;
}

// Collision (Eq. (11), or Eq. (5) with bgk), perturbation (Eq. (9)) and
// recolouring (Eq. (10)) from the node's density deviation, colour
// densities, momentum, trace-adjusted flux S, colour gradient F and - for
// plain BGK only - its populations.  The node relaxes at one rate
// omega = 1/tau, tau = nu/c_s^2 + 1/2, from the mixture viscosity
// 1/nu = sum_k (rho^k/rho)/nu_k; with s = 1/nu that is omega = 2s/(s + 6).
// Opposite directions i and -i share every even term (weights, Q_i, (c.u)^2,
// (F.c)^2, B_i, phi_i) and flip the odd ones (c.u, cos), so the update is
// computed once per pair.
//
// With a CompactOut the recolouring is left to the receiver: the node emits
// its total deviations and the scalars that define every population's
// colour split.
template <class L, typename T, class O>
__device__ __forceinline__ void collide(const Model<T> &mo, T drho, T r36R, T r36B, const T j[3], const T S[6],
                                        const T F[3], const Pops<L, T> *pin, O &o) {
    const T rho = T(1) + drho;
    const T rR = r36R * T(1.0 / 36.0), rB = r36B * T(1.0 / 36.0);
    const T inv_rho = rcp<T>(rho);
    const T ux = j[0] * inv_rho, uy = j[1] * inv_rho, uz = j[2] * inv_rho;
    const T usq = ux * ux + uy * uy + uz * uz;
    const T pR = phat<L, T>(mo.aR), pB = phat<L, T>(mo.aB);
    // colour shares rho^k / rho, the minority one formed directly (exactly 0 in
    // the other colour's bulk) with one correctly rounded division: a rounded
    // constant or an approximate reciprocal would err to one side and bias
    // colour mass through the recolouring.  rec_i / f_i may use the refined
    // reciprocal: rec is odd in i, so a common error cancels between i and -i.
    const T r36 = rho36<T>(drho);
    const bool redmaj = r36R >= r36B;
    const T sB = redmaj ? r36B / r36 : T(1) - r36R / r36;
    const T sR = redmaj ? T(1) - sB : r36R / r36;
    const T sv = sR * mo.ivR + sB * mo.ivB;
    const T om = T(2) * sv * rcp<T>(sv + T(6));
    const T gm = T(1) - om;
    // N = (1 - omega) Pi^neq in Q form: Pi^neq = sum_i f_i c c -
    // sum_k rho^k (phat_k I + u u) = S + sum_k rho^k (1/3 - phat_k) I - rho u u.
    const T cw = gm * rho;
    const T iso = gm * (rR * (T(1.0 / 3.0) - pR) + rB * (T(1.0 / 3.0) - pB));
    T N[6];
    const T uu[6] = {ux * ux, uy * uy, uz * uz, ux * uy, ux * uz, uy * uz};
#pragma unroll
    for (int q = 0; q < 6; ++q) N[q] = gm * S[q] - cw * uu[q];
    N[0] += iso;
    N[1] += iso;
    if (L::D == 3) N[2] += iso;

    const T Fx = F[0], Fy = F[1], Fz = F[2];
    const T F2 = Fx * Fx + Fy * Fy + Fz * Fz;
    const T Fn = sqrt_<T>(F2);
    const bool hasF = Fn > mo.eps_F;
    const T invFn = hasF ? rcp<T>(Fn) : T(0);
    const T seg = mo.beta * rR * rB * inv_rho * inv_rho;
    const T wrho = rho * T(1.5) * usq;  // rho u^2 / (2 c_s^2)
    if constexpr (!O::kCompact) o.red = 0;
    T dsum = T(0);  // sum of the new moving deviations

#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        if (L::opp[i] < i) continue;  // handled with its partner
        const int ib = L::opp[i];
        const T w = T(wgt<L>(i));
        const T cx = T(L::cx[i]), cy = T(L::cy[i]), cz = T(L::cz[i]);
        // the odd parts are formed from the momentum itself (rho c.u = c.j):
        // a rounded velocity would change the node's momentum by a relative
        // ulp per step, in the same direction every step, and so drift the
        // total momentum of a box
        const T cj = cx * j[0] + cy * j[1] + cz * j[2];
        const T cu = cx * ux + cy * uy + cz * uz;
        const T dpR = dphi<L, T>(i, mo.dR0, mo.kR), dpB = dphi<L, T>(i, mo.dB0, mo.kB);
        T ev, od;  // even and odd parts of the new total deviation of direction i
        // (kernels that pass no populations run the regularized form only;
        // the runtime keeps BGK lattices off them)
        if (!mo.bgk || pin == nullptr) {
            T qn = (cx * cx - T(1.0 / 3.0)) * N[0] + (cy * cy - T(1.0 / 3.0)) * N[1];
            if (L::D == 3) qn += (cz * cz - T(1.0 / 3.0)) * N[2];
            qn += T(2) * cx * cy * N[3];
            if (L::D == 3) qn += T(2) * (cx * cz * N[4] + cy * cz * N[5]);
            // sum_k rho^k phi_i^k - w_i  +  w_i rho U  +  w_i/(2 c_s^4) Q_i : N
            ev = w * drho + rR * dpR + rB * dpB + w * (T(4.5) * cj * cu - wrho) + T(4.5) * w * qn;
            od = odd_coef<L, T>(i) * cj;
        } else if (mo.bgk == 1) {
            // (1 - omega) f_i + omega sum_k f_i^{k,eq} - w_i, split into the
            // parts even and odd under i <-> -i (the populations themselves
            // have no symmetry, so both directions are formed here).  The
            // equilibrium's deviation sum_k f_i^{k,eq} - w_i is formed from
            // deviations, as in the regularized form (w_i drho + sum_k rho^k
            // (phi_i^k - w_i) + w_i rho U_i), not as the difference of two
            // full populations, which in FP32 would leave an error of ~1e-9
            // in every population every step.
            const T eq = w * drho + rR * dpR + rB * dpB + w * (T(4.5) * cj * cu - wrho);
            const T lin = om * (odd_coef<L, T>(i) * cj);
            const T di = gm * pin->df[i];
            const T db = gm * pin->df[ib];
            ev = om * eq + T(0.5) * (di + db);
            od = lin + T(0.5) * (di - db);
        } else {
            // Eq. (5) with each colour at its own rate omega_k:
            // sum_k (1 - omega_k) f_i^k + omega_k f_i^{k,eq} - w_i, with the
            // blue part written as f_i - f_i^R and the terms grouped into
            // deviations (as above):
            // (1 - omega_B) df_i + (omega_B - omega_R) (f_i^R - rho^R w_i) +
            // omega_B w_i drho + sum_k omega_k rho^k ((phi_i^k - w_i) + w_i U_i).
            const T U2 = T(4.5) * cu * cu - T(1.5) * usq;
            const T base = mo.omB * w * drho + mo.omR * rR * (dpR + w * U2) + mo.omB * rB * (dpB + w * U2);
            const T lin = (mo.omR * rR + mo.omB * rB) * inv_rho * (odd_coef<L, T>(i) * cj);
            const T dom = mo.omB - mo.omR;
            const T gB = T(1) - mo.omB;
            const T rw = rR * w;
            const T di = gB * pin->df[i] + dom * (pin->fred(i) - rw);
            const T db = gB * pin->df[ib] + dom * (pin->fred(ib) - rw);
            ev = base + T(0.5) * (di + db);
            od = lin + T(0.5) * (di - db);
        }
        if constexpr (O::kCompact) {
            if (hasF) {
                const T Fh = (Fx * cx + Fy * cy + Fz * cz) * invFn;
                ev += mo.Abar * Fn * (w * Fh * Fh - T(bcoef<L>(i)));
            }
            o.df[i] = ev + od;
            o.df[ib] = ev - od;
            dsum += o.df[i] + o.df[ib];
        } else {
        T cosp = T(0);
        if (hasF) {
            const T Fh = (Fx * cx + Fy * cy + Fz * cz) * invFn;
            ev += mo.Abar * Fn * (w * Fh * Fh - T(bcoef<L>(i)));
            cosp = Fh * T(inv_len<L>(i));
        }
        // recolouring, Eq. (10): f_i^R = (rho^R/rho) f_i + rec_i and
        // f_i^B = (rho^B/rho) f_i - rec_i
        const T rec = seg * cosp * (w * rho + rR * dpR + rB * dpB);
        const T d_i = ev + od;
        const T f_i = w + d_i;
        T m;
        bool fl;
        const T q_i = f_i != T(0) ? rec * rcp<T>(f_i) : T(0);
        split_shares<T>(sR + q_i, sB - q_i, m, fl);
        o.df[i] = d_i;
        o.mm[i] = m;
        o.red |= fl ? (1u << i) : 0u;
        const T d_b = ev - od;
        const T f_b = w + d_b;
        const T q_b = f_b != T(0) ? rec * rcp<T>(f_b) : T(0);
        split_shares<T>(sR - q_b, sB + q_b, m, fl);
        o.df[ib] = d_b;
        o.mm[ib] = m;
        o.red |= fl ? (1u << ib) : 0u;
        dsum += d_i + d_b;
        }
    }
    // The rest population is the remainder that keeps the node's mass: the
    // relaxation, the perturbation and the recolouring all conserve it, so
    // this is the same value in exact arithmetic, while rounded constants
    // that should cancel (sum_i (phi_i - w_i), sum_i w_i Q_i : N with
    // phat != 1/3) would otherwise add a small mass of one sign every step.
    // Its recolouring term is zero (cos phi_0 = 0), so its share is rho^R/rho.
    if constexpr (O::kCompact) {
        T m;
        bool fl;
        split_shares<T>(sR, sB, m, fl);
        o.df[0] = drho - dsum;
        o.M = m;
        o.redmaj = fl;
        // 36 x the recolouring term of Eq. (10) as c_i . V_c, signed for the
        // minority colour (f^B_i = (rho^B/rho) f_i - rec_i, f^R_i = ... + rec_i)
        constexpr int ia = first_dir<L>(1), id = first_dir<L>(2);
        const T g = hasF ? (fl ? T(-36) : T(36)) * seg * invFn : T(0);
        const T ka = T(inv_len<L>(ia)) * (T(wgt<L>(ia)) * rho + rR * dphi<L, T>(ia, mo.dR0, mo.kR) +
                                          rB * dphi<L, T>(ia, mo.dB0, mo.kB));
        const T kd = T(inv_len<L>(id)) * (T(wgt<L>(id)) * rho + rR * dphi<L, T>(id, mo.dR0, mo.kR) +
                                          rB * dphi<L, T>(id, mo.dB0, mo.kB));
        const T ga = g * ka, gd = g * kd;
        o.Va[0] = ga * Fx;
        o.Va[1] = ga * Fy;
        o.Va[2] = ga * Fz;
        o.Vd[0] = gd * Fx;
        o.Vd[1] = gd * Fy;
        o.Vd[2] = gd * Fz;
        o.Rd = kd / ka;  // ka > 0: rho^k phi_c^k > 0 for alpha_k < 1
    } else {
        T m;
        bool fl;
        split_shares<T>(sR, sB, m, fl);
        o.df[0] = drho - dsum;
        o.mm[0] = m;
        o.red |= fl ? 1u : 0u;
    }
}

// Encoded new pairs of one node (16-bit storage rounds stochastically with
// the node's generator).
template <class L, typename S, typename T>
__device__ __forceinline__ void encode_out(const PostOut<L, T> &o, uint32_t step, uint32_t node,
                                           typename PairOf<S>::type enc[L::Q]) {
    Dither dz(step, node);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) enc[i] = encode_step<L, S, T>(o.df[i], o.mm[i], (o.red >> i) & 1u, i, dz);
}

// Store a fluid node's encoded new pairs and, with geometry, the boundary
// values of its non-fluid links into the upstream nodes' slots.
template <class L, typename S, typename T>
__device__ __forceinline__ void store_node(const Geo &g, const Model<T> &mo, S *__restrict__ st, int x, int y,
                                           int z, int64_t node, const typename PairOf<S>::type enc[L::Q]) {
    typename PairOf<S>::type *a = reinterpret_cast<typename PairOf<S>::type *>(st);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) put_pair(a + int64_t(i) * g.pitch + node, enc[i]);
    if (!g.mask) return;
    bool own = false;
    OwnMom<T> om{};
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        const int xs = wrap_m1(x - L::cx[i], g.nx);
        const int ys = wrap_m1(y - L::cy[i], g.ny);
        const int zs = wrap_m1(z - L::cz[i], g.nz);
        const int64_t m = xs + int64_t(g.nx) * (ys + int64_t(g.ny) * zs);
        const uint8_t code = g.mask[m];
        if (code == kFluid) continue;
        if (code >= kOutlet0 && !own) {
            om = own_moments<L, S, T>(enc);
            own = true;
        }
        put_pair(a + int64_t(i) * g.pitch + m, boundary_pair<L, S, T>(g, mo, i, code, enc[L::opp[i]], om));
    }
}

}  // namespace lbcg
