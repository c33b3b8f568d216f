#pragma once
// Device code of the fused single-pass D3Q19 RCG step on a compact state
// (arXiv:1711.02003, Sec. II, Eqs. (1)-(11)), periodic lattices, FP32 or
// FP16 storage with FP32 arithmetic, shared by the single-lattice kernels (lbcg_compact.hip) and the batched
// one (lbcg_compact_batch.hip), which are built as separate objects so that
// each gets the code-generation options measured best for it.  The split
// step of lattices with geometry (lbcg_geo.hip) stores and reads the same
// layout through CStore.
//
// The recolouring of Eq. (10) splits each post-collision population f_i into
// colours with coefficients that depend only on the sending node (its colour
// densities, density and colour gradient) and on the speed class of c_i:
//   minority colour part of f_i = M f_i + (c_i . V_c) / 36,
// with M the node's minority share and V_c one 3-vector per speed class
// (axis, diagonal).  Both vectors are the unit colour gradient scaled by a
// class amplitude, so V_diag = R_d V_axis with the node scalar
// R_d = k_diag / k_axis.  So a node need not store the two colours of every
// population: it stores its 19 new total deviations and 5 colour scalars (M
// with the majority flag in its lowest bit, V_axis, R_d), and the receiver
// splits each pulled population with the scalars of the node it came from.
// In exact arithmetic the step is the same as the pair-state step; in FP32
// it moves 2 x (19 x 4 + 20) = 192 bytes per node instead of 2 x 38 x 4 =
// 304, in FP16 2 x (19 x 2 + 12) = 100 instead of 152.
//
// Layout (FP32): 19 arrays of `pitch` floats (array i at i * pitch + node:
// total deviation f_i - w_i), then `pitch` 16-byte records {M, V_axis x, y,
// z} (record n at float 19 * pitch + 4 n) and an array of `pitch` floats R_d
// (at float 23 * pitch + n).  The FP16 layout is given with CStore below.
//
// The sweep is the pair-state sweep's: a block owns a 64 x 8 column tile and
// sweeps a chunk of z planes; plane z+1 is pulled (interior and a one-node
// ring from cache) into psi in a 5-slot LDS ring while plane z collides.  A
// receiver of direction i needs the sender's total of i (a plain pull), its
// M and one (axis) or two (diagonal) components of its V.  Gathered from
// memory per direction that would be ~68 loads per node, more than a wave
// can keep in flight (its memory counter holds 63), so the records are
// staged instead: each plane's records over the tile plus a two-node halo
// (the ring's own senders) are loaded once, with a 16-byte and a 4-byte
// load per node, into a 4-slot LDS ring, three planes ahead of their first
// use, and the receivers read them from there.  The threads of the three
// waves that hold the ring nodes load no records, so every wave keeps fewer
// than 63 memory operations in flight.  The batched form runs the same sweep
// over many lattices from a block table.  The first step after an
// initialisation or a restore reads a pair state instead (the same sweep
// with pair pulls), so the compact state always holds what a recolouring
// produced.
#include <mutex>
#include <set>
#include <utility>

#include "lbcg_buffer.h"
#include "lbcg_internal.h"

namespace lbcg {

namespace {

constexpr int kCTX = 64;                    // tile width of the batched sweep
constexpr int kCR = 8;                      // tile rows
constexpr int kCXCD = 8;
constexpr int kNS = 5;                      // scalars kept in LDS: M, V_axis, R_d
constexpr int kSSlots = 4;
constexpr int kPSlots = 5;

// Shape of a tile TX x kCR (one thread per node) and what follows from it:
// the record tile with a 2-node halo (SW x SH), the psi tile with a 1-node
// halo (PW x PH), the ring nodes (held by the first threads, whose waves
// load no records) and the record loaders (the threads of the other waves,
// PER nodes each), and the LDS of a block.  64 x 8 (512 threads): ring 148
// in waves 0-2, loaders 320 x 3; 32 x 8 (256 threads): ring 84 in waves
// 0-1, loaders 128 x 4.
template <int TX>
struct CTile {
    static constexpr int W = TX, R = kCR, threads = TX * kCR;
    static constexpr int SW = TX + 4, SH = kCR + 4, SN = SW * SH;
    static constexpr int PW = TX + 2, PH = kCR + 2, PN = PW * PH;
    static constexpr int ring = 2 * (TX + 2) + 2 * kCR;
    static constexpr int load0 = (ring + 63) / 64 * 64;
    static constexpr int loaders = threads - load0;
    static constexpr int per = (SN + loaders - 1) / loaders;
    static constexpr size_t lds = (size_t(kPSlots) * PN + size_t(kSSlots) * kNS * SN) * sizeof(float);
    static constexpr size_t lds_pair = size_t(kPSlots) * PN * sizeof(float);
    static_assert(loaders > 0 && per <= 4, "tile shape");
};

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));
typedef unsigned int u2 __attribute__((ext_vector_type(2)));

// Every buffer access takes its wave-uniform byte offset through
// readfirstlane at the point of use: the compiler otherwise may merge equal
// offsets of different accesses into vector registers and then wrap each
// access in a loop over the distinct values of its scalar offset.
__device__ __forceinline__ int su(uint32_t v) { return __builtin_amdgcn_readfirstlane(int(v)); }

// Records are written with stores of at most 8 bytes per lane.  A wider
// store (12 or 16 bytes) may read its data registers after later
// instructions have been issued, and the compiler reuses those registers at
// once (seen: the next store's address written into the first data register
// of a 12-byte store, with its later lanes' data lost under memory
// back-pressure).
__device__ __forceinline__ void store_u2(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, u2 v) {
    __builtin_amdgcn_raw_buffer_store_b64(v, r, int(voff), su(soff), kNonTemporal);
}
__device__ __forceinline__ void store_u1(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, uint32_t v) {
    __builtin_amdgcn_raw_buffer_store_b32(v, r, int(voff), su(soff), kNonTemporal);
}
__device__ __forceinline__ void store_h1(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, uint16_t v) {
    __builtin_amdgcn_raw_buffer_store_b16(v, r, int(voff), su(soff), kNonTemporal);
}

// Storage of the compact state, S = float or _Float16.  The state is 19
// arrays of `pitch` totals (E bytes each), then `pitch` records A of kRecA
// bytes and `pitch` records B of kRecB bytes.
//   FP32: the values as computed; A = {M, V_axis x, y, z}, B = {R_d}
//   (16 B and 4 B; 96 B per node).
//   FP16: totals (f_i - w_i) / w_i, as the FP16 pair state stores them,
//   rounded stochastically; A = {M as FP32, V_axis x, y as FP16},
//   B = {V_axis z, R_d as FP16} (8 B and 4 B; 50 B per node).  M stays FP32
//   because its rounding moves mass between the colours and one M serves
//   all 19 populations of the node: at FP16 it random-walks each colour's
//   mass about four times as fast as the FP16 pair state's independent
//   per-population shares do.  V_axis (|V_axis| <= 9 beta k_axis) and R_d
//   are rounded stochastically; neither changes a colour's mass (the sum of
//   c_i . V over the directions of a class is zero).
// Stochastic rounding takes 13 random bits per value from the node's
// generator (seeded by the time step and x + nx (y + ny z)), so a rounding
// error does not repeat step after step in a steady flow.  A sweep keeps
// pulled totals and loaded records in their stored form while the loads are
// in flight and decodes them at use; the LDS record planes always hold FP32
// entries {M with flag, V_axis} and R_d.
template <typename S>
struct CStore;
template <>
struct CStore<float> {
    static constexpr uint32_t E = 4, kRecA = 16, kRecB = 4;
    typedef uint32_t Raw;
    typedef f4 RawA;
    typedef uint32_t RawB;
    __device__ static __forceinline__ Raw load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
        return __builtin_amdgcn_raw_buffer_load_b32(r, int(voff), su(soff), 0);
    }
    __device__ static __forceinline__ float df(Raw v, int) { return __builtin_bit_cast(float, v); }
    __device__ static __forceinline__ RawA load_a(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
        return __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, int(voff), su(soff), 0));
    }
    __device__ static __forceinline__ RawB load_b(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
        return __builtin_amdgcn_raw_buffer_load_b32(r, int(voff), su(soff), 0);
    }
    __device__ static __forceinline__ f4 entry(RawA v, RawB) { return v; }
    __device__ static __forceinline__ float ratio(RawB v) { return __builtin_bit_cast(float, v); }
    // Compact output of the node at byte column `own` (E bytes per node) of
    // the plane that starts at node zcol.
    __device__ static __forceinline__ void store(__amdgpu_buffer_rsrc_t rout, uint32_t own, uint32_t zcol, uint32_t pitch,
                                                 const CompactOut<D3Q19, float> &o, uint32_t) {
        // the direction stride as a value of its own: shared with the pulls'
        // offsets, the compiler would keep its multiples in vector registers
        const uint32_t cs = uint32_t(uniform(int(pitch * E)));
        const uint32_t zoff = zcol * E;
#pragma unroll
        for (int i = 0; i < D3Q19::Q; ++i)
            store_u1(rout, own, uint32_t(i) * cs + zoff, __builtin_bit_cast(uint32_t, o.df[i]));
        const uint32_t ra = uint32_t(D3Q19::Q) * cs + zcol * kRecA,
                       rb = uint32_t(D3Q19::Q) * cs + pitch * kRecA + zcol * kRecB;
        const f2 a01 = {Codec<float>::enc_col<float>(o.M, o.redmaj), o.Va[0]}, a23 = {o.Va[1], o.Va[2]};
        store_u2(rout, own * (kRecA / E), ra, __builtin_bit_cast(u2, a01));
        store_u2(rout, own * (kRecA / E), ra + 8u, __builtin_bit_cast(u2, a23));
        store_u1(rout, own * (kRecB / E), rb, __builtin_bit_cast(uint32_t, o.Rd));
    }
};
template <>
struct CStore<_Float16> {
    static constexpr uint32_t E = 2, kRecA = 8, kRecB = 4;
    typedef uint16_t Raw;
    typedef u2 RawA;
    typedef uint32_t RawB;
    __device__ static __forceinline__ float h2f(uint32_t b) { return float(__builtin_bit_cast(_Float16, uint16_t(b))); }
    __device__ static __forceinline__ Raw load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
        return __builtin_amdgcn_raw_buffer_load_b16(r, int(voff), su(soff), 0);
    }
    __device__ static __forceinline__ float df(Raw v, int i) {
        return Codec<_Float16>::df<D3Q19, float>(__builtin_bit_cast(_Float16, v), i);
    }
    __device__ static __forceinline__ RawA load_a(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
        return __builtin_amdgcn_raw_buffer_load_b64(r, int(voff), su(soff), 0);
    }
    __device__ static __forceinline__ RawB load_b(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
        return __builtin_amdgcn_raw_buffer_load_b32(r, int(voff), su(soff), 0);
    }
    __device__ static __forceinline__ f4 entry(RawA a, RawB b) {
        const f4 e = {__builtin_bit_cast(float, a[0]), h2f(a[1] & 0xffffu), h2f(a[1] >> 16), h2f(b & 0xffffu)};
        return e;
    }
    __device__ static __forceinline__ float ratio(RawB b) { return h2f(b >> 16); }
    // x rounded stochastically to FP16 with the 13 low random bits of r (the
    // rounding of the FP16 pair state's deviations); the FP16 bits in the
    // low half
    __device__ static __forceinline__ uint32_t sr(float x, uint32_t r) {
        const uint32_t t = Codec<_Float16>::sr_bits<13>(__float_as_uint(x), r);
        return __builtin_bit_cast(uint16_t, _Float16(__uint_as_float(t)));
    }
    // Random bits: 13 per value, two values per 32-bit draw (bits 0-12 and
    // 16-28): draws 0-9 for the 19 totals and R_d, 10-11 for V_axis.
    __device__ static __forceinline__ void store(__amdgpu_buffer_rsrc_t rout, uint32_t own, uint32_t zcol, uint32_t pitch,
                                                 const CompactOut<D3Q19, float> &o, uint32_t step) {
        Dither dz(step, own / E + zcol);
        uint32_t w = 0;
        // the direction stride as a value of its own: shared with the pulls'
        // offsets, the compiler would keep its multiples in vector registers
        const uint32_t cs = uint32_t(uniform(int(pitch * E)));
        const uint32_t zoff = zcol * E;
#pragma unroll
        for (int i = 0; i < D3Q19::Q; ++i) {
            if ((i & 1) == 0) w = dz.next();
            const _Float16 h = Codec<_Float16>::enc_df_sr<D3Q19, float>(o.df[i], i, (i & 1) ? w >> 16 : w);
            store_h1(rout, own, uint32_t(i) * cs + zoff, __builtin_bit_cast(uint16_t, h));
        }
        const uint32_t rd = sr(o.Rd, w >> 16);
        w = dz.next();
        const u2 ra = {__float_as_uint(Codec<float>::enc_col<float>(o.M, o.redmaj)),
                       sr(o.Va[0], w) | (sr(o.Va[1], w >> 16) << 16)};
        const uint32_t rb = sr(o.Va[2], dz.next()) | (rd << 16);
        const uint32_t oa = uint32_t(D3Q19::Q) * cs + zcol * kRecA,
                       ob = uint32_t(D3Q19::Q) * cs + pitch * kRecA + zcol * kRecB;
        store_u2(rout, own * (kRecA / E), oa, ra);
        store_u1(rout, own * (kRecB / E), ob, rb);
    }
};

__device__ __forceinline__ void c_lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

struct CompactArgs {
    const void *in;  // compact state, or pair state (pair_in)
    void *out;       // compact state
    int nx, ny, nz;
    int64_t pitch;
    const uint32_t *ctr_in;
    uint32_t *ctr_out;
    int ntx, nty, zchunks;
};

__device__ __forceinline__ int wrap_any(int a, int n) {
    const int r = a % n;
    return r < 0 ? r + n : r;
}

// Byte offsets (x' + nx y') * E of the 9 source columns of (x, y), entry
// (1 - c_x) + 3 (1 - c_y), periodic.
template <uint32_t E>
__device__ __forceinline__ void col_offsets(const CompactArgs &a, int x, int y, uint32_t t[9]) {
    const uint32_t xs[3] = {uint32_t(x == 0 ? a.nx - 1 : x - 1), uint32_t(x), uint32_t(x == a.nx - 1 ? 0 : x + 1)};
    const uint32_t ys[3] = {uint32_t(y == 0 ? a.ny - 1 : y - 1), uint32_t(y), uint32_t(y == a.ny - 1 ? 0 : y + 1)};
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) t[c + 3 * b] = (xs[c] + uint32_t(a.nx) * ys[b]) * E;
}

// Byte offsets of planes z-1, z, z+1 (periodic) for plane size `plane`.
__device__ __forceinline__ void z_offsets(int z, int nz, uint32_t plane, uint32_t zo[3]) {
    zo[0] = uint32_t(uniform(z == 0 ? nz - 1 : z - 1)) * plane;
    zo[1] = uint32_t(uniform(z)) * plane;
    zo[2] = uint32_t(uniform(z == nz - 1 ? 0 : z + 1)) * plane;
}

__device__ __forceinline__ int wrapz_c(int z, int nz) { return z < 0 ? z + nz : (z >= nz ? z - nz : z); }

// Split of the 19 pulled totals d of a node with its senders' scalars, read
// from the LDS record planes sl[0..2] (planes p-1, p, p+1 of the pulled plane
// p) at tile index c of the node (stride kSW per row).  A record plane holds,
// with ENTRIES, one 16-byte entry {M, V_axis} per node (one LDS read per
// sender), else four arrays M, V_axis x, y, z; then the R_d of every node.
// The single-lattice sweep measured 0.7 % faster with entries, the batched
// one 2.7 % slower, so each uses its own.
template <bool ENTRIES, int kSW, int kSN>
__device__ __forceinline__ void split_pulled(const float d[D3Q19::Q], const float *const sl[3], int c,
                                             CPops<D3Q19, float> &p) {
    using L = D3Q19;
    p.red = 0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const int cv[3] = {L::cx[i], L::cy[i], L::cz[i]};
        const float *s = sl[1 - cv[2]];
        const int k = c - cv[1] * kSW - cv[0];
        bool fl;
        p.df[i] = d[i];
        const int n2 = cv[0] * cv[0] + cv[1] * cv[1] + cv[2] * cv[2];
        if constexpr (ENTRIES) {
            const f4 r = reinterpret_cast<const f4 *>(s)[k];
            p.mm[i] = Codec<float>::col<float>(r[0], fl);
            if (n2 == 0) {
                p.vd[i] = 0.0f;
            } else if (n2 == 1) {
                const int ax = cv[0] ? 0 : (cv[1] ? 1 : 2);
                const float v = r[1 + ax];
                p.vd[i] = cv[ax] > 0 ? v : -v;
            } else {
                const int a0 = cv[0] ? 0 : 1, a1 = cv[2] ? 2 : 1;
                const float v0 = r[1 + a0], v1 = r[1 + a1];
                const float s0 = cv[a0] > 0 ? v0 : -v0;
                p.vd[i] = s[4 * kSN + k] * (cv[a1] > 0 ? s0 + v1 : s0 - v1);
            }
        } else {
            p.mm[i] = Codec<float>::col<float>(s[k], fl);
            if (n2 == 0) {
                p.vd[i] = 0.0f;
            } else if (n2 == 1) {
                const int ax = cv[0] ? 0 : (cv[1] ? 1 : 2);
                const float v = s[(1 + ax) * kSN + k];
                p.vd[i] = cv[ax] > 0 ? v : -v;
            } else {
                const int a0 = cv[0] ? 0 : 1, a1 = cv[2] ? 2 : 1;
                const float v0 = s[(1 + a0) * kSN + k], v1 = s[(1 + a1) * kSN + k];
                const float s0 = cv[a0] > 0 ? v0 : -v0;
                p.vd[i] = s[4 * kSN + k] * (cv[a1] > 0 ? s0 + v1 : s0 - v1);
            }
        }
        p.red |= fl ? (1u << i) : 0u;
    }
}

// ------------------------------------------------------------- compact in
template <bool ENTRIES, int TX, typename S = float>
__device__ __forceinline__ void sweep_compact(const CompactArgs &a, const Model<float> &mo, int tile, int chunk,
                                              float *lds) {
    using L = D3Q19;
    typedef float T;
    typedef CTile<TX> G;
    typedef CStore<S> St;
    constexpr int kCTX = TX, kSW = G::SW, kSN = G::SN, kPW = G::PW, kPN = G::PN;
    constexpr int kLoad0 = G::load0, kLoaders = G::loaders, kPerLoader = G::per;
    const int lane = threadIdx.x % kCTX, row = threadIdx.x / kCTX;
    const int tx = tile % a.ntx, ty = tile / a.ntx;
    const int x0 = tx * kCTX, y0 = ty * kCR;
    const int tw = min(kCTX, a.nx - x0), th = min(kCR, a.ny - y0);
    const int z0 = int((int64_t(chunk) * a.nz) / a.zchunks);
    const int z1 = int((int64_t(chunk + 1) * a.nz) / a.zchunks);
    if (z1 <= z0) return;  // uniform over the block

    const bool intile = lane < tw && row < th;
    const int x = x0 + lane, y = y0 + row;

    // ring node of this thread (at most one; threads below G::ring, all in
    // the waves before kLoad0)
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

    const uint32_t pitch = uint32_t(a.pitch);
    const uint32_t bytes = uint32_t(L::Q) * pitch * St::E + pitch * (St::kRecA + St::kRecB);
    const __amdgpu_buffer_rsrc_t rin = state_rsrc(a.in, bytes);
    const __amdgpu_buffer_rsrc_t rout = state_rsrc(a.out, bytes);
    const uint32_t cs = uint32_t(uniform(int(pitch * St::E)));
    const uint32_t planeE = uint32_t(a.nx) * uint32_t(a.ny) * St::E;
    uint32_t ixy[9], rxy[9];
    col_offsets<St::E>(a, intile ? x : 0, intile ? y : 0, ixy);
    col_offsets<St::E>(a, gx, gy, rxy);
    const uint32_t own = ixy[4];
    uint32_t step = 0;  // seeds the stochastic rounding of FP16 output
    if constexpr (sizeof(S) == 2) step = *a.ctr_in;

    // record loaders: up to kPerLoader nodes of the (tw + 4) x (th + 4) tile
    const int sw = tw + 4, sn = sw * (th + 4);
    uint32_t lcol[kPerLoader];
    int lidx[kPerLoader];
    bool lon[kPerLoader];
#pragma unroll
    for (int k = 0; k < kPerLoader; ++k) {
        const int j = int(threadIdx.x) - kLoad0 + k * kLoaders;
        lon[k] = threadIdx.x >= kLoad0 && j < sn;
        const int sx = lon[k] ? j % sw - 2 : 0, sy = lon[k] ? j / sw - 2 : 0;
        lidx[k] = (sy + 2) * kSW + (sx + 2);
        lcol[k] = uint32_t(wrap_any(x0 + sx, a.nx)) + uint32_t(a.nx) * uint32_t(wrap_any(y0 + sy, a.ny));
    }
    typename St::RawA lq0[kPerLoader];
    typename St::RawB lq1[kPerLoader];

    float *psi_lds = lds;
    float *rec_lds = lds + kPSlots * kPN;
    auto pslot = [&](int zp) { return psi_lds + ((zp - z0 + 1) % kPSlots) * kPN; };
    auto rslot = [&](int q) { return rec_lds + ((q - z0 + 2 * kSSlots) % kSSlots) * (kNS * kSN); };

    auto rec_issue = [&](int q) {
        const uint32_t zq = uint32_t(uniform(wrap_any(q, a.nz))) * (uint32_t(a.nx) * uint32_t(a.ny));
        const uint32_t ra = uint32_t(L::Q) * cs + zq * St::kRecA,
                       rb = uint32_t(L::Q) * cs + pitch * St::kRecA + zq * St::kRecB;
#pragma unroll
        for (int k = 0; k < kPerLoader; ++k)
            if (lon[k]) {
                lq0[k] = St::load_a(rin, lcol[k] * St::kRecA, ra);
                lq1[k] = St::load_b(rin, lcol[k] * St::kRecB, rb);
            }
    };
    auto rec_write = [&](int q) {
        float *s = rslot(q);
#pragma unroll
        for (int k = 0; k < kPerLoader; ++k)
            if (lon[k]) {
                const f4 e = St::entry(lq0[k], lq1[k]);
                if constexpr (ENTRIES) {
                    reinterpret_cast<f4 *>(s)[lidx[k]] = e;
                } else {
                    s[0 * kSN + lidx[k]] = e[0];
                    s[1 * kSN + lidx[k]] = e[1];
                    s[2 * kSN + lidx[k]] = e[2];
                    s[3 * kSN + lidx[k]] = e[3];
                }
                s[4 * kSN + lidx[k]] = St::ratio(lq1[k]);
            }
    };

    // pulled totals of the ring node and of the interior node, as stored
    typename St::Raw rd[L::Q], id[L::Q];
    auto pull = [&](const uint32_t t[9], int zp, typename St::Raw d[L::Q]) {
        uint32_t zo[3];
        z_offsets(wrapz_c(zp, a.nz), a.nz, planeE, zo);
#pragma unroll
        for (int i = 0; i < L::Q; ++i)
            d[i] = St::load(rin, t[(1 - L::cx[i]) + 3 * (1 - L::cy[i])], uint32_t(i) * cs + zo[1 - L::cz[i]]);
    };
    auto ring_issue = [&](int zp) {
        if (has_ring) pull(rxy, zp, rd);
    };
    auto interior_issue = [&](int zp) {
        if (intile) pull(ixy, zp, id);
    };
    auto split = [&](const typename St::Raw raw[L::Q], int zp, int c, CPops<L, T> &q) {
        const float *const sl[3] = {rslot(zp - 1), rslot(zp), rslot(zp + 1)};
        float d[L::Q];
#pragma unroll
        for (int i = 0; i < L::Q; ++i) d[i] = St::df(raw[i], i);
        split_pulled<ENTRIES, kSW, kSN>(d, sl, c, q);
    };
    const int ci = (row + 2) * kSW + lane + 2, cr = (ry + 2) * kSW + rx + 2;
    auto ring_finish = [&](int zp) {
        if (has_ring) {
            CPops<L, T> q;
            split(rd, zp, cr, q);
            T dr, rR, rB;
            densities<L, T>(q, dr, rR, rB);
            pslot(zp)[(ry + 1) * kPW + rx + 1] = float(psi_of<T>(dr, rR, rB));
        }
    };
    auto interior_psi = [&](int zp) {
        if (intile) {
            CPops<L, T> q;
            split(id, zp, ci, q);
            T dr, rR, rB;
            densities<L, T>(q, dr, rR, rB);
            pslot(zp)[(row + 1) * kPW + lane + 1] = float(psi_of<T>(dr, rR, rB));
        }
    };
    auto interior_moments = [&](int zp, T &d, T &r36R, T &r36B, T j[3], T flux[6]) {
        if (intile) {
            CPops<L, T> q;
            split(id, zp, ci, q);
            Mom<T> m;
            moments<L, T>(q, m);
            d = m.drho;
            r36R = m.r36R;
            r36B = m.r36B;
            j[0] = m.j[0];
            j[1] = m.j[1];
            j[2] = m.j[2];
#pragma unroll
            for (int k = 0; k < 6; ++k) flux[k] = m.S[k];
            pslot(zp)[(row + 1) * kPW + lane + 1] = float(psi_of<T>(m.drho, m.r36R, m.r36B));
        }
    };

    // Prologue.  Decoding plane p reads the records of planes p-1..p+1; the
    // loop decodes planes z0+1..z1 and writes record plane z+3 at iteration
    // z into the slot of plane z-1, which no wave reads after the barrier of
    // iteration z-1.
    for (int q = z0 - 2; q <= z0 + 1; ++q) {
        rec_issue(q);
        wait_memory();
        rec_write(q);
    }
    c_lds_barrier();
    ring_issue(z0 - 1);
    interior_issue(z0 - 1);
    wait_memory();
    ring_finish(z0 - 1);
    interior_psi(z0 - 1);
    T cd = 0, cR = 0, cB = 0, cj[3] = {0, 0, 0}, cS[6] = {0, 0, 0, 0, 0, 0};
    ring_issue(z0);
    interior_issue(z0);
    wait_memory();
    ring_finish(z0);
    interior_moments(z0, cd, cR, cB, cj, cS);
    c_lds_barrier();  // plane z0 - 2's slot is free
    rec_issue(z0 + 2);
    wait_memory();
    rec_write(z0 + 2);
    if (z0 + 3 <= z1 + 1) rec_issue(z0 + 3);
    ring_issue(z0 + 1);
    interior_issue(z0 + 1);
    c_lds_barrier();

    for (int z = z0; z < z1; ++z) {
        const bool more = z + 2 <= z1;  // uniform over the block
        T nd = 0, nR = 0, nB = 0, nj[3] = {0, 0, 0}, nS[6] = {0, 0, 0, 0, 0, 0};
        // No wait for all memory operations here: the compiler waits for each
        // loaded register before its use, which does not wait for the stores
        // of the plane before (0.754 -> 0.750 ms per step on 256^3).
        if (z + 3 <= z1 + 1) rec_write(z + 3);
        ring_finish(z + 1);
        interior_moments(z + 1, nd, nR, nB, nj, nS);
        if (more) {
            ring_issue(z + 2);
            interior_issue(z + 2);
        }
        if (z + 4 <= z1 + 1) rec_issue(z + 4);
        c_lds_barrier();
        if (intile) {
            const float *sm = pslot(z - 1), *s0 = pslot(z), *sp = pslot(z + 1);
            const int c = (row + 1) * kPW + lane + 1;
            T fx = 0, fy = 0, fz = 0;
#pragma unroll
            for (int i = 1; i < L::Q; ++i) {
                const float *sl = L::cz[i] > 0 ? sp : (L::cz[i] < 0 ? sm : s0);
                const float pv = sl[c + L::cy[i] * kPW + L::cx[i]];
                const T wp = T(3.0 * wgt<L>(i)) * T(pv);
                if (L::cx[i]) fx += L::cx[i] > 0 ? wp : -wp;
                if (L::cy[i]) fy += L::cy[i] > 0 ? wp : -wp;
                if (L::cz[i]) fz += L::cz[i] > 0 ? wp : -wp;
            }
            const T F[3] = {fx, fy, fz};
            CompactOut<L, T> o;
            collide<L, T>(mo, cd, cR, cB, cj, cS, F, nullptr, o);
            St::store(rout, own, uint32_t(uniform(z)) * (uint32_t(a.nx) * uint32_t(a.ny)), pitch, o, step);
        }
        cd = nd;
        cR = nR;
        cB = nB;
#pragma unroll
        for (int k = 0; k < 3; ++k) cj[k] = nj[k];
#pragma unroll
        for (int k = 0; k < 6; ++k) cS[k] = nS[k];
    }
}

// ------------------------------------------------------------- pair in
// The first step after an initialisation or a restore: pulls (total
// deviation, share) pairs, whose colour split needs no sender scalars.
template <typename S>
struct PendP {
    typename PairOf<S>::type v[D3Q19::Q];
    __device__ __forceinline__ void take(CPops<D3Q19, float> &p) const {
        p.red = 0;
#pragma unroll
        for (int i = 0; i < D3Q19::Q; ++i) {
            bool fl;
            p.df[i] = Codec<S>::template df<D3Q19, float>(v[i].x, i);
            p.mm[i] = Codec<S>::template col<float>(v[i].y, fl);
            p.red |= fl ? (1u << i) : 0u;
            p.vd[i] = 0.0f;
        }
    }
};

template <typename S>
__device__ __forceinline__ void pull_pairs(const CompactArgs &a, __amdgpu_buffer_rsrc_t r, const uint32_t t[9],
                                           int z, PendP<S> &pd) {
    using L = D3Q19;
    typedef typename PairOf<S>::type P;
    const uint32_t plane = uint32_t(a.nx) * uint32_t(a.ny) * uint32_t(sizeof(P));
    const uint32_t cs = uint32_t(uniform(int(uint32_t(a.pitch) * uint32_t(sizeof(P)))));
    uint32_t zo[3];
    z_offsets(z, a.nz, plane, zo);
#pragma unroll
    for (int i = 0; i < L::Q; ++i)
        pd.v[i] = load_pair<P>(r, t[(1 - L::cx[i]) + 3 * (1 - L::cy[i])], uint32_t(su(uint32_t(i) * cs + zo[1 - L::cz[i]])));
}

template <int TX, typename S = float>
__device__ __forceinline__ void sweep_pairs(const CompactArgs &a, const Model<float> &mo, int tile, int chunk,
                                            float *lds) {
    using L = D3Q19;
    typedef float T;
    typedef CStore<S> St;
    constexpr uint32_t PB = sizeof(typename PairOf<S>::type);
    constexpr int kCTX = TX, R = kCR, W = CTile<TX>::PW, PL = CTile<TX>::PN;
    const int lane = threadIdx.x % kCTX, row = threadIdx.x / kCTX;
    const int tx = tile % a.ntx, ty = tile / a.ntx;
    const int x0 = tx * kCTX, y0 = ty * R;
    const int tw = min(kCTX, a.nx - x0), th = min(R, a.ny - y0);
    const int z0 = int((int64_t(chunk) * a.nz) / a.zchunks);
    const int z1 = int((int64_t(chunk + 1) * a.nz) / a.zchunks);
    if (z1 <= z0) return;  // uniform over the block

    const bool intile = lane < tw && row < th;
    const int x = x0 + lane, y = y0 + row;
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

    const uint32_t pitch = uint32_t(a.pitch);
    const __amdgpu_buffer_rsrc_t rin = state_rsrc(a.in, uint32_t(L::Q) * pitch * PB);
    const __amdgpu_buffer_rsrc_t rout = state_rsrc(a.out, uint32_t(L::Q) * pitch * St::E + pitch * (St::kRecA + St::kRecB));
    const uint32_t cs = uint32_t(uniform(int(pitch * St::E)));
    const uint32_t plane = uint32_t(a.nx) * uint32_t(a.ny);
    uint32_t ixy[9], rxy[9], oxy[9];
    col_offsets<PB>(a, intile ? x : 0, intile ? y : 0, ixy);
    col_offsets<PB>(a, gx, gy, rxy);
    col_offsets<St::E>(a, intile ? x : 0, intile ? y : 0, oxy);
    const uint32_t own = oxy[4];
    uint32_t step = 0;  // seeds the stochastic rounding of FP16 output
    if constexpr (sizeof(S) == 2) step = *a.ctr_in;

    auto slot_of = [&](int zp) { return lds + ((zp - z0 + 1) % kPSlots) * PL; };
    PendP<S> rp, pp;
    auto ring_issue = [&](int zp) {
        if (has_ring) pull_pairs(a, rin, rxy, wrapz_c(zp, a.nz), rp);
    };
    auto ring_finish = [&](int zp) {
        if (has_ring) {
            CPops<L, T> q;
            rp.take(q);
            T dr, rR, rB;
            densities<L, T>(q, dr, rR, rB);
            slot_of(zp)[(ry + 1) * W + rx + 1] = float(psi_of<T>(dr, rR, rB));
        }
    };
    auto interior_issue = [&](int zp) {
        if (intile) pull_pairs(a, rin, ixy, wrapz_c(zp, a.nz), pp);
    };
    auto interior_moments = [&](T &d, T &r36R, T &r36B, T j[3], T flux[6]) -> float {
        CPops<L, T> q;
        pp.take(q);
        Mom<T> m;
        moments<L, T>(q, m);
        d = m.drho;
        r36R = m.r36R;
        r36B = m.r36B;
        j[0] = m.j[0];
        j[1] = m.j[1];
        j[2] = m.j[2];
#pragma unroll
        for (int k = 0; k < 6; ++k) flux[k] = m.S[k];
        return float(psi_of<T>(m.drho, m.r36R, m.r36B));
    };

    T cd = 0, cR = 0, cB = 0, cj[3] = {0, 0, 0}, cS[6] = {0, 0, 0, 0, 0, 0};
    ring_issue(z0 - 1);
    interior_issue(z0 - 1);
    if (intile) {
        CPops<L, T> q;
        pp.take(q);
        T dr, rR, rB;
        densities<L, T>(q, dr, rR, rB);
        slot_of(z0 - 1)[(row + 1) * W + lane + 1] = float(psi_of<T>(dr, rR, rB));
    }
    ring_finish(z0 - 1);
    ring_issue(z0);
    interior_issue(z0);
    if (intile) slot_of(z0)[(row + 1) * W + lane + 1] = interior_moments(cd, cR, cB, cj, cS);
    ring_finish(z0);
    ring_issue(z0 + 1);
    interior_issue(z0 + 1);

    for (int z = z0; z < z1; ++z) {
        const bool more = z + 2 <= z1;  // uniform over the block
        T nd = 0, nR = 0, nB = 0, nj[3] = {0, 0, 0}, nS[6] = {0, 0, 0, 0, 0, 0};
        wait_memory();
        ring_finish(z + 1);
        if (intile) slot_of(z + 1)[(row + 1) * W + lane + 1] = interior_moments(nd, nR, nB, nj, nS);
        if (more) {
            ring_issue(z + 2);
            interior_issue(z + 2);
        }
        c_lds_barrier();
        if (intile) {
            const float *sm = slot_of(z - 1), *s0 = slot_of(z), *sp = slot_of(z + 1);
            const int c = (row + 1) * W + lane + 1;
            T fx = 0, fy = 0, fz = 0;
#pragma unroll
            for (int i = 1; i < L::Q; ++i) {
                const float *sl = L::cz[i] > 0 ? sp : (L::cz[i] < 0 ? sm : s0);
                const float pv = sl[c + L::cy[i] * W + L::cx[i]];
                const T wp = T(3.0 * wgt<L>(i)) * T(pv);
                if (L::cx[i]) fx += L::cx[i] > 0 ? wp : -wp;
                if (L::cy[i]) fy += L::cy[i] > 0 ? wp : -wp;
                if (L::cz[i]) fz += L::cz[i] > 0 ? wp : -wp;
            }
            const T F[3] = {fx, fy, fz};
            CompactOut<L, T> o;
            collide<L, T>(mo, cd, cR, cB, cj, cS, F, nullptr, o);
            St::store(rout, own, uint32_t(uniform(z)) * plane, pitch, o, step);
        }
        cd = nd;
        cR = nR;
        cB = nB;
#pragma unroll
        for (int k = 0; k < 3; ++k) cj[k] = nj[k];
#pragma unroll
        for (int k = 0; k < 6; ++k) cS[k] = nS[k];
    }
}

constexpr size_t kCompactLds = CTile<kCTX>::lds;  // the batched sweep's 64 x 8 tiles

// Allows a compact kernel (k = 0, 1: single lattice, FP32, 64 and 32 wide;
// 2: batched; 3, 4: single lattice, FP16, 64 and 32 wide) its LDS beyond
// 64 KiB, once per device and kernel.
void allow_lds(const void *fn, int k, size_t bytes) {
    static std::mutex mu;
    static std::set<std::pair<int, int>> done;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (!done.insert({dev, k}).second) return;
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
    (void)hipGetLastError();
}

}  // namespace

}  // namespace lbcg
