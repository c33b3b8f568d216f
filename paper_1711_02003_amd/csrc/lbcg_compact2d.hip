// Fused single-pass D2Q9 RCG step on a compact state (arXiv:1711.02003,
// Sec. II, Eqs. (1)-(11)), periodic lattices, FP32.
//
// The 2-D counterpart of the compact D3Q19 sweep: a node stores its 9 new
// total deviations and 4 colour scalars (minority share M with the majority
// flag in its lowest bit, V_axis (x, y) and R_d, with V_diag = R_d V_axis),
// from which the receiver of a population splits it into colours (Eq. (10):
// the minority colour part of f_i is M f_i + (c_i . V_c) / 36 with the
// sender's M and the V of the speed class of c_i).  2 x (9 x 4 + 16) = 104
// bytes per node and step instead of 2 x 18 x 4 = 144.
//
// Layout: 9 arrays of `pitch` floats (total deviation f_i - w_i of direction
// i at i * pitch + node), then `pitch` 16-byte records {M, V_axis x, y, R_d}
// (at float 9 * pitch + 4 n).  The records are read with 16-byte loads and
// written with two 8-byte stores per lane (a wider store may read its data
// registers after the compiler has already reused them).
//
// The sweep is the pair-state strip sweep's: each wave owns 64 columns and
// sweeps a chunk of rows, pulling row y+1 (and, on two lanes, the nodes left
// and right of the strip) one row ahead while row y collides, with psi in a
// 3-row LDS ring of its own.  Decoding row p needs the records of rows p-1,
// p, p+1 over the strip plus two columns each side (the side nodes' own
// senders): each row of records is loaded once (68 nodes, two lanes load a
// second node) two rows ahead of its first use into a 3-row LDS ring of the
// wave's own.  A wave's LDS accesses complete in program order, so a
// wave-scope fence for the compiler replaces a workgroup barrier.  The first
// step after an initialisation or a restore reads the pair state instead.
#include "lbcg_buffer.h"
#include "lbcg_internal.h"

namespace lbcg {

namespace {

constexpr int kS2 = 64;             // columns of a strip (one wave)
constexpr int kW2 = 4;              // strips (work items) per block
constexpr int kP2 = kS2 + 2;        // psi row: the strip and one node each side
constexpr int kR2 = kS2 + 4;        // record row: the strip and two nodes each side
constexpr int kNS2 = 4;             // scalars per record: M, V_axis x, y, R_d
constexpr int kRec2 = 16;           // bytes per record
constexpr int kLds2 = 3 * kP2 + 3 * kNS2 * kR2;  // floats per wave

typedef float f2 __attribute__((ext_vector_type(2)));
typedef unsigned int u2 __attribute__((ext_vector_type(2)));

struct Compact2dArgs {
    const float *in;  // compact state, or pair state (pair_in)
    float *out;       // compact state
    int nx, ny;
    int64_t pitch;
    const uint32_t *ctr_in;
    uint32_t *ctr_out;
    int nstrips, ychunks;
};

// Orders the wave's LDS accesses before and after it for the compiler (the
// hardware completes a wave's LDS accesses in order): lanes read what other
// lanes of the wave wrote.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

__device__ __forceinline__ int wrap2(int a, int n) {
    const int r = a % n;
    return r < 0 ? r + n : r;
}

// Every buffer access takes its wave-uniform byte offset through
// readfirstlane at the point of use (see the D3Q19 compact sweep).
__device__ __forceinline__ int su2(uint32_t v) { return __builtin_amdgcn_readfirstlane(int(v)); }
__device__ __forceinline__ float ld1(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, int(voff), su2(soff), 0));
}
typedef float f4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ f4 ld4(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, int(voff), su2(soff), 0));
}
__device__ __forceinline__ f2 ld2(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(f2, __builtin_amdgcn_raw_buffer_load_b64(r, int(voff), su2(soff), 0));
}

// Split of the 9 pulled totals d of a node with its senders' scalars from the
// LDS record rows sl[0..2] (rows p-1, p, p+1 of the pulled row p) at record
// column c of the node.
__device__ __forceinline__ void split2(const float d[D2Q9::Q], const float *const sl[3], int c,
                                       CPops<D2Q9, float> &p) {
    using L = D2Q9;
    p.red = 0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const int cx = L::cx[i], cy = L::cy[i];
        const float *s = sl[1 - cy];
        const int k = c - cx;
        bool fl;
        p.df[i] = d[i];
        p.mm[i] = Codec<float>::col<float>(s[k], fl);
        p.red |= fl ? (1u << i) : 0u;
        const int n2 = cx * cx + cy * cy;
        if (n2 == 0) {
            p.vd[i] = 0.0f;
        } else if (n2 == 1) {
            const float v = cx ? s[1 * kR2 + k] : s[2 * kR2 + k];
            p.vd[i] = (cx + cy) > 0 ? v : -v;
        } else {
            const float vx = s[1 * kR2 + k], vy = s[2 * kR2 + k];
            const float sx = cx > 0 ? vx : -vx;
            p.vd[i] = s[3 * kR2 + k] * (cy > 0 ? sx + vy : sx - vy);
        }
    }
}

template <bool PAIR_IN>
__device__ __forceinline__ void sweep_c2d(const Compact2dArgs &a, const Model<float> &mo, int strip, int chunk,
                                          float *lds) {
    using L = D2Q9;
    using T = float;
    constexpr uint32_t EI = PAIR_IN ? 8u : 4u;  // bytes per input value
    const int lane = threadIdx.x % kS2;
    const int x0 = strip * kS2, tw = min(kS2, a.nx - x0);
    const int y0 = int((int64_t(chunk) * a.ny) / a.ychunks);
    const int y1 = int((int64_t(chunk + 1) * a.ny) / a.ychunks);
    if (y1 <= y0) return;  // uniform over the wave
    const bool intile = lane < tw;
    const int x = x0 + (intile ? lane : 0);

    // lanes 0 and 1 also pull the node left and right of the strip
    const bool has_ring = lane < 2;
    const int gx = lane == 0 ? wrap_m1(x0 - 1, a.nx) : wrap_m1(x0 + tw, a.nx);
    const int rpos = lane == 0 ? -1 : tw;  // strip column of the ring node
    auto cols = [&](int xx, uint32_t t[3]) {
        t[0] = uint32_t(wrap_m1(xx - 1, a.nx)) * EI;
        t[1] = uint32_t(xx) * EI;
        t[2] = uint32_t(wrap_m1(xx + 1, a.nx)) * EI;
    };
    uint32_t it[3], rt[3];
    cols(x, it);
    cols(gx, rt);
    const uint32_t cs = uint32_t(uniform(int(uint32_t(a.pitch) * EI)));
    const uint32_t row = uint32_t(uniform(int(uint32_t(a.nx) * EI)));
    const uint32_t in_bytes = PAIR_IN ? uint32_t(2 * L::Q) * uint32_t(a.pitch) * 4u
                                      : uint32_t(L::Q) * uint32_t(a.pitch) * 4u + uint32_t(a.pitch) * kRec2;
    const uint32_t out_bytes = uint32_t(L::Q) * uint32_t(a.pitch) * 4u + uint32_t(a.pitch) * kRec2;
    const __amdgpu_buffer_rsrc_t rin = state_rsrc(a.in, in_bytes);
    const __amdgpu_buffer_rsrc_t rout = state_rsrc(a.out, out_bytes);
    const uint32_t cso = uint32_t(uniform(int(uint32_t(a.pitch) * 4u)));
    const uint32_t rowo = uint32_t(uniform(int(uint32_t(a.nx) * 4u)));
    const uint32_t own = uint32_t(x);  // node column (the row adds nx per row)

    float *psi = lds;                // 3 rows of kP2
    float *rec = lds + 3 * kP2;      // 3 rows of kNS2 x kR2
    auto pslot = [&](int yy) { return psi + ((yy - y0 + 3) % 3) * kP2; };
    auto rslot = [&](int yy) { return rec + ((yy - y0 + 6) % 3) * (kNS2 * kR2); };
    auto wrapy = [&](int yy) { return wrap2(yy, a.ny); };

    // record loaders: lane l loads record column l (node x0 - 2 + l) and,
    // for l + 64 < tw + 4, column l + 64
    const int rn = tw + 4;
    const bool lon0 = lane < rn, lon1 = lane + kS2 < rn;
    const uint32_t lc0 = uint32_t(wrap2(x0 - 2 + lane, a.nx)), lc1 = uint32_t(wrap2(x0 - 2 + lane + kS2, a.nx));
    f4 ra0, ra1;
    auto rec_issue = [&](int yy) {
        if (PAIR_IN) return;
        const uint32_t n0 = uint32_t(uniform(wrapy(yy))) * uint32_t(a.nx);
        const uint32_t sa = uint32_t(L::Q) * cso + n0 * kRec2;
        if (lon0) {
            ra0 = ld4(rin, lc0 * kRec2, sa);
        }
        if (lon1) {
            ra1 = ld4(rin, lc1 * kRec2, sa);
        }
    };
    auto rec_write = [&](int yy) {
        if (PAIR_IN) return;
        float *s = rslot(yy);
        if (lon0) {
            s[0 * kR2 + lane] = ra0[0];
            s[1 * kR2 + lane] = ra0[1];
            s[2 * kR2 + lane] = ra0[2];
            s[3 * kR2 + lane] = ra0[3];
        }
        if (lon1) {
            s[0 * kR2 + lane + kS2] = ra1[0];
            s[1 * kR2 + lane + kS2] = ra1[1];
            s[2 * kR2 + lane + kS2] = ra1[2];
            s[3 * kR2 + lane + kS2] = ra1[3];
        }
    };

    // pulled values of the interior and the ring node
    float id[L::Q], rd[L::Q], im[L::Q], rm[L::Q];  // totals and (pair input) shares
    auto pull = [&](const uint32_t t[3], int yy, float d[L::Q], float m[L::Q]) {
        const int yw = wrapy(yy);
        const uint32_t yo[3] = {uint32_t(uniform(yw == 0 ? a.ny - 1 : yw - 1)) * row, uint32_t(uniform(yw)) * row,
                                uint32_t(uniform(yw == a.ny - 1 ? 0 : yw + 1)) * row};
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            const uint32_t so = uint32_t(i) * cs + yo[1 - L::cy[i]];
            if (PAIR_IN) {
                const f2 v = ld2(rin, t[1 - L::cx[i]], so);
                d[i] = v[0];
                m[i] = v[1];
            } else {
                d[i] = ld1(rin, t[1 - L::cx[i]], so);
            }
        }
    };
    auto take = [&](const float d[L::Q], const float m[L::Q], int yy, int c, CPops<L, T> &q) {
        if (PAIR_IN) {
            q.red = 0;
#pragma unroll
            for (int i = 0; i < L::Q; ++i) {
                bool fl;
                q.df[i] = d[i];
                q.mm[i] = Codec<float>::col<float>(m[i], fl);
                q.red |= fl ? (1u << i) : 0u;
                q.vd[i] = 0.0f;
            }
        } else {
            const float *const sl[3] = {rslot(yy - 1), rslot(yy), rslot(yy + 1)};
            split2(d, sl, c, q);
        }
    };
    auto issue = [&](int yy) {
        if (has_ring) pull(rt, yy, rd, rm);
        if (intile) pull(it, yy, id, im);
    };
    auto ring_psi = [&](int yy) {
        if (has_ring) {
            CPops<L, T> q;
            take(rd, rm, yy, rpos + 2, q);
            T dr, rR, rB;
            densities<L, T>(q, dr, rR, rB);
            pslot(yy)[rpos + 1] = float(psi_of<T>(dr, rR, rB));
        }
    };
    auto interior = [&](int yy, T &d, T &r36R, T &r36B, T j[3], T flux[6]) {
        if (intile) {
            CPops<L, T> q;
            take(id, im, yy, lane + 2, q);
            Mom<T> m;
            moments<L, T>(q, m);
            d = m.drho;
            r36R = m.r36R;
            r36B = m.r36B;
#pragma unroll
            for (int k = 0; k < 3; ++k) j[k] = m.j[k];
#pragma unroll
            for (int k = 0; k < 6; ++k) flux[k] = m.S[k];
            pslot(yy)[lane + 1] = float(psi_of<T>(m.drho, m.r36R, m.r36B));
        }
    };

    // prologue: records of rows y0-2 .. y0+1, psi of rows y0-1 and y0,
    // moments of y0, requests of y0+1 and of record row y0+2
    T cd = 0, cR = 0, cB = 0, cj[3] = {0, 0, 0}, cS[6] = {0, 0, 0, 0, 0, 0};
    rec_issue(y0 - 2);
    wait_memory();
    rec_write(y0 - 2);
    rec_issue(y0 - 1);
    wait_memory();
    rec_write(y0 - 1);
    rec_issue(y0);
    issue(y0 - 1);
    wait_memory();
    rec_write(y0);
    wave_sync();
    {
        T d, r, b, j[3], f[6];
        ring_psi(y0 - 1);
        interior(y0 - 1, d, r, b, j, f);
    }
    rec_issue(y0 + 1);
    issue(y0);
    wait_memory();
    wave_sync();
    rec_write(y0 + 1);  // into the slot of row y0 - 2, no longer read
    wave_sync();
    ring_psi(y0);
    interior(y0, cd, cR, cB, cj, cS);
    rec_issue(y0 + 2);
    issue(y0 + 1);

    for (int y = y0; y < y1; ++y) {
        T nd = 0, nR = 0, nB = 0, nj[3] = {0, 0, 0}, nS[6] = {0, 0, 0, 0, 0, 0};
        // row y+1 and record row y+2 were requested one iteration ago
        wait_memory();
        rec_write(y + 2);  // into the slot of row y - 1, no longer read
        wave_sync();
        ring_psi(y + 1);
        interior(y + 1, nd, nR, nB, nj, nS);
        if (y + 2 <= y1) {
            issue(y + 2);
            rec_issue(y + 3);
        }
        wave_sync();
        if (intile) {
            const float *sm = pslot(y - 1), *s0 = pslot(y), *sp = pslot(y + 1);
            const int c = lane + 1;
            T fx = 0, fy = 0;
#pragma unroll
            for (int i = 1; i < L::Q; ++i) {
                const float *sl = L::cy[i] > 0 ? sp : (L::cy[i] < 0 ? sm : s0);
                const float pv = sl[c + L::cx[i]];
                const T wp = T(3.0 * wgt<L>(i)) * T(pv);
                if (L::cx[i]) fx += L::cx[i] > 0 ? wp : -wp;
                if (L::cy[i]) fy += L::cy[i] > 0 ? wp : -wp;
            }
            const T F[3] = {fx, fy, T(0)};
            CompactOut<L, T> o;
            collide<L, T>(mo, cd, cR, cB, cj, cS, F, nullptr, o);
            const uint32_t yo = uint32_t(uniform(y)) * rowo;
#pragma unroll
            for (int i = 0; i < L::Q; ++i) store_pair<float>(rout, own * 4u, uint32_t(su2(uint32_t(i) * cso + yo)), o.df[i]);
            const uint32_t n = uint32_t(uniform(y)) * uint32_t(a.nx) + own;
            const f2 qa = {Codec<float>::enc_col<float>(o.M, o.redmaj), o.Va[0]};
            const f2 qb = {o.Va[1], o.Rd};
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, qa), rout, int(n * kRec2),
                                                  su2(uint32_t(L::Q) * cso), kNonTemporal);
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, qb), rout, int(n * kRec2),
                                                  su2(uint32_t(L::Q) * cso + 8u), kNonTemporal);
        }
        wave_sync();
        cd = nd;
        cR = nR;
        cB = nB;
#pragma unroll
        for (int k = 0; k < 3; ++k) cj[k] = nj[k];
#pragma unroll
        for (int k = 0; k < 6; ++k) cS[k] = nS[k];
    }
}

// kW2 work items per block, numbered chunk-major (neighbouring strips of one
// chunk share a block and an L2).
template <bool PAIR_IN>
__global__ void __launch_bounds__(kS2 * kW2) k_step_compact2d(Compact2dArgs a, Model<float> mo) {
    __shared__ float lds[kW2 * kLds2];
    const int wave = threadIdx.x / kS2;
    const int item = blockIdx.x * kW2 + wave;
    if (item == 0 && threadIdx.x == 0) *a.ctr_out = *a.ctr_in + 1u;
    if (item >= a.nstrips * a.ychunks) return;  // uniform over the wave
    sweep_c2d<PAIR_IN>(a, mo, item % a.nstrips, item / a.nstrips, lds + wave * kLds2);
}

// Pair state of nodes [0, N) from a compact D2Q9 state (see k_expand).
__global__ void k_expand2d(const float *__restrict__ cin, typename PairOf<float>::type *__restrict__ pout,
                           int64_t N, int64_t pitch) {
    using L = D2Q9;
    const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const float *ra = cin + int64_t(L::Q) * pitch + 4 * n;
    bool fl;
    const float M = Codec<float>::col<float>(ra[0], fl);
    const float Va[2] = {ra[1], ra[2]}, Rd = ra[3];
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const float d = cin[int64_t(i) * pitch + n];
        const int n2 = csq<L>(i);
        // the receiver's expression: c_i . V_axis, times R_d for a diagonal
        const float cva = float(L::cx[i]) * Va[0] + float(L::cy[i]) * Va[1];
        const float vd = n2 == 0 ? 0.0f : (n2 == 1 ? cva : Rd * cva);
        const float f = float(wgt<L>(i)) + d;
        const float mu36 = M * (float(w36<L>(i)) + 36.0f * d) + vd;
        const float q = f != 0.0f ? mu36 / (36.0f * f) : 0.0f;
        const bool keep = q <= 0.5f;
        pout[int64_t(i) * pitch + n] = encode_pair<L, float, float>(d, keep ? q : 1.0f - q, keep ? fl : !fl, i);
    }
}

}  // namespace

hipError_t launch_step_compact2d(const Geo &g, const ModelD &md, const void *in, bool pair_in, void *out,
                                 const uint32_t *ctr_in, uint32_t *ctr_out, int ychunks, hipStream_t s) {
    if (g.mask || md.bgk || g.nz != 1) return hipErrorInvalidValue;
    if (uint64_t(2 * D2Q9::Q) * uint64_t(g.pitch) * 4u >= (uint64_t(1) << 32)) return hipErrorInvalidValue;
    Compact2dArgs a;
    a.in = static_cast<const float *>(in);
    a.out = static_cast<float *>(out);
    a.nx = g.nx;
    a.ny = g.ny;
    a.pitch = g.pitch;
    a.ctr_in = ctr_in;
    a.ctr_out = ctr_out;
    a.nstrips = (g.nx + kS2 - 1) / kS2;
    a.ychunks = ychunks < 1 ? 1 : (ychunks > g.ny ? g.ny : ychunks);
    const int64_t items = int64_t(a.nstrips) * a.ychunks;
    const int64_t blocks = (items + kW2 - 1) / kW2;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    const Model<float> mo = to_model<float>(md);
    if (pair_in)
        hipLaunchKernelGGL(k_step_compact2d<true>, dim3(unsigned(blocks)), dim3(kS2 * kW2), 0, s, a, mo);
    else
        hipLaunchKernelGGL(k_step_compact2d<false>, dim3(unsigned(blocks)), dim3(kS2 * kW2), 0, s, a, mo);
    return hipGetLastError();
}

hipError_t launch_expand2d(const Geo &g, const void *cin, void *pout, hipStream_t s) {
    if (g.N <= 0) return hipSuccess;
    const int64_t blocks = (g.N + 255) / 256;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_expand2d, dim3(unsigned(blocks)), dim3(256), 0, s, static_cast<const float *>(cin),
                       static_cast<typename PairOf<float>::type *>(pout), g.N, g.pitch);
    return hipGetLastError();
}

}  // namespace lbcg
