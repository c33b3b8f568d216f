// C-ABI runtime of the RCG lattice Boltzmann library: parameter checks, the
// device memory plan, the step loop (generic two-pass or fused single-pass
// kernel, replayed from HIP graphs), field/population export, diagnostics
// and checkpointing.  The arithmetic lives in the kernels; this file only
// moves data and launches work.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/lbcg.h"
#include "lbcg_sim.h"

using namespace lbcg;

namespace {

constexpr size_t kAlign = 256;
constexpr int64_t kStagingMax = int64_t(1) << 18;  // nodes per staging chunk
constexpr int kGraphSteps = 32;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Plan {
    int Q;
    int64_t N, pitch, staging_nodes;
    size_t elem, tsize, state, cstate, psi, moms, mask, links, inl, outl, wall, partials, diag, ctr, staging, total;
};

int validate(const lbcg_params *p) {
    if (!p) return LBCG_E_INVAL;
    if (p->lattice != LBCG_D2Q9 && p->lattice != LBCG_D3Q19) return LBCG_E_INVAL;
    if (p->precision < LBCG_F64 || p->precision > LBCG_F16) return LBCG_E_INVAL;
    if (p->collision != LBCG_REGULARIZED && p->collision != LBCG_BGK && p->collision != LBCG_BGK_COLOUR)
        return LBCG_E_INVAL;
    if (p->kernel < LBCG_KERNEL_AUTO || p->kernel > LBCG_KERNEL_COMPACT) return LBCG_E_INVAL;
    for (int a = 0; a < 3; ++a)
        if (p->dims[a] < 1 || p->dims[a] > (int64_t(1) << 20)) return LBCG_E_INVAL;
    if (p->lattice == LBCG_D2Q9 && p->dims[2] != 1) return LBCG_E_INVAL;
    const int64_t N = p->dims[0] * p->dims[1] * p->dims[2];
    if (N > (int64_t(1) << 34)) return LBCG_E_INVAL;
    if (!(p->tau_R > 0.5) || !(p->tau_B > 0.5) || !std::isfinite(p->tau_R) || !std::isfinite(p->tau_B))
        return LBCG_E_INVAL;
    if (!std::isfinite(p->A_R) || !std::isfinite(p->A_B) || !std::isfinite(p->beta)) return LBCG_E_INVAL;
    if (p->beta < 0.0 || p->beta > 1.0) return LBCG_E_INVAL;
    if (p->alpha_R < 0.0 || p->alpha_R >= 1.0 || p->alpha_B < 0.0 || p->alpha_B >= 1.0) return LBCG_E_INVAL;
    if (p->n_inlets < 0 || p->n_inlets > LBCG_WALL0 - LBCG_INLET0 || p->n_outlets < 0 || p->n_outlets > 128 ||
        p->n_walls < 0 || p->n_walls > LBCG_OUTLET0 - LBCG_WALL0)
        return LBCG_E_INVAL;
    if (p->n_inlets > 0 && !p->inlets) return LBCG_E_INVAL;
    if (p->n_outlets > 0 && !p->outlets) return LBCG_E_INVAL;
    if (p->n_walls > 0 && !p->walls) return LBCG_E_INVAL;
    for (int j = 0; j < p->n_walls; ++j)
        if (!(p->walls[j].psi >= -1.0 && p->walls[j].psi <= 1.0)) return LBCG_E_INVAL;
    for (int j = 0; j < p->n_inlets; ++j) {
        const lbcg_inlet &in = p->inlets[j];
        if (!(in.rho_R >= 0.0) || !(in.rho_B >= 0.0) || !(in.rho_R + in.rho_B > 0.0)) return LBCG_E_INVAL;
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(in.u[a])) return LBCG_E_INVAL;
        if (p->lattice == LBCG_D2Q9 && in.u[2] != 0.0) return LBCG_E_INVAL;
    }
    for (int j = 0; j < p->n_outlets; ++j)
        if (!(p->outlets[j].rho > 0.0) || !std::isfinite(p->outlets[j].rho)) return LBCG_E_INVAL;
    if (p->mask) {
        for (int64_t n = 0; n < N; ++n) {
            const int m = p->mask[n];
            if (m >= LBCG_INLET0 && m < LBCG_WALL0 && m - LBCG_INLET0 >= p->n_inlets) return LBCG_E_INVAL;
            if (m >= LBCG_WALL0 && m < LBCG_OUTLET0 && m - LBCG_WALL0 >= p->n_walls) return LBCG_E_INVAL;
            if (m >= LBCG_OUTLET0 && m - LBCG_OUTLET0 >= p->n_outlets) return LBCG_E_INVAL;
        }
    }
    if (p->tile[0] < 0 || p->tile[1] < 0) return LBCG_E_INVAL;
    if (p->tile[0] != 0 && p->tile[0] != 4 && p->tile[0] != 8) return LBCG_E_INVAL;
    if (p->kernel == LBCG_KERNEL_COMPACT && p->tile[0] == 4) return LBCG_E_INVAL;  // 8-row tiles only
    // the compact state with geometry runs the split step only
    if (p->kernel == LBCG_KERNEL_COMPACT && p->mask && (p->tile[0] || p->tile[1] || p->tile[2])) return LBCG_E_INVAL;
    // plain BGK on the fused D3Q19 sweep: 8-row tiles only
    if (p->collision != LBCG_REGULARIZED && p->lattice == LBCG_D3Q19 && p->precision != LBCG_F64 &&
        p->tile[0] == 4 && p->kernel != LBCG_KERNEL_GENERIC)
        return LBCG_E_INVAL;
    if (p->tile[1] > 4096) return LBCG_E_INVAL;
    // tile width: 64, or 32 on the compact D3Q19 sweep; 0 = automatic
    if (p->tile[2] != 0 && p->tile[2] != 64 &&
        !(p->tile[2] == 32 && p->kernel == LBCG_KERNEL_COMPACT && p->lattice == LBCG_D3Q19))
        return LBCG_E_INVAL;
    return LBCG_OK;
}

Plan make_plan(const lbcg_params *p) {
    Plan pl{};
    pl.Q = p->lattice == LBCG_D2Q9 ? 9 : 19;
    pl.N = p->dims[0] * p->dims[1] * p->dims[2];
    pl.pitch = int64_t(align_up(size_t(pl.N), 64));
    pl.elem = p->precision == LBCG_F64 ? 8 : (p->precision == LBCG_F32 ? 4 : 2);
    pl.tsize = p->precision == LBCG_F64 ? 8 : 4;
    pl.staging_nodes = pl.N < kStagingMax ? pl.N : kStagingMax;
    const int per = 2 * pl.Q > 6 ? 2 * pl.Q : 6;
    pl.state = align_up(size_t(2 * pl.Q) * size_t(pl.pitch) * pl.elem, kAlign);
    pl.cstate = p->kernel == LBCG_KERNEL_COMPACT
                    ? align_up(size_t(p->lattice == LBCG_D2Q9 ? kCompactBytes2d
                                                                  : (p->precision == LBCG_F16 ? kCompactBytes16 : kCompactBytes)) *
                                   size_t(pl.pitch),
                               kAlign)
                    : 0;
    pl.psi = align_up(size_t(pl.pitch) * pl.tsize, kAlign);
    // the split geometry step's moments: D3Q19 with a mask, F32 or F16,
    // regularized collision
    pl.moms = p->mask && p->lattice == LBCG_D3Q19 && p->precision != LBCG_F64 && p->collision == LBCG_REGULARIZED &&
                      (p->kernel == LBCG_KERNEL_AUTO || p->kernel == LBCG_KERNEL_FUSED ||
                       p->kernel == LBCG_KERNEL_COMPACT)
                  ? align_up(split_scratch_bytes(pl.pitch, p->dims[0], p->dims[1], p->dims[2]), kAlign)
                  : 0;
    pl.mask = p->mask ? align_up(size_t(pl.pitch), kAlign) : 0;
    pl.links = p->mask ? align_up(sizeof(uint32_t) * size_t(pl.pitch), kAlign) : 0;
    pl.inl = align_up(sizeof(DevInlet) * size_t(p->n_inlets > 0 ? p->n_inlets : 1), kAlign);
    pl.outl = align_up(sizeof(DevOutlet) * size_t(p->n_outlets > 0 ? p->n_outlets : 1), kAlign);
    pl.wall = align_up(sizeof(DevWall) * size_t(p->n_walls > 0 ? p->n_walls : 1), kAlign);
    pl.partials = align_up(sizeof(double) * kDiagBlocks * kDiagVals, kAlign);
    pl.diag = align_up(sizeof(double) * 16, kAlign);
    pl.ctr = kAlign;
    pl.staging = align_up(sizeof(double) * size_t(per) * size_t(pl.staging_nodes), kAlign);
    pl.total = 2 * pl.state + 2 * pl.cstate + pl.psi + pl.moms + pl.mask + pl.links + pl.inl + pl.outl + pl.wall + pl.partials +
               pl.diag + pl.ctr + pl.staging + kAlign;
    return pl;
}

int dev_err(hipError_t e) { return e == hipSuccess ? LBCG_OK : (e == hipErrorOutOfMemory ? LBCG_E_NOMEM : LBCG_E_DEVICE); }

#define HIP_TRY(expr)                          \
    do {                                       \
        hipError_t e_ = (expr);                \
        if (e_ != hipSuccess) return dev_err(e_); \
    } while (0)

int check_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LBCG_E_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return LBCG_E_DEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return LBCG_E_DEVICE;
    return LBCG_OK;
}

// The fused kernel of a lattice: the D3Q19 column sweep or the D2Q9 strip
// sweep (periodic lattices only).
bool any_fused_supported(int lattice, int prec, const Geo &g) {
    return lattice == LBCG_D3Q19 ? fused_supported(lattice, prec, g) : fused2d_supported(prec, g);
}

hipError_t launch_fused(const lbcg_sim *s, const void *in, void *out, const uint32_t *ctr_in, uint32_t *ctr_out,
                        FusedShape shape) {
    if (shape.rows == 0)
        return launch_step_split(s->prec, s->g, s->md, in, out, s->psi, s->moms, s->split, ctr_in, ctr_out,
                                 s->stream);
    if (s->lattice == LBCG_D2Q9)
        return launch_step_fused2d(s->prec, s->g, s->md, in, out, ctr_in, ctr_out, shape.zchunks, s->stream);
    return launch_step_fused(s->prec, s->g, s->md, in, out, ctr_in, ctr_out, shape, s->stream);
}

// The compact-state sweep of the lattice: D3Q19 column sweep or D2Q9 strip
// sweep (shape.zchunks counts row chunks there).
hipError_t launch_compact(const lbcg_sim *s, const void *in, bool pair_in, void *out, const uint32_t *ctr_in,
                          uint32_t *ctr_out, FusedShape shape) {
    if (s->lattice == LBCG_D2Q9)
        return launch_step_compact2d(s->g, s->md, in, pair_in, out, ctr_in, ctr_out, shape.zchunks, s->stream);
    return launch_step_compact(s->prec, s->g, s->md, in, pair_in, out, ctr_in, ctr_out, shape, s->stream);
}

FusedShape pick_shape(const lbcg_sim *s, const lbcg_params *p) {
    FusedShape sh;
    if (s->lattice == LBCG_D2Q9) {
        // strips of 64 columns, rows split into chunks (zchunks counts them):
        // about 4096 strip chunks fill the device with 4 waves per SIMD, and
        // chunks keep >= 8 rows; with geometry, chunks of 16 rows (the fluid
        // of a channel then still spreads over the device)
        sh.rows = 1;
        int yc = p->tile[1];
        if (!yc && (s->kernel == LBCG_KERNEL_FUSED || s->kernel == LBCG_KERNEL_COMPACT)) {
            const int64_t strips = (s->g.nx + 63) / 64;
            const int64_t want = s->g.mask ? (s->g.ny + 15) / 16 : (4096 + strips - 1) / strips;
            const int64_t cap = s->g.ny / 8 > 1 ? s->g.ny / 8 : 1;
            yc = int(want < 1 ? 1 : (want > cap ? cap : want));
        }
        sh.zchunks = yc < 1 ? 1 : yc;
        return sh;
    }
    if (s->kernel == LBCG_KERNEL_COMPACT && s->g.mask) {
        sh.rows = 0;  // the compact state with geometry: the split step
        sh.zchunks = 1;
        return sh;
    }
    if (s->kernel == LBCG_KERNEL_FUSED && s->moms && !p->tile[0] && !p->tile[1] && p->mask) {
        // With geometry, the split step when at most half the nodes are
        // fluid: the fluid then fills few column tiles, which the sweep can
        // spread over the device only in short z chunks.
        int64_t fluid = 0;
        for (int64_t n = 0; n < s->g.N; ++n) fluid += p->mask[n] == kFluid ? 1 : 0;
        if (2 * fluid <= s->g.N) {
            sh.rows = 0;
            sh.zchunks = 1;
            return sh;
        }
    }
    sh.rows = p->tile[0] ? p->tile[0] : 8;
    sh.tx = p->tile[2] ? p->tile[2] : 64;
    int zc = p->tile[1];
    if (!zc && (s->kernel == LBCG_KERNEL_FUSED || s->kernel == LBCG_KERNEL_COMPACT)) {
        // One wave of resident blocks: each z chunk re-reads two planes, so use
        // as few (long) chunks as fill the device, but keep chunks >= 8 planes.
        const int64_t tiles = int64_t((s->g.nx + sh.tx - 1) / sh.tx) * ((s->g.ny + sh.rows - 1) / sh.rows);
        const int64_t resident = s->kernel == LBCG_KERNEL_COMPACT
                                     ? compact_resident_blocks(sh.tx, s->prec)
                                     : fused_resident_blocks(s->prec, sh.rows, s->g.mask != nullptr,
                                                             s->collision != LBCG_REGULARIZED);
        int64_t want = (resident + tiles - 1) / tiles;
        const int64_t cap = s->g.nz / 8 > 1 ? s->g.nz / 8 : 1;
        zc = int(want < 1 ? 1 : (want > cap ? cap : want));
    }
    sh.zchunks = zc < 1 ? 1 : zc;
    return sh;
}

// One time step from buf[cur] into buf[cur ^ 1].
// With the compact kernel, a pulled step reads cbuf[cur] (or, right after an
// initialisation or a restore, the pair state in buf[cur]) and writes
// cbuf[cur ^ 1].
hipError_t enqueue_step(lbcg_sim *s, bool pulled) {
    const void *in = s->buf[s->cur];
    void *out = s->buf[s->cur ^ 1];
    const uint32_t *ctr_in = s->ctr + s->cur;
    uint32_t *ctr_out = s->ctr + (s->cur ^ 1);
    if (s->kernel == LBCG_KERNEL_COMPACT && pulled) {
        const bool pair_in = !s->compact;
        hipError_t e =
            s->g.mask ? launch_step_cgeo(s->prec, s->g, s->md, pair_in, pair_in ? s->buf[s->cur] : s->cbuf[s->cur],
                                         s->buf[s->cur], s->cbuf[s->cur ^ 1], s->buf[s->cur ^ 1], s->psi, s->moms,
                                         s->split, ctr_in, ctr_out, s->stream)
                      : launch_compact(s, pair_in ? s->buf[s->cur] : s->cbuf[s->cur], pair_in, s->cbuf[s->cur ^ 1],
                                       ctr_in, ctr_out, s->shape);
        if (e == hipSuccess) {
            s->compact = true;
            s->expanded = false;
        }
        return e;
    }
    if (s->kernel == LBCG_KERNEL_FUSED && pulled) return launch_fused(s, in, out, ctr_in, ctr_out, s->shape);
    hipError_t e = launch_psi(s->lattice, s->prec, s->g, s->md, in, pulled, s->psi, s->stream);
    if (e != hipSuccess) return e;
    return launch_step_generic(s->lattice, s->prec, s->g, s->md, in, pulled, s->psi, out, ctr_in, ctr_out,
                               s->stream);
}

// Capture kGraphSteps pulled steps starting from buffer `start` (even count,
// so the graph leaves the state in the buffer it started from).
bool build_graph(lbcg_sim *s, int start) {
    if (s->graph_failed || s->stream == nullptr) return false;
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        s->graph_failed = true;
        return false;
    }
    const int saved = s->cur;
    s->cur = start;
    hipError_t e = hipSuccess;
    for (int k = 0; k < kGraphSteps && e == hipSuccess; ++k) {
        e = enqueue_step(s, true);
        s->cur ^= 1;
    }
    s->cur = saved;
    hipError_t e2 = hipStreamEndCapture(s->stream, &graph);
    if (e != hipSuccess || e2 != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        s->graph_failed = true;
        return false;
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        s->graph_failed = true;
        return false;
    }
    s->graph[start] = exec;
    return true;
}

// Link words of a lattice with geometry (encoding in lbcg_device.h).
template <class L>
std::vector<uint32_t> link_words(int nx, int ny, int nz, const uint8_t *mask) {
    std::vector<uint32_t> out(size_t(nx) * ny * nz, 0u);
    auto wrap = [](int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); };
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const size_t n = size_t(x) + size_t(nx) * (size_t(y) + size_t(ny) * z);
                if (mask[n] != kFluid) {
                    out[n] = uint32_t(mask[n]) << 20;
                    continue;
                }
                // the code of the non-fluid upstream nodes, walls included:
                // one code for all of them, or "mixed"
                uint32_t lk = kLinkFluid;
                int code = -1;
                for (int i = 1; i < L::Q; ++i) {
                    const size_t m = size_t(wrap(x - L::cx[i], nx)) +
                                     size_t(nx) * (size_t(wrap(y - L::cy[i], ny)) + size_t(ny) * wrap(z - L::cz[i], nz));
                    const uint8_t c = mask[m];
                    if (c == kFluid) continue;
                    lk |= 1u << i;
                    if (code < 0)
                        code = c;
                    else if (code != c)
                        lk |= kLinkMixed;
                    if (c >= kOutlet0) lk |= kLinkOutlet;
                }
                if (code >= 0 && !(lk & kLinkMixed)) lk |= uint32_t(code) << 20;
                out[n] = lk;
            }
    return out;
}

void release(lbcg_sim *s) {
    for (int k = 0; k < 2; ++k)
        if (s->graph[k]) (void)hipGraphExecDestroy(s->graph[k]);
    if (s->own_arena && s->arena) (void)hipFree(s->arena);
    if (s->owned_stream) (void)hipStreamDestroy(s->owned_stream);
}

}  // namespace

extern "C" {

const char *lbcg_strerror(int status) {
    switch (status) {
        case LBCG_OK: return "ok";
        case LBCG_E_INVAL: return "invalid argument";
        case LBCG_E_NOMEM: return "out of device memory or buffer too small";
        case LBCG_E_DEVICE: return "HIP runtime error or no gfx950 device";
        case LBCG_E_UNSTABLE: return "non-finite values in the state";
        case LBCG_E_STATE: return "call out of order";
        default: return "unknown status";
    }
}

int lbcg_footprint(const lbcg_params *p, size_t *bytes) {
    if (!bytes) return LBCG_E_INVAL;
    int rc = validate(p);
    if (rc) return rc;
    *bytes = make_plan(p).total;
    return LBCG_OK;
}

int lbcg_create(const lbcg_params *p, void *dev_buf, size_t bytes, void *hip_stream, lbcg_sim **out) {
    if (!out) return LBCG_E_INVAL;
    int rc = validate(p);
    if (rc) return rc;
    rc = check_device();
    if (rc) return rc;
    const Plan pl = make_plan(p);
    if (dev_buf && bytes < pl.total) return LBCG_E_NOMEM;

    lbcg_sim *s = new (std::nothrow) lbcg_sim();
    if (!s) return LBCG_E_NOMEM;
    if (hipGetDevice(&s->device) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return LBCG_E_DEVICE;
    }
    s->lattice = p->lattice;
    s->prec = p->precision;
    s->collision = p->collision;
    s->Q = pl.Q;
    s->D = p->lattice == LBCG_D2Q9 ? 2 : 3;
    s->elem = pl.elem;
    s->g.nx = int(p->dims[0]);
    s->g.ny = int(p->dims[1]);
    s->g.nz = int(p->dims[2]);
    s->g.N = pl.N;
    s->g.pitch = pl.pitch;
    const double w0 = p->lattice == LBCG_D2Q9 ? 4.0 / 9.0 : 1.0 / 3.0;
    s->md.ivR = 3.0 / (p->tau_R - 0.5);  // 1/nu_k, nu_k = c_s^2 (tau_k - 1/2)
    s->md.ivB = 3.0 / (p->tau_B - 0.5);
    s->md.Abar = 0.5 * (p->A_R + p->A_B);
    s->md.beta = p->beta;
    s->md.aR = p->alpha_R > 0.0 ? p->alpha_R : w0;
    s->md.aB = p->alpha_B > 0.0 ? p->alpha_B : w0;
    s->md.eps_F = p->eps_F < 0.0 ? 1e-8 : p->eps_F;
    s->md.w0 = w0;
    s->md.omR = 1.0 / p->tau_R;
    s->md.omB = 1.0 / p->tau_B;
    s->md.bgk = p->collision == LBCG_BGK ? 1 : (p->collision == LBCG_BGK_COLOUR ? 2 : 0);

    if (dev_buf) {
        s->arena = dev_buf;
        s->own_arena = false;
    } else {
        hipError_t e = hipMalloc(&s->arena, pl.total);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            delete s;
            return dev_err(e);
        }
        s->own_arena = true;
    }
    s->arena_bytes = pl.total;
    char *base = reinterpret_cast<char *>(align_up(reinterpret_cast<size_t>(s->arena), kAlign));
    s->buf[0] = base;
    base += pl.state;
    s->buf[1] = base;
    base += pl.state;
    s->cbuf[0] = pl.cstate ? base : nullptr;
    base += pl.cstate;
    s->cbuf[1] = pl.cstate ? base : nullptr;
    base += pl.cstate;
    s->psi = base;
    base += pl.psi;
    s->moms = pl.moms ? base : nullptr;
    base += pl.moms;
    s->mask_dev = p->mask ? reinterpret_cast<uint8_t *>(base) : nullptr;
    base += pl.mask;
    uint32_t *links_dev = pl.links ? reinterpret_cast<uint32_t *>(base) : nullptr;
    base += pl.links;
    s->in_dev = reinterpret_cast<DevInlet *>(base);
    base += pl.inl;
    s->out_dev = reinterpret_cast<DevOutlet *>(base);
    base += pl.outl;
    DevWall *wall_dev = reinterpret_cast<DevWall *>(base);
    base += pl.wall;
    s->partials = reinterpret_cast<double *>(base);
    base += pl.partials;
    s->diag = reinterpret_cast<double *>(base);
    base += pl.diag;
    s->ctr = reinterpret_cast<uint32_t *>(base);
    base += pl.ctr;
    s->staging = reinterpret_cast<double *>(base);
    s->staging_nodes = pl.staging_nodes;
    s->state_bytes = pl.state;

    s->owned_stream = nullptr;
    if (hip_stream) {
        s->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        if (hipStreamCreateWithFlags(&s->owned_stream, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            s->owned_stream = nullptr;
            release(s);
            delete s;
            return LBCG_E_DEVICE;
        }
        s->stream = s->owned_stream;
    }

    s->g.mask = s->mask_dev;
    s->g.inlets = s->in_dev;
    s->g.outlets = s->out_dev;
    s->g.walls = wall_dev;
    s->g.links = links_dev;
    std::vector<DevInlet> ins(size_t(p->n_inlets > 0 ? p->n_inlets : 1));
    for (int j = 0; j < p->n_inlets; ++j) {
        for (int a = 0; a < 3; ++a) ins[j].u[a] = p->inlets[j].u[a];
        ins[j].rhoR = p->inlets[j].rho_R;
        ins[j].rhoB = p->inlets[j].rho_B;
    }
    std::vector<DevOutlet> outs(size_t(p->n_outlets > 0 ? p->n_outlets : 1));
    for (int j = 0; j < p->n_outlets; ++j) outs[j].rho = p->outlets[j].rho;
    std::vector<DevWall> wls(size_t(p->n_walls > 0 ? p->n_walls : 1), DevWall{0.0});
    for (int j = 0; j < p->n_walls; ++j) wls[j].psi = p->walls[j].psi;
    hipError_t e = hipMemcpyAsync(s->in_dev, ins.data(), sizeof(DevInlet) * ins.size(), hipMemcpyHostToDevice,
                                  s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->out_dev, outs.data(), sizeof(DevOutlet) * outs.size(), hipMemcpyHostToDevice,
                           s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(wall_dev, wls.data(), sizeof(DevWall) * wls.size(), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess && p->mask)
        e = hipMemcpyAsync(s->mask_dev, p->mask, size_t(pl.N), hipMemcpyHostToDevice, s->stream);
    std::vector<uint32_t> links;
    if (e == hipSuccess && links_dev) {
        links = s->lattice == LBCG_D3Q19 ? link_words<D3Q19>(s->g.nx, s->g.ny, s->g.nz, p->mask)
                                         : link_words<D2Q9>(s->g.nx, s->g.ny, s->g.nz, p->mask);
        e = hipMemcpyAsync(links_dev, links.data(), sizeof(uint32_t) * links.size(), hipMemcpyHostToDevice,
                           s->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    s->split = SplitPlan{};
    if (e == hipSuccess && s->moms) e = split_prepare(s->g, s->moms, s->split, s->stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        release(s);
        delete s;
        return dev_err(e);
    }

    // plain BGK runs on the D3Q19 column sweep and the D2Q9 strip sweep
    // (not the split step or the compact state)
    const bool fused_ok = any_fused_supported(s->lattice, s->prec, s->g);
    int kind = p->kernel;
    if (kind == LBCG_KERNEL_AUTO) kind = fused_ok ? LBCG_KERNEL_FUSED : LBCG_KERNEL_GENERIC;
    if ((kind == LBCG_KERNEL_FUSED && !fused_ok) ||
        (kind == LBCG_KERNEL_COMPACT &&
         (!compact_supported(s->lattice, s->prec, s->g) || s->collision != LBCG_REGULARIZED))) {
        release(s);
        delete s;
        return LBCG_E_INVAL;
    }
    s->kernel = kind;
    s->shape = pick_shape(s, p);
    s->cur = 0;
    s->compact = false;
    s->expanded = false;
    s->pulled = false;
    s->initialised = false;
    s->step = 0;
    s->graph_steps = kGraphSteps;
    *out = s;
    return LBCG_OK;
}

int lbcg_init_fields(lbcg_sim *s, const double *rhoR, const double *rhoB, const double *u) {
    if (!s || !rhoR || !rhoB) return LBCG_E_INVAL;
    const int64_t N = s->g.N, C = s->staging_nodes;
    for (int64_t n0 = 0; n0 < N; n0 += C) {
        const int64_t cnt = (N - n0) < C ? (N - n0) : C;
        double *sR = s->staging, *sB = s->staging + cnt, *sU = u ? s->staging + 2 * cnt : nullptr;
        HIP_TRY(hipMemcpyAsync(sR, rhoR + n0, sizeof(double) * cnt, hipMemcpyHostToDevice, s->stream));
        HIP_TRY(hipMemcpyAsync(sB, rhoB + n0, sizeof(double) * cnt, hipMemcpyHostToDevice, s->stream));
        if (u)
            for (int a = 0; a < 3; ++a)
                HIP_TRY(hipMemcpyAsync(sU + a * cnt, u + a * N + n0, sizeof(double) * cnt, hipMemcpyHostToDevice,
                                       s->stream));
        HIP_TRY(launch_init(s->lattice, s->prec, s->g, s->md, n0, cnt, sR, sB, sU, s->buf[0], s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
    }
    HIP_TRY(hipMemsetAsync(s->ctr, 0, 2 * sizeof(uint32_t), s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->cur = 0;
    s->compact = false;
    s->pulled = false;
    s->initialised = true;
    s->step = 0;
    return LBCG_OK;
}

int lbcg_step(lbcg_sim *s, int64_t n) {
    if (!s || n < 0) return LBCG_E_INVAL;
    if (!s->initialised) return LBCG_E_STATE;
    while (n > 0) {
        if (!s->pulled) {
            HIP_TRY(enqueue_step(s, false));
            s->cur ^= 1;
            s->pulled = true;
            --n;
            ++s->step;
            continue;
        }
        if (n >= kGraphSteps && !s->graph_failed && (s->kernel != LBCG_KERNEL_COMPACT || s->compact)) {
            if (!s->graph[s->cur] && !build_graph(s, s->cur)) continue;
            HIP_TRY(hipGraphLaunch(s->graph[s->cur], s->stream));
            s->expanded = false;
            n -= kGraphSteps;
            s->step += kGraphSteps;
            continue;
        }
        HIP_TRY(enqueue_step(s, true));
        s->cur ^= 1;
        --n;
        ++s->step;
    }
    return LBCG_OK;
}

// Pair state of a compact state in buf[cur], for the calls that read the
// state (the compact state itself stays the one the next step reads).
static hipError_t ensure_pairs(lbcg_sim *s) {
    if (!s->compact || s->expanded) return hipSuccess;
    hipError_t e = s->lattice == LBCG_D2Q9 ? launch_expand2d(s->g, s->cbuf[s->cur], s->buf[s->cur], s->stream)
                   : s->g.mask           ? launch_expand_cgeo(s->prec, s->g, s->cbuf[s->cur], s->buf[s->cur], s->moms,
                                                              s->split, s->stream)
                                         : launch_expand(s->prec, s->g, s->cbuf[s->cur], s->buf[s->cur], s->stream);
    if (e == hipSuccess) s->expanded = true;
    return e;
}

int lbcg_set_stream(lbcg_sim *s, void *hip_stream) {
    if (!s) return LBCG_E_INVAL;
    if (hip_stream) {
        s->stream = static_cast<hipStream_t>(hip_stream);
        return LBCG_OK;
    }
    if (!s->owned_stream) return LBCG_E_INVAL;
    s->stream = s->owned_stream;
    return LBCG_OK;
}

int lbcg_synchronize(lbcg_sim *s) {
    if (!s) return LBCG_E_INVAL;
    HIP_TRY(hipStreamSynchronize(s->stream));
    return LBCG_OK;
}

int lbcg_fields(lbcg_sim *s, double *rhoR, double *rhoB, double *u, double *psi) {
    if (!s) return LBCG_E_INVAL;
    if (!s->initialised) return LBCG_E_STATE;
    HIP_TRY(ensure_pairs(s));
    const int64_t N = s->g.N, C = s->staging_nodes;
    for (int64_t n0 = 0; n0 < N; n0 += C) {
        const int64_t cnt = (N - n0) < C ? (N - n0) : C;
        HIP_TRY(launch_fields(s->lattice, s->prec, s->g, s->md, s->buf[s->cur], s->pulled, n0, cnt, s->staging,
                              s->stream));
        const size_t b = sizeof(double) * size_t(cnt);
        if (rhoR) HIP_TRY(hipMemcpyAsync(rhoR + n0, s->staging, b, hipMemcpyDeviceToHost, s->stream));
        if (rhoB) HIP_TRY(hipMemcpyAsync(rhoB + n0, s->staging + cnt, b, hipMemcpyDeviceToHost, s->stream));
        if (u)
            for (int a = 0; a < 3; ++a)
                HIP_TRY(hipMemcpyAsync(u + a * N + n0, s->staging + (2 + a) * cnt, b, hipMemcpyDeviceToHost,
                                       s->stream));
        if (psi) HIP_TRY(hipMemcpyAsync(psi + n0, s->staging + 5 * cnt, b, hipMemcpyDeviceToHost, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
    }
    return LBCG_OK;
}

int lbcg_populations(lbcg_sim *s, double *f) {
    if (!s || !f) return LBCG_E_INVAL;
    if (!s->initialised) return LBCG_E_STATE;
    HIP_TRY(ensure_pairs(s));
    const int64_t N = s->g.N, C = s->staging_nodes;
    for (int64_t n0 = 0; n0 < N; n0 += C) {
        const int64_t cnt = (N - n0) < C ? (N - n0) : C;
        HIP_TRY(launch_pops(s->lattice, s->prec, s->g, s->md, s->buf[s->cur], s->pulled, n0, cnt, s->staging,
                            s->stream));
        for (int c = 0; c < 2 * s->Q; ++c)
            HIP_TRY(hipMemcpyAsync(f + int64_t(c) * N + n0, s->staging + int64_t(c) * cnt,
                                   sizeof(double) * size_t(cnt), hipMemcpyDeviceToHost, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
    }
    return LBCG_OK;
}

int lbcg_populations_at(lbcg_sim *s, const int64_t *nodes, int64_t count, double *f) {
    if (!s || count < 0 || (count > 0 && (!nodes || !f))) return LBCG_E_INVAL;
    if (!s->initialised) return LBCG_E_STATE;
    for (int64_t j = 0; j < count; ++j)
        if (nodes[j] < 0 || nodes[j] >= s->g.N) return LBCG_E_INVAL;
    HIP_TRY(ensure_pairs(s));
    // staging holds per-chunk outputs (2Q doubles per node) followed by the
    // chunk's node indices
    const int64_t per = 2 * s->Q;
    const int64_t C = (s->staging_nodes * (per > 6 ? per : 6)) / (per + 1);
    double *outd = s->staging;
    int64_t *idx = reinterpret_cast<int64_t *>(s->staging + C * per);
    for (int64_t j0 = 0; j0 < count; j0 += C) {
        const int64_t cnt = (count - j0) < C ? (count - j0) : C;
        HIP_TRY(hipMemcpyAsync(idx, nodes + j0, sizeof(int64_t) * size_t(cnt), hipMemcpyHostToDevice, s->stream));
        HIP_TRY(launch_pops_at(s->lattice, s->prec, s->g, s->md, s->buf[s->cur], s->pulled, idx, cnt, outd,
                               s->stream));
        HIP_TRY(hipMemcpyAsync(f + j0 * per, outd, sizeof(double) * size_t(cnt * per), hipMemcpyDeviceToHost,
                               s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
    }
    return LBCG_OK;
}

int lbcg_diagnostics(lbcg_sim *s, lbcg_diag *out) {
    if (!s || !out) return LBCG_E_INVAL;
    if (!s->initialised) return LBCG_E_STATE;
    HIP_TRY(ensure_pairs(s));
    HIP_TRY(launch_diag(s->lattice, s->prec, s->g, s->md, s->buf[s->cur], s->pulled, s->partials, s->diag,
                        s->stream));
    double r[kDiagVals];
    HIP_TRY(hipMemcpyAsync(r, s->diag, sizeof(r), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    lbcg_diag d;
    std::memset(&d, 0, sizeof(d));
    d.mass_R = r[0];
    d.mass_B = r[1];
    d.momentum[0] = r[2];
    d.momentum[1] = r[3];
    d.momentum[2] = r[4];
    d.max_u = r[5];
    d.n_in = int64_t(r[7]);
    d.n_out = int64_t(r[9]);
    d.p_in = r[7] > 0 ? r[6] / r[7] : 0.0;
    d.p_out = r[9] > 0 ? r[8] / r[9] : 0.0;
    d.vol_R = r[10];
    d.R_eff = s->D == 2 ? std::sqrt(r[10] / M_PI) : std::cbrt(3.0 * r[10] / (4.0 * M_PI));
    d.nonfinite = int64_t(r[11]);
    d.fluid_nodes = int64_t(r[12]);
    d.step = s->step;
    *out = d;
    return d.nonfinite ? LBCG_E_UNSTABLE : LBCG_OK;
}

// Checkpoint layout: 8 int64 header words, then Q arrays of N (df, m) value pairs.
static const int64_t kMagic = 0x4c42434731LL;  // "LBCG1"

int lbcg_state_bytes(lbcg_sim *s, size_t *bytes) {
    if (!s || !bytes) return LBCG_E_INVAL;
    *bytes = 8 * sizeof(int64_t) + size_t(2 * s->Q) * size_t(s->g.N) * s->elem;
    return LBCG_OK;
}

int lbcg_get_state(lbcg_sim *s, void *host, size_t bytes) {
    size_t need = 0;
    if (!host) return LBCG_E_INVAL;
    int rc = lbcg_state_bytes(s, &need);
    if (rc) return rc;
    if (bytes < need) return LBCG_E_NOMEM;
    if (!s->initialised) return LBCG_E_STATE;
    HIP_TRY(ensure_pairs(s));
    int64_t *h = static_cast<int64_t *>(host);
    h[0] = kMagic;
    h[1] = s->lattice;
    h[2] = s->prec;
    h[3] = s->g.nx;
    h[4] = s->g.ny;
    h[5] = s->g.nz;
    h[6] = s->pulled ? 1 : 0;
    h[7] = s->step;
    char *dst = reinterpret_cast<char *>(h + 8);
    // one array of (df, m) pairs per direction
    const size_t comp = 2 * size_t(s->g.N) * s->elem;
    const char *src = static_cast<const char *>(s->buf[s->cur]);
    for (int c = 0; c < s->Q; ++c)
        HIP_TRY(hipMemcpyAsync(dst + c * comp, src + 2 * size_t(c) * size_t(s->g.pitch) * s->elem, comp,
                               hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return LBCG_OK;
}

int lbcg_set_state(lbcg_sim *s, const void *host, size_t bytes) {
    size_t need = 0;
    if (!host) return LBCG_E_INVAL;
    int rc = lbcg_state_bytes(s, &need);
    if (rc) return rc;
    if (bytes < need) return LBCG_E_INVAL;
    const int64_t *h = static_cast<const int64_t *>(host);
    if (h[0] != kMagic || h[1] != s->lattice || h[2] != s->prec || h[3] != s->g.nx || h[4] != s->g.ny ||
        h[5] != s->g.nz || (h[6] != 0 && h[6] != 1) || h[7] < 0)
        return LBCG_E_INVAL;
    const char *src = reinterpret_cast<const char *>(h + 8);
    const size_t comp = 2 * size_t(s->g.N) * s->elem;
    char *dst = static_cast<char *>(s->buf[s->cur]);
    for (int c = 0; c < s->Q; ++c)
        HIP_TRY(hipMemcpyAsync(dst + 2 * size_t(c) * size_t(s->g.pitch) * s->elem, src + c * comp, comp,
                               hipMemcpyHostToDevice, s->stream));
    const uint32_t ctr = uint32_t(h[7]);  // the step counter continues from the saved step
    HIP_TRY(hipMemcpyAsync(s->ctr + s->cur, &ctr, sizeof(ctr), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->pulled = h[6] == 1;
    s->step = h[7];
    s->compact = false;
    s->initialised = true;
    return LBCG_OK;
}

int lbcg_launch_info(lbcg_sim *s, int32_t *kernel, int32_t *rows, int32_t *zchunks, int32_t *tile_width) {
    if (!s) return LBCG_E_INVAL;
    if (kernel) *kernel = s->kernel;
    if (rows) *rows = s->shape.rows;
    if (zchunks) *zchunks = s->shape.zchunks;
    if (tile_width) *tile_width = s->lattice == LBCG_D3Q19 ? s->shape.tx : 64;
    return LBCG_OK;
}

int lbcg_tune(lbcg_sim *s, int32_t *rows, int32_t *zchunks) {
    if (!s) return LBCG_E_INVAL;
    if (!s->initialised) return LBCG_E_STATE;
    if (s->kernel == LBCG_KERNEL_COMPACT && s->g.mask) {
        // the compact state with geometry has one launch shape: the split step
        if (rows) *rows = s->shape.rows;
        if (zchunks) *zchunks = s->shape.zchunks;
        return LBCG_OK;
    }
    if (s->kernel == LBCG_KERNEL_FUSED || s->kernel == LBCG_KERNEL_COMPACT) {
        const bool cmp = s->kernel == LBCG_KERNEL_COMPACT;
        // Candidate shapes: both tile heights, z splits that fill the device
        // once, twice or four times, and fixed chunk lengths (short chunks
        // balance lattices whose fluid sits in a few tiles).  Each is timed
        // stepping buf[cur] into the other buffer, which leaves the current
        // state untouched.
        const bool masked = s->g.mask != nullptr;
        std::vector<FusedShape> cand;
        if (s->lattice == LBCG_D2Q9) {
            // strip sweep: row chunks of 8 to 512 rows
            for (int len : {8, 16, 32, 64, 128, 256, 512}) {
                const int yc = (s->g.ny + len - 1) / len;
                bool seen = false;
                for (const FusedShape &c : cand) seen = seen || c.zchunks == yc;
                if (!seen) cand.push_back(FusedShape{1, yc});
            }
        }
        // D3Q19: rows 4 or 8 with 64-wide tiles, and with geometry the split
        // step (rows 0); the compact sweep: 8 rows, 64- or 32-wide tiles
        if (s->lattice == LBCG_D3Q19 && !cmp && s->moms) cand.push_back(FusedShape{0, 1, 64});
        const int shapes[3][2] = {{4, 64}, {8, 64}, {8, 32}};
        for (const auto &rt : shapes) {
            const int r = rt[0], tx = rt[1];
            if (s->lattice == LBCG_D2Q9) break;
            if (cmp ? r != 8 : tx != 64) continue;
            const int64_t tiles = int64_t((s->g.nx + tx - 1) / tx) * ((s->g.ny + r - 1) / r);
            if (s->collision != LBCG_REGULARIZED && r != 8) continue;  // plain BGK: 8-row tiles
            const int64_t resident = cmp ? compact_resident_blocks(tx, s->prec)
                                         : fused_resident_blocks(s->prec, r, masked, s->collision != LBCG_REGULARIZED);
            std::vector<int64_t> zs = {1};
            for (int m : {1, 2, 4}) zs.push_back((m * resident + tiles - 1) / tiles);
            for (int planes : {2, 4, 8, 16, 32, 64}) zs.push_back((s->g.nz + planes - 1) / planes);
            for (int64_t z : zs) {
                const int zc = int(z < 1 ? 1 : (z > s->g.nz ? s->g.nz : (z > 4096 ? 4096 : z)));
                bool seen = false;
                for (const FusedShape &c : cand) seen = seen || (c.rows == r && c.zchunks == zc && c.tx == tx);
                if (!seen) cand.push_back(FusedShape{r, zc, tx});
            }
        }
        // The compact kernel is timed as every later step runs it: reading a
        // compact state.  Before the handle's first compact step (the state is
        // still the pair state in buf[cur]) one first-step launch converts the
        // state into the spare compact buffer cbuf[cur ^ 1], and the candidates
        // step that copy into cbuf[cur], which the handle does not use until its
        // own first compact step writes it.  Either way the current state is
        // left as it is.  The counter slot written is the one the next step
        // writes too.
        const uint32_t *ctr_in = s->ctr + s->cur;
        uint32_t *ctr_out = s->ctr + (s->cur ^ 1);
        const void *in = s->buf[s->cur];
        void *out = s->buf[s->cur ^ 1];
        if (cmp) {
            in = s->cbuf[s->cur];
            out = s->cbuf[s->cur ^ 1];
            if (!s->compact) {
                HIP_TRY(launch_compact(s, s->buf[s->cur], true, s->cbuf[s->cur ^ 1], ctr_in, ctr_out, s->shape));
                in = s->cbuf[s->cur ^ 1];
                out = s->cbuf[s->cur];
            }
        }
        hipEvent_t e0 = nullptr, e1 = nullptr;
        HIP_TRY(hipEventCreate(&e0));
        if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            return LBCG_E_DEVICE;
        }
        auto run = [&](const FusedShape &c) {
            return cmp ? launch_compact(s, in, false, out, ctr_in, ctr_out, c)
                       : launch_fused(s, in, out, ctr_in, ctr_out, c);
        };
        // Two passes over the candidates, each keeping its faster time: in a
        // single pass the first candidates ran while the clocks were still
        // rising, and a 7 % faster D2Q9 shape lost to a slower one about
        // half the time.
        std::vector<float> best_ms(cand.size(), 0.0f);
        hipError_t e = hipSuccess;
        for (int pass = 0; pass < 2 && e == hipSuccess; ++pass) {
            for (size_t ci = 0; ci < cand.size(); ++ci) {
                const FusedShape &c = cand[ci];
                for (int k = 0; k < 2 && e == hipSuccess; ++k) e = run(c);
                if (e == hipSuccess) e = hipEventRecord(e0, s->stream);
                for (int k = 0; k < 4 && e == hipSuccess; ++k) e = run(c);
                if (e == hipSuccess) e = hipEventRecord(e1, s->stream);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) break;
                if (best_ms[ci] == 0 || ms < best_ms[ci]) best_ms[ci] = ms;
            }
        }
        FusedShape pick = s->shape;
        float best = 0;
        for (size_t ci = 0; ci < cand.size() && e == hipSuccess; ++ci)
            if (best == 0 || best_ms[ci] < best) {
                best = best_ms[ci];
                pick = cand[ci];
            }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (e != hipSuccess) return dev_err(e);
        if (pick.rows != s->shape.rows || pick.zchunks != s->shape.zchunks || pick.tx != s->shape.tx) {
            for (int k = 0; k < 2; ++k)
                if (s->graph[k]) {
                    (void)hipGraphExecDestroy(s->graph[k]);
                    s->graph[k] = nullptr;
                }
            s->shape = pick;
        }
    }
    if (rows) *rows = s->shape.rows;
    if (zchunks) *zchunks = s->shape.zchunks;
    return LBCG_OK;
}

void lbcg_destroy(lbcg_sim *s) {
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    release(s);
    delete s;
}

}  // extern "C"
