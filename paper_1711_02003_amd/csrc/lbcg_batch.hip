// Batched form of the fused D3Q19 step (pair-state or compact-state sweep):
// many independent lattices advance together, one kernel launch per time level over every lattice that still
// has steps left (two launches when geometry and periodic lattices are
// mixed).  Per lattice the arithmetic is the fused sweep of the single
// lattice form, so each lattice's result is bitwise that of stepping it
// alone.
//
// Work list: every lattice contributes its (tile, z chunk) items; lattices
// are ordered by decreasing step count, so the lattices still running at
// any time level are a prefix of the list and one launch covers them with a
// prefix of the block table.  The kernel deals the prefix to the 8 XCDs in
// contiguous bands.  The items of lattices with the same step count are
// placed so that the bands of a launch over every lattice carry about the
// same work and each band runs its longest items first (z chunks differ by
// up to 2x in planes; on 64 boxes of 32-96 nodes a side this steps 6-7 %
// faster than items placed lattice by lattice).  Runs of
// 32 levels with the same active set are captured into a HIP graph and
// replayed.  The launch shape (rows per tile, z planes per chunk) is chosen
// by timing candidate shapes on the batch itself at creation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <utility>
#include <vector>

#include "lbcg_sim.h"

using namespace lbcg;

namespace {

constexpr int kLevelsPerGraph = 32;
constexpr size_t kGraphCacheMax = 64;
constexpr int kTileX = 64;  // tile width of the fused kernel
constexpr int kMaxPlanes = 1 << 20;

// Both storage types share one descriptor layout.
typedef BatchDesc<float> Desc;
static_assert(sizeof(BatchDesc<float>) == sizeof(BatchDesc<_Float16>), "descriptor layout");

int dev_err(hipError_t e) {
    return e == hipSuccess ? LBCG_OK : (e == hipErrorOutOfMemory ? LBCG_E_NOMEM : LBCG_E_DEVICE);
}

#define HIP_TRY(expr)                                  \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) return dev_err(e_);      \
    } while (0)

}  // namespace

struct lbcg_batch {
    std::vector<lbcg_sim *> sims;
    int prec = 0;
    bool compact = false;  // every lattice on the compact-state kernel
    int rows = 8, zplanes = 32;
    hipStream_t stream = nullptr;
    std::vector<int> zchunks, items;  // per lattice, for the current shape
    int64_t capU = 0, capM = 0;       // table capacity: unmasked / masked groups
    // device and pinned host images of: desc[2][n] | lat/item of group U | lat/item of group M
    void *dmem = nullptr, *hmem = nullptr;
    size_t bytes = 0;
    hipEvent_t staged = nullptr;  // the last staging copy has completed
    bool staged_pending = false;
    std::map<std::pair<int, int>, hipGraphExec_t> graphs;  // (blocks U, blocks M) -> 32 levels
    bool graph_failed = false;

    Desc *desc(void *base, int parity) { return static_cast<Desc *>(base) + size_t(parity) * sims.size(); }
    int *tab(void *base, bool masked, bool item) {
        int *t = reinterpret_cast<int *>(desc(base, 2));
        if (masked) t += 2 * capU;
        return t + (item ? (masked ? capM : capU) : 0);
    }
};

namespace {

bool is_masked(const lbcg_sim *s) { return s->g.mask != nullptr; }

int chunks_for(const lbcg_sim *s, int zplanes) {
    const int64_t z = (int64_t(s->g.nz) + zplanes - 1) / zplanes;
    return int(z < 1 ? 1 : (z > 4096 ? 4096 : z));
}

int64_t items_for(const lbcg_sim *s, int rows, int zc) {
    return int64_t((s->g.nx + kTileX - 1) / kTileX) * ((s->g.ny + rows - 1) / rows) * zc;
}

void set_shape(lbcg_batch *b, int rows, int zplanes) {
    b->rows = rows;
    b->zplanes = zplanes;
    const size_t n = b->sims.size();
    b->zchunks.assign(n, 1);
    b->items.assign(n, 0);
    for (size_t j = 0; j < n; ++j) {
        b->zchunks[j] = chunks_for(b->sims[j], zplanes);
        b->items[j] = int(items_for(b->sims[j], rows, b->zchunks[j]));
    }
}

void drop_graphs(lbcg_batch *b) {
    for (auto &kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    b->graphs.clear();
}

// Work of item i of lattice j in the current shape, in planes: those of
// its z chunk plus the two its sweep pulls first.  A tile that the lattice
// fills only in part takes about as long as a full one (it still steps
// every plane with all its waves): weighting items by their rows or lanes
// measured slower on the 64 boxes.
int64_t item_cost(const lbcg_batch *b, int j, int i) {
    const lbcg_sim *s = b->sims[size_t(j)];
    const int zc = b->zchunks[size_t(j)];
    const int chunk = i % zc;
    const int64_t z0 = int64_t(chunk) * s->g.nz / zc, z1 = int64_t(chunk + 1) * s->g.nz / zc;
    return z1 - z0 + 2;
}

struct Item {
    int64_t cost;
    int lat, item;
};

// Table entries [0, total) of one group (periodic or geometry lattices) for
// the lattices `lats` in table order with step counts `left`.  Each run of
// equal step counts fills its own range of entries (the prefix property).
// Periodic launches deal entries to the XCDs in contiguous bands (the
// kernels' work_index): within a run, items go longest first to the band
// with the least work so far that still has entries in the run's range, and
// each band's entries take its items longest first.  Launches with geometry
// deal consecutive entries to consecutive XCDs, so a run is simply sorted
// longest first.
void place_items(const lbcg_batch *b, const std::vector<int> &lats, const std::vector<int64_t> &left, bool banded,
                 int *lat, int *item) {
    constexpr int kBands = 8;
    int64_t total = 0;
    for (int j : lats) total += b->items[size_t(j)];
    auto band_start = [&](int x) { return int64_t(x) * (total / kBands) + std::min<int64_t>(x, total % kBands); };
    int64_t load[kBands] = {};
    std::vector<Item> run;
    std::vector<int64_t> next(kBands), end(kBands);
    int64_t p = 0;
    for (size_t q = 0; q < lats.size();) {
        size_t r = q;
        run.clear();
        for (; r < lats.size() && left[r] == left[q]; ++r)
            for (int i = 0; i < b->items[size_t(lats[r])]; ++i) run.push_back({item_cost(b, lats[r], i), lats[r], i});
        std::stable_sort(run.begin(), run.end(), [](const Item &u, const Item &v) { return u.cost > v.cost; });
        const int64_t p1 = p + int64_t(run.size());
        if (!banded) {
            for (const Item &it : run) {
                lat[p] = it.lat;
                item[p] = it.item;
                ++p;
            }
        } else {
            // entries [next[x], end[x]) of band x lie in this run's range
            for (int x = 0; x < kBands; ++x) {
                next[x] = std::max(p, band_start(x));
                end[x] = std::min(p1, band_start(x + 1));
            }
            for (const Item &it : run) {
                int pick = -1;
                for (int x = 0; x < kBands; ++x)
                    if (next[x] < end[x] && (pick < 0 || load[x] < load[pick])) pick = x;
                lat[next[pick]] = it.lat;
                item[next[pick]] = it.item;
                ++next[pick];
                load[pick] += it.cost;
            }
            p = p1;
        }
        q = r;
    }
}

// Fill the pinned staging for lattice order `order` (decreasing step count,
// `left` the step counts in that order) and copy it to the device.
// Descriptor parity 0 steps buf[cur] into buf[cur ^ 1], parity 1 the
// reverse.
int stage(lbcg_batch *b, const std::vector<int> &order, const std::vector<int64_t> &left) {
    if (b->staged_pending) {
        HIP_TRY(hipEventSynchronize(b->staged));
        b->staged_pending = false;
    }
    const size_t n = b->sims.size();
    for (int par = 0; par < 2; ++par) {
        Desc *d = b->desc(b->hmem, par);
        for (size_t j = 0; j < n; ++j) {
            const lbcg_sim *s = b->sims[j];
            const FusedShape sh{b->rows, b->zchunks[j]};
            void *const *bufs = b->compact ? s->cbuf : s->buf;
            const void *in = bufs[s->cur ^ par];
            void *out = bufs[s->cur ^ par ^ 1];
            std::memset(&d[j], 0, sizeof(Desc));
            d[j].a = fused_args<float>(s->g, in, out, s->ctr + (s->cur ^ par), s->ctr + (s->cur ^ par ^ 1), sh);
            d[j].mo = to_model<float>(s->md);
        }
    }
    for (int m = 0; m < 2; ++m) {
        std::vector<int> lats;
        std::vector<int64_t> steps;
        for (size_t q = 0; q < order.size(); ++q)
            if (is_masked(b->sims[size_t(order[q])]) == bool(m)) {
                lats.push_back(order[q]);
                steps.push_back(left[q]);
            }
        place_items(b, lats, steps, !m, b->tab(b->hmem, m, false), b->tab(b->hmem, m, true));
    }
    HIP_TRY(hipMemcpyAsync(b->dmem, b->hmem, b->bytes, hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipEventRecord(b->staged, b->stream));
    b->staged_pending = true;
    return LBCG_OK;
}

hipError_t launch_level(lbcg_batch *b, int parity, int nbU, int nbM) {
    if (b->compact)
        return launch_step_compact_batch(b->prec, b->desc(b->dmem, parity), b->tab(b->dmem, false, false),
                                         b->tab(b->dmem, false, true), nbU, b->stream);
    hipError_t e = hipSuccess;
    if (nbU > 0)
        e = launch_step_fused_batch(b->prec, b->desc(b->dmem, parity), b->tab(b->dmem, false, false),
                                    b->tab(b->dmem, false, true), nbU, b->rows, false, b->stream);
    if (e == hipSuccess && nbM > 0)
        e = launch_step_fused_batch(b->prec, b->desc(b->dmem, parity), b->tab(b->dmem, true, false),
                                    b->tab(b->dmem, true, true), nbM, b->rows, true, b->stream);
    return e;
}

hipGraphExec_t graph_for(lbcg_batch *b, int nbU, int nbM) {
    if (b->graph_failed) return nullptr;
    auto it = b->graphs.find({nbU, nbM});
    if (it != b->graphs.end()) return it->second;
    if (b->graphs.size() >= kGraphCacheMax) drop_graphs(b);
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        b->graph_failed = true;
        return nullptr;
    }
    hipError_t e = hipSuccess;
    for (int t = 0; t < kLevelsPerGraph && e == hipSuccess; ++t) e = launch_level(b, t & 1, nbU, nbM);
    hipError_t e2 = hipStreamEndCapture(b->stream, &g);
    hipGraphExec_t exec = nullptr;
    if (e == hipSuccess && e2 == hipSuccess && g) e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess || e2 != hipSuccess || !exec) {
        (void)hipGetLastError();
        b->graph_failed = true;
        return nullptr;
    }
    b->graphs[{nbU, nbM}] = exec;
    return exec;
}

// Time one level over every lattice with the current shape (buf[cur] into
// the other buffer: the lattices' states do not change).
int time_shape(lbcg_batch *b, float *ms) {
    std::vector<int> order(b->sims.size());
    for (size_t j = 0; j < order.size(); ++j) order[j] = int(j);
    int rc = stage(b, order, std::vector<int64_t>(order.size(), 0));
    if (rc) return rc;
    int nbU = 0, nbM = 0;
    for (size_t j = 0; j < order.size(); ++j) (is_masked(b->sims[j]) ? nbM : nbU) += b->items[j];
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    hipError_t e = hipEventCreate(&e1);
    for (int k = 0; k < 2 && e == hipSuccess; ++k) e = launch_level(b, 0, nbU, nbM);
    if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
    for (int k = 0; k < 4 && e == hipSuccess; ++k) e = launch_level(b, 0, nbU, nbM);
    if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return dev_err(e);
}

void destroy(lbcg_batch *b) {
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graphs(b);
    if (b->staged) (void)hipEventDestroy(b->staged);
    if (b->dmem) (void)hipFree(b->dmem);
    if (b->hmem) (void)hipHostFree(b->hmem);
    delete b;
}

}  // namespace

extern "C" {

int lbcg_batch_create(lbcg_sim *const *sims, int32_t n, const int32_t *tile, lbcg_batch **out) {
    if (!sims || n < 1 || !out) return LBCG_E_INVAL;
    const bool tuned = !tile || (tile[0] == 0 && tile[1] == 0);
    if (!tuned && ((tile[0] != 4 && tile[0] != 8) || tile[1] < 1)) return LBCG_E_INVAL;
    for (int j = 0; j < n; ++j) {
        const lbcg_sim *s = sims[j];
        if (!s || !s->initialised || s->lattice != LBCG_D3Q19) return LBCG_E_INVAL;
        if (s->kernel != LBCG_KERNEL_FUSED && s->kernel != LBCG_KERNEL_COMPACT) return LBCG_E_INVAL;
        // the batched sweeps relax with the regularized collision only
        if (s->collision != LBCG_REGULARIZED) return LBCG_E_INVAL;
        // the batched compact sweep: periodic lattices
        if (s->kernel == LBCG_KERNEL_COMPACT && s->g.mask) return LBCG_E_INVAL;
        if (s->kernel != sims[0]->kernel || s->prec != sims[0]->prec || s->stream != sims[0]->stream)
            return LBCG_E_INVAL;
        for (int k = 0; k < j; ++k)
            if (sims[k] == s) return LBCG_E_INVAL;
    }
    lbcg_batch *b = new (std::nothrow) lbcg_batch();
    if (!b) return LBCG_E_NOMEM;
    b->sims.assign(sims, sims + n);
    b->prec = sims[0]->prec;
    b->stream = sims[0]->stream;
    b->compact = sims[0]->kernel == LBCG_KERNEL_COMPACT;
    if (b->compact && !tuned && tile[0] != 8) {  // the compact sweep has 8-row tiles
        delete b;
        return LBCG_E_INVAL;
    }

    // candidate shapes; the tables are sized for the largest
    std::vector<std::pair<int, int>> cand;
    if (tuned) {
        for (int r : {4, 8})
            for (int p : {8, 16, 32, 64, kMaxPlanes})
                if (!b->compact || r == 8) cand.push_back({r, p});
    } else {
        cand.push_back({tile[0], tile[1]});
    }
    for (const auto &c : cand) {
        int64_t u = 0, m = 0;
        for (int j = 0; j < n; ++j)
            (is_masked(sims[j]) ? m : u) += items_for(sims[j], c.first, chunks_for(sims[j], c.second));
        b->capU = std::max(b->capU, u);
        b->capM = std::max(b->capM, m);
    }
    if (b->capU + b->capM > 0x7fffffff) {
        delete b;
        return LBCG_E_INVAL;
    }
    b->bytes = 2 * size_t(n) * sizeof(Desc) + 2 * sizeof(int) * size_t(b->capU + b->capM);
    hipError_t e = hipMalloc(&b->dmem, b->bytes);
    if (e == hipSuccess) e = hipHostMalloc(&b->hmem, b->bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->staged, hipEventDisableTiming);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        destroy(b);
        return dev_err(e);
    }
    if (tuned) {
        float best = 0;
        std::pair<int, int> pick = cand[0];
        for (const auto &c : cand) {
            set_shape(b, c.first, c.second);
            float ms = 0;
            const int rc = time_shape(b, &ms);
            if (rc) {
                destroy(b);
                return rc;
            }
            if (best == 0 || ms < best) {
                best = ms;
                pick = c;
            }
        }
        set_shape(b, pick.first, pick.second);
    } else {
        set_shape(b, tile[0], tile[1]);
    }
    *out = b;
    return LBCG_OK;
}

int lbcg_batch_step(lbcg_batch *b, const int64_t *nsteps) {
    if (!b || !nsteps) return LBCG_E_INVAL;
    const int n = int(b->sims.size());
    std::vector<int64_t> left(nsteps, nsteps + n);
    for (int j = 0; j < n; ++j)
        if (left[j] < 0) return LBCG_E_INVAL;
    // The fused sweep reads post-collision state, and the batched compact
    // sweep a compact one: a lattice fresh from initialisation (or, on the
    // compact kernel, from a restore) takes its first steps alone.
    for (int j = 0; j < n; ++j) {
        lbcg_sim *s = b->sims[j];
        while (left[j] > 0 && (!s->pulled || (b->compact && !s->compact))) {
            const int rc = lbcg_step(s, 1);
            if (rc) return rc;
            --left[j];
        }
    }
    std::vector<int> order;
    for (int j = 0; j < n; ++j)
        if (left[j] > 0) order.push_back(j);
    if (order.empty()) return LBCG_OK;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return left[a] > left[c]; });
    std::vector<int64_t> run_left(order.size());
    for (size_t q = 0; q < order.size(); ++q) run_left[q] = left[size_t(order[q])];
    int rc = stage(b, order, run_left);
    if (rc) return rc;

    // time levels in runs of constant active set: the first k lattices of
    // `order` are active for t < left[order[k - 1]]
    int64_t t = 0;
    int k = int(order.size());
    while (k > 0) {
        const int64_t t1 = left[order[k - 1]];
        int nbU = 0, nbM = 0;
        for (int q = 0; q < k; ++q) (is_masked(b->sims[order[q]]) ? nbM : nbU) += b->items[order[q]];
        while (t < t1) {
            if ((t & 1) == 0 && t1 - t >= kLevelsPerGraph) {
                hipGraphExec_t g = graph_for(b, nbU, nbM);
                if (g) {
                    HIP_TRY(hipGraphLaunch(g, b->stream));
                    t += kLevelsPerGraph;
                    continue;
                }
            }
            HIP_TRY(launch_level(b, int(t & 1), nbU, nbM));
            ++t;
        }
        while (k > 0 && left[order[k - 1]] <= t) --k;
    }
    for (int j : order) {
        lbcg_sim *s = b->sims[j];
        s->cur ^= int(left[j] & 1);
        s->step += left[j];
        s->expanded = false;
    }
    return LBCG_OK;
}

int lbcg_batch_launch_info(lbcg_batch *b, int32_t *rows, int32_t *zplanes, int64_t *blocks) {
    if (!b) return LBCG_E_INVAL;
    if (rows) *rows = b->rows;
    if (zplanes) *zplanes = b->zplanes;
    if (blocks) {
        int64_t t = 0;
        for (int v : b->items) t += v;
        *blocks = t;
    }
    return LBCG_OK;
}

void lbcg_batch_destroy(lbcg_batch *b) {
    if (b) destroy(b);
}

}  // extern "C"
