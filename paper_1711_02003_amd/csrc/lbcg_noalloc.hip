// lbcg_batch_step_noalloc: the batched step without a batch object and
// without any allocation, for callers that cannot allocate.
//
// lbcg_batch_step keeps its descriptors and block tables in device memory and
// pinned host staging that lbcg_batch_create allocates.  This entry point
// keeps them in one fixed area of device memory that the library defines at
// file scope (`scratch` below), sized for LBCG_NOALLOC_MAX_LATTICES lattices
// and LBCG_NOALLOC_MAX_BLOCKS blocks per group and time level.  The host never
// copies into it: two small kernels write the descriptors and the block
// tables from their own kernel arguments (which the runtime passes by value),
// so a call queues kernels only - no memory copy, no pinned memory, no graph.
// The level kernels are those of the batched form, so every lattice's result
// is bitwise the one lbcg_batch_step and lbcg_step give.
//
// The area exists once per device and keeps the last call's contents.  Work
// of successive calls on one stream is ordered; calls whose work overlaps on
// one device (different streams) race on the area.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "lbcg_sim.h"

using namespace lbcg;

namespace {

typedef BatchDesc<float> Desc;  // one layout for both storage types (see lbcg_batch.hip)

constexpr int kMaxLat = LBCG_NOALLOC_MAX_LATTICES;
constexpr int kMaxBlocks = LBCG_NOALLOC_MAX_BLOCKS;
constexpr size_t kDescBytes = (2 * size_t(kMaxLat) * sizeof(Desc) + 255) / 256 * 256;
constexpr size_t kTabBytes = 4 * size_t(kMaxBlocks) * sizeof(int);
constexpr size_t kScratchBytes = kDescBytes + kTabBytes;  // ~1.1 MB
constexpr int kDescPerFill = 8;
constexpr int kMaxDevices = 64;
constexpr int kTileX = 64;

// Descriptors of lattices [first, first + count) for both parities
// (parity 0 steps buf[cur] into buf[cur ^ 1], parity 1 the reverse).
struct DescFill {
    Desc d[2][kDescPerFill];
    int first, count;
};
static_assert(sizeof(DescFill) < 4000, "kernel argument size");
static_assert(sizeof(Desc) % 4 == 0, "descriptor copied in 4-byte words");

// One group's block table: entries [start[q], start[q + 1]) are the work
// items of lattice lat[q], q < n.
struct TabFill {
    int n;
    int start[kMaxLat + 1];
    unsigned char lat[kMaxLat];
};
static_assert(sizeof(TabFill) < 4000, "kernel argument size");
static_assert(kMaxLat <= 256, "lattice numbers fit a byte");

}  // namespace

// The fixed area: descriptors [2][kMaxLat], then the unmasked group's lattice
// and item tables, then the masked group's.  Host code reaches it only
// through the address hipGetSymbolAddress gives for the current device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

__global__ void __launch_bounds__(256) k_fill_desc(DescFill f, unsigned char *area) {
    Desc *desc = reinterpret_cast<Desc *>(area);
    constexpr int words = int(sizeof(Desc) / 4);
    const int per = f.count * words;
    for (int k = int(threadIdx.x); k < 2 * per; k += int(blockDim.x)) {
        const int par = k / per, r = k % per, j = r / words, wd = r % words;
        reinterpret_cast<uint32_t *>(&desc[size_t(par) * kMaxLat + f.first + j])[wd] =
            reinterpret_cast<const uint32_t *>(&f.d[par][j])[wd];
    }
}

__global__ void __launch_bounds__(256) k_fill_tab(TabFill t, int total, int *lat_out, int *item_out) {
    const int k = int(blockIdx.x) * 256 + int(threadIdx.x);
    if (k >= total) return;
    int lo = 0, hi = t.n - 1;  // the last q with start[q] <= k
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (t.start[mid] <= k)
            lo = mid;
        else
            hi = mid - 1;
    }
    lat_out[k] = t.lat[lo];
    item_out[k] = k - t.start[lo];
}

std::mutex g_lock;
void *g_area[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device.
int area_of_device(int dev, unsigned char **out) {
    if (dev < 0 || dev >= kMaxDevices) return LBCG_E_DEVICE;
    std::lock_guard<std::mutex> lk(g_lock);
    if (!g_area[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return LBCG_E_DEVICE;
        }
        g_area[dev] = p;
    }
    *out = static_cast<unsigned char *>(g_area[dev]);
    return LBCG_OK;
}

int dev_err(hipError_t e) {
    return e == hipSuccess ? LBCG_OK : (e == hipErrorOutOfMemory ? LBCG_E_NOMEM : LBCG_E_DEVICE);
}

int chunks_for(const lbcg_sim *s, int zplanes) {
    const int64_t z = (int64_t(s->g.nz) + zplanes - 1) / zplanes;
    return int(z < 1 ? 1 : (z > 4096 ? 4096 : z));
}

}  // namespace

extern "C" int lbcg_batch_step_noalloc(lbcg_sim *const *sims, int32_t n, const int32_t *tile,
                                       const int64_t *nsteps) {
    if (!sims || !tile || !nsteps || n < 1) return LBCG_E_INVAL;
    if (n > kMaxLat) return LBCG_E_INVAL;
    const int rows = tile[0], zplanes = tile[1];
    if ((rows != 4 && rows != 8) || zplanes < 1) return LBCG_E_INVAL;
    const lbcg_sim *s0 = sims[0];
    for (int j = 0; j < n; ++j) {
        const lbcg_sim *s = sims[j];
        if (!s || !s->initialised || s->lattice != LBCG_D3Q19) return LBCG_E_INVAL;
        if (s->kernel != LBCG_KERNEL_FUSED && s->kernel != LBCG_KERNEL_COMPACT) return LBCG_E_INVAL;
        // the batched sweeps relax with the regularized collision only
        if (s->collision != LBCG_REGULARIZED) return LBCG_E_INVAL;
        // the batched compact sweep: periodic lattices
        if (s->kernel == LBCG_KERNEL_COMPACT && s->g.mask) return LBCG_E_INVAL;
        if (s->kernel != s0->kernel || s->prec != s0->prec || s->stream != s0->stream || s->device != s0->device)
            return LBCG_E_INVAL;
        if (nsteps[j] < 0) return LBCG_E_INVAL;
        for (int k = 0; k < j; ++k)
            if (sims[k] == s) return LBCG_E_INVAL;
    }
    const bool compact = s0->kernel == LBCG_KERNEL_COMPACT;
    if (compact && rows != 8) return LBCG_E_INVAL;  // the compact sweep has 8-row tiles
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return LBCG_E_DEVICE;
    }
    if (dev != s0->device) return LBCG_E_INVAL;

    // work items per lattice and the size of each group's table (fixed-size
    // arrays: the call allocates nothing, host memory included)
    int zch[kMaxLat], items[kMaxLat];
    int64_t totU = 0, totM = 0;
    for (int j = 0; j < n; ++j) {
        const lbcg_sim *s = sims[j];
        zch[j] = chunks_for(s, zplanes);
        const int64_t it = int64_t((s->g.nx + kTileX - 1) / kTileX) * ((s->g.ny + rows - 1) / rows) * zch[j];
        if (it > kMaxBlocks) return LBCG_E_INVAL;
        items[j] = int(it);
        (s->g.mask ? totM : totU) += it;
    }
    if (totU > kMaxBlocks || totM > kMaxBlocks) return LBCG_E_INVAL;
    unsigned char *area = nullptr;
    int rc = area_of_device(dev, &area);
    if (rc) return rc;
    Desc *desc = reinterpret_cast<Desc *>(area);
    int *latU = reinterpret_cast<int *>(area + kDescBytes), *itemU = latU + kMaxBlocks;
    int *latM = itemU + kMaxBlocks, *itemM = latM + kMaxBlocks;

    // A lattice fresh from initialisation (or, on the compact kernel, from a
    // restore) takes its first steps alone, as in lbcg_batch_step (single
    // launches: no graph, no allocation).
    int64_t left[kMaxLat];
    for (int j = 0; j < n; ++j) {
        lbcg_sim *s = sims[j];
        left[j] = nsteps[j];
        while (left[j] > 0 && (!s->pulled || (compact && !s->compact))) {
            rc = lbcg_step(s, 1);
            if (rc) return rc;
            --left[j];
        }
    }
    int order[kMaxLat];
    int k = 0;
    for (int j = 0; j < n; ++j)
        if (left[j] > 0) order[k++] = j;
    if (k == 0) return LBCG_OK;
    // decreasing step count; among equal counts, lattices with geometry
    // (whose blocks go to the XCDs in table order) by decreasing planes per
    // z chunk, so that the longest work items start first, and the others in
    // handle order (a stable insertion sort: the library's sorts may take a
    // temporary buffer from the heap)
    int planes[kMaxLat];
    for (int j = 0; j < n; ++j) planes[j] = sims[j]->g.mask ? (sims[j]->g.nz + zch[j] - 1) / zch[j] : 0;
    auto before = [&](int u, int v) { return left[u] > left[v] || (left[u] == left[v] && planes[u] > planes[v]); };
    for (int q = 1; q < k; ++q) {
        const int v = order[q];
        int p = q;
        for (; p > 0 && before(v, order[p - 1]); --p) order[p] = order[p - 1];
        order[p] = v;
    }
    const hipStream_t st = s0->stream;

    // descriptors of every lattice, in chunks of kDescPerFill per launch
    for (int first = 0; first < n; first += kDescPerFill) {
        DescFill f;
        f.first = first;
        f.count = std::min(kDescPerFill, n - first);
        for (int par = 0; par < 2; ++par)
            for (int q = 0; q < f.count; ++q) {
                const lbcg_sim *s = sims[first + q];
                void *const *bufs = compact ? s->cbuf : s->buf;
                const FusedShape sh{rows, zch[first + q]};
                Desc &d = f.d[par][q];
                d = Desc{};
                d.a = fused_args<float>(s->g, bufs[s->cur ^ par], bufs[s->cur ^ par ^ 1], s->ctr + (s->cur ^ par),
                                        s->ctr + (s->cur ^ par ^ 1), sh);
                d.mo = to_model<float>(s->md);
            }
        hipLaunchKernelGGL(k_fill_desc, dim3(1), dim3(256), 0, st, f, area);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return dev_err(e);
    }
    // block tables: each group lists its lattices in `order`, so the lattices
    // still running at a level are a prefix of it
    for (int masked = 0; masked < 2; ++masked) {
        TabFill t;
        t.n = 0;
        int tot = 0;
        for (int q = 0; q < k; ++q) {
            const int j = order[q];
            if ((sims[j]->g.mask != nullptr) != bool(masked)) continue;
            t.lat[t.n] = static_cast<unsigned char>(j);
            t.start[t.n] = tot;
            tot += items[j];
            ++t.n;
        }
        t.start[t.n] = tot;
        if (tot == 0) continue;
        hipLaunchKernelGGL(k_fill_tab, dim3(unsigned((tot + 255) / 256)), dim3(256), 0, st, t, tot,
                           masked ? latM : latU, masked ? itemM : itemU);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return dev_err(e);
    }

    // time levels in runs of a constant active set: the first a lattices of
    // `order` are active for t < left[order[a - 1]]
    int64_t t = 0;
    int a = k;
    while (a > 0) {
        const int64_t t1 = left[order[a - 1]];
        int nbU = 0, nbM = 0;
        for (int q = 0; q < a; ++q) (sims[order[q]]->g.mask ? nbM : nbU) += items[order[q]];
        for (; t < t1; ++t) {
            const int par = int(t & 1);
            hipError_t e = hipSuccess;
            if (compact) {
                e = launch_step_compact_batch(s0->prec, desc + size_t(par) * kMaxLat, latU, itemU, nbU, st);
            } else {
                if (nbU > 0)
                    e = launch_step_fused_batch(s0->prec, desc + size_t(par) * kMaxLat, latU, itemU, nbU, rows, false,
                                                st);
                if (e == hipSuccess && nbM > 0)
                    e = launch_step_fused_batch(s0->prec, desc + size_t(par) * kMaxLat, latM, itemM, nbM, rows, true,
                                                st);
            }
            if (e != hipSuccess) return dev_err(e);
        }
        while (a > 0 && left[order[a - 1]] <= t) --a;
    }
    for (int q = 0; q < k; ++q) {
        lbcg_sim *s = sims[order[q]];
        s->cur ^= int(left[order[q]] & 1);
        s->step += left[order[q]];
        s->expanded = false;
    }
    return LBCG_OK;
}
