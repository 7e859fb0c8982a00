// Host implementation of the C ABI declared in include/lbm.h.
//
// A handle owns the device state of one lattice: two population buffers
// (ping-pong), the cell words, the logical type map and small reduction
// buffers.  Every call validates its arguments, issues its device work on the
// handle's stream and returns a status; no exception crosses the interface.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_internal.h"
#include "lbm_tiles.h"

using namespace lbm;

namespace {

thread_local std::string g_error;

int fail(int code, const std::string &msg) {
    g_error = msg;
    return code;
}

struct HipFail {
    hipError_t e;
    const char *what;
};

#define HIP_TRY(expr)                                         \
    do {                                                      \
        hipError_t e_ = (expr);                               \
        if (e_ != hipSuccess) throw HipFail{e_, #expr};       \
    } while (0)

// Recycled allocations.  hipMalloc and hipFree (and their pinned-host
// counterparts) cost tens of microseconds each, and a server creates and
// destroys a lattice's buffers for every request.  A destroyed handle, whose
// stream has been synchronised first, hands its blocks to this cache, and
// allocations take a cached block of their size class on the same device.
// Sizes are rounded up to a multiple of 1/8 of their power of two (at most
// 12.5 % slack).  At most `cap` bytes wait; the oldest blocks are freed first.
class BlockCache {
  public:
    BlockCache(bool host, size_t cap) : host_(host), cap_(cap) {}
    static size_t size_class(size_t n) {
        if (n <= 4096) return (n + 255) / 256 * 256;
        size_t p = 4096;
        while (p * 2 <= n) p *= 2;
        const size_t step = p / 8;
        return (n + step - 1) / step * step;
    }
    // A block of exactly `cls` bytes on `dev` (-1 for host), or nullptr.
    void *take(int dev, size_t cls) {
        std::lock_guard<std::mutex> g(m_);
        for (auto it = blocks_.begin(); it != blocks_.end(); ++it)
            if (it->dev == dev && it->cls == cls) {
                void *p = it->p;
                total_ -= cls;
                blocks_.erase(it);
                return p;
            }
        return nullptr;
    }
    void give(int dev, size_t cls, void *p) {
        std::lock_guard<std::mutex> g(m_);
        blocks_.push_back({dev, cls, p});
        total_ += cls;
        while (total_ > cap_ && !blocks_.empty()) {
            const Block b = blocks_.front();
            blocks_.pop_front();
            total_ -= b.cls;
            release(b);
        }
    }

  private:
    struct Block {
        int dev;
        size_t cls;
        void *p;
    };
    void release(const Block &b) {
        if (host_) {
            (void)hipHostFree(b.p);
        } else {
            int cur = 0;
            (void)hipGetDevice(&cur);
            (void)hipSetDevice(b.dev);
            (void)hipFree(b.p);
            (void)hipSetDevice(cur);
        }
    }
    bool host_;
    size_t cap_;
    std::mutex m_;
    std::deque<Block> blocks_;
    size_t total_ = 0;
};
// Never destroyed: blocks cached at process exit are left to the runtime.
BlockCache &device_cache() {
    static BlockCache *c = new BlockCache(false, (size_t)4 << 30);
    return *c;
}
BlockCache &host_cache() {
    static BlockCache *c = new BlockCache(true, (size_t)64 << 20);
    return *c;
}

// Pinned host memory of at least `bytes`, from the cache when possible;
// `got` receives the size class actually held.
void *pinned_alloc(size_t bytes, size_t &got) {
    got = BlockCache::size_class(bytes);
    if (void *p = host_cache().take(-1, got)) return p;
    void *p = nullptr;
    const hipError_t e = hipHostMalloc(&p, got, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw std::bad_alloc();
    }
    return p;
}

struct DeviceBuffer {
    void *p = nullptr;
    size_t bytes = 0;
    int dev = 0;
    void reset() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    // Hand the block to the cache; only when no queued work still uses it.
    void recycle() {
        if (p) device_cache().give(dev, bytes, p);
        p = nullptr;
        bytes = 0;
    }
    // Grow to at least `n` bytes (contents are not preserved).
    void ensure(size_t n) {
        if (bytes >= n) return;
        reset();
        if (n == 0) return;
        const size_t cls = BlockCache::size_class(n);
        (void)hipGetDevice(&dev);
        p = device_cache().take(dev, cls);
        if (!p) {
            hipError_t e = hipMalloc(&p, cls);
            if (e != hipSuccess) {
                p = nullptr;
                (void)hipGetLastError();
                throw std::bad_alloc();
            }
        }
        bytes = cls;
    }
    template <typename U>
    U *as() const {
        return static_cast<U *>(p);
    }
    ~DeviceBuffer() { reset(); }
};

int pitch_for(int nx) { return (nx + 63) / 64 * 64; }

size_t elem_size(int precision) {
    switch (precision) {
        case LBM_F64: return sizeof(double);
        case LBM_F32: return sizeof(float);
        default: return 2;  // 16-bit storage forms
    }
}

// Call f with a value of the storage type of `precision`.
template <class F>
decltype(auto) with_storage(int precision, F &&f) {
    switch (precision) {
        case LBM_F64: return f(double{});
        case LBM_F32: return f(float{});
        case LBM_F32_S_F16: return f(h16{});
        default: return f(bf16{});
    }
}

// Flat arborescent distributor: the same construction as the input
// generator used by the tests (branch centres floor((2j+1) ny / 2^(k+1)),
// junction columns round((k+1) nx / (L+1)) with ties to even, level-k bars
// w_k rows wide, connectors w_{k+1} columns wide at each junction).
bool generate_distributor(const lbm_geometry_desc &d, std::vector<uint8_t> &t,
                          std::string &why) {
    const int nx = d.nx, ny = d.ny, L = d.levels;
    if (L < 1 || L > 8) {
        why = "levels must be in 1..8";
        return false;
    }
    int w[9];
    bool all_zero = true;
    for (int k = 0; k <= L; ++k) all_zero &= d.widths[k] == 0;
    for (int k = 0; k <= L; ++k)
        w[k] = all_zero ? std::max(2, (ny / 8) >> k) : d.widths[k];
    for (int k = 0; k <= L; ++k)
        if (w[k] < 2) {
            why = "generator widths must be >= 2";
            return false;
        }
    if (ny / (1 << L) < w[L] + 2) {
        why = "outlet channels do not fit: ny/2^L < w_L + 2";
        return false;
    }
    t.assign((size_t)nx * ny, (uint8_t)LBM_SOLID);
    std::vector<int> xj(L + 1);
    for (int k = 0; k < L; ++k)
        xj[k] = (int)std::nearbyint((double)(k + 1) * nx / (double)(L + 1));
    xj[L] = nx;
    auto yc = [&](int k, int j) { return ((2 * j + 1) * ny) / (1 << (k + 1)); };
    auto fill = [&](int y0, int y1, int x0, int x1) {  // half-open ranges
        y0 = std::max(y0, 0);
        y1 = std::min(y1, ny);
        x0 = std::max(x0, 0);
        x1 = std::min(x1, nx);
        for (int y = y0; y < y1; ++y)
            for (int x = x0; x < x1; ++x) t[(size_t)y * nx + x] = LBM_FLUID;
    };
    for (int k = 0; k <= L; ++k) {
        const int xs = k == 0 ? 0 : xj[k - 1], xe = xj[k];
        for (int j = 0; j < (1 << k); ++j) {
            const int r0 = yc(k, j) - w[k] / 2;
            fill(r0, r0 + w[k], xs, xe);
        }
        if (k < L) {
            const int wc = w[k + 1], c0 = xj[k] - wc / 2;
            for (int j = 0; j < (1 << k); ++j) {
                const int ya = yc(k + 1, 2 * j) - wc / 2;
                const int yb = yc(k + 1, 2 * j + 1) - wc / 2 + wc;
                fill(ya, yb, c0, c0 + wc);
            }
        }
    }
    for (int x = 0; x < nx; ++x) {
        t[x] = LBM_SOLID;
        t[(size_t)(ny - 1) * nx + x] = LBM_SOLID;
    }
    for (int y = 0; y < ny; ++y) {
        uint8_t &a = t[(size_t)y * nx];
        if (a != LBM_SOLID) a = LBM_INLET;
        uint8_t &b = t[(size_t)y * nx + nx - 1];
        if (b != LBM_SOLID) b = LBM_OUTLET;
    }
    return true;
}

bool check_desc(const lbm_geometry_desc *d, std::string &why) {
    if (!d) {
        why = "null descriptor";
        return false;
    }
    if (d->nx < 3 || d->ny < 3) {
        why = "nx and ny must be >= 3";
        return false;
    }
    // work lists pack a tile or block column and row into 16 + 15 bits
    if (d->nx > 65536 || d->ny > 65536 || (int64_t)d->nx * d->ny >= (int64_t)1 << 31) {
        why = "nx and ny must be <= 65536 and nx*ny < 2^31";
        return false;
    }
    if (!(d->tau > 0.5) || !std::isfinite(d->tau)) {
        why = "tau must be a finite value > 1/2";
        return false;
    }
    if (!(d->rho_out > 0.0) || !std::isfinite(d->rho_out)) {
        why = "rho_out must be a finite value > 0";
        return false;
    }
    if (!std::isfinite(d->u_peak) || std::fabs(d->u_peak) >= 1.0) {
        why = "|u_peak| must be < 1";
        return false;
    }
    if (d->precision != LBM_F64 && d->precision != LBM_F32 && d->precision != LBM_F32_S_F16 &&
        d->precision != LBM_F32_S_BF16) {
        why = "unknown precision";
        return false;
    }
    if (d->flags & ~(LBM_NEUMANN_OUTLET | LBM_SYMMETRY_TOP)) {
        why = "unknown boundary flags";
        return false;
    }
    return true;
}

bool check_types(int nx, int ny, const uint8_t *t, std::string &why) {
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const uint8_t v = t[(size_t)y * nx + x];
            if (v > LBM_OUTLET) {
                why = "cell type out of range";
                return false;
            }
            if (v == LBM_INLET && x != 0) {
                why = "inlet cell outside column 0";
                return false;
            }
            if (v == LBM_OUTLET && x != nx - 1) {
                why = "outlet cell outside column nx-1";
                return false;
            }
        }
    return true;
}

}  // namespace

struct lbm_handle {
    int nx = 0, ny = 0, pitch = 0, precision = LBM_F64, device = 0, flags = 0;
    size_t plane = 0;
    double tau = 1, u_peak = 0, rho_out = 1;
    hipStream_t stream = nullptr;

    DeviceBuffer f[2];
    int cur = 0;  // buffer holding the current state
    DeviceBuffer cell, types, uin, uprev, partials, red, out_rows, bnd;
    DeviceBuffer ctl;                    // RunControl of lbm_run_to_steady
    const int *active_stop = nullptr;    // its stop flag while a run is queued
    // While a blocked run is queued: the check launch of the interval being
    // queued writes its partials at run_part, and, when run_prev is set, the
    // interval's first launch carries out the finalize step of interval
    // run_j - 1 from run_prev (SweepArgs::prev) and writes the stop flag to
    // run_stop_rest, which the interval's later launches read.
    double *run_part = nullptr;
    const double *run_prev = nullptr;
    int *run_stop_rest = nullptr;
    int run_j = 0;
    double run_tol = 0.0;
    hipEvent_t run_ev[2 * kRunBatchMax] = {};  // per-interval timing of a run
    DeviceBuffer macro;  // 3*nx*ny doubles (rho, ux, uy), on demand
    DeviceBuffer cand, sel, select_tmp;
    int64_t cand_cap = 0;
    double *pinned = nullptr;  // small host staging for readbacks
    size_t pinned_bytes = 0;

    std::vector<uint8_t> host_types;
    std::vector<float> uin_f;
    std::vector<int32_t> out_y0, out_y1;
    int64_t n_fluid = 0, n_nonsolid = 0, steps = 0;
    double last_residual = std::nan("");
    std::vector<int64_t> last_removed, last_added;
    bool profiling = false;
    int64_t prof_launches = 0;
    double prof_ms = 0.0;

    // Replayable runs of plain sweeps, keyed by (starting buffer, count).
    struct Graph {
        int parity;
        int64_t n;
        hipGraphExec_t exec;
    };
    std::vector<Graph> graphs;
    hipStream_t capture_stream = nullptr;
    bool use_graphs = true;

    // Temporal blocking: tiles holding at least one non-solid cell.
    bool use_tb = true;
    DeviceBuffer tiles;
    std::vector<int32_t> tile_host;
    int32_t *tile_pinned = nullptr;    // staging of the tile-list upload
    size_t tile_pinned_count = 0;
    hipEvent_t tile_copied = nullptr;  // recorded after the last upload
    int n_tiles = 0;
    int tb_variant = 0;         // region shape (index into the compiled shapes)
    int tuned_variant = -1;     // the last autotuner's choice (-1: none, or overridden)
    // Per-shape ms/step of the last lbm_autotune (empty before one), whether
    // its choice then had every tile resident at once, and the device's CU
    // count and LDS per CU (how many workgroups of a shape run at once).
    std::vector<double> tune_ms;
    bool tune_fit = false;
    int cus = 0;
    size_t lds_per_cu = 0;
    uint64_t mask_version = 0;  // bumped whenever the mask changes
    // Non-solid cell counts per tile of a tw x th tiling and the tiles that
    // hold one, row-major, packed (tile row << 16 | tile column); built once
    // per tiling by a scan of the mask, then kept current from the cells each
    // exchange step flips.
    struct Tiling {
        int tw = 0, th = 0, ntx = 0, nty = 0;
        std::vector<int32_t> count, list;
    };
    std::vector<Tiling> tilings;
    int64_t prof_kernels = 0;
    int64_t prof_intervals = 0;  // check intervals seen since profiling was enabled

    size_t N() const { return (size_t)nx * ny; }
    size_t esize() const { return elem_size(precision); }
    void drop_graphs() {
        for (Graph &g : graphs) (void)hipGraphExecDestroy(g.exec);
        graphs.clear();
    }
    // Device bytes the handle holds (each block in its size class).
    size_t device_bytes() {
        DeviceBuffer *bufs[] = {&f[0], &f[1], &cell, &types, &uin, &uprev, &partials,
                                &red, &out_rows, &bnd, &macro, &cand, &sel, &select_tmp,
                                &tiles, &ctl};
        size_t b = 0;
        for (DeviceBuffer *x : bufs) b += x->bytes;
        return b;
    }
    // Hand every device block and both pinned staging areas to the caches;
    // the caller has synchronised the stream.
    void recycle() {
        DeviceBuffer *bufs[] = {&f[0], &f[1], &cell, &types, &uin, &uprev, &partials,
                                &red, &out_rows, &bnd, &macro, &cand, &sel, &select_tmp,
                                &tiles, &ctl};
        for (DeviceBuffer *b : bufs) b->recycle();
        if (pinned) host_cache().give(-1, pinned_bytes, pinned);
        pinned = nullptr;
        pinned_bytes = 0;
        if (tile_copied) (void)hipEventSynchronize(tile_copied);
        if (tile_pinned) host_cache().give(-1, tile_pinned_count * sizeof(int32_t), tile_pinned);
        tile_pinned = nullptr;
        tile_pinned_count = 0;
    }
    ~lbm_handle() {
        drop_graphs();
        if (capture_stream) (void)hipStreamDestroy(capture_stream);
        if (pinned) (void)hipHostFree(pinned);
        if (tile_copied) {
            (void)hipEventSynchronize(tile_copied);
            (void)hipEventDestroy(tile_copied);
        }
        if (tile_pinned) (void)hipHostFree(tile_pinned);
        for (hipEvent_t e : run_ev)
            if (e) (void)hipEventDestroy(e);
    }
};

namespace {

int tb_variant_count(int precision) {
    return with_storage(precision, [](auto t) { return TbVariants<decltype(t)>::count; });
}
TbVariant tb_shape(int precision, int variant) {
    return with_storage(precision, [&](auto t) { return TbVariants<decltype(t)>::v[variant]; });
}
int tile_width(int precision, int variant) { return 64 - 2 * tb_shape(precision, variant).halo; }
int tile_height(int precision, int variant) {
    const TbVariant v = tb_shape(precision, variant);
    return v.rows - 2 * v.halo;
}
int steps_per_launch(int precision, int variant) { return tb_shape(precision, variant).halo; }
// LDS of one workgroup of a shape: the region copies (one when updated in
// place) plus the compacted list.
size_t shape_lds_bytes(int precision, int variant) {
    const TbVariant v = tb_shape(precision, variant);
    return (v.kind == kTbInPlace ? 1 : 2) * 9 * 64 * (size_t)v.rows * elem_size(precision) +
           (v.kind == kTbCompact ? 64 * (size_t)v.rows * 4 : 0);
}
size_t tile_count(int nx, int ny, int precision, int variant) {
    const int w = tile_width(precision, variant), hh = tile_height(precision, variant);
    return (size_t)((nx + w - 1) / w) * ((ny + hh - 1) / hh);
}
// The largest tile count over the compiled shapes (sizes the tile list and
// the per-tile partials once for any shape).
size_t max_tile_count(int nx, int ny, int precision) {
    size_t m = 0;
    for (int v = 0; v < tb_variant_count(precision); ++v)
        m = std::max(m, tile_count(nx, ny, precision, v));
    return m;
}

// Partial slots of a lattice (4 doubles each): one per sweep block, or two
// per tile (a queued run alternates between two halves of the buffer).
size_t partial_slots(int nx, int ny, int precision) {
    return std::max((size_t)sweep_blocks(nx, ny), 2 * max_tile_count(nx, ny, precision));
}

// Initial capacity of each exchange-step candidate list.
int64_t initial_cand_cap(size_t N) { return std::max<int64_t>(4096, (int64_t)(N / 16)); }

size_t footprint(int nx, int ny, int precision) {
    const int pitch = pitch_for(nx);
    const size_t plane = (size_t)ny * pitch, N = (size_t)nx * ny;
    const size_t es = elem_size(precision);
    // each buffer is allocated in its size class
    auto c = [](size_t n) { return BlockCache::size_class(n); };
    size_t b = 2 * c(9 * plane * es);        // populations
    b += c(plane * sizeof(uint16_t));        // cell words
    b += c(N);                               // type map
    b += c((size_t)ny * sizeof(double));     // inlet profile
    b += c(2 * plane * sizeof(double));      // u_prev
    const size_t ntiles = max_tile_count(nx, ny, precision);
    b += c(partial_slots(nx, ny, precision) * 4 * sizeof(double));
    b += c(ntiles * sizeof(int32_t));
    // exchange step, allocated on the first one: the two candidate lists at
    // their initial capacity, the selection scratch and the selections (each
    // at most that capacity); the lists grow when a lattice has more
    // interface cells than N/16 per kind, and the count then exceeds this
    const int64_t cap = initial_cand_cap(N);
    b += c((size_t)cap * 2 * (2 * sizeof(uint64_t) + sizeof(int32_t)));
    b += c(select_scratch_bytes(cap));
    b += c((size_t)cap * (sizeof(double) + 2 * sizeof(int32_t)));
    // the outlet sums of lbm_outlet_stats
    b += c((size_t)(2 * (2 * ny + 5) + 1) * sizeof(double));
    // reduction results, run control, outlet rows (at most one run per two rows)
    b += c(64 * sizeof(double));
    b += c(sizeof(RunControl));
    b += c(2 * (size_t)std::max(1, (ny + 1) / 2) * sizeof(int32_t));
    return b;
}

void compute_ports(lbm_handle *h) {
    const int nx = h->nx, ny = h->ny;
    h->out_y0.clear();
    h->out_y1.clear();
    int y = 0;
    while (y < ny) {
        if (h->host_types[(size_t)y * nx + nx - 1] != LBM_OUTLET) {
            ++y;
            continue;
        }
        const int y0 = y;
        while (y < ny && h->host_types[(size_t)y * nx + nx - 1] == LBM_OUTLET) ++y;
        h->out_y0.push_back(y0);
        h->out_y1.push_back(y - 1);
    }
    h->n_fluid = h->n_nonsolid = 0;
    for (uint8_t v : h->host_types) {
        h->n_fluid += v == LBM_FLUID;
        h->n_nonsolid += v != LBM_SOLID;
    }
}

void list_tiles(lbm_handle::Tiling &t) {
    t.list.clear();
    for (int ty = 0; ty < t.nty; ++ty)
        for (int tx = 0; tx < t.ntx; ++tx)
            if (t.count[(size_t)ty * t.ntx + tx] > 0) t.list.push_back((ty << 16) | tx);
}

// Tiles of a tw x th tiling that hold a non-solid cell (cached per tiling).
const std::vector<int32_t> &tile_list(lbm_handle *h, int tw, int th) {
    for (const auto &t : h->tilings)
        if (t.tw == tw && t.th == th) return t.list;
    lbm_handle::Tiling t;
    t.tw = tw;
    t.th = th;
    t.ntx = (h->nx + tw - 1) / tw;
    t.nty = (h->ny + th - 1) / th;
    t.count.assign((size_t)t.ntx * t.nty, 0);
    for (int y = 0; y < h->ny; ++y) {
        const uint8_t *row = h->host_types.data() + (size_t)y * h->nx;
        int32_t *c = t.count.data() + (size_t)(y / th) * t.ntx;
        for (int tx = 0; tx < t.ntx; ++tx) {
            int n = 0;
            const int x1 = std::min(h->nx, (tx + 1) * tw);
            for (int x = tx * tw; x < x1; ++x) n += row[x] != LBM_SOLID;
            c[tx] += n;
        }
    }
    list_tiles(t);
    h->tilings.push_back(std::move(t));
    return h->tilings.back().list;
}

// Cells made solid (removed) and fluid (added) by an exchange step.
void tilings_flip(lbm_handle *h, const std::vector<int32_t> &removed,
                  const std::vector<int32_t> &added) {
    for (auto &t : h->tilings) {
        for (int32_t n : removed) --t.count[(size_t)((n / h->nx) / t.th) * t.ntx + (n % h->nx) / t.tw];
        for (int32_t n : added) ++t.count[(size_t)((n / h->nx) / t.th) * t.ntx + (n % h->nx) / t.tw];
        list_tiles(t);
    }
}

// Tiles of the temporal-blocking sweep (current shape) whose cells include a
// non-solid one, in launch order, uploaded to the device.
void rebuild_tiles(lbm_handle *h) {
    const bool inplace = tb_shape(h->precision, h->tb_variant).kind == kTbInPlace;
    h->tile_host = dealt_tiles(tile_list(h, tile_width(h->precision, h->tb_variant),
                                         tile_height(h->precision, h->tb_variant)),
                               inplace ? 32 : 8);
    h->n_tiles = (int)h->tile_host.size();
    const size_t cap = max_tile_count(h->nx, h->ny, h->precision);
    h->tiles.ensure(cap * sizeof(int32_t));
    if (!h->tile_copied) HIP_TRY(hipEventCreateWithFlags(&h->tile_copied, hipEventDisableTiming));
    // The staging buffer may still feed the previous upload: wait for it.
    HIP_TRY(hipEventSynchronize(h->tile_copied));
    if (h->tile_pinned_count < cap) {
        if (h->tile_pinned) (void)hipHostFree(h->tile_pinned);
        h->tile_pinned = nullptr;
        h->tile_pinned_count = 0;
        size_t got = 0;
        h->tile_pinned = static_cast<int32_t *>(pinned_alloc(cap * sizeof(int32_t), got));
        h->tile_pinned_count = got / sizeof(int32_t);
    }
    if (h->n_tiles > 0) {
        std::memcpy(h->tile_pinned, h->tile_host.data(), h->n_tiles * sizeof(int32_t));
        HIP_TRY(hipMemcpyAsync(h->tiles.p, h->tile_pinned, h->n_tiles * sizeof(int32_t),
                               hipMemcpyHostToDevice, h->stream));
    }
    HIP_TRY(hipEventRecord(h->tile_copied, h->stream));
}

// Tiles of shape `variant` the device runs at once (one round of workgroups).
size_t resident_tiles(const lbm_handle *h, int variant) {
    const size_t lds = shape_lds_bytes(h->precision, variant);
    return (size_t)h->cus * std::max<size_t>(1, h->lds_per_cu / std::max<size_t>(lds, 1));
}

// After an exchange step: the autotuned shape while its tiles all run in one
// round of workgroups, else the fastest timed shape whose tiles do (the
// shape never changes results); see fitted_shape.
void refit_shape(lbm_handle *h) {
    const int nv = (int)h->tune_ms.size();
    if (nv == 0 || !h->use_tb || !h->tune_fit || h->tuned_variant < 0) return;
    std::vector<size_t> resident(nv);
    for (int v = 0; v < nv; ++v) resident[v] = resident_tiles(h, v);
    const int v = fitted_shape(h->tuned_variant, h->tune_ms, resident, [&](int s) {
        return tile_list(h, tile_width(h->precision, s), tile_height(h->precision, s)).size();
    });
    if (v != h->tb_variant) {
        h->tb_variant = v;
        rebuild_tiles(h);
    }
}

// Parabolic inlet profile (Sec. 3.3) on each maximal run of inlet rows,
// walls half a cell outside the run; the product of the two wall distances
// first, so mirrored rows get bitwise equal values.  Under a symmetry plane
// above the top row, a run reaching row ny-1 is the lower half of an opening
// mirrored about that plane.
std::vector<double> inlet_profile(const lbm_handle *h) {
    std::vector<double> u(h->ny, 0.0);
    int y = 0;
    while (y < h->ny) {
        if (h->host_types[(size_t)y * h->nx] != LBM_INLET) {
            ++y;
            continue;
        }
        const int y0 = y;
        while (y < h->ny && h->host_types[(size_t)y * h->nx] == LBM_INLET) ++y;
        const int last = y - 1;
        const int y1 =
            ((h->flags & LBM_SYMMETRY_TOP) && last == h->ny - 1) ? 2 * h->ny - 1 - y0 : last;
        const double W = (double)(y1 - y0 + 1);
        for (int r = y0; r <= last; ++r) {
            const double a = (double)(r - y0) + 0.5, b = (double)(y1 - r) + 0.5;
            u[r] = 4.0 * h->u_peak * (a * b) / (W * W);
        }
    }
    return u;
}

void ensure_pinned(lbm_handle *h, size_t bytes) {
    if (h->pinned_bytes >= bytes) return;
    if (h->pinned) (void)hipHostFree(h->pinned);
    h->pinned = nullptr;
    h->pinned_bytes = 0;
    size_t got = 0;
    h->pinned = static_cast<double *>(pinned_alloc(bytes, got));
    h->pinned_bytes = got;
}

template <typename T>
SweepArgs<T> sweep_args(lbm_handle *h, bool check) {
    SweepArgs<T> a;
    a.fin = h->f[h->cur].as<T>();
    a.fout = h->f[1 - h->cur].as<T>();
    a.cell = h->cell.as<uint16_t>();
    a.uin = h->uin.as<UinT<T>>();
    a.uprev = check ? h->uprev.as<double>() : nullptr;
    a.partials = !check ? nullptr : h->run_part ? h->run_part : h->partials.as<double>();
    a.stop = !h->use_tb ? nullptr
             : h->active_stop ? h->active_stop
                              : h->ctl.as<RunControl>()->zeros;
    a.nx = h->nx;
    a.ny = h->ny;
    a.pitch = h->pitch;
    a.plane = h->plane;
    a.omega = 1.0 / h->tau;
    a.rho_out = h->rho_out;
    a.one_minus_rho_out = 1.0 - h->rho_out;
    a.flags = h->flags;
    return a;
}

template <typename T>
MacroArgs<T> macro_args(lbm_handle *h) {
    MacroArgs<T> a;
    a.f = h->f[h->cur].as<T>();
    a.cell = h->cell.as<uint16_t>();
    a.rho = a.ux = a.uy = nullptr;
    a.uprev = nullptr;
    a.nx = h->nx;
    a.ny = h->ny;
    a.pitch = h->pitch;
    a.plane = h->plane;
    return a;
}

template <typename T>
void step(lbm_handle *h, bool check) {
    HIP_TRY(launch_sweep<T>(sweep_args<T>(h, check), check, h->stream));
    h->cur = 1 - h->cur;
}

// `n` plain sweeps.  Runs of 8 or more are captured once per (starting
// buffer, n) into a HIP graph of kernel nodes on a private stream and then
// replayed on the handle's stream, which removes the per-launch host cost
// from the time loop.  LBM_GRAPHS=0 in the environment launches directly.
template <typename T>
void plain_sweeps(lbm_handle *h, int64_t n) {
    constexpr int64_t kMaxGraph = 128;
    while (n > 0) {
        const int64_t m = std::min(n, kMaxGraph);
        n -= m;
        if (!h->use_graphs || m < 8) {
            for (int64_t s = 0; s < m; ++s) step<T>(h, false);
            continue;
        }
        hipGraphExec_t exec = nullptr;
        for (const auto &g : h->graphs)
            if (g.parity == h->cur && g.n == m) exec = g.exec;
        if (!exec) {
            if (h->graphs.size() >= 16) h->drop_graphs();
            if (!h->capture_stream)
                HIP_TRY(hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking));
            const int parity = h->cur;
            hipStream_t user = h->stream;
            HIP_TRY(hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeThreadLocal));
            h->stream = h->capture_stream;
            hipError_t err = hipSuccess;
            for (int64_t s = 0; s < m && err == hipSuccess; ++s) {
                err = launch_sweep<T>(sweep_args<T>(h, false), false, h->stream);
                h->cur = 1 - h->cur;
            }
            h->stream = user;
            h->cur = parity;
            hipGraph_t graph = nullptr;
            const hipError_t end = hipStreamEndCapture(h->capture_stream, &graph);
            HIP_TRY(err);
            HIP_TRY(end);
            const hipError_t inst = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            HIP_TRY(inst);
            h->graphs.push_back({parity, m, exec});
        }
        HIP_TRY(hipGraphLaunch(exec, h->stream));
        if (m % 2) h->cur = 1 - h->cur;
    }
}

// Advance `n` >= 1 steps; with `check` the last step also writes residual
// partials (per tile or per sweep block; see partial_count).
template <typename T>
void advance(lbm_handle *h, int64_t n, bool check) {
    if (h->use_tb) {
        bool first = true;
        while (n > 0) {
            const int s =
                (int)std::min<int64_t>(n, steps_per_launch(h->precision, h->tb_variant));
            n -= s;
            SweepArgs<T> a = sweep_args<T>(h, check && n == 0);
            if (first && h->run_prev) {
                a.prev = h->run_prev;
                a.stop_out = h->run_stop_rest;
                a.ctl = h->ctl.as<RunControl>();
                a.prev_j = h->run_j - 1;
                a.prev_count = h->n_tiles;
                a.tol = h->run_tol;
            } else if (!first && h->run_stop_rest) {
                a.stop = h->run_stop_rest;
            }
            first = false;
            HIP_TRY(launch_tb<T>(a, h->tiles.as<int32_t>(), h->n_tiles, s, check && n == 0,
                                 h->tb_variant, h->stream));
            h->cur = 1 - h->cur;
            ++h->prof_kernels;
        }
        return;
    }
    plain_sweeps<T>(h, check ? n - 1 : n);
    h->prof_kernels += check ? n - 1 : n;
    if (check) {
        step<T>(h, true);
        ++h->prof_kernels;
    }
}

int64_t partial_count(const lbm_handle *h) {
    return h->use_tb ? h->n_tiles : sweep_blocks(h->nx, h->ny);
}

template <typename T>
void uprev_from_state(lbm_handle *h) {
    MacroArgs<T> a = macro_args<T>(h);
    a.uprev = h->uprev.as<double>();
    HIP_TRY(launch_macro<T>(a, h->stream));
}

template <typename T>
void macro_to_device(lbm_handle *h) {
    h->macro.ensure(3 * h->N() * sizeof(double));
    MacroArgs<T> a = macro_args<T>(h);
    double *m = h->macro.as<double>();
    a.rho = m;
    a.ux = m + h->N();
    a.uy = m + 2 * h->N();
    HIP_TRY(launch_macro<T>(a, h->stream));
}

void macro_dispatch(lbm_handle *h) {
    with_storage(h->precision, [&](auto t) { macro_to_device<decltype(t)>(h); });
}

// While profiling, the sweep timing of a run covers every kProfileEvery-th
// check interval (two stream markers per timed interval).
constexpr int64_t kProfileEvery = 4;

template <typename T>
int run_impl(lbm_handle *h, int64_t max_steps, double tol, int32_t k,
             int64_t *steps_done, double *residual) {
    ensure_pinned(h, sizeof(RunControl));
    uprev_from_state<T>(h);
    const int64_t nparts = partial_count(h);
    // Check intervals are queued several at a time (temporal blocking only):
    // each interval's finalize step decides on the device whether the run
    // goes on, the launches queued after the deciding one change nothing, and
    // the host waits once per batch instead of once per interval.  The batch
    // grows while the residual is far from the tolerance and shrinks near it.
    // On a lattice of at most kDeferMaxPartials tiles the finalize step of
    // each interval but a batch's last is carried out by the next interval's
    // first launch when that is not also its check launch (the partials
    // alternate between two halves of the buffer), the others by a launch of
    // their own.
    h->ctl.ensure(sizeof(RunControl));
    RunControl *ctl = h->ctl.as<RunControl>();
    HIP_TRY(hipMemsetAsync(ctl, 0, sizeof(RunControl), h->stream));
    struct ActiveStop {  // the stop flag reaches the launches of this run only
        lbm_handle *h;
        ~ActiveStop() {
            h->active_stop = nullptr;
            h->run_part = nullptr;
            h->run_prev = nullptr;
            h->run_stop_rest = nullptr;
        }
    } guard{h};
    const char *no_defer = std::getenv("LBM_DEFER");  // "0": a finalize launch per interval
    const bool defer = h->use_tb && h->n_tiles > 0 && h->n_tiles <= kDeferMaxPartials &&
                       !(no_defer && no_defer[0] == '0');
    double *const part = h->partials.as<double>();
    auto half = [&](int j) { return defer ? part + (size_t)(j % 2) * h->n_tiles * 4 : part; };
    h->run_tol = tol;
    h->active_stop = h->use_tb ? ctl->stop_lanes[0] : nullptr;
    // Timing-only events: without the system-scope fence that an ordinary
    // event record adds (a cache writeback and invalidation between two
    // launches), which cost 4.7 % of the headline solve's time at two
    // records per check interval.  Nothing reads memory through them.
    if (h->profiling)
        for (hipEvent_t &e : h->run_ev)
            if (!e) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    int64_t done = 0;
    double r = h->last_residual, r_prev = std::nan("");
    int status = LBM_OK;
    bool converged = false;
    int batch = 1;
    while (done < max_steps) {
        const int nb = h->use_tb ? batch : 1;
        int64_t chunk[kRunBatchMax];
        int cur_after[kRunBatchMax];
        int64_t kernels[kRunBatchMax];
        bool timed[kRunBatchMax];  // every kProfileEvery-th interval, when profiling
        int planned = 0;
        for (int64_t at = done; planned < nb && at < max_steps; ++planned) {
            chunk[planned] = std::min<int64_t>(k, max_steps - at);
            at += chunk[planned];
            const int64_t k0 = h->prof_kernels;
            timed[planned] = h->profiling && h->prof_intervals++ % kProfileEvery == 0;
            // an interval of one launch (its check launch) leaves the finalize
            // step of the interval before it to a launch of its own
            const bool by_first = defer && planned > 0 &&
                                  chunk[planned] > steps_per_launch(h->precision, h->tb_variant);
            if (defer && planned > 0 && !by_first)
                HIP_TRY(launch_finalize_check(half(planned - 1), nparts, ctl, planned - 1, tol,
                                              h->stream));
            h->run_j = planned;
            h->run_part = half(planned);
            h->run_prev = by_first ? half(planned - 1) : nullptr;
            if (h->use_tb) {
                h->active_stop = ctl->stop_lanes[planned % 2];
                h->run_stop_rest = ctl->stop_lanes[(planned + (by_first ? 1 : 0)) % 2];
            }
            if (timed[planned]) HIP_TRY(hipEventRecord(h->run_ev[2 * planned], h->stream));
            advance<T>(h, chunk[planned], true);
            if (timed[planned])
                HIP_TRY(hipEventRecord(h->run_ev[2 * planned + 1], h->stream));
            kernels[planned] = h->prof_kernels - k0;
            h->prof_kernels = k0;
            if (!defer)
                HIP_TRY(launch_finalize_check(half(planned), nparts, ctl, planned, tol,
                                              h->stream));
            cur_after[planned] = h->cur;
        }
        h->run_part = nullptr;
        h->run_prev = nullptr;
        h->run_stop_rest = nullptr;
        if (defer)
            HIP_TRY(launch_finalize_check(half(planned - 1), nparts, ctl, planned - 1, tol,
                                          h->stream));
        const RunControl *rc = reinterpret_cast<const RunControl *>(h->pinned);
        HIP_TRY(hipMemcpyAsync(h->pinned, ctl, sizeof(RunControl), hipMemcpyDeviceToHost,
                               h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        const int ran = rc->done;
        if (ran < 1 || ran > planned) throw HipFail{hipErrorUnknown, "run control"};
        // every interval before the last one carried out must have gone on
        for (int j = 0; j + 1 < ran; ++j) {
            const double nj = rc->sums[j][0], dj = rc->sums[j][1];
            const double rj = dj == 0.0 ? (nj == 0.0 ? 0.0 : INFINITY) : std::sqrt(nj) / std::sqrt(dj);
            if (rc->sums[j][3] != 0.0 || !std::isfinite(nj) || !std::isfinite(dj) ||
                (tol > 0.0 && rj < tol))
                throw HipFail{hipErrorUnknown, "run control disagrees with the residual"};
        }
        for (int j = 0; j < ran; ++j) {
            done += chunk[j];
            h->steps += chunk[j];
            if (timed[j]) {
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, h->run_ev[2 * j], h->run_ev[2 * j + 1]));
                h->prof_ms += ms;
                h->prof_launches += chunk[j];
                h->prof_kernels += kernels[j];
            }
        }
        h->cur = cur_after[ran - 1];  // launches queued after the last interval did nothing
        const double num = rc->sums[ran - 1][0], den = rc->sums[ran - 1][1],
                     bad = rc->sums[ran - 1][3];
        if (bad != 0.0 || !std::isfinite(num) || !std::isfinite(den)) {
            r = std::nan("");
            status = fail(LBM_EUNSTABLE, "non-finite density or velocity");
            break;
        }
        r = den == 0.0 ? (num == 0.0 ? 0.0 : INFINITY) : std::sqrt(num) / std::sqrt(den);
        if (tol > 0.0 && r < tol) {
            converged = true;
            break;
        }
        if (rc->stop != 0 || ran != planned)  // the device stopped where the host would not
            throw HipFail{hipErrorUnknown, "run control disagrees with the residual"};
        // next batch: about half the intervals the residual's decay rate
        // predicts before the tolerance (one when it does not decay)
        int next = 1;
        if (tol > 0.0 && r_prev > 0.0 && r > 0.0 && r < r_prev) {
            const double per = std::log(r / r_prev) / (double)ran;  // log decay per interval
            const double left = std::log(tol / r) / per;
            next = (int)std::min<double>(kRunBatchMax, std::max(1.0, 0.5 * left));
        } else if (tol <= 0.0) {
            next = kRunBatchMax;
        }
        batch = next;
        r_prev = r;
    }
    if (status == LBM_OK && tol > 0.0 && !converged) status = LBM_NOT_CONVERGED;
    h->last_residual = r;
    if (steps_done) *steps_done = done;
    if (residual) *residual = r;
    return status;
}

// Boundary sums of the current state and of the state one step later (a
// single sweep into the other population buffer, which holds nothing of use
// between steps; the current state and buffer parity are untouched), then
// the mass of the current state.  bout: 2 * (2 n_out + 5) sums, the current
// state's first.
template <typename T>
void stats_impl(lbm_handle *h, std::vector<double> &bout, double &mass) {
    const int n_out = (int)h->out_y0.size();
    const size_t nb = (size_t)(2 * n_out + 5);
    h->bnd.ensure((2 * nb + 1) * sizeof(double));
    ensure_pinned(h, (2 * nb + 1) * sizeof(double));
    MacroArgs<T> a = macro_args<T>(h);
    double *bo = h->bnd.as<double>();
    const int32_t *y0 = h->out_rows.as<int32_t>();
    const int32_t *y1 = y0 + std::max(n_out, 1);
    HIP_TRY(launch_boundary<T>(a, y0, y1, n_out, bo, h->stream));
    HIP_TRY(launch_sweep<T>(sweep_args<T>(h, false), false, h->stream));
    MacroArgs<T> next = a;
    next.f = h->f[1 - h->cur].as<T>();
    HIP_TRY(launch_boundary<T>(next, y0, y1, n_out, bo + nb, h->stream));
    HIP_TRY(launch_mass<T>(a, h->partials.as<double>(), h->stream));
    HIP_TRY(launch_finalize1(h->partials.as<double>(), sweep_blocks(h->nx, h->ny),
                             bo + 2 * nb, h->stream));
    HIP_TRY(hipMemcpyAsync(h->pinned, bo, (2 * nb + 1) * sizeof(double),
                           hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    bout.assign(h->pinned, h->pinned + 2 * nb);
    mass = h->pinned[2 * nb];
}

template <typename T>
void zero_cells(lbm_handle *h, const int32_t *cells, int count) {
    HIP_TRY(launch_rest_cells<T>(h->f[h->cur].as<T>(), h->plane, cells, count,
                                 h->nx, h->pitch, h->stream));
}

template <typename T>
void reset_all(lbm_handle *h) {
    for (int b = 0; b < 2; ++b)
        HIP_TRY(launch_rest_all<T>(h->f[b].as<T>(), h->plane, h->stream));
}

template <typename T>
void export_state(lbm_handle *h, double *f) {
    h->macro.ensure(3 * h->N() * sizeof(double));
    double *stage = h->macro.as<double>();
    for (int i = 0; i < 9; ++i) {
        HIP_TRY(launch_export_plane<T>(h->f[h->cur].as<T>(), h->cell.as<uint16_t>(),
                                       stage, i, h->nx, h->ny, h->pitch, h->plane,
                                       h->stream));
        HIP_TRY(hipMemcpyAsync(f + (size_t)i * h->N(), stage, h->N() * sizeof(double),
                               hipMemcpyDeviceToHost, h->stream));
    }
    HIP_TRY(hipStreamSynchronize(h->stream));
}

template <typename T>
void import_state(lbm_handle *h, const double *f) {
    h->macro.ensure(3 * h->N() * sizeof(double));
    double *stage = h->macro.as<double>();
    for (int i = 0; i < 9; ++i) {
        HIP_TRY(hipMemcpyAsync(stage, f + (size_t)i * h->N(), h->N() * sizeof(double),
                               hipMemcpyHostToDevice, h->stream));
        HIP_TRY(launch_import_plane<T>(h->f[h->cur].as<T>(), h->cell.as<uint16_t>(),
                                       stage, i, h->nx, h->ny, h->pitch, h->plane,
                                       h->stream));
    }
    HIP_TRY(hipStreamSynchronize(h->stream));
}

int guard_hip(const HipFail &f) {
    char buf[256];
    std::snprintf(buf, sizeof buf, "HIP error %d (%s) in %s", (int)f.e,
                  hipGetErrorString(f.e), f.what);
    return fail(LBM_EHIP, buf);
}

}  // namespace

// ---------------------------------------------------------------------------
// Autotuning and batches.

namespace {

// Copies of both population buffers of a handle and its counters: tuning
// trials run real steps and must leave no trace.
struct Saved {
    DeviceBuffer f[2];
    int cur = 0;
    int64_t steps = 0;
    double residual = 0.0;
};

void save_state(lbm_handle *h, Saved &sv) {
    const size_t bytes = 9 * h->plane * h->esize();
    for (int b = 0; b < 2; ++b) {
        sv.f[b].ensure(bytes);
        HIP_TRY(hipMemcpyAsync(sv.f[b].p, h->f[b].p, bytes, hipMemcpyDeviceToDevice,
                               h->stream));
    }
    sv.cur = h->cur;
    sv.steps = h->steps;
    sv.residual = h->last_residual;
}

void restore_state(lbm_handle *h, const Saved &sv) {
    const size_t bytes = 9 * h->plane * h->esize();
    for (int b = 0; b < 2; ++b)
        HIP_TRY(hipMemcpyAsync(h->f[b].p, sv.f[b].p, bytes, hipMemcpyDeviceToDevice,
                               h->stream));
    h->cur = sv.cur;
    h->steps = sv.steps;
    h->last_residual = sv.residual;
}

struct EventPair {
    hipEvent_t e[2] = {nullptr, nullptr};
    EventPair() {
        for (hipEvent_t &x : e) HIP_TRY(hipEventCreate(&x));
    }
    ~EventPair() {
        for (hipEvent_t x : e)
            if (x) (void)hipEventDestroy(x);
    }
    double ms() const {
        float v = 0.f;
        HIP_TRY(hipEventElapsedTime(&v, e[0], e[1]));
        return (double)v;
    }
};

// Mean time per step of `n` steps after one untimed launch's worth.
template <typename T>
double time_handle_steps(lbm_handle *h, int64_t n) {
    EventPair ev;
    advance<T>(h, steps_per_launch(h->precision, h->tb_variant), false);
    HIP_TRY(hipEventRecord(ev.e[0], h->stream));
    advance<T>(h, n, false);
    HIP_TRY(hipEventRecord(ev.e[1], h->stream));
    HIP_TRY(hipEventSynchronize(ev.e[1]));
    return ev.ms() / (double)n;
}

}  // namespace

struct lbm_batch {
    std::vector<lbm_handle *> hs;
    std::vector<uint64_t> versions;
    int precision = 0, device = 0, variant = 0, order = 0;
    hipStream_t stream = nullptr;
    DeviceBuffer args;       // SweepArgs of every member: parity 0, then parity 1
    DeviceBuffer lat, tiles; // work list (lat < 0: padding item)
    int64_t n_items = 0;     // launch grid
    int64_t n_real = 0;      // real tiles
    bool dirty = true;
    bool bc = false;         // some member has boundary-variant flags
    void *pinned = nullptr;
    size_t pinned_bytes = 0;
    // Replayable runs of an even number of launches, starting at parity 0.
    struct Graph {
        int64_t launches;
        hipGraphExec_t exec;
    };
    std::vector<Graph> graphs;
    hipStream_t capture_stream = nullptr;
    bool use_graphs = true;

    void drop_graphs() {
        for (Graph &g : graphs) (void)hipGraphExecDestroy(g.exec);
        graphs.clear();
    }
    ~lbm_batch() {
        drop_graphs();
        if (capture_stream) (void)hipStreamDestroy(capture_stream);
        if (pinned) (void)hipHostFree(pinned);
    }
};

namespace {

// Launches per captured graph (even, so that every replay starts at parity 0).
constexpr int64_t kBatchGraphLaunches = 16;

// Batch variants: 0..count-1 the region shapes of the temporally blocked
// sweep, count = one time step per launch over 64 x 4 blocks.
bool batch_single_step(const lbm_batch *b) {
    return b->variant == tb_variant_count(b->precision);
}
int batch_steps_per_launch(const lbm_batch *b) {
    return batch_single_step(b) ? 1 : steps_per_launch(b->precision, b->variant);
}

void build_work(lbm_batch *b) {
    const bool one = batch_single_step(b);
    const int tw = one ? 64 : tile_width(b->precision, b->variant);
    const int th = one ? 4 : tile_height(b->precision, b->variant);
    std::vector<int32_t> L, Tl;
    for (size_t i = 0; i < b->hs.size(); ++i) {
        lbm_handle *h = b->hs[i];
        for (int32_t t : tile_list(h, tw, th)) {
            L.push_back((int32_t)i);
            Tl.push_back(t);
        }
        b->versions[i] = h->mask_version;
    }
    b->n_real = (int64_t)L.size();
    if (b->order == 1 && !L.empty()) {
        // Workgroup g runs on XCD g mod 8: deal contiguous runs of the list
        // to the eight XCDs so that neighbouring tiles share an L2.
        const int64_t per = (b->n_real + 7) / 8;
        std::vector<int32_t> L2((size_t)per * 8, -1), T2((size_t)per * 8, 0);
        for (int64_t k = 0; k < b->n_real; ++k) {
            const int64_t slot = (k % per) * 8 + k / per;
            L2[slot] = L[k];
            T2[slot] = Tl[k];
        }
        L.swap(L2);
        Tl.swap(T2);
    }
    b->n_items = (int64_t)L.size();
    b->lat.ensure(std::max<size_t>(1, L.size()) * sizeof(int32_t));
    b->tiles.ensure(std::max<size_t>(1, L.size()) * sizeof(int32_t));
    if (!L.empty()) {
        HIP_TRY(hipMemcpyAsync(b->lat.p, L.data(), L.size() * sizeof(int32_t),
                               hipMemcpyHostToDevice, b->stream));
        HIP_TRY(hipMemcpyAsync(b->tiles.p, Tl.data(), Tl.size() * sizeof(int32_t),
                               hipMemcpyHostToDevice, b->stream));
    }
    HIP_TRY(hipStreamSynchronize(b->stream));
    b->drop_graphs();
    b->dirty = false;
}

bool work_stale(const lbm_batch *b) {
    if (b->dirty) return true;
    for (size_t i = 0; i < b->hs.size(); ++i)
        if (b->versions[i] != b->hs[i]->mask_version) return true;
    return false;
}

template <typename T>
hipError_t batch_launch(lbm_batch *b, int parity, int steps, hipStream_t s) {
    const SweepArgs<T> *A = b->args.as<SweepArgs<T>>() + (size_t)parity * b->hs.size();
    if (batch_single_step(b))
        return launch_step_batch<T>(A, b->lat.as<int32_t>(), b->tiles.as<int32_t>(),
                                    (int)b->n_items, b->bc, s);
    return launch_tb_batch<T>(A, b->lat.as<int32_t>(), b->tiles.as<int32_t>(),
                              (int)b->n_items, steps, b->variant, b->bc, s);
}

template <typename T>
hipGraphExec_t batch_graph(lbm_batch *b, int64_t launches) {
    for (const auto &g : b->graphs)
        if (g.launches == launches) return g.exec;
    if (!b->capture_stream)
        HIP_TRY(hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking));
    const int H = batch_steps_per_launch(b);
    // Kernel attributes are set outside the capture (an empty launch does it).
    if (!batch_single_step(b))
        HIP_TRY(launch_tb_batch<T>(nullptr, nullptr, nullptr, 0, H, b->variant, b->bc, b->stream));
    HIP_TRY(hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal));
    hipError_t err = hipSuccess;
    for (int64_t k = 0; k < launches && err == hipSuccess; ++k)
        err = batch_launch<T>(b, (int)(k % 2), H, b->capture_stream);
    hipGraph_t graph = nullptr;
    const hipError_t end = hipStreamEndCapture(b->capture_stream, &graph);
    HIP_TRY(err);
    HIP_TRY(end);
    hipGraphExec_t exec = nullptr;
    const hipError_t inst = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HIP_TRY(inst);
    b->graphs.push_back({launches, exec});
    return exec;
}

template <typename T>
double batch_run_impl(lbm_batch *b, int64_t steps) {
    if (work_stale(b)) build_work(b);
    // The members' own queued work comes first.
    for (size_t i = 0; i < b->hs.size(); ++i) {
        bool seen = false;
        for (size_t j = 0; j < i && !seen; ++j) seen = b->hs[j]->stream == b->hs[i]->stream;
        if (!seen) HIP_TRY(hipStreamSynchronize(b->hs[i]->stream));
    }
    const size_t n = b->hs.size();
    const size_t bytes = 2 * n * sizeof(SweepArgs<T>);
    if (b->pinned_bytes < bytes) {
        if (b->pinned) (void)hipHostFree(b->pinned);
        b->pinned = nullptr;
        b->pinned_bytes = 0;
        size_t got = 0;
        b->pinned = pinned_alloc(bytes, got);
        b->pinned_bytes = got;
    }
    SweepArgs<T> *pa = static_cast<SweepArgs<T> *>(b->pinned);
    for (size_t i = 0; i < n; ++i) {
        lbm_handle *h = b->hs[i];
        pa[i] = sweep_args<T>(h, false);
        pa[n + i] = pa[i];
        pa[n + i].fin = pa[i].fout;
        pa[n + i].fout = const_cast<T *>(pa[i].fin);
    }
    HIP_TRY(hipMemcpyAsync(b->args.p, pa, bytes, hipMemcpyHostToDevice, b->stream));

    const int H = batch_steps_per_launch(b);
    const int64_t full = steps / H;
    const int rem = (int)(steps % H);
    int64_t done = 0;
    hipGraphExec_t exec = nullptr;
    if (b->use_graphs && full >= kBatchGraphLaunches && b->n_items > 0)
        exec = batch_graph<T>(b, kBatchGraphLaunches);
    EventPair ev;
    HIP_TRY(hipEventRecord(ev.e[0], b->stream));
    if (exec)
        for (; done + kBatchGraphLaunches <= full; done += kBatchGraphLaunches)
            HIP_TRY(hipGraphLaunch(exec, b->stream));
    for (; done < full; ++done) HIP_TRY(batch_launch<T>(b, (int)(done % 2), H, b->stream));
    if (rem > 0) {
        HIP_TRY(batch_launch<T>(b, (int)(done % 2), rem, b->stream));
        ++done;
    }
    HIP_TRY(hipEventRecord(ev.e[1], b->stream));
    HIP_TRY(hipEventSynchronize(ev.e[1]));
    for (lbm_handle *h : b->hs) {
        if (done % 2) h->cur = 1 - h->cur;
        h->steps += steps;
        if (steps > 0) h->last_residual = std::nan("");
    }
    return ev.ms();
}

}  // namespace

// ---------------------------------------------------------------------------
extern "C" {

const char *lbm_last_error(void) { return g_error.c_str(); }

size_t lbm_footprint_bytes(const lbm_geometry_desc *d) {
    std::string why;
    if (!check_desc(d, why)) return 0;
    return footprint(d->nx, d->ny, d->precision);
}

}  // extern "C"

namespace lbm {
void handle_set_stream(lbm_handle *h, hipStream_t s) {
    h->drop_graphs();  // captured for the old stream
    h->stream = s;
}
}  // namespace lbm

extern "C" {

int lbm_device_bytes(lbm_handle *h, size_t *bytes) {
    g_error.clear();
    if (!h || !bytes) return fail(LBM_EINVAL, "null argument");
    *bytes = h->device_bytes();
    return LBM_OK;
}

int lbm_create_geometry(const lbm_geometry_desc *d, const uint8_t *cell_types,
                        void *hip_stream, lbm_handle **out) {
    g_error.clear();
    if (!out) return fail(LBM_EINVAL, "null output handle pointer");
    *out = nullptr;
    std::string why;
    if (!check_desc(d, why)) return fail(LBM_EINVAL, why);
    lbm_handle *h = new (std::nothrow) lbm_handle();
    if (!h) return fail(LBM_ENOMEM, "host allocation failed");
    try {
        h->nx = d->nx;
        h->ny = d->ny;
        h->pitch = pitch_for(d->nx);
        h->plane = (size_t)h->ny * h->pitch;
        h->precision = d->precision;
        h->tau = d->tau;
        h->u_peak = d->u_peak;
        h->rho_out = d->rho_out;
        h->flags = d->flags;
        h->stream = static_cast<hipStream_t>(hip_stream);
        const char *g = std::getenv("LBM_GRAPHS");
        h->use_graphs = !(g && g[0] == '0');
        const char *tb = std::getenv("LBM_TB");
        h->use_tb = !(tb && tb[0] == '0');
        HIP_TRY(hipGetDevice(&h->device));
        HIP_TRY(hipDeviceGetAttribute(&h->cus, hipDeviceAttributeMultiprocessorCount, h->device));
        int lds = 0;
        HIP_TRY(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                                      h->device));
        h->lds_per_cu = (size_t)lds;
        if (cell_types) {
            if (!check_types(h->nx, h->ny, cell_types, why)) {
                delete h;
                return fail(LBM_EINVAL, why);
            }
            h->host_types.assign(cell_types, cell_types + h->N());
        } else if (!generate_distributor(*d, h->host_types, why)) {
            delete h;
            return fail(LBM_EINVAL, why);
        }
        compute_ports(h);
        const size_t es = h->esize();
        for (int b = 0; b < 2; ++b) h->f[b].ensure(9 * h->plane * es);
        h->cell.ensure(h->plane * sizeof(uint16_t));
        h->types.ensure(h->N());
        h->uin.ensure((size_t)h->ny * sizeof(double));
        h->uprev.ensure(2 * h->plane * sizeof(double));
        h->partials.ensure(partial_slots(h->nx, h->ny, h->precision) * 4 * sizeof(double));
        h->red.ensure(64 * sizeof(double));
        h->ctl.ensure(sizeof(RunControl));
        HIP_TRY(hipMemsetAsync(h->ctl.p, 0, sizeof(RunControl), h->stream));
        const int n_out = (int)h->out_y0.size();
        h->out_rows.ensure(2 * (size_t)std::max(n_out, 1) * sizeof(int32_t));
        ensure_pinned(h, 64 * sizeof(double));

        HIP_TRY(hipMemcpyAsync(h->types.p, h->host_types.data(), h->N(),
                               hipMemcpyHostToDevice, h->stream));
        if (n_out > 0) {
            HIP_TRY(hipMemcpyAsync(h->out_rows.p, h->out_y0.data(), n_out * sizeof(int32_t),
                                   hipMemcpyHostToDevice, h->stream));
            HIP_TRY(hipMemcpyAsync(h->out_rows.as<int32_t>() + n_out, h->out_y1.data(),
                                   n_out * sizeof(int32_t), hipMemcpyHostToDevice,
                                   h->stream));
        }
        // inlet velocities: double for the double form, float otherwise (the
        // offset forms read them through their arithmetic type)
        const std::vector<double> u = inlet_profile(h);
        if (h->precision == LBM_F64) {
            HIP_TRY(hipMemcpyAsync(h->uin.p, u.data(), h->ny * sizeof(double),
                                   hipMemcpyHostToDevice, h->stream));
        } else {
            h->uin_f.assign(u.begin(), u.end());
            HIP_TRY(hipMemcpyAsync(h->uin.p, h->uin_f.data(), h->ny * sizeof(float),
                                   hipMemcpyHostToDevice, h->stream));
        }
        with_storage(h->precision, [&](auto t) { reset_all<decltype(t)>(h); });
        HIP_TRY(launch_build_cells(h->types.as<uint8_t>(), h->cell.as<uint16_t>(), h->nx,
                                   h->ny, h->pitch, h->flags, h->stream));
        rebuild_tiles(h);
        HIP_TRY(hipStreamSynchronize(h->stream));
    } catch (const std::bad_alloc &) {
        delete h;
        return fail(LBM_ENOMEM, "device allocation failed");
    } catch (const HipFail &e) {
        delete h;
        return guard_hip(e);
    }
    *out = h;
    return LBM_OK;
}

void lbm_destroy(lbm_handle *h) {
    if (!h) return;
    (void)hipSetDevice(h->device);
    // Batches synchronise before returning, so after this no queued work
    // reads the handle's memory and its blocks can be recycled.
    if (hipStreamSynchronize(h->stream) == hipSuccess) h->recycle();
    delete h;
}

int lbm_run_to_steady(lbm_handle *h, int64_t max_steps, double tol,
                      int32_t check_every, int64_t *steps_done,
                      double *residual) {
    g_error.clear();
    if (!h) return fail(LBM_EINVAL, "null handle");
    if (max_steps < 0 || check_every < 1 || std::isnan(tol))
        return fail(LBM_EINVAL, "max_steps >= 0 and check_every >= 1 required");
    try {
        HIP_TRY(hipSetDevice(h->device));
        return with_storage(h->precision, [&](auto t) {
            return run_impl<decltype(t)>(h, max_steps, tol, check_every, steps_done, residual);
        });
    } catch (const HipFail &e) {
        return guard_hip(e);
    } catch (const std::bad_alloc &) {
        return fail(LBM_ENOMEM, "allocation failed");
    }
}

int lbm_bench_sweep(lbm_handle *h, int32_t steps, double *ms_per_step) {
    g_error.clear();
    if (!h || steps < 1 || !ms_per_step) return fail(LBM_EINVAL, "bad arguments");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    try {
        HIP_TRY(hipSetDevice(h->device));
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        // warm the graph cache and kernel setup outside the timed region
        const int64_t warm = std::min<int64_t>(steps, 128);
        with_storage(h->precision, [&](auto t) { advance<decltype(t)>(h, warm, false); });
        HIP_TRY(hipEventRecord(e0, h->stream));
        with_storage(h->precision, [&](auto t) { advance<decltype(t)>(h, steps, false); });
        HIP_TRY(hipEventRecord(e1, h->stream));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        *ms_per_step = (double)ms / steps;
        h->steps += steps + warm;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return LBM_OK;
    } catch (const HipFail &e) {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        return guard_hip(e);
    }
}

int lbm_profile_sweeps(lbm_handle *h, int32_t enable, int64_t *steps,
                       int64_t *launches, double *total_ms) {
    g_error.clear();
    if (!h) return fail(LBM_EINVAL, "null handle");
    try {
        HIP_TRY(hipSetDevice(h->device));
        if (enable) {
            h->prof_launches = 0;
            h->prof_kernels = 0;
            h->prof_ms = 0.0;
            h->prof_intervals = 0;
        }
        h->profiling = enable != 0;
    } catch (const HipFail &e) {
        return guard_hip(e);
    }
    if (steps) *steps = h->prof_launches;
    if (launches) *launches = h->prof_kernels;
    if (total_ms) *total_ms = h->prof_ms;
    return LBM_OK;
}

}  // extern "C"

namespace {

// Fill s (and flow) from the boundary sums b of the current state (b[0, nb))
// and of the state one step later (b[nb, 2 nb)), nb = 2 n_out + 5, and the
// current state's mass: the steady flow rates are the two-step means, which
// cancel the undamped period-two oscillation of the boundary fluxes; Eqs.
// 9-11 on the means.
void finish_stats(const lbm_handle *h, const double *b, double mass, double *flow,
                  lbm_stats *s) {
    const int n_out = (int)h->out_y0.size();
    const size_t nb = (size_t)(2 * n_out + 5);
    auto dp_of = [&](const double *c) {  // Eq. 4 with c_s^2 = 1/3
        const double rho_in_sum = c[2 * n_out + 1], cnt_in = c[2 * n_out + 2];
        const double cnt_out = c[2 * n_out + 3], rho_out_sum = c[2 * n_out + 4];
        const double rin = cnt_in > 0 ? rho_in_sum / cnt_in : 0.0;
        const double rout = cnt_out > 0 ? rho_out_sum / cnt_out : 0.0;
        return (rin - rout) / 3.0;
    };
    double p2 = 0.0;
    for (int k = 0; k < n_out; ++k) {
        p2 = std::max(p2, std::fabs(b[k] - b[nb + k]) * 0.5);
        flow[k] = 0.5 * (b[k] + b[nb + k]);
    }
    s->flow_in = 0.5 * (b[2 * n_out] + b[nb + 2 * n_out]);
    s->dp = 0.5 * (dp_of(b) + dp_of(b + nb));
    s->flow_p2 = p2;
    s->mass = mass;
    if (n_out > 0) {
        double mx = flow[0], mn = flow[0], sum = 0.0;
        for (int k = 0; k < n_out; ++k) {
            mx = std::max(mx, flow[k]);
            mn = std::min(mn, flow[k]);
            sum += flow[k];
        }
        const double ave = sum / n_out;  // Eq. 11
        double dev = 0.0;
        for (int k = 0; k < n_out; ++k) {
            const double e = flow[k] / ave - 1.0;
            dev += e * e;
        }
        s->theta = mx / mn;                                         // Eq. 9
        s->dg = n_out > 1 ? std::sqrt(dev / (double)(n_out - 1)) : 0.0;  // Eq. 10
        s->flow_ave = ave;
    }
}

// Arguments every statistics call checks; fills the counts of s.
int begin_stats(lbm_handle *h, double *flow, int32_t flow_cap, lbm_stats *s) {
    if (!h || !s) return fail(LBM_EINVAL, "null handle or stats");
    const int n_out = (int)h->out_y0.size();
    std::memset(s, 0, sizeof *s);
    s->n_outlets = n_out;
    s->n_fluid = h->n_fluid;
    s->n_nonsolid = h->n_nonsolid;
    s->residual = h->last_residual;
    s->steps = h->steps;
    if (n_out > 0 && (!flow || flow_cap < n_out))
        return fail(LBM_EINVAL, "flow_cap smaller than the number of outlets");
    return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_outlet_stats(lbm_handle *h, double *flow, int32_t flow_cap,
                     lbm_stats *s) {
    g_error.clear();
    const int rc = begin_stats(h, flow, flow_cap, s);
    if (rc != LBM_OK) return rc;
    std::vector<double> b;
    double mass = 0.0;
    try {
        HIP_TRY(hipSetDevice(h->device));
        with_storage(h->precision, [&](auto t) { stats_impl<decltype(t)>(h, b, mass); });
    } catch (const HipFail &e) {
        return guard_hip(e);
    } catch (const std::bad_alloc &) {
        return fail(LBM_ENOMEM, "allocation failed");
    }
    finish_stats(h, b.data(), mass, flow, s);
    return LBM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Statistics without allocation.

// Device scratch of lbm_outlet_stats_noalloc, one copy per GPU, held until the
// process ends: the boundary sums of two states (2 (2 n_out + 5) doubles),
// the mass (one double), then the per-block mass partials.  Host code never
// uses this name as an address (it is a host-side stand-in): it uses the
// device address that hipGetSymbolAddress returns for each device.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[64] = {};  // per device ordinal

// The scratch's device address on `device`, which must be current; looked up
// once per device.
int scratch_on(int device, double **out) {
    if (device < 0 || device >= 64) return fail(LBM_EINVAL, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(LBM_EHIP, std::string("hipGetSymbolAddress of the scratch failed: ") +
                                      hipGetErrorString(e));
        g_scratch_ptr[device] = p;
    }
    *out = static_cast<double *>(g_scratch_ptr[device]);
    return LBM_OK;
}

// The kernels of stats_impl with every intermediate in `scr` (device) and the
// sums copied to `host` (2 nb + 1 doubles): no buffer of the handle's is
// grown and no pinned staging is used.
template <typename T>
void stats_noalloc_impl(lbm_handle *h, double *scr, double *host) {
    const int n_out = (int)h->out_y0.size();
    const size_t nb = (size_t)(2 * n_out + 5);
    MacroArgs<T> a = macro_args<T>(h);
    const int32_t *y0 = h->out_rows.as<int32_t>();
    const int32_t *y1 = y0 + std::max(n_out, 1);
    double *partials = scr + 2 * nb + 1;
    HIP_TRY(launch_boundary<T>(a, y0, y1, n_out, scr, h->stream));
    HIP_TRY(launch_sweep<T>(sweep_args<T>(h, false), false, h->stream));
    MacroArgs<T> next = a;
    next.f = h->f[1 - h->cur].as<T>();
    HIP_TRY(launch_boundary<T>(next, y0, y1, n_out, scr + nb, h->stream));
    HIP_TRY(launch_mass<T>(a, partials, h->stream));
    HIP_TRY(launch_finalize1(partials, sweep_blocks(h->nx, h->ny), scr + 2 * nb, h->stream));
    HIP_TRY(hipMemcpyAsync(host, scr, (2 * nb + 1) * sizeof(double), hipMemcpyDeviceToHost,
                           h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
}

}  // namespace

extern "C" {

int lbm_outlet_stats_noalloc(lbm_handle *h, double *flow, int32_t flow_cap, lbm_stats *s) {
    g_error.clear();
    const int rc = begin_stats(h, flow, flow_cap, s);
    if (rc != LBM_OK) return rc;
    const int n_out = (int)h->out_y0.size();
    if (n_out > kNoAllocMaxOutlets)
        return fail(LBM_EINVAL, "lbm_outlet_stats_noalloc: more outlets than its limit");
    const size_t nb = (size_t)(2 * n_out + 5);
    const size_t need = (2 * nb + 1 + (size_t)sweep_blocks(h->nx, h->ny)) * sizeof(double);
    if (need > kNoAllocScratchBytes)
        return fail(LBM_EINVAL, "lbm_outlet_stats_noalloc: lattice too large for its scratch");
    double host[2 * (2 * kNoAllocMaxOutlets + 5) + 1];
    try {
        HIP_TRY(hipSetDevice(h->device));
        double *scr = nullptr;
        const int e = scratch_on(h->device, &scr);
        if (e != LBM_OK) return e;
        with_storage(h->precision, [&](auto t) { stats_noalloc_impl<decltype(t)>(h, scr, host); });
    } catch (const HipFail &e) {
        return guard_hip(e);
    }
    finish_stats(h, host, host[2 * nb], flow, s);
    return LBM_OK;
}

}  // extern "C"

namespace {

// One exchange step (Steps 3-4 of Sec. 2.3) split into the phases between
// which the host waits for the device, so that lbm_shape_update_many can run
// each phase for many handles before waiting once.
struct Exchange {
    lbm_handle *h = nullptr;
    lbm_shape_params p{};
    const double *field = nullptr;  // host override of (rho, ux, uy), or NULL
    lbm_shape_result *r = nullptr;
    int status = LBM_OK;
    int64_t keff = 0, nf = 0;
    unsigned long long cnt[2] = {0, 0};
    size_t rb_al = 0;  // pinned offset of the selection kernels' error flag
};

int exchange_check(lbm_handle *h, const lbm_shape_params *p, lbm_shape_result *r) {
    if (!h || !p || !r) return fail(LBM_EINVAL, "null argument");
    if (!(p->frac >= 0.0 && p->frac <= 1.0)) return fail(LBM_EINVAL, "frac must be in [0, 1]");
    if (p->band_x < 1 || p->band_y < 1 || 2 * p->band_x >= h->nx || 2 * p->band_y >= h->ny)
        return fail(LBM_EINVAL, "band_x, band_y must be >= 1 and leave an interior");
    if (p->criterion != LBM_CRIT_PAPER && p->criterion != LBM_CRIT_SPEED)
        return fail(LBM_EINVAL, "unknown criterion");
    if (p->reinit != LBM_WARM && p->reinit != LBM_COLD)
        return fail(LBM_EINVAL, "unknown reinit mode");
    return LBM_OK;
}

unsigned long long *exchange_counters(lbm_handle *h) {
    return h->red.as<unsigned long long>() + 32;
}
int *exchange_error(lbm_handle *h) {
    return reinterpret_cast<int *>(h->red.as<unsigned long long>() + 36);
}

// Phase 1: the field (the current state's moments, or the override), then the
// candidates and their keys; the counts and the error flag are copied to the
// pinned staging.  No wait.
void exchange_keys(Exchange &e) {
    lbm_handle *h = e.h;
    const size_t N = h->N();
    HIP_TRY(hipSetDevice(h->device));
    // The keys read the field the caller gave, else the stored state itself
    // (only the interface cells and their neighbours).
    const double *m = nullptr;
    if (e.field) {
        h->macro.ensure(3 * N * sizeof(double));
        HIP_TRY(hipMemcpyAsync(h->macro.p, e.field, 3 * N * sizeof(double),
                               hipMemcpyHostToDevice, h->stream));
        m = h->macro.as<double>();
    }
    ensure_pinned(h, 64 * sizeof(double));
    // candidate lists: 2 x (u64 key, u64 hash, i32 idx) per entry
    if (h->cand_cap == 0) h->cand_cap = initial_cand_cap(N);
    const int64_t cap = h->cand_cap;
    h->cand.ensure((size_t)cap * 2 * (2 * sizeof(uint64_t) + sizeof(int32_t)));
    uint64_t *kf = h->cand.as<uint64_t>();
    unsigned long long *counters = exchange_counters(h);
    // counters[0..3] and the error flag (counters + 4) in one fill
    HIP_TRY(hipMemsetAsync(counters, 0, 5 * sizeof(unsigned long long), h->stream));
    KeysArgs ka;
    ka.types = h->types.as<uint8_t>();
    ka.rho = m;
    ka.ux = m ? m + N : nullptr;
    ka.uy = m ? m + 2 * N : nullptr;
    ka.f = h->f[h->cur].p;
    ka.plane = h->plane;
    ka.pitch = h->pitch;
    ka.nx = h->nx;
    ka.ny = h->ny;
    ka.band_x = e.p.band_x;
    ka.band_y = e.p.band_y;
    ka.criterion = e.p.criterion;
    ka.seed = e.p.seed;
    ka.cap = cap;
    ka.count_f = counters;
    ka.count_s = counters + 1;
    ka.error = exchange_error(h);
    ka.kf = kf;
    ka.hf = kf + cap;
    ka.ks = kf + 2 * cap;
    ka.hs = kf + 3 * cap;
    ka.if_ = reinterpret_cast<int32_t *>(kf + 4 * cap);
    ka.is = ka.if_ + cap;
    with_storage(h->precision, [&](auto t) { HIP_TRY(launch_keys<decltype(t)>(ka, h->stream)); });
    HIP_TRY(hipMemcpyAsync(h->pinned, counters, 5 * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, h->stream));
}

// After the wait: the candidate counts.  False when a list outgrew its
// capacity (the capacity is then raised; phase 1 must run again).
bool exchange_counts(Exchange &e) {
    lbm_handle *h = e.h;
    const unsigned long long *pc = reinterpret_cast<unsigned long long *>(h->pinned);
    e.cnt[0] = pc[0];
    e.cnt[1] = pc[1];
    if (*reinterpret_cast<const int *>(pc + 4) != 0) {
        e.status = fail(LBM_EINVAL, "NaN or negative exchange key");
        return true;
    }
    const int64_t need = (int64_t)std::max(e.cnt[0], e.cnt[1]);
    if (need <= h->cand_cap) return true;
    h->cand_cap = need;  // grow and recompute
    h->cand.reset();
    return false;
}

// Phase 2: selection, flips, re-initialisation of the flipped cells; the
// selections, removed densities and the error flag are copied to the pinned
// staging.  No wait.
void exchange_select(Exchange &e) {
    lbm_handle *h = e.h;
    const int64_t cap = h->cand_cap;
    uint64_t *kf = h->cand.as<uint64_t>();
    uint64_t *hf = kf + cap, *ks = kf + 2 * cap, *hs = kf + 3 * cap;
    int32_t *if_ = reinterpret_cast<int32_t *>(kf + 4 * cap), *is = if_ + cap;
    e.nf = h->n_fluid;
    int64_t K = (int64_t)std::floor(e.p.frac * (double)e.nf);
    if (K < 1) K = 1;
    e.keff = std::min<int64_t>(K, std::min<int64_t>(e.cnt[0], e.cnt[1]));
    e.r->n_cand_fluid = (int64_t)e.cnt[0];
    e.r->n_cand_solid = (int64_t)e.cnt[1];
    e.r->n_fluid_before = e.nf;
    const int64_t keff = e.keff;
    if (keff <= 0) return;
    // sel: the removed cells' densities, then the removed and the added cell
    // lists (the layout the pinned readback mirrors)
    h->sel.ensure((size_t)keff * (sizeof(double) + 2 * sizeof(int32_t)));
    double *rrho = h->sel.as<double>();
    int32_t *srem = reinterpret_cast<int32_t *>(rrho + keff), *sadd = srem + keff;
    h->select_tmp.ensure(select_scratch_bytes(keff));
    int *err = exchange_error(h);
    HIP_TRY(launch_select_pair(kf, hf, if_, (int64_t)e.cnt[0], ks, hs, is, (int64_t)e.cnt[1], keff,
                               srem, sadd, h->select_tmp.p, keff, err, h->stream));
    FlipArgs fa;
    fa.types = h->types.as<uint8_t>();
    fa.removed = srem;
    fa.added = sadd;
    fa.k_eff = (int)keff;
    fa.removed_rho = rrho;
    fa.rho = e.field ? h->macro.as<double>() : nullptr;
    fa.f = h->f[h->cur].p;
    fa.plane = h->plane;
    fa.nx = h->nx;
    fa.pitch = h->pitch;
    with_storage(h->precision, [&](auto t) { HIP_TRY(launch_flip<decltype(t)>(fa, h->stream)); });
    if (e.p.reinit == LBM_WARM)  // removed and added cells, adjacent in sel
        with_storage(h->precision,
                     [&](auto t) { zero_cells<decltype(t)>(h, srem, 2 * (int)keff); });
    // the selections and removed densities, then the error flag the
    // selection kernels may have set
    const size_t rb = (size_t)keff * (sizeof(double) + 2 * sizeof(int32_t));
    e.rb_al = (rb + 7) / 8 * 8;
    ensure_pinned(h, e.rb_al + sizeof(double));
    HIP_TRY(hipMemcpyAsync(h->pinned, rrho, rb, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipMemcpyAsync(reinterpret_cast<char *>(h->pinned) + e.rb_al, err, sizeof(int),
                           hipMemcpyDeviceToHost, h->stream));
}

// After the wait: the removed mass in selection order, the whole-lattice
// reset (COLD), the wall links, and the constant-volume check on the host
// mirror as the flips apply (every removed cell must have been fluid and
// every added one solid, each listed once).
void exchange_finish(Exchange &e) {
    lbm_handle *h = e.h;
    const int64_t keff = e.keff, nf = e.nf;
    std::vector<int32_t> rem(std::max<int64_t>(keff, 0)), add(std::max<int64_t>(keff, 0));
    double mass_removed = 0.0;
    if (keff > 0) {
        if (*reinterpret_cast<const int *>(reinterpret_cast<const char *>(h->pinned) + e.rb_al)) {
            e.status = fail(LBM_EHIP, "the selection kernels found an inconsistent candidate list");
            return;
        }
        const double *rr = h->pinned;
        const int32_t *ix = reinterpret_cast<const int32_t *>(h->pinned + keff);
        std::memcpy(rem.data(), ix, keff * sizeof(int32_t));
        std::memcpy(add.data(), ix + keff, keff * sizeof(int32_t));
        for (int64_t k = 0; k < keff; ++k) mass_removed += rr[k];  // selection order
    }
    if (e.p.reinit == LBM_COLD) {
        with_storage(h->precision, [&](auto t) { reset_all<decltype(t)>(h); });
    }
    // the wall links around the flipped cells (removed then added, adjacent
    // in the selection buffer)
    if (keff > 0) {
        const int32_t *flipped = reinterpret_cast<const int32_t *>(h->sel.as<double>() + keff);
        HIP_TRY(launch_build_cells_at(h->types.as<uint8_t>(), h->cell.as<uint16_t>(), flipped,
                                      (int)(2 * keff), h->nx, h->ny, h->pitch, h->flags,
                                      h->stream));
    }
    int64_t nf_after = nf;
    for (int64_t k = 0; k < keff; ++k) {
        uint8_t &tr = h->host_types[rem[k]];
        nf_after -= tr == LBM_FLUID ? 1 : 0;
        tr = tr == LBM_FLUID ? (uint8_t)LBM_SOLID : (uint8_t)0xff;
    }
    for (int64_t k = 0; k < keff; ++k) {
        uint8_t &ta = h->host_types[add[k]];
        nf_after += ta == LBM_SOLID ? 1 : 0;
        ta = ta == LBM_SOLID ? (uint8_t)LBM_FLUID : (uint8_t)0xff;
    }
    for (int64_t k = 0; k < keff; ++k)
        if (h->host_types[rem[k]] == 0xff || h->host_types[add[k]] == 0xff) nf_after = -1;
    h->last_removed.assign(rem.begin(), rem.end());
    h->last_added.assign(add.begin(), add.end());
    if (keff > 0) {
        tilings_flip(h, rem, add);
        rebuild_tiles(h);
        refit_shape(h);
        ++h->mask_version;
    }
    e.r->k_eff = (int32_t)keff;
    e.r->n_fluid_after = nf_after;
    e.r->mass_removed = mass_removed;
    e.r->mass_added = (double)keff;
    if (nf_after != nf) e.status = fail(LBM_EHIP, "fluid volume changed by the exchange step");
}

// Run one phase on every exchange still going; a HIP or allocation failure
// ends that exchange only.
template <typename F>
void exchange_phase(std::vector<Exchange> &ex, F &&f) {
    for (Exchange &e : ex) {
        if (e.status != LBM_OK) continue;
        try {
            f(e);
        } catch (const HipFail &x) {
            e.status = guard_hip(x);
        } catch (const std::bad_alloc &) {
            e.status = fail(LBM_ENOMEM, "device allocation failed");
        }
    }
}

// Wait for the streams of the exchanges still going (each stream once).
void exchange_wait(std::vector<Exchange> &ex) {
    std::vector<hipStream_t> done;
    for (Exchange &e : ex) {
        if (e.status != LBM_OK) continue;
        if (std::find(done.begin(), done.end(), e.h->stream) != done.end()) continue;
        const hipError_t err = hipStreamSynchronize(e.h->stream);
        if (err != hipSuccess) {
            for (Exchange &o : ex)
                if (o.status == LBM_OK && o.h->stream == e.h->stream)
                    o.status = guard_hip(HipFail{err, "hipStreamSynchronize"});
        }
        done.push_back(e.h->stream);
    }
}

// Exchange steps on many handles, phase by phase: two waits in all (plus one
// per handle whose candidate list outgrew its capacity).
void exchange_all(std::vector<Exchange> &ex) {
    exchange_phase(ex, [](Exchange &e) { exchange_keys(e); });
    exchange_wait(ex);
    for (Exchange &e : ex) {
        if (e.status != LBM_OK || exchange_counts(e)) continue;
        // a list outgrew its capacity (now raised): recompute once
        std::vector<Exchange> one(1, e);
        exchange_phase(one, [](Exchange &x) { exchange_keys(x); });
        exchange_wait(one);
        e.status = one[0].status;
        if (e.status == LBM_OK && !exchange_counts(e))
            e.status = fail(LBM_EHIP, "candidate count changed between passes");
    }
    exchange_phase(ex, [](Exchange &e) { exchange_select(e); });
    exchange_wait(ex);
    exchange_phase(ex, [](Exchange &e) { exchange_finish(e); });
}

}  // namespace

extern "C" {

int lbm_shape_update(lbm_handle *h, const lbm_shape_params *p,
                     const double *rho_ux_uy, lbm_shape_result *r) {
    g_error.clear();
    const int rc = exchange_check(h, p, r);
    if (rc != LBM_OK) return rc;
    std::memset(r, 0, sizeof *r);
    std::vector<Exchange> ex(1);
    ex[0].h = h;
    ex[0].p = *p;
    ex[0].field = rho_ux_uy;
    ex[0].r = r;
    exchange_all(ex);
    if (ex[0].status != LBM_OK) return ex[0].status;
    return LBM_OK;
}

int lbm_shape_update_many(lbm_handle *const *hs, const lbm_shape_params *ps, int32_t n,
                          lbm_shape_result *rs, int32_t *status) {
    g_error.clear();
    if (n < 0 || (n > 0 && (!hs || !ps || !rs || !status)))
        return fail(LBM_EINVAL, "null array or negative count");
    std::vector<Exchange> ex(n);
    int worst = LBM_OK;
    for (int32_t k = 0; k < n; ++k) {
        for (int32_t j = 0; j < k; ++j)
            if (hs[j] == hs[k]) return fail(LBM_EINVAL, "a handle is listed twice");
        status[k] = exchange_check(hs[k], &ps[k], &rs[k]);
        if (status[k] == LBM_OK) std::memset(&rs[k], 0, sizeof rs[k]);
        ex[k].h = hs[k];
        ex[k].p = ps[k];
        ex[k].r = &rs[k];
        ex[k].status = status[k];
    }
    exchange_all(ex);
    for (int32_t k = 0; k < n; ++k) {
        status[k] = ex[k].status;
        if (status[k] < worst) worst = status[k];
    }
    return worst;
}

int lbm_last_exchange(lbm_handle *h, int64_t *removed, int64_t *added,
                      int32_t cap) {
    g_error.clear();
    if (!h) return fail(LBM_EINVAL, "null handle");
    const size_t k = h->last_removed.size();
    if ((size_t)std::max(cap, 0) < k || (k > 0 && (!removed || !added)))
        return fail(LBM_EINVAL, "cap smaller than the last exchange count");
    for (size_t i = 0; i < k; ++i) {
        removed[i] = h->last_removed[i];
        added[i] = h->last_added[i];
    }
    return (int)k;
}

int lbm_get_mask(lbm_handle *h, uint8_t *types, size_t n) {
    g_error.clear();
    if (!h || !types || n < h->N()) return fail(LBM_EINVAL, "bad arguments");
    try {
        HIP_TRY(hipSetDevice(h->device));
        HIP_TRY(hipMemcpyAsync(types, h->types.p, h->N(), hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
    } catch (const HipFail &e) {
        return guard_hip(e);
    }
    return LBM_OK;
}

int lbm_get_macro(lbm_handle *h, double *rho, double *ux, double *uy, size_t n) {
    g_error.clear();
    if (!h || !rho || !ux || !uy || n < h->N()) return fail(LBM_EINVAL, "bad arguments");
    try {
        HIP_TRY(hipSetDevice(h->device));
        macro_dispatch(h);
        const double *m = h->macro.as<double>();
        const size_t N = h->N();
        HIP_TRY(hipMemcpyAsync(rho, m, N * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipMemcpyAsync(ux, m + N, N * sizeof(double), hipMemcpyDeviceToHost,
                               h->stream));
        HIP_TRY(hipMemcpyAsync(uy, m + 2 * N, N * sizeof(double), hipMemcpyDeviceToHost,
                               h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
    } catch (const HipFail &e) {
        return guard_hip(e);
    } catch (const std::bad_alloc &) {
        return fail(LBM_ENOMEM, "allocation failed");
    }
    return LBM_OK;
}

int lbm_get_state(lbm_handle *h, double *f, size_t n) {
    g_error.clear();
    if (!h || !f || n < 9 * h->N()) return fail(LBM_EINVAL, "bad arguments");
    try {
        HIP_TRY(hipSetDevice(h->device));
        with_storage(h->precision, [&](auto t) { export_state<decltype(t)>(h, f); });
    } catch (const HipFail &e) {
        return guard_hip(e);
    } catch (const std::bad_alloc &) {
        return fail(LBM_ENOMEM, "allocation failed");
    }
    return LBM_OK;
}

int lbm_set_state(lbm_handle *h, const double *f, size_t n) {
    g_error.clear();
    if (!h || !f || n < 9 * h->N()) return fail(LBM_EINVAL, "bad arguments");
    try {
        HIP_TRY(hipSetDevice(h->device));
        with_storage(h->precision, [&](auto t) { import_state<decltype(t)>(h, f); });
        h->steps = 0;
        h->last_residual = std::nan("");
    } catch (const HipFail &e) {
        return guard_hip(e);
    } catch (const std::bad_alloc &) {
        return fail(LBM_ENOMEM, "allocation failed");
    }
    return LBM_OK;
}

int32_t lbm_tb_variant_count(int32_t precision) {
    if (precision < LBM_F64 || precision > LBM_F32_S_BF16) return 0;
    return tb_variant_count(precision);
}

int lbm_tb_variant_info(int32_t precision, int32_t variant, int32_t *rows, int32_t *halo,
                        int32_t *tile_w, int32_t *tile_h) {
    g_error.clear();
    if (variant < 0 || variant >= lbm_tb_variant_count(precision))
        return fail(LBM_EINVAL, "unknown precision or shape");
    const TbVariant v = tb_shape(precision, variant);
    if (rows) *rows = v.rows;
    if (halo) *halo = v.halo;
    if (tile_w) *tile_w = tile_width(precision, variant);
    if (tile_h) *tile_h = tile_height(precision, variant);
    return LBM_OK;
}

int lbm_tb_variant_kind(int32_t precision, int32_t variant, int32_t *kind,
                        int32_t *lds_bytes) {
    g_error.clear();
    if (variant < 0 || variant >= lbm_tb_variant_count(precision))
        return fail(LBM_EINVAL, "unknown precision or shape");
    const TbVariant v = tb_shape(precision, variant);
    if (kind) *kind = v.kind;
    // the region copies (one when updated in place), plus the compacted list
    if (lds_bytes) *lds_bytes = (int32_t)shape_lds_bytes(precision, variant);
    return LBM_OK;
}

int lbm_precision_info(int32_t precision, int32_t *storage_bytes, int32_t *arith_bytes) {
    g_error.clear();
    if (precision < LBM_F64 || precision > LBM_F32_S_BF16 || !storage_bytes || !arith_bytes)
        return fail(LBM_EINVAL, "unknown precision or null pointer");
    with_storage(precision, [&](auto t) {
        using T = decltype(t);
        *storage_bytes = (int32_t)sizeof(T);
        *arith_bytes = (int32_t)sizeof(ArithT<T>);
    });
    return LBM_OK;
}

int lbm_get_tb_variant(lbm_handle *h, int32_t *variant) {
    g_error.clear();
    if (!h || !variant) return fail(LBM_EINVAL, "null argument");
    *variant = h->use_tb ? h->tb_variant : -1;
    return LBM_OK;
}

int lbm_set_tb_variant(lbm_handle *h, int32_t variant) {
    g_error.clear();
    if (!h) return fail(LBM_EINVAL, "null handle");
    if (variant < 0 || variant >= tb_variant_count(h->precision))
        return fail(LBM_EINVAL, "shape out of range");
    try {
        HIP_TRY(hipSetDevice(h->device));
        h->tb_variant = variant;
        h->tuned_variant = -1;
        h->tune_ms.clear();  // an explicit choice is kept through exchange steps
        rebuild_tiles(h);
    } catch (const HipFail &e) {
        return guard_hip(e);
    } catch (const std::bad_alloc &) {
        return fail(LBM_ENOMEM, "allocation failed");
    }
    return LBM_OK;
}

int lbm_autotune(lbm_handle *h, int32_t trial_steps, int32_t *best, double *ms,
                 int32_t ms_cap) {
    g_error.clear();
    if (!h || trial_steps < 1) return fail(LBM_EINVAL, "null handle or trial_steps < 1");
    const int nv = tb_variant_count(h->precision);
    if (ms && ms_cap < nv) return fail(LBM_EINVAL, "ms_cap below the shape count");
    try {
        HIP_TRY(hipSetDevice(h->device));
        Saved sv;
        save_state(h, sv);
        int bv = h->tb_variant;
        double bms = INFINITY;
        std::vector<double> times(nv);
        for (int v = 0; v < nv; ++v) {
            h->tb_variant = v;
            rebuild_tiles(h);
            const double t = with_storage(h->precision, [&](auto x) {
                return time_handle_steps<decltype(x)>(h, trial_steps);
            });
            restore_state(h, sv);
            times[v] = t;
            if (ms) ms[v] = t;
            if (t < bms) {
                bms = t;
                bv = v;
            }
        }
        h->tb_variant = bv;
        h->tuned_variant = bv;
        rebuild_tiles(h);
        h->tune_ms = times;
        h->tune_fit = (size_t)h->n_tiles <= resident_tiles(h, bv);
        HIP_TRY(hipStreamSynchronize(h->stream));
        if (best) *best = bv;
    } catch (const HipFail &e) {
        return guard_hip(e);
    } catch (const std::bad_alloc &) {
        return fail(LBM_ENOMEM, "allocation failed");
    }
    return LBM_OK;
}

int lbm_batch_create(lbm_handle *const *handles, int32_t count, void *hip_stream,
                     lbm_batch **out) {
    g_error.clear();
    if (!out) return fail(LBM_EINVAL, "null output pointer");
    *out = nullptr;
    if (!handles || count < 1) return fail(LBM_EINVAL, "at least one handle required");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(LBM_EHIP, "no current device");
    for (int32_t i = 0; i < count; ++i) {
        if (!handles[i]) return fail(LBM_EINVAL, "null handle in the list");
        if (handles[i]->precision != handles[0]->precision)
            return fail(LBM_EINVAL, "handles of different precision");
        if (handles[i]->device != dev)
            return fail(LBM_EINVAL, "handle not on the current device");
        for (int32_t j = 0; j < i; ++j)
            if (handles[j] == handles[i]) return fail(LBM_EINVAL, "handle listed twice");
    }
    lbm_batch *b = new (std::nothrow) lbm_batch;
    if (!b) return fail(LBM_ENOMEM, "host allocation failed");
    try {
        b->hs.assign(handles, handles + count);
        for (int32_t i = 0; i < count; ++i) b->bc = b->bc || handles[i]->flags != 0;
        b->versions.assign((size_t)count, 0);
        b->precision = handles[0]->precision;
        b->device = dev;
        b->stream = static_cast<hipStream_t>(hip_stream);
        const char *g = std::getenv("LBM_GRAPHS");
        b->use_graphs = !(g && g[0] == '0');
        const size_t args_bytes = with_storage(b->precision, [&](auto t) {
            return 2 * (size_t)count * sizeof(SweepArgs<decltype(t)>);
        });
        b->args.ensure(args_bytes);
        build_work(b);
    } catch (const std::bad_alloc &) {
        delete b;
        return fail(LBM_ENOMEM, "device allocation failed");
    } catch (const HipFail &e) {
        delete b;
        return guard_hip(e);
    }
    *out = b;
    return LBM_OK;
}

int lbm_batch_run(lbm_batch *b, int64_t steps, double *elapsed_ms) {
    g_error.clear();
    if (!b || steps < 0) return fail(LBM_EINVAL, "null batch or steps < 0");
    try {
        HIP_TRY(hipSetDevice(b->device));
        const double ms = with_storage(b->precision, [&](auto t) {
            return batch_run_impl<decltype(t)>(b, steps);
        });
        if (elapsed_ms) *elapsed_ms = ms;
    } catch (const HipFail &e) {
        return guard_hip(e);
    } catch (const std::bad_alloc &) {
        return fail(LBM_ENOMEM, "allocation failed");
    }
    return LBM_OK;
}

int lbm_batch_configure(lbm_batch *b, int32_t variant, int32_t order) {
    g_error.clear();
    if (!b) return fail(LBM_EINVAL, "null batch");
    if (variant < 0 || variant > tb_variant_count(b->precision) || order < 0 || order > 1)
        return fail(LBM_EINVAL, "shape or order out of range");
    if (variant != b->variant || order != b->order) {
        b->variant = variant;
        b->order = order;
        b->dirty = true;
    }
    return LBM_OK;
}

int lbm_batch_tune(lbm_batch *b, int32_t trial_steps, int32_t *best_variant,
                   int32_t *best_order, double *ms, int32_t ms_cap) {
    g_error.clear();
    if (!b || trial_steps < 1) return fail(LBM_EINVAL, "null batch or trial_steps < 1");
    const int nv = tb_variant_count(b->precision) + 1;  // shapes + single step
    if (ms && ms_cap < 2 * nv) return fail(LBM_EINVAL, "ms_cap below 2 x (shape count + 1)");
    try {
        HIP_TRY(hipSetDevice(b->device));
        std::vector<Saved> sv(b->hs.size());
        for (size_t i = 0; i < b->hs.size(); ++i) save_state(b->hs[i], sv[i]);
        for (lbm_handle *h : b->hs) HIP_TRY(hipStreamSynchronize(h->stream));
        int bv = b->variant, bo = b->order;
        double bms = INFINITY;
        for (int v = 0; v < nv; ++v)
            for (int o = 0; o < 2; ++o) {
                b->variant = v;
                b->order = o;
                b->dirty = true;
                const int H = batch_steps_per_launch(b);
                const double t = with_storage(b->precision, [&](auto x) {
                    batch_run_impl<decltype(x)>(b, H);  // untimed
                    return batch_run_impl<decltype(x)>(b, trial_steps) / trial_steps;
                });
                for (size_t i = 0; i < b->hs.size(); ++i) restore_state(b->hs[i], sv[i]);
                for (lbm_handle *h : b->hs) HIP_TRY(hipStreamSynchronize(h->stream));
                if (ms) ms[2 * v + o] = t;
                if (t < bms) {
                    bms = t;
                    bv = v;
                    bo = o;
                }
            }
        b->variant = bv;
        b->order = bo;
        b->dirty = true;
        build_work(b);
        if (best_variant) *best_variant = bv;
        if (best_order) *best_order = bo;
    } catch (const HipFail &e) {
        return guard_hip(e);
    } catch (const std::bad_alloc &) {
        return fail(LBM_ENOMEM, "allocation failed");
    }
    return LBM_OK;
}

int lbm_batch_info(lbm_batch *b, int64_t *items, int32_t *steps_per_launch_out,
                   int64_t *nonsolid_cells) {
    g_error.clear();
    if (!b) return fail(LBM_EINVAL, "null batch");
    try {
        HIP_TRY(hipSetDevice(b->device));
        if (work_stale(b)) build_work(b);
    } catch (const HipFail &e) {
        return guard_hip(e);
    } catch (const std::bad_alloc &) {
        return fail(LBM_ENOMEM, "allocation failed");
    }
    if (items) *items = b->n_real;
    if (steps_per_launch_out) *steps_per_launch_out = batch_steps_per_launch(b);
    if (nonsolid_cells) {
        int64_t c = 0;
        for (const lbm_handle *h : b->hs) c += h->n_nonsolid;
        *nonsolid_cells = c;
    }
    return LBM_OK;
}

void lbm_batch_destroy(lbm_batch *b) {
    if (!b) return;
    (void)hipSetDevice(b->device);
    if (hipStreamSynchronize(b->stream) == hipSuccess) {  // nothing queued reads them now
        b->args.recycle();
        b->lat.recycle();
        b->tiles.recycle();
        if (b->pinned) host_cache().give(-1, b->pinned_bytes, b->pinned);
        b->pinned = nullptr;
        b->pinned_bytes = 0;
    }
    delete b;
}

int lbm_batch_set_graphs(lbm_batch *b, int32_t enable) {
    g_error.clear();
    if (!b) return fail(LBM_EINVAL, "null batch");
    b->use_graphs = enable != 0;
    if (!b->use_graphs) b->drop_graphs();
    return LBM_OK;
}

int lbm_state_digest(lbm_handle *h, uint64_t *digest) {
    g_error.clear();
    if (!h || !digest) return fail(LBM_EINVAL, "null argument");
    try {
        HIP_TRY(hipSetDevice(h->device));
        ensure_pinned(h, 64 * sizeof(double));
        unsigned long long *acc = h->red.as<unsigned long long>() + 52;
        HIP_TRY(hipMemsetAsync(acc, 0, sizeof(unsigned long long), h->stream));
        with_storage(h->precision, [&](auto t) {
            using T = decltype(t);
            HIP_TRY(launch_digest<T>(h->f[h->cur].as<T>(), h->cell.as<uint16_t>(),
                                     h->types.as<uint8_t>(), h->nx, h->ny, h->pitch, h->plane,
                                     acc, h->stream));
        });
        HIP_TRY(hipMemcpyAsync(h->pinned, acc, sizeof(unsigned long long),
                               hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        *digest = *reinterpret_cast<const uint64_t *>(h->pinned);
    } catch (const HipFail &e) {
        return guard_hip(e);
    } catch (const std::bad_alloc &) {
        return fail(LBM_ENOMEM, "allocation failed");
    }
    return LBM_OK;
}

}  // extern "C"
