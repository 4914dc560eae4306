// C ABI and host-side orchestration of one time step (single-process form of
// Alg. 2: detection, colouring, accumulator init, NBGS sweeps, integration).
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <new>
#include <algorithm>

#include "scene.h"

namespace nbgs {

namespace {
thread_local std::string g_last_error;
}

const char *last_error_cstr() { return g_last_error.c_str(); }

void set_error(const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

}  // namespace nbgs

namespace nbgs {

// ------------------------------------------------------------------ arena

void Arena::reset(void *base, size_t bytes) {
    free_.clear();
    live_.clear();
    moved_.clear();
    used_ = peak_ = 0;
    base_ = nullptr;
    size_ = 0;
    const uintptr_t b = reinterpret_cast<uintptr_t>(base);
    const uintptr_t a = (b + kAlign - 1) & ~(uintptr_t)(kAlign - 1);
    if (!base || bytes < (a - b) + kAlign) return;
    base_ = reinterpret_cast<char *>(a);
    size_ = (bytes - (a - b)) & ~(size_t)(kAlign - 1);
    free_[0] = size_;
}

void *Arena::alloc(size_t bytes, ArenaBuf *owner) {
    if (!base_) return nullptr;
    const size_t len = (bytes + kAlign - 1) & ~(size_t)(kAlign - 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second < len) continue;
        const size_t off = it->first, rest = it->second - len;
        free_.erase(it);
        if (rest) free_[off + len] = rest;
        live_[off] = {len, owner};
        used_ += len;
        peak_ = std::max(peak_, used_);
        return base_ + off;
    }
    return nullptr;
}

void Arena::release(void *p) {
    if (!p || !base_) return;
    const size_t off = (size_t)(static_cast<char *>(p) - base_);
    auto it = live_.find(off);
    if (it == live_.end()) return;
    size_t start = off, len = it->second.first;
    used_ -= len;
    live_.erase(it);
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && nx->first == off + len) {  // join the free run after it
        len += nx->second;
        nx = free_.erase(nx);
    }
    if (nx != free_.begin()) {  // and the one before it
        auto pv = std::prev(nx);
        if (pv->first + pv->second == start) {
            start = pv->first;
            len += pv->second;
            free_.erase(pv);
        }
    }
    free_[start] = len;
}

nbgs_status Arena::move_to(void *base, size_t bytes, hipStream_t s) {
    Arena fresh;
    fresh.reset(base, bytes);
    if (!fresh.bound()) {
        set_error("the new workspace is NULL or smaller than %zu bytes", (size_t)kAlign);
        return NBGS_ERR_INVALID_ARG;
    }
    if (base_ && fresh.base_ < base_ + size_ && fresh.base_ + fresh.size_ > base_) {
        set_error("the new workspace overlaps the current one");
        return NBGS_ERR_INVALID_ARG;
    }
    size_t need = 0;
    for (const auto &kv : live_) need += kv.second.first;
    if (need > fresh.size_) {
        set_error("the new workspace (%zu bytes) cannot hold the %zu bytes in use", fresh.size_, need);
        return NBGS_ERR_CAPACITY;
    }
    std::vector<std::array<uintptr_t, 3>> moved;
    std::map<size_t, std::pair<size_t, ArenaBuf *>> live;
    size_t off = 0;
    for (const auto &kv : live_) {
        const size_t len = kv.second.first;
        char *src = base_ + kv.first, *dst = fresh.base_ + off;
        NBGS_HIP(hipMemcpyAsync(dst, src, len, hipMemcpyDeviceToDevice, s));
        moved.push_back({reinterpret_cast<uintptr_t>(src), reinterpret_cast<uintptr_t>(src) + len,
                         reinterpret_cast<uintptr_t>(dst)});
        live[off] = kv.second;
        off += len;
    }
    NBGS_HIP(hipStreamSynchronize(s));
    for (const auto &kv : live) kv.second.second->arena_moved(fresh.base_ + kv.first);
    base_ = fresh.base_;
    size_ = fresh.size_;
    live_ = std::move(live);
    free_.clear();
    if (off < size_) free_[off] = size_ - off;
    used_ = off;
    peak_ = std::max(peak_, used_);
    moved_ = std::move(moved);
    g_alloc_generation.fetch_add(1, std::memory_order_relaxed);
    return NBGS_OK;
}

const void *Arena::relocate(const void *old) const {
    const uintptr_t a = reinterpret_cast<uintptr_t>(old);
    for (const auto &m : moved_)
        if (a >= m[0] && a < m[1]) return reinterpret_cast<const void *>(m[2] + (a - m[0]));
    return old;
}

// Upper bound of a sphere scene's device memory (nbgs_workspace_query): every
// buffer at its largest size for n bodies in `scenes` scenes and c contacts,
// with the growth slack of the buffers that grow, in every sweep order,
// precision and warm start.  Per body 567 B (detection 180 B, accumulator
// records of both precisions 96 B, block and subdomain tables of blocks
// holding eight bodies or more on average 165 B, cell ranges of 8 B and
// their occupancy bits at most eight per body 82 B, the touched flags of the
// few-contact solve 1 B, and the rest); per
// contact 1000 B (two contact tables 192 B, sweep
// records of both precisions 168 B, colouring 36 B, learned start 156 B,
// subdomain ends, slots and corrections 208 B, partial sums and tuning copies
// 40 B, times 1.25); per scene its cell table of at least 2^16 cells and its
// tables; a fixed 16 MiB (residual history of 131,072 sweeps, sort
// scratch); ten per cent for the alignment of every buffer and for runs left
// between freed buffers.  The per-id tables of the block-local order and of the
// subdomain solver come on top (scene_need_bytes).
size_t scene_workspace_bytes(int64_t n, int64_t c, int64_t scenes) {
    const double per_body = 567.0, per_contact = 1000.0, per_scene = 65536.0 * 9.0 * 1.25 + 4096.0;
    const double fixed = 16.0 * 1024.0 * 1024.0;
    const double b = 1.1 * (per_body * (double)n + per_contact * (double)c + per_scene * (double)scenes + fixed);
    return ((size_t)b + Arena::kAlign - 1) & ~(size_t)(Arena::kAlign - 1);  // all of it usable at an aligned base
}

// Per id of the block-local order or of the subdomain solver: contact range
// (8 B), its count (4 B), slot count and range (8 B), colour runs and their
// count (8 B), residual partial sums (16 B), scan scratch, times 1.25 for the
// growth slack, rounded up.
constexpr double kPerIdBytes = 80.0;
constexpr double kRecPerBody = 3.0 * 4.0;

nbgs_status scene_need_bytes(nbgs_scene_t sc, int64_t c, size_t *bytes) {
    int64_t ids = 0;
    NBGS_TRY(order_ids(sc, &ids));
    const size_t id_bytes = ids > 0 ? (size_t)(1.1 * kPerIdBytes * (double)(ids + 2)) : 0;
    // the block-local order's record layout: per body its three index tables, per contact its two ends as records
    // and its at most two slots
    const size_t rec_bytes =
        sc->blk_edge > 0.0 ? (size_t)(1.1 * (kRecPerBody * (double)sc->b.n + 16.0 * (double)c) + 8 * Arena::kAlign) : 0;
    *bytes = scene_workspace_bytes(sc->b.n, c, sc->n_scenes) +
             ((id_bytes + Arena::kAlign - 1) & ~(size_t)(Arena::kAlign - 1)) +
             ((rec_bytes + Arena::kAlign - 1) & ~(size_t)(Arena::kAlign - 1));
    return NBGS_OK;
}

nbgs_status check_params(const nbgs_params *p) {
    if (!p) {
        set_error("params is NULL");
        return NBGS_ERR_INVALID_ARG;
    }
    if (!(p->dt > 0.0) || !std::isfinite(p->dt)) {
        set_error("dt must be positive and finite");
        return NBGS_ERR_INVALID_ARG;
    }
    if (!(p->relax > 0.0 && p->relax <= 1.0)) {
        set_error("relax must lie in (0, 1]");
        return NBGS_ERR_INVALID_ARG;
    }
    if (!(p->erp >= 0.0 && p->erp <= 1.0)) {
        set_error("erp must lie in [0, 1]");
        return NBGS_ERR_INVALID_ARG;
    }
    if (!(p->mu >= 0.0) || !std::isfinite(p->mu)) {
        set_error("mu must be non-negative");
        return NBGS_ERR_INVALID_ARG;
    }
    if (!(p->tau >= 0.0) || !std::isfinite(p->tau)) {
        set_error("tau must be non-negative");
        return NBGS_ERR_INVALID_ARG;
    }
    if (p->precision != NBGS_FP64 && p->precision != NBGS_FP32_SWEEP) {
        set_error("unknown precision %d", p->precision);
        return NBGS_ERR_INVALID_ARG;
    }
    if (p->warm_start != NBGS_WS_ZERO && p->warm_start != NBGS_WS_PREVIOUS && p->warm_start != NBGS_WS_LEARNED) {
        set_error("unknown warm start mode %d", p->warm_start);
        return NBGS_ERR_INVALID_ARG;
    }
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(p->gravity[a])) {
            set_error("gravity must be finite");
            return NBGS_ERR_INVALID_ARG;
        }
    return NBGS_OK;
}

nbgs_status check_domain(const nbgs_domain *domain) {
    if (!domain) {
        set_error("domain is NULL");
        return NBGS_ERR_INVALID_ARG;
    }
    if (domain->n_planes < 0 || domain->n_planes > PlaneSet::kMax || (domain->n_planes > 0 && !domain->planes)) {
        set_error("n_planes must lie in [0, %d] with a plane array", PlaneSet::kMax);
        return NBGS_ERR_INVALID_ARG;
    }
    for (int a = 0; a < 3; ++a)
        if (!(domain->hi[a] > domain->lo[a]) || !std::isfinite(domain->hi[a] - domain->lo[a])) {
            set_error("domain box must have hi > lo on every axis");
            return NBGS_ERR_INVALID_ARG;
        }
    for (int w = 0; w < domain->n_planes; ++w) {
        const double *nm = domain->planes[w].normal;
        const double len = std::sqrt(nm[0] * nm[0] + nm[1] * nm[1] + nm[2] * nm[2]);
        if (!(std::fabs(len - 1.0) < 1e-12)) {
            set_error("plane %d normal is not unit length", w);
            return NBGS_ERR_INVALID_ARG;
        }
    }
    return NBGS_OK;
}

PlaneSet plane_set(const nbgs_domain *domain) {
    PlaneSet ps{};
    ps.n = domain->n_planes;
    for (int w = 0; w < domain->n_planes; ++w)
        for (int a = 0; a < 3; ++a) {
            ps.p[w][a] = domain->planes[w].point[a];
            ps.nrm[w][a] = domain->planes[w].normal[a];
        }
    return ps;
}

int bits_for(int64_t n) {
    int b = 0;
    while (((int64_t)1 << b) < n) ++b;
    return b;
}

// Cell grid of one box for the largest hull diameter 2 max(r + h), with at
// most max(8 n, 2^16) cells for n bodies.
Grid grid_for_box(const double lo[3], const double hi[3], const int32_t periodic[3], int64_t n, double max_reach) {
    Grid g{};
    const double cell = 2.0 * max_reach * (1.0 + 1e-9);
    int64_t dims[3];
    double edge[3];
    for (int a = 0; a < 3; ++a) {
        const double L = hi[a] - lo[a];
        g.lo[a] = lo[a];
        g.hi[a] = hi[a];
        g.L[a] = L;
        g.periodic[a] = periodic[a];
        double c = std::floor(L / cell);
        if (!(c >= 1.0)) c = 1.0;
        if (c > 1.0e6) c = 1.0e6;
        if (periodic[a] && c < 3.0) c = 1.0;  // one cell: every partner is tested by minimum image
        dims[a] = (int64_t)c;
        edge[a] = periodic[a] ? L / c : cell;
    }
    // keep the table within a few cells per body (a finer grid means fewer hull tests; the neighbour search reads
    // the records of occupied cells only)
    const int64_t cap = std::max<int64_t>(8 * n, 1 << 16);
    while (dims[0] * dims[1] * dims[2] > cap) {
        for (int a = 0; a < 3; ++a) {
            if (dims[a] <= 1) continue;
            int64_t c = std::max<int64_t>(1, dims[a] / 2);
            if (periodic[a] && c < 3) c = 1;
            dims[a] = c;
            edge[a] = periodic[a] ? g.L[a] / (double)c : edge[a] * 2.0;
        }
    }
    for (int a = 0; a < 3; ++a) {
        g.dims[a] = (int32_t)dims[a];
        g.edge[a] = edge[a];
    }
    g.ncells = (int32_t)(dims[0] * dims[1] * dims[2]);
    g.key_bits = bits_for(g.ncells);
    g.cell_off = 0;
    const int32_t identity[3] = {0, 1, 2};
    grid_set_axes(g, identity);
    return g;
}

void grid_set_axes(Grid &g, const int32_t axis[3]) {
    for (int k = 0; k < 3; ++k) {
        g.axis[k] = axis[k];
        g.kdims[k] = g.dims[axis[k]];
        g.kperiodic[k] = g.periodic[axis[k]];
    }
}

}  // namespace nbgs

using namespace nbgs;

namespace {


void update_scales(nbgs_scene_t sc) {
    const double g = std::sqrt(sc->p.gravity[0] * sc->p.gravity[0] + sc->p.gravity[1] * sc->p.gravity[1] +
                               sc->p.gravity[2] * sc->p.gravity[2]);
    sc->fs.vs = g * sc->p.dt > 0.0 ? g * sc->p.dt : 1e-3;
    sc->fs.ms = sc->mean_mass;
    sc->fs.rs = sc->mean_radius;
}

void record(nbgs_scene_t sc, int i) {
    if (sc->ev[i]) sc->ev_ok[i] = hipEventRecord(sc->ev[i], sc->s) == hipSuccess;
}



// The scene's grid, or for batched scenes one grid per scene laid out one
// after another in a shared cell table (sc->grid then only carries the total
// cell count and key width).
// The key order of the cell grid: the axis along which the caller's numbering
// advances fastest runs fastest in the keys, so that the sorted order follows
// the numbering as far as it can and the gathers by body index in sorted order
// read neighbouring records (a lattice numbered with z fastest would otherwise
// be read two megabytes apart).  The numbering advances along an axis when
// consecutive bodies step along it: measured once, on the first detection, as
// the mean |x_{i+1} - x_i| per axis over up to 2^22 pairs, the largest first;
// an axis other than x leads only when its mean is more than twice x's (a
// numbering that follows no axis keeps x fastest).
nbgs_status choose_key_axes(nbgs_scene_t sc) {
    if (sc->key_axes_set) return NBGS_OK;
    sc->key_axes_set = true;
    const int64_t pairs = std::min<int64_t>((int64_t)sc->b.n - 1, (int64_t)1 << 22);
    if (pairs < 64) return NBGS_OK;
    constexpr int kBlocks = 256;
    DevBuf<double> part;
    NBGS_TRY(part.reserve(3 * kBlocks, 1.0));
    NBGS_TRY(launch_numbering_steps(sc->b, pairs, part.p, kBlocks, sc->s));
    std::vector<double> h(3 * kBlocks);
    NBGS_HIP(hipMemcpyAsync(h.data(), part.p, sizeof(double) * 3 * kBlocks, hipMemcpyDeviceToHost, sc->s));
    NBGS_HIP(hipStreamSynchronize(sc->s));
    double m[3] = {0.0, 0.0, 0.0};
    for (int b = 0; b < kBlocks; ++b)
        for (int a = 0; a < 3; ++a) m[a] += h[(size_t)3 * b + a];
    int order[3] = {0, 1, 2};
    std::sort(order, order + 3, [&](int a, int c) { return m[a] > m[c] || (m[a] == m[c] && a < c); });
    if (!(order[0] != 0 && m[order[0]] > 2.0 * m[0])) {  // keep x fastest unless another axis clearly leads
        order[0] = 0;
        order[1] = m[1] >= m[2] ? 1 : 2;
        order[2] = 3 - order[1];
    }
    for (int k = 0; k < 3; ++k) sc->key_axes[k] = order[k];
    return NBGS_OK;
}

nbgs_status make_grid(nbgs_scene_t sc, double max_reach) {
    NBGS_TRY(choose_key_axes(sc));
    if (sc->n_scenes <= 1) {
        sc->grid = grid_for_box(sc->lo, sc->hi, sc->periodic, sc->b.n, max_reach);
        grid_set_axes(sc->grid, sc->key_axes);
        return NBGS_OK;
    }
    int64_t off = 0;
    for (int s = 0; s < sc->n_scenes; ++s) {
        const int64_t ns = sc->body_off_h[s + 1] - sc->body_off_h[s];
        Grid g = grid_for_box(&sc->lo_h[3 * s], &sc->hi_h[3 * s], &sc->periodic_h[3 * s], ns, max_reach);
        grid_set_axes(g, sc->key_axes);
        g.cell_off = (uint32_t)off;
        off += g.ncells;
        if (off > (int64_t)0x7fffffff) {
            set_error("the cell tables of the batched scenes exceed 2^31 cells");
            return NBGS_ERR_CAPACITY;
        }
        sc->grids_pinned[s] = g;
    }
    Grid total{};
    total.ncells = (int32_t)off;
    total.key_bits = bits_for(off);
    sc->grid = total;
    NBGS_HIP(hipMemcpyAsync(sc->grids_d.p, sc->grids_pinned, sizeof(Grid) * sc->n_scenes, hipMemcpyHostToDevice,
                            sc->s));
    return NBGS_OK;
}

template <class T>
SweepBuf<T> &sweep_buf(nbgs_scene_t sc);
template <>
SweepBuf<double> &sweep_buf<double>(nbgs_scene_t sc) {
    return sc->sw64;
}
template <>
SweepBuf<float> &sweep_buf<float>(nbgs_scene_t sc) {
    return sc->sw32;
}
template <class T>
DevBuf<T> &vel_buf(nbgs_scene_t sc);
template <>
DevBuf<double> &vel_buf<double>(nbgs_scene_t sc) {
    return sc->vel64;
}
template <>
DevBuf<float> &vel_buf<float>(nbgs_scene_t sc) {
    return sc->vel32;
}

// body -> solver record while the records are in the block-local sweeps' order, else null (body order)
const int32_t *rec_map(nbgs_scene_t sc) { return sc->rec_on ? sc->rec_of.p : nullptr; }

template <class T>
DevBuf<T> &corr_buf(nbgs_scene_t sc);
template <>
DevBuf<double> &corr_buf<double>(nbgs_scene_t sc) {
    return sc->corr64;
}
template <>
DevBuf<float> &corr_buf<float>(nbgs_scene_t sc) {
    return sc->corr32;
}

nbgs_status sync_small(nbgs_scene_t sc, int first, int count) {
    NBGS_HIP(hipMemcpyAsync(sc->pinned + first, sc->small.p + first, sizeof(int32_t) * count, hipMemcpyDeviceToHost,
                            sc->s));
    NBGS_HIP(hipStreamSynchronize(sc->s));
    return NBGS_OK;
}

// The last completed sweep's residual, staged beside the control words so that
// one copy brings both to the host.
__global__ void __launch_bounds__(64) k_last_residual(const int32_t *ctrl, const double *hist, double *out) {
    if (threadIdx.x != 0) return;
    const int32_t k = ctrl[1];
    out[0] = k > 0 ? hist[k - 1] : 0.0;
}

// Stop flag, sweeps completed, numeric-error flag and the last residual of a
// solve in one host round trip.
nbgs_status read_solve_result(nbgs_scene_t sc, int32_t &sweeps, double &R) {
    k_last_residual<<<1, 64, 0, sc->s>>>(sc->ctrl(), sc->res_hist.p, reinterpret_cast<double *>(sc->small.p + 12));
    NBGS_HIP(hipGetLastError());
    NBGS_TRY(sync_small(sc, 8, 6));
    sweeps = sc->pinned[8 + 1];
    R = 0.0;
    if (sweeps > 0) std::memcpy(&R, sc->pinned + 12, sizeof(double));
    return NBGS_OK;
}

template <class T>
nbgs_status gather_for_sweeps(nbgs_scene_t sc, bool indices) {
    SweepBuf<T> &sw = sweep_buf<T>(sc);
    sw.per_contact_mu = sc->n_scenes > 1;
    sw.sub = sc->sub_active || sc->blk_active;
    NBGS_TRY(sw.reserve((size_t)sc->nc));
    return launch_gather_sweep<T>(sc->cb[sc->cur].view(), sc->perm, sw.sub ? sc->sdom.p : nullptr, sc->nc,
                                  sc->p.dt, sc->p.erp, sc->table(), sw.view(), indices, sc->s);
}

nbgs_status colour_and_order(nbgs_scene_t sc, ContactBuf &cb, const SceneTable &tab, const int32_t *sdom,
                             bool warm_colours);

// The broad and narrow phase on the cell grid (Sect. 4) with hull radii `hull`
// and the largest reach `reach`: cell keys, sort, cell ranges, pair counts and
// their scan; *total = the pair count, checked against the 32-bit and
// candidate limits.  The emit follows separately.
static nbgs_status grid_pairs(nbgs_scene_t sc, const double *hull, double reach, int64_t *total) {
    hipStream_t s = sc->s;
    const int32_t N = sc->b.n;
    NBGS_TRY(make_grid(sc, reach));
    const SceneTable tab = sc->table();
    NBGS_HIP(hipMemsetAsync(sc->maxbits.p + 1, 0, 2 * sizeof(unsigned long long), s));
    NBGS_TRY(launch_cell_keys(sc->b, sc->grid, tab, hull, sc->keys.p, sc->ids.p, sc->xr.p, s));
    bool alt = false;
    NBGS_TRY(radix_sort_pairs(sc->keys.p, sc->ids.p, sc->keys2.p, sc->ids2.p, N, sc->grid.key_bits,
                              sc->radix_hist.p, sc->scan_tmp.p, sc->scan_tmp.cap, &alt, s));
    sc->skeys = alt ? sc->keys2.p : sc->keys.p;
    sc->sids = alt ? sc->ids2.p : sc->ids.p;
    // cell ranges (entries of occupied cells are rewritten every step) and the occupancy bitmap
    NBGS_TRY(sc->cells.reserve(sc->grid.ncells));
    NBGS_TRY(sc->occ.reserve(((size_t)sc->grid.ncells + 31) / 32));
    NBGS_TRY(launch_cells(N, sc->grid.ncells, sc->skeys, sc->sids, sc->xr.p, sc->cells.p, sc->occ.p, sc->sxr.p, s));
    // count, scan
    NBGS_TRY(launch_pair_count(sc->b, sc->grid, sc->planes, tab, sc->p.tau, sc->skeys, sc->sids, sc->sxr.p, hull,
                               sc->cells.p, sc->occ.p, sc->cnt.p,
                               sc->npart.p, sc->partners.p, sc->cellpos.p, sc->maxbits.p + 1, s));
    NBGS_TRY(exclusive_scan_i32(sc->cnt.p, sc->off.p, N, sc->total(), sc->scan_tmp.p, sc->scan_tmp.cap, s));
    NBGS_HIP(hipMemcpyAsync(sc->pinned + 4, sc->maxbits.p + 1, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                            s));
    NBGS_TRY(sync_small(sc, 0, 1));
    unsigned long long total64 = 0, over = 0;
    std::memcpy(&total64, sc->pinned + 4, sizeof(total64));
    std::memcpy(&over, sc->pinned + 6, sizeof(over));
    if (over) {
        set_error("a body meets more than 2^18 hull candidates in its 27 cells: the cell grid, sized by the largest "
                  "hull (radius %g), is too coarse for this state (a diverged solve or a very fast body)",
                  reach);
        return NBGS_ERR_CAPACITY;
    }
    if (total64 > 0x7fffff00ull) {
        set_error("%llu contacts exceed the 2^31 entries of the contact list (largest hull radius %g)",
                  (unsigned long long)total64, reach);
        return NBGS_ERR_CAPACITY;
    }
    if (sc->pinned[0] != (int32_t)total64) {
        set_error("contact count %lld disagrees with its 64-bit total %llu", (long long)sc->pinned[0],
                  (unsigned long long)total64);
        return NBGS_ERR_DEVICE;
    }
    *total = (int64_t)total64;
    return NBGS_OK;
}

// The pair list: every pair (and body-wall pair) whose reaches with hull radius
// `skin` overlap, in canonical order, built by the grid phase with that hull;
// with it the positions, radii and static flags of the build.  A later step
// tests these pairs only, as long as every body's displacement plus hull plus
// radius growth stays below the skin (checked by the hull pass): a pair further
// apart than r_i + r_k + 2 skin at the build cannot overlap its hulls then, and
// a wall further than skin + tau cannot be met.  The contacts are those of the
// grid phase, bit for bit (the same predicates on the same values); the list
// saves the sort and the neighbour search of the steps in between.  It is kept
// only when the workspace has room for it; otherwise every step uses the grid.
// Bytes of the pair list of nl pairs for n bodies: per pair its two ends, flag
// and scan offset (16 B), per body the build's position, radius, hull and
// static flag (41 B), ten per cent and the alignment of eight buffers.
static size_t list_bytes(int64_t nl, int64_t n) {
    return (size_t)(1.1 * (16.0 * (double)nl + 41.0 * (double)n)) + 8 * Arena::kAlign;
}

static nbgs_status build_pair_list(nbgs_scene_t sc, double max_reach, double max_h, bool *built) {
    hipStream_t s = sc->s;
    const int32_t N = sc->b.n;
    *built = false;
    sc->vl_valid = false;
    const double skin = std::max(4.0 * max_h, 0.02 * max_reach);
    if (!(skin > 0.0) || !std::isfinite(skin)) return NBGS_OK;
    // room for the list beside everything the step may need (the list is not part of the workspace bound)
    auto drop = [&]() {
        for (DevBuf<int32_t> *b : {&sc->vl_j1, &sc->vl_j2, &sc->vl_flag, &sc->vl_off}) b->release();
        for (DevBuf<double> *b : {&sc->vl_h, &sc->vl_x0, &sc->vl_r0}) b->release();
        sc->vl_static0.release();
        set_error("");
        return NBGS_OK;
    };
    for (DevBuf<int32_t> *b : {&sc->vl_j1, &sc->vl_j2, &sc->vl_flag, &sc->vl_off}) b->release();  // the old list
    if (sc->vl_blocked) return drop();
    // the contacts the list will serve: a quarter more than the last detection found (all listed pairs on the
    // first); a step that finds more than fit beside the list gives the list's room back (nbgs_detect)
    auto contacts_served = [&](int64_t nl) { return sc->nc > 0 ? std::min(nl, sc->nc + sc->nc / 4 + 64) : nl; };
    size_t base = 0;
    NBGS_TRY(scene_need_bytes(sc, sc->nc, &base));
    if (base + list_bytes(0, N) > sc->arena.size()) return drop();
    if (sc->vl_h.reserve((size_t)N, 1.0) != NBGS_OK || sc->vl_x0.reserve(3 * (size_t)N + 1, 1.0) != NBGS_OK ||
        sc->vl_r0.reserve((size_t)N, 1.0) != NBGS_OK || sc->vl_static0.reserve((size_t)N, 1.0) != NBGS_OK)
        return drop();
    NBGS_TRY(launch_fill_f64(sc->vl_h.p, N, skin, s));
    int64_t nl = 0;
    NBGS_TRY(grid_pairs(sc, sc->vl_h.p, max_reach + skin, &nl));
    size_t need = 0;
    NBGS_TRY(scene_need_bytes(sc, contacts_served(nl), &need));
    if (need + list_bytes(nl, N) > sc->arena.size()) return drop();
    if (sc->vl_j1.reserve((size_t)(nl > 0 ? nl : 1)) != NBGS_OK ||
        sc->vl_j2.reserve((size_t)(nl > 0 ? nl : 1)) != NBGS_OK || sc->vl_flag.reserve((size_t)nl + 1) != NBGS_OK ||
        sc->vl_off.reserve((size_t)nl + 1) != NBGS_OK)
        return drop();
    ContactsView lv{};
    lv.j1 = sc->vl_j1.p;
    lv.j2 = sc->vl_j2.p;
    NBGS_TRY(launch_pair_emit(sc->b, sc->grid, sc->planes, sc->table(), sc->p.tau, sc->skeys, sc->sids, sc->sxr.p,
                              sc->vl_h.p, sc->cells.p, sc->occ.p, sc->cnt.p, sc->off.p, sc->cellpos.p, sc->npart.p,
                              sc->partners.p, lv, nl, false, s));
    NBGS_HIP(hipMemcpyAsync(sc->vl_x0.p, sc->b.x, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    NBGS_HIP(hipMemcpyAsync(sc->vl_x0.p + N, sc->b.y, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    NBGS_HIP(hipMemcpyAsync(sc->vl_x0.p + 2 * (size_t)N, sc->b.z, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    NBGS_HIP(hipMemcpyAsync(sc->vl_r0.p, sc->b.radius, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    NBGS_TRY(launch_static_flags(sc->b.inv_mass, N, sc->vl_static0.p, s));
    sc->vl_skin = skin;
    sc->vl_n = nl;
    sc->vl_valid = true;
    sc->vl_builds += 1;
    *built = true;
    return NBGS_OK;
}

nbgs_status detect_impl(nbgs_scene_t sc, nbgs_stats *stats) {
    hipStream_t s = sc->s;
    const int32_t N = sc->b.n;
    record(sc, kDetect);
    if (sc->table_in_cur) {  // the solved impulses of the last step become the lookup table
        sc->cur = 1 - sc->cur;
        sc->table_in_cur = false;
    }
    ContactBuf &prev = sc->cb[1 - sc->cur];
    // hull radii, the largest reach and hull and, with a pair list, its validity
    // maxbits: [0] largest r + h (bits of a non-negative double), [1] contact total in 64 bits, [2] candidate
    // overflow of the pair count, [3] largest h, [4] largest displacement + h + radius growth since the list's build
    const bool have_list = sc->vl_enabled && sc->vl_valid;
    NBGS_HIP(hipMemsetAsync(sc->maxbits.p, 0, 5 * sizeof(unsigned long long), s));
    // every body's dynamic bit, compared with the last detection's (kept current at every detection): small[7]
    // counts the words that changed
    NBGS_TRY(sc->dyn_bits.reserve((size_t)((sc->b.n + 63) / 64 + 1), 1.0));
    NBGS_HIP(hipMemsetAsync(sc->small.p + 7, 0, sizeof(int32_t), s));
    NBGS_TRY(launch_hull(sc->b, sc->p.dt, sc->p.tau, sc->h.p, sc->maxbits.p, have_list ? sc->vl_x0.p : nullptr,
                         have_list ? sc->vl_r0.p : nullptr, have_list ? sc->vl_static0.p : nullptr, sc->dyn_bits.p,
                         sc->small.p + 7, s));
    unsigned long long mb[5];
    NBGS_HIP(hipMemcpyAsync(sc->pinned, sc->maxbits.p, sizeof(mb), hipMemcpyDeviceToHost, s));
    NBGS_HIP(hipStreamSynchronize(s));
    std::memcpy(mb, sc->pinned, sizeof(mb));
    double max_reach, max_h, max_moved;
    std::memcpy(&max_reach, &mb[0], sizeof(double));
    std::memcpy(&max_h, &mb[3], sizeof(double));
    std::memcpy(&max_moved, &mb[4], sizeof(double));
    if (!std::isfinite(max_reach)) {
        set_error("non-finite velocity or radius in the body state");
        return NBGS_ERR_NUMERIC;
    }
    const SceneTable tab = sc->table();
    // contacts: from the pair list while it holds (rebuilt when it does not), else from the cell grid
    bool use_list = have_list && max_moved <= 0.999 * sc->vl_skin;
    if (sc->vl_enabled && !use_list) NBGS_TRY(build_pair_list(sc, max_reach, max_h, &use_list));
    int64_t nc = 0;
    if (use_list) {
        const int64_t nl = sc->vl_n;
        NBGS_TRY(launch_list_test(sc->b, sc->grid, sc->planes, tab, sc->p.tau, sc->h.p, sc->vl_j1.p, sc->vl_j2.p, nl,
                                  sc->vl_flag.p, s));
        const size_t need_tmp = exclusive_scan_tmp_bytes(nl + 1);
        if (need_tmp > sc->scan_tmp.cap) NBGS_TRY(sc->scan_tmp.reserve(need_tmp));
        NBGS_TRY(exclusive_scan_i32(sc->vl_flag.p, sc->vl_off.p, nl, sc->total(), sc->scan_tmp.p, sc->scan_tmp.cap,
                                    s));
        NBGS_TRY(sync_small(sc, 0, 1));
        nc = nl > 0 ? sc->pinned[0] : 0;
    } else {
        NBGS_TRY(grid_pairs(sc, sc->h.p, max_reach, &nc));
    }
    if ((sc->sub_edge > 0.0 || sc->blk_edge > 0.0) && 2 * nc > (int64_t)0x7fffff00) {
        set_error("%lld contacts: the subdomain solver indexes both ends of a contact in 32 bits (at most 2^30 "
                  "contacts)", (long long)nc);
        return NBGS_ERR_CAPACITY;
    }
    // from here on a CAPACITY is the workspace's: its count is reported (the refusals above report none)
    sc->nc_needed = nc;
    // the contact capacity of the workspace (nbgs_scene_workspace_query's sizes): refused before any list is touched
    size_t need = 0;
    NBGS_TRY(scene_need_bytes(sc, nc, &need));
    if (need > sc->arena.size()) {
        set_error("%lld contacts need a workspace of %zu bytes in this sweep order (nbgs_scene_workspace_query), "
                  "this one has %zu", (long long)nc, need, sc->arena.size());
        return NBGS_ERR_CAPACITY;
    }
    sc->nc_needed = -1;  // a later refusal (colours, block sizes) is not lifted by a larger workspace
    sc->nc = nc;
    ContactBuf &cb = sc->cb[sc->cur];
    NBGS_TRY(cb.reserve((size_t)nc));
    if (use_list) {
        NBGS_TRY(launch_list_emit(sc->vl_j1.p, sc->vl_j2.p, sc->vl_n, sc->vl_flag.p, sc->vl_off.p, cb.view(), s));
        NBGS_TRY(launch_pair_geometry(sc->b, sc->grid, sc->planes, tab, cb.view(), nc, s));
        NBGS_TRY(launch_contact_runs(cb.j1.p, nc, N, sc->cnt.p, sc->off.p, s));  // the colouring's per-body runs
    } else {
        NBGS_TRY(launch_pair_emit(sc->b, sc->grid, sc->planes, tab, sc->p.tau, sc->skeys, sc->sids, sc->sxr.p,
                                  sc->h.p, sc->cells.p, sc->occ.p, sc->cnt.p, sc->off.p, sc->cellpos.p, sc->npart.p,
                                  sc->partners.p, cb.view(), nc, true, s));
    }
    // initial impulses and, when the previous table carries colours, the start of the colouring
    const bool warm_impulses = sc->p.warm_start != NBGS_WS_ZERO && sc->n_prev > 0;
    const bool warm_colours = sc->prev_colours && sc->n_prev > 0 && nc > 0;
    // new pairs are counted when the previous colouring may be reused whole (same pair count)
    const bool maybe_same = warm_colours && nc == sc->n_prev;
    if (maybe_same) NBGS_HIP(hipMemsetAsync(sc->small.p + 4, 0, 3 * sizeof(int32_t), s));  // small[7]: the hull pass
    const bool dyn_bits_known = sc->dyn_bits_valid;
    sc->dyn_bits_valid = true;
    NBGS_TRY(launch_match_prev(cb.view(), nc, prev.key.p, prev.px.p, prev.py.p, prev.pz.p, prev.colour.p, sc->n_prev,
                               sc->p.mu, tab, warm_impulses, warm_colours, maybe_same ? sc->small.p + 4 : nullptr,
                               s));
    if (!warm_impulses) NBGS_TRY(launch_zero_impulses(cb.view(), nc, s));
    if (!warm_impulses && !warm_colours) NBGS_TRY(launch_fill_i32(cb.matched.p, nc, 0, s));
    // network features and prediction (from the state before the step and the previous impulses)
    sc->have_features = false;
    sc->have_learned = false;
    sc->solved = false;
    const bool learned = sc->p.warm_start == NBGS_WS_LEARNED && sc->mlp;
    if ((sc->capture || learned) && nc > 0) {
        NBGS_TRY(sc->feat.reserve(12 * (size_t)nc));
        NBGS_TRY(sc->frame.reserve(9 * (size_t)nc));
        NBGS_TRY(launch_features(sc->b, cb.view(), nc, sc->p.gravity, sc->p.dt, sc->p.mu, sc->p.erp, sc->fs,
                                 sc->feat.p, sc->frame.p, s));
        sc->have_features = true;
        if (learned) {
            NBGS_TRY(sc->yout.reserve(3 * (size_t)nc));
            for (DevBuf<double> *b : {&sc->lpx, &sc->lpy, &sc->lpz}) NBGS_TRY(b->reserve((size_t)nc));
            NBGS_TRY(launch_mlp_forward(mlp_frag_ptr(sc->mlp), mlp_weight_ptr(sc->mlp), sc->feat.p, nc, sc->yout.p, s));
            NBGS_TRY(launch_decode(sc->yout.p, sc->frame.p, cb.view(), nc, sc->fs, sc->p.mu, sc->lpx.p, sc->lpy.p,
                                   sc->lpz.p, s));
            sc->have_learned = true;
        }
    }
    record(sc, kColour);
    // subdomain solver: the colouring is restricted to the contacts of one subdomain
    sc->sub_active = sc->sub_edge > 0.0 && nc > 0;
    sc->blk_active = !sc->sub_active && sc->blk_edge > 0.0 && nc > 0;
    if (sc->sub_active) NBGS_TRY(subdomain_assign(sc));
    if (!sc->blk_active) sc->xg_prev_valid = false;  // the last ids kept are not this order's
    if (sc->blk_active)
        NBGS_TRY(block_assign(sc, sc->small.p + 6, maybe_same && dyn_bits_known && sc->prev_sig_valid));
    const int32_t *sdom = sc->sub_active || sc->blk_active ? sc->sdom.p : nullptr;
    // The greedy colouring and the (id, colour, key) order are functions of the pair keys, the ids, the seed and
    // which bodies are dynamic only.  When every pair of this step is a pair of the last one (same count, none new),
    // every id and every body's dynamic bit is the same and the mode and seed are too, the last colours (already
    // copied by the match), colour counts and sweep permutation are this step's.
    const double sig[4] = {(double)sc->p.colour_seed, sc->sub_active ? sc->sub_edge : -1.0,
                           sc->blk_active ? sc->blk_edge : -1.0, (double)(sdom ? sc->n_sub : 0)};
    bool same = maybe_same && dyn_bits_known && sc->prev_sig_valid &&
                std::memcmp(sig, sc->prev_sig, sizeof(sig)) == 0 && sc->prev_seed == sc->p.colour_seed &&
                sc->perm != nullptr;
    if (same && sdom) NBGS_TRY(launch_ids_changed(sdom, sc->prev_sdom.p, cb.matched.p, nc, sc->small.p + 5, s));
    // the block set-up (slots, per-id ranges, cross colours) depends on these and on every body's block
    bool prep_same = false;
    if (same) {
        NBGS_TRY(sync_small(sc, 4, 4));
        same = sc->pinned[4] == 0 && sc->pinned[5] == 0 && sc->pinned[7] == 0;
        prep_same = same && sc->blk_active && sc->bblk_compared && sc->pinned[6] == 0 &&
                    sc->prev_precision == sc->p.precision;
    }
    sc->colouring_reused = same;
    if (same) sc->colour_passes = 0;
    else NBGS_TRY(colour_and_order(sc, cb, tab, sdom, warm_colours));
    // ids of this step's pairs, for the next step's comparison
    if (sdom) {
        NBGS_TRY(sc->prev_sdom.reserve((size_t)nc));
        NBGS_HIP(hipMemcpyAsync(sc->prev_sdom.p, sdom, sizeof(int32_t) * nc, hipMemcpyDeviceToDevice, s));
    }
    std::memcpy(sc->prev_sig, sig, sizeof(sig));
    sc->prev_seed = sc->p.colour_seed;
    sc->prev_sig_valid = nc > 0;
    sc->precision_used = sc->p.precision;
    // a reused order keeps the sweep record's ends, order, colours and ids (same precision, same buffers)
    NBGS_TRY(scene_gather(sc, !(same && sc->prev_precision == sc->p.precision)));
    if (sc->sub_active) NBGS_TRY(subdomain_prepare(sc));
    if (sc->blk_active && !prep_same) NBGS_TRY(block_prepare(sc));
    sc->blk_prep_reused = prep_same;
    sc->prev_precision = sc->p.precision;
    if (sc->blk_active) sc->bblk_cur = 1 - sc->bblk_cur;
    sc->bblk_valid = sc->blk_active;
    sc->state = 1;
    sc->stats.n_contacts = nc;
    sc->stats.n_colours = sc->n_colours;
    sc->stats.sweeps = 0;
    sc->stats.residual = 0.0;
    record(sc, kInit);
    if (stats) *stats = sc->stats;
    return NBGS_OK;
}

// Greedy colouring (from the previous colours where the match supplied them, else Jones-Plassmann rounds from
// scratch), the colour histogram and the colour-major (id, colour, key) permutation.
nbgs_status colour_and_order(nbgs_scene_t sc, ContactBuf &cb, const SceneTable &tab, const int32_t *sdom,
                             bool warm_colours) {
    hipStream_t s = sc->s;
    const int32_t N = sc->b.n;
    const int64_t nc = sc->nc;
    // colouring: body -> contacts where it is j2 (as j1 it owns the segment off[i] .. off[i] + cnt[i])
    NBGS_TRY(sc->inc2.reserve((size_t)(nc > 0 ? nc : 1)));
    NBGS_TRY(sc->prio.reserve((size_t)(nc > 0 ? nc : 1)));
    NBGS_TRY(launch_prio(cb.view(), nc, sc->p.colour_seed, tab, N, sc->prio.p, s));
    NBGS_TRY(launch_j2_degree(cb.view(), nc, N, sc->b.inv_mass, sc->deg2.p, s));
    NBGS_TRY(exclusive_scan_i32(sc->deg2.p, sc->off2.p, (int64_t)N + 1, nullptr, sc->scan_tmp.p, sc->scan_tmp.cap, s));
    NBGS_HIP(hipMemcpyAsync(sc->cursor.p, sc->off2.p, sizeof(int32_t) * ((size_t)N + 1), hipMemcpyDeviceToDevice, s));
    NBGS_TRY(launch_j2_fill(cb.view(), nc, N, sc->b.inv_mass, sc->cursor.p, sc->inc2.p, s));
    sc->colour_passes = 0;
    if (nc > 0 && warm_colours) {
        // greedy rule repeated from the previous colours until a pass changes nothing; after the first pass only
        // the contacts a change reached are evaluated
        NBGS_TRY(sc->dirty[0].reserve((size_t)nc));
        NBGS_TRY(sc->dirty[1].reserve((size_t)nc));
        // passes go out in growing batches between host checks (a pass after the fixed point finds nothing
        // marked and changes nothing); the count read back is the last pass's
        // (one change counter per pass and flag arrays the passes leave clear: no clearing launch between passes)
        NBGS_TRY(sc->fixcnt.reserve(kFixCounters, 1.0));
        NBGS_HIP(hipMemsetAsync(sc->fixcnt.p, 0, sizeof(int32_t) * kFixCounters, s));
        NBGS_HIP(hipMemsetAsync(sc->overflow(), 0, sizeof(int32_t), s));
        NBGS_TRY(launch_fill_u8(sc->dirty[0].p, nc, 0, s));
        NBGS_TRY(launch_fill_u8(sc->dirty[1].p, nc, 0, s));
        int pass = 0, batch = 1;
        for (;;) {
            for (int r = 0; r < batch; ++r, ++pass) {
                int32_t *cnt = sc->fixcnt.p + pass % kFixCounters;
                if (pass >= kFixCounters) NBGS_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t), s));
                uint8_t *din = pass == 0 ? nullptr : sc->dirty[(pass + 1) & 1].p;
                uint8_t *dout = sc->dirty[pass & 1].p;
                NBGS_TRY(launch_colour_fix(cb.view(), sc->prio.p, nc, N, sc->b.inv_mass, sc->off.p, sc->cnt.p,
                                           sc->off2.p, sc->inc2.p, sdom, din, dout, cnt, sc->overflow(), false, s));
            }
            NBGS_HIP(hipMemcpyAsync(sc->pinned + 1, sc->fixcnt.p + (pass - 1) % kFixCounters, sizeof(int32_t),
                                    hipMemcpyDeviceToHost, s));
            NBGS_TRY(sync_small(sc, 2, 1));
            sc->colour_passes = pass;
            if (sc->pinned[2]) {
                set_error("more than 255 colours needed");
                return NBGS_ERR_CAPACITY;
            }
            if (sc->pinned[1] == 0) break;
            if (pass > 100000) {
                set_error("colouring did not settle");
                return NBGS_ERR_DEVICE;
            }
            batch = batch < 8 ? 2 * batch : 8;
        }
    } else if (nc > 0) {
        NBGS_HIP(hipMemsetAsync(cb.colour.p, 0xff, sizeof(int32_t) * nc, s));
        sc->pinned[1] = (int32_t)nc;
        sc->pinned[2] = 0;
        NBGS_HIP(hipMemcpyAsync(sc->remaining(), sc->pinned + 1, 2 * sizeof(int32_t), hipMemcpyHostToDevice, s));
        int batch = 2, rounds = 0;
        for (;;) {
            for (int r = 0; r < batch; ++r)
                NBGS_TRY(launch_jp_round(cb.view(), sc->prio.p, nc, N, sc->b.inv_mass, sc->off.p, sc->cnt.p,
                                         sc->off2.p, sc->inc2.p, sdom, sc->remaining(), sc->overflow(), s));
            rounds += batch;
            NBGS_TRY(sync_small(sc, 1, 2));
            if (sc->pinned[2]) {
                set_error("more than 255 colours needed");
                return NBGS_ERR_CAPACITY;
            }
            if (sc->pinned[1] == 0) break;
            if (rounds > 100000) {
                set_error("colouring did not finish");
                return NBGS_ERR_DEVICE;
            }
            batch = batch < 8 ? batch * 2 : 8;
        }
        sc->colour_passes = -rounds;
    }
    // colour-major order: stable sort of (colour, canonical index)
    NBGS_TRY(launch_colour_hist(cb.view(), nc, N, sc->b.inv_mass, sc->chist(), s));
    NBGS_TRY(sync_small(sc, 16, 512));
    sc->n_colours = 0;
    for (int c = 0; c < 256; ++c)
        if (sc->pinned[16 + c]) sc->n_colours = c + 1;
    sc->col_off.assign((size_t)sc->n_colours + 1, 0);
    sc->col_dyn.assign((size_t)sc->n_colours, 0);
    for (int c = 0; c < sc->n_colours; ++c) {
        sc->col_off[c + 1] = sc->col_off[c] + sc->pinned[16 + c];
        sc->col_dyn[c] = sc->pinned[16 + 256 + c];
    }
    NBGS_TRY(sc->ckeys.reserve((size_t)nc + 1));
    NBGS_TRY(sc->cids.reserve((size_t)nc + 1));
    NBGS_TRY(sc->ckeys2.reserve((size_t)nc + 1));
    NBGS_TRY(sc->cids2.reserve((size_t)nc + 1));
    NBGS_TRY(launch_colour_keys(cb.view(), sdom, nc, sc->ckeys.p, sc->cids.p, s));
    if ((size_t)radix_hist_entries(nc) > sc->radix_hist.cap) NBGS_TRY(sc->radix_hist.reserve(radix_hist_entries(nc)));
    const size_t need_tmp = exclusive_scan_tmp_bytes((int64_t)radix_hist_entries(nc));
    if (need_tmp > sc->scan_tmp.cap) NBGS_TRY(sc->scan_tmp.reserve(need_tmp));
    bool calt = false;
    NBGS_TRY(radix_sort_pairs(sc->ckeys.p, sc->cids.p, sc->ckeys2.p, sc->cids2.p, nc,
                              sdom ? 8 + bits_for(sc->n_sub) : 8, sc->radix_hist.p, sc->scan_tmp.p, sc->scan_tmp.cap,
                              &calt, s));
    const uint32_t *perm = calt ? sc->cids2.p : sc->cids.p;
    if (nc == 1) perm = sc->cids.p;
    sc->perm = perm;
    return NBGS_OK;
}

nbgs_status ensure_profile_events(nbgs_scene_t sc, size_t launches) {
    while (sc->pev.size() < 2 * launches) {
        hipEvent_t e;
        NBGS_HIP(hipEventCreate(&e));
        sc->pev.push_back(e);
    }
    return NBGS_OK;
}

// Compulsory bytes of one sweep launch: the contact record (ids, normal,
// xi/dt, arms, impulse read and written) plus, per dynamic body touched, its
// record read (v', w', 1/m, 1/I) and v', w' written.
template <class T>
constexpr double contact_bytes() {
    return 2 * 4 + 6 * sizeof(T) + 2 * 3 * sizeof(T);
}
template <class T>
constexpr double body_bytes() {
    return 8 * sizeof(T) + 6 * sizeof(T);
}

template <class T>
nbgs_status accumulate_profile(nbgs_scene_t sc, int32_t sweeps) {
    NBGS_HIP(hipStreamSynchronize(sc->s));
    if (sc->graph_pairs > 0) {  // graph replay: one event pair per replayed block of sweeps, residuals included
        for (int q = 0; q < sc->graph_pairs; ++q) {
            float ms = 0.0f;
            NBGS_HIP(hipEventElapsedTime(&ms, sc->pev[2 * q], sc->pev[2 * q + 1]));
            sc->prof.sweep_kernel_ms += ms;
        }
        for (int c = 0; c < sc->n_colours; ++c) {
            const int64_t m = sc->col_off[c + 1] - sc->col_off[c];
            if (m == 0) continue;
            sc->prof.sweep_launches += sweeps;
            sc->prof.contact_updates += (int64_t)sweeps * m;
            sc->prof.sweep_bytes +=
                (double)sweeps * (contact_bytes<T>() * (double)m + body_bytes<T>() * (double)sc->col_dyn[c]);
        }
        return NBGS_OK;
    }
    size_t pe = 0;
    for (int32_t k = 0; k < sweeps; ++k)
        for (int c = 0; c < sc->n_colours; ++c, ++pe) {
            float ms = 0.0f;
            NBGS_HIP(hipEventElapsedTime(&ms, sc->pev[2 * pe], sc->pev[2 * pe + 1]));
            const int64_t m = sc->col_off[c + 1] - sc->col_off[c];
            if (m == 0) continue;
            sc->prof.sweep_kernel_ms += ms;
            sc->prof.sweep_launches += 1;
            sc->prof.contact_updates += m;
            sc->prof.sweep_bytes += contact_bytes<T>() * (double)m + body_bytes<T>() * (double)sc->col_dyn[c];
        }
    return NBGS_OK;
}

// The solver's records at the start of a solve: every body's, or with few contacts the touched bodies' only; in
// the block-local sweeps' order while rec_on.
template <class T>
nbgs_status init_records(nbgs_scene_t sc, T *vel) {
    if (sc->sparse_bodies) return launch_init_touched<T>(sc->b, sc->p.gravity, sc->p.dt, sc->touched.p, vel, sc->s);
    return launch_init_bodies<T>(sc->b, sc->p.gravity, sc->p.dt, vel, rec_map(sc), sc->s);
}

// Jacobi residual of the previous-step and of the learned initial impulses;
// the sweep record keeps the better one (ties: the network).
template <class T>
nbgs_status judge_warm_start(nbgs_scene_t sc) {
    hipStream_t s = sc->s;
    const int32_t N = sc->b.n;
    SweepBuf<T> &sw = sweep_buf<T>(sc);
    DevBuf<T> &vel = vel_buf<T>(sc);
    NBGS_TRY(sc->jpart.reserve(2 * (size_t)((sc->nc + 255) / 256 + 1)));
    NBGS_TRY(sc->jres.reserve(2));
    ContactBuf &cb = sc->cb[sc->cur];
    for (int cand = 0; cand < 2; ++cand) {
        if (cand == 1) NBGS_TRY(launch_set_sweep_impulses<T>(sw.view(), sc->nc, sc->lpx.p, sc->lpy.p, sc->lpz.p, s));
        NBGS_TRY(init_records<T>(sc, vel.p));
        for (int c = 0; c < sc->n_colours; ++c)
            NBGS_TRY(launch_warm_scatter<T>(sw.view(), sc->col_off[c], sc->col_off[c + 1], N, vel.p, s));
        NBGS_TRY(launch_jacobi_residual<T>(sw.view(), sc->nc, N, vel.p, sc->p.mu, sc->jpart.p, sc->jres.p + cand, s));
    }
    double r[2];
    NBGS_HIP(hipMemcpyAsync(sc->pinned + 64, sc->jres.p, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    NBGS_HIP(hipStreamSynchronize(s));
    std::memcpy(r, sc->pinned + 64, sizeof(r));
    sc->winfo.r_previous = r[0];
    sc->winfo.r_learned = r[1];
    sc->winfo.choice = r[1] <= r[0] ? 1 : 0;
    if (sc->winfo.choice == 0)
        NBGS_TRY(launch_set_sweep_impulses<T>(sw.view(), sc->nc, cb.px.p, cb.py.p, cb.pz.p, s));
    return NBGS_OK;
}

// Enqueue k sweeps (every colour from its device-side range, then the
// residual) on stream cs.
template <class T>
nbgs_status enqueue_dev_sweeps(nbgs_scene_t sc, int32_t k, double target, const SweepTune &tune, unsigned grid,
                               hipStream_t cs, bool residuals) {
    SweepBuf<T> &sw = sweep_buf<T>(sc);
    DevBuf<T> &vel = vel_buf<T>(sc);
    const SweepParams sp{sc->p.mu, sc->p.relax};
    const int C = sc->n_colours;
    for (int32_t it = 0; it < k; ++it) {
        for (int c = 0; c < C; ++c)
            NBGS_TRY(launch_sweep_colour_dev<T>(sw.view(), sc->col_d.p, c, sc->b.n, vel.p, sp, tune,
                                                sc->partials.p + 2 * (size_t)c * grid, sc->ctrl(), cs));
        if (residuals)
            NBGS_TRY(launch_residual(sc->partials.p, (int32_t)((int64_t)C * grid), target, sc->ctrl(), sc->res_hist.p,
                                     cs));
    }
    return NBGS_OK;
}

}  // namespace

namespace nbgs {

nbgs_status scene_sync_small(nbgs_scene_t sc, int first, int count) { return sync_small(sc, first, count); }

nbgs_status scene_gather(nbgs_scene_t sc, bool indices) {
    if (indices) sc->rec_valid = false;  // new ends in the sweep record
    if (sc->precision_used == NBGS_FP32_SWEEP) return gather_for_sweeps<float>(sc, indices);
    return gather_for_sweeps<double>(sc, indices);
}

// The sweep loop replayed from a captured graph: blocks of up to 32 sweeps
// are captured once (on a private stream, re-captured when the colour count,
// launch shape, buffers or parameters change) and launched on the scene's
// stream; the colour ranges are uploaded per solve, so one graph serves every
// step.  Sweeps after the target is met exit at once, as in the direct loop.
template <class T>
nbgs_status scene_sweep_loop(nbgs_scene_t sc, int32_t max_sweeps, double target, const SweepTune &tune) {
    hipStream_t s = sc->s;
    SweepBuf<T> &sw = sweep_buf<T>(sc);
    DevBuf<T> &vel = vel_buf<T>(sc);
    const int C = sc->n_colours;
    const unsigned grid = sweep_graph_grid<T>(tune);
    if (grid == 0) {
        set_error("unsupported sweep tuning for graph replay");
        return NBGS_ERR_INVALID_ARG;
    }
    NBGS_TRY(sc->partials.reserve(2 * (size_t)((int64_t)C * grid + 1)));
    NBGS_TRY(sc->col_d.reserve((size_t)C + 1));
    if (sc->col_pinned_cap < (size_t)C + 1) {
        if (sc->col_pinned) (void)hipHostFree(sc->col_pinned);
        sc->col_pinned = nullptr;
        sc->col_pinned_cap = 0;
        const size_t want = (size_t)C + 65;
        NBGS_HIP(hipHostMalloc((void **)&sc->col_pinned, want * sizeof(int64_t)));
        sc->col_pinned_cap = want;
    }
    // the previous upload from this staging area has completed: every solve ends with a stream synchronisation
    // before the next one starts, or the caller synchronised after a solve without statistics
    NBGS_HIP(hipStreamSynchronize(s));
    for (int c = 0; c <= C; ++c) sc->col_pinned[c] = sc->col_off[c];
    NBGS_HIP(hipMemcpyAsync(sc->col_d.p, sc->col_pinned, sizeof(int64_t) * (C + 1), hipMemcpyHostToDevice, s));
    const int32_t K = std::min<int32_t>(max_sweeps, 32);
    nbgs_scene_s::GraphKey key;
    key.sweeps = K;
    key.colours = C;
    key.prec = (int32_t)sizeof(T);
    key.grid = grid;
    key.tune = tune;
    key.ptrs[0] = sw.j1.p;
    key.ptrs[1] = sw.px.p;
    key.ptrs[2] = sw.mu.p;
    key.ptrs[3] = vel.p;
    key.ptrs[4] = sc->partials.p;
    key.ptrs[5] = sc->res_hist.p;
    key.col = sc->col_d.p;
    key.target = target;
    key.mu = sc->p.mu;
    key.relax = sc->p.relax;
    // without a target and without history only the last sweep's residual is formed (after the replays)
    const bool every = target > 0.0 || sc->res_history;
    key.every = every;
    key.alloc_gen = g_alloc_generation.load(std::memory_order_relaxed);
    if (!sc->gexec || !(key == sc->gkey)) {
        if (sc->gexec) (void)hipGraphExecDestroy(sc->gexec);
        sc->gexec = nullptr;
        if (!sc->cap_stream) NBGS_HIP(hipStreamCreateWithFlags(&sc->cap_stream, hipStreamNonBlocking));
        NBGS_HIP(hipStreamBeginCapture(sc->cap_stream, hipStreamCaptureModeRelaxed));
        const nbgs_status st = enqueue_dev_sweeps<T>(sc, K, target, tune, grid, sc->cap_stream, every);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(sc->cap_stream, &g);
        if (st != NBGS_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        NBGS_HIP(e);
        const hipError_t ei = hipGraphInstantiate(&sc->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        NBGS_HIP(ei);
        sc->gkey = key;
    }
    const int32_t reps = max_sweeps / K, rem = max_sweeps % K;
    const bool prof = sc->profiling;
    if (prof) NBGS_TRY(ensure_profile_events(sc, (size_t)reps + 1));
    int q = 0;
    bool done = false;
    for (int32_t r = 0; r < reps && !done; ++r) {
        if (prof) NBGS_HIP(hipEventRecord(sc->pev[2 * q], s));
        NBGS_HIP(hipGraphLaunch(sc->gexec, s));
        if (prof) NBGS_HIP(hipEventRecord(sc->pev[2 * q + 1], s));
        ++q;
        if (target > 0.0 && (r + 1 < reps || rem > 0)) {
            NBGS_TRY(sync_small(sc, 8, 3));
            done = sc->pinned[8] != 0;
        }
    }
    if (!done && rem > 0) {
        if (prof) NBGS_HIP(hipEventRecord(sc->pev[2 * q], s));
        NBGS_TRY(enqueue_dev_sweeps<T>(sc, rem, target, tune, grid, s, every));
        if (prof) NBGS_HIP(hipEventRecord(sc->pev[2 * q + 1], s));
        ++q;
    }
    if (!every)
        NBGS_TRY(launch_residual(sc->partials.p, (int32_t)((int64_t)C * grid), target, sc->ctrl(), sc->res_hist.p, s,
                                 max_sweeps - 1));
    sc->graph_pairs = prof ? q : 0;
    return NBGS_OK;
}

template nbgs_status scene_sweep_loop<double>(nbgs_scene_t, int32_t, double, const SweepTune &);
template nbgs_status scene_sweep_loop<float>(nbgs_scene_t, int32_t, double, const SweepTune &);

}  // namespace nbgs

namespace {

constexpr int kSolveColour = 0, kSolveSubdomain = 1, kSolveBlock = 2;

// Stop flag, sweep count and last residual after a solve; NUMERIC / NOT_CONVERGED as nbgs_solve reports them.
// mode: which solver ran (the profile's byte count of the subdomain and block-local solvers is made here).
template <class T>
nbgs_status finish_solve(nbgs_scene_t sc, int32_t max_sweeps, double target, nbgs_stats *stats, int mode) {
    hipStream_t s = sc->s;
    SweepBuf<T> &sw = sweep_buf<T>(sc);
    NBGS_TRY(launch_save_impulses<T>(sw.view(), sc->nc, sc->cb[sc->cur].view(), s));
    record(sc, kIntegrate);
    sc->state = 2;
    sc->solved = true;
    int32_t sweeps = 0;
    double R = 0.0;
    NBGS_TRY(read_solve_result(sc, sweeps, R));
    sc->stats.sweeps = sweeps;
    sc->stats.residual = R;
    if (stats) *stats = sc->stats;
    if (mode != kSolveColour && sc->profiling) {
        for (int32_t k = 0; k < sweeps && k < max_sweeps; ++k) {
            float ms = 0.0f;
            NBGS_HIP(hipEventElapsedTime(&ms, sc->pev[2 * k], sc->pev[2 * k + 1]));
            sc->prof.sweep_kernel_ms += ms;
        }
        const double tb = (double)sizeof(T);
        double per_sweep;
        if (mode == kSolveSubdomain) {
            // every contact record and its two slot indices, every slot read (v', w', 1/m, 1/I) and its
            // correction written and read back, every corrected body's v', w' read and written
            per_sweep = (2 * 4 + 12 * tb) * (double)sc->nc + 4 * 2 * (double)sc->nc +
                        (8 * tb + 6 * tb + 6 * tb) * (double)sc->n_slots + 12 * tb * (double)sc->b.n;
        } else {
            // every contact record, the two 16-bit slot indices of every local contact, every slot read and
            // written once, every dynamic end of a contact between blocks read and written
            double xd = 0.0;
            for (int64_t d : sc->xdyn) xd += (double)d;
            per_sweep = (2 * 4 + 12 * tb) * (double)sc->nc + 2 * 2 * (double)sc->blk_n_local +
                        14 * tb * ((double)sc->blk_dyn_local + xd);
        }
        sc->prof.sweep_launches += sweeps;
        sc->prof.contact_updates += (int64_t)sweeps * sc->nc;
        sc->prof.sweep_bytes += per_sweep * sweeps;
    }
    if (sc->pinned[8 + 2]) {
        set_error("non-finite residual after sweep %d", sweeps);
        return NBGS_ERR_NUMERIC;
    }
    if (target > 0.0 && !(R <= target)) {
        set_error("residual %.3e above target %.3e after %d sweeps", R, target, sweeps);
        return NBGS_ERR_NOT_CONVERGED;
    }
    return NBGS_OK;
}

// Subdomain NBGS: the initial impulses enter as a first correction pass, then
// sweeps until the target or the sweep count, one pass (all subdomains) plus
// the correction reduction per sweep.
template <class T>
nbgs_status sub_solve(nbgs_scene_t sc, int32_t max_sweeps, double target, nbgs_stats *stats) {
    hipStream_t s = sc->s;
    DevBuf<T> &vel = vel_buf<T>(sc);
    DevBuf<T> &corr = corr_buf<T>(sc);
    NBGS_TRY(corr.reserve(6 * (size_t)(sc->n_slots > 0 ? sc->n_slots : 1)));
    NBGS_TRY(sc->partials.reserve(2 * (size_t)sc->n_sub));
    NBGS_HIP(hipMemsetAsync(sc->ctrl(), 0, 4 * sizeof(int32_t), s));
    // with a fixed sweep count and the history off only the last sweep's residual is formed
    const bool every = target > 0.0 || sc->res_history;
    sc->hist_partial = !every;
    sc->graph_pairs = 0;
    NBGS_TRY(subdomain_pass<T>(sc, 0, vel.p, corr.p));
    record(sc, kSweeps);
    const bool prof = sc->profiling;
    if (prof) NBGS_TRY(ensure_profile_events(sc, (size_t)max_sweeps));
    int32_t launched = 0, chunk = target > 0.0 ? 4 : max_sweeps;
    bool done = false;
    while (launched < max_sweeps && !done) {
        const int32_t k = std::min(chunk, max_sweeps - launched);
        for (int32_t it = 0; it < k; ++it) {
            if (prof) NBGS_HIP(hipEventRecord(sc->pev[2 * (launched + it)], s));
            NBGS_TRY(subdomain_pass<T>(sc, 1, vel.p, corr.p));
            if (prof) NBGS_HIP(hipEventRecord(sc->pev[2 * (launched + it) + 1], s));
            if (every) NBGS_TRY(launch_residual(sc->partials.p, sc->n_sub, target, sc->ctrl(), sc->res_hist.p, s));
            else if (launched + it + 1 == max_sweeps)
                NBGS_TRY(launch_residual(sc->partials.p, sc->n_sub, target, sc->ctrl(), sc->res_hist.p, s,
                                         max_sweeps - 1));
        }
        launched += k;
        if (target > 0.0 && launched < max_sweeps) {
            NBGS_TRY(sync_small(sc, 8, 3));
            done = sc->pinned[8] != 0;
            chunk = std::min(chunk * 2, 64);
        }
    }
    return finish_solve<T>(sc, max_sweeps, target, stats, kSolveSubdomain);
}

// Block-local order: the initial impulses (the local part in the block pass,
// then the contacts between blocks colour by colour), then per sweep the block
// pass and the cross colours, and the residual over the blocks' and the cross
// tiles' partial sums.  The sequence of contacts is that of the sweep record:
// blocks in ascending id, each in (colour, key) order, then the cross
// contacts in (colour, key) order.
template <class T>
nbgs_status blk_solve(nbgs_scene_t sc, int32_t max_sweeps, double target, nbgs_stats *stats) {
    hipStream_t s = sc->s;
    const int32_t N = sc->b.n;
    SweepBuf<T> &sw = sweep_buf<T>(sc);
    DevBuf<T> &vel = vel_buf<T>(sc);
    const SweepTune &tune = sc->tune[sc->precision_used == NBGS_FP32_SWEEP ? 1 : 0];
    const int nx = (int)sc->xcol.size() - 1;
    const int64_t tile = sweep_tile<T>(tune);
    sc->xpart_off.assign((size_t)nx + 1, (int64_t)(sc->n_sub - 1));  // after the partials of the blocks and groups
    for (int c = 0; c < nx; ++c) {
        const int64_t m = sc->xcol[c + 1] - sc->xcol[c];
        sc->xpart_off[c + 1] = sc->xpart_off[c] + (m + tile - 1) / tile;
    }
    const int64_t n_partials = sc->xpart_off[(size_t)nx];
    if (n_partials > 0x7fffffff) {
        set_error("too many partial sums");
        return NBGS_ERR_CAPACITY;
    }
    NBGS_TRY(sc->partials.reserve(2 * (size_t)(n_partials > 0 ? n_partials : 1)));
    NBGS_HIP(hipMemsetAsync(sc->ctrl(), 0, 4 * sizeof(int32_t), s));
    // with a fixed sweep count and the history off only the last sweep's residual is formed
    const bool every = target > 0.0 || sc->res_history;
    sc->hist_partial = !every;
    sc->graph_pairs = 0;
    // records in the first grid's slot order (rec_on, set before they were written): the contacts' ends are records
    T *rv = vel.p;
    SweepView<T> xv = sw.view();
    if (sc->rec_on) {
        xv.j1 = sc->j1r.p;
        xv.j2 = sc->j2r.p;
    }
    if (sc->p.warm_start != NBGS_WS_ZERO) {
        NBGS_TRY(block_pass<T>(sc, 0, rv));
        for (int c = 0; c < nx; ++c)
            NBGS_TRY(launch_warm_scatter<T>(xv, sc->xcol[c], sc->xcol[c + 1], N, rv, s));
    }
    record(sc, kSweeps);
    const bool prof = sc->profiling;
    if (prof) NBGS_TRY(ensure_profile_events(sc, (size_t)max_sweeps));
    const SweepParams sp{sc->p.mu, sc->p.relax};
    int32_t launched = 0, chunk = target > 0.0 ? 4 : max_sweeps;
    bool done = false;
    while (launched < max_sweeps && !done) {
        const int32_t k = std::min(chunk, max_sweeps - launched);
        for (int32_t it = 0; it < k; ++it) {
            if (prof) NBGS_HIP(hipEventRecord(sc->pev[2 * (launched + it)], s));
            NBGS_TRY(block_pass<T>(sc, 1, rv));
            for (int c = 0; c < nx; ++c)
                NBGS_TRY(launch_sweep_colour<T>(xv, sc->xcol[c], sc->xcol[c + 1], N, rv, sp, tune,
                                                sc->partials.p + 2 * sc->xpart_off[c], sc->ctrl(), s));
            if (prof) NBGS_HIP(hipEventRecord(sc->pev[2 * (launched + it) + 1], s));
            if (every)
                NBGS_TRY(launch_residual(sc->partials.p, (int32_t)n_partials, target, sc->ctrl(), sc->res_hist.p, s));
            else if (launched + it + 1 == max_sweeps)
                NBGS_TRY(launch_residual(sc->partials.p, (int32_t)n_partials, target, sc->ctrl(), sc->res_hist.p, s,
                                         max_sweeps - 1));
        }
        launched += k;
        if (target > 0.0 && launched < max_sweeps) {
            NBGS_TRY(sync_small(sc, 8, 3));
            done = sc->pinned[8] != 0;
            chunk = std::min(chunk * 2, 64);
        }
    }
    return finish_solve<T>(sc, max_sweeps, target, stats, kSolveBlock);
}

template <class T>
nbgs_status solve_impl(nbgs_scene_t sc, int32_t max_sweeps, double target, nbgs_stats *stats) {
    hipStream_t s = sc->s;
    const int32_t N = sc->b.n;
    SweepBuf<T> &sw = sweep_buf<T>(sc);
    DevBuf<T> &vel = vel_buf<T>(sc);
    NBGS_TRY(vel.reserve(8 * (size_t)N));
    NBGS_TRY(sc->res_hist.reserve((size_t)max_sweeps));
    record(sc, kInit);
    sc->rec_on = false;  // body order until the block-local order's tables are in place (below)
    sc->winfo = nbgs_warm_info{-1, 0.0, 0.0};
    // few contacts on many bodies: records only for the bodies they touch (the sweeps read no other; the
    // integration and the export form the rest from the state); a small scene keeps the two launches fewer
    sc->sparse_bodies = N >= (1 << 16) && sc->nc < (int64_t)N / 8;
    if (sc->sparse_bodies) {
        NBGS_TRY(sc->touched.reserve((size_t)N + 1, 1.0));
        const ContactBuf &cb = sc->cb[sc->cur];
        NBGS_TRY(launch_mark_touched(cb.j1.p, cb.j2.p, sc->nc, N, sc->touched.p, s));
    }
    if (sc->p.warm_start == NBGS_WS_LEARNED && sc->have_learned) NBGS_TRY(judge_warm_start<T>(sc));
    // the block-local sweeps read and write each first-grid block's records as one contiguous range: the records
    // of this solve, its integration and its export are laid out in that order (same arithmetic, same order of
    // the contacts; only where each record lies changes)
    if (sc->blk_active && !sc->sub_active) NBGS_TRY(block_records(sc));
    NBGS_TRY(init_records<T>(sc, vel.p));
    if (sc->sub_active) return sub_solve<T>(sc, max_sweeps, target, stats);
    if (sc->blk_active) return blk_solve<T>(sc, max_sweeps, target, stats);
    if (sc->p.warm_start != NBGS_WS_ZERO)
        for (int c = 0; c < sc->n_colours; ++c)
            NBGS_TRY(launch_warm_scatter<T>(sw.view(), sc->col_off[c], sc->col_off[c + 1], N, vel.p, s));
    record(sc, kSweeps);
    const SweepTune &tune = sc->tune[sc->precision_used == NBGS_FP32_SWEEP ? 1 : 0];
    sc->part_off.assign((size_t)sc->n_colours + 1, 0);
    for (int c = 0; c < sc->n_colours; ++c) {
        const int64_t m = sc->col_off[c + 1] - sc->col_off[c];
        sc->part_off[c + 1] = sc->part_off[c] + (m + sweep_tile<T>(tune) - 1) / sweep_tile<T>(tune);
    }
    sc->n_partials = sc->part_off[sc->n_colours];
    NBGS_TRY(sc->partials.reserve(2 * (size_t)(sc->n_partials > 0 ? sc->n_partials : 1)));
    NBGS_HIP(hipMemsetAsync(sc->ctrl(), 0, 4 * sizeof(int32_t), s));
    SweepParams sp{sc->p.mu, sc->p.relax};
    int32_t launched = 0, chunk = target > 0.0 ? 4 : max_sweeps;
    bool done = false;
    const bool prof = sc->profiling;
    sc->graph_pairs = 0;
    if (tune.graph) {
        NBGS_TRY(scene_sweep_loop<T>(sc, max_sweeps, target, tune));
        done = true;
    } else if (prof) {
        NBGS_TRY(ensure_profile_events(sc, (size_t)max_sweeps * sc->n_colours));
    }
    size_t pe = 0;
    const bool every = target > 0.0 || sc->res_history;
    sc->hist_partial = !every;
    while (launched < max_sweeps && !done) {
        const int32_t k = std::min(chunk, max_sweeps - launched);
        for (int32_t it = 0; it < k; ++it) {
            for (int c = 0; c < sc->n_colours; ++c) {
                if (prof) NBGS_HIP(hipEventRecord(sc->pev[2 * pe], s));
                NBGS_TRY(launch_sweep_colour<T>(sw.view(), sc->col_off[c], sc->col_off[c + 1], N, vel.p, sp, tune,
                                                sc->partials.p + 2 * sc->part_off[c], sc->ctrl(), s));
                if (prof) NBGS_HIP(hipEventRecord(sc->pev[2 * pe + 1], s));
                ++pe;
            }
            const bool last = launched + it + 1 == max_sweeps;
            if (every) NBGS_TRY(launch_residual(sc->partials.p, (int32_t)sc->n_partials, target, sc->ctrl(), sc->res_hist.p, s));
            else if (last)
                NBGS_TRY(launch_residual(sc->partials.p, (int32_t)sc->n_partials, target, sc->ctrl(), sc->res_hist.p, s,
                                         max_sweeps - 1));
        }
        launched += k;
        if (target > 0.0 && launched < max_sweeps) {
            NBGS_TRY(sync_small(sc, 8, 3));
            done = sc->pinned[8] != 0;
            chunk = std::min(chunk * 2, 64);
        }
    }
    NBGS_TRY(launch_save_impulses<T>(sw.view(), sc->nc, sc->cb[sc->cur].view(), s));
    record(sc, kIntegrate);
    sc->state = 2;
    sc->solved = true;
    if (stats || target > 0.0) {
        int32_t sweeps = 0;
        double R = 0.0;
        NBGS_TRY(read_solve_result(sc, sweeps, R));
        sc->stats.sweeps = sweeps;
        sc->stats.residual = R;
        if (stats) *stats = sc->stats;
        if (prof) NBGS_TRY(accumulate_profile<T>(sc, sweeps));
        if (sc->pinned[8 + 2]) {
            set_error("non-finite residual after sweep %d", sweeps);
            return NBGS_ERR_NUMERIC;
        }
        if (target > 0.0 && !(R <= target)) {
            set_error("residual %.3e above target %.3e after %d sweeps", R, target, sweeps);
            return NBGS_ERR_NOT_CONVERGED;
        }
    } else {
        sc->stats.sweeps = max_sweeps;
        if (prof) NBGS_TRY(accumulate_profile<T>(sc, max_sweeps));
    }
    return NBGS_OK;
}

template <class T>
nbgs_status integrate_impl(nbgs_scene_t sc) {
    record(sc, kIntegrate);
    NBGS_TRY(launch_integrate<T>(sc->b, sc->grid, sc->table(), sc->p.dt, vel_buf<T>(sc).p,
                                 sc->sparse_bodies ? sc->touched.p : nullptr, sc->p.gravity, rec_map(sc), sc->s));
    record(sc, kNumPhases);
    sc->table_in_cur = true;
    sc->n_prev = sc->nc;
    sc->prev_colours = true;
    sc->state = 0;
    return NBGS_OK;
}



// Per-scene tables of a batch: body -> scene, body and wall offsets, walls,
// friction coefficients and colouring seeds (device copies), boxes (host).
nbgs_status setup_scene_tables(nbgs_scene_t sc, int32_t n_scenes, const int64_t *body_off, const nbgs_domain *domains,
                               const nbgs_params *params) {
    const int32_t N = sc->b.n;
    sc->body_off_h.resize((size_t)n_scenes + 1);
    sc->wall_off_h.resize((size_t)n_scenes + 1);
    sc->planes_h.resize((size_t)n_scenes);
    sc->lo_h.resize(3 * (size_t)n_scenes);
    sc->hi_h.resize(3 * (size_t)n_scenes);
    sc->periodic_h.resize(3 * (size_t)n_scenes);
    sc->mu_h.resize((size_t)n_scenes);
    sc->seed_h.resize((size_t)n_scenes);
    std::vector<int32_t> body_scene((size_t)N);
    int32_t walls = 0;
    for (int32_t s = 0; s < n_scenes; ++s) {
        sc->body_off_h[s] = (int32_t)body_off[s];
        sc->wall_off_h[s] = walls;
        walls += domains[s].n_planes;
        sc->planes_h[s] = plane_set(&domains[s]);
        for (int a = 0; a < 3; ++a) {
            sc->lo_h[3 * s + a] = domains[s].lo[a];
            sc->hi_h[3 * s + a] = domains[s].hi[a];
            sc->periodic_h[3 * s + a] = domains[s].periodic[a] ? 1 : 0;
        }
        sc->mu_h[s] = params[s].mu;
        sc->seed_h[s] = params[s].colour_seed;
        for (int64_t i = body_off[s]; i < body_off[s + 1]; ++i) body_scene[(size_t)i] = s;
    }
    sc->body_off_h[n_scenes] = N;
    sc->wall_off_h[n_scenes] = walls;
    NBGS_TRY(sc->body_scene_d.reserve((size_t)N, 1.0));
    NBGS_TRY(sc->body_off_d.reserve((size_t)n_scenes + 1, 1.0));
    NBGS_TRY(sc->wall_off_d.reserve((size_t)n_scenes + 1, 1.0));
    NBGS_TRY(sc->grids_d.reserve((size_t)n_scenes, 1.0));
    NBGS_TRY(sc->planes_d.reserve((size_t)n_scenes, 1.0));
    NBGS_TRY(sc->mu_d.reserve((size_t)n_scenes, 1.0));
    NBGS_TRY(sc->seed_d.reserve((size_t)n_scenes, 1.0));
    NBGS_HIP(hipMemcpy(sc->body_scene_d.p, body_scene.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice));
    NBGS_HIP(hipMemcpy(sc->body_off_d.p, sc->body_off_h.data(), sizeof(int32_t) * (n_scenes + 1), hipMemcpyHostToDevice));
    NBGS_HIP(hipMemcpy(sc->wall_off_d.p, sc->wall_off_h.data(), sizeof(int32_t) * (n_scenes + 1), hipMemcpyHostToDevice));
    NBGS_HIP(hipMemcpy(sc->planes_d.p, sc->planes_h.data(), sizeof(PlaneSet) * n_scenes, hipMemcpyHostToDevice));
    NBGS_HIP(hipMemcpy(sc->mu_d.p, sc->mu_h.data(), sizeof(double) * n_scenes, hipMemcpyHostToDevice));
    NBGS_HIP(hipMemcpy(sc->seed_d.p, sc->seed_h.data(), sizeof(uint64_t) * n_scenes, hipMemcpyHostToDevice));
    NBGS_HIP(hipHostMalloc((void **)&sc->grids_pinned, sizeof(Grid) * n_scenes));
    // batches replay their sweeps from a captured graph over a resident grid unless tuned otherwise
    for (SweepTune &t : sc->tune) {
        t.graph = 1;
        t.persistent = 1;
    }
    return NBGS_OK;
}

}  // namespace

namespace nbgs {

nbgs_status scene_create(void *workspace, size_t workspace_bytes, const nbgs_bodies *bodies, int32_t n_scenes,
                         const int64_t *body_off,
                         const nbgs_domain *domains, const nbgs_params *params, void *hip_stream, nbgs_scene_t *out) {
    *out = nullptr;
    if (!bodies || !domains || !params || !body_off) {
        set_error("bodies, domains, params or body offsets is NULL");
        return NBGS_ERR_INVALID_ARG;
    }
    if (n_scenes < 1) {
        set_error("at least one scene is needed");
        return NBGS_ERR_INVALID_ARG;
    }
    if (bodies->n < 1 || bodies->n >= (int64_t)0x7fffffc0) {
        set_error("body count %lld out of range", (long long)bodies->n);
        return NBGS_ERR_INVALID_ARG;
    }
    int64_t n_walls = 0;
    for (int32_t s = 0; s < n_scenes; ++s) {
        NBGS_TRY(check_params(&params[s]));
        NBGS_TRY(check_domain(&domains[s]));
        if (!(body_off[s + 1] > body_off[s])) {
            set_error("scene %d holds no body (offsets must increase)", s);
            return NBGS_ERR_INVALID_ARG;
        }
        n_walls += domains[s].n_planes;
        if (s > 0) {
            const nbgs_params &a = params[0], &b = params[s];
            if (a.dt != b.dt || a.gravity[0] != b.gravity[0] || a.gravity[1] != b.gravity[1] ||
                a.gravity[2] != b.gravity[2] || a.tau != b.tau || a.relax != b.relax || a.erp != b.erp ||
                a.precision != b.precision || a.warm_start != b.warm_start) {
                set_error("batched scenes may differ only in mu and colour_seed (scene %d differs)", s);
                return NBGS_ERR_INVALID_ARG;
            }
        }
    }
    if (body_off[0] != 0 || body_off[n_scenes] != bodies->n) {
        set_error("body offsets must run from 0 to the body count");
        return NBGS_ERR_INVALID_ARG;
    }
    if (n_scenes > 1 && params[0].warm_start == NBGS_WS_LEARNED) {
        set_error("the learned warm start is not available for batched scenes");
        return NBGS_ERR_UNSUPPORTED;
    }
    if (bodies->n + n_walls >= (int64_t)0x7fffffc0) {
        set_error("too many bodies and walls");
        return NBGS_ERR_INVALID_ARG;
    }
    const nbgs_domain *domain = &domains[0];
    const void *ptrs[] = {bodies->x,  bodies->y,  bodies->z,  bodies->qw, bodies->qx, bodies->qy,
                          bodies->qz, bodies->vx, bodies->vy, bodies->vz, bodies->wx, bodies->wy,
                          bodies->wz, bodies->radius, bodies->inv_mass, bodies->inv_inertia};
    for (const void *q : ptrs)
        if (!q) {
            set_error("a body array pointer is NULL");
            return NBGS_ERR_INVALID_ARG;
        }
    nbgs_scene_t sc = new (std::nothrow) nbgs_scene_s();
    if (!sc) {
        set_error("host allocation failed");
        return NBGS_ERR_OUT_OF_MEMORY;
    }
    sc->s = (hipStream_t)hip_stream;
    sc->arena.reset(workspace, workspace_bytes);
    if (!sc->arena.bound()) {
        delete sc;
        set_error("the workspace is NULL or too small (nbgs_workspace_query gives its size)");
        return NBGS_ERR_INVALID_ARG;
    }
    ArenaScope arena_scope(&sc->arena);
    // default launch shapes, the fastest measured on the dense 1M packing: lane groups with non-temporal contact
    // loads in FP64, lane groups over a resident grid in FP32
    sc->tune[0].lanes = 1;
    sc->tune[0].nontemporal = 1;
    sc->tune[1].lanes = 1;
    sc->tune[1].persistent = 1;
    BodiesView &b = sc->b;
    b.n = (int32_t)bodies->n;
    b.x = bodies->x;
    b.y = bodies->y;
    b.z = bodies->z;
    b.qw = bodies->qw;
    b.qx = bodies->qx;
    b.qy = bodies->qy;
    b.qz = bodies->qz;
    b.vx = bodies->vx;
    b.vy = bodies->vy;
    b.vz = bodies->vz;
    b.wx = bodies->wx;
    b.wy = bodies->wy;
    b.wz = bodies->wz;
    b.radius = bodies->radius;
    b.inv_mass = bodies->inv_mass;
    b.inv_inertia = bodies->inv_inertia;
    sc->planes = plane_set(domain);
    for (int a = 0; a < 3; ++a) {
        sc->lo[a] = domain->lo[a];
        sc->hi[a] = domain->hi[a];
        sc->periodic[a] = domain->periodic[a] ? 1 : 0;
    }
    sc->p = params[0];
    sc->n_scenes = n_scenes;
    const size_t N = (size_t)b.n;
    nbgs_status st = NBGS_OK;
    auto chk = [&](nbgs_status x) {
        if (st == NBGS_OK) st = x;
    };
    chk(sc->h.reserve(N, 1.0));
    chk(sc->keys.reserve(N, 1.0));
    chk(sc->ids.reserve(N, 1.0));
    chk(sc->keys2.reserve(N, 1.0));
    chk(sc->ids2.reserve(N, 1.0));
    chk(sc->sxr.reserve(N, 1.0));
    chk(sc->xr.reserve(N, 1.0));
    chk(sc->cnt.reserve(N + 1, 1.0));
    chk(sc->npart.reserve(N, 1.0));
    chk(sc->partners.reserve((size_t)kPartnerCap * N, 1.0));
    chk(sc->cellpos.reserve(N, 1.0));
    chk(sc->off.reserve(N + 1, 1.0));
    chk(sc->deg2.reserve(N + 1, 1.0));
    chk(sc->off2.reserve(N + 1, 1.0));
    chk(sc->cursor.reserve(N + 1, 1.0));
    chk(sc->radix_hist.reserve(radix_hist_entries((int64_t)N + 1), 1.0));
    chk(sc->scan_tmp.reserve(exclusive_scan_tmp_bytes((int64_t)radix_hist_entries((int64_t)N + 1) + N + 1), 1.0));
    chk(sc->small.reserve(kSmallInts, 1.0));
    chk(sc->maxbits.reserve(5, 1.0));
    if (st == NBGS_OK && hipHostMalloc((void **)&sc->pinned, sizeof(int32_t) * kSmallInts * 2) != hipSuccess) {
        set_error("pinned host allocation failed");
        st = NBGS_ERR_OUT_OF_MEMORY;
    }
    for (int i = 0; i <= kNumPhases && st == NBGS_OK; ++i)
        if (hipEventCreate(&sc->ev[i]) != hipSuccess) sc->ev[i] = nullptr;
    if (st == NBGS_OK) {
        // static bodies must not rotate either (walls and fixed spheres have infinite inertia)
        std::vector<double> im(N), ii(N);
        if (hipMemcpy(im.data(), b.inv_mass, N * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(ii.data(), b.inv_inertia, N * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
            set_error("could not read inv_mass / inv_inertia (not device pointers?)");
            st = NBGS_ERR_INVALID_ARG;
        } else {
            for (size_t i = 0; i < N; ++i)
                if (!(im[i] >= 0.0) || !(ii[i] >= 0.0) || (im[i] == 0.0 && ii[i] != 0.0)) {
                    set_error("body %zu: inverse mass/inertia must be >= 0 and a static body (1/m = 0) needs 1/I = 0",
                              i);
                    st = NBGS_ERR_INVALID_ARG;
                    break;
                }
            std::vector<double> rad(N);
            if (st == NBGS_OK && hipMemcpy(rad.data(), b.radius, N * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
                set_error("could not read radius");
                st = NBGS_ERR_INVALID_ARG;
            }
            if (st == NBGS_OK) {
                double sm = 0.0, sr = 0.0;
                size_t nd = 0;
                for (size_t i = 0; i < N; ++i) {
                    sr += rad[i];
                    if (im[i] > 0.0) {
                        sm += 1.0 / im[i];
                        ++nd;
                    }
                }
                sc->mean_mass = nd ? sm / (double)nd : 1.0;
                sc->mean_radius = sr / (double)N;
                update_scales(sc);
            }
        }
    }
    if (st == NBGS_OK && n_scenes > 1) st = setup_scene_tables(sc, n_scenes, body_off, domains, params);
    if (st != NBGS_OK) {
        nbgs_scene_destroy(sc);
        return st;
    }
    *out = sc;
    return NBGS_OK;
}

}  // namespace nbgs


namespace nbgs {
const char *last_error_cstr();
}

// A NULL handle is refused; the handle's arena takes the buffers allocated
// until the entry point returns.
#define NBGS_GUARD(sc)                                                                                          \
    if (!(sc)) {                                                                                                \
        set_error("scene handle is NULL");                                                                      \
        return NBGS_ERR_INVALID_ARG;                                                                            \
    }                                                                                                           \
    ArenaScope arena_scope_(&(sc)->arena)

extern "C" {

int32_t nbgs_abi_version(void) { return NBGS_ABI_VERSION; }

const char *nbgs_last_error(void) { return nbgs::last_error_cstr(); }

nbgs_status nbgs_workspace_query(int64_t n_bodies, int64_t contact_capacity, const nbgs_params *params,
                                 size_t *bytes) {
    if (!bytes || n_bodies < 0 || contact_capacity < 0) {
        set_error("bad arguments to nbgs_workspace_query");
        return NBGS_ERR_INVALID_ARG;
    }
    if (params) NBGS_TRY(check_params(params));
    *bytes = scene_workspace_bytes(n_bodies, contact_capacity, 1);
    return NBGS_OK;
}

nbgs_status nbgs_scene_workspace_query(nbgs_scene_t sc, int64_t contact_capacity, size_t *bytes) {
    if (!sc || !bytes || contact_capacity < 0) {
        set_error("bad arguments to nbgs_scene_workspace_query");
        return NBGS_ERR_INVALID_ARG;
    }
    return scene_need_bytes(sc, contact_capacity, bytes);
}

nbgs_status nbgs_scene_create(const nbgs_bodies *bodies, const nbgs_domain *domain, const nbgs_params *params,
                              void *workspace, size_t workspace_bytes, void *hip_stream, nbgs_scene_t *out) {
    if (!out) {
        set_error("out is NULL");
        return NBGS_ERR_INVALID_ARG;
    }
    *out = nullptr;
    if (!bodies) {
        set_error("bodies is NULL");
        return NBGS_ERR_INVALID_ARG;
    }
    const int64_t off[2] = {0, bodies->n};
    return scene_create(workspace, workspace_bytes, bodies, 1, off, domain, params, hip_stream, out);
}

nbgs_status nbgs_scene_set_workspace(nbgs_scene_t sc, void *workspace, size_t bytes) {
    NBGS_GUARD(sc);
    NBGS_TRY(sc->arena.move_to(workspace, bytes, sc->s));
    // addresses kept inside moved buffers
    sc->perm = static_cast<const uint32_t *>(sc->arena.relocate(sc->perm));
    sc->skeys = static_cast<const uint32_t *>(sc->arena.relocate(sc->skeys));
    sc->sids = static_cast<const uint32_t *>(sc->arena.relocate(sc->sids));
    sc->vl_blocked = false;  // a new workspace may hold the pair list
    sc->body_slots = static_cast<const uint32_t *>(sc->arena.relocate(sc->body_slots));
    return NBGS_OK;
}

nbgs_status nbgs_scene_workspace_usage(nbgs_scene_t sc, size_t *size, size_t *used, size_t *peak) {
    NBGS_GUARD(sc);
    if (size) *size = sc->arena.size();
    if (used) *used = sc->arena.used();
    if (peak) *peak = sc->arena.peak();
    return NBGS_OK;
}

nbgs_status nbgs_scene_destroy(nbgs_scene_t sc) {
    if (!sc) return NBGS_OK;
    (void)hipStreamSynchronize(sc->s);
    for (int i = 0; i <= kNumPhases; ++i)
        if (sc->ev[i]) (void)hipEventDestroy(sc->ev[i]);
    for (hipEvent_t e : sc->pev) (void)hipEventDestroy(e);
    if (sc->pinned) (void)hipHostFree(sc->pinned);
    if (sc->grids_pinned) (void)hipHostFree(sc->grids_pinned);
    if (sc->col_pinned) (void)hipHostFree(sc->col_pinned);
    if (sc->gexec) (void)hipGraphExecDestroy(sc->gexec);
    if (sc->cap_stream) (void)hipStreamDestroy(sc->cap_stream);
    delete sc;
    return NBGS_OK;
}

nbgs_status nbgs_scene_set_params(nbgs_scene_t sc, const nbgs_params *params) {
    NBGS_GUARD(sc);
    NBGS_TRY(check_params(params));
    if (sc->n_scenes > 1 && params->warm_start == NBGS_WS_LEARNED) {
        set_error("the learned warm start is not available for batched scenes");
        return NBGS_ERR_UNSUPPORTED;
    }
    if (sc->sub_edge > 0.0 && params->warm_start == NBGS_WS_LEARNED) {
        set_error("the subdomain solver does not combine with the learned warm start");
        return NBGS_ERR_UNSUPPORTED;
    }
    if (sc->blk_edge > 0.0 && params->warm_start == NBGS_WS_LEARNED) {
        set_error("the block-local order does not combine with the learned warm start");
        return NBGS_ERR_UNSUPPORTED;
    }
    if (sc->sub_edge > 0.0 && !(params->relax < 1.0)) {
        set_error("the subdomain solver needs a relaxation below 1: switch it off first");
        return NBGS_ERR_INVALID_ARG;
    }
    sc->p = *params;
    sc->vl_valid = false;  // the pair list was built for the old margin (tau) and step
    update_scales(sc);
    return NBGS_OK;
}

nbgs_status nbgs_detect(nbgs_scene_t sc, nbgs_stats *stats) {
    NBGS_GUARD(sc);
    sc->state = 0;
    sc->nc_needed = -1;
    nbgs_status st = detect_impl(sc, stats);
    if (st == NBGS_ERR_CAPACITY && sc->nc_needed < 0 && (sc->vl_h.p || sc->vl_j1.p)) {
        // A buffer did not fit beside the pair list although the contact count did: the list gives its room back
        // and is built no more in this workspace; the detection runs once more with the cell grid (the colouring
        // of the failed run is not reused).
        for (DevBuf<int32_t> *b : {&sc->vl_j1, &sc->vl_j2, &sc->vl_flag, &sc->vl_off}) b->release();
        for (DevBuf<double> *b : {&sc->vl_h, &sc->vl_x0, &sc->vl_r0}) b->release();
        sc->vl_static0.release();
        sc->vl_valid = false;
        sc->vl_blocked = true;
        sc->prev_sig_valid = false;
        sc->dyn_bits_valid = false;
        st = detect_impl(sc, stats);
    }
    // a failed detection may have updated per-body state (hull radii, dynamic bits): the next one reuses nothing
    if (st != NBGS_OK) sc->prev_sig_valid = false;
    if (st == NBGS_ERR_CAPACITY) {
        // what was lacking: the contact count found, for nbgs_workspace_query
        if (stats) {
            *stats = nbgs_stats{};
            stats->n_contacts = sc->nc_needed;
        }
    }
    return st;
}

nbgs_status nbgs_solve(nbgs_scene_t sc, int32_t max_sweeps, double residual_target, nbgs_stats *stats) {
    NBGS_GUARD(sc);
    if (sc->state < 1) {
        set_error("nbgs_solve needs a preceding nbgs_detect");
        return NBGS_ERR_STATE;
    }
    if (max_sweeps < 1) {
        set_error("max_sweeps must be >= 1");
        return NBGS_ERR_INVALID_ARG;
    }
    if (sc->precision_used == NBGS_FP32_SWEEP) return solve_impl<float>(sc, max_sweeps, residual_target, stats);
    return solve_impl<double>(sc, max_sweeps, residual_target, stats);
}

nbgs_status nbgs_integrate(nbgs_scene_t sc) {
    NBGS_GUARD(sc);
    if (sc->state != 2) {
        set_error("nbgs_integrate needs a preceding nbgs_solve");
        return NBGS_ERR_STATE;
    }
    if (sc->precision_used == NBGS_FP32_SWEEP) return integrate_impl<float>(sc);
    return integrate_impl<double>(sc);
}

nbgs_status nbgs_step(nbgs_scene_t sc, int32_t max_sweeps, double residual_target, nbgs_stats *stats) {
    NBGS_GUARD(sc);
    nbgs_stats dst{};
    const nbgs_status ds = nbgs_detect(sc, &dst);
    if (ds != NBGS_OK) {
        if (ds == NBGS_ERR_CAPACITY && stats) *stats = dst;  // the contact count the workspace lacks
        return ds;
    }
    nbgs_status st = nbgs_solve(sc, max_sweeps, residual_target, stats);
    if (st != NBGS_OK && st != NBGS_ERR_NOT_CONVERGED) return st;
    NBGS_TRY(nbgs_integrate(sc));
    return st;
}

nbgs_status nbgs_get_contacts(nbgs_scene_t sc, int64_t cap, int32_t *j1, int32_t *j2, uint64_t *key,
                              int32_t *colour, double *normal, double *xi, double *impulse, int64_t *n_out) {
    NBGS_GUARD(sc);
    if (n_out) *n_out = sc->nc;
    if (sc->nc > cap) {
        set_error("%lld contacts do not fit into %lld", (long long)sc->nc, (long long)cap);
        return NBGS_ERR_CAPACITY;
    }
    const int64_t m = sc->nc;
    if (m == 0) return NBGS_OK;
    ContactBuf &cb = sc->cb[sc->table_in_cur ? sc->cur : sc->cur];
    hipStream_t s = sc->s;
    auto cp = [&](void *dst, const void *src, size_t bytes) -> nbgs_status {
        if (!dst) return NBGS_OK;
        NBGS_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s));
        return NBGS_OK;
    };
    NBGS_TRY(cp(j1, cb.j1.p, m * sizeof(int32_t)));
    NBGS_TRY(cp(j2, cb.j2.p, m * sizeof(int32_t)));
    NBGS_TRY(cp(key, cb.key.p, m * sizeof(uint64_t)));
    NBGS_TRY(cp(colour, cb.colour.p, m * sizeof(int32_t)));
    NBGS_TRY(cp(xi, cb.xi.p, m * sizeof(double)));
    if (normal) {
        NBGS_TRY(cp(normal, cb.nx.p, m * sizeof(double)));
        NBGS_TRY(cp(normal + cap, cb.ny.p, m * sizeof(double)));
        NBGS_TRY(cp(normal + 2 * cap, cb.nz.p, m * sizeof(double)));
    }
    if (impulse) {
        NBGS_TRY(cp(impulse, cb.px.p, m * sizeof(double)));
        NBGS_TRY(cp(impulse + cap, cb.py.p, m * sizeof(double)));
        NBGS_TRY(cp(impulse + 2 * cap, cb.pz.p, m * sizeof(double)));
    }
    NBGS_HIP(hipStreamSynchronize(s));
    return NBGS_OK;
}

nbgs_status nbgs_get_accumulators(nbgs_scene_t sc, double *v, double *w) {
    NBGS_GUARD(sc);
    if (!v || !w) {
        set_error("v and w must be device buffers of 3 n doubles");
        return NBGS_ERR_INVALID_ARG;
    }
    if (sc->precision_used == NBGS_FP32_SWEEP) {
        if (!sc->vel32.p) {
            set_error("no solve yet");
            return NBGS_ERR_STATE;
        }
        return launch_export_accumulators<float>(sc->vel32.p, sc->b.n, v, w, sc->b,
                                                 sc->sparse_bodies ? sc->touched.p : nullptr, sc->state == 2,
                                                 sc->p.gravity, sc->p.dt, rec_map(sc), sc->s);
    }
    if (!sc->vel64.p) {
        set_error("no solve yet");
        return NBGS_ERR_STATE;
    }
    return launch_export_accumulators<double>(sc->vel64.p, sc->b.n, v, w, sc->b,
                                              sc->sparse_bodies ? sc->touched.p : nullptr, sc->state == 2,
                                              sc->p.gravity, sc->p.dt, rec_map(sc), sc->s);
}

nbgs_status nbgs_get_residuals(nbgs_scene_t sc, int32_t cap, double *hist, int32_t *n_out) {
    NBGS_GUARD(sc);
    NBGS_HIP(hipStreamSynchronize(sc->s));
    int32_t ctrl[4] = {0, 0, 0, 0};
    if (sc->small.p) NBGS_HIP(hipMemcpy(ctrl, sc->ctrl(), sizeof(ctrl), hipMemcpyDeviceToHost));
    const int32_t n = ctrl[1];
    if (n_out) *n_out = n;
    const int32_t k = std::min(cap, n);
    if (k > 0 && hist) {
        NBGS_HIP(hipMemcpy(hist, sc->res_hist.p, sizeof(double) * k, hipMemcpyDeviceToHost));
        if (sc->hist_partial)  // only the last sweep was summed
            for (int32_t i = 0; i < k && i < n - 1; ++i) hist[i] = std::nan("");
    }
    return NBGS_OK;
}

nbgs_status nbgs_set_subdomains(nbgs_scene_t sc, double edge) {
    NBGS_GUARD(sc);
    if (!(edge >= 0.0) || !std::isfinite(edge)) {
        set_error("the subdomain edge must be finite and >= 0");
        return NBGS_ERR_INVALID_ARG;
    }
    if (edge > 0.0 && sc->n_scenes > 1) {
        set_error("the subdomain solver is not available for batched scenes");
        return NBGS_ERR_UNSUPPORTED;
    }
    if (edge > 0.0 && sc->p.warm_start == NBGS_WS_LEARNED) {
        set_error("the subdomain solver does not combine with the learned warm start");
        return NBGS_ERR_UNSUPPORTED;
    }
    if (edge > 0.0 && sc->blk_edge > 0.0) {
        set_error("the block-local order is set: switch it off first");
        return NBGS_ERR_INVALID_ARG;
    }
    if (edge > 0.0 && !(sc->p.relax < 1.0)) {
        set_error("the subdomain solver needs a relaxation below 1 (across subdomains it is a Jacobi iteration, "
                  "which diverges unrelaxed on dense packings); the paper's runs use 0.75");
        return NBGS_ERR_INVALID_ARG;
    }
    sc->sub_edge = edge;
    sc->state = 0;  // the next step starts with a detection
    return NBGS_OK;
}

nbgs_status nbgs_set_block_order(nbgs_scene_t sc, double edge) {
    NBGS_GUARD(sc);
    if (!(edge >= 0.0) || !std::isfinite(edge)) {
        set_error("the block edge must be finite and >= 0");
        return NBGS_ERR_INVALID_ARG;
    }
    if (edge > 0.0 && sc->n_scenes > 1) {
        set_error("the block-local order is not available for batched scenes");
        return NBGS_ERR_UNSUPPORTED;
    }
    if (edge > 0.0 && sc->p.warm_start == NBGS_WS_LEARNED) {
        set_error("the block-local order does not combine with the learned warm start");
        return NBGS_ERR_UNSUPPORTED;
    }
    if (edge > 0.0 && sc->sub_edge > 0.0) {
        set_error("the subdomain solver is set: switch it off first");
        return NBGS_ERR_INVALID_ARG;
    }
    sc->blk_edge = edge;
    sc->state = 0;  // the next step starts with a detection
    return NBGS_OK;
}

nbgs_status nbgs_set_block_grids(nbgs_scene_t sc, int32_t grids) {
    NBGS_GUARD(sc);
    if (grids < 1 || grids > 8) {
        set_error("block grids must be 1 .. 8");
        return NBGS_ERR_INVALID_ARG;
    }
    sc->blk_grids = grids;
    sc->state = 0;  // the next step starts with a detection
    return NBGS_OK;
}

nbgs_status nbgs_set_pair_list(nbgs_scene_t sc, int32_t enable) {
    NBGS_GUARD(sc);
    sc->vl_enabled = enable != 0;
    sc->vl_valid = false;
    return NBGS_OK;
}

nbgs_status nbgs_get_pair_list_info(nbgs_scene_t sc, int64_t *pairs, double *skin, int64_t *builds) {
    NBGS_GUARD(sc);
    if (pairs) *pairs = sc->vl_valid ? sc->vl_n : -1;
    if (skin) *skin = sc->vl_valid ? sc->vl_skin : 0.0;
    if (builds) *builds = sc->vl_builds;
    return NBGS_OK;
}

nbgs_status nbgs_set_residual_history(nbgs_scene_t sc, int32_t enable) {
    NBGS_GUARD(sc);
    sc->res_history = enable != 0;
    return NBGS_OK;
}

nbgs_status nbgs_set_warm_start(nbgs_scene_t sc, int64_t n, const uint64_t *keys, const double *impulse) {
    NBGS_GUARD(sc);
    if (n < 0 || (n > 0 && (!keys || !impulse))) {
        set_error("bad warm-start table");
        return NBGS_ERR_INVALID_ARG;
    }
    if (sc->table_in_cur) {
        sc->cur = 1 - sc->cur;
        sc->table_in_cur = false;
    }
    ContactBuf &prev = sc->cb[1 - sc->cur];
    NBGS_TRY(prev.reserve((size_t)(n > 0 ? n : 1)));
    if (n > 0) {
        NBGS_HIP(hipMemcpyAsync(prev.key.p, keys, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, sc->s));
        NBGS_HIP(hipMemcpyAsync(prev.px.p, impulse, n * sizeof(double), hipMemcpyDeviceToDevice, sc->s));
        NBGS_HIP(hipMemcpyAsync(prev.py.p, impulse + n, n * sizeof(double), hipMemcpyDeviceToDevice, sc->s));
        NBGS_HIP(hipMemcpyAsync(prev.pz.p, impulse + 2 * n, n * sizeof(double), hipMemcpyDeviceToDevice, sc->s));
    }
    sc->n_prev = n;
    sc->prev_colours = false;
    return NBGS_OK;
}

nbgs_status nbgs_get_phase_times(nbgs_scene_t sc, int32_t n, double *out) {
    NBGS_GUARD(sc);
    if (!out || n < 0 || n > kNumPhases) {
        set_error("out must hold up to %d values", kNumPhases);
        return NBGS_ERR_INVALID_ARG;
    }
    NBGS_HIP(hipStreamSynchronize(sc->s));
    for (int i = 0; i < n; ++i) {
        float ms = 0.0f;
        if (sc->ev_ok[i] && sc->ev_ok[i + 1] && hipEventElapsedTime(&ms, sc->ev[i], sc->ev[i + 1]) == hipSuccess)
            out[i] = ms;
        else
            out[i] = 0.0;
    }
    return NBGS_OK;
}

nbgs_status nbgs_scene_attach_mlp(nbgs_scene_t sc, nbgs_mlp_t mlp) {
    NBGS_GUARD(sc);
    if (sc->n_scenes > 1) {
        set_error("the learned warm start is not available for batched scenes");
        return NBGS_ERR_UNSUPPORTED;
    }
    sc->mlp = mlp;
    return NBGS_OK;
}

nbgs_status nbgs_set_feature_capture(nbgs_scene_t sc, int32_t enable) {
    NBGS_GUARD(sc);
    if (sc->n_scenes > 1 && enable) {
        set_error("network features are not available for batched scenes");
        return NBGS_ERR_UNSUPPORTED;
    }
    sc->capture = enable != 0;
    return NBGS_OK;
}

nbgs_status nbgs_get_feature_scales(nbgs_scene_t sc, double *out) {
    NBGS_GUARD(sc);
    if (!out) {
        set_error("out is NULL");
        return NBGS_ERR_INVALID_ARG;
    }
    out[0] = sc->fs.vs;
    out[1] = sc->fs.ms;
    out[2] = sc->fs.rs;
    return NBGS_OK;
}

nbgs_status nbgs_get_training_data(nbgs_scene_t sc, int64_t cap, float *feat, float *target, int64_t *n_out) {
    NBGS_GUARD(sc);
    if (n_out) *n_out = sc->nc;
    if (!sc->have_features || !sc->solved) {
        set_error("training data needs features from nbgs_detect (capture or learned warm start) and a solve");
        return NBGS_ERR_STATE;
    }
    if (sc->nc > cap) {
        set_error("%lld contacts do not fit into %lld", (long long)sc->nc, (long long)cap);
        return NBGS_ERR_CAPACITY;
    }
    if (sc->nc == 0) return NBGS_OK;
    if (feat)
        NBGS_HIP(hipMemcpyAsync(feat, sc->feat.p, sizeof(float) * 12 * sc->nc, hipMemcpyDeviceToDevice, sc->s));
    if (target) NBGS_TRY(launch_targets(sc->frame.p, sc->cb[sc->cur].view(), sc->nc, sc->fs, target, sc->s));
    NBGS_HIP(hipStreamSynchronize(sc->s));
    return NBGS_OK;
}

nbgs_status nbgs_mlp_collect(nbgs_scene_t sc, nbgs_mlp_t mlp, int64_t *n_stored) {
    NBGS_GUARD(sc);
    if (!mlp) {
        set_error("network handle is NULL");
        return NBGS_ERR_INVALID_ARG;
    }
    if (!sc->have_features || !sc->solved) {
        set_error("collecting needs features from nbgs_detect (capture or learned warm start) and a solve");
        return NBGS_ERR_STATE;
    }
    float *feat = nullptr, *tgt = nullptr;
    NBGS_TRY(mlp_store_slot(mlp, sc->nc, &feat, &tgt));
    if (sc->nc > 0) {
        NBGS_HIP(hipMemcpyAsync(feat, sc->feat.p, sizeof(float) * 12 * sc->nc, hipMemcpyDeviceToDevice, sc->s));
        NBGS_TRY(launch_targets(sc->frame.p, sc->cb[sc->cur].view(), sc->nc, sc->fs, tgt, sc->s));
        NBGS_HIP(hipStreamSynchronize(sc->s));  // the network's stream reads the store next
    }
    mlp_store_commit(mlp, sc->nc);
    if (n_stored) NBGS_TRY(nbgs_mlp_collected(mlp, n_stored, nullptr, nullptr));
    return NBGS_OK;
}

nbgs_status nbgs_get_warm_start_info(nbgs_scene_t sc, nbgs_warm_info *out) {
    NBGS_GUARD(sc);
    if (!out) {
        set_error("out is NULL");
        return NBGS_ERR_INVALID_ARG;
    }
    *out = sc->winfo;
    return NBGS_OK;
}

nbgs_status nbgs_get_learned_start(nbgs_scene_t sc, int64_t cap, double *impulse, int64_t *n_out) {
    NBGS_GUARD(sc);
    if (n_out) *n_out = sc->nc;
    if (!sc->have_learned) {
        set_error("no learned start: the last nbgs_detect ran without NBGS_WS_LEARNED and an attached network");
        return NBGS_ERR_STATE;
    }
    if (sc->nc > cap) {
        set_error("%lld contacts do not fit into %lld", (long long)sc->nc, (long long)cap);
        return NBGS_ERR_CAPACITY;
    }
    if (sc->nc == 0 || !impulse) return NBGS_OK;
    const size_t bytes = sizeof(double) * (size_t)sc->nc;
    NBGS_HIP(hipMemcpyAsync(impulse, sc->lpx.p, bytes, hipMemcpyDeviceToDevice, sc->s));
    NBGS_HIP(hipMemcpyAsync(impulse + cap, sc->lpy.p, bytes, hipMemcpyDeviceToDevice, sc->s));
    NBGS_HIP(hipMemcpyAsync(impulse + 2 * cap, sc->lpz.p, bytes, hipMemcpyDeviceToDevice, sc->s));
    NBGS_HIP(hipStreamSynchronize(sc->s));
    return NBGS_OK;
}

nbgs_status nbgs_set_tuning(nbgs_scene_t sc, int32_t precision, const nbgs_tuning *t) {
    NBGS_GUARD(sc);
    if (!t || (precision != NBGS_FP64 && precision != NBGS_FP32_SWEEP)) {
        set_error("bad tuning arguments");
        return NBGS_ERR_INVALID_ARG;
    }
    SweepTune st;
    st.block = t->block;
    st.cpt = t->contacts_per_thread;
    st.xcd_remap = t->xcd_remap;
    st.nontemporal = t->nontemporal;
    st.full_store = t->full_store;
    st.persistent = t->persistent;
    st.graph = t->graph;
    st.lanes = t->lane_groups;
    if (!sweep_tune_supported(st)) {
        set_error("unsupported tuning: block %d, contacts_per_thread %d, xcd_remap %d, nontemporal %d, full_store %d, "
                  "persistent %d, graph %d, lane_groups %d",
                  t->block, t->contacts_per_thread, t->xcd_remap, t->nontemporal, t->full_store, t->persistent,
                  t->graph, t->lane_groups);
        return NBGS_ERR_INVALID_ARG;
    }
    sc->tune[precision] = st;
    sc->tuned[precision] = true;
    return NBGS_OK;
}

nbgs_status nbgs_get_tuning(nbgs_scene_t sc, int32_t precision, nbgs_tuning *t) {
    NBGS_GUARD(sc);
    if (!t || (precision != NBGS_FP64 && precision != NBGS_FP32_SWEEP)) {
        set_error("bad tuning arguments");
        return NBGS_ERR_INVALID_ARG;
    }
    const SweepTune &st = sc->tune[precision];
    t->block = st.block;
    t->contacts_per_thread = st.cpt;
    t->xcd_remap = st.xcd_remap;
    t->nontemporal = st.nontemporal;
    t->full_store = st.full_store;
    t->persistent = st.persistent;
    t->graph = st.graph;
    t->lane_groups = st.lanes;
    return NBGS_OK;
}

nbgs_status nbgs_set_profiling(nbgs_scene_t sc, int32_t enable) {
    NBGS_GUARD(sc);
    sc->profiling = enable != 0;
    sc->prof = nbgs_profile{};
    return NBGS_OK;
}

nbgs_status nbgs_get_profile(nbgs_scene_t sc, nbgs_profile *out) {
    NBGS_GUARD(sc);
    if (!out) {
        set_error("out is NULL");
        return NBGS_ERR_INVALID_ARG;
    }
    *out = sc->prof;
    return NBGS_OK;
}

}  // extern "C"
