// Internal declarations of the gfx950 hard-contact solver library.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/nbgs.h"
#include "sweep_types.h"

namespace nbgs {

// ----------------------------------------------------------------- errors

void set_error(const char *fmt, ...);

#define NBGS_HIP(call)                                                                                          \
    do {                                                                                                        \
        hipError_t e_ = (call);                                                                                 \
        if (e_ != hipSuccess) {                                                                                 \
            ::nbgs::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__);       \
            return NBGS_ERR_DEVICE;                                                                             \
        }                                                                                                       \
    } while (0)

#define NBGS_TRY(expr)                                                                                          \
    do {                                                                                                        \
        nbgs_status s_ = (expr);                                                                                \
        if (s_ != NBGS_OK) return s_;                                                                           \
    } while (0)

// Bumped by every (re)allocation or move of a device buffer: a captured graph
// holds raw device addresses and stays valid only while no buffer has moved
// since.
inline std::atomic<uint64_t> g_alloc_generation{0};

// A buffer that lives in an Arena and can be told where it moved.
struct ArenaBuf {
    virtual void arena_moved(void *p) = 0;

   protected:
    ~ArenaBuf() = default;
};

// The device memory of one handle (scene, batch, composite scene, network):
// a region the caller allocated (a torch byte tensor) from which the handle's
// buffers are carved, first fit, 256-byte aligned.  The library allocates no
// device memory of its own.  Host-side bookkeeping only; every buffer is used
// on the handle's stream, so a released range can be handed out again at
// once (later work on the stream runs after earlier work).
class Arena {
   public:
    static constexpr size_t kAlign = 256;
    Arena() = default;
    Arena(const Arena &) = delete;
    Arena &operator=(const Arena &) = delete;
    // an empty arena over [base, base + bytes) (the base is aligned up to kAlign)
    void reset(void *base, size_t bytes);
    bool bound() const { return base_ != nullptr; }
    size_t size() const { return size_; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    // nullptr when no free run of that many bytes is left
    void *alloc(size_t bytes, ArenaBuf *owner);
    void release(void *p);
    // Copy every live buffer, packed, into the region [base, base + bytes) on
    // stream s, tell each one where it went, and continue in that region; the
    // old region is free once the call returns (it synchronises the stream).
    // CAPACITY (nothing moved) if the live buffers do not fit.
    nbgs_status move_to(void *base, size_t bytes, hipStream_t s);
    // Where an address inside a buffer moved by the last move_to went (the
    // address itself if it was not inside a moved buffer).
    const void *relocate(const void *old) const;

   private:
    char *base_ = nullptr;
    size_t size_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;                         // offset -> length, coalesced
    std::map<size_t, std::pair<size_t, ArenaBuf *>> live_;  // offset -> (length, owner)
    std::vector<std::array<uintptr_t, 3>> moved_;           // old begin, old end, new begin
};

// The arena that buffers allocated now are carved from (bound by each entry
// point for the handle it works on).
inline thread_local Arena *tl_arena = nullptr;

struct ArenaScope {
    Arena *prev;
    explicit ArenaScope(Arena *a) : prev(tl_arena) { tl_arena = a; }
    ~ArenaScope() { tl_arena = prev; }
    ArenaScope(const ArenaScope &) = delete;
    ArenaScope &operator=(const ArenaScope &) = delete;
};

// A device buffer carved from the arena of its handle that only grows.
// Contents are not preserved on growth.
template <class T>
struct DevBuf final : ArenaBuf {
    T *p = nullptr;
    size_t cap = 0;
    Arena *owner = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p && owner) owner->release(p);
        p = nullptr;
        cap = 0;
        owner = nullptr;
    }
    void arena_moved(void *np) override { p = static_cast<T *>(np); }
    nbgs_status reserve(size_t n, double slack = 1.25) {
        if (n <= cap && p) return NBGS_OK;
        Arena *a = owner ? owner : tl_arena;
        if (!a || !a->bound()) {
            set_error("no workspace is bound to the handle");
            return NBGS_ERR_STATE;
        }
        release();
        size_t want = n < 16 ? 16 : (size_t)((double)n * slack) + 16;
        void *q = a->alloc(want * sizeof(T), this);
        if (!q && want > n) {  // without the growth slack
            want = n < 16 ? 16 : n;
            q = a->alloc(want * sizeof(T), this);
        }
        if (!q) {
            set_error("the workspace (%zu bytes, %zu in use) cannot hold another %zu bytes: give the handle a larger "
                      "one (nbgs_workspace_query, then nbgs_scene_set_workspace or its composite/network form)",
                      a->size(), a->used(), want * sizeof(T));
            return NBGS_ERR_CAPACITY;
        }
        p = static_cast<T *>(q);
        cap = want;
        owner = a;
        g_alloc_generation.fetch_add(1, std::memory_order_relaxed);
        return NBGS_OK;
    }
};

// ------------------------------------------------------------ device views

struct BodiesView {  // borrowed caller arrays
    int32_t n;
    double *x, *y, *z, *qw, *qx, *qy, *qz, *vx, *vy, *vz, *wx, *wy, *wz;
    const double *radius, *inv_mass, *inv_inertia;
};

struct PlaneSet {  // walls, passed by value to kernels
    static constexpr int kMax = 16;
    int32_t n;
    double p[kMax][3];
    double nrm[kMax][3];
};

struct Grid {
    double lo[3];
    double hi[3];
    double edge[3];
    int32_t dims[3];
    int32_t periodic[3];
    double L[3];
    int32_t ncells;
    int32_t key_bits;
    uint32_t cell_off;  // first global cell of this grid (several scenes share one cell table)
    // Cell keys run fastest along axis[0], then axis[1], then axis[2]; kdims and
    // kperiodic are dims and periodic in that order (the neighbour search works
    // in key order, so the three cells of a stencil row are neighbours in the
    // table).  The scene picks the order in which its bodies' numbering is
    // most coherent.
    int32_t axis[3];
    int32_t kdims[3];
    int32_t kperiodic[3];
};

// Key order of a grid's axes (axis[0] fastest); fills kdims and kperiodic.
void grid_set_axes(Grid &g, const int32_t axis[3]);

// Several independent scenes held in one body array (batching).  Every array
// is indexed by scene except body_scene (by body).  All null for a single
// scene, whose grid, walls and friction coefficient come as plain arguments.
// Scene s owns bodies body_off[s] .. body_off[s + 1] - 1 and walls with ids
// n + wall_off[s] .. n + wall_off[s + 1] - 1 (n = all bodies); its contacts are
// coloured with the priorities of its own numbering (body i -> i - body_off[s],
// wall -> n_s + w) and its own seed, so it is coloured, ordered and relaxed
// exactly as it would be alone.
struct SceneTable {
    const int32_t *body_scene = nullptr;
    const int32_t *body_off = nullptr;
    const int32_t *wall_off = nullptr;
    const Grid *grids = nullptr;
    const PlaneSet *planes = nullptr;
    const double *mu = nullptr;
    const uint64_t *seed = nullptr;
    int32_t n_scenes = 1;
};

// Canonical (key-ordered) contact list, structure of arrays.
struct ContactsView {
    int32_t *j1, *j2;
    uint64_t *key;
    double *nx, *ny, *nz, *xi, *a1, *a2;
    double *px, *py, *pz;  // initial / solved impulse (world frame)
    int32_t *colour;
    int32_t *matched;  // 1 + the previous step's index of the same pair, 0 for a new pair
};

// ------------------------------------------------------- host helpers (api.hip)

nbgs_status check_params(const nbgs_params *p);
nbgs_status check_domain(const nbgs_domain *domain);  // box, walls (at most PlaneSet::kMax, unit normals)
PlaneSet plane_set(const nbgs_domain *domain);
int bits_for(int64_t n);
// Cell grid of one box whose cells are at least 2 max_reach wide, with at most max(8 n, 2^16) cells.
Grid grid_for_box(const double lo[3], const double hi[3], const int32_t periodic[3], int64_t n, double max_reach);

// ------------------------------------------------------- kernel launchers

// scan.hip / sort.hip
nbgs_status exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, int32_t *total_dev, void *tmp,
                               size_t tmp_bytes, hipStream_t s);
size_t exclusive_scan_tmp_bytes(int64_t n);
nbgs_status radix_sort_pairs(uint32_t *keys, uint32_t *vals, uint32_t *keys_alt, uint32_t *vals_alt, int64_t n,
                             int32_t key_bits, int32_t *hist_tmp, void *scan_tmp, size_t scan_tmp_bytes,
                             bool *result_in_alt, hipStream_t s);
size_t radix_hist_entries(int64_t n);

// detect.hip
// Partners (k > i) of a body kept by the pair count for the emit; longer lists are searched again.
constexpr int kPartnerCap = 16;
// Hull radii, their maxima, the pair list's validity and every body's dynamic bit (dyn_bits, one word per 64
// bodies; *dyn_changed += the words that changed), in one pass over the bodies.
nbgs_status launch_hull(const BodiesView &b, double dt, double tau, double *h, unsigned long long *max_bits,
                        const double *x0, const double *r0, const uint8_t *static0, uint64_t *dyn_bits,
                        int32_t *dyn_changed, hipStream_t s);
nbgs_status launch_fill_f64(double *p, int64_t n, double v, hipStream_t s);
nbgs_status launch_static_flags(const double *inv_mass, int64_t n, uint8_t *flags, hipStream_t s);
// The pair list (see detect.hip): test its pairs with this step's hulls, compact the contacts, geometry.
nbgs_status launch_list_test(const BodiesView &b, const Grid &g, const PlaneSet &pl, const SceneTable &st,
                             double tau, const double *h, const int32_t *lj1, const int32_t *lj2, int64_t nl,
                             int32_t *flag, hipStream_t s);
// Each body's run of contacts as first body in a key-ordered list: its start
// in off and its length in cnt (zero for bodies without one), as the pair
// count and its scan leave them for the colouring.
nbgs_status launch_contact_runs(const int32_t *j1, int64_t nc, int32_t n, int32_t *cnt, int32_t *off, hipStream_t s);
nbgs_status launch_list_emit(const int32_t *lj1, const int32_t *lj2, int64_t nl, const int32_t *flag,
                             const int32_t *off, ContactsView c, hipStream_t s);
nbgs_status launch_pair_geometry(const BodiesView &b, const Grid &g, const PlaneSet &pl, const SceneTable &st,
                                 ContactsView c, int64_t nc, hipStream_t s);
nbgs_status launch_cell_keys(const BodiesView &b, const Grid &g, const SceneTable &st, const double *h,
                             uint32_t *keys, uint32_t *ids, double4 *xr, hipStream_t s);
// Per workgroup b (gridDim.x of them) the sums over its sampled consecutive
// body pairs (i, i + 1) of |x_{i+1} - x_i|, |y..|, |z..|: part[3 b + a].
nbgs_status launch_numbering_steps(const BodiesView &b, int64_t pairs, double *part, int blocks, hipStream_t s);
nbgs_status launch_cells(int32_t n, int64_t ncells, const uint32_t *skeys, const uint32_t *sids, const double4 *xr,
                         int2 *cells, uint32_t *occ, double4 *sxr, hipStream_t s);
nbgs_status launch_pair_count(const BodiesView &b, const Grid &g, const PlaneSet &pl, const SceneTable &st, double tau,
                              const uint32_t *skeys, const uint32_t *sids, const double4 *sxr, const double *h,
                              const int2 *cells, const uint32_t *occ, int32_t *cnt, int32_t *npart,
                              int32_t *partners, int32_t *cellpos, unsigned long long *total, hipStream_t s);
nbgs_status launch_pair_emit(const BodiesView &b, const Grid &g, const PlaneSet &pl, const SceneTable &st, double tau,
                             const uint32_t *skeys, const uint32_t *sids, const double4 *sxr, const double *h,
                             const int2 *cells, const uint32_t *occ, const int32_t *cnt, const int32_t *off,
                             const int32_t *cellpos, const int32_t *npart, const int32_t *partners, ContactsView c,
                             int64_t nc, bool geometry, hipStream_t s);
nbgs_status launch_match_prev(ContactsView c, int64_t nc, const uint64_t *prev_key, const double *prev_px,
                              const double *prev_py, const double *prev_pz, const int32_t *prev_colour,
                              int64_t n_prev, double mu, const SceneTable &st, bool impulses, bool colours,
                              int32_t *unmatched, hipStream_t s);
nbgs_status launch_ids_changed(const int32_t *sdom, const int32_t *prev_sdom, const int32_t *matched, int64_t nc,
                               int32_t *changed, hipStream_t s);
// One bit per body (1/m > 0) in (n + 63) / 64 words; words that differ from the stored ones are rewritten and
// counted into changed.
nbgs_status launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
nbgs_status launch_zero_impulses(ContactsView c, int64_t nc, hipStream_t s);

// colour.hip
nbgs_status launch_j2_degree(const ContactsView &c, int64_t nc, int32_t nb, const double *inv_mass, int32_t *deg2,
                             hipStream_t s);
nbgs_status launch_j2_fill(const ContactsView &c, int64_t nc, int32_t nb, const double *inv_mass, int32_t *cursor,
                           int32_t *inc2, hipStream_t s);
nbgs_status launch_prio(const ContactsView &c, int64_t nc, uint64_t seed, const SceneTable &st, int32_t nb,
                        uint64_t *prio, hipStream_t s);
nbgs_status launch_jp_round(const ContactsView &c, const uint64_t *prio, int64_t nc, int32_t nb,
                            const double *inv_mass, const int32_t *off1, const int32_t *cnt1, const int32_t *off2,
                            const int32_t *inc2, const int32_t *sdom, int32_t *remaining, int32_t *overflow,
                            hipStream_t s);
nbgs_status launch_fill_u8(uint8_t *p, int64_t n, uint8_t v, hipStream_t s);
// One pass of the greedy rule; each contact it evaluates clears its dirty_in flag (so the two flag arrays stay
// clear between the passes that write them); clear_out: clear dirty_out first (it was not left clear).
nbgs_status launch_colour_fix(const ContactsView &c, const uint64_t *prio, int64_t nc, int32_t nb,
                              const double *inv_mass, const int32_t *off1, const int32_t *cnt1, const int32_t *off2,
                              const int32_t *inc2, const int32_t *sdom, uint8_t *dirty_in, uint8_t *dirty_out,
                              int32_t *changed, int32_t *overflow, bool clear_out, hipStream_t s);
// Per-pass change counters of a colour-fix loop (zeroed once per colouring; a pass far beyond them re-zeroes its
// slot), and the host check after a batch of passes: the last pass's count and the overflow flag into pinned[1..2].
constexpr int kFixCounters = 64;
nbgs_status launch_colour_hist(const ContactsView &c, int64_t nc, int32_t nb, const double *inv_mass, int32_t *hist,
                               hipStream_t s);
nbgs_status launch_colour_keys(const ContactsView &c, const int32_t *sdom, int64_t nc, uint32_t *keys, uint32_t *ids,
                               hipStream_t s);
nbgs_status launch_invert(const uint32_t *perm, int64_t nc, int32_t *pos, hipStream_t s);
template <class T>
nbgs_status launch_gather_sweep(const ContactsView &c, const uint32_t *perm, const int32_t *sdom, int64_t nc,
                                double dt, double erp, const SceneTable &st, SweepView<T> sv, bool indices,
                                hipStream_t s);

// sweep.hip
// rec (null: body order): body i's solver record is record rec[i] of vel (the block-local sweeps' order); the
// integration and the export take the same map.
template <class T>
nbgs_status launch_init_bodies(const BodiesView &b, const double g[3], double dt, T *vel, const int32_t *rec,
                               hipStream_t s);
template <class T>
nbgs_status launch_warm_scatter(SweepView<T> sv, int64_t begin, int64_t end, int32_t nb, T *vel, hipStream_t s);
// Contacts per tile (one partial residual sum each).
template <class T>
int64_t sweep_tile(const SweepTune &t);
bool sweep_tune_supported(const SweepTune &t);
template <class T>
nbgs_status launch_sweep_colour(SweepView<T> sv, int64_t begin, int64_t end, int32_t nb, T *vel, SweepParams sp,
                                const SweepTune &t, double *partials, const int32_t *ctrl, hipStream_t s);
// The same sweep for colour c whose range col[c] .. col[c + 1] is read on the
// device, over a fixed number of workgroups (sweep_graph_grid); workgroup b
// writes its partial sums to partials[2 b], [2 b + 1].
template <class T>
unsigned sweep_graph_grid(const SweepTune &t);
template <class T>
nbgs_status launch_sweep_colour_dev(SweepView<T> sv, const int64_t *col, int32_t c, int32_t nb, T *vel, SweepParams sp,
                                    const SweepTune &t, double *partials, const int32_t *ctrl, hipStream_t s);
nbgs_status launch_residual(const double *partials, int32_t n_partials, double target, int32_t *ctrl,
                            double *hist, hipStream_t s, int32_t at = -1);
template <class T>
nbgs_status launch_integrate(const BodiesView &b, const Grid &g, const SceneTable &st, double dt, const T *vel,
                             const uint8_t *touched, const double grav[3], const int32_t *rec, hipStream_t s);
// Few contacts: touched[i] = 1 for every body a contact of the step touches (launch_mark_touched), the solver's
// records written for those bodies only (launch_init_touched); the integration and the export take every other
// body's record from its state (touched passed to them; NULL: every record is read).
nbgs_status launch_mark_touched(const int32_t *j1, const int32_t *j2, int64_t nc, int32_t nb, uint8_t *touched,
                                hipStream_t s);
template <class T>
nbgs_status launch_init_touched(const BodiesView &b, const double g[3], double dt, const uint8_t *touched, T *vel,
                                hipStream_t s);
template <class T>
nbgs_status launch_save_impulses(SweepView<T> sv, int64_t nc, ContactsView c, hipStream_t s);
template <class T>
nbgs_status launch_export_accumulators(const T *vel, int32_t nb, double *v, double *w, const BodiesView &b,
                                       const uint8_t *touched, bool pending, const double g[3], double dt,
                                       const int32_t *rec, hipStream_t s);

// warmstart.hip
struct FeatureScales {
    double vs, ms, rs;  // velocity, mass, length
};
nbgs_status launch_features(const BodiesView &b, const ContactsView &c, int64_t nc, const double g[3], double dt,
                            double mu, double erp, const FeatureScales &fs, float *feat, double *frame,
                            hipStream_t s);
nbgs_status launch_decode(const float *y, const double *frame, const ContactsView &c, int64_t nc,
                          const FeatureScales &fs, double mu, double *px, double *py, double *pz, hipStream_t s);
nbgs_status launch_targets(const double *frame, const ContactsView &c, int64_t nc, const FeatureScales &fs, float *t,
                           hipStream_t s);
template <class T>
nbgs_status launch_set_sweep_impulses(SweepView<T> sv, int64_t nc, const double *px, const double *py,
                                      const double *pz, hipStream_t s);
template <class T>
nbgs_status launch_jacobi_residual(SweepView<T> sv, int64_t nc, int32_t nb, const T *vel, double mu,
                                   double *partials, double *out, hipStream_t s);

// mlp.hip
int mlp_param_count();
int mlp_frag_count();
int mlp_grad_blocks(int64_t bsz);
nbgs_status launch_mlp_pack(const float *w, unsigned short *fr, hipStream_t s);
nbgs_status launch_mlp_forward(const unsigned short *fr, const float *w, const float *x, int64_t n, float *y,
                               hipStream_t s);
nbgs_status launch_mlp_grad(const unsigned short *fr, const float *w, const float *x, const float *t,
                            const int32_t *idx, int64_t off, int64_t bsz, float *part, float *lpart, float *grad,
                            hipStream_t s);
nbgs_status launch_mlp_adam(float *w, const float *g, float *m, float *v, int64_t step, float lr, hipStream_t s);
const unsigned short *mlp_frag_ptr(nbgs_mlp_t mlp);
const float *mlp_weight_ptr(nbgs_mlp_t mlp);
// The network's store of collected training pairs: room for n more (CAPACITY past its size), then taken.
nbgs_status mlp_store_slot(nbgs_mlp_t mlp, int64_t n, float **feat, float **tgt);
void mlp_store_commit(nbgs_mlp_t mlp, int64_t n);

constexpr int kSweepBlock = 256;

}  // namespace nbgs
