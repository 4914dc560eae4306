// The scene object behind the C ABI: borrowed body arrays, per-step device
// buffers, the contact tables of this and the previous step, and the host-side
// state of one time step (shared by the scene, batch and tuning entry points).
#pragma once

#include <string>
#include <vector>

#include "nbgs_internal.h"

namespace nbgs {

struct ContactBuf {
    DevBuf<int32_t> j1, j2, colour, matched;
    DevBuf<uint64_t> key;
    DevBuf<double> nx, ny, nz, xi, a1, a2, px, py, pz;
    nbgs_status reserve(size_t n) {
        NBGS_TRY(j1.reserve(n));
        NBGS_TRY(j2.reserve(n));
        NBGS_TRY(colour.reserve(n));
        NBGS_TRY(matched.reserve(n));
        NBGS_TRY(key.reserve(n));
        for (DevBuf<double> *b : {&nx, &ny, &nz, &xi, &a1, &a2, &px, &py, &pz}) NBGS_TRY(b->reserve(n));
        return NBGS_OK;
    }
    ContactsView view() {
        ContactsView v;
        v.j1 = j1.p;
        v.j2 = j2.p;
        v.key = key.p;
        v.nx = nx.p;
        v.ny = ny.p;
        v.nz = nz.p;
        v.xi = xi.p;
        v.a1 = a1.p;
        v.a2 = a2.p;
        v.px = px.p;
        v.py = py.p;
        v.pz = pz.p;
        v.colour = colour.p;
        v.matched = matched.p;
        return v;
    }
};

template <class T>
struct SweepBuf {
    DevBuf<int32_t> j1, j2, perm, col, sdom;
    DevBuf<int16_t> ls;  // slot of each contact end inside its block or subdomain (block-local and subdomain modes)
    DevBuf<T> nx, ny, nz, bias, a1, a2, px, py, pz, mu;
    bool per_contact_mu = false;
    bool sub = false;  // subdomain solver: colour and subdomain per position, local slots per contact end
    nbgs_status reserve(size_t n) {
        NBGS_TRY(j1.reserve(n));
        NBGS_TRY(j2.reserve(n));
        NBGS_TRY(perm.reserve(n));
        for (DevBuf<T> *b : {&nx, &ny, &nz, &bias, &a1, &a2, &px, &py, &pz}) NBGS_TRY(b->reserve(n));
        if (per_contact_mu) NBGS_TRY(mu.reserve(n));
        if (sub) {
            NBGS_TRY(col.reserve(n));
            NBGS_TRY(sdom.reserve(n));
            NBGS_TRY(ls.reserve(2 * n));
        }
        return NBGS_OK;
    }
    SweepView<T> view() {
        SweepView<T> v;
        v.j1 = j1.p;
        v.j2 = j2.p;
        v.perm = perm.p;
        v.nx = nx.p;
        v.ny = ny.p;
        v.nz = nz.p;
        v.bias = bias.p;
        v.a1 = a1.p;
        v.a2 = a2.p;
        v.px = px.p;
        v.py = py.p;
        v.pz = pz.p;
        v.mu = per_contact_mu ? mu.p : nullptr;
        v.col = sub ? col.p : nullptr;
        v.sdom = sub ? sdom.p : nullptr;
        return v;
    }
};

enum Phase { kDetect = 0, kColour = 1, kInit = 2, kSweeps = 3, kIntegrate = 4, kNumPhases = 5 };

}  // namespace nbgs

using namespace nbgs;

struct nbgs_scene_s {
    // device memory of the scene (the caller's workspace); first, so that it outlives every buffer carved from it
    Arena arena;
    BodiesView b{};
    PlaneSet planes{};
    double lo[3], hi[3];
    int32_t periodic[3];
    nbgs_params p{};
    hipStream_t s = nullptr;
    Grid grid{};

    // per body
    DevBuf<double> h;
    DevBuf<uint32_t> keys, ids, keys2, ids2;
    DevBuf<double4> sxr;  // packed records (centre, +-(r + h)) in sorted order
    DevBuf<double4> xr;   // the same in body order
    int32_t key_axes[3] = {0, 1, 2};  // cell key order (axis[0] fastest), chosen on the first detection
    bool key_axes_set = false;
    const uint32_t *skeys = nullptr, *sids = nullptr;  // the last grid phase's sorted keys and bodies
    // pair list (detect_impl): its pairs, their flags and scan offsets, and the build's positions (3 n), radii,
    // hull (the skin) and static flags
    bool vl_enabled = true, vl_valid = false;
    bool vl_blocked = false;  // a buffer did not fit beside the list in this workspace: no list until it changes
    double vl_skin = 0.0;
    int64_t vl_n = 0, vl_builds = 0;
    DevBuf<int32_t> vl_j1, vl_j2, vl_flag, vl_off;
    DevBuf<double> vl_h, vl_x0, vl_r0;
    DevBuf<uint8_t> vl_static0;
    DevBuf<int32_t> cnt, off, cellpos;
    DevBuf<int32_t> npart, partners;  // the pair count's partner store (kPartnerCap per body) for the emit
    DevBuf<int32_t> deg2, off2, cursor;
    DevBuf<double> vel64;
    DevBuf<float> vel32;
    // cells
    DevBuf<int2> cells;     // per occupied cell (start, end) of its sorted range
    DevBuf<uint32_t> occ;   // occupancy bitmap of the cells, rebuilt every step
    // scratch
    DevBuf<int32_t> radix_hist;
    DevBuf<char> scan_tmp;
    DevBuf<int32_t> fixcnt;  // per-pass change counters of the colour-fix loop
    DevBuf<int32_t> small;  // [0] total, [1] remaining, [2] overflow, [4] new pairs, [5] changed ids, [6] changed
                            // blocks, [7] changed dynamic bits, [8..12) ctrl, [12..14) last residual, [16..528)
                            // colour histograms
    DevBuf<unsigned long long> maxbits;
    int32_t *pinned = nullptr;  // host mirror of small
    // contacts
    ContactBuf cb[2];
    int cur = 0;
    bool table_in_cur = false;
    int64_t nc = 0, n_prev = 0;
    int64_t nc_needed = -1;  // the contact count the last detection found (reported with CAPACITY)
    DevBuf<int32_t> inc2;
    DevBuf<uint8_t> dirty[2];  // colouring passes: the contacts a change reached (ping-pong)
    DevBuf<uint64_t> prio;
    bool prev_colours = false;  // the previous table holds the colours of its contact set
    int32_t colour_passes = 0;  // > 0: passes from the previous colours, < 0: Jones-Plassmann rounds
    DevBuf<uint32_t> ckeys, cids, ckeys2, cids2;
    const uint32_t *perm = nullptr;  // sweep position -> canonical index (in ckeys/cids storage)
    // the last step's colouring inputs: ids of its pairs (canonical order), mode and seed; reused whole when equal
    DevBuf<int32_t> prev_sdom;
    double prev_sig[4] = {0.0, 0.0, 0.0, 0.0};
    uint64_t prev_seed = 0;
    bool prev_sig_valid = false;
    // every body's dynamic bit (1/m > 0) as the last detection saw it; the colouring and the block slots depend
    // on it, so a change forbids their reuse
    DevBuf<uint64_t> dyn_bits;
    bool dyn_bits_valid = false;
    bool colouring_reused = false;
    int32_t prev_precision = -1;
    // every body's block in the block-local order, this step's and the last one's (alternating)
    DevBuf<uint32_t> bblk[2];
    int bblk_cur = 0;
    bool bblk_valid = false, bblk_compared = false, blk_prep_reused = false;
    int64_t bblk_nblocks = 0;
    SweepBuf<double> sw64;
    SweepBuf<float> sw32;
    int32_t n_colours = 0;
    std::vector<int64_t> col_off;
    std::vector<int64_t> part_off;
    SweepTune tune[2];  // per precision (NBGS_FP64, NBGS_FP32_SWEEP)
    int64_t n_partials = 0;
    DevBuf<double> partials;
    DevBuf<double> res_hist;
    int32_t precision_used = NBGS_FP64;
    int state = 0;  // 0 idle, 1 detected, 2 solved
    nbgs_stats stats{};
    hipEvent_t ev[kNumPhases + 1] = {};
    bool ev_ok[kNumPhases + 1] = {};
    std::vector<int64_t> col_dyn;  // dynamic bodies touched per colour
    // learned warm start
    nbgs_mlp_t mlp = nullptr;
    bool capture = false;
    FeatureScales fs{1.0, 1.0, 1.0};
    double mean_mass = 1.0, mean_radius = 1.0;
    DevBuf<float> feat, yout;
    DevBuf<double> frame, lpx, lpy, lpz, jpart, jres;
    bool have_features = false, have_learned = false;
    bool solved = false;  // a solve ran since the last detect
    nbgs_warm_info winfo{-1, 0.0, 0.0};
    // sweep-kernel profiling (event pair around every sweep launch)
    bool profiling = false;
    std::vector<hipEvent_t> pev;
    nbgs_profile prof{};

    // batched scenes (n_scenes > 1): per-scene boxes, walls, friction, seeds
    int32_t n_scenes = 1;
    std::vector<int32_t> body_off_h, wall_off_h;
    std::vector<PlaneSet> planes_h;
    std::vector<double> lo_h, hi_h, mu_h;  // 3 per scene for lo, hi
    std::vector<int32_t> periodic_h;        // 3 per scene
    std::vector<uint64_t> seed_h;
    DevBuf<int32_t> body_scene_d, body_off_d, wall_off_d;
    DevBuf<Grid> grids_d;
    DevBuf<PlaneSet> planes_d;
    DevBuf<double> mu_d;
    DevBuf<uint64_t> seed_d;
    Grid *grids_pinned = nullptr;
    std::vector<int64_t> scene_contacts;  // per scene, last detect (filled on request)
    // sweeps replayed from a captured graph
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec = nullptr;
    struct GraphKey {
        int32_t sweeps = -1, colours = -1, prec = -1;
        unsigned grid = 0;
        SweepTune tune{};
        const void *ptrs[6] = {};
        const void *col = nullptr;
        double target = 0.0, mu = 0.0, relax = 0.0;
        bool every = true;  // residual after every sweep
        uint64_t alloc_gen = 0;  // no device buffer (re)allocated since the capture
        bool operator==(const GraphKey &o) const {
            if (sweeps != o.sweeps || colours != o.colours || prec != o.prec || grid != o.grid || col != o.col ||
                target != o.target || mu != o.mu || relax != o.relax || every != o.every || alloc_gen != o.alloc_gen)
                return false;
            if (std::memcmp(&tune, &o.tune, sizeof(tune)) != 0) return false;
            for (int i = 0; i < 6; ++i)
                if (ptrs[i] != o.ptrs[i]) return false;
            return true;
        }
    } gkey;
    int graph_pairs = 0;  // profiling event pairs of the last graph-replayed solve
    bool res_history = true;   // residual of every sweep even without a target
    bool hist_partial = false;  // the last solve summed only its last sweep
    DevBuf<int64_t> col_d;
    int64_t *col_pinned = nullptr;
    size_t col_pinned_cap = 0;
    // subdomain solver (Alg. 1 with block subdomains), off when sub_edge == 0
    double sub_edge = 0.0;
    bool sub_active = false;  // the current step uses it (edge > 0 and contacts)
    int32_t n_sub = 0;
    int64_t n_slots = 0;
    int32_t max_slots = 0;
    // block-local order: the launches of the block pass (first id, ids, the largest block's slots)
    std::vector<int32_t> launch_id0, launch_n, launch_slots;
    DevBuf<int32_t> sdom, tile_cnt, tile_off32, tile_scnt, tile_slot_off, eflags, eex, slot_body, slot_sdom, body_cnt,
        body_slot_off;
    DevBuf<int64_t> tile_off;
    DevBuf<int32_t> blk_cs;    // block-local order: per block its colour runs (k_blk_colour_runs)
    DevBuf<int32_t> blk_nrun;  // and their count
    DevBuf<uint32_t> ekeys, evals, ekeys2, evals2, bkeys, bvals, bkeys2, bvals2;
    const uint32_t *body_slots = nullptr;
    DevBuf<double> corr64;
    DevBuf<float> corr32;
    // block-local sweep order of the plain NBGS, off when blk_edge == 0: the
    // ids of the contacts are their blocks (local) or n_blk (between blocks);
    // the tables above then describe the local part, the cross part is swept
    // colour by colour over xcol[c] .. xcol[c + 1] of the sweep record
    double blk_edge = 0.0;
    bool blk_active = false;
    int32_t n_blk = 0;
    int32_t blk_grids = 1;     // block grids shifted by 1/blk_grids of an edge (nbgs_set_block_grids)
    int32_t blk_grid_ids = 0;  // ids (blocks) per grid: n_blk = blk_grids * blk_grid_ids
    // groups of the clusters of contacts no grid holds (ids n_blk .. n_blk + blk_groups - 1, swept by the block
    // pass; 0: those contacts keep the id n_blk and are swept by colour)
    int32_t blk_groups = 0;
    bool blk_group_cross = true;
    // few contacts (fewer than one per eight bodies, at least 2^16 bodies): the solver's records are kept for the
    // touched bodies only
    bool sparse_bodies = false;
    DevBuf<uint8_t> touched;
    bool xg_prev_valid = false;  // the last detection formed its groups in this order (n_blk blocks)
    int32_t xg_prev_nblk = 0;
    DevBuf<int32_t> xg_ctl, xg_cnt;
    int64_t blk_first_cross = 0;  // first sweep position of the contacts between blocks
    std::vector<int64_t> xcol;       // positions of the cross colours' ranges (size colours + 1)
    std::vector<int64_t> xdyn;       // dynamic contact ends per cross colour
    std::vector<int64_t> xpart_off;  // first partial of every cross colour, after the n_blk block partials
    int64_t blk_dyn_local = 0;       // slots of the local part (each read and written once per sweep)
    int64_t blk_n_local = 0;         // contacts of the local part
    // the solver records in the first grid's slot order (record s: slot s of the first grid's blocks, then every
    // other body in index order), so that a block of the first grid reads and writes one contiguous range: rec_of
    // (body -> record), body_of (record -> body), the slot table and the sweep record's ends as records; rebuilt
    // with the block set-up or the sweep record's ends (rec_valid); rec_on from a solve's initialisation of the
    // records to the next one (its sweeps, integration and export use the order)
    int64_t slot_s0 = 0;  // slots of the first grid's blocks
    DevBuf<int32_t> rec_of, body_of, rec_tmp, slot_rec, j1r, j2r;
    bool rec_valid = false, rec_on = false;
    DevBuf<int64_t> xcol_d;
    DevBuf<int32_t> xncol_d;
    // sweep-tuning cache file (empty: none)
    std::string tune_cache;
    bool tuned[2] = {false, false};

    nbgs::SceneTable table() const {
        nbgs::SceneTable t;
        if (n_scenes <= 1) return t;
        t.body_scene = body_scene_d.p;
        t.body_off = body_off_d.p;
        t.wall_off = wall_off_d.p;
        t.grids = grids_d.p;
        t.planes = planes_d.p;
        t.mu = mu_d.p;
        t.seed = seed_d.p;
        t.n_scenes = n_scenes;
        return t;
    }
    int32_t *total() { return small.p + 0; }
    int32_t *remaining() { return small.p + 1; }
    int32_t *overflow() { return small.p + 2; }
    int32_t *ctrl() { return small.p + 8; }
    int32_t *chist() { return small.p + 16; }
};


namespace nbgs {

constexpr int kSmallInts = 16 + 512;

// Scene set-up shared by nbgs_scene_create (one scene) and nbgs_batch_create
// (n_scenes scenes in one body array; body_off: n_scenes + 1 host offsets).
// Device bytes a scene (or a batch of `scenes` scenes) of n bodies with up to c contacts needs.
size_t scene_workspace_bytes(int64_t n, int64_t c, int64_t scenes);
// scene_workspace_bytes plus the per-id tables of the scene's current sweep order.
nbgs_status scene_need_bytes(nbgs_scene_t sc, int64_t c, size_t *bytes);
nbgs_status scene_create(void *workspace, size_t workspace_bytes, const nbgs_bodies *bodies, int32_t n_scenes,
                         const int64_t *body_off,
                         const nbgs_domain *domains, const nbgs_params *params, void *hip_stream, nbgs_scene_t *out);
// Sweep tuning: the cached choice for this scene's size, else a search over
// launch shapes on the scene's current contacts whose trial sweeps leave no
// trace (the initial impulses are restored afterwards).
nbgs_status scene_autotune(nbgs_scene_t sc, int32_t sweeps, nbgs_tuning *chosen, double *best_ms);
// The sweep record from the canonical contacts; indices = false rewrites only geometry and impulses.
nbgs_status scene_gather(nbgs_scene_t sc, bool indices = true);
nbgs_status scene_sync_small(nbgs_scene_t sc, int first, int count);
// Subdomain solver: subdomain of every contact (before colouring), then the
// tile and slot tables (after the sweep record is gathered), and one pass
// (mode 0: initial impulses, 1: relaxation) with the correction reduction.
nbgs_status subdomain_assign(nbgs_scene_t sc);
nbgs_status order_ids(nbgs_scene_t sc, int64_t *ids);
nbgs_status subdomain_prepare(nbgs_scene_t sc);
template <class T>
nbgs_status subdomain_pass(nbgs_scene_t sc, int mode, T *vel, T *corr);
// Block-local order: ids of the contacts (before colouring), then the local
// tables and the cross colours' ranges (after the gather), and the pass over
// the local part (mode 0: initial impulses, 1: relaxation), each block's
// velocities updated in place in LDS.
// Contact ids of the block-local order; every body's block, the number that changed since the last step added to
// changed.
nbgs_status block_assign(nbgs_scene_t sc, int32_t *changed, bool maybe_reuse);
nbgs_status block_prepare(nbgs_scene_t sc);
template <class T>
nbgs_status block_pass(nbgs_scene_t sc, int mode, T *vel);
// The block-local sweeps' record order: builds its tables when the order changed and, with room in the workspace,
// sets rec_on (off: the records stay in body order, with the same results).
nbgs_status block_records(nbgs_scene_t sc);
template <class T>
nbgs_status scene_sweep_loop(nbgs_scene_t sc, int32_t max_sweeps, double target, const SweepTune &tune);

}  // namespace nbgs
