/*
 * nbgs.h -- C ABI of the MI355X (gfx950) hard-contact granular solver.
 *
 * One time step of the method of Preclik & Ruede, "Ultrascale Simulations of
 * Non-smooth Granular Dynamics" (single-process form of Alg. 2, Sect. 6.6):
 *   nbgs_detect     contact detection with intersection hulls (Sect. 4,
 *                   eq. (expansionradius), eq. (contactpos) for spheres and
 *                   wall planes), colouring of the contacts, initial impulses
 *                   (zero or previous step, Sect. 5);
 *   nbgs_solve      nonlinear block Gauss-Seidel sweeps (Alg. 1 with one
 *                   subdomain, run colour by colour; per contact the 3x3
 *                   Coulomb one-contact problem of eqs. (nonpenetration) and
 *                   (coulomb) is solved and projected onto the friction cone);
 *   nbgs_integrate  semi-implicit Euler of eq. (integrationscheme) with
 *                   quaternion renormalisation (Sect. 3);
 *   nbgs_step       the three in sequence.
 *
 * Conventions (shared by every entry point)
 *   - Pointers marked [device] are HIP device pointers, [host] are host
 *     pointers.  Body arrays are owned by the caller (e.g. torch tensors) and
 *     borrowed by the scene for its lifetime; nbgs_integrate / nbgs_step write
 *     positions, orientations and velocities in place.
 *   - Device memory: the library allocates none.  Every handle (scene, batch,
 *     composite scene, network) is given a workspace [device] by its caller
 *     (e.g. a torch byte tensor), sized by the matching *_workspace_query, and
 *     carves all its buffers from it; the workspace stays owned by the caller
 *     and must outlive the handle.  A detection whose contacts exceed the
 *     workspace's contact capacity returns CAPACITY with the contact count in
 *     nbgs_stats.n_contacts and leaves the scene as it was: query the size for
 *     that count, allocate, nbgs_scene_set_workspace, detect again.  (Every
 *     other CAPACITY, a limit that no workspace lifts, reports -1 there.)
 *   - All device work is enqueued on the stream passed to nbgs_scene_create
 *     (NULL = the legacy default stream).  Entry points that return counts in a
 *     host nbgs_stats synchronise that stream before returning.
 *   - Every entry point returns an nbgs_status and never throws; the detail of
 *     the last non-OK status of the calling thread is in nbgs_last_error().
 *   - Units: the solver works with contact impulses P = dt * lambda, where
 *     lambda is the contact force of eq. (integrationscheme).
 *   - Contact j joins bodies j1 < j2; wall plane w acts as body n_bodies + w and
 *     is always j2.  The normal points from j2 towards j1 (outward from j2),
 *     the contact point lies on the surface of j2 (eq. (contactpos)), and the
 *     impulse acts +P on j1 and -P on j2 (eq. (wrench)).  The pair key is
 *     (j1 << 32) | j2; the canonical contact order is ascending key.
 */
#ifndef NBGS_H
#define NBGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NBGS_ABI_VERSION 2

typedef enum {
    NBGS_OK = 0,
    NBGS_ERR_INVALID_ARG = 1,   /* bad pointer, size or parameter value */
    NBGS_ERR_OUT_OF_MEMORY = 2, /* a device allocation failed */
    NBGS_ERR_CAPACITY = 3,      /* a fixed limit was exceeded (colours > 255, counts >= 2^31, buffer too small) */
    NBGS_ERR_DEVICE = 4,        /* a HIP call failed */
    NBGS_ERR_NOT_CONVERGED = 5, /* residual target not reached within max_sweeps (impulses are still valid) */
    NBGS_ERR_STATE = 6,         /* wrong call order, e.g. solve before detect */
    NBGS_ERR_NUMERIC = 7,       /* NaN or Inf met in the residual */
    NBGS_ERR_UNSUPPORTED = 8
} nbgs_status;

typedef struct nbgs_scene_s *nbgs_scene_t;

/* Arithmetic of the sweeps.  Detection, the residual and integration are FP64
 * in both modes; NBGS_FP32_SWEEP keeps the velocity accumulators, the impulses
 * and the per-contact sweep record in FP32. */
typedef enum { NBGS_FP64 = 0, NBGS_FP32_SWEEP = 1 } nbgs_precision;

/* Initial impulses of a solve (Sect. 5: zero, or the previous step's; any
 * other guess is admissible).  NBGS_WS_LEARNED predicts them with an attached
 * network (nbgs_scene_attach_mlp) and keeps the prediction only if its Jacobi
 * residual (every contact's one-contact solution against the accumulators
 * with the initial impulses applied, |P* - P0|_2 / |P*|_2) is not larger than
 * that of the previous-step impulses; without a network it is
 * NBGS_WS_PREVIOUS. */
typedef enum { NBGS_WS_ZERO = 0, NBGS_WS_PREVIOUS = 1, NBGS_WS_LEARNED = 2 } nbgs_warm_start;

/* Body state, structure of arrays of length n, FP64, [device].  Spheres only:
 * radius is the bounding radius r_i of eq. (expansionradius).  inv_mass = 0
 * marks a static body, which must then also have inv_inertia = 0;
 * inv_inertia = 0 with inv_mass > 0 is a rotation-locked body.  The inertia is
 * isotropic (inv_inertia is 1/I of a body whose principal moments are equal,
 * Sect. 2), so the gyroscopic term w x I w vanishes. */
typedef struct {
    int64_t n;
    double *x, *y, *z;
    double *qw, *qx, *qy, *qz;
    double *vx, *vy, *vz;
    double *wx, *wy, *wz;
    const double *radius, *inv_mass, *inv_inertia;
} nbgs_bodies;

/* A wall: a global body of infinite inertia and zero velocity (Sect. 6.4). */
typedef struct {
    double point[3];
    double normal[3]; /* unit length, pointing into the domain */
} nbgs_plane;

/* Domain box [lo, hi).  Periodic axes use minimum-image separations and wrap
 * positions after integration; they need hi - lo >= 3 cell edges (a cell edge
 * is at least twice the largest r + h).  planes: [host], copied at create. */
typedef struct {
    double lo[3], hi[3];
    int32_t periodic[3];
    int32_t n_planes;
    const nbgs_plane *planes;
} nbgs_domain;

typedef struct {
    double dt;          /* time step, > 0 */
    double gravity[3];  /* external acceleration of every dynamic body */
    double mu;          /* coefficient of friction, eq. (coulomb), >= 0 */
    double tau;         /* hull safety margin of eq. (expansionradius), >= 0 */
    double relax;       /* relaxation parameter omega of Alg. 1, in (0, 1] */
    double erp;         /* scale of the xi/dt penetration correction when xi < 0 (Sect. 3), in [0, 1] */
    int32_t precision;  /* nbgs_precision */
    int32_t warm_start; /* nbgs_warm_start */
    uint64_t colour_seed; /* seed of the contact priorities of the colouring */
} nbgs_params;

typedef struct {
    int64_t n_contacts;
    int32_t n_colours;
    int32_t sweeps;   /* sweeps done by the last solve */
    double residual;  /* R of the last sweep: |dP|_2 / |P|_2 over all contacts of that sweep */
} nbgs_stats;

/* ABI version of the loaded library (NBGS_ABI_VERSION). */
int32_t nbgs_abi_version(void);

/* Message of the calling thread's last non-OK status ("" if none).  The
 * pointer stays valid until the next failing call on the same thread. */
const char *nbgs_last_error(void);

/* Bytes of device workspace a scene of n_bodies bodies with up to
 * contact_capacity contacts needs, in the classic order in every precision
 * and warm start (an upper bound: per body 567 B, per contact 1,000 B, plus a
 * cell table of 2^16 cells, 16 MiB, and ten per cent), a multiple of 256 (all
 * of it usable from a 256-byte aligned base).  The block-local order and the
 * subdomain solver add 88 B per id, the block-local order also the tables
 * of its record order, 12 B per body and 16 B per contact, plus ten per cent
 * (nbgs_scene_workspace_query).  params
 * [host] may be NULL (checked when given).  *bytes [host].  Pure host
 * computation: no device is touched.  Errors: INVALID_ARG. */
nbgs_status nbgs_workspace_query(int64_t n_bodies, int64_t contact_capacity, const nbgs_params *params,
                                 size_t *bytes);

/* Create a scene that borrows the body arrays.  bodies, domain, params:
 * [host] structs (the body pointers inside are [device]).  workspace
 * [device], workspace_bytes: the caller's region the scene carves all its
 * device buffers from (nbgs_workspace_query; at least 256-byte aligned use is
 * made of it), borrowed until nbgs_scene_destroy or the next
 * nbgs_scene_set_workspace.  hip_stream: a hipStream_t or NULL.  Errors:
 * INVALID_ARG (n < 1, n >= 2^31 - 64, null pointer or workspace, dt <= 0,
 * relax not in (0,1], a static body with inv_inertia != 0, a non-unit plane
 * normal), CAPACITY (the workspace cannot hold the per-body buffers),
 * OUT_OF_MEMORY (host), DEVICE.  *out receives the handle, which the caller
 * releases with nbgs_scene_destroy. */
nbgs_status nbgs_scene_create(const nbgs_bodies *bodies, const nbgs_domain *domain, const nbgs_params *params,
                              void *workspace, size_t workspace_bytes, void *hip_stream, nbgs_scene_t *out);

/* Move the scene into another workspace [device] of `bytes` (typically a
 * larger one after nbgs_detect returned CAPACITY): every buffer in use is
 * copied, packed, into the new region on the scene's stream, which is then
 * synchronised, so the old workspace may be released once this returns.  The
 * regions must not overlap.  Errors: INVALID_ARG (NULL, too small, overlap),
 * CAPACITY (the buffers in use do not fit; nothing moved), DEVICE. */
nbgs_status nbgs_scene_set_workspace(nbgs_scene_t scene, void *workspace, size_t bytes);

/* Bytes of workspace this scene needs for contact_capacity contacts in its
 * current sweep order: nbgs_workspace_query's figure plus, for the
 * block-local order (nbgs_set_block_order) or the subdomain solver
 * (nbgs_set_subdomains), 88 B per id (every block of every grid and the id of
 * the contacts between blocks, or every subdomain), rounded up to 256.  This
 * is the size a detection checks its workspace against.  *bytes [host].  Host
 * arithmetic only.  Errors: INVALID_ARG (NULL, negative capacity, an edge
 * giving too many blocks). */
nbgs_status nbgs_scene_workspace_query(nbgs_scene_t scene, int64_t contact_capacity, size_t *bytes);

/* Size of the scene's workspace, the bytes its buffers use now and the most
 * they used at once, each [host] and NULL-able. */
nbgs_status nbgs_scene_workspace_usage(nbgs_scene_t scene, size_t *size, size_t *used, size_t *peak);

/* Release the scene (synchronises its stream).  The body arrays and the
 * workspace are not touched.  NULL is accepted. */
nbgs_status nbgs_scene_destroy(nbgs_scene_t scene);

/* Replace the parameters (e.g. switch precision or warm start between steps).
 * Same checks as nbgs_scene_create. */
nbgs_status nbgs_scene_set_params(nbgs_scene_t scene, const nbgs_params *params);

/* Contact detection for the current body state (Sect. 4): hull radii
 * h_i = dt(|v_i| + |w_i| r_i) + tau, every pair whose hulls intersect
 * (|x_i - x_k| <= (r_i + h_i) + (r_k + h_k)) and every sphere/wall pair with
 * gap <= h_i + tau becomes a contact; pairs of two static bodies are skipped.
 * Then the contacts are coloured (greedy first-fit in descending
 * splitmix64(key ^ colour_seed) priority, conflicts = shared body with
 * inv_mass > 0) and ordered by (colour, key) for the sweeps, and the initial
 * impulses are set (params.warm_start).  stats: [host] or NULL (then only
 * n_contacts of the scene is known after the next synchronising call).
 * Errors: CAPACITY (more contacts than the workspace holds, found before
 * any list is written: stats->n_contacts = the contact count, the scene
 * unchanged, see nbgs_scene_set_workspace; for every other CAPACITY, which
 * no workspace can lift, stats->n_contacts = -1: more than 255 colours; more than
 * 2^31 - 256 contacts, counted in 64 bits before any list is sized; a body
 * meeting more than 2^18 hull candidates in its 27 cells, which happens when
 * one hull, e.g. of a diverged state, makes the cell grid too coarse; in
 * subdomain mode more than 2^30 contacts; block or subdomain tables larger
 * than the workspace allows), OUT_OF_MEMORY, DEVICE. */
nbgs_status nbgs_detect(nbgs_scene_t scene, nbgs_stats *stats);

/* NBGS sweeps over the detected contacts (Alg. 1, one subdomain, colour
 * order).  max_sweeps >= 1.  residual_target > 0: stop after the first sweep
 * whose R <= residual_target (NOT_CONVERGED if none within max_sweeps);
 * residual_target <= 0: exactly max_sweeps sweeps.  stats: [host] or NULL.
 * Errors: STATE (no detect since the last integrate), NUMERIC (NaN residual),
 * NOT_CONVERGED, DEVICE. */
nbgs_status nbgs_solve(nbgs_scene_t scene, int32_t max_sweeps, double residual_target, nbgs_stats *stats);

/* Semi-implicit Euler (eq. (integrationscheme)): v <- v', w <- w',
 * x <- x + dt v', q <- normalise(q + dt Q(q) w'), periodic wrap.  Saves the
 * (key, impulse) table for the next step's warm start.  Errors: STATE (no
 * solve since the last detect), DEVICE. */
nbgs_status nbgs_integrate(nbgs_scene_t scene);

/* nbgs_detect + nbgs_solve + nbgs_integrate.  NOT_CONVERGED from the solve is
 * returned after the integration has still been done. */
nbgs_status nbgs_step(nbgs_scene_t scene, int32_t max_sweeps, double residual_target, nbgs_stats *stats);

/* Copy the current contact list in canonical (key) order into caller buffers
 * [device], each NULL-able: j1, j2, key, colour of length cap; normal and
 * impulse as three consecutive planes of cap doubles (x[cap], y[cap], z[cap]);
 * xi of length cap.  impulse holds the initial impulses after nbgs_detect and
 * the solved ones after nbgs_solve.  *n_out [host] receives the contact
 * count; CAPACITY if it exceeds cap (nothing copied).  Synchronises. */
nbgs_status nbgs_get_contacts(nbgs_scene_t scene, int64_t cap, int32_t *j1, int32_t *j2, uint64_t *key,
                              int32_t *colour, double *normal, double *xi, double *impulse, int64_t *n_out);

/* Copy the velocity accumulators v', w' after the last solve into [device]
 * buffers of 3 n doubles each (planes x[n], y[n], z[n]).  STATE before the
 * first solve. */
nbgs_status nbgs_get_accumulators(nbgs_scene_t scene, double *v, double *w);

/* Residual history of the last solve: R of sweeps 1..min(cap, sweeps) into
 * hist [host]; *n_out [host] = number of sweeps.  Entries of sweeps whose
 * residual was not formed (see nbgs_set_residual_history) are NaN.
 * Synchronises. */
nbgs_status nbgs_get_residuals(nbgs_scene_t scene, int32_t cap, double *hist, int32_t *n_out);

/* Solver of later steps: edge = 0 (default) the NBGS in colour order (one
 * subdomain, the classic Gauss-Seidel of Alg. 1); edge > 0 the subdomain
 * NBGS of Alg. 1, whose subdomain affinity s_c(j) is the block holding body
 * j1's centre when the box is cut into max(1, floor(L_a / edge)) blocks of
 * edge L_a / that count per axis (domain partitioning, Sect. 6.1).  A contact
 * sees the newest impulses of the contacts of its subdomain relaxed before it
 * (colouring restricted to the subdomain, order (subdomain, colour, key)) and
 * the last iteration's impulses of all others; with accumulated velocities
 * and per-subdomain velocity corrections summed at the end of every sweep in
 * ascending subdomain (Sect. 6.3).  The relaxation must be below 1 (the
 * paper's runs use 0.75): across subdomains the iteration is a Jacobi one,
 * which diverges unrelaxed on dense packings; INVALID_ARG at relaxation 1
 * here and from nbgs_scene_set_params while the solver is on.
 * CAPACITY at detection if a subdomain touches too many bodies for the
 * workgroup's local memory (about 540 in FP64): use a smaller edge.
 * UNSUPPORTED for batches and with the learned warm start. */
nbgs_status nbgs_set_subdomains(nbgs_scene_t scene, double edge);

/* Sweep order of later steps: edge = 0 (default) the (colour, key) order;
 * edge > 0 the block-local order of the same plain NBGS (Alg. 1 with one
 * subdomain: every contact sees the newest impulses of all others, only the
 * order in which the contacts are visited changes).  With the box cut into
 * blocks as for nbgs_set_subdomains, a contact whose dynamic bodies lie in
 * one block is local to it; a contact between dynamic bodies of two blocks
 * is a cross contact.  A sweep takes every block's local contacts in
 * (colour, key) order, blocks in ascending order (local contacts of different
 * blocks share no dynamic body, so the blocks run as independent workgroups
 * with their bodies' velocities held in LDS), then the cross contacts in
 * (colour, key) order; each colouring covers one block's local contacts or
 * the cross contacts.  The initial impulses are applied in the same order.
 * CAPACITY at detection if a block holds too many bodies for the
 * workgroup's local memory (about 960 in FP64, 1,900 in FP32): use a smaller
 * edge.  INVALID_ARG while the subdomain solver is on; UNSUPPORTED for
 * batches and with the learned warm start. */
nbgs_status nbgs_set_block_order(nbgs_scene_t scene, double edge);

/* Number of block grids of the block-local order (1 .. 8, default 1): grid g
 * is the block grid of nbgs_set_block_order shifted by g/grids of a block edge
 * along every axis (taken modulo the box along a periodic axis; along another
 * axis a shifted grid has one block more).  A contact is local to the first
 * grid in one of whose blocks all its dynamic bodies lie, with the id g B +
 * block (B blocks per grid), or a contact between blocks if there is none.  A
 * sweep takes the local contacts grid by grid (blocks ascending, each in
 * (colour, key) order; the local contacts of two blocks of a grid share no
 * dynamic body, so a grid's blocks run as independent workgroups), then the
 * rest in (colour, key) order: the same plain NBGS (Alg. 1 with one
 * subdomain), visited in another order.  With four grids a contact whose
 * centres differ by less than a quarter block edge along every axis is
 * always local.  With two or more grids the rest, which touch each other only
 * through shared dynamic bodies, are swept by cluster (the components of
 * "shares a dynamic body", packed whole into groups that the block pass runs
 * as it runs blocks): each cluster in its (colour, key) order, so every
 * contact is relaxed as in the colour-ordered sweep of the rest, bit for bit;
 * when a group would exceed the workgroup's local memory they are swept
 * colour by colour.  Takes effect at the next detection; INVALID_ARG outside
 * 1 .. 8. */
nbgs_status nbgs_set_block_grids(nbgs_scene_t scene, int32_t grids);

/* The pair list of the detection (Sect. 4 broad phase), enable = 1 (the
 * default) or 0.  With it a detection keeps every pair whose hulls would
 * overlap with hull radius `skin` (max(4 max h, 0.02 max(r + h)) at the
 * build) and, while every body's displacement since the build plus its hull
 * plus its radius growth stays below the skin and no body changed between
 * static and dynamic, finds the step's contacts by testing those pairs only
 * (the same predicates as the cell-grid phase, so the same contacts, bit for
 * bit); otherwise it rebuilds the list.  The list is kept only when the
 * workspace has room for it beside everything the step may need (16 B per
 * listed pair, 41 B per body); else every detection uses the cell grid.
 * Setting it drops the current list.  Errors: INVALID_ARG (NULL). */
nbgs_status nbgs_set_pair_list(nbgs_scene_t scene, int32_t enable);

/* The pair list's state [host, each NULL-able]: *pairs = listed pairs (-1
 * when no list is held), *skin its hull radius, *builds how many lists the
 * scene has built. */
nbgs_status nbgs_get_pair_list_info(nbgs_scene_t scene, int64_t *pairs, double *skin, int64_t *builds);

/* enable = 1 (default): the residual R_k of every sweep is formed.  enable =
 * 0: a solve without a residual target forms only the last sweep's residual
 * (the one nbgs_stats reports); impulses and velocities are unchanged.  A
 * solve with a target always forms every sweep's residual. */
nbgs_status nbgs_set_residual_history(nbgs_scene_t scene, int32_t enable);

/* Replace the previous-step table used by NBGS_WS_PREVIOUS: n entries, keys
 * [device] strictly ascending, impulse [device] three planes of n doubles.
 * The next nbgs_detect matches every contact's key in it, re-projects the
 * impulse onto the new normal and cone (P_n = max(0, n.P), |P_t| <= mu P_n)
 * and starts unmatched contacts at zero. */
nbgs_status nbgs_set_warm_start(nbgs_scene_t scene, int64_t n, const uint64_t *keys, const double *impulse);

/* Device milliseconds of the phases of the last step (HIP events on the
 * scene's stream): out[0] detect (hull, sort, cells, pairs, narrow phase),
 * out[1] colouring and ordering, out[2] accumulator init, out[3] sweeps
 * incl. residuals, out[4] integrate.  n: entries wanted (<= 5).
 * Synchronises. */
nbgs_status nbgs_get_phase_times(nbgs_scene_t scene, int32_t n, double *out);

/* Launch shape of the sweep kernel (results do not depend on it: every
 * contact is relaxed by the same arithmetic).  block: threads per workgroup,
 * 64, 128, 256 or 512; contacts_per_thread: 1, 2 or 4; xcd_remap: 1 maps
 * consecutive workgroups, which the dispatcher deals round-robin over the
 * 8 XCDs, onto contiguous contact ranges per XCD (shared body records stay
 * in one L2), 0 keeps the identity mapping; nontemporal: 1 puts the
 * non-temporal hint on the streamed per-contact arrays; full_store: 1 writes
 * each touched body record back whole (its constants unchanged), so the write
 * covers the record's aligned bytes; persistent: 1 launches at most the
 * workgroups the device holds resident at once, each walking several tiles,
 * a multiple of 8 launches at most that many workgroups, 0 one per tile;
 * graph: 1 replays the sweeps from a captured HIP graph (blocks of up to 32
 * sweeps, colour ranges read on the device, persistent workgroups: the
 * resident count unless persistent gives a multiple of 8); lane_groups: 1
 * relaxes each contact by a group of lanes, one per 16 B piece of a body
 * record (4 lanes in FP64, 2 in FP32; needs contacts_per_thread 1): the group
 * loads and stores each touched record whole in one instruction and shares it
 * by lane broadcasts, every lane evaluating the contact.  Impulses and
 * velocities do not depend on any of these; the residual's partial sums are
 * grouped per tile (per workgroup with graph), so only its rounding may.
 * Defaults (block / contacts_per_thread / xcd_remap / nontemporal /
 * full_store / persistent / graph / lane_groups): FP64 256/1/1/1/0/0/0/1,
 * FP32 256/1/1/0/0/1/0/1 for a scene; a batch also sets graph 1 and
 * persistent 1. */
typedef struct {
    int32_t block;
    int32_t contacts_per_thread;
    int32_t xcd_remap;
    int32_t nontemporal;
    int32_t full_store;
    int32_t persistent;
    int32_t graph;
    int32_t lane_groups;
} nbgs_tuning;

/* Set / read the sweep launch shape used for precision (nbgs_precision).
 * INVALID_ARG for an unsupported shape.  A shape set here is kept: a batch
 * does not autotune that precision afterwards. */
nbgs_status nbgs_set_tuning(nbgs_scene_t scene, int32_t precision, const nbgs_tuning *tuning);
nbgs_status nbgs_get_tuning(nbgs_scene_t scene, int32_t precision, nbgs_tuning *tuning);

/* Choose the sweep launch shape for the scene's precision by timing trial
 * solves of `sweeps` sweeps on the contacts of the current step (call after
 * nbgs_detect, before nbgs_solve): coordinate descent over the nbgs_tuning
 * fields from the current shape (UNSUPPORTED with the subdomain solver or
 * the block-local order).  The trials leave no trace: the initial
 * impulses are restored, and the solve that follows gives the same impulses
 * and velocities as without tuning.  cache_path [host, may be NULL]: a text
 * file of earlier choices, one line per (GPU architecture, precision,
 * scene or batch, ceil log2 of the contact count); a cached choice is taken
 * without trials and a new one is appended.  *chosen [host, may be NULL]
 * receives the shape, *ms_per_sweep [host, may be NULL] its time per sweep.
 * STATE unless a step is detected and not solved.  Synchronises. */
nbgs_status nbgs_autotune(nbgs_scene_t scene, int32_t sweeps, const char *cache_path, nbgs_tuning *chosen,
                          double *ms_per_sweep);

/* Sweep-kernel profile accumulated while profiling is enabled. */
typedef struct {
    double sweep_kernel_ms;  /* sum of device times of the sweep launches (HIP event pair per launch) */
    int64_t sweep_launches;  /* non-empty colour launches timed */
    double sweep_bytes;      /* compulsory bytes of those launches: per contact its record (ids, normal, xi/dt,
                                arms, impulse read + write: 104 B FP64, 56 B FP32), per dynamic body touched its
                                record read + v', w' written (112 B FP64, 56 B FP32) */
    int64_t contact_updates; /* contact relaxations done by those launches */
} nbgs_profile;

/* Enable (1) or disable (0) profiling of the sweep launches of later
 * nbgs_solve calls; enabling resets the accumulated profile.  While enabled,
 * every sweep launch is bracketed by two HIP events on the scene's stream and
 * nbgs_solve synchronises at its end. */
nbgs_status nbgs_set_profiling(nbgs_scene_t scene, int32_t enable);

/* Copy the accumulated profile into *out [host]. */
nbgs_status nbgs_get_profile(nbgs_scene_t scene, nbgs_profile *out);

/* ------------------------------------------------------- batched scenes
 *
 * Many independent scenes of uneven size stepped together.  Each scene is a
 * separate granular system (its own box, periodicity, walls, friction
 * coefficient and colouring seed; Alg. 2 per scene); they share one body
 * array and one set of launches: colour c of every scene is relaxed by the
 * same sweep launch.  Each scene is detected, coloured, ordered and relaxed
 * exactly as it would be alone (same contacts, colours and FP arithmetic), so
 * its impulses and velocities after a fixed number of sweeps equal those of a
 * scene created for it alone.  The residual of a batch is that of all its
 * contacts together, so a residual target stops all scenes at one sweep. */
typedef struct nbgs_batch_s *nbgs_batch_t;

/* n_scenes >= 1 scenes; body_offsets [host, n_scenes + 1 int64]: scene s owns
 * bodies body_offsets[s] .. body_offsets[s + 1] - 1 of `bodies` (device SoA
 * as for nbgs_scene_create, borrowed), body_offsets[0] = 0 and
 * body_offsets[n_scenes] = bodies->n, every scene non-empty.  domains,
 * params [host, n_scenes each]: per-scene box and walls; params may differ
 * between scenes only in mu and colour_seed (INVALID_ARG otherwise);
 * NBGS_WS_LEARNED is UNSUPPORTED.  Wall w of scene s has body id
 * bodies->n + (walls of scenes 0 .. s-1) + w in contact lists.
 * tune_cache_path [host, may be NULL, copied]: autotuner cache file (see
 * nbgs_autotune).  workspace [device], workspace_bytes: as for
 * nbgs_scene_create, sized by nbgs_batch_workspace_query; a batch moves to a
 * larger one with nbgs_scene_set_workspace on nbgs_batch_scene's handle.  The
 * batch autotunes the launch shape of its sweeps on its first step of each
 * precision unless nbgs_set_tuning set one (the candidates include replay of
 * the sweeps from a captured HIP graph over resident workgroups). */
nbgs_status nbgs_batch_create(int32_t n_scenes, const int64_t *body_offsets, const nbgs_bodies *bodies,
                              const nbgs_domain *domains, const nbgs_params *params, const char *tune_cache_path,
                              void *workspace, size_t workspace_bytes, void *hip_stream, nbgs_batch_t *out);

/* Bytes of device workspace a batch of n_scenes scenes, n_bodies bodies in all
 * and up to contact_capacity contacts in all needs (nbgs_workspace_query's
 * bound with one cell table per scene).  params [host, n_scenes, may be
 * NULL].  Errors: INVALID_ARG. */
nbgs_status nbgs_batch_workspace_query(int32_t n_scenes, int64_t n_bodies, int64_t contact_capacity,
                                       const nbgs_params *params, size_t *bytes);
nbgs_status nbgs_batch_destroy(nbgs_batch_t batch);

/* The scene handle behind the batch (owned by the batch): every nbgs_scene_t
 * entry point except the learned warm start applies to the batch as a whole
 * (contacts in the shared numbering, accumulators of all bodies, tuning,
 * profiling, phase times, residual history). */
nbgs_status nbgs_batch_scene(nbgs_batch_t batch, nbgs_scene_t *scene);

/* n_steps time steps of every scene (detect, solve with max_sweeps /
 * residual_target as nbgs_solve, integrate).  *stats [host, may be NULL]: the
 * last step's totals.  *steps_done [host, may be NULL]: steps completed.
 * NOT_CONVERGED if the last solve missed its target.  CAPACITY when a
 * detection finds more contacts than the workspace holds: that step has not
 * run, stats->n_contacts holds the count (grow the workspace through
 * nbgs_batch_scene's handle and continue with the remaining steps). */
nbgs_status nbgs_batch_step(nbgs_batch_t batch, int32_t n_steps, int32_t max_sweeps, double residual_target,
                            nbgs_stats *stats, int32_t *steps_done);

/* Per-scene contact and colour counts of the last detected step into
 * n_contacts, n_colours [host, n entries, n = the scene count].  Synchronises. */
nbgs_status nbgs_batch_scene_stats(nbgs_batch_t batch, int32_t n, int64_t *n_contacts, int32_t *n_colours);

/* ------------------------------------------------ learned warm start (MLP)
 *
 * A 12-128-128-3 ReLU network that predicts each contact's impulse at the
 * start of a step from local features (the initial solution of Alg. 1 may be
 * any guess, Sect. 5).  BF16 matrix-core inference and training with FP32
 * accumulation and FP32 master weights.  Weight vector layout (18,563 floats):
 * W1[12][128], b1[128], W2[128][128], b2[128], W3[128][3], b3[3], layer
 * y = x W + b, ReLU after the first two layers. */
typedef struct nbgs_mlp_s *nbgs_mlp_t;

/* Number of weights (18,563). */
int32_t nbgs_mlp_param_count(void);

/* Bytes of device workspace of a network whose store of collected training
 * pairs holds max_samples samples and which trains on at most that many at a
 * time (weights, Adam moments, gradient partials of up to 1,024 blocks, and
 * 64 B per sample).  Errors: INVALID_ARG. */
nbgs_status nbgs_mlp_workspace_query(int64_t max_samples, size_t *bytes);

/* Create a network with deterministic initial weights (He-uniform hidden
 * layers, output layer scaled by 0.1, zero biases; uniforms from
 * splitmix64(seed + index)).  max_samples: capacity of its store of collected
 * training pairs (nbgs_mlp_collect).  workspace [device], workspace_bytes:
 * the caller's region (nbgs_mlp_workspace_query), borrowed until
 * nbgs_mlp_destroy.  hip_stream as for scenes. */
nbgs_status nbgs_mlp_create(uint64_t seed, int64_t max_samples, void *workspace, size_t workspace_bytes,
                            void *hip_stream, nbgs_mlp_t *out);
nbgs_status nbgs_mlp_destroy(nbgs_mlp_t mlp);

/* Replace / read the FP32 master weights ([host], 18,563 floats).  Setting
 * weights resets the Adam state. */
nbgs_status nbgs_mlp_set_weights(nbgs_mlp_t mlp, const float *weights);
nbgs_status nbgs_mlp_get_weights(nbgs_mlp_t mlp, float *weights);

/* out[n][3] = network(feat[n][12]); [device] row-major FP32, feat 16-byte
 * aligned (INVALID_ARG otherwise).  Features and hidden activations are
 * rounded to BF16 for the matrix cores. */
nbgs_status nbgs_mlp_forward(nbgs_mlp_t mlp, const float *feat, int64_t n, float *out);

/* Gradient of L = 1/(2n) sum |out - target|^2 over the n samples into grad
 * [device, 18,563 floats, may be NULL]; *loss [host, may be NULL] = L.
 * Deterministic (fixed reduction order). */
nbgs_status nbgs_mlp_loss_grad(nbgs_mlp_t mlp, const float *feat, const float *target, int64_t n, float *grad,
                               double *loss);

/* nbgs_mlp_loss_grad for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * kernels, with the per-block gradient and loss partials in a fixed device
 * array of the library (4.75 MB, one per GPU, kept until the process ends)
 * instead of the network's workspace; no allocation of any kind.  At most
 * 4,096 samples per call (INVALID_ARG beyond); grad [device] must be given.
 * Every call on one GPU shares that array: calls that overlap in time on one
 * GPU (several streams or threads) race and must be serialised by the caller.
 * Results equal nbgs_mlp_loss_grad's bit for bit. */
nbgs_status nbgs_mlp_loss_grad_static(nbgs_mlp_t mlp, const float *feat, const float *target, int64_t n,
                                      float *grad, double *loss);

/* Adam (lr, beta1 0.9, beta2 0.999, eps 1e-8) over `epochs` passes of
 * minibatches of `batch` samples drawn in a splitmix64 Fisher-Yates order
 * from shuffle_seed; feat [device n x 12], target [device n x 3].
 * *final_loss [host, may be NULL] = mean L over the last epoch. */
nbgs_status nbgs_mlp_train(nbgs_mlp_t mlp, const float *feat, const float *target, int64_t n, int32_t epochs,
                           int32_t batch, float lr, uint64_t shuffle_seed, double *final_loss);

/* Append the training pairs of the scene's last solved step (every contact's
 * features at the step's start and its solved impulse in the contact frame
 * scaled by 1/(ms vs), the network being trained on impulses the solver
 * itself produced) to the network's store.  The step's nbgs_detect must have
 * computed features (learned warm start or nbgs_set_feature_capture).
 * *n_stored [host, may be NULL] = samples held afterwards.  Synchronises the
 * scene's stream.  Errors: STATE (no features or no solve), CAPACITY (the
 * store's max_samples would be exceeded; nothing appended). */
nbgs_status nbgs_mlp_collect(nbgs_scene_t scene, nbgs_mlp_t mlp, int64_t *n_stored);

/* nbgs_mlp_train on every collected pair.  STATE if none. */
nbgs_status nbgs_mlp_train_collected(nbgs_mlp_t mlp, int32_t epochs, int32_t batch, float lr, uint64_t shuffle_seed,
                                     double *final_loss);

/* The collected store: *n [host] pairs, *feat [device n x 12], *target
 * [device n x 3] (FP32, owned by the network, valid until the next collect or
 * clear); each output NULL-able. */
nbgs_status nbgs_mlp_collected(nbgs_mlp_t mlp, int64_t *n, const float **feat, const float **target);

/* Empty the store. */
nbgs_status nbgs_mlp_clear_collected(nbgs_mlp_t mlp);

/* Use `mlp` (NULL detaches) for NBGS_WS_LEARNED; the scene borrows it. */
nbgs_status nbgs_scene_attach_mlp(nbgs_scene_t scene, nbgs_mlp_t mlp);

/* Compute the network features of every contact at each nbgs_detect even when
 * the warm start is not learned (for collecting training data). */
nbgs_status nbgs_set_feature_capture(nbgs_scene_t scene, int32_t enable);

/* Velocity, mass and length scales of the features: vs = |g| dt (1e-3 if
 * g = 0), ms = mean mass of the dynamic bodies, rs = mean radius.  out [host]
 * receives (vs, ms, rs). */
nbgs_status nbgs_get_feature_scales(nbgs_scene_t scene, double *out);

/* After nbgs_solve (and until the next nbgs_detect) of a step whose
 * nbgs_detect computed features: the
 * features [device cap x 12] and the solved impulses in the contact frame
 * divided by ms vs [device cap x 3] (training pairs), canonical order.
 * *n_out [host] = contact count; CAPACITY if it exceeds cap; STATE if no
 * features or no solve.  Either output may be NULL. */
nbgs_status nbgs_get_training_data(nbgs_scene_t scene, int64_t cap, float *feat, float *target, int64_t *n_out);

/* Outcome of the last learned warm start: choice 1 = network, 0 = previous
 * step, -1 = not judged; the two Jacobi residuals. */
typedef struct {
    int32_t choice;
    double r_previous;
    double r_learned;
} nbgs_warm_info;
nbgs_status nbgs_get_warm_start_info(nbgs_scene_t scene, nbgs_warm_info *out);

/* The learned initial impulses of the last nbgs_detect (NBGS_WS_LEARNED with
 * a network attached): for a contact the previous step also had, its
 * re-projected previous impulse; for a new contact the network output decoded
 * from the contact frame and projected onto the friction cone (the initial
 * solution of Alg. 1 may be any estimate, Sect. 5).  impulse [device]: three
 * planes of cap doubles (x[cap], y[cap], z[cap]), canonical (key) order.
 * *n_out [host] = contact count; CAPACITY if it exceeds cap; STATE if the
 * last detection made no learned start.  Synchronises. */
nbgs_status nbgs_get_learned_start(nbgs_scene_t scene, int64_t cap, double *impulse, int64_t *n_out);

/* ------------------------------------------------------------------------
 * Composite particles: rigid clusters of element spheres (Sect. 2 builds
 * non-spherical particles from primitives glued together; the granular gas of
 * Sect. 7.2.1 uses two to four spheres per particle).
 *
 * A body is its centre of mass x, an orientation q (unit quaternion mapping
 * the principal body frame to the world), velocities v and w (world frame),
 * 1/m, the principal inverse moments (body frame), the bounding radius rbar
 * about the centre of mass and its elements: spheres of radius r_e centred at
 * o_e in body coordinates.  One time step:
 *   detect     hull radius h = dt (|v| + |w| rbar) + tau (eq. (expansionradius));
 *              every pair of elements of different bodies whose spheres grown
 *              by their bodies' h meet, and every element whose grown sphere
 *              reaches a wall, is a contact (eq. (contactpos) of two spheres:
 *              normal from the centre of j2's element to j1's, contact point
 *              on the surface of j2's element); then colouring as for
 *              spheres and initial impulses (zero or the previous step's);
 *   solve      accumulators v' = v + dt g, w' = w + dt I^-1 (-w x I w) (the
 *              gyroscopic term of eq. (integrationscheme)), then NBGS sweeps
 *              colour by colour with the full 3x3 Delassus block of the two
 *              bodies at the contact (eq. (wrench)) and the exact solution of
 *              the one-contact problem of eqs. (nonpenetration), (coulomb):
 *              separate, stick, or slide with the tangential multiplier found
 *              by safeguarded Newton steps;
 *   integrate  eq. (integrationscheme) as for spheres.
 * Conventions as above, except that a contact joins ELEMENTS: j1 < j2 are the
 * bodies, the key is (element of j1 << 32) | element of j2, a wall w is body
 * n_bodies + w and element n_elements + w, and the lever arms r1 = x_hat - x_j1,
 * r2 = x_hat - x_j2 (zero for a wall) are part of the contact.  FP64 only.
 * ------------------------------------------------------------------------ */

typedef struct nbgs_composite_s *nbgs_composite_t;

typedef struct {
    int64_t n; /* bodies */
    /* [device] body state, n each, updated in place by integrate / step */
    double *x, *y, *z, *qw, *qx, *qy, *qz, *vx, *vy, *vz, *wx, *wy, *wz;
    const double *inv_mass;    /* [device] n; 0: static body */
    const double *inv_inertia; /* [device] 3 n principal inverse moments, xyz interleaved; 0 0 0: no rotation */
    const double *bound;       /* [device] n bounding radius about the centre of mass */
    const int32_t *elem_start; /* [device] n + 1: body i owns elements elem_start[i] .. elem_start[i+1]-1 */
    int64_t n_elements;
    const double *elem_offset; /* [device] 3 E element centres in body coordinates, xyz interleaved */
    const double *elem_radius; /* [device] E */
} nbgs_composite_bodies;

/* Bytes of device workspace of a composite scene of n_bodies bodies,
 * n_elements elements and up to contact_capacity contacts (an upper bound:
 * per element 352 B, per body 164 B, per contact 525 B, a cell table of 2^16
 * cells, 16 MiB, ten per cent).  params may be NULL.  Errors: INVALID_ARG. */
nbgs_status nbgs_composite_workspace_query(int64_t n_bodies, int64_t n_elements, int64_t contact_capacity,
                                           const nbgs_params *params, size_t *bytes);

/* Create a composite scene that borrows the arrays.  bodies, domain, params:
 * [host] structs.  workspace [device], workspace_bytes: as for
 * nbgs_scene_create (nbgs_composite_workspace_query).  Errors: INVALID_ARG
 * (null pointer or workspace, n < 1, fewer elements than bodies, elem_start
 * not running from 0 to n_elements, bad parameters or domain as for
 * nbgs_scene_create), UNSUPPORTED (precision other than NBGS_FP64, learned
 * warm start), CAPACITY, OUT_OF_MEMORY (host), DEVICE.  Release the handle
 * with nbgs_composite_destroy.  nbgs_composite_detect returns CAPACITY with
 * the contact count in stats->n_contacts when the workspace holds fewer, and
 * with stats->n_contacts = -1 for the limits no workspace lifts. */
nbgs_status nbgs_composite_create(const nbgs_composite_bodies *bodies, const nbgs_domain *domain,
                                  const nbgs_params *params, void *workspace, size_t workspace_bytes,
                                  void *hip_stream, nbgs_composite_t *out);

/* Move the composite scene into another workspace, as nbgs_scene_set_workspace. */
nbgs_status nbgs_composite_set_workspace(nbgs_composite_t scene, void *workspace, size_t bytes);
nbgs_status nbgs_composite_destroy(nbgs_composite_t scene);

/* Detection, colouring, initial impulses (see above).  stats [host, may be
 * NULL]: contact and colour counts.  Errors: STATE (detected twice without a
 * solve and integrate), CAPACITY (an element meets more than 2^18 hull
 * candidates, 2^31 contacts or more, more than 255 colours), NUMERIC (a
 * non-finite body state). */
nbgs_status nbgs_composite_detect(nbgs_composite_t scene, nbgs_stats *stats);

/* Accumulator init and NBGS sweeps: exactly max_sweeps (residual_target <= 0)
 * or until R <= residual_target (checked after every sweep; the host looks
 * every 8 sweeps, later sweeps are no-ops).  Errors: STATE (not detected, or
 * solved already), NOT_CONVERGED (impulses still valid), NUMERIC. */
nbgs_status nbgs_composite_solve(nbgs_composite_t scene, int32_t max_sweeps, double residual_target,
                                 nbgs_stats *stats);

/* Semi-implicit Euler of the body state with the solved accumulators.
 * STATE if the step is not solved. */
nbgs_status nbgs_composite_integrate(nbgs_composite_t scene);

/* detect + solve + integrate; returns NOT_CONVERGED after integrating if the
 * target was missed. */
nbgs_status nbgs_composite_step(nbgs_composite_t scene, int32_t max_sweeps, double residual_target,
                                nbgs_stats *stats);

/* The current contact list in canonical (key) order into [device] buffers of
 * capacity cap (any may be NULL): j1, j2 (bodies), key, colour, impulse
 * (3 cap doubles: planes x[cap], y[cap], z[cap], the solved impulse after a
 * solve, else the initial one) and geometry (10 cap doubles, planes n_x, n_y,
 * n_z, xi, r1 (3), r2 (3)).  *n_out [host] = contact count.  cap = 0 only
 * queries the count.  CAPACITY if 0 < cap < count; STATE before the first
 * detection.  Synchronises. */
nbgs_status nbgs_composite_get_contacts(nbgs_composite_t scene, int64_t cap, int32_t *j1, int32_t *j2, uint64_t *key,
                                        int32_t *colour, double *impulse, double *geometry, int64_t *n_out);

/* Velocity accumulators v', w' after the last solve into [device] buffers of
 * 3 n doubles each (planes x[n], y[n], z[n]).  STATE before the first solve. */
nbgs_status nbgs_composite_get_accumulators(nbgs_composite_t scene, double *v, double *w);

/* Residuals R of sweeps 1 .. min(cap, sweeps) of the last solve into hist
 * [host]; *n_out [host] = sweeps done.  Synchronises. */
nbgs_status nbgs_composite_get_residuals(nbgs_composite_t scene, int32_t cap, double *hist, int32_t *n_out);

/* Wall-clock milliseconds [host, n <= 5] of the last step's phases from
 * events on the scene's stream: detection, colouring and sweep order,
 * accumulator init with initial impulses, sweeps, integration (-1 where a
 * phase did not run).  Synchronises. */
nbgs_status nbgs_composite_get_phase_times(nbgs_composite_t scene, int32_t n, double *out);

#ifdef __cplusplus
}
#endif

#endif /* NBGS_H */
