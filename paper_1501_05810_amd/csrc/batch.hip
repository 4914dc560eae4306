// Many independent scenes of uneven size in one set of launches.
//
// The scenes share one body array (scene s owns a contiguous range of it) and
// one contact table.  Detection runs one cell grid per scene laid out in a
// shared cell table, so a body only meets bodies and walls of its own scene;
// colouring uses each scene's own pair numbering and seed, so a scene gets the
// colours, order and arithmetic it would get alone (the per-scene friction
// coefficient travels with each contact).  Colour c of every scene is relaxed
// by the same launch, so a sweep costs as many launches as the largest
// colour count, not the sum over scenes.  nbgs_batch_step drives each step
// from the host (detection, colouring, solve, integration enqueued one after
// another on the batch's stream); the launch shape of the sweeps comes from
// the autotuner on the first step of each precision, whose candidates
// include persistent workgroups and replay of the sweeps from a captured HIP
// graph.
#include <algorithm>
#include <new>

#include "scene.h"

struct nbgs_batch_s {
    nbgs_scene_t sc = nullptr;
    int32_t tune_sweeps = 8;
};

using namespace nbgs;

extern "C" {

nbgs_status nbgs_batch_workspace_query(int32_t n_scenes, int64_t n_bodies, int64_t contact_capacity,
                                       const nbgs_params *params, size_t *bytes) {
    if (!bytes || n_scenes < 1 || n_bodies < 0 || contact_capacity < 0) {
        set_error("bad arguments to nbgs_batch_workspace_query");
        return NBGS_ERR_INVALID_ARG;
    }
    if (params)
        for (int32_t s = 0; s < n_scenes; ++s) NBGS_TRY(check_params(&params[s]));
    *bytes = scene_workspace_bytes(n_bodies, contact_capacity, n_scenes);
    return NBGS_OK;
}

nbgs_status nbgs_batch_create(int32_t n_scenes, const int64_t *body_offsets, const nbgs_bodies *bodies,
                              const nbgs_domain *domains, const nbgs_params *params, const char *tune_cache_path,
                              void *workspace, size_t workspace_bytes, void *hip_stream, nbgs_batch_t *out) {
    if (!out) {
        set_error("out is NULL");
        return NBGS_ERR_INVALID_ARG;
    }
    *out = nullptr;
    nbgs_batch_t bt = new (std::nothrow) nbgs_batch_s();
    if (!bt) {
        set_error("host allocation failed");
        return NBGS_ERR_OUT_OF_MEMORY;
    }
    const nbgs_status st = scene_create(workspace, workspace_bytes, bodies, n_scenes, body_offsets, domains, params,
                                        hip_stream, &bt->sc);
    if (st != NBGS_OK) {
        delete bt;
        return st;
    }
    if (tune_cache_path) bt->sc->tune_cache = tune_cache_path;
    *out = bt;
    return NBGS_OK;
}

nbgs_status nbgs_batch_destroy(nbgs_batch_t bt) {
    if (!bt) return NBGS_OK;
    const nbgs_status st = nbgs_scene_destroy(bt->sc);
    delete bt;
    return st;
}

nbgs_status nbgs_batch_scene(nbgs_batch_t bt, nbgs_scene_t *scene) {
    if (!bt || !scene) {
        set_error("batch handle or output is NULL");
        return NBGS_ERR_INVALID_ARG;
    }
    *scene = bt->sc;
    return NBGS_OK;
}

nbgs_status nbgs_batch_step(nbgs_batch_t bt, int32_t n_steps, int32_t max_sweeps, double residual_target,
                            nbgs_stats *stats, int32_t *steps_done) {
    if (steps_done) *steps_done = 0;
    if (!bt) {
        set_error("batch handle is NULL");
        return NBGS_ERR_INVALID_ARG;
    }
    if (n_steps < 0 || max_sweeps < 1) {
        set_error("n_steps must be >= 0 and max_sweeps >= 1");
        return NBGS_ERR_INVALID_ARG;
    }
    nbgs_scene_t sc = bt->sc;
    ArenaScope arena_scope(&sc->arena);
    nbgs_status last = NBGS_OK;
    for (int32_t k = 0; k < n_steps; ++k) {
        nbgs_stats dst{};
        const nbgs_status ds = nbgs_detect(sc, &dst);
        if (ds != NBGS_OK) {
            if (ds == NBGS_ERR_CAPACITY && stats) *stats = dst;  // the contact count the workspace lacks
            return ds;
        }
        const int prec = sc->precision_used == NBGS_FP32_SWEEP ? 1 : 0;
        if (!sc->tuned[prec] && sc->nc > 0)
            NBGS_TRY(scene_autotune(sc, std::min(max_sweeps, bt->tune_sweeps), nullptr, nullptr));
        last = nbgs_solve(sc, max_sweeps, residual_target, k + 1 == n_steps ? stats : nullptr);
        if (last != NBGS_OK && last != NBGS_ERR_NOT_CONVERGED) return last;
        NBGS_TRY(nbgs_integrate(sc));
        if (steps_done) *steps_done = k + 1;
    }
    return last;
}

nbgs_status nbgs_batch_scene_stats(nbgs_batch_t bt, int32_t n, int64_t *n_contacts, int32_t *n_colours) {
    if (!bt || n < 0 || (n > 0 && (!n_contacts || !n_colours))) {
        set_error("bad arguments");
        return NBGS_ERR_INVALID_ARG;
    }
    nbgs_scene_t sc = bt->sc;
    if (n != sc->n_scenes) {
        set_error("the batch holds %d scenes, not %d", sc->n_scenes, n);
        return NBGS_ERR_INVALID_ARG;
    }
    std::fill(n_contacts, n_contacts + n, 0);
    std::fill(n_colours, n_colours + n, 0);
    const int64_t m = sc->nc;
    if (m == 0) return NBGS_OK;
    std::vector<int32_t> j1((size_t)m), col((size_t)m);
    ContactBuf &cb = sc->cb[sc->cur];
    NBGS_HIP(hipStreamSynchronize(sc->s));
    NBGS_HIP(hipMemcpy(j1.data(), cb.j1.p, sizeof(int32_t) * m, hipMemcpyDeviceToHost));
    NBGS_HIP(hipMemcpy(col.data(), cb.colour.p, sizeof(int32_t) * m, hipMemcpyDeviceToHost));
    for (int64_t j = 0; j < m; ++j) {
        const int32_t s = (int32_t)(std::upper_bound(sc->body_off_h.begin(), sc->body_off_h.end(), j1[(size_t)j]) -
                                    sc->body_off_h.begin()) - 1;
        ++n_contacts[s];
        n_colours[s] = std::max(n_colours[s], col[(size_t)j] + 1);
    }
    return NBGS_OK;
}

}  // extern "C"
