/*
 * nbgs_ref.c -- ORACLE.  Test infrastructure only: the plain, slow, sequential
 * FP64 CPU reference for the per-time-step hard-contact solve of Preclik & Ruede,
 * "Ultrascale Simulations of Non-smooth Granular Dynamics".  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the GPU
 * library never does, and the two share no code.
 *
 * One time step (the single-process form of Alg. 2, Sect. 6.6):
 *   hull radii, eq. (expansionradius)                  -> nbgs_ref_hull_radii
 *   contact detection (Sect. 4; eq. (contactpos) solved
 *     analytically for spheres and planes)             -> nbgs_ref_detect_brute / _grid
 *   colouring of contacts (no two contacts in a colour
 *     share a dynamic body; replaces the subdomain
 *     affinity s_c(j) of Alg. 1)                       -> nbgs_ref_colour, nbgs_ref_sweep_order
 *   block-local sweep order (block by block, then the
 *     contacts between blocks)                         -> nbgs_ref_block_local, nbgs_ref_sweep_order_sub
 *   subdomain NBGS (Alg. 1 with block subdomains,
 *     Sect. 6.1, 6.3)                                  -> nbgs_ref_subdomains, nbgs_ref_solve_sub
 *   warm start from the previous step (Sect. 5)        -> nbgs_ref_warm_match
 *   accumulator init + NBGS sweeps (Alg. 1 with one
 *     subdomain, Sect. 6.3 velocity accumulators,
 *     eqs. (nonpenetration), (coulomb))                -> nbgs_ref_solve
 *   semi-implicit Euler, eq. (integrationscheme),
 *     quaternion renormalisation (Sect. 3)             -> nbgs_ref_integrate
 *
 * Units: the solver works with contact impulses P = dt * lambda (lambda is the
 * contact force of eq. (integrationscheme)), so v' = v + dt g + M^-1 (sum of P).
 *
 * Readings where the paper is silent (documented in the design notes):
 *   j1 is the lower body index, planes are always j2 and carry index n + w;
 *   contact point on the surface of j2 as in eq. (contactpos);
 *   coincident centres get n = +z;
 *   one-contact solve = exact solution of the 3x3 problem with the diagonal
 *     Delassus block of two spheres (normal clamp, then radial cone clip);
 *   colouring = greedy first-fit in descending splitmix64 priority;
 *   sweep order = (colour, key);  convergence = relative L2 impulse change.
 *
 * Compile with -ffp-contract=off: every expression is evaluated as written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "nbgs_ref.h"

/* ------------------------------------------------------------ hull radii */

/* eq. (expansionradius): h_i = dt (|v_i| + |omega_i| r_i) + tau, with the
 * bounding radius of a sphere equal to its radius. */
void nbgs_ref_hull_radii(const ref_bodies *b, const ref_params *p, double *h)
{
    for (int64_t i = 0; i < b->n; ++i) {
        double speed = sqrt(b->vx[i] * b->vx[i] + b->vy[i] * b->vy[i] + b->vz[i] * b->vz[i]);
        double spin = sqrt(b->wx[i] * b->wx[i] + b->wy[i] * b->wy[i] + b->wz[i] * b->wz[i]);
        h[i] = p->dt * (speed + spin * b->radius[i]) + p->tau;
    }
}

/* Minimum-image separation along one axis (periodic axes only). */
static double min_image(double d, const ref_domain *dom, int axis)
{
    if (!dom->periodic[axis]) return d;
    double L = dom->hi[axis] - dom->lo[axis];
    if (d > 0.5 * L) return d - L;
    if (d < -0.5 * L) return d + L;
    return d;
}

static int is_static(const ref_bodies *b, int64_t i) { return b->inv_mass[i] == 0.0; }

/* Sphere i (j1) against sphere k (j2), k > i.  The hulls S + ball(h) of
 * Sect. 4 intersect iff |x_i - x_k| <= (r_i + h_i) + (r_k + h_k).  For two
 * spheres eq. (contactpos) has the closed form: n points from the centre of
 * j2 to the centre of j1, the contact point sits on the surface of j2,
 * x_hat = x_k + r_k n, and xi = |x_i - x_k| - r_i - r_k. */
static int sphere_pair(const ref_bodies *b, const ref_domain *dom, const double *h, int64_t i, int64_t k,
                       double *n, double *xi, double *a1, double *a2)
{
    double dx = min_image(b->x[i] - b->x[k], dom, 0);
    double dy = min_image(b->y[i] - b->y[k], dom, 1);
    double dz = min_image(b->z[i] - b->z[k], dom, 2);
    double d2 = dx * dx + dy * dy + dz * dz;
    double reach = (b->radius[i] + h[i]) + (b->radius[k] + h[k]);
    if (!(d2 <= reach * reach)) return 0;
    double d = sqrt(d2);
    if (d2 > 0.0) {
        n[0] = dx / d;
        n[1] = dy / d;
        n[2] = dz / d;
    } else {
        n[0] = 0.0;
        n[1] = 0.0;
        n[2] = 1.0;
    }
    *xi = (d - b->radius[i]) - b->radius[k];
    *a1 = b->radius[i] + *xi;
    *a2 = b->radius[k];
    return 1;
}

/* Sphere i (j1) against wall plane w (j2, infinite inertia, Sect. 6.4).  The
 * plane's hull radius is tau (it does not move).  Signed distance of the
 * centre s = n_w . (x_i - p_w); xi = s - r_i; the contact point is the foot
 * of the perpendicular on the plane. */
static int sphere_plane(const ref_bodies *b, const ref_plane *pl, double h_i, double tau, int64_t i,
                        double *n, double *xi, double *a1, double *a2)
{
    double s = pl->normal[0] * (b->x[i] - pl->point[0]) + pl->normal[1] * (b->y[i] - pl->point[1]) +
               pl->normal[2] * (b->z[i] - pl->point[2]);
    double gap = s - b->radius[i];
    if (!(gap <= h_i + tau)) return 0;
    n[0] = pl->normal[0];
    n[1] = pl->normal[1];
    n[2] = pl->normal[2];
    *xi = gap;
    *a1 = b->radius[i] + gap;
    *a2 = 0.0;
    return 1;
}

static void put_contact(ref_contacts *c, int64_t m, int64_t j1, int64_t j2, const double *n, double xi, double a1,
                        double a2)
{
    if (m >= c->cap) return;
    c->j1[m] = (int32_t)j1;
    c->j2[m] = (int32_t)j2;
    c->key[m] = ((uint64_t)(uint32_t)j1 << 32) | (uint64_t)(uint32_t)j2;
    c->nx[m] = n[0];
    c->ny[m] = n[1];
    c->nz[m] = n[2];
    c->xi[m] = xi;
    c->a1[m] = a1;
    c->a2[m] = a2;
}

/* Contact detection by exhaustive pair testing (the definition of the
 * potential-contact set C of Sect. 4).  Pairs of two static bodies are not
 * contacts.  Output is in ascending key order.  Returns the number of
 * contacts; only the first cap are written. */
int64_t nbgs_ref_detect_brute(const ref_bodies *b, const ref_domain *dom, const ref_params *p, ref_contacts *out)
{
    double *h = (double *)malloc(sizeof(double) * (size_t)(b->n > 0 ? b->n : 1));
    nbgs_ref_hull_radii(b, p, h);
    int64_t m = 0;
    double n[3], xi, a1, a2;
    for (int64_t i = 0; i < b->n; ++i) {
        for (int64_t k = i + 1; k < b->n; ++k) {
            if (is_static(b, i) && is_static(b, k)) continue;
            if (sphere_pair(b, dom, h, i, k, n, &xi, &a1, &a2)) put_contact(out, m++, i, k, n, xi, a1, a2);
        }
        if (is_static(b, i)) continue;
        for (int32_t w = 0; w < dom->n_planes; ++w)
            if (sphere_plane(b, &dom->planes[w], h[i], p->tau, i, n, &xi, &a1, &a2))
                put_contact(out, m++, i, b->n + w, n, xi, a1, a2);
    }
    free(h);
    return m;
}

/* Contacts of one body i only, by testing it against every other body and
 * every wall (the definition restricted to pairs containing i), in key order.
 * Lets large scenes be checked on sampled bodies.  Returns the count. */
int64_t nbgs_ref_detect_body(const ref_bodies *b, const ref_domain *dom, const ref_params *p, int64_t i,
                             ref_contacts *out)
{
    /* hull radii of body i and of each partner, eq. (expansionradius) */
    double h_i, h_k;
    int64_t m = 0;
    double n[3], xi, a1, a2;
    {
        double speed = sqrt(b->vx[i] * b->vx[i] + b->vy[i] * b->vy[i] + b->vz[i] * b->vz[i]);
        double spin = sqrt(b->wx[i] * b->wx[i] + b->wy[i] * b->wy[i] + b->wz[i] * b->wz[i]);
        h_i = p->dt * (speed + spin * b->radius[i]) + p->tau;
    }
    for (int64_t k = 0; k < b->n; ++k) {
        if (k == i) continue;
        if (is_static(b, i) && is_static(b, k)) continue;
        double speed = sqrt(b->vx[k] * b->vx[k] + b->vy[k] * b->vy[k] + b->vz[k] * b->vz[k]);
        double spin = sqrt(b->wx[k] * b->wx[k] + b->wy[k] * b->wy[k] + b->wz[k] * b->wz[k]);
        h_k = p->dt * (speed + spin * b->radius[k]) + p->tau;
        int64_t lo = k < i ? k : i, hi = k < i ? i : k;
        const double h_lo = lo == i ? h_i : h_k, h_hi = hi == i ? h_i : h_k;
        double dx = min_image(b->x[lo] - b->x[hi], dom, 0);
        double dy = min_image(b->y[lo] - b->y[hi], dom, 1);
        double dz = min_image(b->z[lo] - b->z[hi], dom, 2);
        double d2 = dx * dx + dy * dy + dz * dz;
        double reach = (b->radius[lo] + h_lo) + (b->radius[hi] + h_hi);
        if (!(d2 <= reach * reach)) continue;
        double d = sqrt(d2);
        if (d2 > 0.0) {
            n[0] = dx / d;
            n[1] = dy / d;
            n[2] = dz / d;
        } else {
            n[0] = 0.0;
            n[1] = 0.0;
            n[2] = 1.0;
        }
        xi = (d - b->radius[lo]) - b->radius[hi];
        a1 = b->radius[lo] + xi;
        a2 = b->radius[hi];
        put_contact(out, m++, lo, hi, n, xi, a1, a2);
    }
    if (!is_static(b, i))
        for (int32_t w = 0; w < dom->n_planes; ++w)
            if (sphere_plane(b, &dom->planes[w], h_i, p->tau, i, n, &xi, &a1, &a2))
                put_contact(out, m++, i, b->n + w, n, xi, a1, a2);
    /* partners k < i give keys (k, i), then (i, k > i), then walls: ascending already */
    return m;
}

static void contacts_alloc(ref_contacts *c, int64_t cap);
static void contacts_free(ref_contacts *c);
static int32_t ref_threads;

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* The cell lists of one grid detection. */
typedef struct {
    const ref_bodies *b;
    const ref_domain *dom;
    const ref_params *p;
    const double *h;
    const int64_t *dims, *head, *next, *cidx;
} grid_lists;

/* The contacts of body i found through the cell lists (its partners k > i in
 * ascending index, then its walls), written from position m of out; returns
 * the new count. */
static int64_t grid_body(const grid_lists *g, int64_t i, int64_t **cand_p, int64_t *cand_cap_p, ref_contacts *out,
                         int64_t m)
{
    const ref_bodies *b = g->b;
    const ref_domain *dom = g->dom;
    const ref_params *p = g->p;
    const double *h = g->h;
    const int64_t *dims = g->dims, *head = g->head, *next = g->next, *cidx = g->cidx;
    const int64_t N = b->n;
    int64_t *cand = *cand_p, cand_cap = *cand_cap_p;
    double n[3], xi, a1, a2;
    int64_t nc = 0;
    int64_t lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        if (dims[a] == 1) {
            lo[a] = 0;
            hi[a] = 0;
        } else {
            lo[a] = cidx[3 * i + a] - 1;
            hi[a] = cidx[3 * i + a] + 1;
        }
    }
    for (int64_t cz = lo[2]; cz <= hi[2]; ++cz)
        for (int64_t cy = lo[1]; cy <= hi[1]; ++cy)
            for (int64_t cx = lo[0]; cx <= hi[0]; ++cx) {
                int64_t c3[3] = {cx, cy, cz}, ok = 1;
                for (int a = 0; a < 3; ++a) {
                    if (c3[a] < 0 || c3[a] >= dims[a]) {
                        if (!dom->periodic[a]) ok = 0;
                        else c3[a] = (c3[a] + dims[a]) % dims[a];
                    }
                }
                if (!ok) continue;
                int64_t lin = (c3[2] * dims[1] + c3[1]) * dims[0] + c3[0];
                for (int64_t k = head[lin]; k >= 0; k = next[k]) {
                    if (k <= i) continue;
                    if (nc == cand_cap) {
                        cand_cap *= 2;
                        cand = (int64_t *)realloc(cand, sizeof(int64_t) * (size_t)cand_cap);
                    }
                    cand[nc++] = k;
                }
            }
    *cand_p = cand;
    *cand_cap_p = cand_cap;
    qsort(cand, (size_t)nc, sizeof(int64_t), cmp_i64);
    for (int64_t t = 0; t < nc; ++t) {
        int64_t k = cand[t];
        if (t > 0 && cand[t - 1] == k) continue; /* a periodic axis with one cell lists a body once per image */
        if (is_static(b, i) && is_static(b, k)) continue;
        if (sphere_pair(b, dom, h, i, k, n, &xi, &a1, &a2)) put_contact(out, m++, i, k, n, xi, a1, a2);
    }
    if (is_static(b, i)) return m;
    for (int32_t w = 0; w < dom->n_planes; ++w)
        if (sphere_plane(b, &dom->planes[w], h[i], p->tau, i, n, &xi, &a1, &a2))
            put_contact(out, m++, i, N + w, n, xi, a1, a2);
    return m;
}

/* Same contact set with a uniform cell grid (broad phase by spatial
 * partitioning, Sect. 4) so that larger scenes stay tractable.  Cell edge >=
 * the largest possible reach 2 max(r + h), so every contact partner lies in
 * one of the 27 surrounding cells.  Candidates of body i with k > i are
 * sorted ascending before testing, giving the same order as the brute force.
 * In the OpenMP mode runs of consecutive bodies are searched in parallel,
 * each into a list of its own, and the lists joined in body order. */
int64_t nbgs_ref_detect_grid(const ref_bodies *b, const ref_domain *dom, const ref_params *p, ref_contacts *out)
{
    int64_t N = b->n;
    if (N == 0) return 0;
    double *h = (double *)malloc(sizeof(double) * (size_t)N);
    nbgs_ref_hull_radii(b, p, h);
    double reach = 0.0;
    for (int64_t i = 0; i < N; ++i)
        if (b->radius[i] + h[i] > reach) reach = b->radius[i] + h[i];
    double cell = 2.0 * reach * (1.0 + 1e-9);
    int64_t dims[3];
    double edge[3];
    for (int a = 0; a < 3; ++a) {
        double L = dom->hi[a] - dom->lo[a];
        int64_t c = (int64_t)floor(L / cell);
        if (c < 1) c = 1;
        if (dom->periodic[a] && c < 3) c = 1; /* too few cells for a periodic axis: one cell, all images */
        dims[a] = c;
        edge[a] = dom->periodic[a] ? L / (double)c : cell;
    }
    int64_t ncell = dims[0] * dims[1] * dims[2];
    int64_t *head = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncell);
    int64_t *next = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
    int64_t *cidx = (int64_t *)malloc(sizeof(int64_t) * (size_t)N * 3);
    for (int64_t c = 0; c < ncell; ++c) head[c] = -1;
    for (int64_t i = N - 1; i >= 0; --i) {
        double pos[3] = {b->x[i], b->y[i], b->z[i]};
        int64_t ci[3];
        for (int a = 0; a < 3; ++a) {
            int64_t c = (int64_t)floor((pos[a] - dom->lo[a]) / edge[a]);
            if (c < 0) c = 0;
            if (c > dims[a] - 1) c = dims[a] - 1;
            ci[a] = c;
            cidx[3 * i + a] = c;
        }
        int64_t lin = (ci[2] * dims[1] + ci[1]) * dims[0] + ci[0];
        next[i] = head[lin];
        head[lin] = i;
    }
    const grid_lists g = {b, dom, p, h, dims, head, next, cidx};
    int64_t m = 0;
    if (ref_threads > 1) {
        /* OpenMP mode: contiguous runs of bodies, each into a list of its own,
         * joined in run order: the same contacts in the same order. */
        const int64_t runs = 8 * (int64_t)ref_threads;
        ref_contacts *part = (ref_contacts *)calloc((size_t)runs, sizeof(ref_contacts));
        int64_t *pm = (int64_t *)calloc((size_t)runs, sizeof(int64_t));
        #pragma omp parallel for num_threads(ref_threads) schedule(dynamic, 1)
        for (int64_t r = 0; r < runs; ++r) {
            const int64_t i0 = N * r / runs, i1 = N * (r + 1) / runs;
            int64_t cap = 64, cand_cap = 64, k;
            int64_t *cand = (int64_t *)malloc(sizeof(int64_t) * (size_t)cand_cap);
            for (;;) {
                contacts_alloc(&part[r], cap);
                k = 0;
                for (int64_t i = i0; i < i1; ++i) k = grid_body(&g, i, &cand, &cand_cap, &part[r], k);
                if (k <= cap) break;
                contacts_free(&part[r]);
                cap = 2 * k;
            }
            free(cand);
            pm[r] = k;
        }
        for (int64_t r = 0; r < runs; ++r) {
            const ref_contacts *c = &part[r];
            for (int64_t q = 0; q < pm[r]; ++q, ++m) {
                if (m >= out->cap) continue;
                out->j1[m] = c->j1[q];
                out->j2[m] = c->j2[q];
                out->key[m] = c->key[q];
                out->nx[m] = c->nx[q];
                out->ny[m] = c->ny[q];
                out->nz[m] = c->nz[q];
                out->xi[m] = c->xi[q];
                out->a1[m] = c->a1[q];
                out->a2[m] = c->a2[q];
            }
            contacts_free(&part[r]);
        }
        free(pm);
        free(part);
    } else {
        int64_t cand_cap = 64;
        int64_t *cand = (int64_t *)malloc(sizeof(int64_t) * (size_t)cand_cap);
        for (int64_t i = 0; i < N; ++i) m = grid_body(&g, i, &cand, &cand_cap, out, m);
        free(cand);
    }
    free(cidx);
    free(next);
    free(head);
    free(h);
    return m;
}

/* ------------------------------------------------------------- colouring */

/* splitmix64 finaliser (Steele, Lea, Flood 2014; constants as published by
 * Vigna): a counter-based 64-bit mixing function used for contact priorities. */
uint64_t nbgs_ref_splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static const uint64_t *g_prio;
static const uint64_t *g_key;
static int cmp_priority(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    if (g_prio[x] != g_prio[y]) return g_prio[x] > g_prio[y] ? -1 : 1; /* descending priority */
    return (g_key[x] > g_key[y]) - (g_key[x] < g_key[y]);             /* then ascending key */
}

/* Greedy first-fit colouring of the contact conflict graph, visiting contacts
 * in descending priority pi_j = splitmix64(key_j ^ seed) (ties: ascending
 * key).  Two contacts conflict iff they share a body with inverse mass > 0
 * (and, when sdom is given, lie in the same subdomain); planes (index >=
 * n_bodies) and static spheres never conflict.  Each contact takes the
 * smallest colour not used by an already coloured conflicting contact.
 * Returns the number of colours. */
int32_t nbgs_ref_colour(int64_t n_bodies, const double *inv_mass, int64_t nc, const int32_t *j1, const int32_t *j2,
                        const uint64_t *key, uint64_t seed, const int32_t *sdom, int32_t *colour)
{
    if (nc == 0) return 0;
    /* body -> incident contacts */
    int64_t *deg = (int64_t *)calloc((size_t)n_bodies + 1, sizeof(int64_t));
    for (int64_t j = 0; j < nc; ++j) {
        if (j1[j] < n_bodies && inv_mass[j1[j]] > 0.0) deg[j1[j] + 1]++;
        if (j2[j] < n_bodies && inv_mass[j2[j]] > 0.0) deg[j2[j] + 1]++;
    }
    for (int64_t i = 0; i < n_bodies; ++i) deg[i + 1] += deg[i];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_bodies + 1));
    memcpy(fill, deg, sizeof(int64_t) * (size_t)(n_bodies + 1));
    int64_t *inc = (int64_t *)malloc(sizeof(int64_t) * (size_t)(deg[n_bodies] > 0 ? deg[n_bodies] : 1));
    for (int64_t j = 0; j < nc; ++j) {
        if (j1[j] < n_bodies && inv_mass[j1[j]] > 0.0) inc[fill[j1[j]]++] = j;
        if (j2[j] < n_bodies && inv_mass[j2[j]] > 0.0) inc[fill[j2[j]]++] = j;
    }
    uint64_t *prio = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)nc);
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)nc);
    for (int64_t j = 0; j < nc; ++j) {
        prio[j] = nbgs_ref_splitmix64(key[j] ^ seed);
        order[j] = j;
        colour[j] = -1;
    }
    g_prio = prio;
    g_key = key;
    qsort(order, (size_t)nc, sizeof(int64_t), cmp_priority);
    int32_t ncol = 0;
    size_t used_cap = 64;
    unsigned char *used = (unsigned char *)malloc(used_cap);
    for (int64_t t = 0; t < nc; ++t) {
        int64_t j = order[t];
        memset(used, 0, used_cap);
        int32_t ends[2] = {j1[j], j2[j]};
        for (int e = 0; e < 2; ++e) {
            int64_t body = ends[e];
            if (body >= n_bodies || !(inv_mass[body] > 0.0)) continue;
            for (int64_t q = deg[body]; q < deg[body + 1]; ++q) {
                int32_t c = colour[inc[q]];
                if (c < 0) continue;
                if (sdom && sdom[inc[q]] != sdom[j]) continue;
                if ((size_t)c >= used_cap) {
                    size_t nc2 = used_cap;
                    while ((size_t)c >= nc2) nc2 *= 2;
                    used = (unsigned char *)realloc(used, nc2);
                    memset(used + used_cap, 0, nc2 - used_cap);
                    used_cap = nc2;
                }
                used[c] = 1;
            }
        }
        int32_t c = 0;
        while ((size_t)c < used_cap && used[c]) ++c;
        colour[j] = c;
        if (c + 1 > ncol) ncol = c + 1;
    }
    free(used);
    free(order);
    free(prio);
    free(inc);
    free(fill);
    free(deg);
    return ncol;
}

/* Sweep order: contacts sorted by (colour, key).  The list is in key order
 * already, so a stable grouping by colour suffices. */
void nbgs_ref_sweep_order(int64_t nc, const int32_t *colour, int32_t n_colours, int64_t *order)
{
    int64_t t = 0;
    for (int32_t c = 0; c < n_colours; ++c)
        for (int64_t j = 0; j < nc; ++j)
            if (colour[j] == c) order[t++] = j;
}

/* Subdomains (Alg. 1's s_c(j), the domain partitioning of Sect. 6.1): the
 * box is cut into nb_a = max(1, floor(L_a / edge)) blocks per axis of edge
 * L_a / nb_a, and contact j belongs to the block holding the centre of body
 * j1 (block coordinates clamped into the box).  Block id (c_z nb_y + c_y)
 * nb_x + c_x.  Returns the number of blocks. */
static void block_grid(const ref_domain *dom, double edge, int64_t nb[3], double e[3])
{
    for (int a = 0; a < 3; ++a) {
        double L = dom->hi[a] - dom->lo[a];
        double c = floor(L / edge);
        if (!(c >= 1.0)) c = 1.0;
        nb[a] = (int64_t)c;
        e[a] = L / c;
    }
}

/* Block holding the centre of body i (coordinates clamped into the box). */
static int32_t block_of(const ref_bodies *b, const ref_domain *dom, const int64_t nb[3], const double e[3], int64_t i)
{
    double x[3] = {b->x[i], b->y[i], b->z[i]};
    int64_t c[3];
    for (int a = 0; a < 3; ++a) {
        double f = floor((x[a] - dom->lo[a]) / e[a]);
        f = fmax(0.0, fmin(f, (double)(nb[a] - 1)));
        c[a] = (int64_t)f;
    }
    return (int32_t)((c[2] * nb[1] + c[1]) * nb[0] + c[0]);
}

int32_t nbgs_ref_subdomains(const ref_bodies *b, const ref_domain *dom, double edge, int64_t nc, const int32_t *j1,
                            int32_t *sdom)
{
    int64_t nb[3];
    double e[3];
    block_grid(dom, edge, nb, e);
    for (int64_t j = 0; j < nc; ++j) sdom[j] = block_of(b, dom, nb, e, j1[j]);
    return (int32_t)(nb[0] * nb[1] * nb[2]);
}

/* Block-local sweep order of the plain NBGS (one subdomain in Alg. 1; any
 * order of the contacts is a Gauss-Seidel sweep).  With the blocks of
 * nbgs_ref_subdomains, a contact whose dynamic bodies all lie in one block
 * is local to that block and gets its id; a contact between dynamic bodies of
 * two different blocks gets the id nblocks.  Sorting by (id, colour, key),
 * the colouring restricted to equal ids, sweeps every block's local contacts
 * (blocks share no dynamic body through them) and then the others.  Returns
 * nblocks + 1, the number of ids. */
int32_t nbgs_ref_block_local(const ref_bodies *b, const ref_domain *dom, double edge, int64_t nc, const int32_t *j1,
                             const int32_t *j2, int32_t *id)
{
    int64_t nb[3];
    double e[3];
    block_grid(dom, edge, nb, e);
    int32_t nblocks = (int32_t)(nb[0] * nb[1] * nb[2]);
    int64_t N = b->n;
    for (int64_t j = 0; j < nc; ++j) {
        int d1 = b->inv_mass[j1[j]] > 0.0;
        int d2 = j2[j] < N && b->inv_mass[j2[j]] > 0.0;
        if (d1 && d2) {
            int32_t k1 = block_of(b, dom, nb, e, j1[j]), k2 = block_of(b, dom, nb, e, j2[j]);
            id[j] = k1 == k2 ? k1 : nblocks;
        } else {
            id[j] = block_of(b, dom, nb, e, d1 ? j1[j] : j2[j]);
        }
    }
    return nblocks + 1;
}

/* Block of body i in grid g of `grids` grids shifted by g/grids of a block
 * edge along every axis: c_a = floor((x_a - lo_a) / e_a + g / grids), taken
 * modulo nb_a along a periodic axis (the block across the boundary is one
 * block) and clamped along another one, to [0, nb_a - 1] in grid 0 (as
 * block_of) and to [0, nb_a] in a shifted grid (whose last block reaches past
 * the box).  Block id (c_z M_y + c_y) M_x + c_x with M_a = nb_a, plus one
 * along a non-periodic axis when there are several grids. */
static int64_t block_in_grid(const ref_bodies *b, const ref_domain *dom, const int64_t nb[3], const double e[3],
                             const int64_t M[3], int g, int grids, int64_t i)
{
    double x[3] = {b->x[i], b->y[i], b->z[i]};
    int64_t c[3];
    for (int a = 0; a < 3; ++a) {
        double f = floor((x[a] - dom->lo[a]) / e[a] + (double)g / (double)grids);
        if (dom->periodic[a]) {
            int64_t q = (int64_t)f % nb[a];
            c[a] = q < 0 ? q + nb[a] : q;
        } else {
            double top = g == 0 ? (double)(nb[a] - 1) : (double)nb[a];
            c[a] = (int64_t)fmax(0.0, fmin(f, top));
        }
    }
    return (c[2] * M[1] + c[1]) * M[0] + c[0];
}

/* Block-local order over several shifted block grids (the same plain NBGS,
 * visited in another order).  Grid g (g = 0 .. grids - 1) cuts the box as
 * nbgs_ref_block_local does, shifted by g/grids of a block edge along every
 * axis.  A contact is local to grid g if all its dynamic bodies lie in one
 * block of that grid; it takes the id g B + block for the first such grid
 * (B blocks per grid), or the id grids B if it is local to none.  Sorted by
 * (id, colour, key) with the colouring restricted to equal ids, a sweep takes
 * grid 0's blocks, then grid 1's, ..., then the remaining contacts; the local
 * contacts of two blocks of one grid share no dynamic body.  A contact whose
 * centres differ by less than a quarter of the block edge along every axis is
 * local to one of four grids (along each axis the faces of the four grids are a
 * quarter edge apart, so at most one grid has a face between the centres).
 * grids = 1 is nbgs_ref_block_local.  Returns grids B + 1, the number of ids. */
int32_t nbgs_ref_block_local_grids(const ref_bodies *b, const ref_domain *dom, double edge, int32_t grids,
                                   int64_t nc, const int32_t *j1, const int32_t *j2, int32_t *id)
{
    if (grids <= 1) return nbgs_ref_block_local(b, dom, edge, nc, j1, j2, id);
    int64_t nb[3], M[3];
    double e[3];
    block_grid(dom, edge, nb, e);
    for (int a = 0; a < 3; ++a) M[a] = nb[a] + (dom->periodic[a] ? 0 : 1);
    int64_t B = M[0] * M[1] * M[2];
    int64_t N = b->n;
    for (int64_t j = 0; j < nc; ++j) {
        int d1 = b->inv_mass[j1[j]] > 0.0;
        int d2 = j2[j] < N && b->inv_mass[j2[j]] > 0.0;
        int64_t out = (int64_t)grids * B;
        for (int g = 0; g < grids; ++g) {
            int64_t k1 = block_in_grid(b, dom, nb, e, M, g, grids, d1 ? j1[j] : j2[j]);
            int64_t k2 = d1 && d2 ? block_in_grid(b, dom, nb, e, M, g, grids, j2[j]) : k1;
            if (k1 == k2) {
                out = (int64_t)g * B + k1;
                break;
            }
        }
        id[j] = (int32_t)out;
    }
    return (int32_t)((int64_t)grids * B + 1);
}

/* Sweep order of the subdomain solver: contacts sorted by (subdomain, colour,
 * key); the list is in key order, so a stable grouping suffices. */
void nbgs_ref_sweep_order_sub(int64_t nc, const int32_t *sdom, int32_t n_sub, const int32_t *colour, int32_t n_colours,
                              int64_t *order)
{
    int64_t nbin = (int64_t)n_sub * (n_colours > 0 ? n_colours : 1);
    int64_t *start = (int64_t *)calloc((size_t)nbin + 1, sizeof(int64_t));
    for (int64_t j = 0; j < nc; ++j) start[(int64_t)sdom[j] * n_colours + colour[j] + 1]++;
    for (int64_t q = 0; q < nbin; ++q) start[q + 1] += start[q];
    for (int64_t j = 0; j < nc; ++j) order[start[(int64_t)sdom[j] * n_colours + colour[j]]++] = j;
    free(start);
}

/* ----------------------------------------------------------- warm start */

/* Project a world-frame impulse P onto the contact's friction cone around n:
 * normal part clamped at zero (non-adhesion), tangential part scaled down to
 * mu times the normal part (eq. (coulomb), first condition). */
static void cone_project(const double *n, double mu, double *P)
{
    double pn = n[0] * P[0] + n[1] * P[1] + n[2] * P[2];
    double t0 = P[0] - pn * n[0], t1 = P[1] - pn * n[1], t2 = P[2] - pn * n[2];
    if (pn < 0.0) pn = 0.0;
    double tl = sqrt(t0 * t0 + t1 * t1 + t2 * t2);
    double lim = mu * pn;
    if (tl > lim) {
        double s = tl > 0.0 ? lim / tl : 0.0;
        t0 = t0 * s;
        t1 = t1 * s;
        t2 = t2 * s;
    }
    P[0] = pn * n[0] + t0;
    P[1] = pn * n[1] + t1;
    P[2] = pn * n[2] + t2;
}

/* Initial impulses from the previous time step (Sect. 5 allows the previous
 * step's reactions as initial solution): each contact looks up its pair key in
 * the previous step's (key-sorted) table, re-projects that world impulse onto
 * its new normal and friction cone, and starts at zero if the pair is new. */
void nbgs_ref_warm_match(int64_t nc, const uint64_t *key, const double *nx, const double *ny, const double *nz,
                         double mu, int64_t n_prev, const uint64_t *prev_key, const double *prev_px,
                         const double *prev_py, const double *prev_pz, double *px, double *py, double *pz)
{
    for (int64_t j = 0; j < nc; ++j) {
        int64_t lo = 0, hi = n_prev; /* first index with prev_key >= key */
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            if (prev_key[mid] < key[j]) lo = mid + 1;
            else hi = mid;
        }
        if (lo < n_prev && prev_key[lo] == key[j]) {
            double P[3] = {prev_px[lo], prev_py[lo], prev_pz[lo]};
            double n[3] = {nx[j], ny[j], nz[j]};
            cone_project(n, mu, P);
            px[j] = P[0];
            py[j] = P[1];
            pz[j] = P[2];
        } else {
            px[j] = 0.0;
            py[j] = 0.0;
            pz[j] = 0.0;
        }
    }
}

/* ----------------------------------------------------------------- solve */

/* Apply impulse dP at contact j (acting +dP on j1 and -dP on j2 at the
 * contact point, eq. (wrench)) to the velocity accumulators.  With
 * r1 = x_hat - x_j1 = -a1 n and r2 = x_hat - x_j2 = a2 n:
 *   v1 += m1^-1 dP,  w1 += I1^-1 (r1 x dP) = -I1^-1 a1 (n x dP),
 *   v2 -= m2^-1 dP,  w2 -= I2^-1 (r2 x dP) = -I2^-1 a2 (n x dP). */
static void apply_impulse(int64_t N, const double *im, const double *ii, double *v, double *w, int32_t b1,
                          int32_t b2, const double *n, double a1, double a2, const double *dP)
{
    double m0 = n[1] * dP[2] - n[2] * dP[1];
    double m1 = n[2] * dP[0] - n[0] * dP[2];
    double m2 = n[0] * dP[1] - n[1] * dP[0];
    if (im[b1] > 0.0) {
        v[3 * b1 + 0] = v[3 * b1 + 0] + im[b1] * dP[0];
        v[3 * b1 + 1] = v[3 * b1 + 1] + im[b1] * dP[1];
        v[3 * b1 + 2] = v[3 * b1 + 2] + im[b1] * dP[2];
        w[3 * b1 + 0] = w[3 * b1 + 0] - ii[b1] * a1 * m0;
        w[3 * b1 + 1] = w[3 * b1 + 1] - ii[b1] * a1 * m1;
        w[3 * b1 + 2] = w[3 * b1 + 2] - ii[b1] * a1 * m2;
    }
    if (b2 < N && im[b2] > 0.0) {
        v[3 * b2 + 0] = v[3 * b2 + 0] - im[b2] * dP[0];
        v[3 * b2 + 1] = v[3 * b2 + 1] - im[b2] * dP[1];
        v[3 * b2 + 2] = v[3 * b2 + 2] - im[b2] * dP[2];
        w[3 * b2 + 0] = w[3 * b2 + 0] - ii[b2] * a2 * m0;
        w[3 * b2 + 1] = w[3 * b2 + 1] - ii[b2] * a2 * m1;
        w[3 * b2 + 2] = w[3 * b2 + 2] - ii[b2] * a2 * m2;
    }
}

/* The one-contact problem F_j(P) = 0 of Sect. 3 for two spheres.  In the
 * contact frame the post-step relative velocity is u = b + W P with the
 * diagonal Delassus block W = diag(w_n, w_t, w_t),
 *   w_n = 1/m1 + 1/m2,  w_t = w_n + a1^2/I1 + a2^2/I2,
 * and b the relative velocity (plus the xi/dt term) without this contact's
 * impulse.  Because W is diagonal the problem decouples:
 *   normal:  u_n >= 0 complementary to P_n >= 0  =>  P_n = max(0, -b_n / w_n);
 *   friction: stick P_t = -b_t / w_t if |P_t| <= mu P_n, otherwise slide with
 *            P_t = -mu P_n b_t / |b_t|, which is the stick value scaled onto
 *            the cone; then u_t is parallel to b_t and P_t opposes it, as
 *            eq. (coulomb) demands. */
static void one_contact(double bn, const double *bt, double wn, double wt, double mu, const double *n, double *P)
{
    double pn = -bn / wn;
    if (!(pn > 0.0)) pn = 0.0;
    double t0 = -bt[0] / wt, t1 = -bt[1] / wt, t2 = -bt[2] / wt;
    double tl = sqrt(t0 * t0 + t1 * t1 + t2 * t2);
    double lim = mu * pn;
    if (tl > lim) {
        double s = lim / tl;
        t0 = t0 * s;
        t1 = t1 * s;
        t2 = t2 * s;
    }
    P[0] = pn * n[0] + t0;
    P[1] = pn * n[1] + t1;
    P[2] = pn * n[2] + t2;
}

/* The arrays one sweep reads and writes. */
typedef struct {
    int64_t N;
    const double *im, *ii;
    const ref_params *p;
    const int32_t *j1, *j2;
    const double *nx, *ny, *nz, *xi, *a1, *a2;
    double *px, *py, *pz, *v, *w;
} sweep_arrays;

/* The one-contact solution P* = F_j^-1(0, P_jbar) of contact j against the
 * accumulators as they stand (its own impulse P_j taken out of them); P
 * receives the contact's current impulse P_j. */
static void contact_target(const sweep_arrays *s, int64_t j, double *P, double *Ps)
{
    const int64_t N = s->N;
    const double *im = s->im, *ii = s->ii, *v = s->v, *w = s->w;
    const ref_params *p = s->p;
    int32_t b1 = s->j1[j], b2 = s->j2[j];
    double n[3] = {s->nx[j], s->ny[j], s->nz[j]};
    double im1 = im[b1], ii1 = ii[b1];
    double im2 = 0.0, ii2 = 0.0;
    double v2[3] = {0.0, 0.0, 0.0}, w2[3] = {0.0, 0.0, 0.0};
    if (b2 < N) {
        im2 = im[b2];
        ii2 = ii[b2];
        for (int a = 0; a < 3; ++a) {
            v2[a] = v[3 * b2 + a];
            w2[a] = w[3 * b2 + a];
        }
    }
    double s0 = s->a1[j] * w[3 * b1 + 0] + s->a2[j] * w2[0];
    double s1 = s->a1[j] * w[3 * b1 + 1] + s->a2[j] * w2[1];
    double s2 = s->a1[j] * w[3 * b1 + 2] + s->a2[j] * w2[2];
    double du[3];
    du[0] = (v[3 * b1 + 0] - v2[0]) - (s1 * n[2] - s2 * n[1]);
    du[1] = (v[3 * b1 + 1] - v2[1]) - (s2 * n[0] - s0 * n[2]);
    du[2] = (v[3 * b1 + 2] - v2[2]) - (s0 * n[1] - s1 * n[0]);
    double dun = n[0] * du[0] + n[1] * du[1] + n[2] * du[2];
    double corr = s->xi[j] < 0.0 ? p->erp * s->xi[j] : s->xi[j];
    double un = corr / p->dt + dun;
    double ut[3] = {du[0] - dun * n[0], du[1] - dun * n[1], du[2] - dun * n[2]};
    P[0] = s->px[j];
    P[1] = s->py[j];
    P[2] = s->pz[j];
    double Pn = n[0] * P[0] + n[1] * P[1] + n[2] * P[2];
    double Pt[3] = {P[0] - Pn * n[0], P[1] - Pn * n[1], P[2] - Pn * n[2]};
    double wn = im1 + im2;
    double wt = wn + ii1 * s->a1[j] * s->a1[j] + ii2 * s->a2[j] * s->a2[j];
    double bn = un - wn * Pn;
    double bt[3] = {ut[0] - wt * Pt[0], ut[1] - wt * Pt[1], ut[2] - wt * Pt[2]};
    one_contact(bn, bt, wn, wt, p->mu, n, Ps);
}

/* One relaxation of contact j (the loop body of a sweep below); *dp2 = |dP|^2
 * and *p2 = |P_new|^2 for the residual. */
static void relax_one(const sweep_arrays *s, int64_t j, double *dp2, double *p2)
{
    const ref_params *p = s->p;
    double n[3] = {s->nx[j], s->ny[j], s->nz[j]};
    double P[3], Ps[3];
    contact_target(s, j, P, Ps);
    double Pnew[3], dP[3];
    for (int a = 0; a < 3; ++a) {
        Pnew[a] = p->relax * Ps[a] + (1.0 - p->relax) * P[a];
        dP[a] = Pnew[a] - P[a];
    }
    apply_impulse(s->N, s->im, s->ii, s->v, s->w, s->j1[j], s->j2[j], n, s->a1[j], s->a2[j], dP);
    s->px[j] = Pnew[0];
    s->py[j] = Pnew[1];
    s->pz[j] = Pnew[2];
    *dp2 = dP[0] * dP[0] + dP[1] * dP[1] + dP[2] * dP[2];
    *p2 = Pnew[0] * Pnew[0] + Pnew[1] * Pnew[1] + Pnew[2] * Pnew[2];
}

/* The initial impulse of contact j applied to its bodies (nothing when zero). */
static void apply_initial(const sweep_arrays *s, int64_t j)
{
    double n[3] = {s->nx[j], s->ny[j], s->nz[j]};
    double P0[3] = {s->px[j], s->py[j], s->pz[j]};
    if (P0[0] != 0.0 || P0[1] != 0.0 || P0[2] != 0.0)
        apply_impulse(s->N, s->im, s->ii, s->v, s->w, s->j1[j], s->j2[j], n, s->a1[j], s->a2[j], P0);
}

/* Threads of the OpenMP mode (1: the plain sequential loops). */
static int32_t ref_threads = 1;

void nbgs_ref_set_threads(int32_t threads) { ref_threads = threads > 1 ? threads : 1; }

int32_t nbgs_ref_get_threads(void) { return ref_threads; }

/* Dependency levels of a sweep order (the OpenMP mode).  Position t of the
 * order waits for the last earlier position that shares one of its dynamic
 * bodies (a wall or a static body is never written, so it links nothing):
 *   level(t) = 1 + the largest level among those positions, 1 without any.
 * Two positions of one level share no dynamic body, and each body meets its
 * contacts level by level in the order's sequence; so running the levels one
 * after another, each in any order or in parallel, gives every body the same
 * impulses in the same sequence as the sequential loop: the same result to the
 * last bit.  lev_pos (nc entries) receives the positions grouped by level,
 * ascending inside a level; *lev_start (levels + 1 entries, allocated here and
 * freed by the caller) where level l (0-based) starts.  Returns the number of
 * levels. */
int64_t nbgs_ref_order_levels(int64_t N, const double *inv_mass, int64_t nc, const int32_t *j1, const int32_t *j2,
                              const int64_t *order, int64_t *lev_pos, int64_t **lev_start)
{
    int64_t *last = (int64_t *)calloc((size_t)(N > 0 ? N : 1), sizeof(int64_t));
    int64_t *lev = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nc > 0 ? nc : 1));
    int64_t L = 0;
    for (int64_t t = 0; t < nc; ++t) {
        int64_t j = order[t];
        int32_t b1 = j1[j], b2 = j2[j];
        int d1 = inv_mass[b1] > 0.0, d2 = b2 < N && inv_mass[b2] > 0.0;
        int64_t l = 0;
        if (d1 && last[b1] > l) l = last[b1];
        if (d2 && last[b2] > l) l = last[b2];
        l += 1;
        if (d1) last[b1] = l;
        if (d2) last[b2] = l;
        lev[t] = l - 1;
        if (l > L) L = l;
    }
    int64_t *start = (int64_t *)calloc((size_t)L + 1, sizeof(int64_t));
    for (int64_t t = 0; t < nc; ++t) start[lev[t] + 1] += 1;
    for (int64_t l = 0; l < L; ++l) start[l + 1] += start[l];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(L > 0 ? L : 1));
    memcpy(fill, start, sizeof(int64_t) * (size_t)L);
    for (int64_t t = 0; t < nc; ++t) lev_pos[fill[lev[t]]++] = t;
    free(fill);
    free(lev);
    free(last);
    *lev_start = start;
    return L;
}

/* NBGS solve of one time step.
 *
 * Accumulators (Sect. 6.3, velocity form; the paper's experiments use it):
 *   v' = v + dt g (dynamic bodies), w' = w  (spheres: w x I w = 0), then the
 *   initial impulses P (warm start, or zero) are applied contact by contact in
 *   sweep order.
 * Sweep k (Alg. 1 with a single subdomain: every contact sees the newest
 * impulses of all contacts relaxed before it):
 *   for each contact j in sweep order:
 *     du   = v'_1 - v'_2 - (a1 w'_1 + a2 w'_2) x n       (relative velocity, Sect. 3)
 *     u_n  = xi'/dt + n.du,   u_t = du - (n.du) n         (eq. (nonpenetration); xi' = erp xi if xi < 0)
 *     b    = u - W P_j                                    (the contact's own impulse taken out)
 *     P*   = one_contact(b)                               (F_j^-1(0, P_jbar))
 *     P_new = omega P* + (1 - omega) P_j                  (Alg. 1, relaxation)
 *     apply dP = P_new - P_j to both bodies, P_j = P_new
 *   residual R_k = |dP|_2 / |P_new|_2 over all contacts of the sweep
 *   stop when R_k <= target (target > 0) or k = max_sweeps.
 *
 * order[t] is the t-th contact of the sweep; P arrays are in contact order,
 * in/out.  v_out, w_out (3 n each, interleaved xyz) receive v', w'.
 * residual_hist (max_sweeps entries, may be NULL) receives R_k.
 *
 * With more than one thread (nbgs_ref_set_threads) the initial impulses and
 * every sweep run level by level (nbgs_ref_order_levels), the contacts of a
 * level in parallel; the per-contact residual terms are kept by position and
 * summed in the order's sequence, so every output is the sequential one. */
void nbgs_ref_solve(const ref_bodies *b, const ref_params *p, int64_t nc, const int32_t *j1, const int32_t *j2,
                    const double *nx, const double *ny, const double *nz, const double *xi, const double *a1,
                    const double *a2, const int64_t *order, double *px, double *py, double *pz, int32_t max_sweeps,
                    double target, double *v_out, double *w_out, double *residual_hist, ref_solve_stats *stats)
{
    int64_t N = b->n;
    const double *im = b->inv_mass, *ii = b->inv_inertia;
    double *v = v_out, *w = w_out;
    for (int64_t i = 0; i < N; ++i) {
        int dyn = im[i] > 0.0;
        v[3 * i + 0] = dyn ? b->vx[i] + p->dt * p->gravity[0] : b->vx[i];
        v[3 * i + 1] = dyn ? b->vy[i] + p->dt * p->gravity[1] : b->vy[i];
        v[3 * i + 2] = dyn ? b->vz[i] + p->dt * p->gravity[2] : b->vz[i];
        w[3 * i + 0] = b->wx[i];
        w[3 * i + 1] = b->wy[i];
        w[3 * i + 2] = b->wz[i];
    }
    const sweep_arrays s = {N, im, ii, p, j1, j2, nx, ny, nz, xi, a1, a2, px, py, pz, v, w};
    const int par = ref_threads > 1 && nc > 0;
    int64_t L = 0, *lev_pos = NULL, *lev_start = NULL;
    double *term_dp = NULL, *term_p = NULL;
    if (par) {
        lev_pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)nc);
        L = nbgs_ref_order_levels(N, im, nc, j1, j2, order, lev_pos, &lev_start);
        term_dp = (double *)malloc(sizeof(double) * (size_t)nc);
        term_p = (double *)malloc(sizeof(double) * (size_t)nc);
        #pragma omp parallel num_threads(ref_threads)
        for (int64_t l = 0; l < L; ++l) {
            #pragma omp for schedule(static)
            for (int64_t q = lev_start[l]; q < lev_start[l + 1]; ++q) apply_initial(&s, order[lev_pos[q]]);
        }
    } else {
        for (int64_t t = 0; t < nc; ++t) apply_initial(&s, order[t]);
    }
    int32_t k = 0;
    double R = 0.0;
    while (k < max_sweeps) {
        double sum_dp = 0.0, sum_p = 0.0;
        if (par) {
            #pragma omp parallel num_threads(ref_threads)
            for (int64_t l = 0; l < L; ++l) {
                #pragma omp for schedule(static)
                for (int64_t q = lev_start[l]; q < lev_start[l + 1]; ++q) {
                    int64_t t = lev_pos[q];
                    relax_one(&s, order[t], &term_dp[t], &term_p[t]);
                }
            }
            for (int64_t t = 0; t < nc; ++t) {
                sum_dp += term_dp[t];
                sum_p += term_p[t];
            }
        } else {
            for (int64_t t = 0; t < nc; ++t) {
                double dp2, p2;
                relax_one(&s, order[t], &dp2, &p2);
                sum_dp += dp2;
                sum_p += p2;
            }
        }
        double den = sqrt(sum_p);
        R = sqrt(sum_dp) / (den > 1e-300 ? den : 1e-300);
        if (residual_hist) residual_hist[k] = R;
        ++k;
        if (target > 0.0 && R <= target) break;
    }
    free(lev_pos);
    free(lev_start);
    free(term_dp);
    free(term_p);
    if (stats) {
        stats->sweeps = k;
        stats->residual = R;
    }
}

/* Jacobi residual of an initial impulse (the judge of a learned warm start,
 * Sect. 5: any initial solution may start Alg. 1, so two candidates are
 * compared by how far each is from its own one-contact solutions).
 *
 * Definition: from the accumulators of the initial impulses P0 (v' = v + dt g
 * for dynamic bodies, w' = w, then every contact's P0 applied in sweep
 * order, exactly as a solve starts), every contact takes its one-contact
 * solution P*_j with its own impulse taken out, all against the same
 * accumulators and nothing written back (one nonlinear Jacobi step); then
 *   R_J = |P* - P0|_2 / max(|P*|_2, 1e-300)
 * over all contacts, the squares summed in sweep order.  P* of every contact
 * (contact order) is written to ps_x/ps_y/ps_z when they are not NULL; v_out
 * and w_out (3 n each, may be NULL) receive the accumulators.  Returns R_J
 * (0 when there is no contact). */
double nbgs_ref_jacobi_residual(const ref_bodies *b, const ref_params *p, int64_t nc, const int32_t *j1,
                                const int32_t *j2, const double *nx, const double *ny, const double *nz,
                                const double *xi, const double *a1, const double *a2, const int64_t *order,
                                const double *px, const double *py, const double *pz, double *ps_x, double *ps_y,
                                double *ps_z, double *v_out, double *w_out)
{
    int64_t N = b->n;
    const double *im = b->inv_mass;
    double *v = (double *)malloc(sizeof(double) * 3 * (size_t)(N > 0 ? N : 1));
    double *w = (double *)malloc(sizeof(double) * 3 * (size_t)(N > 0 ? N : 1));
    for (int64_t i = 0; i < N; ++i) {
        int dyn = im[i] > 0.0;
        v[3 * i + 0] = dyn ? b->vx[i] + p->dt * p->gravity[0] : b->vx[i];
        v[3 * i + 1] = dyn ? b->vy[i] + p->dt * p->gravity[1] : b->vy[i];
        v[3 * i + 2] = dyn ? b->vz[i] + p->dt * p->gravity[2] : b->vz[i];
        w[3 * i + 0] = b->wx[i];
        w[3 * i + 1] = b->wy[i];
        w[3 * i + 2] = b->wz[i];
    }
    /* the sweep arrays read the initial impulses only (nothing is relaxed) */
    const sweep_arrays s = {N, im, b->inv_inertia, p, j1, j2, nx, ny, nz, xi, a1, a2,
                            (double *)px, (double *)py, (double *)pz, v, w};
    for (int64_t t = 0; t < nc; ++t) apply_initial(&s, order[t]);
    double sum_d = 0.0, sum_s = 0.0;
    for (int64_t t = 0; t < nc; ++t) {
        int64_t j = order[t];
        double P[3], Ps[3];
        contact_target(&s, j, P, Ps);
        double d0 = Ps[0] - P[0], d1 = Ps[1] - P[1], d2 = Ps[2] - P[2];
        sum_d += d0 * d0 + d1 * d1 + d2 * d2;
        sum_s += Ps[0] * Ps[0] + Ps[1] * Ps[1] + Ps[2] * Ps[2];
        if (ps_x) {
            ps_x[j] = Ps[0];
            ps_y[j] = Ps[1];
            ps_z[j] = Ps[2];
        }
    }
    if (v_out) memcpy(v_out, v, sizeof(double) * 3 * (size_t)N);
    if (w_out) memcpy(w_out, w, sizeof(double) * 3 * (size_t)N);
    free(v);
    free(w);
    double den = sqrt(sum_s);
    return nc > 0 ? sqrt(sum_d) / (den > 1e-300 ? den : 1e-300) : 0.0;
}

/* Velocities of body i as a contact of subdomain s sees them: accumulator
 * plus the subdomain's correction (Sect. 6.3); zero for a wall. */
static void seen_velocity(int64_t N, const double *V, const double *Wv, const double *dv, const double *dw, int64_t i,
                          double *v, double *w)
{
    for (int a = 0; a < 3; ++a) {
        v[a] = i < N ? V[3 * i + a] + dv[3 * i + a] : 0.0;
        w[a] = i < N ? Wv[3 * i + a] + dw[3 * i + a] : 0.0;
    }
}

/* One pass over all subdomains.  mode 0 applies the initial impulses, mode 1
 * relaxes every contact (Alg. 1).  Within subdomain s the contacts are taken
 * in sweep order and see the accumulators V, W of the last iteration plus the
 * corrections dv, dw of the contacts of s relaxed before them; afterwards the
 * corrections are added to the next accumulators Vn, Wn, subdomain by
 * subdomain in ascending order. */
static void sub_pass(int mode, const ref_bodies *b, const ref_params *p, int64_t nc, const int32_t *j1,
                     const int32_t *j2, const double *nx, const double *ny, const double *nz, const double *xi,
                     const double *a1, const double *a2, const int64_t *order, const int32_t *sdom, double *px,
                     double *py, double *pz, double *V, double *Wv, double *Vn, double *Wn, double *dv, double *dw,
                     int64_t *stamp, int64_t *touched, double *sum_dp, double *sum_p)
{
    int64_t N = b->n;
    const double *im = b->inv_mass, *ii = b->inv_inertia;
    memcpy(Vn, V, sizeof(double) * 3 * (size_t)N);
    memcpy(Wn, Wv, sizeof(double) * 3 * (size_t)N);
    *sum_dp = 0.0;
    *sum_p = 0.0;
    int64_t t = 0;
    while (t < nc) {
        int32_t s = sdom[order[t]];
        int64_t u = t;
        while (u < nc && sdom[order[u]] == s) ++u;
        /* corrections of subdomain s start at zero */
        int64_t nt = 0;
        for (int64_t q = t; q < u; ++q) {
            int64_t j = order[q];
            int64_t ends[2] = {j1[j], j2[j]};
            for (int e = 0; e < 2; ++e) {
                int64_t i = ends[e];
                if (i >= N || !(im[i] > 0.0) || stamp[i] == (int64_t)s + 1) continue;
                stamp[i] = (int64_t)s + 1;
                touched[nt++] = i;
                for (int a = 0; a < 3; ++a) {
                    dv[3 * i + a] = 0.0;
                    dw[3 * i + a] = 0.0;
                }
            }
        }
        for (int64_t q = t; q < u; ++q) {
            int64_t j = order[q];
            int32_t b1 = j1[j], b2 = j2[j];
            double n[3] = {nx[j], ny[j], nz[j]};
            double P[3] = {px[j], py[j], pz[j]};
            if (mode == 0) {
                if (P[0] != 0.0 || P[1] != 0.0 || P[2] != 0.0) apply_impulse(N, im, ii, dv, dw, b1, b2, n, a1[j], a2[j], P);
                continue;
            }
            double v1[3], w1[3], v2[3], w2[3];
            seen_velocity(N, V, Wv, dv, dw, b1, v1, w1);
            seen_velocity(N, V, Wv, dv, dw, b2, v2, w2);
            double im1 = im[b1], ii1 = ii[b1];
            double im2 = b2 < N ? im[b2] : 0.0, ii2 = b2 < N ? ii[b2] : 0.0;
            double s0 = a1[j] * w1[0] + a2[j] * w2[0];
            double s1 = a1[j] * w1[1] + a2[j] * w2[1];
            double s2 = a1[j] * w1[2] + a2[j] * w2[2];
            double du[3];
            du[0] = (v1[0] - v2[0]) - (s1 * n[2] - s2 * n[1]);
            du[1] = (v1[1] - v2[1]) - (s2 * n[0] - s0 * n[2]);
            du[2] = (v1[2] - v2[2]) - (s0 * n[1] - s1 * n[0]);
            double dun = n[0] * du[0] + n[1] * du[1] + n[2] * du[2];
            double corr = xi[j] < 0.0 ? p->erp * xi[j] : xi[j];
            double un = corr / p->dt + dun;
            double ut[3] = {du[0] - dun * n[0], du[1] - dun * n[1], du[2] - dun * n[2]};
            double Pn = n[0] * P[0] + n[1] * P[1] + n[2] * P[2];
            double Pt[3] = {P[0] - Pn * n[0], P[1] - Pn * n[1], P[2] - Pn * n[2]};
            double wn = im1 + im2;
            double wt = wn + ii1 * a1[j] * a1[j] + ii2 * a2[j] * a2[j];
            double bn = un - wn * Pn;
            double bt[3] = {ut[0] - wt * Pt[0], ut[1] - wt * Pt[1], ut[2] - wt * Pt[2]};
            double Ps[3];
            one_contact(bn, bt, wn, wt, p->mu, n, Ps);
            double Pnew[3], dP[3];
            for (int a = 0; a < 3; ++a) {
                Pnew[a] = p->relax * Ps[a] + (1.0 - p->relax) * P[a];
                dP[a] = Pnew[a] - P[a];
            }
            apply_impulse(N, im, ii, dv, dw, b1, b2, n, a1[j], a2[j], dP);
            px[j] = Pnew[0];
            py[j] = Pnew[1];
            pz[j] = Pnew[2];
            *sum_dp += dP[0] * dP[0] + dP[1] * dP[1] + dP[2] * dP[2];
            *sum_p += Pnew[0] * Pnew[0] + Pnew[1] * Pnew[1] + Pnew[2] * Pnew[2];
        }
        for (int64_t k = 0; k < nt; ++k) {
            int64_t i = touched[k];
            for (int a = 0; a < 3; ++a) {
                Vn[3 * i + a] = Vn[3 * i + a] + dv[3 * i + a];
                Wn[3 * i + a] = Wn[3 * i + a] + dw[3 * i + a];
            }
        }
        t = u;
    }
    memcpy(V, Vn, sizeof(double) * 3 * (size_t)N);
    memcpy(Wv, Wn, sizeof(double) * 3 * (size_t)N);
}

/* Subdomain NBGS of one time step (Alg. 1 with the subdomain affinity sdom),
 * in the velocity form of Sect. 6.3.  Contact j of subdomain s sees the
 * newest impulses of the contacts of s relaxed before it and the last
 * iteration's impulses of every other contact: its bodies' velocities are the
 * accumulators of the last iteration plus the corrections made by s in this
 * iteration.  At the end of an iteration the corrections of all subdomains
 * are added to the accumulators.  The initial impulses enter the same way, as
 * the corrections of a first pass.  order lists the contacts grouped by
 * ascending subdomain (sweep order inside each).  Arguments as
 * nbgs_ref_solve. */
void nbgs_ref_solve_sub(const ref_bodies *b, const ref_params *p, int64_t nc, const int32_t *j1, const int32_t *j2,
                        const double *nx, const double *ny, const double *nz, const double *xi, const double *a1,
                        const double *a2, const int64_t *order, const int32_t *sdom, double *px, double *py,
                        double *pz, int32_t max_sweeps, double target, double *v_out, double *w_out,
                        double *residual_hist, ref_solve_stats *stats)
{
    int64_t N = b->n;
    size_t n3 = 3 * (size_t)(N > 0 ? N : 1);
    const double *im = b->inv_mass;
    double *V = v_out, *Wv = w_out;
    for (int64_t i = 0; i < N; ++i) {
        int dyn = im[i] > 0.0;
        V[3 * i + 0] = dyn ? b->vx[i] + p->dt * p->gravity[0] : b->vx[i];
        V[3 * i + 1] = dyn ? b->vy[i] + p->dt * p->gravity[1] : b->vy[i];
        V[3 * i + 2] = dyn ? b->vz[i] + p->dt * p->gravity[2] : b->vz[i];
        Wv[3 * i + 0] = b->wx[i];
        Wv[3 * i + 1] = b->wy[i];
        Wv[3 * i + 2] = b->wz[i];
    }
    double *Vn = (double *)malloc(sizeof(double) * n3), *Wn = (double *)malloc(sizeof(double) * n3);
    double *dv = (double *)calloc(n3, sizeof(double)), *dw = (double *)calloc(n3, sizeof(double));
    int64_t *stamp = (int64_t *)calloc((size_t)(N > 0 ? N : 1), sizeof(int64_t));
    int64_t *touched = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
    double sdp, sp;
    sub_pass(0, b, p, nc, j1, j2, nx, ny, nz, xi, a1, a2, order, sdom, px, py, pz, V, Wv, Vn, Wn, dv, dw, stamp,
             touched, &sdp, &sp);
    int32_t k = 0;
    double R = 0.0;
    while (k < max_sweeps) {
        for (int64_t i = 0; i < N; ++i) stamp[i] = 0;
        sub_pass(1, b, p, nc, j1, j2, nx, ny, nz, xi, a1, a2, order, sdom, px, py, pz, V, Wv, Vn, Wn, dv, dw, stamp,
                 touched, &sdp, &sp);
        double den = sqrt(sp);
        R = sqrt(sdp) / (den > 1e-300 ? den : 1e-300);
        if (residual_hist) residual_hist[k] = R;
        ++k;
        if (target > 0.0 && R <= target) break;
    }
    free(Vn);
    free(Wn);
    free(dv);
    free(dw);
    free(stamp);
    free(touched);
    if (stats) {
        stats->sweeps = k;
        stats->residual = R;
    }
}

/* ------------------------------------------------------------- integrate */

/* eq. (integrationscheme): v <- v', w <- w', x <- x + dt v',
 * q <- q + dt Q(q) w' with the quaternion block
 *   Q(q) = 1/2 [ -qx -qy -qz ;  qw  qz -qy ; -qz  qw  qx ;  qy -qx  qw ],
 * then q is renormalised (Sect. 3).  Periodic axes wrap positions into
 * [lo, hi). */
void nbgs_ref_integrate(ref_bodies *b, const ref_domain *dom, const ref_params *p, const double *v, const double *w)
{
    double dt = p->dt;
    for (int64_t i = 0; i < b->n; ++i) {
        b->vx[i] = v[3 * i + 0];
        b->vy[i] = v[3 * i + 1];
        b->vz[i] = v[3 * i + 2];
        b->wx[i] = w[3 * i + 0];
        b->wy[i] = w[3 * i + 1];
        b->wz[i] = w[3 * i + 2];
        b->x[i] = b->x[i] + dt * b->vx[i];
        b->y[i] = b->y[i] + dt * b->vy[i];
        b->z[i] = b->z[i] + dt * b->vz[i];
        double qw = b->qw[i], qx = b->qx[i], qy = b->qy[i], qz = b->qz[i];
        double ox = b->wx[i], oy = b->wy[i], oz = b->wz[i];
        double dw = 0.5 * (-qx * ox - qy * oy - qz * oz);
        double dx = 0.5 * (qw * ox + qz * oy - qy * oz);
        double dy = 0.5 * (-qz * ox + qw * oy + qx * oz);
        double dz = 0.5 * (qy * ox - qx * oy + qw * oz);
        qw = qw + dt * dw;
        qx = qx + dt * dx;
        qy = qy + dt * dy;
        qz = qz + dt * dz;
        double len = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
        b->qw[i] = qw / len;
        b->qx[i] = qx / len;
        b->qy[i] = qy / len;
        b->qz[i] = qz / len;
        double *pos[3] = {&b->x[i], &b->y[i], &b->z[i]};
        for (int a = 0; a < 3; ++a) {
            if (!dom->periodic[a]) continue;
            double L = dom->hi[a] - dom->lo[a];
            if (*pos[a] >= dom->hi[a]) *pos[a] = *pos[a] - L;
            else if (*pos[a] < dom->lo[a]) *pos[a] = *pos[a] + L;
        }
    }
}

/* ------------------------------------------------- stateful time stepping */

/* A scene that owns its contact list and the previous step's impulse table,
 * so that trajectories can be run step by step (Alg. 2 on one process). */
typedef struct {
    ref_bodies b;
    ref_domain dom;
    ref_plane *planes;
    ref_params p;
    ref_contacts c;
    int64_t nc;
    int32_t n_colours;
    int32_t *colour;
    int64_t *order;
    double *px, *py, *pz;
    double *v, *w;
    int64_t n_prev, prev_cap;
    uint64_t *prev_key;
    double *prev_px, *prev_py, *prev_pz;
    ref_solve_stats stats;
    double *residual_hist;
    int32_t hist_cap;
    double sub_edge; /* > 0: subdomain NBGS with blocks of about this edge */
    double blk_edge; /* > 0: plain NBGS in the block-local order with blocks of about this edge */
    int32_t blk_grids; /* shifted block grids of that order (1: one grid) */
    int32_t *sdom;
    int32_t n_sub;
} ref_world;

/* Read-only view of a world's current contact state. */
typedef struct {
    int64_t n_contacts;
    int32_t n_colours, sweeps;
    double residual;
    const int32_t *j1, *j2, *colour;
    const uint64_t *key;
    const double *nx, *ny, *nz, *xi, *a1, *a2;
    const double *px, *py, *pz; /* impulses, contact (key) order */
    const int64_t *order;       /* sweep order */
    const double *v, *w;        /* accumulators v', w' after the last solve, xyz interleaved */
    const double *residual_hist;
    const int32_t *sdom; /* subdomain of every contact (subdomain mode), else NULL */
    int32_t n_sub;
} ref_world_view;

static void contacts_alloc(ref_contacts *c, int64_t cap)
{
    c->cap = cap;
    size_t n = (size_t)(cap > 0 ? cap : 1);
    c->j1 = (int32_t *)malloc(n * sizeof(int32_t));
    c->j2 = (int32_t *)malloc(n * sizeof(int32_t));
    c->key = (uint64_t *)malloc(n * sizeof(uint64_t));
    c->nx = (double *)malloc(n * sizeof(double));
    c->ny = (double *)malloc(n * sizeof(double));
    c->nz = (double *)malloc(n * sizeof(double));
    c->xi = (double *)malloc(n * sizeof(double));
    c->a1 = (double *)malloc(n * sizeof(double));
    c->a2 = (double *)malloc(n * sizeof(double));
}

static void contacts_free(ref_contacts *c)
{
    free(c->j1);
    free(c->j2);
    free(c->key);
    free(c->nx);
    free(c->ny);
    free(c->nz);
    free(c->xi);
    free(c->a1);
    free(c->a2);
    memset(c, 0, sizeof(*c));
}

ref_world *nbgs_ref_world_create(const ref_bodies *b, const ref_domain *dom, const ref_params *p)
{
    ref_world *W = (ref_world *)calloc(1, sizeof(ref_world));
    W->b = *b;
    W->dom = *dom;
    W->planes = (ref_plane *)malloc(sizeof(ref_plane) * (size_t)(dom->n_planes > 0 ? dom->n_planes : 1));
    if (dom->n_planes > 0) memcpy(W->planes, dom->planes, sizeof(ref_plane) * (size_t)dom->n_planes);
    W->dom.planes = W->planes;
    W->p = *p;
    contacts_alloc(&W->c, 1024);
    W->v = (double *)malloc(sizeof(double) * 3 * (size_t)(b->n > 0 ? b->n : 1));
    W->w = (double *)malloc(sizeof(double) * 3 * (size_t)(b->n > 0 ? b->n : 1));
    return W;
}

void nbgs_ref_world_destroy(ref_world *W)
{
    if (!W) return;
    contacts_free(&W->c);
    free(W->planes);
    free(W->colour);
    free(W->order);
    free(W->px);
    free(W->py);
    free(W->pz);
    free(W->v);
    free(W->w);
    free(W->prev_key);
    free(W->prev_px);
    free(W->prev_py);
    free(W->prev_pz);
    free(W->residual_hist);
    free(W->sdom);
    free(W);
}

/* Detection, colouring and initial impulses.  warm: 0 = zero start,
 * 1 = previous step's impulses.  use_grid: 0 = exhaustive pair test. */
void nbgs_ref_world_detect(ref_world *W, int32_t use_grid, int32_t warm)
{
    int64_t m;
    for (;;) {
        m = use_grid ? nbgs_ref_detect_grid(&W->b, &W->dom, &W->p, &W->c)
                     : nbgs_ref_detect_brute(&W->b, &W->dom, &W->p, &W->c);
        if (m <= W->c.cap) break;
        contacts_free(&W->c);
        contacts_alloc(&W->c, 2 * m);
    }
    W->nc = m;
    size_t n = (size_t)(m > 0 ? m : 1);
    W->colour = (int32_t *)realloc(W->colour, n * sizeof(int32_t));
    W->order = (int64_t *)realloc(W->order, n * sizeof(int64_t));
    W->px = (double *)realloc(W->px, n * sizeof(double));
    W->py = (double *)realloc(W->py, n * sizeof(double));
    W->pz = (double *)realloc(W->pz, n * sizeof(double));
    if (W->sub_edge > 0.0) {
        W->sdom = (int32_t *)realloc(W->sdom, n * sizeof(int32_t));
        W->n_sub = nbgs_ref_subdomains(&W->b, &W->dom, W->sub_edge, m, W->c.j1, W->sdom);
        W->n_colours =
            nbgs_ref_colour(W->b.n, W->b.inv_mass, m, W->c.j1, W->c.j2, W->c.key, W->p.colour_seed, W->sdom, W->colour);
        nbgs_ref_sweep_order_sub(m, W->sdom, W->n_sub, W->colour, W->n_colours, W->order);
    } else if (W->blk_edge > 0.0) {
        W->sdom = (int32_t *)realloc(W->sdom, n * sizeof(int32_t));
        W->n_sub = nbgs_ref_block_local_grids(&W->b, &W->dom, W->blk_edge, W->blk_grids > 1 ? W->blk_grids : 1, m,
                                              W->c.j1, W->c.j2, W->sdom);
        W->n_colours =
            nbgs_ref_colour(W->b.n, W->b.inv_mass, m, W->c.j1, W->c.j2, W->c.key, W->p.colour_seed, W->sdom, W->colour);
        nbgs_ref_sweep_order_sub(m, W->sdom, W->n_sub, W->colour, W->n_colours, W->order);
    } else {
        W->n_colours =
            nbgs_ref_colour(W->b.n, W->b.inv_mass, m, W->c.j1, W->c.j2, W->c.key, W->p.colour_seed, NULL, W->colour);
        nbgs_ref_sweep_order(m, W->colour, W->n_colours, W->order);
    }
    if (warm && W->n_prev > 0) {
        nbgs_ref_warm_match(m, W->c.key, W->c.nx, W->c.ny, W->c.nz, W->p.mu, W->n_prev, W->prev_key, W->prev_px,
                            W->prev_py, W->prev_pz, W->px, W->py, W->pz);
    } else {
        for (int64_t j = 0; j < m; ++j) {
            W->px[j] = 0.0;
            W->py[j] = 0.0;
            W->pz[j] = 0.0;
        }
    }
}

/* Overwrite the initial impulses (contact order) before a solve. */
void nbgs_ref_world_set_impulses(ref_world *W, const double *px, const double *py, const double *pz)
{
    memcpy(W->px, px, sizeof(double) * (size_t)W->nc);
    memcpy(W->py, py, sizeof(double) * (size_t)W->nc);
    memcpy(W->pz, pz, sizeof(double) * (size_t)W->nc);
}

void nbgs_ref_world_solve(ref_world *W, int32_t max_sweeps, double target)
{
    if (max_sweeps > W->hist_cap) {
        W->residual_hist = (double *)realloc(W->residual_hist, sizeof(double) * (size_t)max_sweeps);
        W->hist_cap = max_sweeps;
    }
    if (W->sub_edge > 0.0)
        nbgs_ref_solve_sub(&W->b, &W->p, W->nc, W->c.j1, W->c.j2, W->c.nx, W->c.ny, W->c.nz, W->c.xi, W->c.a1,
                           W->c.a2, W->order, W->sdom, W->px, W->py, W->pz, max_sweeps, target, W->v, W->w,
                           W->residual_hist, &W->stats);
    else
        nbgs_ref_solve(&W->b, &W->p, W->nc, W->c.j1, W->c.j2, W->c.nx, W->c.ny, W->c.nz, W->c.xi, W->c.a1, W->c.a2,
                       W->order, W->px, W->py, W->pz, max_sweeps, target, W->v, W->w, W->residual_hist, &W->stats);
    /* keep (key, impulse) for the next step's warm start */
    if (W->nc > W->prev_cap) {
        W->prev_cap = W->nc;
        W->prev_key = (uint64_t *)realloc(W->prev_key, sizeof(uint64_t) * (size_t)W->nc);
        W->prev_px = (double *)realloc(W->prev_px, sizeof(double) * (size_t)W->nc);
        W->prev_py = (double *)realloc(W->prev_py, sizeof(double) * (size_t)W->nc);
        W->prev_pz = (double *)realloc(W->prev_pz, sizeof(double) * (size_t)W->nc);
    }
    W->n_prev = W->nc;
    if (W->nc > 0) {
        memcpy(W->prev_key, W->c.key, sizeof(uint64_t) * (size_t)W->nc);
        memcpy(W->prev_px, W->px, sizeof(double) * (size_t)W->nc);
        memcpy(W->prev_py, W->py, sizeof(double) * (size_t)W->nc);
        memcpy(W->prev_pz, W->pz, sizeof(double) * (size_t)W->nc);
    }
}

void nbgs_ref_world_integrate(ref_world *W) { nbgs_ref_integrate(&W->b, &W->dom, &W->p, W->v, W->w); }

/* One full time step: detect, colour, warm start, solve, integrate. */
void nbgs_ref_world_step(ref_world *W, int32_t use_grid, int32_t warm, int32_t max_sweeps, double target)
{
    nbgs_ref_world_detect(W, use_grid, warm);
    nbgs_ref_world_solve(W, max_sweeps, target);
    nbgs_ref_world_integrate(W);
}

void nbgs_ref_world_view_get(const ref_world *W, ref_world_view *out)
{
    out->n_contacts = W->nc;
    out->n_colours = W->n_colours;
    out->sweeps = W->stats.sweeps;
    out->residual = W->stats.residual;
    out->j1 = W->c.j1;
    out->j2 = W->c.j2;
    out->colour = W->colour;
    out->key = W->c.key;
    out->nx = W->c.nx;
    out->ny = W->c.ny;
    out->nz = W->c.nz;
    out->xi = W->c.xi;
    out->a1 = W->c.a1;
    out->a2 = W->c.a2;
    out->px = W->px;
    out->py = W->py;
    out->pz = W->pz;
    out->order = W->order;
    out->v = W->v;
    out->w = W->w;
    out->residual_hist = W->residual_hist;
    out->sdom = W->sub_edge > 0.0 || W->blk_edge > 0.0 ? W->sdom : NULL;
    out->n_sub = W->sub_edge > 0.0 || W->blk_edge > 0.0 ? W->n_sub : 0;
}

/* edge > 0: later detections assign subdomains and solves run the subdomain
 * NBGS; edge = 0: one subdomain, the classic NBGS. */
void nbgs_ref_world_set_subdomains(ref_world *W, double edge) { W->sub_edge = edge > 0.0 ? edge : 0.0; }

/* edge > 0: later detections sweep in the block-local order (plain NBGS);
 * edge = 0: (colour, key) order. */
void nbgs_ref_world_set_block_order(ref_world *W, double edge) { W->blk_edge = edge > 0.0 ? edge : 0.0; }

/* Shifted block grids of the block-local order (nbgs_ref_block_local_grids); 1 by default. */
void nbgs_ref_world_set_block_grids(ref_world *W, int32_t grids) { W->blk_grids = grids > 1 ? grids : 1; }

/* Replace the previous-step impulse table (key-sorted) used by the warm start. */
void nbgs_ref_world_set_prev(ref_world *W, int64_t n, const uint64_t *key, const double *px, const double *py,
                             const double *pz)
{
    if (n > W->prev_cap) {
        W->prev_cap = n;
        W->prev_key = (uint64_t *)realloc(W->prev_key, sizeof(uint64_t) * (size_t)n);
        W->prev_px = (double *)realloc(W->prev_px, sizeof(double) * (size_t)n);
        W->prev_py = (double *)realloc(W->prev_py, sizeof(double) * (size_t)n);
        W->prev_pz = (double *)realloc(W->prev_pz, sizeof(double) * (size_t)n);
    }
    W->n_prev = n;
    if (n > 0) {
        memcpy(W->prev_key, key, sizeof(uint64_t) * (size_t)n);
        memcpy(W->prev_px, px, sizeof(double) * (size_t)n);
        memcpy(W->prev_py, py, sizeof(double) * (size_t)n);
        memcpy(W->prev_pz, pz, sizeof(double) * (size_t)n);
    }
}
