/*
 * nbgs_ref.h -- ORACLE (test infrastructure only).  Types shared by the
 * sphere oracle (nbgs_ref.c) and the composite-particle oracle
 * (composite_ref.c), and the sphere-oracle routines the latter reuses.
 */
#pragma once
#include <stdint.h>

typedef struct {
    int64_t n;
    double *x, *y, *z;
    double *qw, *qx, *qy, *qz;
    double *vx, *vy, *vz;
    double *wx, *wy, *wz;
    const double *radius, *inv_mass, *inv_inertia;
} ref_bodies;

typedef struct {
    double point[3];
    double normal[3]; /* unit, pointing into the domain */
} ref_plane;

typedef struct {
    double lo[3], hi[3];
    int32_t periodic[3];
    int32_t n_planes;
    const ref_plane *planes;
} ref_domain;

typedef struct {
    double dt;
    double gravity[3];
    double mu;    /* coefficient of friction, eq. (coulomb) */
    double tau;   /* hull safety margin, eq. (expansionradius) */
    double relax; /* relaxation parameter omega of Alg. 1 */
    double erp;   /* scale of the penetration correction xi/dt when xi < 0, Sect. 3 */
    uint64_t colour_seed;
} ref_params;

/* Contact list, structure of arrays, capacity cap. */
typedef struct {
    int64_t cap;
    int32_t *j1, *j2;
    uint64_t *key;
    double *nx, *ny, *nz; /* unit normal, outward from body j2 */
    double *xi;           /* signed contact distance */
    double *a1, *a2;      /* lever arms: x_hat - x_j1 = -a1 n, x_hat - x_j2 = a2 n */
} ref_contacts;

typedef struct {
    int32_t sweeps;
    double residual;
} ref_solve_stats;

int32_t nbgs_ref_colour(int64_t n_bodies, const double *inv_mass, int64_t nc, const int32_t *j1, const int32_t *j2,
                        const uint64_t *key, uint64_t seed, const int32_t *sdom, int32_t *colour);
void nbgs_ref_sweep_order(int64_t nc, const int32_t *colour, int32_t n_colours, int64_t *order);
void nbgs_ref_warm_match(int64_t nc, const uint64_t *key, const double *nx, const double *ny, const double *nz,
                         double mu, int64_t n_prev, const uint64_t *prev_key, const double *prev_px,
                         const double *prev_py, const double *prev_pz, double *px, double *py, double *pz);
void nbgs_ref_integrate(ref_bodies *b, const ref_domain *dom, const ref_params *p, const double *v, const double *w);
/* OpenMP mode of the sweeps (1 thread: the sequential loops; results identical either way). */
void nbgs_ref_set_threads(int32_t threads);
int32_t nbgs_ref_get_threads(void);
int64_t nbgs_ref_order_levels(int64_t N, const double *inv_mass, int64_t nc, const int32_t *j1, const int32_t *j2,
                              const int64_t *order, int64_t *lev_pos, int64_t **lev_start);
