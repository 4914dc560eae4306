/*
 * composite_ref.c -- ORACLE.  Test infrastructure only: the plain, slow,
 * sequential FP64 CPU reference of one time step for composite particles,
 * rigid clusters of element spheres (Sect. 2 builds non-spherical shapes from
 * primitives glued together; the granular gas of Sect. 7.2.1 uses two to four
 * spheres per particle).  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the GPU library never does.
 *
 * One time step:
 *   hull radii with the bounding radius, eq. (expansionradius)   -> comp_hull
 *   contacts between elements of different bodies and between
 *     elements and walls (Sect. 4; eq. (contactpos) of two
 *     spheres), lever arms from each body's centre of mass        -> nbgs_ref_comp_detect_brute / _element
 *   colouring and (colour, key) sweep order as for spheres        -> nbgs_ref_colour, nbgs_ref_sweep_order
 *   accumulators v' = v + dt g, w' = w + dt I^-1 (-w x I w)
 *     (eq. (integrationscheme) with its gyroscopic term)           -> comp_init
 *   NBGS sweeps (Alg. 1 with one subdomain) with the full 3x3
 *     Delassus block of eq. (wrench) and the exact solution of
 *     the one-contact problem (eqs. (nonpenetration), (coulomb))  -> nbgs_ref_comp_solve, nbgs_ref_comp_one_contact
 *   semi-implicit Euler as for spheres                            -> nbgs_ref_integrate
 *
 * Readings where the paper is silent (documented in the design notes):
 *   j1 is the lower body index, a wall is always j2 (body n + w, element E + w);
 *   a contact is a pair of element spheres, key = (element of j1 << 32) | element of j2;
 *   orientation q maps the principal (body) frame to the world, R(q) the usual
 *     rotation matrix of a unit quaternion, which the quaternion block Q(q) of
 *     Sect. 2 integrates for a world-frame angular velocity;
 *   the one-contact solve is exact: separate if the free normal velocity is
 *     non-negative, else stick if the unconstrained 3x3 solution lies in the
 *     cone, else slide on the cone's boundary, found as the root of a scalar
 *     equation in the multiplier of the tangential constraint (safeguarded
 *     Newton steps);
 *   a body with any principal inverse moment zero gets no gyroscopic term.
 *
 * Compile with -ffp-contract=off: every expression is evaluated as written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "nbgs_ref.h"

typedef struct {
    int64_t n;
    double *x, *y, *z;
    double *qw, *qx, *qy, *qz;
    double *vx, *vy, *vz;
    double *wx, *wy, *wz;
    const double *inv_mass;    /* n; 0: static */
    const double *inv_inertia; /* 3 n: principal inverse moments (body frame), xyz interleaved */
    const double *bound;       /* n: bounding radius about the centre of mass */
    const int32_t *elem_start; /* n + 1 */
    int64_t n_elem;
    const double *elem_offset; /* 3 E: element centres in body coordinates, xyz interleaved */
    const double *elem_radius; /* E */
} ref_comp_bodies;

typedef struct {
    int64_t cap;
    int32_t *j1, *j2; /* bodies (a wall is n + w) */
    int32_t *e1, *e2; /* elements (a wall is E + w) */
    uint64_t *key;
    double *nx, *ny, *nz; /* unit normal, outward from the element of j2 */
    double *xi;           /* signed contact distance */
    double *r1x, *r1y, *r1z; /* lever arm x_hat - x_j1 */
    double *r2x, *r2y, *r2z; /* lever arm x_hat - x_j2 (zero for a wall) */
} ref_comp_contacts;

/* ----------------------------------------------------------- geometry */

/* Rotation matrix (row major) of the unit quaternion (w, x, y, z). */
static void rotation(double qw, double qx, double qy, double qz, double R[9])
{
    R[0] = 1.0 - 2.0 * (qy * qy + qz * qz);
    R[1] = 2.0 * (qx * qy - qw * qz);
    R[2] = 2.0 * (qx * qz + qw * qy);
    R[3] = 2.0 * (qx * qy + qw * qz);
    R[4] = 1.0 - 2.0 * (qx * qx + qz * qz);
    R[5] = 2.0 * (qy * qz - qw * qx);
    R[6] = 2.0 * (qx * qz - qw * qy);
    R[7] = 2.0 * (qy * qz + qw * qx);
    R[8] = 1.0 - 2.0 * (qx * qx + qy * qy);
}

static void body_rotation(const ref_comp_bodies *b, int64_t i, double R[9])
{
    rotation(b->qw[i], b->qx[i], b->qy[i], b->qz[i], R);
}

/* World-frame offset R o of element e (from its body's centre of mass). */
static void world_offset(const ref_comp_bodies *b, const double R[9], int64_t e, double out[3])
{
    const double *o = &b->elem_offset[3 * e];
    for (int a = 0; a < 3; ++a) out[a] = R[3 * a + 0] * o[0] + R[3 * a + 1] * o[1] + R[3 * a + 2] * o[2];
}

static double min_image(double d, const ref_domain *dom, int axis)
{
    if (!dom->periodic[axis]) return d;
    double L = dom->hi[axis] - dom->lo[axis];
    if (d > 0.5 * L) return d - L;
    if (d < -0.5 * L) return d + L;
    return d;
}

/* eq. (expansionradius): h_i = dt (|v_i| + |omega_i| rbar_i) + tau with the
 * bounding radius rbar_i of the whole particle; every element's hull is the
 * element grown by h_i (the hull of a union is the union of the hulls). */
static double comp_hull(const ref_comp_bodies *b, const ref_params *p, int64_t i)
{
    double speed = sqrt(b->vx[i] * b->vx[i] + b->vy[i] * b->vy[i] + b->vz[i] * b->vz[i]);
    double spin = sqrt(b->wx[i] * b->wx[i] + b->wy[i] * b->wy[i] + b->wz[i] * b->wz[i]);
    return p->dt * (speed + spin * b->bound[i]) + p->tau;
}

static int is_static(const ref_comp_bodies *b, int64_t i) { return b->inv_mass[i] == 0.0; }

static void put(ref_comp_contacts *c, int64_t m, int64_t j1, int64_t j2, int64_t e1, int64_t e2, const double n[3],
                double xi, const double r1[3], const double r2[3])
{
    if (m >= c->cap) return;
    c->j1[m] = (int32_t)j1;
    c->j2[m] = (int32_t)j2;
    c->e1[m] = (int32_t)e1;
    c->e2[m] = (int32_t)e2;
    c->key[m] = ((uint64_t)(uint32_t)e1 << 32) | (uint64_t)(uint32_t)e2;
    c->nx[m] = n[0];
    c->ny[m] = n[1];
    c->nz[m] = n[2];
    c->xi[m] = xi;
    c->r1x[m] = r1[0];
    c->r1y[m] = r1[1];
    c->r1z[m] = r1[2];
    c->r2x[m] = r2[0];
    c->r2y[m] = r2[1];
    c->r2z[m] = r2[2];
}

/* Element e (body A, j1) against element f (body B > A, j2).  The two hulls
 * intersect iff |c_e - c_f| <= (r_e + h_A) + (r_f + h_B).  For two spheres
 * eq. (contactpos) puts the contact point on the surface of f's sphere along
 * the line of centres: n from c_f to c_e, x_hat = c_f + r_f n,
 * xi = |c_e - c_f| - r_e - r_f.  Lever arms from the centres of mass:
 * x_hat - x_A = R_A o_e - (r_e + xi) n,  x_hat - x_B = R_B o_f + r_f n. */
static int elem_pair(const ref_comp_bodies *b, const ref_domain *dom, int64_t A, int64_t e, const double oe[3],
                     double hA, int64_t B, int64_t f, const double of[3], double hB, double n[3], double *xi,
                     double r1[3], double r2[3])
{
    double ce[3] = {b->x[A] + oe[0], b->y[A] + oe[1], b->z[A] + oe[2]};
    double cf[3] = {b->x[B] + of[0], b->y[B] + of[1], b->z[B] + of[2]};
    double dx = min_image(ce[0] - cf[0], dom, 0);
    double dy = min_image(ce[1] - cf[1], dom, 1);
    double dz = min_image(ce[2] - cf[2], dom, 2);
    double d2 = dx * dx + dy * dy + dz * dz;
    double re = b->elem_radius[e], rf = b->elem_radius[f];
    double reach = (re + hA) + (rf + hB);
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
    *xi = (d - re) - rf;
    double a1 = re + *xi;
    for (int a = 0; a < 3; ++a) {
        r1[a] = oe[a] - a1 * n[a];
        r2[a] = of[a] + rf * n[a];
    }
    return 1;
}

/* Element e (body A) against wall w: signed distance of the element centre
 * s = n_w . (c_e - p_w), xi = s - r_e, contact iff xi <= h_A + tau (the wall's
 * hull is tau); the contact point is the foot of the perpendicular on the wall. */
static int elem_plane(const ref_comp_bodies *b, const ref_plane *pl, int64_t A, int64_t e, const double oe[3],
                      double hA, double tau, double n[3], double *xi, double r1[3], double r2[3])
{
    double ce[3] = {b->x[A] + oe[0], b->y[A] + oe[1], b->z[A] + oe[2]};
    double s = pl->normal[0] * (ce[0] - pl->point[0]) + pl->normal[1] * (ce[1] - pl->point[1]) +
               pl->normal[2] * (ce[2] - pl->point[2]);
    double gap = s - b->elem_radius[e];
    if (!(gap <= hA + tau)) return 0;
    n[0] = pl->normal[0];
    n[1] = pl->normal[1];
    n[2] = pl->normal[2];
    *xi = gap;
    double a1 = b->elem_radius[e] + gap;
    for (int a = 0; a < 3; ++a) {
        r1[a] = oe[a] - a1 * n[a];
        r2[a] = 0.0;
    }
    return 1;
}

static int64_t *body_of_elements(const ref_comp_bodies *b)
{
    int64_t *body = (int64_t *)malloc(sizeof(int64_t) * (size_t)(b->n_elem > 0 ? b->n_elem : 1));
    for (int64_t i = 0; i < b->n; ++i)
        for (int64_t e = b->elem_start[i]; e < b->elem_start[i + 1]; ++e) body[e] = i;
    return body;
}

/* World offsets of all elements (3 E) and hull radii of all bodies (n). */
static void offsets_and_hulls(const ref_comp_bodies *b, const ref_params *p, double *ow, double *h)
{
    double R[9];
    for (int64_t i = 0; i < b->n; ++i) {
        body_rotation(b, i, R);
        for (int64_t e = b->elem_start[i]; e < b->elem_start[i + 1]; ++e) world_offset(b, R, e, &ow[3 * e]);
        h[i] = comp_hull(b, p, i);
    }
}

/* Contact detection by exhaustive testing of element pairs of different
 * bodies (the definition of the potential-contact set of Sect. 4 for
 * composites) and of elements against walls.  Pairs of two static bodies are
 * not contacts, nor are walls with a static body.  Output in ascending key
 * order; returns the count, only the first cap are written. */
int64_t nbgs_ref_comp_detect_brute(const ref_comp_bodies *b, const ref_domain *dom, const ref_params *p,
                                   ref_comp_contacts *out)
{
    const int64_t E = b->n_elem;
    double *ow = (double *)malloc(sizeof(double) * 3 * (size_t)(E > 0 ? E : 1));
    double *h = (double *)malloc(sizeof(double) * (size_t)(b->n > 0 ? b->n : 1));
    int64_t *body = body_of_elements(b);
    offsets_and_hulls(b, p, ow, h);
    int64_t m = 0;
    double n[3], xi, r1[3], r2[3];
    for (int64_t e = 0; e < E; ++e) {
        int64_t A = body[e];
        for (int64_t f = b->elem_start[A + 1]; f < E; ++f) {
            int64_t B = body[f];
            if (is_static(b, A) && is_static(b, B)) continue;
            if (elem_pair(b, dom, A, e, &ow[3 * e], h[A], B, f, &ow[3 * f], h[B], n, &xi, r1, r2))
                put(out, m++, A, B, e, f, n, xi, r1, r2);
        }
        if (is_static(b, A)) continue;
        for (int32_t w = 0; w < dom->n_planes; ++w)
            if (elem_plane(b, &dom->planes[w], A, e, &ow[3 * e], h[A], p->tau, n, &xi, r1, r2))
                put(out, m++, A, b->n + w, e, E + w, n, xi, r1, r2);
    }
    free(body);
    free(h);
    free(ow);
    return m;
}

/* Contacts of one element e only (e on either side), by testing it against
 * every element of every other body and every wall, in ascending key order, so
 * that large scenes can be checked on sampled elements.  Returns the count. */
int64_t nbgs_ref_comp_detect_element(const ref_comp_bodies *b, const ref_domain *dom, const ref_params *p,
                                     int64_t e, ref_comp_contacts *out)
{
    const int64_t E = b->n_elem;
    int64_t *body = body_of_elements(b);
    const int64_t A = body[e];
    double R[9], oe[3], of[3];
    body_rotation(b, A, R);
    world_offset(b, R, e, oe);
    const double hA = comp_hull(b, p, A);
    int64_t m = 0;
    double n[3], xi, r1[3], r2[3];
    /* partners f of lower bodies give keys (f, e) < (e, .); then higher bodies; then walls */
    for (int64_t f = 0; f < E; ++f) {
        int64_t B = body[f];
        if (B == A) continue;
        if (is_static(b, A) && is_static(b, B)) continue;
        body_rotation(b, B, R);
        world_offset(b, R, f, of);
        const double hB = comp_hull(b, p, B);
        if (B < A) {
            if (elem_pair(b, dom, B, f, of, hB, A, e, oe, hA, n, &xi, r1, r2)) put(out, m++, B, A, f, e, n, xi, r1, r2);
        } else {
            if (elem_pair(b, dom, A, e, oe, hA, B, f, of, hB, n, &xi, r1, r2)) put(out, m++, A, B, e, f, n, xi, r1, r2);
        }
    }
    if (!is_static(b, A))
        for (int32_t w = 0; w < dom->n_planes; ++w)
            if (elem_plane(b, &dom->planes[w], A, e, oe, hA, p->tau, n, &xi, r1, r2))
                put(out, m++, A, b->n + w, e, E + w, n, xi, r1, r2);
    free(body);
    return m;
}

/* --------------------------------------------------- one-contact problem */

/* Sliding case for the multiplier lam >= 0 of the constraint |p_t| = mu p_n.
 * In the contact frame (n, t, o) the post-step relative velocity is u = Wc p + b
 * with
 *     Wc = [ a  c^T ]      b = [ b_n ]
 *          [ c  B   ],         [ b_t ].
 * Sliding means u_n = 0 and u_t = -lam p_t (opposite to the friction impulse,
 * eq. (coulomb)), so with M = B + lam 1:  p_t = p_n alpha + beta,
 * alpha = -M^-1 c, beta = -M^-1 b_t, and p_n = -(b_n + c.beta) / (a + c.alpha).
 * Returns phi(lam) = |p_t| - mu p_n and its derivative (d alpha = -M^-1 alpha,
 * d beta = -M^-1 beta). */
static double slide_eval(const double Wc[6], const double bc[3], double mu, double lam, double *pn, double *pt0,
                         double *pt1, double *dphi)
{
    double a = Wc[0], c0 = Wc[1], c1 = Wc[2], B00 = Wc[3], B01 = Wc[4], B11 = Wc[5];
    double m00 = B00 + lam, m11 = B11 + lam;
    double r = 1.0 / (m00 * m11 - B01 * B01);
    double al0 = -(m11 * c0 - B01 * c1) * r;
    double al1 = -(m00 * c1 - B01 * c0) * r;
    double be0 = -(m11 * bc[1] - B01 * bc[2]) * r;
    double be1 = -(m00 * bc[2] - B01 * bc[1]) * r;
    double da0 = -(m11 * al0 - B01 * al1) * r;
    double da1 = -(m00 * al1 - B01 * al0) * r;
    double db0 = -(m11 * be0 - B01 * be1) * r;
    double db1 = -(m00 * be1 - B01 * be0) * r;
    double D = a + (c0 * al0 + c1 * al1);
    double q = -(bc[0] + (c0 * be0 + c1 * be1)) / D;
    double dq = (-(c0 * db0 + c1 * db1) - q * (c0 * da0 + c1 * da1)) / D;
    double t0 = q * al0 + be0, t1 = q * al1 + be1;
    double d0 = (dq * al0 + q * da0) + db0, d1 = (dq * al1 + q * da1) + db1;
    double tl = sqrt(t0 * t0 + t1 * t1);
    *pn = q;
    *pt0 = t0;
    *pt1 = t1;
    *dphi = (tl > 0.0 ? (t0 * d0 + t1 * d1) / tl : 0.0) - mu * dq;
    return tl - mu * q;
}

/* The one-contact problem F_j(P) = 0 of Sect. 3 with a full symmetric
 * positive definite Delassus block, in the contact frame: Wc = (a, c0, c1,
 * B00, B01, B11) as above, bc = (b_n, b_t0, b_t1), result p = (p_n, p_t0, p_t1).
 * Cases, taken in this order:
 *   separate: b_n >= 0 -> p = 0 (u = b has u_n >= 0, eq. (nonpenetration));
 *   frictionless (mu = 0): p_n = -b_n / a, p_t = 0;
 *   stick: p = -Wc^-1 b if p_n > 0 and |p_t| <= mu p_n (then u = 0);
 *   slide: the root lam* > 0 of phi(lam) = |p_t(lam)| - mu p_n(lam), by Newton
 *     steps from lam = 0 (where phi >= 0) kept inside the bracket of the
 *     points seen so far (a step that leaves it bisects the bracket, or, with
 *     no point beyond the root yet, doubles the lower end, starting from
 *     B00 + B11); it stops when the Newton correction falls below 2^-50 lam or
 *     a step no longer moves lam, after 40 steps at most, and returns the
 *     impulse at the last lam, clipped onto the cone.
 *     For two spheres (c = 0, B = w_t 1) phi = |b_t| / (w_t + lam) - mu p_n and
 *     Newton from the left converges quadratically from the first step.
 * For a block that is diagonal in the contact frame the cases reduce to the
 * normal clamp and radial cone clip of the sphere solver. */
void nbgs_ref_comp_one_contact(const double Wc[6], const double bc[3], double mu, double p[3])
{
    double a = Wc[0], c0 = Wc[1], c1 = Wc[2], B00 = Wc[3], B01 = Wc[4], B11 = Wc[5];
    double bn = bc[0], bt0 = bc[1], bt1 = bc[2];
    p[0] = 0.0;
    p[1] = 0.0;
    p[2] = 0.0;
    if (!(bn < 0.0)) return;
    if (!(mu > 0.0)) {
        p[0] = -bn / a;
        return;
    }
    /* stick: adjugate of the symmetric Wc over its determinant */
    double i00 = B00 * B11 - B01 * B01;
    double i01 = c1 * B01 - c0 * B11;
    double i02 = c0 * B01 - c1 * B00;
    double i11 = a * B11 - c1 * c1;
    double i12 = c0 * c1 - a * B01;
    double i22 = a * B00 - c0 * c0;
    double det = a * i00 + c0 * i01 + c1 * i02;
    double sn = -(i00 * bn + i01 * bt0 + i02 * bt1) / det;
    double s0 = -(i01 * bn + i11 * bt0 + i12 * bt1) / det;
    double s1 = -(i02 * bn + i12 * bt0 + i22 * bt1) / det;
    if (sn > 0.0 && sqrt(s0 * s0 + s1 * s1) <= mu * sn) {
        p[0] = sn;
        p[1] = s0;
        p[2] = s1;
        return;
    }
    /* slide */
    double pn, pt0, pt1, dphi;
    double lo = 0.0, hi = INFINITY, lam = 0.0;
    for (int k = 0; k < 40; ++k) {
        double phi = slide_eval(Wc, bc, mu, lam, &pn, &pt0, &pt1, &dphi);
        if (phi > 0.0) lo = lam;
        else hi = lam;
        double step = phi / dphi;
        if (fabs(step) <= 0x1p-50 * lam) break; /* the Newton correction is below the last bits of lam */
        double next = lam - step;
        if (!(next > lo && next < hi)) next = hi < INFINITY ? 0.5 * (lo + hi) : (lo > 0.0 ? 2.0 * lo : B00 + B11);
        if (next == lam) break;
        lam = next;
    }
    slide_eval(Wc, bc, mu, lam, &pn, &pt0, &pt1, &dphi);
    if (!(pn > 0.0)) return;
    double tl = sqrt(pt0 * pt0 + pt1 * pt1);
    double lim = mu * pn;
    if (tl > lim) {
        double s = lim / tl;
        pt0 = pt0 * s;
        pt1 = pt1 * s;
    }
    p[0] = pn;
    p[1] = pt0;
    p[2] = pt1;
}

/* A right-handed orthonormal frame (n, t, o): t = (n x e) / |n x e| with e
 * the coordinate axis of the smallest |n_k| (lowest index on ties), o = n x t. */
static void tangent_frame(const double n[3], double t[3], double o[3])
{
    int k = 0;
    if (fabs(n[1]) < fabs(n[k])) k = 1;
    if (fabs(n[2]) < fabs(n[k])) k = 2;
    double e[3] = {0.0, 0.0, 0.0};
    e[k] = 1.0;
    t[0] = n[1] * e[2] - n[2] * e[1];
    t[1] = n[2] * e[0] - n[0] * e[2];
    t[2] = n[0] * e[1] - n[1] * e[0];
    double l = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    t[0] = t[0] / l;
    t[1] = t[1] / l;
    t[2] = t[2] / l;
    o[0] = n[1] * t[2] - n[2] * t[1];
    o[1] = n[2] * t[0] - n[0] * t[2];
    o[2] = n[0] * t[1] - n[1] * t[0];
}

static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void mat_vec(const double M[9], const double x[3], double y[3])
{
    for (int a = 0; a < 3; ++a) y[a] = M[3 * a + 0] * x[0] + M[3 * a + 1] * x[1] + M[3 * a + 2] * x[2];
}

/* K = -[r]x Iw [r]x, the velocity at lever arm r produced by a unit impulse
 * there through the body's rotation: dw = Iw (r x P), du = dw x r = K P
 * (eq. (wrench) and the relative contact velocity of Sect. 2).  Computed as
 * X^T (Iw X) with X = [r]x (X^T = -X). */
static void rot_block(const double r[3], const double Iw[9], double K[9])
{
    double X[9] = {0.0, -r[2], r[1], r[2], 0.0, -r[0], -r[1], r[0], 0.0};
    double A[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) A[3 * i + j] = Iw[3 * i + 0] * X[0 + j] + Iw[3 * i + 1] * X[3 + j] + Iw[3 * i + 2] * X[6 + j];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) K[3 * i + j] = X[0 + i] * A[0 + j] + X[3 + i] * A[3 + j] + X[6 + i] * A[6 + j];
}

/* ----------------------------------------------------------------- solve */

/* Body i's world inverse inertia Iw = R diag(ii) R^T. */
static void world_inv_inertia(const ref_comp_bodies *b, int64_t i, const double R[9], double Iw[9])
{
    const double *ii = &b->inv_inertia[3 * i];
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c)
            Iw[3 * a + c] = (R[3 * a + 0] * ii[0]) * R[3 * c + 0] + (R[3 * a + 1] * ii[1]) * R[3 * c + 1] +
                            (R[3 * a + 2] * ii[2]) * R[3 * c + 2];
}

/* Accumulators before any contact impulse, eq. (integrationscheme) without
 * the contact wrenches: v' = v + dt g and w' = w + dt I^-1 (-w x I w) for a
 * dynamic body (I = R diag(1/ii) R^T, evaluated in the body frame:
 * wb = R^T w, L = diag(1/ii) wb, dwb = dt diag(ii) (-(wb x L)), w' = w + R dwb). */
static void comp_init(const ref_comp_bodies *b, const ref_params *p, int64_t i, const double R[9], double v[3],
                      double w[3])
{
    int dyn = b->inv_mass[i] > 0.0;
    v[0] = dyn ? b->vx[i] + p->dt * p->gravity[0] : b->vx[i];
    v[1] = dyn ? b->vy[i] + p->dt * p->gravity[1] : b->vy[i];
    v[2] = dyn ? b->vz[i] + p->dt * p->gravity[2] : b->vz[i];
    w[0] = b->wx[i];
    w[1] = b->wy[i];
    w[2] = b->wz[i];
    const double *ii = &b->inv_inertia[3 * i];
    if (!dyn || !(ii[0] > 0.0) || !(ii[1] > 0.0) || !(ii[2] > 0.0)) return;
    double wb[3], L[3], g[3], dwb[3];
    for (int k = 0; k < 3; ++k) wb[k] = R[0 + k] * w[0] + R[3 + k] * w[1] + R[6 + k] * w[2];
    for (int k = 0; k < 3; ++k) L[k] = wb[k] / ii[k];
    g[0] = -(wb[1] * L[2] - wb[2] * L[1]);
    g[1] = -(wb[2] * L[0] - wb[0] * L[2]);
    g[2] = -(wb[0] * L[1] - wb[1] * L[0]);
    for (int k = 0; k < 3; ++k) dwb[k] = p->dt * (ii[k] * g[k]);
    for (int a = 0; a < 3; ++a) w[a] = w[a] + (R[3 * a + 0] * dwb[0] + R[3 * a + 1] * dwb[1] + R[3 * a + 2] * dwb[2]);
}

/* Impulse dP at contact j: +dP on j1, -dP on j2 at the contact point
 * (eq. (wrench)):  v1 += m1^-1 dP, w1 += Iw1 (r1 x dP), v2 -= m2^-1 dP,
 * w2 -= Iw2 (r2 x dP).  Static bodies and walls are left alone. */
static void comp_apply(int64_t N, const double *im, const double *Iw, double *v, double *w, int32_t b1, int32_t b2,
                       const double r1[3], const double r2[3], const double dP[3])
{
    double m[3], t[3];
    if (im[b1] > 0.0) {
        m[0] = r1[1] * dP[2] - r1[2] * dP[1];
        m[1] = r1[2] * dP[0] - r1[0] * dP[2];
        m[2] = r1[0] * dP[1] - r1[1] * dP[0];
        mat_vec(&Iw[9 * b1], m, t);
        for (int a = 0; a < 3; ++a) {
            v[3 * b1 + a] = v[3 * b1 + a] + im[b1] * dP[a];
            w[3 * b1 + a] = w[3 * b1 + a] + t[a];
        }
    }
    if (b2 < N && im[b2] > 0.0) {
        m[0] = r2[1] * dP[2] - r2[2] * dP[1];
        m[1] = r2[2] * dP[0] - r2[0] * dP[2];
        m[2] = r2[0] * dP[1] - r2[1] * dP[0];
        mat_vec(&Iw[9 * b2], m, t);
        for (int a = 0; a < 3; ++a) {
            v[3 * b2 + a] = v[3 * b2 + a] - im[b2] * dP[a];
            w[3 * b2 + a] = w[3 * b2 + a] - t[a];
        }
    }
}

/* NBGS solve of one time step for composite bodies (Alg. 1 with a single
 * subdomain, contacts in the given sweep order).  Per contact:
 *   u    = (v'_1 + w'_1 x r1) - (v'_2 + w'_2 x r2)        relative contact velocity
 *   W    = (m1^-1 + m2^-1) 1 + K(r1, Iw1) + K(r2, Iw2)    Delassus block (eq. (wrench))
 *   b    = u + (xi'/dt) n - W P_j                        (own impulse taken out; xi' = erp xi if xi < 0)
 *   P*   = the one-contact solution in the frame (n, t, o), back in world coordinates
 *   P_new = omega P* + (1 - omega) P_j, apply dP = P_new - P_j.
 * Residual R_k = |dP|_2 / |P_new|_2 per sweep; stop at R_k <= target (> 0)
 * or k = max_sweeps.  v_out, w_out (3 n, xyz interleaved) receive v', w';
 * iw_out (9 n, may be NULL) the world inverse inertias. */
void nbgs_ref_comp_solve(const ref_comp_bodies *b, const ref_params *p, int64_t nc, const ref_comp_contacts *c,
                         const int64_t *order, double *px, double *py, double *pz, int32_t max_sweeps, double target,
                         double *v_out, double *w_out, double *iw_out, double *residual_hist, ref_solve_stats *stats)
{
    const int64_t N = b->n;
    const double *im = b->inv_mass;
    double *v = v_out, *w = w_out;
    double *Iw = (double *)malloc(sizeof(double) * 9 * (size_t)(N > 0 ? N : 1));
    double R[9];
    for (int64_t i = 0; i < N; ++i) {
        body_rotation(b, i, R);
        world_inv_inertia(b, i, R, &Iw[9 * i]);
        comp_init(b, p, i, R, &v[3 * i], &w[3 * i]);
    }
    if (iw_out) memcpy(iw_out, Iw, sizeof(double) * 9 * (size_t)N);
    for (int64_t t = 0; t < nc; ++t) {
        int64_t j = order[t];
        double r1[3] = {c->r1x[j], c->r1y[j], c->r1z[j]}, r2[3] = {c->r2x[j], c->r2y[j], c->r2z[j]};
        double P0[3] = {px[j], py[j], pz[j]};
        if (P0[0] != 0.0 || P0[1] != 0.0 || P0[2] != 0.0) comp_apply(N, im, Iw, v, w, c->j1[j], c->j2[j], r1, r2, P0);
    }
    int32_t k = 0;
    double Rk = 0.0;
    while (k < max_sweeps) {
        double sum_dp = 0.0, sum_p = 0.0;
        for (int64_t t = 0; t < nc; ++t) {
            int64_t j = order[t];
            int32_t b1 = c->j1[j], b2 = c->j2[j];
            double n[3] = {c->nx[j], c->ny[j], c->nz[j]};
            double r1[3] = {c->r1x[j], c->r1y[j], c->r1z[j]}, r2[3] = {c->r2x[j], c->r2y[j], c->r2z[j]};
            double vp1[3], vp2[3] = {0.0, 0.0, 0.0};
            const double *V1 = &v[3 * b1], *W1 = &w[3 * b1];
            vp1[0] = V1[0] + (W1[1] * r1[2] - W1[2] * r1[1]);
            vp1[1] = V1[1] + (W1[2] * r1[0] - W1[0] * r1[2]);
            vp1[2] = V1[2] + (W1[0] * r1[1] - W1[1] * r1[0]);
            double im2 = 0.0;
            if (b2 < N) {
                const double *V2 = &v[3 * b2], *W2 = &w[3 * b2];
                vp2[0] = V2[0] + (W2[1] * r2[2] - W2[2] * r2[1]);
                vp2[1] = V2[1] + (W2[2] * r2[0] - W2[0] * r2[2]);
                vp2[2] = V2[2] + (W2[0] * r2[1] - W2[1] * r2[0]);
                im2 = im[b2];
            }
            double K1[9], K2[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, W[9];
            rot_block(r1, &Iw[9 * b1], K1);
            if (b2 < N) rot_block(r2, &Iw[9 * b2], K2);
            double wsum = im[b1] + im2;
            for (int a = 0; a < 3; ++a)
                for (int e = 0; e < 3; ++e) W[3 * a + e] = ((a == e ? wsum : 0.0) + K1[3 * a + e]) + K2[3 * a + e];
            double corr = c->xi[j] < 0.0 ? p->erp * c->xi[j] : c->xi[j];
            double bias = corr / p->dt;
            double P[3] = {px[j], py[j], pz[j]};
            double WP[3], bw[3];
            mat_vec(W, P, WP);
            for (int a = 0; a < 3; ++a) bw[a] = ((vp1[a] - vp2[a]) + bias * n[a]) - WP[a];
            double tt[3], oo[3];
            tangent_frame(n, tt, oo);
            double Wn[3], Wt[3], Wo[3];
            mat_vec(W, n, Wn);
            mat_vec(W, tt, Wt);
            mat_vec(W, oo, Wo);
            double Wc[6] = {dot3(n, Wn), dot3(tt, Wn), dot3(oo, Wn), dot3(tt, Wt), dot3(tt, Wo), dot3(oo, Wo)};
            double bc[3] = {dot3(n, bw), dot3(tt, bw), dot3(oo, bw)};
            double pc[3];
            nbgs_ref_comp_one_contact(Wc, bc, p->mu, pc);
            double Pnew[3], dP[3];
            for (int a = 0; a < 3; ++a) {
                double Ps = (pc[0] * n[a] + pc[1] * tt[a]) + pc[2] * oo[a];
                Pnew[a] = p->relax * Ps + (1.0 - p->relax) * P[a];
                dP[a] = Pnew[a] - P[a];
            }
            comp_apply(N, im, Iw, v, w, b1, b2, r1, r2, dP);
            px[j] = Pnew[0];
            py[j] = Pnew[1];
            pz[j] = Pnew[2];
            sum_dp += dP[0] * dP[0] + dP[1] * dP[1] + dP[2] * dP[2];
            sum_p += Pnew[0] * Pnew[0] + Pnew[1] * Pnew[1] + Pnew[2] * Pnew[2];
        }
        double den = sqrt(sum_p);
        Rk = sqrt(sum_dp) / (den > 1e-300 ? den : 1e-300);
        if (residual_hist) residual_hist[k] = Rk;
        ++k;
        if (target > 0.0 && Rk <= target) break;
    }
    free(Iw);
    if (stats) {
        stats->sweeps = k;
        stats->residual = Rk;
    }
}

/* eq. (integrationscheme) for the body state (positions, orientations,
 * velocities), exactly as for spheres. */
void nbgs_ref_comp_integrate(ref_comp_bodies *b, const ref_domain *dom, const ref_params *p, const double *v,
                             const double *w)
{
    ref_bodies s;
    memset(&s, 0, sizeof(s));
    s.n = b->n;
    s.x = b->x;
    s.y = b->y;
    s.z = b->z;
    s.qw = b->qw;
    s.qx = b->qx;
    s.qy = b->qy;
    s.qz = b->qz;
    s.vx = b->vx;
    s.vy = b->vy;
    s.vz = b->vz;
    s.wx = b->wx;
    s.wy = b->wy;
    s.wz = b->wz;
    nbgs_ref_integrate(&s, dom, p, v, w);
}

/* ------------------------------------------------- stateful time stepping */

typedef struct {
    ref_comp_bodies b;
    ref_domain dom;
    ref_plane *planes;
    ref_params p;
    ref_comp_contacts c;
    int64_t nc;
    int32_t n_colours;
    int32_t *colour;
    int64_t *order;
    double *px, *py, *pz;
    double *v, *w, *iw;
    int64_t n_prev, prev_cap;
    uint64_t *prev_key;
    double *prev_px, *prev_py, *prev_pz;
    ref_solve_stats stats;
    double *residual_hist;
    int32_t hist_cap;
} ref_comp_world;

typedef struct {
    int64_t n_contacts;
    int32_t n_colours, sweeps;
    double residual;
    const int32_t *j1, *j2, *e1, *e2, *colour;
    const uint64_t *key;
    const double *nx, *ny, *nz, *xi, *r1x, *r1y, *r1z, *r2x, *r2y, *r2z;
    const double *px, *py, *pz;
    const int64_t *order;
    const double *v, *w, *iw;
    const double *residual_hist;
} ref_comp_view;

static void comp_contacts_alloc(ref_comp_contacts *c, int64_t cap)
{
    size_t n = (size_t)(cap > 0 ? cap : 1);
    c->cap = cap;
    c->j1 = (int32_t *)malloc(n * sizeof(int32_t));
    c->j2 = (int32_t *)malloc(n * sizeof(int32_t));
    c->e1 = (int32_t *)malloc(n * sizeof(int32_t));
    c->e2 = (int32_t *)malloc(n * sizeof(int32_t));
    c->key = (uint64_t *)malloc(n * sizeof(uint64_t));
    double **f[] = {&c->nx, &c->ny, &c->nz, &c->xi, &c->r1x, &c->r1y, &c->r1z, &c->r2x, &c->r2y, &c->r2z};
    for (size_t k = 0; k < sizeof(f) / sizeof(f[0]); ++k) *f[k] = (double *)malloc(n * sizeof(double));
}

static void comp_contacts_free(ref_comp_contacts *c)
{
    free(c->j1);
    free(c->j2);
    free(c->e1);
    free(c->e2);
    free(c->key);
    double *f[] = {c->nx, c->ny, c->nz, c->xi, c->r1x, c->r1y, c->r1z, c->r2x, c->r2y, c->r2z};
    for (size_t k = 0; k < sizeof(f) / sizeof(f[0]); ++k) free(f[k]);
    memset(c, 0, sizeof(*c));
}

ref_comp_world *nbgs_ref_comp_world_create(const ref_comp_bodies *b, const ref_domain *dom, const ref_params *p)
{
    ref_comp_world *W = (ref_comp_world *)calloc(1, sizeof(ref_comp_world));
    W->b = *b;
    W->dom = *dom;
    W->planes = (ref_plane *)malloc(sizeof(ref_plane) * (size_t)(dom->n_planes > 0 ? dom->n_planes : 1));
    if (dom->n_planes > 0) memcpy(W->planes, dom->planes, sizeof(ref_plane) * (size_t)dom->n_planes);
    W->dom.planes = W->planes;
    W->p = *p;
    comp_contacts_alloc(&W->c, 1024);
    size_t n = (size_t)(b->n > 0 ? b->n : 1);
    W->v = (double *)malloc(sizeof(double) * 3 * n);
    W->w = (double *)malloc(sizeof(double) * 3 * n);
    W->iw = (double *)malloc(sizeof(double) * 9 * n);
    return W;
}

void nbgs_ref_comp_world_destroy(ref_comp_world *W)
{
    if (!W) return;
    comp_contacts_free(&W->c);
    free(W->planes);
    free(W->colour);
    free(W->order);
    free(W->px);
    free(W->py);
    free(W->pz);
    free(W->v);
    free(W->w);
    free(W->iw);
    free(W->prev_key);
    free(W->prev_px);
    free(W->prev_py);
    free(W->prev_pz);
    free(W->residual_hist);
    free(W);
}

/* Detection, colouring (conflicts between contacts that share a dynamic
 * body), (colour, key) order and initial impulses (warm: previous step's
 * impulses matched by key and re-projected onto the new cone; else zero). */
void nbgs_ref_comp_world_detect(ref_comp_world *W, int32_t warm)
{
    int64_t m;
    for (;;) {
        m = nbgs_ref_comp_detect_brute(&W->b, &W->dom, &W->p, &W->c);
        if (m <= W->c.cap) break;
        comp_contacts_free(&W->c);
        comp_contacts_alloc(&W->c, 2 * m);
    }
    W->nc = m;
    size_t n = (size_t)(m > 0 ? m : 1);
    W->colour = (int32_t *)realloc(W->colour, n * sizeof(int32_t));
    W->order = (int64_t *)realloc(W->order, n * sizeof(int64_t));
    W->px = (double *)realloc(W->px, n * sizeof(double));
    W->py = (double *)realloc(W->py, n * sizeof(double));
    W->pz = (double *)realloc(W->pz, n * sizeof(double));
    W->n_colours =
        nbgs_ref_colour(W->b.n, W->b.inv_mass, m, W->c.j1, W->c.j2, W->c.key, W->p.colour_seed, NULL, W->colour);
    nbgs_ref_sweep_order(m, W->colour, W->n_colours, W->order);
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

void nbgs_ref_comp_world_set_impulses(ref_comp_world *W, const double *px, const double *py, const double *pz)
{
    memcpy(W->px, px, sizeof(double) * (size_t)W->nc);
    memcpy(W->py, py, sizeof(double) * (size_t)W->nc);
    memcpy(W->pz, pz, sizeof(double) * (size_t)W->nc);
}

void nbgs_ref_comp_world_solve(ref_comp_world *W, int32_t max_sweeps, double target)
{
    if (max_sweeps > W->hist_cap) {
        W->residual_hist = (double *)realloc(W->residual_hist, sizeof(double) * (size_t)max_sweeps);
        W->hist_cap = max_sweeps;
    }
    nbgs_ref_comp_solve(&W->b, &W->p, W->nc, &W->c, W->order, W->px, W->py, W->pz, max_sweeps, target, W->v, W->w,
                        W->iw, W->residual_hist, &W->stats);
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

void nbgs_ref_comp_world_integrate(ref_comp_world *W) { nbgs_ref_comp_integrate(&W->b, &W->dom, &W->p, W->v, W->w); }

void nbgs_ref_comp_world_step(ref_comp_world *W, int32_t warm, int32_t max_sweeps, double target)
{
    nbgs_ref_comp_world_detect(W, warm);
    nbgs_ref_comp_world_solve(W, max_sweeps, target);
    nbgs_ref_comp_world_integrate(W);
}

void nbgs_ref_comp_world_view_get(const ref_comp_world *W, ref_comp_view *out)
{
    out->n_contacts = W->nc;
    out->n_colours = W->n_colours;
    out->sweeps = W->stats.sweeps;
    out->residual = W->stats.residual;
    out->j1 = W->c.j1;
    out->j2 = W->c.j2;
    out->e1 = W->c.e1;
    out->e2 = W->c.e2;
    out->colour = W->colour;
    out->key = W->c.key;
    out->nx = W->c.nx;
    out->ny = W->c.ny;
    out->nz = W->c.nz;
    out->xi = W->c.xi;
    out->r1x = W->c.r1x;
    out->r1y = W->c.r1y;
    out->r1z = W->c.r1z;
    out->r2x = W->c.r2x;
    out->r2y = W->c.r2y;
    out->r2z = W->c.r2z;
    out->px = W->px;
    out->py = W->py;
    out->pz = W->pz;
    out->order = W->order;
    out->v = W->v;
    out->w = W->w;
    out->iw = W->iw;
    out->residual_hist = W->residual_hist;
}
