/*
 * mlp_ref.c -- ORACLE (test infrastructure only) for the learned warm start:
 * per-contact features, a 12-128-128-3 ReLU multilayer perceptron in FP64
 * (forward, loss, gradient), Adam, the decoding of its output into an
 * initial impulse and the training targets.  The Jacobi residual that judges
 * an initial impulse is nbgs_ref_jacobi_residual in nbgs_ref.c (it needs the
 * solve's one-contact problem).
 *
 * The network predicts each contact's impulse at the start of a time step
 * (the paper allows any initial solution of Alg. 1, Sect. 5).  Features are
 * taken in a contact frame (n, e_t, e_o) so that they do not depend on the
 * orientation of the contact in space.
 *
 * Weight vector layout (18,563 values): W1[12][128], b1[128], W2[128][128],
 * b2[128], W3[128][3], b3[3]; layer l computes y = x W_l + b_l, ReLU after
 * layers 1 and 2.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NF 12
#define NH 128
#define NO 3
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + NF * NH)
#define OFF_W2 (OFF_B1 + NH)
#define OFF_B2 (OFF_W2 + NH * NH)
#define OFF_W3 (OFF_B2 + NH)
#define OFF_B3 (OFF_W3 + NH * NO)
#define N_PARAMS (OFF_B3 + NO)

int32_t nbgs_ref_mlp_param_count(void) { return N_PARAMS; }

/* Forward pass of one sample; h1, h2 receive the post-ReLU activations. */
static void forward_one(const double *w, const double *x, double *h1, double *h2, double *y)
{
    for (int j = 0; j < NH; ++j) {
        double a = w[OFF_B1 + j];
        for (int i = 0; i < NF; ++i) a += x[i] * w[OFF_W1 + i * NH + j];
        h1[j] = a > 0.0 ? a : 0.0;
    }
    for (int j = 0; j < NH; ++j) {
        double a = w[OFF_B2 + j];
        for (int i = 0; i < NH; ++i) a += h1[i] * w[OFF_W2 + i * NH + j];
        h2[j] = a > 0.0 ? a : 0.0;
    }
    for (int j = 0; j < NO; ++j) {
        double a = w[OFF_B3 + j];
        for (int i = 0; i < NH; ++i) a += h2[i] * w[OFF_W3 + i * NO + j];
        y[j] = a;
    }
}

/* y[n][3] = MLP(x[n][12]). */
void nbgs_ref_mlp_forward(const double *w, int64_t n, const double *x, double *y)
{
    double h1[NH], h2[NH];
    for (int64_t s = 0; s < n; ++s) forward_one(w, x + NF * s, h1, h2, y + NO * s);
}

/* Loss L = 1/(2n) sum_s |y_s - t_s|^2 and its gradient with respect to the
 * weight vector (back-propagation through the three layers). */
double nbgs_ref_mlp_loss_grad(const double *w, int64_t n, const double *x, const double *t, double *grad)
{
    double h1[NH], h2[NH], y[NO], dy[NO], dh2[NH], dh1[NH];
    memset(grad, 0, sizeof(double) * N_PARAMS);
    double loss = 0.0;
    for (int64_t s = 0; s < n; ++s) {
        const double *xs = x + NF * s;
        forward_one(w, xs, h1, h2, y);
        for (int j = 0; j < NO; ++j) {
            double e = y[j] - t[NO * s + j];
            loss += 0.5 * e * e;
            dy[j] = e / (double)n;
        }
        for (int i = 0; i < NH; ++i) {
            double a = 0.0;
            for (int j = 0; j < NO; ++j) {
                grad[OFF_W3 + i * NO + j] += h2[i] * dy[j];
                a += dy[j] * w[OFF_W3 + i * NO + j];
            }
            dh2[i] = h2[i] > 0.0 ? a : 0.0;
        }
        for (int j = 0; j < NO; ++j) grad[OFF_B3 + j] += dy[j];
        for (int i = 0; i < NH; ++i) {
            double a = 0.0;
            for (int j = 0; j < NH; ++j) {
                grad[OFF_W2 + i * NH + j] += h1[i] * dh2[j];
                a += dh2[j] * w[OFF_W2 + i * NH + j];
            }
            dh1[i] = h1[i] > 0.0 ? a : 0.0;
        }
        for (int j = 0; j < NH; ++j) grad[OFF_B2 + j] += dh2[j];
        for (int i = 0; i < NF; ++i)
            for (int j = 0; j < NH; ++j) grad[OFF_W1 + i * NH + j] += xs[i] * dh1[j];
        for (int j = 0; j < NH; ++j) grad[OFF_B1 + j] += dh1[j];
    }
    return loss / (double)n;
}

/* Adam update (Kingma & Ba 2015) of the weight vector, step k >= 1. */
void nbgs_ref_mlp_adam(double *w, const double *g, double *m, double *v, int64_t k, double lr, double beta1,
                       double beta2, double eps)
{
    double c1 = 1.0 - pow(beta1, (double)k), c2 = 1.0 - pow(beta2, (double)k);
    for (int i = 0; i < N_PARAMS; ++i) {
        m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
        v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
        w[i] = w[i] - lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}

/* Contact frame: n; e_t along the tangential relative velocity u_t if it is
 * not negligible, else along the tangential part of the previous impulse, else
 * n x (the world axis least aligned with n); e_o = n x e_t. */
static void contact_frame(const double *n, const double *ut, const double *Pt, double vtiny, double ptiny, double *et,
                          double *eo)
{
    double lu = sqrt(ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2]);
    double lp = sqrt(Pt[0] * Pt[0] + Pt[1] * Pt[1] + Pt[2] * Pt[2]);
    if (lu > vtiny) {
        et[0] = ut[0] / lu;
        et[1] = ut[1] / lu;
        et[2] = ut[2] / lu;
    } else if (lp > ptiny) {
        et[0] = Pt[0] / lp;
        et[1] = Pt[1] / lp;
        et[2] = Pt[2] / lp;
    } else {
        int a = 0;
        if (fabs(n[1]) < fabs(n[a])) a = 1;
        if (fabs(n[2]) < fabs(n[a])) a = 2;
        double e[3] = {0.0, 0.0, 0.0};
        e[a] = 1.0;
        double c0 = n[1] * e[2] - n[2] * e[1], c1 = n[2] * e[0] - n[0] * e[2], c2 = n[0] * e[1] - n[1] * e[0];
        double lc = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
        et[0] = c0 / lc;
        et[1] = c1 / lc;
        et[2] = c2 / lc;
    }
    eo[0] = n[1] * et[2] - n[2] * et[1];
    eo[1] = n[2] * et[0] - n[0] * et[2];
    eo[2] = n[0] * et[1] - n[1] * et[0];
}

/* Features of every contact at the start of a step.  Velocities are the
 * accumulators before any impulse, v0 = v + dt g (dynamic bodies), w0 = w;
 * P0 is the previous-step impulse re-projected onto the new cone (zero if
 * the pair is new).  Scales: vs (velocity), ms (mass), rs (length).
 *   f0 = u_n / vs          u_n = xi'/dt + n.du   (free normal velocity)
 *   f1 = u_t.e_t / vs,  f2 = u_t.e_o / vs
 *   f3 = xi / rs
 *   f4 = w_n ms,  f5 = w_t ms   (Delassus diagonal, see the solve)
 *   f6 = r_j1 / rs,  f7 = r_j2 / rs (0 for a wall)
 *   f8 = mu
 *   f9..f11 = (P0.n, P0.e_t, P0.e_o) / (ms vs)
 * frame[9 j ..] receives n, e_t, e_o. */
void nbgs_ref_mlp_features(int64_t nb, const double *vx, const double *vy, const double *vz, const double *wx,
                           const double *wy, const double *wz, const double *radius, const double *inv_mass,
                           const double *inv_inertia, const double *gravity, double dt, double mu, double erp,
                           int64_t nc, const int32_t *j1, const int32_t *j2, const double *nx, const double *ny,
                           const double *nz, const double *xi, const double *a1, const double *a2, const double *px,
                           const double *py, const double *pz, double vs, double ms, double rs, double *feat,
                           double *frame)
{
    for (int64_t j = 0; j < nc; ++j) {
        int32_t b1 = j1[j], b2 = j2[j];
        double n[3] = {nx[j], ny[j], nz[j]};
        double v1[3], w1[3], v2[3] = {0.0, 0.0, 0.0}, w2[3] = {0.0, 0.0, 0.0};
        double im1 = inv_mass[b1], ii1 = inv_inertia[b1], im2 = 0.0, ii2 = 0.0, r2 = 0.0;
        int dyn1 = im1 > 0.0;
        v1[0] = dyn1 ? vx[b1] + dt * gravity[0] : vx[b1];
        v1[1] = dyn1 ? vy[b1] + dt * gravity[1] : vy[b1];
        v1[2] = dyn1 ? vz[b1] + dt * gravity[2] : vz[b1];
        w1[0] = wx[b1];
        w1[1] = wy[b1];
        w1[2] = wz[b1];
        if (b2 < nb) {
            int dyn2 = inv_mass[b2] > 0.0;
            im2 = inv_mass[b2];
            ii2 = inv_inertia[b2];
            r2 = radius[b2];
            v2[0] = dyn2 ? vx[b2] + dt * gravity[0] : vx[b2];
            v2[1] = dyn2 ? vy[b2] + dt * gravity[1] : vy[b2];
            v2[2] = dyn2 ? vz[b2] + dt * gravity[2] : vz[b2];
            w2[0] = wx[b2];
            w2[1] = wy[b2];
            w2[2] = wz[b2];
        }
        double s0 = a1[j] * w1[0] + a2[j] * w2[0];
        double s1 = a1[j] * w1[1] + a2[j] * w2[1];
        double s2 = a1[j] * w1[2] + a2[j] * w2[2];
        double du[3];
        du[0] = (v1[0] - v2[0]) - (s1 * n[2] - s2 * n[1]);
        du[1] = (v1[1] - v2[1]) - (s2 * n[0] - s0 * n[2]);
        du[2] = (v1[2] - v2[2]) - (s0 * n[1] - s1 * n[0]);
        double dun = n[0] * du[0] + n[1] * du[1] + n[2] * du[2];
        double corr = xi[j] < 0.0 ? erp * xi[j] : xi[j];
        double un = corr / dt + dun;
        double ut[3] = {du[0] - dun * n[0], du[1] - dun * n[1], du[2] - dun * n[2]};
        double P[3] = {px[j], py[j], pz[j]};
        double Pn = n[0] * P[0] + n[1] * P[1] + n[2] * P[2];
        double Pt[3] = {P[0] - Pn * n[0], P[1] - Pn * n[1], P[2] - Pn * n[2]};
        double et[3], eo[3];
        contact_frame(n, ut, Pt, 1e-9 * vs, 1e-9 * ms * vs, et, eo);
        double wn = im1 + im2;
        double wt = wn + ii1 * a1[j] * a1[j] + ii2 * a2[j] * a2[j];
        double *f = feat + NF * j;
        f[0] = un / vs;
        f[1] = (ut[0] * et[0] + ut[1] * et[1] + ut[2] * et[2]) / vs;
        f[2] = (ut[0] * eo[0] + ut[1] * eo[1] + ut[2] * eo[2]) / vs;
        f[3] = xi[j] / rs;
        f[4] = wn * ms;
        f[5] = wt * ms;
        f[6] = radius[b1] / rs;
        f[7] = r2 / rs;
        f[8] = mu;
        f[9] = Pn / (ms * vs);
        f[10] = (P[0] * et[0] + P[1] * et[1] + P[2] * et[2]) / (ms * vs);
        f[11] = (P[0] * eo[0] + P[1] * eo[1] + P[2] * eo[2]) / (ms * vs);
        double *fr = frame + 9 * j;
        for (int a = 0; a < 3; ++a) {
            fr[a] = n[a];
            fr[3 + a] = et[a];
            fr[6 + a] = eo[a];
        }
    }
}

/* Network output y (frame components scaled by ms vs) -> world impulse,
 * projected onto the cone (P_n >= 0, |P_t| <= mu P_n).  The learned start of
 * a contact that the previous step also had (matched[j] != 0) is its
 * previous impulse P0 (the initial solution may be the previous step's
 * reactions, Sect. 5); the network supplies the start of new contacts only.
 * matched may be NULL (every contact decoded). */
void nbgs_ref_mlp_decode(int64_t nc, const double *y, const double *frame, double ms, double vs, double mu,
                         const int32_t *matched, const double *p0x, const double *p0y, const double *p0z, double *px,
                         double *py, double *pz)
{
    for (int64_t j = 0; j < nc; ++j) {
        if (matched && matched[j]) {
            px[j] = p0x[j];
            py[j] = p0y[j];
            pz[j] = p0z[j];
            continue;
        }
        const double *fr = frame + 9 * j;
        double s = ms * vs;
        double pn = y[NO * j + 0] * s, pt = y[NO * j + 1] * s, po = y[NO * j + 2] * s;
        if (pn < 0.0) pn = 0.0;
        double tl = sqrt(pt * pt + po * po);
        double lim = mu * pn;
        if (tl > lim) {
            double k = tl > 0.0 ? lim / tl : 0.0;
            pt = pt * k;
            po = po * k;
        }
        px[j] = pn * fr[0] + pt * fr[3] + po * fr[6];
        py[j] = pn * fr[1] + pt * fr[4] + po * fr[7];
        pz[j] = pn * fr[2] + pt * fr[5] + po * fr[8];
    }
}

/* Training target of a contact: its solved impulse P in the contact frame,
 * scaled by 1/(ms vs). */
void nbgs_ref_mlp_targets(int64_t nc, const double *frame, const double *px, const double *py, const double *pz,
                          double ms, double vs, double *t)
{
    for (int64_t j = 0; j < nc; ++j) {
        const double *fr = frame + 9 * j;
        double P[3] = {px[j], py[j], pz[j]};
        for (int c = 0; c < 3; ++c)
            t[NO * j + c] = (P[0] * fr[3 * c + 0] + P[1] * fr[3 * c + 1] + P[2] * fr[3 * c + 2]) / (ms * vs);
    }
}
