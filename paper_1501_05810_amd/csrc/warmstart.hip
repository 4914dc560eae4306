// Learned warm start around the MLP: per-contact features, decoding of the
// network output into an initial impulse, training targets, and the residual
// that judges an initial impulse.
//
// Features (FP64 arithmetic, stored FP32) of contact j at the start of a step,
// from the accumulators before any impulse (v0 = v + dt g for dynamic bodies,
// w0 = w) and the previous-step impulse P0 re-projected onto the new cone,
// in the frame (n, e_t, e_o):
//   e_t along the tangential relative velocity u_t if it is not negligible,
//   else along the tangential part of P0, else n x (world axis least aligned
//   with n); e_o = n x e_t.
//   f0 = u_n / vs (u_n = xi'/dt + n.du), f1 = u_t.e_t / vs, f2 = u_t.e_o / vs,
//   f3 = xi / rs, f4 = w_n ms, f5 = w_t ms, f6 = r_j1 / rs, f7 = r_j2 / rs
//   (0 for a wall), f8 = mu, f9..f11 = (P0.n, P0.e_t, P0.e_o) / (ms vs).
// The network output y is the initial impulse in that frame scaled by
// 1 / (ms vs); it is projected onto the friction cone after decoding.
#include "nbgs_internal.h"

namespace nbgs {

namespace {

constexpr int kBlock = 256;
inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

__device__ inline void frame_of(const double n[3], const double ut[3], const double Pt[3], double vtiny, double ptiny,
                                double et[3], double eo[3]) {
    const double lu = sqrt(ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2]);
    const double lp = sqrt(Pt[0] * Pt[0] + Pt[1] * Pt[1] + Pt[2] * Pt[2]);
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
        const double e0 = a == 0 ? 1.0 : 0.0, e1 = a == 1 ? 1.0 : 0.0, e2 = a == 2 ? 1.0 : 0.0;
        const double c0 = n[1] * e2 - n[2] * e1, c1 = n[2] * e0 - n[0] * e2, c2 = n[0] * e1 - n[1] * e0;
        const double lc = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
        et[0] = c0 / lc;
        et[1] = c1 / lc;
        et[2] = c2 / lc;
    }
    eo[0] = n[1] * et[2] - n[2] * et[1];
    eo[1] = n[2] * et[0] - n[0] * et[2];
    eo[2] = n[0] * et[1] - n[1] * et[0];
}

__global__ void __launch_bounds__(kBlock) k_features(BodiesView b, ContactsView c, int64_t nc, double gx, double gy,
                                                     double gz, double dt, double mu, double erp, FeatureScales fs,
                                                     float *feat, double *frame) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nc) return;
    const int b1 = c.j1[j], b2 = c.j2[j];
    const double n[3] = {c.nx[j], c.ny[j], c.nz[j]};
    const double im1 = b.inv_mass[b1], ii1 = b.inv_inertia[b1];
    const bool dyn1 = im1 > 0.0;
    double v1[3], w1[3], v2[3] = {0.0, 0.0, 0.0}, w2[3] = {0.0, 0.0, 0.0};
    v1[0] = dyn1 ? b.vx[b1] + dt * gx : b.vx[b1];
    v1[1] = dyn1 ? b.vy[b1] + dt * gy : b.vy[b1];
    v1[2] = dyn1 ? b.vz[b1] + dt * gz : b.vz[b1];
    w1[0] = b.wx[b1];
    w1[1] = b.wy[b1];
    w1[2] = b.wz[b1];
    double im2 = 0.0, ii2 = 0.0, r2 = 0.0;
    if (b2 < b.n) {
        im2 = b.inv_mass[b2];
        ii2 = b.inv_inertia[b2];
        r2 = b.radius[b2];
        const bool dyn2 = im2 > 0.0;
        v2[0] = dyn2 ? b.vx[b2] + dt * gx : b.vx[b2];
        v2[1] = dyn2 ? b.vy[b2] + dt * gy : b.vy[b2];
        v2[2] = dyn2 ? b.vz[b2] + dt * gz : b.vz[b2];
        w2[0] = b.wx[b2];
        w2[1] = b.wy[b2];
        w2[2] = b.wz[b2];
    }
    const double a1 = c.a1[j], a2 = c.a2[j], xi = c.xi[j];
    const double s0 = a1 * w1[0] + a2 * w2[0];
    const double s1 = a1 * w1[1] + a2 * w2[1];
    const double s2 = a1 * w1[2] + a2 * w2[2];
    double du[3];
    du[0] = (v1[0] - v2[0]) - (s1 * n[2] - s2 * n[1]);
    du[1] = (v1[1] - v2[1]) - (s2 * n[0] - s0 * n[2]);
    du[2] = (v1[2] - v2[2]) - (s0 * n[1] - s1 * n[0]);
    const double dun = n[0] * du[0] + n[1] * du[1] + n[2] * du[2];
    const double corr = xi < 0.0 ? erp * xi : xi;
    const double un = corr / dt + dun;
    const double ut[3] = {du[0] - dun * n[0], du[1] - dun * n[1], du[2] - dun * n[2]};
    const double P[3] = {c.px[j], c.py[j], c.pz[j]};
    const double Pn = n[0] * P[0] + n[1] * P[1] + n[2] * P[2];
    const double Pt[3] = {P[0] - Pn * n[0], P[1] - Pn * n[1], P[2] - Pn * n[2]};
    double et[3], eo[3];
    frame_of(n, ut, Pt, 1e-9 * fs.vs, 1e-9 * fs.ms * fs.vs, et, eo);
    const double wn = im1 + im2;
    const double wt = wn + ii1 * a1 * a1 + ii2 * a2 * a2;
    float *f = feat + 12 * j;
    f[0] = (float)(un / fs.vs);
    f[1] = (float)((ut[0] * et[0] + ut[1] * et[1] + ut[2] * et[2]) / fs.vs);
    f[2] = (float)((ut[0] * eo[0] + ut[1] * eo[1] + ut[2] * eo[2]) / fs.vs);
    f[3] = (float)(xi / fs.rs);
    f[4] = (float)(wn * fs.ms);
    f[5] = (float)(wt * fs.ms);
    f[6] = (float)(b.radius[b1] / fs.rs);
    f[7] = (float)(r2 / fs.rs);
    f[8] = (float)mu;
    f[9] = (float)(Pn / (fs.ms * fs.vs));
    f[10] = (float)((P[0] * et[0] + P[1] * et[1] + P[2] * et[2]) / (fs.ms * fs.vs));
    f[11] = (float)((P[0] * eo[0] + P[1] * eo[1] + P[2] * eo[2]) / (fs.ms * fs.vs));
    double *fr = frame + 9 * j;
    for (int a = 0; a < 3; ++a) {
        fr[a] = n[a];
        fr[3 + a] = et[a];
        fr[6 + a] = eo[a];
    }
}

// The learned start of a contact the previous step also had is its previous
// impulse (Sect. 5); the network supplies the start of new contacts.
__global__ void __launch_bounds__(kBlock) k_decode(const float *y, const double *frame, ContactsView c, int64_t nc,
                                                   FeatureScales fs, double mu, double *px, double *py, double *pz) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nc) return;
    if (c.matched[j]) {
        px[j] = c.px[j];
        py[j] = c.py[j];
        pz[j] = c.pz[j];
        return;
    }
    const double *fr = frame + 9 * j;
    const double s = fs.ms * fs.vs;
    double pn = (double)y[3 * j + 0] * s, pt = (double)y[3 * j + 1] * s, po = (double)y[3 * j + 2] * s;
    if (!(pn > 0.0)) pn = 0.0;
    const double tl = sqrt(pt * pt + po * po);
    const double lim = mu * pn;
    if (tl > lim) {
        const double k = tl > 0.0 ? lim / tl : 0.0;
        pt = pt * k;
        po = po * k;
    }
    px[j] = pn * fr[0] + pt * fr[3] + po * fr[6];
    py[j] = pn * fr[1] + pt * fr[4] + po * fr[7];
    pz[j] = pn * fr[2] + pt * fr[5] + po * fr[8];
}

__global__ void __launch_bounds__(kBlock) k_targets(const double *frame, ContactsView c, int64_t nc, FeatureScales fs,
                                                    float *t) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nc) return;
    const double *fr = frame + 9 * j;
    const double P[3] = {c.px[j], c.py[j], c.pz[j]};
    for (int k = 0; k < 3; ++k)
        t[3 * j + k] = (float)((P[0] * fr[3 * k + 0] + P[1] * fr[3 * k + 1] + P[2] * fr[3 * k + 2]) / (fs.ms * fs.vs));
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_set_sweep_impulses(SweepView<T> sv, int64_t nc, const double *px,
                                                               const double *py, const double *pz) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= nc) return;
    const int j = sv.perm[p];
    sv.px[p] = (T)px[j];
    sv.py[p] = (T)py[j];
    sv.pz[p] = (T)pz[j];
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Jacobi residual of an initial impulse: every contact solves its
// one-contact problem against the same accumulators (nothing is written
// back); partial sums of |P* - P|^2 and |P*|^2 per block.
template <class T>
__global__ void __launch_bounds__(kBlock) k_jacobi(SweepView<T> sv, int64_t nc, int32_t nb, const T *vel, T mu,
                                                   double *partials) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double sd = 0.0, sp = 0.0;
    if (p < nc) {
        const int b1 = sv.j1[p], b2 = sv.j2[p];
        const T n[3] = {sv.nx[p], sv.ny[p], sv.nz[p]};
        const T a1 = sv.a1[p], a2 = sv.a2[p];
        const T P[3] = {sv.px[p], sv.py[p], sv.pz[p]};
        const T *r1 = vel + 8 * (int64_t)b1;
        T v2[3] = {T(0), T(0), T(0)}, w2[3] = {T(0), T(0), T(0)}, im2 = T(0), ii2 = T(0);
        if (b2 < nb) {
            const T *r2 = vel + 8 * (int64_t)b2;
            for (int a = 0; a < 3; ++a) {
                v2[a] = r2[a];
                w2[a] = r2[3 + a];
            }
            im2 = r2[6];
            ii2 = r2[7];
        }
        const T s0 = a1 * r1[3] + a2 * w2[0], s1 = a1 * r1[4] + a2 * w2[1], s2 = a1 * r1[5] + a2 * w2[2];
        const T du[3] = {(r1[0] - v2[0]) - (s1 * n[2] - s2 * n[1]), (r1[1] - v2[1]) - (s2 * n[0] - s0 * n[2]),
                         (r1[2] - v2[2]) - (s0 * n[1] - s1 * n[0])};
        const T dun = n[0] * du[0] + n[1] * du[1] + n[2] * du[2];
        const T un = sv.bias[p] + dun;
        const T ut[3] = {du[0] - dun * n[0], du[1] - dun * n[1], du[2] - dun * n[2]};
        const T Pn = n[0] * P[0] + n[1] * P[1] + n[2] * P[2];
        const T Pt[3] = {P[0] - Pn * n[0], P[1] - Pn * n[1], P[2] - Pn * n[2]};
        const T wn = r1[6] + im2;
        const T wt = wn + r1[7] * a1 * a1 + ii2 * a2 * a2;
        const T bn = un - wn * Pn;
        T pn = -bn / wn;
        if (!(pn > T(0))) pn = T(0);
        T t[3] = {-(ut[0] - wt * Pt[0]) / wt, -(ut[1] - wt * Pt[1]) / wt, -(ut[2] - wt * Pt[2]) / wt};
        const T tl = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
        if (tl > mu * pn) {
            const T k = mu * pn / tl;
            t[0] *= k;
            t[1] *= k;
            t[2] *= k;
        }
        for (int a = 0; a < 3; ++a) {
            const double ps = (double)(pn * n[a] + t[a]);
            const double d = ps - (double)P[a];
            sd += d * d;
            sp += ps * ps;
        }
    }
    __shared__ double red[2][kBlock / 64];
    sd = wave_sum(sd);
    sp = wave_sum(sp);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][wave] = sd;
        red[1][wave] = sp;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) {
            a += red[0][w];
            b += red[1][w];
        }
        partials[2 * blockIdx.x] = a;
        partials[2 * blockIdx.x + 1] = b;
    }
}

__global__ void __launch_bounds__(kBlock) k_ratio(const double *partials, int32_t n, double *out) {
    double a = 0.0, b = 0.0;
    for (int q = threadIdx.x; q < n; q += kBlock) {
        a += partials[2 * q];
        b += partials[2 * q + 1];
    }
    __shared__ double red[2][kBlock];
    red[0][threadIdx.x] = a;
    red[1][threadIdx.x] = b;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double den = sqrt(red[1][0]);
        *out = sqrt(red[0][0]) / (den > 1e-300 ? den : 1e-300);
    }
}

}  // namespace

nbgs_status launch_features(const BodiesView &b, const ContactsView &c, int64_t nc, const double g[3], double dt,
                            double mu, double erp, const FeatureScales &fs, float *feat, double *frame,
                            hipStream_t s) {
    if (nc == 0) return NBGS_OK;
    k_features<<<grid_for(nc), kBlock, 0, s>>>(b, c, nc, g[0], g[1], g[2], dt, mu, erp, fs, feat, frame);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

nbgs_status launch_decode(const float *y, const double *frame, const ContactsView &c, int64_t nc,
                          const FeatureScales &fs, double mu, double *px, double *py, double *pz, hipStream_t s) {
    if (nc == 0) return NBGS_OK;
    k_decode<<<grid_for(nc), kBlock, 0, s>>>(y, frame, c, nc, fs, mu, px, py, pz);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

nbgs_status launch_targets(const double *frame, const ContactsView &c, int64_t nc, const FeatureScales &fs, float *t,
                           hipStream_t s) {
    if (nc == 0) return NBGS_OK;
    k_targets<<<grid_for(nc), kBlock, 0, s>>>(frame, c, nc, fs, t);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

template <class T>
nbgs_status launch_set_sweep_impulses(SweepView<T> sv, int64_t nc, const double *px, const double *py,
                                      const double *pz, hipStream_t s) {
    if (nc == 0) return NBGS_OK;
    k_set_sweep_impulses<T><<<grid_for(nc), kBlock, 0, s>>>(sv, nc, px, py, pz);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

template <class T>
nbgs_status launch_jacobi_residual(SweepView<T> sv, int64_t nc, int32_t nb, const T *vel, double mu,
                                   double *partials, double *out, hipStream_t s) {
    const unsigned g = grid_for(nc > 0 ? nc : 1);
    k_jacobi<T><<<g, kBlock, 0, s>>>(sv, nc, nb, vel, (T)mu, partials);
    NBGS_HIP(hipGetLastError());
    k_ratio<<<1, kBlock, 0, s>>>(partials, (int32_t)g, out);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

template nbgs_status launch_set_sweep_impulses<double>(SweepView<double>, int64_t, const double *, const double *,
                                                       const double *, hipStream_t);
template nbgs_status launch_set_sweep_impulses<float>(SweepView<float>, int64_t, const double *, const double *,
                                                      const double *, hipStream_t);
template nbgs_status launch_jacobi_residual<double>(SweepView<double>, int64_t, int32_t, const double *, double,
                                                    double *, double *, hipStream_t);
template nbgs_status launch_jacobi_residual<float>(SweepView<float>, int64_t, int32_t, const float *, double,
                                                   double *, double *, hipStream_t);

}  // namespace nbgs
