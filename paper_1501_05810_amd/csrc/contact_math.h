// The one-contact relaxation shared by every sweep kernel (the colour-ordered
// sweeps and the block-local pass), so that all of them agree bit for bit.
//
// Body record {v'x, v'y, v'z, w'x, w'y, w'z, 1/m, 1/I} of the velocity
// accumulators (Sect. 6.3).  Relaxing contact j (Alg. 1, eqs. (nonpenetration)
// and (coulomb)):
//   du   = v'1 - v'2 - (a1 w'1 + a2 w'2) x n      relative contact velocity
//   u_n  = xi'/dt + n.du,  u_t = du - (n.du) n
//   W    = diag(w_n, w_t, w_t),  w_n = 1/m1 + 1/m2,  w_t = w_n + a1^2/I1 + a2^2/I2
//   b    = u - W P_j                               own impulse taken out
//   P*_n = max(0, -b_n / w_n);  P*_t = -b_t / w_t, scaled onto |P*_t| <= mu P*_n
//   P_j <- omega P* + (1 - omega) P_j; the change is applied to both bodies
//   (eq. (wrench)).
#pragma once

#include <hip/hip_runtime.h>

namespace nbgs {

template <class T>
struct Rec {
    T v[3], w[3], im, ii;
};

template <class T>
__device__ inline Rec<T> zero_rec() {
    Rec<T> r;
    r.v[0] = r.v[1] = r.v[2] = T(0);
    r.w[0] = r.w[1] = r.w[2] = T(0);
    r.im = r.ii = T(0);
    return r;
}

// Impulse change dP at the contact point: +dP on body 1 (arm -a1 n),
// -dP on body 2 (arm +a2 n), eq. (wrench).
template <class T>
__device__ inline void apply(Rec<T> &r1, Rec<T> &r2, const T n[3], T a1, T a2, const T dP[3]) {
    const T m0 = n[1] * dP[2] - n[2] * dP[1];
    const T m1 = n[2] * dP[0] - n[0] * dP[2];
    const T m2 = n[0] * dP[1] - n[1] * dP[0];
    r1.v[0] = r1.v[0] + r1.im * dP[0];
    r1.v[1] = r1.v[1] + r1.im * dP[1];
    r1.v[2] = r1.v[2] + r1.im * dP[2];
    r1.w[0] = r1.w[0] - r1.ii * a1 * m0;
    r1.w[1] = r1.w[1] - r1.ii * a1 * m1;
    r1.w[2] = r1.w[2] - r1.ii * a1 * m2;
    r2.v[0] = r2.v[0] - r2.im * dP[0];
    r2.v[1] = r2.v[1] - r2.im * dP[1];
    r2.v[2] = r2.v[2] - r2.im * dP[2];
    r2.w[0] = r2.w[0] - r2.ii * a2 * m0;
    r2.w[1] = r2.w[1] - r2.ii * a2 * m1;
    r2.w[2] = r2.w[2] - r2.ii * a2 * m2;
}

// Relaxation of one contact against the body records r1, r2 (which receive
// the impulse change): relative velocity at the contact point, the contact's
// own impulse taken out, the one-contact solution (normal clamp, radial
// projection onto the cone), relaxation.  One definition for every kernel
// variant, so that they agree bit for bit.
template <class T>
__device__ inline void relax_contact(const T nk[3], T bias, T a1, T a2, const T Pk[3], T mu, T relax, Rec<T> &r1,
                                     Rec<T> &r2, T Pnew[3], T dP[3]) {
    // relative velocity at the contact point
    const T s0 = a1 * r1.w[0] + a2 * r2.w[0];
    const T s1 = a1 * r1.w[1] + a2 * r2.w[1];
    const T s2 = a1 * r1.w[2] + a2 * r2.w[2];
    T du[3];
    du[0] = (r1.v[0] - r2.v[0]) - (s1 * nk[2] - s2 * nk[1]);
    du[1] = (r1.v[1] - r2.v[1]) - (s2 * nk[0] - s0 * nk[2]);
    du[2] = (r1.v[2] - r2.v[2]) - (s0 * nk[1] - s1 * nk[0]);
    const T dun = nk[0] * du[0] + nk[1] * du[1] + nk[2] * du[2];
    const T un = bias + dun;
    const T ut[3] = {du[0] - dun * nk[0], du[1] - dun * nk[1], du[2] - dun * nk[2]};
    // own impulse in the contact frame
    const T Pn = nk[0] * Pk[0] + nk[1] * Pk[1] + nk[2] * Pk[2];
    const T Pt[3] = {Pk[0] - Pn * nk[0], Pk[1] - Pn * nk[1], Pk[2] - Pn * nk[2]};
    const T wn = r1.im + r2.im;
    const T wt = wn + r1.ii * a1 * a1 + r2.ii * a2 * a2;
    const T bn = un - wn * Pn;
    const T bt[3] = {ut[0] - wt * Pt[0], ut[1] - wt * Pt[1], ut[2] - wt * Pt[2]};
    // one-contact solve: normal clamp, radial projection onto the cone
    T pn = -bn / wn;
    if (!(pn > T(0))) pn = T(0);
    T t0 = -bt[0] / wt, t1 = -bt[1] / wt, t2 = -bt[2] / wt;
    const T tl = sqrt(t0 * t0 + t1 * t1 + t2 * t2);
    const T lim = mu * pn;
    if (tl > lim) {
        const T sc = lim / tl;
        t0 = t0 * sc;
        t1 = t1 * sc;
        t2 = t2 * sc;
    }
    const T Ps[3] = {pn * nk[0] + t0, pn * nk[1] + t1, pn * nk[2] + t2};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        Pnew[a] = relax * Ps[a] + (T(1) - relax) * Pk[a];
        dP[a] = Pnew[a] - Pk[a];
    }
    apply(r1, r2, nk, a1, a2, dP);
}

}  // namespace nbgs
