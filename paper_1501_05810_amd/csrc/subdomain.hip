// Subdomain NBGS: Alg. 1 with the subdomain affinity s_c(j) = the block of
// the box that holds the centre of body j1 (domain partitioning, Sect. 6.1),
// in the velocity form of Sect. 6.3.
//
// One workgroup treats one subdomain per pass.  It copies the accumulated
// velocities of the bodies its contacts touch (its "slots") into LDS, zeroes
// their corrections, and relaxes its contacts colour by colour (a colouring
// restricted to the subdomain, so no two contacts of a colour share a slot);
// a contact sees accumulator + correction of its bodies, i.e. the newest
// impulses of the subdomain's contacts relaxed before it and the last
// iteration's impulses of all others.  The corrections are then written out
// per slot, and a second kernel adds them to the accumulators, body by body
// in ascending subdomain order.  The initial impulses enter the same way, as
// the corrections of a first pass.  Both orders of addition are fixed, so the
// result does not depend on scheduling.
//
// Per-step preparation: subdomain of every contact; the sweep order
// (subdomain, colour, key) from the colour sort; contact ranges per
// subdomain; slots = distinct (subdomain, dynamic body) pairs, found by
// sorting the contact ends by body and then, stably, by subdomain; each end's
// slot index local to its subdomain; per body the list of its slots in
// ascending subdomain.
#include <algorithm>

#include "scene.h"

namespace nbgs {

namespace {

constexpr int kBlock = 256;
constexpr int kMaxCol = 256;

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

struct Blocks {
    double lo[3], e[3];
    int32_t nb[3];
};

__global__ void __launch_bounds__(kBlock) k_subdomain(BodiesView b, const int32_t *j1, int64_t nc, Blocks bl,
                                                      int32_t *sdom) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nc) return;
    const int i = j1[j];
    const double x[3] = {b.x[i], b.y[i], b.z[i]};
    int64_t c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double f = floor((x[a] - bl.lo[a]) / bl.e[a]);
        f = fmax(0.0, fmin(f, (double)(bl.nb[a] - 1)));
        c[a] = (int64_t)f;
    }
    sdom[j] = (int32_t)((c[2] * bl.nb[1] + c[1]) * bl.nb[0] + c[0]);
}

__global__ void __launch_bounds__(kBlock) k_hist(const int32_t *v, int64_t n, int32_t *cnt) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) atomicAdd(&cnt[v[i]], 1);
}

__global__ void __launch_bounds__(kBlock) k_fill(int32_t *p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}

// Contact end e = 2 p + k (k = 0: j1, 1: j2) of sweep position p; its body if
// dynamic, else nb (sorts after every body).
__device__ inline int32_t end_body(const int32_t *sj1, const int32_t *sj2, int32_t nb, const double *inv_mass,
                                   uint32_t e) {
    const int32_t b = (e & 1u) ? sj2[e >> 1] : sj1[e >> 1];
    return (b < nb && inv_mass[b] > 0.0) ? b : nb;
}

__global__ void __launch_bounds__(kBlock) k_ends(const int32_t *sj1, const int32_t *sj2, int64_t nends, int32_t nb,
                                                 const double *inv_mass, uint32_t *keys, uint32_t *vals) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= nends) return;
    keys[e] = (uint32_t)end_body(sj1, sj2, nb, inv_mass, (uint32_t)e);
    vals[e] = (uint32_t)e;
}

__global__ void __launch_bounds__(kBlock) k_end_tiles(const uint32_t *vals, int64_t n, const int32_t *ssd,
                                                      uint32_t *keys) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) keys[i] = (uint32_t)ssd[vals[i] >> 1];
}

// First end of every (subdomain, dynamic body) group, ends sorted by (subdomain, body).
__global__ void __launch_bounds__(kBlock) k_slot_flags(const uint32_t *vals, int64_t n, const int32_t *sj1,
                                                       const int32_t *sj2, const int32_t *ssd, int32_t nb,
                                                       const double *inv_mass, int32_t *flags) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t e = vals[i];
    const int32_t b = end_body(sj1, sj2, nb, inv_mass, e);
    int f = 0;
    if (b < nb) {
        if (i == 0) {
            f = 1;
        } else {
            const uint32_t e0 = vals[i - 1];
            f = (ssd[e0 >> 1] != ssd[e >> 1] || end_body(sj1, sj2, nb, inv_mass, e0) != b) ? 1 : 0;
        }
    }
    flags[i] = f;
}

__global__ void __launch_bounds__(kBlock) k_slot_write(const uint32_t *vals, int64_t n, const int32_t *sj1,
                                                       const int32_t *sj2, const int32_t *ssd, int32_t nb,
                                                       const double *inv_mass, const int32_t *flags,
                                                       const int32_t *ex, int32_t *slot_body, int32_t *slot_sdom) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n || !flags[i]) return;
    const uint32_t e = vals[i];
    slot_body[ex[i]] = end_body(sj1, sj2, nb, inv_mass, e);
    slot_sdom[ex[i]] = ssd[e >> 1];
}

// Local slot of every contact end (-1: wall or static body).
__global__ void __launch_bounds__(kBlock) k_end_slots(const uint32_t *vals, int64_t n, const int32_t *sj1,
                                                      const int32_t *sj2, const int32_t *ssd, int32_t nb,
                                                      const double *inv_mass, const int32_t *flags,
                                                      const int32_t *ex, const int32_t *tile_slot_off,
                                                      int32_t *ls) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t e = vals[i];
    const int32_t b = end_body(sj1, sj2, nb, inv_mass, e);
    ls[e] = b < nb ? ex[i] + flags[i] - 1 - tile_slot_off[ssd[e >> 1]] : -1;
}

__global__ void __launch_bounds__(kBlock) k_iota(uint32_t *v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) v[i] = (uint32_t)i;
}

__global__ void __launch_bounds__(kBlock) k_copy_u32(const int32_t *a, int64_t n, uint32_t *b) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) b[i] = (uint32_t)a[i];
}

// ----------------------------------------------------------------- passes

template <class T>
struct Rec6 {
    T v[3], w[3];
};

// mode 0: the initial impulses become corrections; mode 1: relax (Alg. 1).
template <class T, int MODE>
__global__ void __launch_bounds__(kBlock) k_sub_pass(SubView<T> sv, int32_t nb, const T *vel, T mu, T relax,
                                                     const int64_t *tile_off, const int32_t *tile_slot_off,
                                                     const int32_t *slot_body, T *corr, double *partials,
                                                     const int32_t *ctrl) {
    if (MODE == 1 && ctrl[0]) return;  // an earlier sweep met the target (uniform over the grid)
    extern __shared__ __align__(16) unsigned char smem[];
    const int s = blockIdx.x;
    const int64_t c0 = tile_off[s], c1 = tile_off[s + 1];
    const int s0 = tile_slot_off[s], ns = tile_slot_off[s + 1] - s0;
    T *Vs = reinterpret_cast<T *>(smem);  // [6][ns] accumulators, then [6][ns] corrections, [ns] 1/m, [ns] 1/I
    T *Ds = Vs + 6 * ns;
    T *IM = Ds + 6 * ns;
    T *II = IM + ns;
    __shared__ int64_t cstart[kMaxCol + 1];
    __shared__ int ncol;
    for (int i = threadIdx.x; i < ns; i += kBlock) {
        const T *r = vel + 8 * (int64_t)slot_body[s0 + i];
#pragma unroll
        for (int a = 0; a < 6; ++a) {
            Vs[a * ns + i] = r[a];
            Ds[a * ns + i] = T(0);
        }
        IM[i] = r[6];
        II[i] = r[7];
    }
    // colour ranges of the subdomain's contacts (sorted by colour)
    for (int c = threadIdx.x; c <= kMaxCol; c += kBlock) cstart[c] = c1;
    if (threadIdx.x == 0) ncol = 0;
    __syncthreads();
    for (int64_t p = c0 + threadIdx.x; p < c1; p += kBlock) {
        const int cp = sv.col[p];
        if (p == c0 || sv.col[p - 1] != cp) cstart[cp] = p;
        if (p == c1 - 1) ncol = cp + 1;
    }
    __syncthreads();
    if (threadIdx.x == 0)  // empty colours start where the next one does
        for (int c = ncol - 1; c >= 0; --c)
            if (cstart[c] == c1 && c + 1 <= kMaxCol) cstart[c] = cstart[c + 1];
    __syncthreads();
    double sd = 0.0, sp = 0.0;
    for (int c = 0; c < ncol; ++c) {
        const int64_t pa = cstart[c], pb = c + 1 < ncol ? cstart[c + 1] : c1;
        for (int64_t p = pa + threadIdx.x; p < pb; p += kBlock) {
            const int l1 = sv.ls[2 * p], l2 = sv.ls[2 * p + 1];
            const int b1 = sv.j1[p], b2 = sv.j2[p];
            const T n[3] = {sv.nx[p], sv.ny[p], sv.nz[p]};
            const T a1 = sv.a1[p], a2 = sv.a2[p];
            const T P[3] = {sv.px[p], sv.py[p], sv.pz[p]};
            // velocities seen: accumulator + correction of a slot; a static body's record (never corrected: + 0);
            // a wall: zero
            Rec6<T> u1, u2;
            T im1, ii1, im2 = T(0), ii2 = T(0);
            if (l1 >= 0) {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    u1.v[a] = Vs[a * ns + l1] + Ds[a * ns + l1];
                    u1.w[a] = Vs[(3 + a) * ns + l1] + Ds[(3 + a) * ns + l1];
                }
                im1 = IM[l1];
                ii1 = II[l1];
            } else {
                const T *r = vel + 8 * (int64_t)b1;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    u1.v[a] = r[a] + T(0);
                    u1.w[a] = r[3 + a] + T(0);
                }
                im1 = r[6];
                ii1 = r[7];
            }
            if (l2 >= 0) {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    u2.v[a] = Vs[a * ns + l2] + Ds[a * ns + l2];
                    u2.w[a] = Vs[(3 + a) * ns + l2] + Ds[(3 + a) * ns + l2];
                }
                im2 = IM[l2];
                ii2 = II[l2];
            } else if (b2 < nb) {
                const T *r = vel + 8 * (int64_t)b2;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    u2.v[a] = r[a] + T(0);
                    u2.w[a] = r[3 + a] + T(0);
                }
                im2 = r[6];
                ii2 = r[7];
            } else {
#pragma unroll
                for (int a = 0; a < 3; ++a) u2.v[a] = u2.w[a] = T(0);
            }
            T dP[3];
            if (MODE == 0) {
                if (P[0] == T(0) && P[1] == T(0) && P[2] == T(0)) continue;
                dP[0] = P[0];
                dP[1] = P[1];
                dP[2] = P[2];
            } else {
                const T s0 = a1 * u1.w[0] + a2 * u2.w[0];
                const T s1 = a1 * u1.w[1] + a2 * u2.w[1];
                const T s2 = a1 * u1.w[2] + a2 * u2.w[2];
                T du[3];
                du[0] = (u1.v[0] - u2.v[0]) - (s1 * n[2] - s2 * n[1]);
                du[1] = (u1.v[1] - u2.v[1]) - (s2 * n[0] - s0 * n[2]);
                du[2] = (u1.v[2] - u2.v[2]) - (s0 * n[1] - s1 * n[0]);
                const T dun = n[0] * du[0] + n[1] * du[1] + n[2] * du[2];
                const T un = sv.bias[p] + dun;
                const T ut[3] = {du[0] - dun * n[0], du[1] - dun * n[1], du[2] - dun * n[2]};
                const T Pn = n[0] * P[0] + n[1] * P[1] + n[2] * P[2];
                const T Pt[3] = {P[0] - Pn * n[0], P[1] - Pn * n[1], P[2] - Pn * n[2]};
                const T wn = im1 + im2;
                const T wt = wn + ii1 * a1 * a1 + ii2 * a2 * a2;
                const T bn = un - wn * Pn;
                const T bt[3] = {ut[0] - wt * Pt[0], ut[1] - wt * Pt[1], ut[2] - wt * Pt[2]};
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
                const T Ps[3] = {pn * n[0] + t0, pn * n[1] + t1, pn * n[2] + t2};
                T Pnew[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    Pnew[a] = relax * Ps[a] + (T(1) - relax) * P[a];
                    dP[a] = Pnew[a] - P[a];
                }
                sv.px[p] = Pnew[0];
                sv.py[p] = Pnew[1];
                sv.pz[p] = Pnew[2];
                const double d0 = dP[0], d1 = dP[1], d2 = dP[2];
                const double q0 = Pnew[0], q1 = Pnew[1], q2 = Pnew[2];
                sd += d0 * d0 + d1 * d1 + d2 * d2;
                sp += q0 * q0 + q1 * q1 + q2 * q2;
            }
            // corrections (eq. (wrench)): +dP on j1 at arm -a1 n, -dP on j2 at arm +a2 n
            const T m0 = n[1] * dP[2] - n[2] * dP[1];
            const T m1 = n[2] * dP[0] - n[0] * dP[2];
            const T m2 = n[0] * dP[1] - n[1] * dP[0];
            if (l1 >= 0 && im1 > T(0)) {
                Ds[0 * ns + l1] = Ds[0 * ns + l1] + im1 * dP[0];
                Ds[1 * ns + l1] = Ds[1 * ns + l1] + im1 * dP[1];
                Ds[2 * ns + l1] = Ds[2 * ns + l1] + im1 * dP[2];
                Ds[3 * ns + l1] = Ds[3 * ns + l1] - ii1 * a1 * m0;
                Ds[4 * ns + l1] = Ds[4 * ns + l1] - ii1 * a1 * m1;
                Ds[5 * ns + l1] = Ds[5 * ns + l1] - ii1 * a1 * m2;
            }
            if (l2 >= 0 && im2 > T(0)) {
                Ds[0 * ns + l2] = Ds[0 * ns + l2] - im2 * dP[0];
                Ds[1 * ns + l2] = Ds[1 * ns + l2] - im2 * dP[1];
                Ds[2 * ns + l2] = Ds[2 * ns + l2] - im2 * dP[2];
                Ds[3 * ns + l2] = Ds[3 * ns + l2] - ii2 * a2 * m0;
                Ds[4 * ns + l2] = Ds[4 * ns + l2] - ii2 * a2 * m1;
                Ds[5 * ns + l2] = Ds[5 * ns + l2] - ii2 * a2 * m2;
            }
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < ns; i += kBlock)
#pragma unroll
        for (int a = 0; a < 6; ++a) corr[6 * (int64_t)(s0 + i) + a] = Ds[a * ns + i];
    if (MODE == 1) {
        __shared__ double red[2][kBlock / 64];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            sd += __shfl_xor(sd, o, 64);
            sp += __shfl_xor(sp, o, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            red[0][threadIdx.x >> 6] = sd;
            red[1][threadIdx.x >> 6] = sp;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double a = 0.0, c = 0.0;
#pragma unroll
            for (int w = 0; w < kBlock / 64; ++w) {
                a += red[0][w];
                c += red[1][w];
            }
            partials[2 * s + 0] = a;
            partials[2 * s + 1] = c;
        }
    }
}

// Accumulators + corrections of every slot of the body, in ascending subdomain.
template <class T>
__global__ void __launch_bounds__(kBlock) k_sub_reduce(T *vel, int32_t nb, const int32_t *body_slot_off,
                                                       const uint32_t *body_slots, const T *corr,
                                                       const int32_t *ctrl, int mode) {
    if (mode == 1 && ctrl[0]) return;
    const int b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= nb) return;
    const int q0 = body_slot_off[b], q1 = body_slot_off[b + 1];
    if (q0 == q1) return;
    T *r = vel + 8 * (int64_t)b;
    T v[6];
#pragma unroll
    for (int a = 0; a < 6; ++a) v[a] = r[a];
    for (int q = q0; q < q1; ++q) {
        const T *d = corr + 6 * (int64_t)body_slots[q];
#pragma unroll
        for (int a = 0; a < 6; ++a) v[a] = v[a] + d[a];
    }
#pragma unroll
    for (int a = 0; a < 6; ++a) r[a] = v[a];
}

}  // namespace

// Subdomains of the contacts and, when the colouring is done, the tile and slot tables.
nbgs_status subdomain_assign(nbgs_scene_t sc) {
    hipStream_t s = sc->s;
    Blocks bl;
    int64_t nsub = 1;
    for (int a = 0; a < 3; ++a) {
        const double L = sc->hi[a] - sc->lo[a];
        double c = std::floor(L / sc->sub_edge);
        if (!(c >= 1.0)) c = 1.0;
        if (c > 4096.0) c = 4096.0;
        bl.lo[a] = sc->lo[a];
        bl.nb[a] = (int32_t)c;
        bl.e[a] = L / c;
        nsub *= (int64_t)c;
    }
    if (nsub > (1 << 23)) {
        set_error("%lld subdomains are too many: use a larger edge", (long long)nsub);
        return NBGS_ERR_INVALID_ARG;
    }
    sc->n_sub = (int32_t)nsub;
    const int64_t nc = sc->nc;
    NBGS_TRY(sc->sdom.reserve((size_t)nc + 1));
    k_subdomain<<<grid_for(nc), kBlock, 0, s>>>(sc->b, sc->cb[sc->cur].j1.p, nc, bl, sc->sdom.p);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

template <class T>
static nbgs_status prepare_impl(nbgs_scene_t sc) {
    hipStream_t s = sc->s;
    const int64_t nc = sc->nc;
    const int32_t N = sc->b.n;
    const int32_t nsub = sc->n_sub;
    SweepBuf<T> &sw = sc->precision_used == NBGS_FP32_SWEEP ? *reinterpret_cast<SweepBuf<T> *>(&sc->sw32)
                                                            : *reinterpret_cast<SweepBuf<T> *>(&sc->sw64);
    const int32_t *sj1 = sw.j1.p, *sj2 = sw.j2.p, *ssd = sw.sdom.p;
    // contact ranges per subdomain
    NBGS_TRY(sc->tile_cnt.reserve((size_t)nsub + 1));
    NBGS_TRY(sc->tile_off.reserve((size_t)nsub + 1));
    k_fill<<<grid_for(nsub + 1), kBlock, 0, s>>>(sc->tile_cnt.p, nsub + 1, 0);
    k_hist<<<grid_for(nc), kBlock, 0, s>>>(ssd, nc, sc->tile_cnt.p);
    NBGS_HIP(hipGetLastError());
    const size_t need_tmp = exclusive_scan_tmp_bytes(std::max<int64_t>(2 * nc, (int64_t)N) + 2);
    if (need_tmp > sc->scan_tmp.cap) NBGS_TRY(sc->scan_tmp.reserve(need_tmp));
    // contact ends sorted by body, then stably by subdomain
    const int64_t ne = 2 * nc;
    for (DevBuf<uint32_t> *b : {&sc->ekeys, &sc->evals, &sc->ekeys2, &sc->evals2}) NBGS_TRY(b->reserve((size_t)ne + 1));
    if ((size_t)radix_hist_entries(ne) > sc->radix_hist.cap) NBGS_TRY(sc->radix_hist.reserve(radix_hist_entries(ne)));
    const size_t need_tmp2 = exclusive_scan_tmp_bytes((int64_t)radix_hist_entries(ne));
    if (need_tmp2 > sc->scan_tmp.cap) NBGS_TRY(sc->scan_tmp.reserve(need_tmp2));
    k_ends<<<grid_for(ne), kBlock, 0, s>>>(sj1, sj2, ne, N, sc->b.inv_mass, sc->ekeys.p, sc->evals.p);
    NBGS_HIP(hipGetLastError());
    auto bits_for = [](int64_t n) {
        int b = 0;
        while (((int64_t)1 << b) < n) ++b;
        return b;
    };
    bool alt = false;
    NBGS_TRY(radix_sort_pairs(sc->ekeys.p, sc->evals.p, sc->ekeys2.p, sc->evals2.p, ne, bits_for((int64_t)N + 1),
                              sc->radix_hist.p, sc->scan_tmp.p, sc->scan_tmp.cap, &alt, s));
    uint32_t *vals = alt ? sc->evals2.p : sc->evals.p;
    uint32_t *keys = alt ? sc->ekeys2.p : sc->ekeys.p;
    uint32_t *vals_o = alt ? sc->evals.p : sc->evals2.p;
    uint32_t *keys_o = alt ? sc->ekeys.p : sc->ekeys2.p;
    k_end_tiles<<<grid_for(ne), kBlock, 0, s>>>(vals, ne, ssd, keys);
    NBGS_HIP(hipGetLastError());
    bool alt2 = false;
    NBGS_TRY(radix_sort_pairs(keys, vals, keys_o, vals_o, ne, std::max(1, bits_for(nsub)), sc->radix_hist.p,
                              sc->scan_tmp.p, sc->scan_tmp.cap, &alt2, s));
    const uint32_t *svals = alt2 ? vals_o : vals;
    // slots
    NBGS_TRY(sc->eflags.reserve((size_t)ne + 1));
    NBGS_TRY(sc->eex.reserve((size_t)ne + 1));
    k_slot_flags<<<grid_for(ne), kBlock, 0, s>>>(svals, ne, sj1, sj2, ssd, N, sc->b.inv_mass, sc->eflags.p);
    NBGS_HIP(hipGetLastError());
    NBGS_TRY(exclusive_scan_i32(sc->eflags.p, sc->eex.p, ne, sc->total(), sc->scan_tmp.p, sc->scan_tmp.cap, s));
    NBGS_TRY(scene_sync_small(sc, 0, 1));
    const int64_t nslots = sc->pinned[0];
    sc->n_slots = nslots;
    NBGS_TRY(sc->slot_body.reserve((size_t)nslots + 1));
    NBGS_TRY(sc->slot_sdom.reserve((size_t)nslots + 1));
    k_slot_write<<<grid_for(ne), kBlock, 0, s>>>(svals, ne, sj1, sj2, ssd, N, sc->b.inv_mass, sc->eflags.p, sc->eex.p,
                                                 sc->slot_body.p, sc->slot_sdom.p);
    NBGS_HIP(hipGetLastError());
    NBGS_TRY(sc->tile_scnt.reserve((size_t)nsub + 1));
    NBGS_TRY(sc->tile_slot_off.reserve((size_t)nsub + 1));
    k_fill<<<grid_for(nsub + 1), kBlock, 0, s>>>(sc->tile_scnt.p, nsub + 1, 0);
    k_hist<<<grid_for(nslots), kBlock, 0, s>>>(sc->slot_sdom.p, nslots, sc->tile_scnt.p);
    NBGS_HIP(hipGetLastError());
    NBGS_TRY(exclusive_scan_i32(sc->tile_scnt.p, sc->tile_slot_off.p, (int64_t)nsub + 1, nullptr, sc->scan_tmp.p,
                                sc->scan_tmp.cap, s));
    NBGS_TRY(sw.ls.reserve((size_t)ne + 1));
    k_end_slots<<<grid_for(ne), kBlock, 0, s>>>(svals, ne, sj1, sj2, ssd, N, sc->b.inv_mass, sc->eflags.p, sc->eex.p,
                                                sc->tile_slot_off.p, sw.ls.p);
    NBGS_HIP(hipGetLastError());
    // per body its slots in ascending subdomain (slots are numbered in (subdomain, body) order)
    for (DevBuf<uint32_t> *b : {&sc->bkeys, &sc->bvals, &sc->bkeys2, &sc->bvals2})
        NBGS_TRY(b->reserve((size_t)nslots + 1));
    if (nslots == 0) {
        set_error("no dynamic body in any subdomain");
        return NBGS_ERR_STATE;
    }
    k_copy_u32<<<grid_for(nslots), kBlock, 0, s>>>(sc->slot_body.p, nslots, sc->bkeys.p);
    k_iota<<<grid_for(nslots), kBlock, 0, s>>>(sc->bvals.p, nslots);
    NBGS_HIP(hipGetLastError());
    bool alt3 = false;
    NBGS_TRY(radix_sort_pairs(sc->bkeys.p, sc->bvals.p, sc->bkeys2.p, sc->bvals2.p, nslots, bits_for((int64_t)N + 1),
                              sc->radix_hist.p, sc->scan_tmp.p, sc->scan_tmp.cap, &alt3, s));
    sc->body_slots = alt3 ? sc->bvals2.p : sc->bvals.p;
    if (nslots <= 1) sc->body_slots = sc->bvals.p;
    NBGS_TRY(sc->body_cnt.reserve((size_t)N + 1));
    NBGS_TRY(sc->body_slot_off.reserve((size_t)N + 1));
    k_fill<<<grid_for((int64_t)N + 1), kBlock, 0, s>>>(sc->body_cnt.p, (int64_t)N + 1, 0);
    k_hist<<<grid_for(nslots), kBlock, 0, s>>>(sc->slot_body.p, nslots, sc->body_cnt.p);
    NBGS_HIP(hipGetLastError());
    NBGS_TRY(exclusive_scan_i32(sc->body_cnt.p, sc->body_slot_off.p, (int64_t)N + 1, nullptr, sc->scan_tmp.p,
                                sc->scan_tmp.cap, s));
    // tile sizes against the kernel's limits
    std::vector<int32_t> cnt((size_t)nsub), scnt((size_t)nsub);
    NBGS_HIP(hipMemcpyAsync(cnt.data(), sc->tile_cnt.p, sizeof(int32_t) * nsub, hipMemcpyDeviceToHost, s));
    NBGS_HIP(hipMemcpyAsync(scnt.data(), sc->tile_scnt.p, sizeof(int32_t) * nsub, hipMemcpyDeviceToHost, s));
    NBGS_HIP(hipStreamSynchronize(s));
    int32_t max_slots = 0;
    for (int32_t t = 0; t < nsub; ++t) max_slots = std::max(max_slots, scnt[(size_t)t]);
    const size_t lds = (size_t)max_slots * 14 * sizeof(T);
    if (lds > 60 * 1024) {
        set_error("a subdomain touches %d bodies (%zu bytes of LDS); use a smaller subdomain edge", max_slots, lds);
        return NBGS_ERR_CAPACITY;
    }
    sc->max_slots = max_slots;
    // 64-bit contact offsets of the tiles
    std::vector<int64_t> toff((size_t)nsub + 1, 0);
    for (int32_t t = 0; t < nsub; ++t) toff[(size_t)t + 1] = toff[(size_t)t] + cnt[(size_t)t];
    NBGS_HIP(hipMemcpyAsync(sc->tile_off.p, toff.data(), sizeof(int64_t) * (nsub + 1), hipMemcpyHostToDevice, s));
    NBGS_HIP(hipStreamSynchronize(s));  // toff is a host temporary
    return NBGS_OK;
}

nbgs_status subdomain_prepare(nbgs_scene_t sc) {
    if (sc->precision_used == NBGS_FP32_SWEEP) return prepare_impl<float>(sc);
    return prepare_impl<double>(sc);
}

template <class T>
nbgs_status subdomain_pass(nbgs_scene_t sc, int mode, T *vel, T *corr) {
    hipStream_t s = sc->s;
    SweepBuf<T> &sw = sc->precision_used == NBGS_FP32_SWEEP ? *reinterpret_cast<SweepBuf<T> *>(&sc->sw32)
                                                            : *reinterpret_cast<SweepBuf<T> *>(&sc->sw64);
    SubView<T> v;
    v.j1 = sw.j1.p;
    v.j2 = sw.j2.p;
    v.ls = sw.ls.p;
    v.col = sw.col.p;
    v.nx = sw.nx.p;
    v.ny = sw.ny.p;
    v.nz = sw.nz.p;
    v.bias = sw.bias.p;
    v.a1 = sw.a1.p;
    v.a2 = sw.a2.p;
    v.px = sw.px.p;
    v.py = sw.py.p;
    v.pz = sw.pz.p;
    const size_t lds = (size_t)std::max(sc->max_slots, 1) * 14 * sizeof(T);
    const unsigned grid = (unsigned)sc->n_sub;
    const T mu = (T)sc->p.mu, relax = (T)sc->p.relax;
    if (mode == 0)
        k_sub_pass<T, 0><<<grid, kBlock, lds, s>>>(v, sc->b.n, vel, mu, relax, sc->tile_off.p, sc->tile_slot_off.p,
                                                   sc->slot_body.p, corr, sc->partials.p, sc->ctrl());
    else
        k_sub_pass<T, 1><<<grid, kBlock, lds, s>>>(v, sc->b.n, vel, mu, relax, sc->tile_off.p, sc->tile_slot_off.p,
                                                   sc->slot_body.p, corr, sc->partials.p, sc->ctrl());
    NBGS_HIP(hipGetLastError());
    k_sub_reduce<T><<<grid_for(sc->b.n), kBlock, 0, s>>>(vel, sc->b.n, sc->body_slot_off.p, sc->body_slots, corr,
                                                         sc->ctrl(), mode);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

template nbgs_status subdomain_pass<double>(nbgs_scene_t, int, double *, double *);
template nbgs_status subdomain_pass<float>(nbgs_scene_t, int, float *, float *);

}  // namespace nbgs
