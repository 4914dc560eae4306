// Composite particles: rigid clusters of element spheres.
//
// Sect. 2 builds non-spherical shapes from primitives glued rigidly together,
// and the granular gas of Sect. 7.2.1 uses particles of two to four spheres.
// A composite body carries its centre of mass, an orientation quaternion that
// maps its principal (body) frame to the world, a diagonal body-frame inertia
// and a list of element spheres in body coordinates.  One time step:
//
//   detection   every element is a sphere grown by its body's hull radius
//               h = dt (|v| + |w| rbar) + tau (eq. (expansionradius), rbar the
//               bounding radius of the body); elements are binned on a cell
//               grid, radix sorted, and pairs of elements of different bodies
//               (and elements against walls) are tested as spheres
//               (eq. (contactpos)); the contact keeps its lever arms from the
//               two centres of mass;
//   colouring   as for spheres: no two contacts of a colour share a dynamic
//               body (several contacts may join the same two bodies); after
//               the first step the passes start from the previous colours;
//   init        v' = v + dt g, w' = w + dt I^-1 (-w x I w): the gyroscopic
//               term of eq. (integrationscheme), zero for spheres;
//   sweeps      per colour, per contact: relative velocity at the contact
//               point, the full 3x3 Delassus block
//               W = (1/m1 + 1/m2) 1 - [r1]x Iw1 [r1]x - [r2]x Iw2 [r2]x
//               (eq. (wrench)), and the exact one-contact solution of
//               eqs. (nonpenetration) and (coulomb): separate, stick, or slide
//               with the tangential multiplier found by safeguarded Newton steps;
//   integrate   as for spheres.
//
// Every contact is relaxed with the same operations in the same order as the
// plain definition, compiled without contraction, so results are bit-exact
// rather than close.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "nbgs_internal.h"

namespace nbgs {

struct CompBodies {  // borrowed caller arrays
    int32_t n;
    int64_t ne;
    double *x, *y, *z, *qw, *qx, *qy, *qz, *vx, *vy, *vz, *wx, *wy, *wz;
    const double *inv_mass, *inv_inertia, *bound;
    const int32_t *elem_start;
    const double *elem_offset, *elem_radius;
};

struct CompContactsView {
    int32_t *j1, *j2, *e1, *e2;
    uint64_t *key;
    double *nx, *ny, *nz, *xi, *r1x, *r1y, *r1z, *r2x, *r2y, *r2z;
    double *px, *py, *pz;
    int32_t *colour, *matched;
};

// Sweep-ordered record: ends, normal, bias, lever arms, impulse.
struct CompSweepView {
    int32_t *j1, *j2, *perm;
    double *nx, *ny, *nz, *bias, *r1x, *r1y, *r1z, *r2x, *r2y, *r2z, *px, *py, *pz;
};

namespace {

constexpr int kBlock = 256;
constexpr int kMaxCandidates = 1 << 18;

inline unsigned grid_for(int64_t n, int block = kBlock) { return (unsigned)((n + block - 1) / block); }

// Rotation matrix (row major) of the unit quaternion (w, x, y, z).
__device__ inline void rotation(double qw, double qx, double qy, double qz, double R[9]) {
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

__global__ void __launch_bounds__(kBlock) k_elem_body(const int32_t *elem_start, int32_t n, int32_t *ebody) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    for (int e = elem_start[i]; e < elem_start[i + 1]; ++e) ebody[e] = i;
}

// Per body: hull radius, rotation; per element: world offset R o and the
// grown sphere (centre x + R o, reach r + h, negative for a static body).
__global__ void __launch_bounds__(kBlock) k_hull(CompBodies b, double dt, double tau, double *h, double *owx,
                                                 double *owy, double *owz, double4 *ec,
                                                 unsigned long long *max_bits) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double rmax = 0.0;
    if (i < b.n) {
        const double speed = sqrt(b.vx[i] * b.vx[i] + b.vy[i] * b.vy[i] + b.vz[i] * b.vz[i]);
        const double spin = sqrt(b.wx[i] * b.wx[i] + b.wy[i] * b.wy[i] + b.wz[i] * b.wz[i]);
        const double hi = dt * (speed + spin * b.bound[i]) + tau;
        h[i] = hi;
        double R[9];
        rotation(b.qw[i], b.qx[i], b.qy[i], b.qz[i], R);
        const bool stat = b.inv_mass[i] == 0.0;
        for (int e = b.elem_start[i]; e < b.elem_start[i + 1]; ++e) {
            const double *o = b.elem_offset + 3 * (int64_t)e;
            const double o0 = R[0] * o[0] + R[1] * o[1] + R[2] * o[2];
            const double o1 = R[3] * o[0] + R[4] * o[1] + R[5] * o[2];
            const double o2 = R[6] * o[0] + R[7] * o[1] + R[8] * o[2];
            owx[e] = o0;
            owy[e] = o1;
            owz[e] = o2;
            const double reach = b.elem_radius[e] + hi;
            ec[e] = make_double4(b.x[i] + o0, b.y[i] + o1, b.z[i] + o2, stat ? -reach : reach);
            double rr = reach;
            if (!(rr == rr)) rr = __longlong_as_double(0x7ff0000000000000ll);  // NaN -> +inf: caught on the host
            rmax = fmax(rmax, rr);
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) rmax = fmax(rmax, __shfl_xor(rmax, o, 64));
    __shared__ double wmax[kBlock / 64];
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = rmax;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = wmax[0];
        for (int w = 1; w < kBlock / 64; ++w) m = fmax(m, wmax[w]);
        atomicMax(max_bits, (unsigned long long)__double_as_longlong(m));
    }
}

// Cell of an element centre.  A centre may lie outside the box by up to its
// body's bounding radius: periodic axes wrap it into [lo, hi), others clamp it
// into the border cells (partners within reach still land in a neighbour).
__device__ inline int elem_cell(double x, const Grid &g, int a) {
    double t = x - g.lo[a];
    if (g.periodic[a]) t = t - g.L[a] * floor(t / g.L[a]);
    double c = floor(t / g.edge[a]);
    c = fmax(0.0, fmin(c, (double)(g.dims[a] - 1)));  // NaN -> 0
    return (int)c;
}

__global__ void __launch_bounds__(kBlock) k_cell_keys(const double4 *ec, int64_t ne, Grid g, uint32_t *keys,
                                                      uint32_t *ids) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= ne) return;
    const double4 c = ec[e];
    const int cx = elem_cell(c.x, g, 0), cy = elem_cell(c.y, g, 1), cz = elem_cell(c.z, g, 2);
    keys[e] = (uint32_t)((cz * g.dims[1] + cy) * g.dims[0] + cx);
    ids[e] = (uint32_t)e;
}

__global__ void __launch_bounds__(kBlock) k_cells(int64_t ne, const uint32_t *skeys, const uint32_t *sids,
                                                  const double4 *ec, const int32_t *ebody, int4 *cells, uint32_t stamp,
                                                  double4 *sec, int32_t *sbody) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= ne) return;
    const uint32_t key = skeys[p];
    if (p == 0 || skeys[p - 1] != key) {
        cells[key].x = (int32_t)p;
        cells[key].z = (int)stamp;
    }
    if (p == ne - 1 || skeys[p + 1] != key) cells[key].y = (int32_t)(p + 1);
    const int e = (int)sids[p];
    sec[p] = ec[e];
    sbody[p] = ebody[e];
}

__device__ inline double min_image(double d, int periodic, double L) {
    if (!periodic) return d;
    if (d > 0.5 * L) return d - L;
    if (d < -0.5 * L) return d + L;
    return d;
}

// Partner elements f of element e (sorted position p, body A) on bodies B > A
// whose grown spheres meet it; the count variant returns -1 past
// kMaxCandidates and keeps the first `cap` partners found in out (the emit
// variant keeps all).
template <bool kEmit>
__device__ inline int visit_partners(const Grid &g, const uint32_t *skeys, const uint32_t *sids, const double4 *sec,
                                     const int32_t *sbody, const int4 *cells, uint32_t stamp, int p, int A, int32_t *out,
                                     int cap = 0) {
    const double4 me = sec[p];
    const uint32_t key = skeys[p];
    int c[3];
    c[0] = (int)(key % (uint32_t)g.dims[0]);
    const uint32_t t = key / (uint32_t)g.dims[0];
    c[1] = (int)(t % (uint32_t)g.dims[1]);
    c[2] = (int)(t / (uint32_t)g.dims[1]);
    int lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = g.dims[a] == 1 ? 0 : -1;
        hi[a] = g.dims[a] == 1 ? 0 : 1;
    }
    int m = 0, seen = 0;
    // the entries of one sorted range [q0, q1)
    auto scan = [&](int q0, int q1) -> bool {
        if (!kEmit) {
            seen += q1 - q0;
            if (seen > kMaxCandidates) return false;
        }
        for (int s = q0; s < q1; ++s) {
            const int B = sbody[s];
            const double4 o = sec[s];
            if (B <= A) continue;
            if (me.w < 0.0 && o.w < 0.0) continue;  // two static bodies
            const double ddx = min_image(me.x - o.x, g.periodic[0], g.L[0]);
            const double ddy = min_image(me.y - o.y, g.periodic[1], g.L[1]);
            const double ddz = min_image(me.z - o.z, g.periodic[2], g.L[2]);
            const double d2 = ddx * ddx + ddy * ddy + ddz * ddz;
            const double reach = fabs(me.w) + fabs(o.w);
            if (!(d2 <= reach * reach)) continue;
            if (kEmit || m < cap) out[m] = (int32_t)sids[s];
            ++m;
        }
        return true;
    };
    for (int dz = lo[2]; dz <= hi[2]; ++dz)
        for (int dy = lo[1]; dy <= hi[1]; ++dy) {
            int qy = c[1] + dy, qz = c[2] + dz;
            bool out_of_box = false;
            if (qy < 0 || qy >= g.dims[1]) {
                if (!g.periodic[1]) out_of_box = true;
                qy = qy < 0 ? qy + g.dims[1] : qy - g.dims[1];
            }
            if (qz < 0 || qz >= g.dims[2]) {
                if (!g.periodic[2]) out_of_box = true;
                qz = qz < 0 ? qz + g.dims[2] : qz - g.dims[2];
            }
            if (out_of_box) continue;
            const int row = (qz * g.dims[1] + qy) * g.dims[0];  // the row's cell at x = 0
            // consecutive x cells hold consecutive sorted entries, so unless the row wraps round a periodic x
            // axis its stamped cells form one range, from the first one's start to the last one's end (cells
            // between them without a stamp hold no entries)
            int xa = c[0] + lo[0], xb = c[0] + hi[0];
            bool wrap = false;
            if (xa < 0) {
                if (g.periodic[0]) wrap = true;
                else xa = 0;
            }
            if (xb >= g.dims[0]) {
                if (g.periodic[0]) wrap = true;
                else xb = g.dims[0] - 1;
            }
            if (!wrap) {
                int q0 = 0, q1 = 0;
                bool any = false;
#pragma unroll
                for (int x = 0; x < 3; ++x) {
                    const int cell = row + (xa + x <= xb ? xa + x : xa);  // past xb: a repeat, left unused
                    const int4 cr = cells[cell];
                    const uint32_t cs = (uint32_t)cr.z;
                    const int s0 = cr.x, s1 = cr.y;
                    if (xa + x > xb || cs != stamp) continue;
                    if (!any) q0 = s0;
                    q1 = s1;
                    any = true;
                }
                if (any && !scan(q0, q1)) return -1;
            } else {
                for (int dx = lo[0]; dx <= hi[0]; ++dx) {
                    int qx = c[0] + dx;
                    if (qx < 0) qx += g.dims[0];
                    else if (qx >= g.dims[0]) qx -= g.dims[0];
                    const int cell = row + qx;
                    // the cell's stamp and range are read together (one round trip); a range whose stamp is
                    // stale is left unused
                    const int4 cr = cells[cell];
                    const uint32_t cs = (uint32_t)cr.z;
                    const int q0 = cr.x, q1 = cr.y;
                    if (cs != stamp) continue;
                    if (!scan(q0, q1)) return -1;
                }
            }
        }
    return m;
}

__device__ inline bool plane_hit(const PlaneSet &pl, int w, const double4 &c, double r, double hA, double tau,
                                 double *gap_out) {
    const double s = pl.nrm[w][0] * (c.x - pl.p[w][0]) + pl.nrm[w][1] * (c.y - pl.p[w][1]) +
                     pl.nrm[w][2] * (c.z - pl.p[w][2]);
    const double gap = s - r;
    *gap_out = gap;
    return gap <= hA + tau;
}

// Workgroups are dispatched to the 8 XCDs in turn (b mod 8), each XCD with its
// own L2: this bijection hands XCD x a contiguous run of the tiles, so that the
// neighbour reads of an element find what its XCD's earlier workgroups loaded.
__device__ inline unsigned xcd_tile(unsigned b, unsigned nb) {
    const unsigned q = nb / 8, r = nb % 8, x = b % 8, l = b / 8;
    return x * q + (x < r ? x : r) + l;
}

// One thread per sorted position (elements of a cell search the same cells).
// cnt holds zeros (filled before the count): only elements with contacts are
// written, with their partner count and sorted position (the emit reads those
// of such elements alone).
__global__ void __launch_bounds__(kBlock) k_pair_count(int64_t ne, Grid g, PlaneSet pl, double tau,
                                                       const uint32_t *skeys, const uint32_t *sids,
                                                       const double4 *sec, const int32_t *sbody,
                                                       const double *erad, const double *h,
                                                       const int4 *cells, uint32_t stamp, int32_t *cnt,
                                                       int32_t *npart, int32_t *partners, int32_t *cellpos,
                                                       unsigned long long *total) {
    const int64_t p = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    unsigned long long m64 = 0;
    int over = 0;
    if (p < ne) {
        const int e = (int)sids[p];
        const int A = sbody[p];
        int m = visit_partners<false>(g, skeys, sids, sec, sbody, cells, stamp, (int)p, A,
                                      partners + (int64_t)kPartnerCap * e, kPartnerCap);
        if (m < 0) {
            over = 1;
            m = 0;
        }
        const int mp = m;
        const double4 me = sec[p];
        if (me.w >= 0.0 && pl.n > 0) {
            double gap;
            for (int w = 0; w < pl.n; ++w)
                if (plane_hit(pl, w, me, erad[e], h[A], tau, &gap)) ++m;
        }
        if (m > 0) {
            cnt[e] = m;
            npart[e] = mp;
            cellpos[e] = (int32_t)p;
        }
        m64 = (unsigned long long)m;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m64 += __shfl_xor(m64, o, 64);
    over = __any(over);
    __shared__ unsigned long long wsum[kBlock / 64];
    __shared__ int wover[kBlock / 64];
    if ((threadIdx.x & 63) == 0) {
        wsum[threadIdx.x >> 6] = m64;
        wover[threadIdx.x >> 6] = over;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        int ov = 0;
        for (int w = 0; w < kBlock / 64; ++w) {
            t += wsum[w];
            ov |= wover[w];
        }
        if (t) atomicAdd(&total[0], t);
        if (ov) atomicOr(&total[1], 1ull);
    }
}

// Ascending partner indices: insertion sort for short lists, heap sort above.
__device__ inline void sort_partners(int32_t *ks, int m) {
    if (m <= 32) {
        for (int a = 1; a < m; ++a) {
            const int v = ks[a];
            int t = a - 1;
            while (t >= 0 && ks[t] > v) {
                ks[t + 1] = ks[t];
                --t;
            }
            ks[t + 1] = v;
        }
        return;
    }
    auto sift = [ks](int root, int end) {
        const int v = ks[root];
        for (;;) {
            int child = 2 * root + 1;
            if (child >= end) break;
            if (child + 1 < end && ks[child + 1] > ks[child]) ++child;
            if (v >= ks[child]) break;
            ks[root] = ks[child];
            root = child;
        }
        ks[root] = v;
    };
    for (int r = m / 2 - 1; r >= 0; --r) sift(r, m);
    for (int e = m - 1; e > 0; --e) {
        const int top = ks[0];
        ks[0] = ks[e];
        ks[e] = top;
        sift(0, e);
    }
}

// One thread per element in index order: its segment of the canonical list,
// partners on higher bodies in ascending element index, then walls.  The
// partners come from the count's store when they all fit, else from a new
// search.
// Geometry of a pair (eq. (contactpos) for two spheres): n from c_f to c_e,
// xi = |c_e - c_f| - r_e - r_f, lever arms from the centres of mass
// r1 = R_A o_e - (r_e + xi) n, r2 = R_B o_f + r_f n.
__global__ void __launch_bounds__(kBlock) k_pair_emit(int64_t ne, int32_t nb, Grid g, PlaneSet pl, double tau,
                                                      const uint32_t *skeys, const uint32_t *sids,
                                                      const double4 *sec, const int32_t *sbody,
                                                      const int4 *cells, uint32_t stamp,
                                                      const int32_t *cnt, const int32_t *off,
                                                      const int32_t *npart, const int32_t *partners,
                                                      const int32_t *cellpos, const double4 *ec,
                                                      const int32_t *ebody, const double *erad, const double *h,
                                                      const double *owx, const double *owy, const double *owz,
                                                      CompContactsView c) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= ne || cnt[e] == 0) return;
    const int p = cellpos[e];
    const int A = ebody[e];
    const int base = off[e];
    int32_t *ks = c.e2 + base;
    int m = npart[e];
    if (m <= kPartnerCap) {
        const int32_t *kept = partners + (int64_t)kPartnerCap * e;
        for (int t = 0; t < m; ++t) ks[t] = kept[t];
    } else {
        m = visit_partners<true>(g, skeys, sids, sec, sbody, cells, stamp, p, A, ks);
    }
    sort_partners(ks, m);
    const double4 ce = ec[e];
    const double re = erad[e];
    const double oe[3] = {owx[e], owy[e], owz[e]};
    for (int t = 0; t < m; ++t) {
        const int f = ks[t];
        const int j = base + t;
        const double4 cf = ec[f];
        const double rf = erad[f];
        const double dx = min_image(ce.x - cf.x, g.periodic[0], g.L[0]);
        const double dy = min_image(ce.y - cf.y, g.periodic[1], g.L[1]);
        const double dz = min_image(ce.z - cf.z, g.periodic[2], g.L[2]);
        const double d2 = dx * dx + dy * dy + dz * dz;
        const double d = sqrt(d2);
        double n[3];
        if (d2 > 0.0) {
            n[0] = dx / d;
            n[1] = dy / d;
            n[2] = dz / d;
        } else {
            n[0] = 0.0;
            n[1] = 0.0;
            n[2] = 1.0;
        }
        const double xi = (d - re) - rf;
        const double a1 = re + xi;
        const double of[3] = {owx[f], owy[f], owz[f]};
        c.j1[j] = A;
        c.j2[j] = ebody[f];
        c.e1[j] = (int32_t)e;
        c.key[j] = ((uint64_t)(uint32_t)e << 32) | (uint64_t)(uint32_t)f;
        c.nx[j] = n[0];
        c.ny[j] = n[1];
        c.nz[j] = n[2];
        c.xi[j] = xi;
        c.r1x[j] = oe[0] - a1 * n[0];
        c.r1y[j] = oe[1] - a1 * n[1];
        c.r1z[j] = oe[2] - a1 * n[2];
        c.r2x[j] = of[0] + rf * n[0];
        c.r2y[j] = of[1] + rf * n[1];
        c.r2z[j] = of[2] + rf * n[2];
    }
    if (ce.w < 0.0) return;  // static body: no wall contacts
    int t = m;
    for (int w = 0; w < pl.n; ++w) {
        double gap;
        if (!plane_hit(pl, w, ce, re, h[A], tau, &gap)) continue;
        const int j = base + t++;
        const double n[3] = {pl.nrm[w][0], pl.nrm[w][1], pl.nrm[w][2]};
        const double a1 = re + gap;
        c.j1[j] = A;
        c.j2[j] = nb + w;
        c.e1[j] = (int32_t)e;
        c.e2[j] = (int32_t)(ne + w);
        c.key[j] = ((uint64_t)(uint32_t)e << 32) | (uint64_t)(uint32_t)(ne + w);
        c.nx[j] = n[0];
        c.ny[j] = n[1];
        c.nz[j] = n[2];
        c.xi[j] = gap;
        c.r1x[j] = oe[0] - a1 * n[0];
        c.r1y[j] = oe[1] - a1 * n[1];
        c.r1z[j] = oe[2] - a1 * n[2];
        c.r2x[j] = 0.0;
        c.r2y[j] = 0.0;
        c.r2z[j] = 0.0;
    }
}

// Segment of body i as j1 in the canonical list (its elements' segments are
// consecutive), for the colouring's body -> contacts lookup.
__global__ void __launch_bounds__(kBlock) k_segments(const int32_t *elem_start, int32_t n, const int32_t *off,
                                                     int32_t *off1, int32_t *cnt1) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int a = off[elem_start[i]], b = off[elem_start[i + 1]];
    off1[i] = a;
    cnt1[i] = b - a;
}

__global__ void __launch_bounds__(kBlock) k_gather(CompContactsView c, const int32_t *pos, int64_t nc, double dt,
                                                   double erp, CompSweepView sv) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nc) return;
    const int64_t p = pos[j];
    sv.perm[p] = (int32_t)j;
    sv.j1[p] = c.j1[j];
    sv.j2[p] = c.j2[j];
    sv.nx[p] = c.nx[j];
    sv.ny[p] = c.ny[j];
    sv.nz[p] = c.nz[j];
    const double xi = c.xi[j];
    const double corr = xi < 0.0 ? erp * xi : xi;  // scaled-down penetration correction (Sect. 3)
    sv.bias[p] = corr / dt;
    sv.r1x[p] = c.r1x[j];
    sv.r1y[p] = c.r1y[j];
    sv.r1z[p] = c.r1z[j];
    sv.r2x[p] = c.r2x[j];
    sv.r2y[p] = c.r2y[j];
    sv.r2z[p] = c.r2z[j];
    sv.px[p] = c.px[j];
    sv.py[p] = c.py[j];
    sv.pz[p] = c.pz[j];
}

// Accumulators and world inverse inertia Iw = R diag(ii) R^T (9 entries per
// body, row major).  vel record: v'(3), w'(3), 1/m, 0.  The gyroscopic term of
// eq. (integrationscheme), in the body frame: wb = R^T w, L = wb / ii,
// dwb = dt ii (-(wb x L)), w' = w + R dwb; skipped for static bodies and for
// bodies with any principal inverse moment zero.
__global__ void __launch_bounds__(kBlock) k_init(CompBodies b, double gx, double gy, double gz, double dt,
                                                 double *vel, double *iw) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= b.n) return;
    double R[9];
    rotation(b.qw[i], b.qx[i], b.qy[i], b.qz[i], R);
    const double *ii = b.inv_inertia + 3 * (int64_t)i;
    const double ii0 = ii[0], ii1 = ii[1], ii2 = ii[2];
    double *I = iw + 9 * (int64_t)i;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            I[3 * a + c] = (R[3 * a + 0] * ii0) * R[3 * c + 0] + (R[3 * a + 1] * ii1) * R[3 * c + 1] +
                           (R[3 * a + 2] * ii2) * R[3 * c + 2];
    const double im = b.inv_mass[i];
    const bool dyn = im > 0.0;
    double v[3], w[3];
    v[0] = dyn ? b.vx[i] + dt * gx : b.vx[i];
    v[1] = dyn ? b.vy[i] + dt * gy : b.vy[i];
    v[2] = dyn ? b.vz[i] + dt * gz : b.vz[i];
    w[0] = b.wx[i];
    w[1] = b.wy[i];
    w[2] = b.wz[i];
    if (dyn && ii0 > 0.0 && ii1 > 0.0 && ii2 > 0.0) {
        const double iv[3] = {ii0, ii1, ii2};
        double wb[3], L[3], gg[3], dwb[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) wb[k] = R[0 + k] * w[0] + R[3 + k] * w[1] + R[6 + k] * w[2];
#pragma unroll
        for (int k = 0; k < 3; ++k) L[k] = wb[k] / iv[k];
        gg[0] = -(wb[1] * L[2] - wb[2] * L[1]);
        gg[1] = -(wb[2] * L[0] - wb[0] * L[2]);
        gg[2] = -(wb[0] * L[1] - wb[1] * L[0]);
#pragma unroll
        for (int k = 0; k < 3; ++k) dwb[k] = dt * (iv[k] * gg[k]);
#pragma unroll
        for (int a = 0; a < 3; ++a) w[a] = w[a] + (R[3 * a + 0] * dwb[0] + R[3 * a + 1] * dwb[1] + R[3 * a + 2] * dwb[2]);
    }
    double *r = vel + 8 * (int64_t)i;
    r[0] = v[0];
    r[1] = v[1];
    r[2] = v[2];
    r[3] = w[0];
    r[4] = w[1];
    r[5] = w[2];
    r[6] = im;
    r[7] = 0.0;
}

__device__ inline void mat_vec(const double *M, const double x[3], double y[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) y[a] = M[3 * a + 0] * x[0] + M[3 * a + 1] * x[1] + M[3 * a + 2] * x[2];
}

__device__ inline double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// dP at lever arm r of body b with sign s (+1 for j1, -1 for j2):
// v += s m^-1 dP, w += s Iw (r x dP).
__device__ inline void apply_end(double *vel, const double *iw, int b, const double r[3], const double dP[3],
                                 bool plus) {
    double *rec = vel + 8 * (int64_t)b;
    const double im = rec[6];
    double m[3], t[3];
    m[0] = r[1] * dP[2] - r[2] * dP[1];
    m[1] = r[2] * dP[0] - r[0] * dP[2];
    m[2] = r[0] * dP[1] - r[1] * dP[0];
    mat_vec(iw + 9 * (int64_t)b, m, t);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (plus) {
            rec[a] = rec[a] + im * dP[a];
            rec[3 + a] = rec[3 + a] + t[a];
        } else {
            rec[a] = rec[a] - im * dP[a];
            rec[3 + a] = rec[3 + a] - t[a];
        }
    }
}

// Initial impulses in colour order (one launch per colour).
__global__ void __launch_bounds__(kBlock) k_warm(CompSweepView sv, int64_t begin, int64_t end, int32_t nb,
                                                 double *vel, const double *iw) {
    const int64_t p = begin + (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= end) return;
    const double P[3] = {sv.px[p], sv.py[p], sv.pz[p]};
    if (P[0] == 0.0 && P[1] == 0.0 && P[2] == 0.0) return;
    const int b1 = sv.j1[p], b2 = sv.j2[p];
    const double r1[3] = {sv.r1x[p], sv.r1y[p], sv.r1z[p]}, r2[3] = {sv.r2x[p], sv.r2y[p], sv.r2z[p]};
    if (vel[8 * (int64_t)b1 + 6] > 0.0) apply_end(vel, iw, b1, r1, P, true);
    if (b2 < nb && vel[8 * (int64_t)b2 + 6] > 0.0) apply_end(vel, iw, b2, r2, P, false);
}

// K = X^T (Iw X) with X = [r]x: the velocity at r caused by a unit impulse at
// r through the body's rotation.
__device__ inline void rot_block(const double r[3], const double *Iw, double K[9]) {
    const double X[9] = {0.0, -r[2], r[1], r[2], 0.0, -r[0], -r[1], r[0], 0.0};
    double A[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) A[3 * i + j] = Iw[3 * i + 0] * X[0 + j] + Iw[3 * i + 1] * X[3 + j] + Iw[3 * i + 2] * X[6 + j];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) K[3 * i + j] = X[0 + i] * A[0 + j] + X[3 + i] * A[3 + j] + X[6 + i] * A[6 + j];
}

// Sliding case for the multiplier lam of the constraint |p_t| = mu p_n: with
// M = B + lam 1, p_t = p_n alpha + beta, alpha = -M^-1 c, beta = -M^-1 b_t,
// p_n = -(b_n + c.beta) / (a + c.alpha).  Returns phi = |p_t| - mu p_n and
// its derivative in lam (d alpha = -M^-1 alpha, d beta = -M^-1 beta).
__device__ inline double slide_eval(const double Wc[6], const double bc[3], double mu, double lam, double *pn,
                                    double *pt0, double *pt1, double *dphi) {
    const double a = Wc[0], c0 = Wc[1], c1 = Wc[2], B00 = Wc[3], B01 = Wc[4], B11 = Wc[5];
    const double m00 = B00 + lam, m11 = B11 + lam;
    const double r = 1.0 / (m00 * m11 - B01 * B01);
    const double al0 = -(m11 * c0 - B01 * c1) * r;
    const double al1 = -(m00 * c1 - B01 * c0) * r;
    const double be0 = -(m11 * bc[1] - B01 * bc[2]) * r;
    const double be1 = -(m00 * bc[2] - B01 * bc[1]) * r;
    const double da0 = -(m11 * al0 - B01 * al1) * r;
    const double da1 = -(m00 * al1 - B01 * al0) * r;
    const double db0 = -(m11 * be0 - B01 * be1) * r;
    const double db1 = -(m00 * be1 - B01 * be0) * r;
    const double D = a + (c0 * al0 + c1 * al1);
    const double q = -(bc[0] + (c0 * be0 + c1 * be1)) / D;
    const double dq = (-(c0 * db0 + c1 * db1) - q * (c0 * da0 + c1 * da1)) / D;
    const double t0 = q * al0 + be0, t1 = q * al1 + be1;
    const double d0 = (dq * al0 + q * da0) + db0, d1 = (dq * al1 + q * da1) + db1;
    const double tl = sqrt(t0 * t0 + t1 * t1);
    *pn = q;
    *pt0 = t0;
    *pt1 = t1;
    *dphi = (tl > 0.0 ? (t0 * d0 + t1 * d1) / tl : 0.0) - mu * dq;
    return tl - mu * q;
}

// Exact solution of the one-contact problem in the contact frame: separate
// (b_n >= 0), frictionless, stick (unconstrained solution inside the cone),
// or slide: Newton steps on phi from lam = 0 kept inside the bracket of the
// points seen (bisection, or doubling the lower end while no point beyond the
// root is known), stopping when the correction falls below 2^-50 lam or a step
// no longer moves lam (40 steps at most); the impulse at the last lam is
// clipped onto the cone.
__device__ inline void one_contact(const double Wc[6], const double bc[3], double mu, double p[3]) {
    const double a = Wc[0], c0 = Wc[1], c1 = Wc[2], B00 = Wc[3], B01 = Wc[4], B11 = Wc[5];
    const double bn = bc[0], bt0 = bc[1], bt1 = bc[2];
    p[0] = 0.0;
    p[1] = 0.0;
    p[2] = 0.0;
    if (!(bn < 0.0)) return;
    if (!(mu > 0.0)) {
        p[0] = -bn / a;
        return;
    }
    const double i00 = B00 * B11 - B01 * B01;
    const double i01 = c1 * B01 - c0 * B11;
    const double i02 = c0 * B01 - c1 * B00;
    const double i11 = a * B11 - c1 * c1;
    const double i12 = c0 * c1 - a * B01;
    const double i22 = a * B00 - c0 * c0;
    const double det = a * i00 + c0 * i01 + c1 * i02;
    const double sn = -(i00 * bn + i01 * bt0 + i02 * bt1) / det;
    const double s0 = -(i01 * bn + i11 * bt0 + i12 * bt1) / det;
    const double s1 = -(i02 * bn + i12 * bt0 + i22 * bt1) / det;
    if (sn > 0.0 && sqrt(s0 * s0 + s1 * s1) <= mu * sn) {
        p[0] = sn;
        p[1] = s0;
        p[2] = s1;
        return;
    }
    double pn, pt0, pt1, dphi;
    double lo = 0.0, hi = INFINITY, lam = 0.0;
    for (int k = 0; k < 40; ++k) {
        const double phi = slide_eval(Wc, bc, mu, lam, &pn, &pt0, &pt1, &dphi);
        if (phi > 0.0) lo = lam;
        else hi = lam;
        const double step = phi / dphi;
        if (fabs(step) <= 0x1p-50 * lam) break;
        double next = lam - step;
        if (!(next > lo && next < hi)) next = hi < INFINITY ? 0.5 * (lo + hi) : (lo > 0.0 ? 2.0 * lo : B00 + B11);
        if (next == lam) break;
        lam = next;
    }
    slide_eval(Wc, bc, mu, lam, &pn, &pt0, &pt1, &dphi);
    if (!(pn > 0.0)) return;
    const double tl = sqrt(pt0 * pt0 + pt1 * pt1);
    const double lim = mu * pn;
    if (tl > lim) {
        const double s = lim / tl;
        pt0 = pt0 * s;
        pt1 = pt1 * s;
    }
    p[0] = pn;
    p[1] = pt0;
    p[2] = pt1;
}

// Right-handed frame (n, t, o): t = (n x e) / |n x e|, e the axis of the
// smallest |n_k| (lowest index on ties), o = n x t.
__device__ inline void tangent_frame(const double n[3], double t[3], double o[3]) {
    int k = 0;
    if (fabs(n[1]) < fabs(n[k])) k = 1;
    if (fabs(n[2]) < fabs(n[k])) k = 2;
    const double e[3] = {k == 0 ? 1.0 : 0.0, k == 1 ? 1.0 : 0.0, k == 2 ? 1.0 : 0.0};
    t[0] = n[1] * e[2] - n[2] * e[1];
    t[1] = n[2] * e[0] - n[0] * e[2];
    t[2] = n[0] * e[1] - n[1] * e[0];
    const double l = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    t[0] = t[0] / l;
    t[1] = t[1] / l;
    t[2] = t[2] / l;
    o[0] = n[1] * t[2] - n[2] * t[1];
    o[1] = n[2] * t[0] - n[0] * t[2];
    o[2] = n[0] * t[1] - n[1] * t[0];
}

// Contacts begin .. end - 1 of one colour (no two share a dynamic body), one
// thread each.  Workgroup b writes (sum |dP|^2, sum |P_new|^2) of its
// contacts to partials[2 b], [2 b + 1].  ctrl[0] != 0 (set by the residual
// kernel once the target is met) turns the remaining sweeps into no-ops.
__global__ void __launch_bounds__(kBlock) k_sweep(CompSweepView sv, int64_t begin, int64_t end, int32_t nb,
                                                  double *vel, const double *iw, double mu, double relax,
                                                  double *partials, const int32_t *ctrl) {
    if (ctrl[0]) return;  // the residual target was met after an earlier sweep
    const int64_t p = begin + (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double sdp = 0.0, sp = 0.0;
    if (p < end) {
        const int b1 = sv.j1[p], b2 = sv.j2[p];
        const double n[3] = {sv.nx[p], sv.ny[p], sv.nz[p]};
        const double r1[3] = {sv.r1x[p], sv.r1y[p], sv.r1z[p]}, r2[3] = {sv.r2x[p], sv.r2y[p], sv.r2z[p]};
        const double *V1 = vel + 8 * (int64_t)b1;
        double vp1[3], vp2[3] = {0.0, 0.0, 0.0};
        vp1[0] = V1[0] + (V1[4] * r1[2] - V1[5] * r1[1]);
        vp1[1] = V1[1] + (V1[5] * r1[0] - V1[3] * r1[2]);
        vp1[2] = V1[2] + (V1[3] * r1[1] - V1[4] * r1[0]);
        const double im1 = V1[6];
        double im2 = 0.0;
        double K1[9], K2[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, W[9];
        rot_block(r1, iw + 9 * (int64_t)b1, K1);
        if (b2 < nb) {
            const double *V2 = vel + 8 * (int64_t)b2;
            vp2[0] = V2[0] + (V2[4] * r2[2] - V2[5] * r2[1]);
            vp2[1] = V2[1] + (V2[5] * r2[0] - V2[3] * r2[2]);
            vp2[2] = V2[2] + (V2[3] * r2[1] - V2[4] * r2[0]);
            im2 = V2[6];
            rot_block(r2, iw + 9 * (int64_t)b2, K2);
        }
        const double wsum = im1 + im2;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int e = 0; e < 3; ++e) W[3 * a + e] = ((a == e ? wsum : 0.0) + K1[3 * a + e]) + K2[3 * a + e];
        const double bias = sv.bias[p];
        const double P[3] = {sv.px[p], sv.py[p], sv.pz[p]};
        double WP[3], bw[3];
        mat_vec(W, P, WP);
#pragma unroll
        for (int a = 0; a < 3; ++a) bw[a] = ((vp1[a] - vp2[a]) + bias * n[a]) - WP[a];
        double tt[3], oo[3];
        tangent_frame(n, tt, oo);
        double Wn[3], Wt[3], Wo[3];
        mat_vec(W, n, Wn);
        mat_vec(W, tt, Wt);
        mat_vec(W, oo, Wo);
        const double Wc[6] = {dot3(n, Wn), dot3(tt, Wn), dot3(oo, Wn), dot3(tt, Wt), dot3(tt, Wo), dot3(oo, Wo)};
        const double bc[3] = {dot3(n, bw), dot3(tt, bw), dot3(oo, bw)};
        double pc[3];
        one_contact(Wc, bc, mu, pc);
        double Pnew[3], dP[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double Ps = (pc[0] * n[a] + pc[1] * tt[a]) + pc[2] * oo[a];
            Pnew[a] = relax * Ps + (1.0 - relax) * P[a];
            dP[a] = Pnew[a] - P[a];
        }
        if (im1 > 0.0) apply_end(vel, iw, b1, r1, dP, true);
        if (b2 < nb && im2 > 0.0) apply_end(vel, iw, b2, r2, dP, false);
        sv.px[p] = Pnew[0];
        sv.py[p] = Pnew[1];
        sv.pz[p] = Pnew[2];
        sdp = dP[0] * dP[0] + dP[1] * dP[1] + dP[2] * dP[2];
        sp = Pnew[0] * Pnew[0] + Pnew[1] * Pnew[1] + Pnew[2] * Pnew[2];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        sdp += __shfl_xor(sdp, o, 64);
        sp += __shfl_xor(sp, o, 64);
    }
    __shared__ double red[2][kBlock / 64];
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = sdp;
        red[1][threadIdx.x >> 6] = sp;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, c = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) {
            a += red[0][w];
            c += red[1][w];
        }
        partials[2 * (int64_t)blockIdx.x] = a;
        partials[2 * (int64_t)blockIdx.x + 1] = c;
    }
}

__global__ void __launch_bounds__(kBlock) k_save(CompSweepView sv, int64_t nc, CompContactsView c) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= nc) return;
    const int j = sv.perm[p];
    c.px[j] = sv.px[p];
    c.py[j] = sv.py[p];
    c.pz[j] = sv.pz[p];
}

__global__ void __launch_bounds__(kBlock) k_export_contacts(CompContactsView c, int64_t nc, int64_t cap,
                                                            int32_t *j1, int32_t *j2, uint64_t *key,
                                                            int32_t *colour, double *imp, double *geo) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nc) return;
    if (j1) j1[j] = c.j1[j];
    if (j2) j2[j] = c.j2[j];
    if (key) key[j] = c.key[j];
    if (colour) colour[j] = c.colour[j];
    if (imp) {
        imp[j] = c.px[j];
        imp[cap + j] = c.py[j];
        imp[2 * cap + j] = c.pz[j];
    }
    if (geo) {
        const double g[10] = {c.nx[j], c.ny[j], c.nz[j], c.xi[j], c.r1x[j], c.r1y[j], c.r1z[j],
                              c.r2x[j], c.r2y[j], c.r2z[j]};
#pragma unroll
        for (int k = 0; k < 10; ++k) geo[k * cap + j] = g[k];
    }
}

struct CompContactBuf {
    DevBuf<int32_t> j1, j2, e1, e2, colour, matched;
    DevBuf<uint64_t> key;
    DevBuf<double> nx, ny, nz, xi, r1x, r1y, r1z, r2x, r2y, r2z, px, py, pz;
    nbgs_status reserve(size_t n) {
        for (DevBuf<int32_t> *b : {&j1, &j2, &e1, &e2, &colour, &matched}) NBGS_TRY(b->reserve(n));
        NBGS_TRY(key.reserve(n));
        for (DevBuf<double> *b : {&nx, &ny, &nz, &xi, &r1x, &r1y, &r1z, &r2x, &r2y, &r2z, &px, &py, &pz})
            NBGS_TRY(b->reserve(n));
        return NBGS_OK;
    }
    CompContactsView view() {
        return CompContactsView{j1.p,  j2.p,  e1.p,  e2.p,  key.p, nx.p, ny.p, nz.p,     xi.p,     r1x.p, r1y.p,
                                r1z.p, r2x.p, r2y.p, r2z.p, px.p,  py.p, pz.p, colour.p, matched.p};
    }
    // The fields the shared colouring and warm-start kernels read.
    ContactsView shared_view() {
        ContactsView v{};
        v.j1 = j1.p;
        v.j2 = j2.p;
        v.key = key.p;
        v.nx = nx.p;
        v.ny = ny.p;
        v.nz = nz.p;
        v.px = px.p;
        v.py = py.p;
        v.pz = pz.p;
        v.colour = colour.p;
        v.matched = matched.p;
        return v;
    }
};

struct CompSweepBuf {
    DevBuf<int32_t> j1, j2, perm;
    DevBuf<double> nx, ny, nz, bias, r1x, r1y, r1z, r2x, r2y, r2z, px, py, pz;
    nbgs_status reserve(size_t n) {
        for (DevBuf<int32_t> *b : {&j1, &j2, &perm}) NBGS_TRY(b->reserve(n));
        for (DevBuf<double> *b : {&nx, &ny, &nz, &bias, &r1x, &r1y, &r1z, &r2x, &r2y, &r2z, &px, &py, &pz})
            NBGS_TRY(b->reserve(n));
        return NBGS_OK;
    }
    CompSweepView view() {
        return CompSweepView{j1.p,  j2.p,  perm.p, nx.p,  ny.p,  nz.p, bias.p, r1x.p,
                             r1y.p, r1z.p, r2x.p,  r2y.p, r2z.p, px.p, py.p,   pz.p};
    }
};

enum { kPhDetect = 0, kPhColour, kPhInit, kPhSweeps, kPhIntegrate, kPhEnd, kPhN };

}  // namespace
}  // namespace nbgs

using namespace nbgs;

struct nbgs_composite_s {
    // device memory of the scene (the caller's workspace); first, so that it outlives every buffer carved from it
    Arena arena;
    int64_t nc_needed = -1;  // the contact count the last detection found (reported with CAPACITY)
    hipStream_t s = nullptr;
    CompBodies b{};
    BodiesView bv{};  // the body state as the shared integrator reads it
    PlaneSet planes{};
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    int32_t periodic[3] = {0, 0, 0};
    nbgs_params p{};
    Grid grid{};
    DevBuf<int4> cells;  // per cell (start, end, stamp, -) of its sorted range
    DevBuf<int32_t> ebody, sbody, cellpos, cnt, off, off1, cnt1, deg2, off2, cursor, inc2,
        radix_hist, spos, small, ctrl, npart, partners;
    DevBuf<uint8_t> dirty[2];  // colouring passes: the contacts a change reached (ping-pong)
    DevBuf<uint32_t> keys, ids, keys2, ids2, ckeys, cids, ckeys2, cids2;
    DevBuf<double4> ec, sec;
    DevBuf<double> h, owx, owy, owz, vel, iw, partials, hist;
    DevBuf<unsigned long long> maxbits;
    DevBuf<uint64_t> prio;
    DevBuf<unsigned char> scan_tmp;
    uint32_t stamp = 0;
    CompContactBuf cb[2];
    int cur = 0;
    bool table_in_cur = false;
    int64_t n_prev = 0;
    CompSweepBuf sw;
    int64_t nc = 0;
    int32_t n_colours = 0;
    std::vector<int64_t> col_off;
    int32_t *pinned = nullptr;  // host: [0] scan total, [1] remaining, [2] overflow, [4..7] two 64-bit words,
                                // [16..528) colour histogram, [600..) residual bytes
    int state = 0;              // 0: fresh or integrated, 1: detected, 2: solved
    nbgs_stats stats{};
    int32_t hist_n = 0;
    hipEvent_t ev[kPhN] = {};
    bool ev_ok[kPhN] = {};
};

// Upper bound of a composite scene's device memory (nbgs_composite_workspace_query):
// per element 352 B (its world offset, grown sphere, sorted copies, partner
// store, sort keys 192 B; cells of 16 B at most eight per element 160 B), per body
// 164 B (accumulator record, world inverse inertia, hull radius, colouring
// counters), per contact 525 B (two contact tables 272 B, the sweep record
// 116 B, colouring 32 B, times 1.25), a cell table of at least 2^16 cells and
// a fixed 16 MiB; ten per cent for alignment and the runs between freed
// buffers.
size_t composite_workspace_bytes(int64_t n, int64_t e, int64_t c) {
    const double b = 1.1 * (352.0 * (double)e + 164.0 * (double)n + 525.0 * (double)c + 65536.0 * 16.0 * 1.25 +
                            16.0 * 1024.0 * 1024.0);
    return ((size_t)b + Arena::kAlign - 1) & ~(size_t)(Arena::kAlign - 1);
}

namespace {

void record(nbgs_composite_t sc, int i) {
    if (sc->ev[i]) sc->ev_ok[i] = hipEventRecord(sc->ev[i], sc->s) == hipSuccess;
}

nbgs_status sync_small(nbgs_composite_t sc, int first, int count) {
    NBGS_HIP(hipMemcpyAsync(sc->pinned + first, sc->small.p + first, sizeof(int32_t) * count, hipMemcpyDeviceToHost,
                            sc->s));
    NBGS_HIP(hipStreamSynchronize(sc->s));
    return NBGS_OK;
}

nbgs_status comp_detect(nbgs_composite_t sc, nbgs_stats *stats) {
    hipStream_t s = sc->s;
    const int32_t N = sc->b.n;
    const int64_t E = sc->b.ne;
    record(sc, kPhDetect);
    if (sc->table_in_cur) {  // the solved impulses of the last step become the lookup table
        sc->cur = 1 - sc->cur;
        sc->table_in_cur = false;
    }
    CompContactBuf &prev = sc->cb[1 - sc->cur];
    NBGS_HIP(hipMemsetAsync(sc->maxbits.p, 0, 3 * sizeof(unsigned long long), s));
    k_hull<<<grid_for(N), kBlock, 0, s>>>(sc->b, sc->p.dt, sc->p.tau, sc->h.p, sc->owx.p, sc->owy.p, sc->owz.p,
                                          sc->ec.p, sc->maxbits.p);
    NBGS_HIP(hipGetLastError());
    NBGS_HIP(hipMemcpyAsync(sc->pinned + 4, sc->maxbits.p, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    NBGS_HIP(hipStreamSynchronize(s));
    double max_reach;
    std::memcpy(&max_reach, sc->pinned + 4, sizeof(max_reach));
    if (!std::isfinite(max_reach)) {
        set_error("non-finite velocity, orientation or radius in the body state");
        return NBGS_ERR_NUMERIC;
    }
    sc->grid = grid_for_box(sc->lo, sc->hi, sc->periodic, E, max_reach);
    const Grid g = sc->grid;
    k_cell_keys<<<grid_for(E), kBlock, 0, s>>>(sc->ec.p, E, g, sc->keys.p, sc->ids.p);
    NBGS_HIP(hipGetLastError());
    bool alt = false;
    NBGS_TRY(radix_sort_pairs(sc->keys.p, sc->ids.p, sc->keys2.p, sc->ids2.p, E, g.key_bits, sc->radix_hist.p,
                              sc->scan_tmp.p, sc->scan_tmp.cap, &alt, s));
    const uint32_t *skeys = alt ? sc->keys2.p : sc->keys.p;
    const uint32_t *sids = alt ? sc->ids2.p : sc->ids.p;
    if ((size_t)g.ncells > sc->cells.cap) {
        NBGS_TRY(sc->cells.reserve(g.ncells));
        NBGS_HIP(hipMemsetAsync(sc->cells.p, 0, sizeof(int4) * sc->cells.cap, s));
        sc->stamp = 0;
    }
    if (++sc->stamp == 0) {
        NBGS_HIP(hipMemsetAsync(sc->cells.p, 0, sizeof(int4) * sc->cells.cap, s));
        sc->stamp = 1;
    }
    k_cells<<<grid_for(E), kBlock, 0, s>>>(E, skeys, sids, sc->ec.p, sc->ebody.p, sc->cells.p, sc->stamp, sc->sec.p,
                                           sc->sbody.p);
    NBGS_HIP(hipGetLastError());
    NBGS_HIP(hipMemsetAsync(sc->cnt.p, 0, sizeof(int32_t) * (E + 1), s));  // zeros; cnt[E] makes off[E] the total
    k_pair_count<<<grid_for(E), kBlock, 0, s>>>(E, g, sc->planes, sc->p.tau, skeys, sids, sc->sec.p, sc->sbody.p,
                                                sc->b.elem_radius, sc->h.p, sc->cells.p, sc->stamp, sc->cnt.p,
                                                sc->npart.p, sc->partners.p, sc->cellpos.p, sc->maxbits.p + 1);
    NBGS_HIP(hipGetLastError());
    NBGS_TRY(exclusive_scan_i32(sc->cnt.p, sc->off.p, E + 1, sc->small.p, sc->scan_tmp.p, sc->scan_tmp.cap, s));
    NBGS_HIP(hipMemcpyAsync(sc->pinned + 4, sc->maxbits.p + 1, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                            s));
    NBGS_TRY(sync_small(sc, 0, 1));
    unsigned long long total64 = 0, over = 0;
    std::memcpy(&total64, sc->pinned + 4, sizeof(total64));
    std::memcpy(&over, sc->pinned + 6, sizeof(over));
    if (over) {
        set_error("an element meets more than 2^18 hull candidates in its 27 cells (largest grown element %g)",
                  max_reach);
        return NBGS_ERR_CAPACITY;
    }
    if (total64 > 0x7fffff00ull) {
        set_error("%llu contacts exceed the 2^31 entries of the contact list", (unsigned long long)total64);
        return NBGS_ERR_CAPACITY;
    }
    const int64_t nc = sc->pinned[0];
    if (nc != (int64_t)total64) {
        set_error("contact count %lld disagrees with its 64-bit total %llu", (long long)nc,
                  (unsigned long long)total64);
        return NBGS_ERR_DEVICE;
    }
    sc->nc_needed = nc;
    const size_t need = composite_workspace_bytes(N, E, nc);
    if (need > sc->arena.size()) {
        set_error("%lld contacts need a workspace of %zu bytes (nbgs_composite_workspace_query), this one has %zu",
                  (long long)nc, need, sc->arena.size());
        return NBGS_ERR_CAPACITY;
    }
    sc->nc_needed = -1;  // a later refusal (colours, block sizes) is not lifted by a larger workspace
    sc->nc = nc;
    CompContactBuf &cb = sc->cb[sc->cur];
    NBGS_TRY(cb.reserve((size_t)(nc > 0 ? nc : 1)));
    k_pair_emit<<<grid_for(E), kBlock, 0, s>>>(E, N, g, sc->planes, sc->p.tau, skeys, sids, sc->sec.p, sc->sbody.p,
                                               sc->cells.p, sc->stamp,
                                               sc->cnt.p, sc->off.p, sc->npart.p, sc->partners.p, sc->cellpos.p,
                                               sc->ec.p, sc->ebody.p,
                                               sc->b.elem_radius, sc->h.p, sc->owx.p, sc->owy.p, sc->owz.p, cb.view());
    NBGS_HIP(hipGetLastError());
    // initial impulses: the previous step's, matched by key and re-projected onto the new cone, else zero
    // and, when the previous step was coloured, its colours as the start of the colouring passes
    const bool warm = sc->p.warm_start == NBGS_WS_PREVIOUS && sc->n_prev > 0;
    const bool warm_colours = sc->n_prev > 0 && nc > 0;
    const SceneTable tab{};
    NBGS_TRY(launch_match_prev(cb.shared_view(), nc, prev.key.p, prev.px.p, prev.py.p, prev.pz.p, prev.colour.p,
                               sc->n_prev, sc->p.mu, tab, warm, warm_colours, nullptr, s));
    if (!warm && nc > 0) {
        NBGS_HIP(hipMemsetAsync(cb.px.p, 0, sizeof(double) * nc, s));
        NBGS_HIP(hipMemsetAsync(cb.py.p, 0, sizeof(double) * nc, s));
        NBGS_HIP(hipMemsetAsync(cb.pz.p, 0, sizeof(double) * nc, s));
    }
    record(sc, kPhColour);
    // colouring: per body its j1 segment and the contacts where it is j2
    k_segments<<<grid_for(N), kBlock, 0, s>>>(sc->b.elem_start, N, sc->off.p, sc->off1.p, sc->cnt1.p);
    NBGS_HIP(hipGetLastError());
    const ContactsView cv = cb.shared_view();
    NBGS_TRY(sc->inc2.reserve((size_t)(nc > 0 ? nc : 1)));
    NBGS_TRY(sc->prio.reserve((size_t)(nc > 0 ? nc : 1)));
    NBGS_TRY(launch_prio(cv, nc, sc->p.colour_seed, tab, N, sc->prio.p, s));
    NBGS_TRY(launch_j2_degree(cv, nc, N, sc->b.inv_mass, sc->deg2.p, s));
    NBGS_TRY(exclusive_scan_i32(sc->deg2.p, sc->off2.p, (int64_t)N + 1, nullptr, sc->scan_tmp.p, sc->scan_tmp.cap, s));
    NBGS_HIP(hipMemcpyAsync(sc->cursor.p, sc->off2.p, sizeof(int32_t) * ((size_t)N + 1), hipMemcpyDeviceToDevice, s));
    NBGS_TRY(launch_j2_fill(cv, nc, N, sc->b.inv_mass, sc->cursor.p, sc->inc2.p, s));
    if (warm_colours) {
        // the greedy rule repeated from the previous colours until a pass changes nothing: its fixed point is the
        // greedy colouring in priority order, the one the Jones-Plassmann rounds build from scratch; after the first
        // pass only the contacts a change reached are evaluated
        NBGS_TRY(sc->dirty[0].reserve((size_t)(nc > 0 ? nc : 1)));
        NBGS_TRY(sc->dirty[1].reserve((size_t)(nc > 0 ? nc : 1)));
        NBGS_HIP(hipMemsetAsync(sc->small.p + 2, 0, sizeof(int32_t), s));
        int pass = 0, batch = 1;
        for (;;) {
            for (int r = 0; r < batch; ++r, ++pass) {
                NBGS_HIP(hipMemsetAsync(sc->small.p + 1, 0, sizeof(int32_t), s));
                uint8_t *din = pass == 0 ? nullptr : sc->dirty[(pass + 1) & 1].p;
                NBGS_TRY(launch_colour_fix(cv, sc->prio.p, nc, N, sc->b.inv_mass, sc->off1.p, sc->cnt1.p, sc->off2.p,
                                           sc->inc2.p, nullptr, din, sc->dirty[pass & 1].p, sc->small.p + 1,
                                           sc->small.p + 2, true, s));
            }
            NBGS_TRY(sync_small(sc, 1, 2));
            if (sc->pinned[2]) {
                set_error("more than 255 colours needed");
                return NBGS_ERR_CAPACITY;
            }
            if (sc->pinned[1] == 0) break;
            if (pass > 100000) {
                set_error("colouring did not settle");
                return NBGS_ERR_DEVICE;
            }
            batch = batch < 8 ? 2 * batch : 8;
        }
    } else if (nc > 0) {
        NBGS_HIP(hipMemsetAsync(cb.colour.p, 0xff, sizeof(int32_t) * nc, s));
        sc->pinned[1] = (int32_t)nc;
        sc->pinned[2] = 0;
        NBGS_HIP(hipMemcpyAsync(sc->small.p + 1, sc->pinned + 1, 2 * sizeof(int32_t), hipMemcpyHostToDevice, s));
        int batch = 2, rounds = 0;
        for (;;) {
            for (int r = 0; r < batch; ++r)
                NBGS_TRY(launch_jp_round(cv, sc->prio.p, nc, N, sc->b.inv_mass, sc->off1.p, sc->cnt1.p, sc->off2.p,
                                         sc->inc2.p, nullptr, sc->small.p + 1, sc->small.p + 2, s));
            rounds += batch;
            NBGS_TRY(sync_small(sc, 1, 2));
            if (sc->pinned[2]) {
                set_error("more than 255 colours needed");
                return NBGS_ERR_CAPACITY;
            }
            if (sc->pinned[1] == 0) break;
            if (rounds > 100000) {
                set_error("colouring did not finish");
                return NBGS_ERR_DEVICE;
            }
            batch = batch < 8 ? batch * 2 : 8;
        }
    }
    NBGS_TRY(launch_colour_hist(cv, nc, N, sc->b.inv_mass, sc->small.p + 16, s));
    NBGS_TRY(sync_small(sc, 16, 512));
    sc->n_colours = 0;
    for (int c = 0; c < 256; ++c)
        if (sc->pinned[16 + c]) sc->n_colours = c + 1;
    sc->col_off.assign((size_t)sc->n_colours + 1, 0);
    for (int c = 0; c < sc->n_colours; ++c) sc->col_off[c + 1] = sc->col_off[c] + sc->pinned[16 + c];
    for (DevBuf<uint32_t> *bb : {&sc->ckeys, &sc->cids, &sc->ckeys2, &sc->cids2}) NBGS_TRY(bb->reserve((size_t)nc + 1));
    NBGS_TRY(launch_colour_keys(cv, nullptr, nc, sc->ckeys.p, sc->cids.p, s));
    if ((size_t)radix_hist_entries(nc) > sc->radix_hist.cap) NBGS_TRY(sc->radix_hist.reserve(radix_hist_entries(nc)));
    const size_t need_tmp = exclusive_scan_tmp_bytes((int64_t)radix_hist_entries(nc));
    if (need_tmp > sc->scan_tmp.cap) NBGS_TRY(sc->scan_tmp.reserve(need_tmp));
    bool calt = false;
    NBGS_TRY(radix_sort_pairs(sc->ckeys.p, sc->cids.p, sc->ckeys2.p, sc->cids2.p, nc, 8, sc->radix_hist.p,
                              sc->scan_tmp.p, sc->scan_tmp.cap, &calt, s));
    const uint32_t *perm = calt ? sc->cids2.p : sc->cids.p;
    if (nc == 1) perm = sc->cids.p;
    NBGS_TRY(sc->spos.reserve((size_t)nc + 1));
    NBGS_TRY(launch_invert(perm, nc, sc->spos.p, s));
    NBGS_TRY(sc->sw.reserve((size_t)(nc > 0 ? nc : 1)));
    if (nc > 0) {
        k_gather<<<grid_for(nc), kBlock, 0, s>>>(cb.view(), sc->spos.p, nc, sc->p.dt, sc->p.erp, sc->sw.view());
        NBGS_HIP(hipGetLastError());
    }
    sc->state = 1;
    sc->stats.n_contacts = nc;
    sc->stats.n_colours = sc->n_colours;
    sc->stats.sweeps = 0;
    sc->stats.residual = 0.0;
    record(sc, kPhInit);
    if (stats) *stats = sc->stats;
    return NBGS_OK;
}

nbgs_status comp_solve(nbgs_composite_t sc, int32_t max_sweeps, double target, nbgs_stats *stats) {
    if (sc->state != 1) {
        set_error(sc->state == 2 ? "already solved: integrate, then detect again" : "solve before detect");
        return NBGS_ERR_STATE;
    }
    if (max_sweeps < 0) {
        set_error("max_sweeps must be >= 0");
        return NBGS_ERR_INVALID_ARG;
    }
    hipStream_t s = sc->s;
    const int32_t N = sc->b.n;
    const int64_t nc = sc->nc;
    record(sc, kPhInit);
    k_init<<<grid_for(N), kBlock, 0, s>>>(sc->b, sc->p.gravity[0], sc->p.gravity[1], sc->p.gravity[2], sc->p.dt,
                                          sc->vel.p, sc->iw.p);
    NBGS_HIP(hipGetLastError());
    const CompSweepView sv = sc->sw.view();
    for (int c = 0; c < sc->n_colours; ++c) {
        const int64_t b0 = sc->col_off[c], b1 = sc->col_off[c + 1];
        if (b1 <= b0) continue;
        k_warm<<<grid_for(b1 - b0), kBlock, 0, s>>>(sv, b0, b1, N, sc->vel.p, sc->iw.p);
        NBGS_HIP(hipGetLastError());
    }
    record(sc, kPhSweeps);
    // residual partials: one pair per workgroup of every colour launch
    int64_t n_part = 0;
    std::vector<int64_t> part_off((size_t)sc->n_colours + 1, 0);
    for (int c = 0; c < sc->n_colours; ++c) {
        n_part += grid_for(sc->col_off[c + 1] - sc->col_off[c]);
        part_off[c + 1] = n_part;
    }
    NBGS_TRY(sc->partials.reserve((size_t)(2 * n_part + 2)));
    NBGS_TRY(sc->hist.reserve((size_t)max_sweeps + 1));
    NBGS_HIP(hipMemsetAsync(sc->ctrl.p, 0, 4 * sizeof(int32_t), s));
    int32_t done = 0;
    double R = 0.0;
    const int32_t check = 8;  // sweeps between host checks of the residual target
    for (int32_t k = 0; k < max_sweeps && nc > 0; ++k) {
        for (int c = 0; c < sc->n_colours; ++c) {
            const int64_t b0 = sc->col_off[c], b1 = sc->col_off[c + 1];
            if (b1 <= b0) continue;
            k_sweep<<<grid_for(b1 - b0), kBlock, 0, s>>>(sv, b0, b1, N, sc->vel.p, sc->iw.p, sc->p.mu, sc->p.relax,
                                                         sc->partials.p + 2 * part_off[c], sc->ctrl.p);
            NBGS_HIP(hipGetLastError());
        }
        NBGS_TRY(launch_residual(sc->partials.p, (int32_t)(n_part > 0 ? n_part : 1), target, sc->ctrl.p, sc->hist.p,
                                 s, k));
        done = k + 1;
        if (target > 0.0 && (done % check == 0 || done == max_sweeps)) {
            NBGS_HIP(hipMemcpyAsync(sc->pinned + 8, sc->ctrl.p, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            NBGS_HIP(hipStreamSynchronize(s));
            if (sc->pinned[8]) {
                done = sc->pinned[9];
                break;
            }
        }
    }
    if (nc == 0) done = max_sweeps;
    record(sc, kPhIntegrate);
    if (nc > 0) {
        k_save<<<grid_for(nc), kBlock, 0, s>>>(sv, nc, sc->cb[sc->cur].view());
        NBGS_HIP(hipGetLastError());
    }
    sc->hist_n = done;
    sc->state = 2;
    sc->stats.sweeps = done;
    sc->stats.residual = 0.0;
    if (stats || target > 0.0) {
        if (done > 0 && nc > 0) {
            NBGS_HIP(hipMemcpyAsync(sc->pinned + 600, sc->hist.p + (done - 1), sizeof(double), hipMemcpyDeviceToHost,
                                    s));
        }
        NBGS_HIP(hipMemcpyAsync(sc->pinned + 8, sc->ctrl.p, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        NBGS_HIP(hipStreamSynchronize(s));
        if (done > 0 && nc > 0) std::memcpy(&R, sc->pinned + 600, sizeof(double));
        sc->stats.residual = R;
        if (stats) *stats = sc->stats;
        if (sc->pinned[8 + 2]) {
            set_error("non-finite residual after sweep %d", done);
            return NBGS_ERR_NUMERIC;
        }
        if (target > 0.0 && nc > 0 && !(R <= target)) {
            set_error("residual %.3e above target %.3e after %d sweeps", R, target, done);
            return NBGS_ERR_NOT_CONVERGED;
        }
    }
    return NBGS_OK;
}

nbgs_status comp_integrate(nbgs_composite_t sc) {
    if (sc->state != 2) {
        set_error("integrate needs a solved step");
        return NBGS_ERR_STATE;
    }
    record(sc, kPhIntegrate);
    const SceneTable tab{};
    NBGS_TRY(launch_integrate<double>(sc->bv, sc->grid, tab, sc->p.dt, sc->vel.p, nullptr, sc->p.gravity, nullptr,
                                      sc->s));
    record(sc, kPhEnd);
    sc->table_in_cur = true;
    sc->n_prev = sc->nc;
    sc->state = 0;
    return NBGS_OK;
}

}  // namespace

// A NULL handle is refused; the handle's arena takes the buffers allocated
// until the entry point returns.
#define NBGS_CGUARD(sc)                                                                                         \
    if (!(sc)) {                                                                                                \
        set_error("composite scene handle is NULL");                                                            \
        return NBGS_ERR_INVALID_ARG;                                                                            \
    }                                                                                                           \
    ArenaScope arena_scope_(&(sc)->arena)

extern "C" {

nbgs_status nbgs_composite_workspace_query(int64_t n_bodies, int64_t n_elements, int64_t contact_capacity,
                                           const nbgs_params *params, size_t *bytes) {
    if (!bytes || n_bodies < 0 || n_elements < 0 || contact_capacity < 0) {
        set_error("bad arguments to nbgs_composite_workspace_query");
        return NBGS_ERR_INVALID_ARG;
    }
    if (params) NBGS_TRY(check_params(params));
    *bytes = composite_workspace_bytes(n_bodies, n_elements, contact_capacity);
    return NBGS_OK;
}

nbgs_status nbgs_composite_set_workspace(nbgs_composite_t sc, void *workspace, size_t bytes) {
    NBGS_CGUARD(sc);
    return sc->arena.move_to(workspace, bytes, sc->s);
}

nbgs_status nbgs_composite_create(const nbgs_composite_bodies *bodies, const nbgs_domain *domain,
                                  const nbgs_params *params, void *workspace, size_t workspace_bytes,
                                  void *hip_stream, nbgs_composite_t *out) {
    if (!out) {
        set_error("out is NULL");
        return NBGS_ERR_INVALID_ARG;
    }
    *out = nullptr;
    if (!bodies) {
        set_error("bodies is NULL");
        return NBGS_ERR_INVALID_ARG;
    }
    NBGS_TRY(check_params(params));
    NBGS_TRY(check_domain(domain));
    if (params->precision != NBGS_FP64) {
        set_error("composite particles are solved in FP64 only");
        return NBGS_ERR_UNSUPPORTED;
    }
    if (params->warm_start == NBGS_WS_LEARNED) {
        set_error("the learned warm start is not available for composite particles");
        return NBGS_ERR_UNSUPPORTED;
    }
    if (bodies->n < 1 || bodies->n >= (int64_t)0x7fffffc0 - domain->n_planes) {
        set_error("body count %lld out of range", (long long)bodies->n);
        return NBGS_ERR_INVALID_ARG;
    }
    if (bodies->n_elements < bodies->n || bodies->n_elements >= (int64_t)0x7fffffc0 - domain->n_planes) {
        set_error("element count %lld out of range (every body needs at least one element)",
                  (long long)bodies->n_elements);
        return NBGS_ERR_INVALID_ARG;
    }
    const void *ptrs[] = {bodies->x,  bodies->y,  bodies->z,  bodies->qw, bodies->qx, bodies->qy, bodies->qz,
                          bodies->vx, bodies->vy, bodies->vz, bodies->wx, bodies->wy, bodies->wz, bodies->inv_mass,
                          bodies->inv_inertia, bodies->bound, bodies->elem_start, bodies->elem_offset,
                          bodies->elem_radius};
    for (const void *q : ptrs)
        if (!q) {
            set_error("a body or element array pointer is NULL");
            return NBGS_ERR_INVALID_ARG;
        }
    nbgs_composite_t sc = new (std::nothrow) nbgs_composite_s();
    if (!sc) {
        set_error("host allocation failed");
        return NBGS_ERR_OUT_OF_MEMORY;
    }
    struct Guard {
        nbgs_composite_t sc;
        bool keep = false;
        ~Guard() {
            if (!keep) nbgs_composite_destroy(sc);
        }
    } guard{sc};
    sc->s = (hipStream_t)hip_stream;
    sc->arena.reset(workspace, workspace_bytes);
    if (!sc->arena.bound()) {
        set_error("the workspace is NULL or too small (nbgs_composite_workspace_query gives its size)");
        return NBGS_ERR_INVALID_ARG;
    }
    ArenaScope arena_scope(&sc->arena);
    CompBodies &b = sc->b;
    b.n = (int32_t)bodies->n;
    b.ne = bodies->n_elements;
    b.x = bodies->x;
    b.y = bodies->y;
    b.z = bodies->z;
    b.qw = bodies->qw;
    b.qx = bodies->qx;
    b.qy = bodies->qy;
    b.qz = bodies->qz;
    b.vx = bodies->vx;
    b.vy = bodies->vy;
    b.vz = bodies->vz;
    b.wx = bodies->wx;
    b.wy = bodies->wy;
    b.wz = bodies->wz;
    b.inv_mass = bodies->inv_mass;
    b.inv_inertia = bodies->inv_inertia;
    b.bound = bodies->bound;
    b.elem_start = bodies->elem_start;
    b.elem_offset = bodies->elem_offset;
    b.elem_radius = bodies->elem_radius;
    BodiesView &bv = sc->bv;
    bv.n = b.n;
    bv.x = b.x;
    bv.y = b.y;
    bv.z = b.z;
    bv.qw = b.qw;
    bv.qx = b.qx;
    bv.qy = b.qy;
    bv.qz = b.qz;
    bv.vx = b.vx;
    bv.vy = b.vy;
    bv.vz = b.vz;
    bv.wx = b.wx;
    bv.wy = b.wy;
    bv.wz = b.wz;
    bv.inv_mass = b.inv_mass;
    sc->planes = plane_set(domain);
    for (int a = 0; a < 3; ++a) {
        sc->lo[a] = domain->lo[a];
        sc->hi[a] = domain->hi[a];
        sc->periodic[a] = domain->periodic[a] ? 1 : 0;
    }
    sc->p = *params;
    const size_t N = (size_t)b.n, E = (size_t)b.ne;
    // the body -> elements ranges are checked on the host before any kernel indexes with them
    {
        std::vector<int32_t> es(N + 1);
        if (hipMemcpy(es.data(), b.elem_start, sizeof(int32_t) * (N + 1), hipMemcpyDeviceToHost) != hipSuccess) {
            set_error("elem_start is not readable device memory");
            return NBGS_ERR_INVALID_ARG;
        }
        if (es[0] != 0 || (int64_t)es[N] != b.ne) {
            set_error("elem_start must run from 0 to the element count (got %d .. %d for %lld elements)", es[0],
                      es[N], (long long)b.ne);
            return NBGS_ERR_INVALID_ARG;
        }
        for (size_t i = 0; i < N; ++i)
            if (!(es[i + 1] > es[i])) {
                set_error("elem_start must increase: body %zu holds no element", i);
                return NBGS_ERR_INVALID_ARG;
            }
    }
    for (DevBuf<int32_t> *bb : {&sc->ebody, &sc->sbody, &sc->cellpos}) NBGS_TRY(bb->reserve(E, 1.0));
    NBGS_TRY(sc->cnt.reserve(E + 1, 1.0));
    NBGS_TRY(sc->npart.reserve(E, 1.0));
    NBGS_TRY(sc->partners.reserve((size_t)kPartnerCap * E, 1.0));
    NBGS_TRY(sc->off.reserve(E + 1, 1.0));
    for (DevBuf<int32_t> *bb : {&sc->off1, &sc->cnt1}) NBGS_TRY(bb->reserve(N, 1.0));
    for (DevBuf<int32_t> *bb : {&sc->deg2, &sc->off2, &sc->cursor}) NBGS_TRY(bb->reserve(N + 1, 1.0));
    for (DevBuf<uint32_t> *bb : {&sc->keys, &sc->ids, &sc->keys2, &sc->ids2}) NBGS_TRY(bb->reserve(E, 1.0));
    NBGS_TRY(sc->ec.reserve(E, 1.0));
    NBGS_TRY(sc->sec.reserve(E, 1.0));
    for (DevBuf<double> *bb : {&sc->owx, &sc->owy, &sc->owz}) NBGS_TRY(bb->reserve(E, 1.0));
    NBGS_TRY(sc->h.reserve(N, 1.0));
    NBGS_TRY(sc->vel.reserve(8 * N, 1.0));
    NBGS_TRY(sc->iw.reserve(9 * N, 1.0));
    NBGS_TRY(sc->maxbits.reserve(4, 1.0));
    NBGS_TRY(sc->small.reserve(1024, 1.0));
    NBGS_TRY(sc->ctrl.reserve(4, 1.0));
    NBGS_TRY(sc->radix_hist.reserve(radix_hist_entries((int64_t)E), 1.0));
    NBGS_TRY(sc->scan_tmp.reserve(
        exclusive_scan_tmp_bytes((int64_t)radix_hist_entries((int64_t)E + 1) + (int64_t)std::max(E, N) + 1), 1.0));
    NBGS_TRY(sc->cb[0].reserve(1024));
    NBGS_TRY(sc->cb[1].reserve(1024));
    NBGS_HIP(hipHostMalloc((void **)&sc->pinned, 1024 * sizeof(int32_t), hipHostMallocDefault));
    std::memset(sc->pinned, 0, 1024 * sizeof(int32_t));
    for (int i = 0; i < kPhN; ++i)
        if (hipEventCreate(&sc->ev[i]) != hipSuccess) sc->ev[i] = nullptr;
    k_elem_body<<<grid_for((int64_t)N), kBlock, 0, sc->s>>>(b.elem_start, b.n, sc->ebody.p);
    NBGS_HIP(hipGetLastError());
    NBGS_HIP(hipStreamSynchronize(sc->s));
    guard.keep = true;
    *out = sc;
    return NBGS_OK;
}

nbgs_status nbgs_composite_destroy(nbgs_composite_t sc) {
    if (!sc) return NBGS_OK;
    if (sc->s) (void)hipStreamSynchronize(sc->s);
    else (void)hipDeviceSynchronize();
    for (int i = 0; i < kPhN; ++i)
        if (sc->ev[i]) (void)hipEventDestroy(sc->ev[i]);
    if (sc->pinned) (void)hipHostFree(sc->pinned);
    delete sc;
    return NBGS_OK;
}

nbgs_status nbgs_composite_detect(nbgs_composite_t sc, nbgs_stats *stats) {
    NBGS_CGUARD(sc);
    if (sc->state == 1 || sc->state == 2) {
        set_error("detect after detect: solve and integrate first");
        return NBGS_ERR_STATE;
    }
    sc->nc_needed = -1;
    const nbgs_status st = comp_detect(sc, stats);
    if (st == NBGS_ERR_CAPACITY && stats) {
        *stats = nbgs_stats{};
        stats->n_contacts = sc->nc_needed;
    }
    return st;
}

nbgs_status nbgs_composite_solve(nbgs_composite_t sc, int32_t max_sweeps, double residual_target,
                                 nbgs_stats *stats) {
    NBGS_CGUARD(sc);
    return comp_solve(sc, max_sweeps, residual_target, stats);
}

nbgs_status nbgs_composite_integrate(nbgs_composite_t sc) {
    NBGS_CGUARD(sc);
    return comp_integrate(sc);
}

nbgs_status nbgs_composite_step(nbgs_composite_t sc, int32_t max_sweeps, double residual_target, nbgs_stats *stats) {
    NBGS_CGUARD(sc);
    if (sc->state != 0) {
        set_error("step needs an integrated (or fresh) scene");
        return NBGS_ERR_STATE;
    }
    sc->nc_needed = -1;
    const nbgs_status ds = comp_detect(sc, nullptr);
    if (ds != NBGS_OK) {
        if (ds == NBGS_ERR_CAPACITY && stats) {  // the contact count the workspace lacks
            *stats = nbgs_stats{};
            stats->n_contacts = sc->nc_needed;
        }
        return ds;
    }
    const nbgs_status st = comp_solve(sc, max_sweeps, residual_target, stats);
    if (st != NBGS_OK && st != NBGS_ERR_NOT_CONVERGED) return st;
    NBGS_TRY(comp_integrate(sc));
    return st;
}

nbgs_status nbgs_composite_get_contacts(nbgs_composite_t sc, int64_t cap, int32_t *j1, int32_t *j2, uint64_t *key,
                                        int32_t *colour, double *impulse, double *geometry, int64_t *n_out) {
    NBGS_CGUARD(sc);
    if (n_out) *n_out = sc->nc;
    if (sc->state == 0 && !sc->table_in_cur) {
        if (cap == 0) return NBGS_OK;
        set_error("no detected step");
        return NBGS_ERR_STATE;
    }
    if (cap == 0) return NBGS_OK;
    if (cap < sc->nc) {
        set_error("capacity %lld below the contact count %lld", (long long)cap, (long long)sc->nc);
        return NBGS_ERR_CAPACITY;
    }
    if (sc->nc == 0) return NBGS_OK;
    CompContactBuf &cb = sc->cb[sc->cur];
    k_export_contacts<<<grid_for(sc->nc), kBlock, 0, sc->s>>>(cb.view(), sc->nc, cap, j1, j2, key, colour, impulse,
                                                              geometry);
    NBGS_HIP(hipGetLastError());
    NBGS_HIP(hipStreamSynchronize(sc->s));
    return NBGS_OK;
}

nbgs_status nbgs_composite_get_accumulators(nbgs_composite_t sc, double *v, double *w) {
    NBGS_CGUARD(sc);
    if (sc->state != 2 && !(sc->state == 0 && sc->table_in_cur)) {
        set_error("no solved step");
        return NBGS_ERR_STATE;
    }
    if (!v || !w) {
        set_error("v or w is NULL");
        return NBGS_ERR_INVALID_ARG;
    }
    NBGS_TRY(launch_export_accumulators<double>(sc->vel.p, sc->b.n, v, w, sc->bv, nullptr, false, sc->p.gravity,
                                                sc->p.dt, nullptr, sc->s));
    NBGS_HIP(hipStreamSynchronize(sc->s));
    return NBGS_OK;
}

nbgs_status nbgs_composite_get_residuals(nbgs_composite_t sc, int32_t cap, double *hist, int32_t *n_out) {
    NBGS_CGUARD(sc);
    if (n_out) *n_out = sc->hist_n;
    const int32_t m = std::min(cap, sc->hist_n);
    if (m > 0 && hist && sc->nc > 0) {
        NBGS_HIP(hipMemcpyAsync(hist, sc->hist.p, sizeof(double) * (size_t)m, hipMemcpyDeviceToHost, sc->s));
        NBGS_HIP(hipStreamSynchronize(sc->s));
    }
    return NBGS_OK;
}

nbgs_status nbgs_composite_get_phase_times(nbgs_composite_t sc, int32_t n, double *out) {
    NBGS_CGUARD(sc);
    if (!out || n < 1) {
        set_error("out is NULL or n < 1");
        return NBGS_ERR_INVALID_ARG;
    }
    NBGS_HIP(hipStreamSynchronize(sc->s));
    const int pairs[5][2] = {{kPhDetect, kPhColour}, {kPhColour, kPhInit}, {kPhInit, kPhSweeps},
                             {kPhSweeps, kPhIntegrate}, {kPhIntegrate, kPhEnd}};
    for (int k = 0; k < n && k < 5; ++k) {
        float ms = 0.0f;
        const int a = pairs[k][0], c = pairs[k][1];
        out[k] = (sc->ev[a] && sc->ev[c] && sc->ev_ok[a] && sc->ev_ok[c] &&
                  hipEventElapsedTime(&ms, sc->ev[a], sc->ev[c]) == hipSuccess)
                     ? (double)ms
                     : -1.0;
    }
    return NBGS_OK;
}

}  // extern "C"
