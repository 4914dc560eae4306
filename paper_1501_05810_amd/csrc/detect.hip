// Contact detection on a uniform cell grid (Sect. 4 of the paper).
//
// Broad phase: every body's intersection hull S_i + ball(h_i), with
// h_i = dt (|v_i| + |w_i| r_i) + tau (eq. (expansionradius)), lies in the cell
// of its centre, and the cell edge is at least the largest hull diameter, so
// partners of a body are found in the 27 surrounding cells.  Bodies are radix
// sorted by cell key; a table gives each occupied cell its range of sorted
// positions, and a bitmap of the occupied cells (cleared every step, 1 bit per
// cell) says which entries of the table are current, so that the neighbour
// search loads the records of occupied cells only.
//
// Narrow phase: eq. (contactpos) has a closed form for spheres (contact point
// on the surface of j2, normal from j2 to j1) and for wall planes.
//
// Output order: body i's contacts with partners k > i, ascending k, then its
// wall contacts; bodies in ascending index.  That is ascending pair key, the
// canonical order, built by count -> exclusive scan -> emit, so it does not
// depend on thread scheduling.
//
// The hull test and the geometry are evaluated with the same operations in
// the same order as the plain definition (compiled without contraction), so
// the contact set is bit-exact, not merely close.
#include "nbgs_internal.h"

namespace nbgs {

namespace {

constexpr int kBlock = 256;

inline unsigned grid_for(int64_t n, int block = kBlock) { return (unsigned)((n + block - 1) / block); }

// Workgroups of the hull pass: each walks bodies i, i + kHullBlocks kBlock, ...
// and adds one atomic maximum, so a few thousand atomics meet on the largest
// hull rather than one per 256 bodies.
constexpr int kHullBlocks = 2048;

// State of the pair list at its build (see launch_hull): positions, radii and
// which bodies were static.
struct ListRef {
    const double *x0, *y0, *z0, *r0;
    const uint8_t *static0;
};

// Hull radii h_i and the largest r_i + h_i (max_bits[0]), the largest h_i
// (max_bits[3]) and, when a pair list is held (ref.x0 set), the largest
// |x_i - x_i(build)| + h_i + max(0, r_i - r_i(build)) (max_bits[4]; +inf when
// a body's static flag changed).  The list stays exact while that stays below
// its skin: a pair further apart than r_i + r_k + 2 skin at the build cannot
// overlap its hulls then.  The same pass keeps every body's dynamic bit
// (bit i of bits, one word per wave of 64 bodies) and adds the number of
// words that changed since the last detection to *changed (the colouring and
// the block slots depend on which bodies are dynamic, so a colouring is
// reused only while no word changed).  Waves walk the
// bodies in steps of whole 64-body words, so every lane of a wave takes part
// in each ballot.
__global__ void __launch_bounds__(kBlock) k_hull(BodiesView b, double dt, double tau, double *h,
                                                 unsigned long long *max_bits, ListRef ref, uint64_t *bits,
                                                 int32_t *changed) {
    double rmax = 0.0, hmax = 0.0, dmax = 0.0;
    int diff = 0;
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i0 = (int64_t)blockIdx.x * kBlock + (threadIdx.x & ~63); i0 < b.n; i0 += stride) {
        const int64_t i = i0 + lane;
        bool dyn = false;
        if (i < b.n) {
            const double vx = b.vx[i], vy = b.vy[i], vz = b.vz[i];
            const double wx = b.wx[i], wy = b.wy[i], wz = b.wz[i];
            const double r = b.radius[i];
            const double im = b.inv_mass[i];
            dyn = im > 0.0;
            const double speed = sqrt(vx * vx + vy * vy + vz * vz);
            const double spin = sqrt(wx * wx + wy * wy + wz * wz);
            const double hi = dt * (speed + spin * r) + tau;
            h[i] = hi;
            double rh = r + hi;
            if (!(rh == rh)) rh = __longlong_as_double(0x7ff0000000000000ll);  // NaN -> +inf: caught on the host
            rmax = fmax(rmax, rh);
            hmax = fmax(hmax, hi);
            if (ref.x0) {
                const double dx = b.x[i] - ref.x0[i], dy = b.y[i] - ref.y0[i], dz = b.z[i] - ref.z0[i];
                double d = sqrt(dx * dx + dy * dy + dz * dz) + hi + fmax(0.0, r - ref.r0[i]);
                if (!(d == d) || (uint8_t)(im == 0.0) != ref.static0[i]) d = __longlong_as_double(0x7ff0000000000000ll);
                dmax = fmax(dmax, d);
            }
        }
        const unsigned long long m = __ballot(dyn);
        if (lane == 0) {
            const int64_t word = i0 >> 6;
            if (bits[word] != (uint64_t)m) {
                bits[word] = (uint64_t)m;
                ++diff;
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        rmax = fmax(rmax, __shfl_xor(rmax, o, 64));
        hmax = fmax(hmax, __shfl_xor(hmax, o, 64));
        dmax = fmax(dmax, __shfl_xor(dmax, o, 64));
    }
    __shared__ double wmax[3][kBlock / 64];
    __shared__ int wdiff[kBlock / 64];
    if (lane == 0) {
        wmax[0][threadIdx.x >> 6] = rmax;
        wmax[1][threadIdx.x >> 6] = hmax;
        wmax[2][threadIdx.x >> 6] = dmax;
        wdiff[threadIdx.x >> 6] = diff;
    }
    __syncthreads();
    if (threadIdx.x < 3) {  // the maxima are order-independent
        const int k = threadIdx.x;
        double m = wmax[k][0];
        for (int w = 1; w < kBlock / 64; ++w) m = fmax(m, wmax[k][w]);
        if (k == 0 || m > 0.0) atomicMax(&max_bits[k == 0 ? 0 : k + 2], (unsigned long long)__double_as_longlong(m));
    } else if (threadIdx.x == 64) {  // one atomic per workgroup (the first detection changes every word)
        int t = 0;
        for (int w = 0; w < kBlock / 64; ++w) t += wdiff[w];
        if (t) atomicAdd(changed, t);
    }
}

__device__ inline int cell_coord(double x, double lo, double edge, int dims) {
    double c = floor((x - lo) / edge);
    c = fmax(0.0, fmin(c, (double)(dims - 1)));  // NaN -> 0
    return (int)c;
}

// The grid of body i: its scene's (batched scenes) or the single one.
__device__ inline const Grid &grid_of(const Grid &g, const SceneTable &st, int i) {
    return st.body_scene ? st.grids[st.body_scene[i]] : g;
}

// Cell key of every body and its packed record (centre, +-(r + h), the sign
// marking static bodies) in body order, for the one gather of k_cells.
__global__ void __launch_bounds__(kBlock) k_cell_keys(BodiesView b, Grid g0, SceneTable st, const double *h,
                                                      uint32_t *keys, uint32_t *ids, double4 *xr) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= b.n) return;
    const Grid &g = grid_of(g0, st, i);
    const double x = b.x[i], y = b.y[i], z = b.z[i];
    const int cx = cell_coord(x, g.lo[0], g.edge[0], g.dims[0]);
    const int cy = cell_coord(y, g.lo[1], g.edge[1], g.dims[1]);
    const int cz = cell_coord(z, g.lo[2], g.edge[2], g.dims[2]);
    // the cell's coordinates in key order (g.axis[0] fastest)
    auto along = [&](int a) { return a == 0 ? cx : (a == 1 ? cy : cz); };
    keys[i] = g.cell_off + (uint32_t)((along(g.axis[2]) * g.kdims[1] + along(g.axis[1])) * g.kdims[0] + along(g.axis[0]));
    ids[i] = (uint32_t)i;
    const double rh = b.radius[i] + h[i];
    xr[i] = make_double4(x, y, z, b.inv_mass[i] == 0.0 ? -rh : rh);
}

// Cell ranges from the sorted keys (the first body of a cell's run writes its
// start, the last one the end), the cells' occupancy bits, and the packed
// records in sorted order (for coalesced neighbour reads).  The keys rise
// along the wave, so lanes whose cells share a bitmap word are neighbours: the
// word's bits are OR-ed across them and set by one atomic.
__global__ void __launch_bounds__(kBlock) k_cells(int32_t n, const uint32_t *skeys, const uint32_t *sids,
                                                  const double4 *xr, int2 *cells, uint32_t *occ, double4 *sxr) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool valid = p < n;
    const uint32_t key = valid ? skeys[p] : 0xffffffffu;
    const bool first = valid && (p == 0 || skeys[p - 1] != key);
    if (first) cells[key].x = p;
    if (valid && (p == n - 1 || skeys[p + 1] != key)) cells[key].y = p + 1;
    if (valid) sxr[p] = xr[sids[p]];
    const uint32_t word = key >> 5;
    uint32_t bits = first ? (1u << (key & 31u)) : 0u;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {  // OR over the following lanes of the same word
        const uint32_t ow = __shfl_down(word, o, 64), ob = __shfl_down(bits, o, 64);
        if (lane + o < 64 && ow == word) bits |= ob;
    }
    const uint32_t prev_word = __shfl_up(word, 1, 64);
    if (valid && bits && (lane == 0 || prev_word != word)) atomicOr(&occ[word], bits);
}

__device__ inline double min_image(double d, int periodic, double L) {
    if (!periodic) return d;
    if (d > 0.5 * L) return d - L;
    if (d < -0.5 * L) return d + L;
    return d;
}

struct NeighbourRange {
    int lo[3], hi[3];
};

// The cell of a key in key order (c[0] along the fastest key axis) and the
// stencil's extent per key axis.
__device__ inline NeighbourRange neighbour_range(uint32_t gkey, const Grid &g, int c[3]) {
    const uint32_t key = gkey - g.cell_off;
    c[0] = (int)(key % (uint32_t)g.kdims[0]);
    const uint32_t t = key / (uint32_t)g.kdims[0];
    c[1] = (int)(t % (uint32_t)g.kdims[1]);
    c[2] = (int)(t / (uint32_t)g.kdims[1]);
    NeighbourRange r;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (g.kdims[a] == 1) {
            r.lo[a] = 0;
            r.hi[a] = 0;
        } else {
            r.lo[a] = -1;
            r.hi[a] = 1;
        }
    }
    return r;
}

// Linear index of neighbour cell c + d (key order), or -1 outside a
// non-periodic axis.
__device__ inline int neighbour_cell(const Grid &g, const int c[3], int dx, int dy, int dz) {
    int q[3] = {c[0] + dx, c[1] + dy, c[2] + dz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (q[a] < 0 || q[a] >= g.kdims[a]) {
            if (!g.kperiodic[a]) return -1;
            q[a] = q[a] < 0 ? q[a] + g.kdims[a] : q[a] - g.kdims[a];
        }
    }
    return (int)g.cell_off + (q[2] * g.kdims[1] + q[1]) * g.kdims[0] + q[0];
}

// Hull overlap of sorted entries (own, other): |x_i - x_k|^2 <= ((r_i + h_i) + (r_k + h_k))^2.
__device__ inline bool hull_hit(const double4 &a, const double4 &o, const Grid &g) {
    const double dx = min_image(a.x - o.x, g.periodic[0], g.L[0]);
    const double dy = min_image(a.y - o.y, g.periodic[1], g.L[1]);
    const double dz = min_image(a.z - o.z, g.periodic[2], g.L[2]);
    const double d2 = dx * dx + dy * dy + dz * dz;
    const double reach = fabs(a.w) + fabs(o.w);
    return d2 <= reach * reach;
}

__device__ inline bool plane_hit(const PlaneSet &pl, int w, double x, double y, double z, double r, double h,
                                 double tau, double *gap_out) {
    const double s = pl.nrm[w][0] * (x - pl.p[w][0]) + pl.nrm[w][1] * (y - pl.p[w][1]) + pl.nrm[w][2] * (z - pl.p[w][2]);
    const double gap = s - r;
    *gap_out = gap;
    return gap <= h + tau;
}

// Hull candidates one body may meet in its 27 cells.  The cell edge follows
// the largest hull, so a single fast body coarsens the whole grid; past this
// bound the count gives up (the host reports it) instead of scanning for
// minutes.  A dense monodisperse packing meets a few hundred.
constexpr int kMaxCandidates = 1 << 18;

// Partners of body i with k > i, hull overlap tested on the sorted entries;
// the count variant returns -1 once the candidates pass kMaxCandidates and
// keeps the first `cap` partners found in out_k (the emit variant keeps all).
template <bool kEmit>
__device__ inline int visit_partners(const Grid &g, const uint32_t *skeys, const uint32_t *sids, const double4 *sxr,
                                     const int2 *cells, const uint32_t *occ, int p, int i, int32_t *out_k,
                                     int cap = 0) {
    const double4 me = sxr[p];
    int c[3];
    const NeighbourRange nr = neighbour_range(skeys[p], g, c);
    int m = 0, seen = 0;
    for (int dz = nr.lo[2]; dz <= nr.hi[2]; ++dz)
        for (int dy = nr.lo[1]; dy <= nr.hi[1]; ++dy) {
            // the row's (up to) three cells: their occupancy bits first, then the ranges (start, end) of the
            // occupied ones, loaded together
            int cell[3];
            bool used[3];
            int2 cr[3];
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                const int dx = nr.lo[0] + t;
                cell[t] = dx <= nr.hi[0] ? neighbour_cell(g, c, dx, dy, dz) : -1;
                const uint32_t cc = cell[t] < 0 ? 0u : (uint32_t)cell[t];
                used[t] = cell[t] >= 0 && ((occ[cc >> 5] >> (cc & 31u)) & 1u);
            }
#pragma unroll
            for (int t = 0; t < 3; ++t) cr[t] = used[t] ? cells[cell[t]] : make_int2(0, 0);
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                if (!used[t]) continue;
                const int q0 = cr[t].x, q1 = cr[t].y;
                if (!kEmit) {
                    seen += q1 - q0;
                    if (seen > kMaxCandidates) return -1;
                }
                for (int q = q0; q < q1; ++q) {
                    const int k = (int)sids[q];
                    const double4 o = sxr[q];
                    if (k <= i) continue;
                    if (me.w < 0.0 && o.w < 0.0) continue;  // two static bodies
                    if (!hull_hit(me, o, g)) continue;
                    if (kEmit || m < cap) out_k[m] = k;
                    ++m;
                }
            }
        }
    return m;
}

// Workgroups are dispatched to the 8 XCDs in turn (b mod 8), each XCD with its
// own L2.  This bijection hands XCD x a contiguous run of the tiles, so the
// neighbour reads of a body (cells one row and one plane away in sorted
// order) find the data its XCD's earlier workgroups loaded.
__device__ inline unsigned xcd_tile(unsigned b, unsigned nb) {
    const unsigned q = nb / 8, r = nb % 8, x = b % 8, l = b / 8;
    return x * q + (x < r ? x : r) + l;
}

__global__ void __launch_bounds__(kBlock) k_pair_count(BodiesView b, Grid g0, PlaneSet pl0, SceneTable st, double tau,
                                                       const uint32_t *skeys, const uint32_t *sids,
                                                       const double4 *sxr, const double *h,
                                                       const int2 *cells, const uint32_t *occ, int32_t *cnt,
                                                       int32_t *npart, int32_t *partners, int32_t *cellpos,
                                                       unsigned long long *total) {
    const int64_t p64 = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    const int p = (int)(p64 < b.n ? p64 : 0);  // (the sorted position, below 2^31 when in range)
    unsigned long long m64 = 0;
    int over = 0;
    if (p64 < b.n) {
        const int i = (int)sids[p];
        const int sc = st.body_scene ? st.body_scene[i] : 0;
        const Grid g = st.body_scene ? st.grids[sc] : g0;  // a copy: read once, not at every cell and candidate
        const PlaneSet &pl = st.body_scene ? st.planes[sc] : pl0;
        int m = visit_partners<false>(g, skeys, sids, sxr, cells, occ, p, i,
                                      partners + (int64_t)kPartnerCap * i, kPartnerCap);
        if (m < 0) {
            over = 1;
            m = 0;
        }
        const int mp = m;
        const double4 me = sxr[p];
        if (pl.n > 0 && me.w >= 0.0) {  // a dynamic body (the sign of its packed reach) meets the walls
            const double r = b.radius[i], hi = h[i];
            double gap;
            for (int w = 0; w < pl.n; ++w)
                if (plane_hit(pl, w, me.x, me.y, me.z, r, hi, tau, &gap)) ++m;
        }
        // cnt holds zeros (filled before the count); only bodies with contacts are written, and the emit reads
        // npart and the sorted position of those alone
        if (m > 0) {
            cnt[i] = m;
            npart[i] = mp;
            cellpos[i] = p;
        }
        m64 = (unsigned long long)m;
    }
    // The list length in 64 bits (the 32-bit scan of the counts would wrap
    // silently past 2^31) and the candidate overflow: one atomic per block.
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

// Ascending partner indices: insertion sort for the usual short list, heap
// sort (bounded work) for the long one of a body with a wide hull.  Partners
// are distinct, so both give the same order.
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

// The canonical list in two passes.  First one thread per body: its segment
// of body indices (partners ascending, then the walls its hull meets); a body
// whose partners all fit in the count's store copies them from there, only a
// longer list is searched again; bodies without contacts leave at once.
__global__ void __launch_bounds__(kBlock) k_pair_emit(BodiesView b, Grid g0, PlaneSet pl0, SceneTable st, double tau,
                                                      const uint32_t *skeys, const uint32_t *sids,
                                                      const double4 *sxr, const double *h,
                                                      const int2 *cells, const uint32_t *occ, const int32_t *cnt,
                                                      const int32_t *off, const int32_t *cellpos,
                                                      const int32_t *npart, const int32_t *partners, ContactsView c) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= b.n || cnt[i] == 0) return;
    const int p = cellpos[i];
    const int sc = st.body_scene ? st.body_scene[i] : 0;
    const Grid g = st.body_scene ? st.grids[sc] : g0;
    const PlaneSet &pl = st.body_scene ? st.planes[sc] : pl0;
    const int wall0 = b.n + (st.body_scene ? st.wall_off[sc] : 0);
    const int base = off[i];
    int32_t *ks = c.j2 + base;
    int m = npart[i];
    if (m <= kPartnerCap) {
        const int32_t *kept = partners + (int64_t)kPartnerCap * i;
        for (int t = 0; t < m; ++t) ks[t] = kept[t];
    } else {
        m = visit_partners<true>(g, skeys, sids, sxr, cells, occ, p, i, ks);
    }
    sort_partners(ks, m);
    for (int t = 0; t < m; ++t) c.j1[base + t] = i;
    if (b.inv_mass[i] != 0.0) {
        int t = m;
        const double xi_ = b.x[i], yi = b.y[i], zi = b.z[i], ri = b.radius[i], hi = h[i];
        double gap;
        for (int w = 0; w < pl.n; ++w) {
            if (!plane_hit(pl, w, xi_, yi, zi, ri, hi, tau, &gap)) continue;
            const int j = base + t++;
            c.j1[j] = i;
            c.j2[j] = wall0 + w;
        }
    }
}

// Then one thread per contact, so that neighbouring threads write neighbouring
// entries: the key and the geometry of eq. (contactpos) for two spheres (n from
// the centre of j2 to that of j1, xi = |x1 - x2| - r1 - r2, arms r1 + xi and
// r2) or for a sphere and a wall (the wall's normal, xi its gap to the sphere,
// arms r1 + xi and 0).
__global__ void __launch_bounds__(kBlock) k_pair_geometry(BodiesView b, Grid g0, PlaneSet pl0, SceneTable st,
                                                          int64_t nc, ContactsView c) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nc) return;
    const int i = c.j1[j], k = c.j2[j];
    c.key[j] = ((uint64_t)(uint32_t)i << 32) | (uint64_t)(uint32_t)k;
    const double xi_ = b.x[i], yi = b.y[i], zi = b.z[i], ri = b.radius[i];
    if (k < b.n) {
        const int sc = st.body_scene ? st.body_scene[i] : 0;
        const Grid &g = st.body_scene ? st.grids[sc] : g0;
        const double dx = min_image(xi_ - b.x[k], g.periodic[0], g.L[0]);
        const double dy = min_image(yi - b.y[k], g.periodic[1], g.L[1]);
        const double dz = min_image(zi - b.z[k], g.periodic[2], g.L[2]);
        const double d2 = dx * dx + dy * dy + dz * dz;
        const double d = sqrt(d2);
        double nx, ny, nz;
        if (d2 > 0.0) {
            nx = dx / d;
            ny = dy / d;
            nz = dz / d;
        } else {
            nx = 0.0;
            ny = 0.0;
            nz = 1.0;
        }
        const double rk = b.radius[k];
        const double xi = (d - ri) - rk;
        c.nx[j] = nx;
        c.ny[j] = ny;
        c.nz[j] = nz;
        c.xi[j] = xi;
        c.a1[j] = ri + xi;
        c.a2[j] = rk;
    } else {
        const int sc = st.body_scene ? st.body_scene[i] : 0;
        const PlaneSet &pl = st.body_scene ? st.planes[sc] : pl0;
        const int w = k - (b.n + (st.body_scene ? st.wall_off[sc] : 0));
        double gap;
        (void)plane_hit(pl, w, xi_, yi, zi, ri, 0.0, 0.0, &gap);  // the gap the first pass tested
        c.nx[j] = pl.nrm[w][0];
        c.ny[j] = pl.nrm[w][1];
        c.nz[j] = pl.nrm[w][2];
        c.xi[j] = gap;
        c.a1[j] = ri + gap;
        c.a2[j] = 0.0;
    }
}

// Look each contact's pair key up in the previous step's key-sorted table.
// matched: 1 + the previous index of the same pair, 0 if the pair is new;
// unmatched (may be null): the number of new pairs is added to it.
// impulses: the previous impulse of the same pair re-projected onto the new
// cone (P_n = max(0, n.P), tangential part clipped to mu P_n), zero if the pair
// is new.  colours: the previous colour as the start of the colouring passes
// (0 if new).
__global__ void __launch_bounds__(kBlock) k_match_prev(ContactsView c, int64_t nc, const uint64_t *prev_key,
                                                       const double *prev_px, const double *prev_py,
                                                       const double *prev_pz, const int32_t *prev_colour,
                                                       int64_t n_prev, double mu0, SceneTable st, int impulses,
                                                       int colours, int32_t *unmatched) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    bool found = false;
    int64_t lo = 0;
    if (j < nc) {
        const uint64_t key = c.key[j];
        if (j < n_prev && prev_key[j] == key) {
            // the same place in the last list (keys are unique there): what the search below would find, without
            // its dependent reads; in a settled packing this holds for every pair
            lo = j;
            found = true;
        } else {
            int64_t hi = n_prev;
            while (lo < hi) {
                const int64_t mid = lo + ((hi - lo) >> 1);
                if (prev_key[mid] < key) lo = mid + 1;
                else hi = mid;
            }
            found = lo < n_prev && prev_key[lo] == key;
        }
    }
    if (unmatched) {
        const unsigned long long nf = __ballot(j < nc && !found);
        __shared__ int wcount[kBlock / 64];
        if ((threadIdx.x & 63) == 0) wcount[threadIdx.x >> 6] = __popcll(nf);
        __syncthreads();
        if (threadIdx.x == 0) {
            int t = 0;
            for (int w = 0; w < kBlock / 64; ++w) t += wcount[w];
            if (t) atomicAdd(unmatched, t);
        }
    }
    if (j >= nc) return;
    const double mu = st.body_scene ? st.mu[st.body_scene[c.j1[j]]] : mu0;
    c.matched[j] = found ? (int32_t)(lo + 1) : 0;
    if (colours) c.colour[j] = found ? prev_colour[lo] : 0;
    if (!impulses) return;
    double P0 = 0.0, P1 = 0.0, P2 = 0.0;
    if (found) {
        const double n0 = c.nx[j], n1 = c.ny[j], n2 = c.nz[j];
        const double q0 = prev_px[lo], q1 = prev_py[lo], q2 = prev_pz[lo];
        double pn = n0 * q0 + n1 * q1 + n2 * q2;
        double t0 = q0 - pn * n0, t1 = q1 - pn * n1, t2 = q2 - pn * n2;
        if (pn < 0.0) pn = 0.0;
        const double tl = sqrt(t0 * t0 + t1 * t1 + t2 * t2);
        const double lim = mu * pn;
        if (tl > lim) {
            const double s = tl > 0.0 ? lim / tl : 0.0;
            t0 = t0 * s;
            t1 = t1 * s;
            t2 = t2 * s;
        }
        P0 = pn * n0 + t0;
        P1 = pn * n1 + t1;
        P2 = pn * n2 + t2;
    }
    c.px[j] = P0;
    c.py[j] = P1;
    c.pz[j] = P2;
}

// Contacts whose id (block or subdomain) differs from the one the same pair had
// in the previous step (matched = 1 + previous index); every contact is matched.
__global__ void __launch_bounds__(kBlock) k_ids_changed(const int32_t *sdom, const int32_t *prev_sdom,
                                                        const int32_t *matched, int64_t nc, int32_t *changed) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    // a new pair (matched 0: no previous id) counts as a change; the host checks the new pairs as well
    const bool diff = j < nc && (matched[j] == 0 || sdom[j] != prev_sdom[matched[j] - 1]);
    const unsigned long long m = __ballot(diff);
    __shared__ int wcount[kBlock / 64];
    if ((threadIdx.x & 63) == 0) wcount[threadIdx.x >> 6] = __popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < kBlock / 64; ++w) t += wcount[w];
        if (t) atomicAdd(changed, t);
    }
}

// The pair list's pairs (canonical order) tested with this step's hulls by
// exactly the predicates of the pair count: two bodies' reaches (r + h, the
// same roundings) against their minimum-image distance, two static bodies
// never; a dynamic body's wall by its gap.  flag[q] = 1 for a contact.
__global__ void __launch_bounds__(kBlock) k_list_test(BodiesView b, Grid g0, PlaneSet pl0, SceneTable st, double tau,
                                                      const double *h, const int32_t *lj1, const int32_t *lj2,
                                                      int64_t nl, int32_t *flag) {
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= nl) return;
    const int i = lj1[q], k = lj2[q];
    const int sc = st.body_scene ? st.body_scene[i] : 0;
    int hit = 0;
    if (k < b.n) {
        const Grid &g = st.body_scene ? st.grids[sc] : g0;
        const double rhi = b.radius[i] + h[i], rhk = b.radius[k] + h[k];
        const bool si = b.inv_mass[i] == 0.0, sk = b.inv_mass[k] == 0.0;
        if (!(si && sk)) {
            const double dx = min_image(b.x[i] - b.x[k], g.periodic[0], g.L[0]);
            const double dy = min_image(b.y[i] - b.y[k], g.periodic[1], g.L[1]);
            const double dz = min_image(b.z[i] - b.z[k], g.periodic[2], g.L[2]);
            const double d2 = dx * dx + dy * dy + dz * dz;
            const double reach = rhi + rhk;
            hit = d2 <= reach * reach;
        }
    } else if (b.inv_mass[i] != 0.0) {
        const PlaneSet &pl = st.body_scene ? st.planes[sc] : pl0;
        const int w = k - (b.n + (st.body_scene ? st.wall_off[sc] : 0));
        double gap;
        hit = plane_hit(pl, w, b.x[i], b.y[i], b.z[i], b.radius[i], h[i], tau, &gap);
    }
    flag[q] = hit;
}

// The listed pairs that are contacts, in list order (canonical), at their
// positions of the exclusive scan of the flags.
__global__ void __launch_bounds__(kBlock) k_list_emit(const int32_t *lj1, const int32_t *lj2, int64_t nl,
                                                      const int32_t *flag, const int32_t *off, ContactsView c) {
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= nl || !flag[q]) return;
    const int32_t o = off[q];
    c.j1[o] = lj1[q];
    c.j2[o] = lj2[q];
}

// The run of contacts of body j1[j] starts at j when j1[j - 1] differs; its
// first thread walks to the run's end (runs are a body's few partners).
__global__ void __launch_bounds__(kBlock) k_contact_runs(const int32_t *j1, int64_t nc, int32_t *cnt, int32_t *off) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nc) return;
    const int32_t b = j1[j];
    if (j > 0 && j1[j - 1] == b) return;
    int64_t e = j + 1;
    while (e < nc && j1[e] == b) ++e;
    off[b] = (int32_t)j;
    cnt[b] = (int32_t)(e - j);
}

// Sums of the steps between consecutive bodies per axis (pairs i, i + 1 for
// i < pairs), one partial per workgroup.
__global__ void __launch_bounds__(kBlock) k_numbering_steps(BodiesView b, int64_t pairs, double *part) {
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < pairs; i += (int64_t)gridDim.x * kBlock) {
        sx += fabs(b.x[i + 1] - b.x[i]);
        sy += fabs(b.y[i + 1] - b.y[i]);
        sz += fabs(b.z[i + 1] - b.z[i]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        sx += __shfl_xor(sx, o, 64);
        sy += __shfl_xor(sy, o, 64);
        sz += __shfl_xor(sz, o, 64);
    }
    __shared__ double w[3][kBlock / 64];
    if ((threadIdx.x & 63) == 0) {
        w[0][threadIdx.x >> 6] = sx;
        w[1][threadIdx.x >> 6] = sy;
        w[2][threadIdx.x >> 6] = sz;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double t = 0.0;
        for (int k = 0; k < kBlock / 64; ++k) t += w[threadIdx.x][k];
        part[3 * blockIdx.x + threadIdx.x] = t;
    }
}

__global__ void __launch_bounds__(kBlock) k_fill_f64(double *p, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void __launch_bounds__(kBlock) k_static_flags(const double *inv_mass, int64_t n, uint8_t *flags) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) flags[i] = (uint8_t)(inv_mass[i] == 0.0);
}

__global__ void __launch_bounds__(kBlock) k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

nbgs_status launch_hull(const BodiesView &b, double dt, double tau, double *h, unsigned long long *max_bits,
                        const double *x0, const double *r0, const uint8_t *static0, uint64_t *dyn_bits,
                        int32_t *dyn_changed, hipStream_t s) {
    if (b.n <= 0) return NBGS_OK;
    const unsigned blocks = std::min<unsigned>(grid_for(b.n), (unsigned)kHullBlocks);
    ListRef ref{x0, x0 ? x0 + b.n : nullptr, x0 ? x0 + 2 * (int64_t)b.n : nullptr, r0, static0};
    k_hull<<<blocks, kBlock, 0, s>>>(b, dt, tau, h, max_bits, ref, dyn_bits, dyn_changed);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

nbgs_status launch_fill_f64(double *p, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return NBGS_OK;
    k_fill_f64<<<grid_for(n), kBlock, 0, s>>>(p, n, v);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

nbgs_status launch_static_flags(const double *inv_mass, int64_t n, uint8_t *flags, hipStream_t s) {
    if (n <= 0) return NBGS_OK;
    k_static_flags<<<grid_for(n), kBlock, 0, s>>>(inv_mass, n, flags);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

nbgs_status launch_list_test(const BodiesView &b, const Grid &g, const PlaneSet &pl, const SceneTable &st,
                             double tau, const double *h, const int32_t *lj1, const int32_t *lj2, int64_t nl,
                             int32_t *flag, hipStream_t s) {
    if (nl <= 0) return NBGS_OK;
    k_list_test<<<grid_for(nl), kBlock, 0, s>>>(b, g, pl, st, tau, h, lj1, lj2, nl, flag);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

nbgs_status launch_list_emit(const int32_t *lj1, const int32_t *lj2, int64_t nl, const int32_t *flag,
                             const int32_t *off, ContactsView c, hipStream_t s) {
    if (nl <= 0) return NBGS_OK;
    k_list_emit<<<grid_for(nl), kBlock, 0, s>>>(lj1, lj2, nl, flag, off, c);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

nbgs_status launch_contact_runs(const int32_t *j1, int64_t nc, int32_t n, int32_t *cnt, int32_t *off, hipStream_t s) {
    NBGS_TRY(launch_fill_i32(cnt, n, 0, s));
    if (nc <= 0) return NBGS_OK;
    k_contact_runs<<<grid_for(nc), kBlock, 0, s>>>(j1, nc, cnt, off);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

nbgs_status launch_pair_geometry(const BodiesView &b, const Grid &g, const PlaneSet &pl, const SceneTable &st,
                                 ContactsView c, int64_t nc, hipStream_t s) {
    if (nc <= 0) return NBGS_OK;
    k_pair_geometry<<<grid_for(nc), kBlock, 0, s>>>(b, g, pl, st, nc, c);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

nbgs_status launch_cell_keys(const BodiesView &b, const Grid &g, const SceneTable &st, const double *h,
                             uint32_t *keys, uint32_t *ids, double4 *xr, hipStream_t s) {
    if (b.n <= 0) return NBGS_OK;
    k_cell_keys<<<grid_for(b.n), kBlock, 0, s>>>(b, g, st, h, keys, ids, xr);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

nbgs_status launch_numbering_steps(const BodiesView &b, int64_t pairs, double *part, int blocks, hipStream_t s) {
    k_numbering_steps<<<blocks, kBlock, 0, s>>>(b, pairs, part);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

nbgs_status launch_cells(int32_t n, int64_t ncells, const uint32_t *skeys, const uint32_t *sids, const double4 *xr,
                         int2 *cells, uint32_t *occ, double4 *sxr, hipStream_t s) {
    const int64_t words = (ncells + 31) / 32;
    k_fill_i32<<<grid_for(words), kBlock, 0, s>>>(reinterpret_cast<int32_t *>(occ), words, 0);
    NBGS_HIP(hipGetLastError());
    if (n <= 0) return NBGS_OK;
    k_cells<<<grid_for(n), kBlock, 0, s>>>(n, skeys, sids, xr, cells, occ, sxr);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

nbgs_status launch_pair_count(const BodiesView &b, const Grid &g, const PlaneSet &pl, const SceneTable &st, double tau,
                              const uint32_t *skeys, const uint32_t *sids, const double4 *sxr, const double *h,
                              const int2 *cells, const uint32_t *occ, int32_t *cnt, int32_t *npart,
                              int32_t *partners, int32_t *cellpos,
                              unsigned long long *total, hipStream_t s) {
    if (b.n <= 0) return NBGS_OK;
    k_fill_i32<<<grid_for(b.n), kBlock, 0, s>>>(cnt, b.n, 0);
    k_pair_count<<<grid_for(b.n), kBlock, 0, s>>>(b, g, pl, st, tau, skeys, sids, sxr, h, cells, occ, cnt, npart,
                                                  partners, cellpos, total);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

nbgs_status launch_pair_emit(const BodiesView &b, const Grid &g, const PlaneSet &pl, const SceneTable &st, double tau,
                             const uint32_t *skeys, const uint32_t *sids, const double4 *sxr, const double *h,
                             const int2 *cells, const uint32_t *occ, const int32_t *cnt, const int32_t *off,
                             const int32_t *cellpos,
                             const int32_t *npart, const int32_t *partners, ContactsView c, int64_t nc,
                             bool geometry, hipStream_t s) {
    k_pair_emit<<<grid_for(b.n), kBlock, 0, s>>>(b, g, pl, st, tau, skeys, sids, sxr, h, cells, occ, cnt, off, cellpos, npart, partners, c);
    NBGS_HIP(hipGetLastError());
    if (geometry && nc > 0) {
        k_pair_geometry<<<grid_for(nc), kBlock, 0, s>>>(b, g, pl, st, nc, c);
        NBGS_HIP(hipGetLastError());
    }
    return NBGS_OK;
}

nbgs_status launch_match_prev(ContactsView c, int64_t nc, const uint64_t *prev_key, const double *prev_px,
                              const double *prev_py, const double *prev_pz, const int32_t *prev_colour,
                              int64_t n_prev, double mu, const SceneTable &st, bool impulses, bool colours,
                              int32_t *unmatched, hipStream_t s) {
    if (nc == 0 || (!impulses && !colours)) return NBGS_OK;
    k_match_prev<<<grid_for(nc), kBlock, 0, s>>>(c, nc, prev_key, prev_px, prev_py, prev_pz, prev_colour, n_prev, mu,
                                                 st, impulses ? 1 : 0, colours ? 1 : 0, unmatched);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

nbgs_status launch_ids_changed(const int32_t *sdom, const int32_t *prev_sdom, const int32_t *matched, int64_t nc,
                               int32_t *changed, hipStream_t s) {
    if (nc == 0) return NBGS_OK;
    k_ids_changed<<<grid_for(nc), kBlock, 0, s>>>(sdom, prev_sdom, matched, nc, changed);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

nbgs_status launch_zero_impulses(ContactsView c, int64_t nc, hipStream_t s) {
    if (nc == 0) return NBGS_OK;
    NBGS_HIP(hipMemsetAsync(c.px, 0, sizeof(double) * nc, s));
    NBGS_HIP(hipMemsetAsync(c.py, 0, sizeof(double) * nc, s));
    NBGS_HIP(hipMemsetAsync(c.pz, 0, sizeof(double) * nc, s));
    return NBGS_OK;
}

nbgs_status launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return NBGS_OK;
    k_fill_i32<<<grid_for(n), kBlock, 0, s>>>(p, n, v);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

}  // namespace nbgs
