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

#include "contact_math.h"
#include "scene.h"

namespace nbgs {

namespace {

constexpr int kBlock = 256;
constexpr int kMaxCol = 256;

// At least one workgroup: counts here may be zero (no slot at all when every
// contact of the block-local order lies between blocks), and every element
// kernel below guards its index.
inline unsigned grid_for(int64_t n) { return n > 0 ? (unsigned)((n + kBlock - 1) / kBlock) : 1u; }

struct Blocks {
    double lo[3], e[3];
    int32_t nb[3];
};

// Block holding the centre of body i (coordinates clamped into the box).
__device__ inline int32_t block_of(const BodiesView &b, const Blocks &bl, int i) {
    const double x[3] = {b.x[i], b.y[i], b.z[i]};
    int64_t c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double f = floor((x[a] - bl.lo[a]) / bl.e[a]);
        f = fmax(0.0, fmin(f, (double)(bl.nb[a] - 1)));
        c[a] = (int64_t)f;
    }
    return (int32_t)((c[2] * bl.nb[1] + c[1]) * bl.nb[0] + c[0]);
}

__global__ void __launch_bounds__(kBlock) k_subdomain(BodiesView b, const int32_t *j1, int64_t nc, Blocks bl,
                                                      int32_t *sdom) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nc) return;
    sdom[j] = block_of(b, bl, j1[j]);
}

// Block-local id: the block of the contact's dynamic bodies if they share one,
// else nblocks (a contact between blocks).
__global__ void __launch_bounds__(kBlock) k_block_local(BodiesView b, const int32_t *j1, const int32_t *j2,
                                                        int64_t nc, Blocks bl, int32_t nblocks, int32_t *id) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nc) return;
    const int i1 = j1[j], i2 = j2[j];
    const bool d1 = b.inv_mass[i1] > 0.0;
    const bool d2 = i2 < b.n && b.inv_mass[i2] > 0.0;
    if (d1 && d2) {
        const int32_t k1 = block_of(b, bl, i1), k2 = block_of(b, bl, i2);
        id[j] = k1 == k2 ? k1 : nblocks;
    } else {
        id[j] = block_of(b, bl, d1 ? i1 : i2);
    }
}

// Block of body i in grid g of `grids` grids shifted by g/grids of an edge:
// c_a = floor((x_a - lo_a) / e_a + g / grids), modulo nb_a along a periodic
// axis, clamped to [0, nb_a - 1] in grid 0 and to [0, nb_a] in a shifted grid
// along another axis; id (c_z M_y + c_y) M_x + c_x.
__device__ inline int32_t block_in_grid(const BodiesView &b, const Blocks &bl, const int32_t M[3],
                                        const int32_t periodic[3], int g, int grids, int i) {
    const double x[3] = {b.x[i], b.y[i], b.z[i]};
    int64_t c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double f = floor((x[a] - bl.lo[a]) / bl.e[a] + (double)g / (double)grids);
        if (periodic[a]) {
            const int64_t q = (int64_t)f % bl.nb[a];
            c[a] = q < 0 ? q + bl.nb[a] : q;
        } else {
            const double top = g == 0 ? (double)(bl.nb[a] - 1) : (double)bl.nb[a];
            c[a] = (int64_t)fmax(0.0, fmin(f, top));
        }
    }
    return (int32_t)((c[2] * M[1] + c[1]) * M[0] + c[0]);
}

// Ids of the block-local order over several grids: g B + block for the first
// grid g whose block holds every dynamic body of the contact, grids B if none.
__global__ void __launch_bounds__(kBlock) k_block_local_grids(BodiesView b, const int32_t *j1, const int32_t *j2,
                                                              int64_t nc, Blocks bl, int32_t grids, int32_t Mx,
                                                              int32_t My, int32_t Mz, int32_t px, int32_t py,
                                                              int32_t pz, int32_t *id) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nc) return;
    const int32_t M[3] = {Mx, My, Mz}, per[3] = {px, py, pz};
    const int32_t B = Mx * My * Mz;
    const int i1 = j1[j], i2 = j2[j];
    const bool d1 = b.inv_mass[i1] > 0.0;
    const bool d2 = i2 < b.n && b.inv_mass[i2] > 0.0;
    int32_t out = grids * B;
    for (int g = 0; g < grids; ++g) {
        const int32_t k1 = block_in_grid(b, bl, M, per, g, grids, d1 ? i1 : i2);
        const int32_t k2 = d1 && d2 ? block_in_grid(b, bl, M, per, g, grids, i2) : k1;
        if (k1 == k2) {
            out = g * B + k1;
            break;
        }
    }
    id[j] = out;
}

// Groups of the contacts no grid holds (the block-local order over several
// grids).  Two such contacts interact only through a shared dynamic body, and
// in a settled packing they form small clusters, each swept in its own
// (colour, key) order.  Sweeping whole clusters in the block pass, packed
// into groups, one workgroup each with the group's bodies in LDS, gives every
// contact the arithmetic and the order of the colour launches (no cluster
// reaches another) in a single launch.  Clusters are the connected components
// of the contacts under "shares a dynamic body": every contact takes the
// smallest list position in its component by alternating minima over bodies
// and contacts.
__global__ void __launch_bounds__(kBlock) k_cross_flags(const int32_t *id, int64_t nc, int32_t cross,
                                                        int32_t *flag) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j < nc) flag[j] = id[j] == cross ? 1 : 0;
}

// The list of those contacts (pos: exclusive scan of the flags) and their start labels (own position).
__global__ void __launch_bounds__(kBlock) k_cross_list(const int32_t *id, const int32_t *pos, int64_t nc,
                                                       int32_t cross, int32_t *xl, int32_t *lab) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nc || id[j] != cross) return;
    xl[pos[j]] = (int32_t)j;
    lab[pos[j]] = pos[j];
}

__device__ inline int32_t dyn_end(const int32_t *jj, int32_t j, int32_t nb, const double *inv_mass) {
    const int32_t b = jj[j];
    return b < nb && inv_mass[b] > 0.0 ? b : -1;
}

// Every dynamic body of a listed contact: the smallest label of its listed contacts.
__global__ void __launch_bounds__(kBlock) k_cc_push(const int32_t *xl, int32_t nx, const int32_t *j1,
                                                    const int32_t *j2, int32_t nb, const double *inv_mass,
                                                    const int32_t *lab, int32_t *blab) {
    const int32_t q = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (q >= nx) return;
    const int32_t j = xl[q], l = lab[q];
    const int32_t b1 = dyn_end(j1, j, nb, inv_mass), b2 = dyn_end(j2, j, nb, inv_mass);
    if (b1 >= 0) atomicMin(&blab[b1], l);
    if (b2 >= 0) atomicMin(&blab[b2], l);
}

// Every listed contact: the smallest label of its dynamic bodies, if smaller; changed counts the moves.
__global__ void __launch_bounds__(kBlock) k_cc_pull(const int32_t *xl, int32_t nx, const int32_t *j1,
                                                    const int32_t *j2, int32_t nb, const double *inv_mass,
                                                    int32_t *lab, const int32_t *blab, int32_t *changed) {
    const int32_t q = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    int moved = 0;
    if (q < nx) {
        const int32_t j = xl[q];
        int32_t l = lab[q];
        const int32_t b1 = dyn_end(j1, j, nb, inv_mass), b2 = dyn_end(j2, j, nb, inv_mass);
        if (b1 >= 0) l = min(l, blab[b1]);
        if (b2 >= 0) l = min(l, blab[b2]);
        if (l < lab[q]) {
            lab[q] = l;
            moved = 1;
        }
    }
    if (__ballot(moved) && (threadIdx.x & 63) == 0) atomicAdd(changed, 1);
}

// Group ids: the cluster of label l goes to group l / per (labels are list positions, so a group holds the
// clusters whose first contact is among `per` consecutive ones); cnt counts each group's contacts.
__global__ void __launch_bounds__(kBlock) k_cc_ids(const int32_t *xl, int32_t nx, const int32_t *lab, int32_t base,
                                                   int32_t per, int32_t *id, int32_t *cnt) {
    const int32_t q = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (q >= nx) return;
    const int32_t g = lab[q] / per;
    id[xl[q]] = base + g;
    atomicAdd(&cnt[g], 1);
}

__global__ void __launch_bounds__(kBlock) k_cc_reset(const int32_t *xl, int32_t nx, int32_t cross, int32_t *id) {
    const int32_t q = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (q < nx) id[xl[q]] = cross;
}

// This step's ids from the grids (id n_blk: local in none) against the last step's final ids of the same pairs
// (matched[j] - 1; ids n_blk and above: local in none, in a group or swept by colour): *changed counts the pairs
// whose grid id differs or that became or stopped being local in none.
__global__ void __launch_bounds__(kBlock) k_raw_ids_changed(const int32_t *id, const int32_t *prev,
                                                            const int32_t *matched, int64_t nc, int32_t nblk,
                                                            int32_t *changed) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    bool diff = false;
    if (j < nc) {
        const int32_t m = matched[j];  // 0: a new pair (counted as a change; the host checks the new pairs too)
        const int32_t a = id[j], b = m > 0 ? prev[m - 1] : -1;
        diff = m == 0 || (a >= nblk) != (b >= nblk) || (a < nblk && a != b);
    }
    if (__ballot(diff) && (threadIdx.x & 63) == 0) atomicAdd(changed, 1);
}

// The last step's final ids for the same pairs.
__global__ void __launch_bounds__(kBlock) k_ids_from_prev(const int32_t *prev, const int32_t *matched, int64_t nc,
                                                          int32_t *id) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j < nc && matched[j] > 0) id[j] = prev[matched[j] - 1];  // launched only when no pair is new
}

__global__ void __launch_bounds__(kBlock) k_max_i32(const int32_t *v, int32_t n, int32_t *out) {
    const int32_t i = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    int32_t m = i < n ? v[i] : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0 && m > 0) atomicMax(out, m);
}

// cnt[v[i]] += 1 for every i.  The inputs here are sorted (ids of a sweep
// record, slots by id), so equal values sit in neighbouring lanes: each run of
// equal values in a wave adds its length with one atomic (exact for any input).
__global__ void __launch_bounds__(kBlock) k_hist(const int32_t *v, int64_t n, int32_t *cnt) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool valid = i < n;
    const int32_t x = valid ? v[i] : 0;
    const int32_t xl = __shfl_up(x, 1, 64);
    const bool start = valid && (lane == 0 || xl != x);
    const unsigned long long starts = __ballot(start);
    const int nvalid = __popcll(__ballot(valid));  // the valid lanes are a prefix of the wave
    if (start) {
        const unsigned long long above = lane == 63 ? 0ull : (starts & (~0ull << (lane + 1)));
        int next = above ? __ffsll((long long)above) - 1 : 64;
        if (next > nvalid) next = nvalid;
        atomicAdd(&cnt[x], next - lane);
    }
}

__global__ void __launch_bounds__(kBlock) k_fill(int32_t *p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}

// Contact end e = 2 p + k (k = 0: j1, 1: j2) of sweep position p; its body if
// dynamic, else nb (sorts after every body).  The ends of contacts with the id
// no_slot (the contacts between blocks of the block-local order, swept from
// global memory) count as not dynamic: they take no slot.
__device__ inline int32_t end_body(const int32_t *sj1, const int32_t *sj2, int32_t nb, const double *inv_mass,
                                   uint32_t e, const int32_t *ssd = nullptr, int32_t no_slot = -1) {
    if (no_slot >= 0 && ssd[e >> 1] == no_slot) return nb;
    const int32_t b = (e & 1u) ? sj2[e >> 1] : sj1[e >> 1];
    return (b < nb && inv_mass[b] > 0.0) ? b : nb;
}

__global__ void __launch_bounds__(kBlock) k_ends(const int32_t *sj1, const int32_t *sj2, int64_t nends, int32_t nb,
                                                 const double *inv_mass, uint32_t *keys, uint32_t *vals,
                                                 const int32_t *ssd, int32_t no_slot) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= nends) return;
    keys[e] = (uint32_t)end_body(sj1, sj2, nb, inv_mass, (uint32_t)e, ssd, no_slot);
    vals[e] = (uint32_t)e;
}

__global__ void __launch_bounds__(kBlock) k_end_tiles(const uint32_t *vals, int64_t n, const int32_t *ssd,
                                                      uint32_t *keys) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) keys[i] = (uint32_t)ssd[vals[i] >> 1];
}

// The same key in the block-local order over several grids, with the slots of
// a first-grid block sub-ordered by the cell of the body's centre among the
// grids^3 cells the shifted grids cut the block into (sb bits): the sweeps'
// records follow the first grid's slot order, and a later grid's block then
// reads its records in a few short runs.  Which slot a body takes inside its
// block changes nothing else.
__global__ void __launch_bounds__(kBlock) k_end_tiles_sub(const uint32_t *vals, int64_t n, const int32_t *ssd,
                                                          const int32_t *sj1, const int32_t *sj2, BodiesView b,
                                                          Blocks bl, int32_t grids, int32_t grid_ids,
                                                          int32_t no_slot, int32_t sb, uint32_t *keys) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t e = vals[i];
    const int32_t sd = ssd[e >> 1];
    uint32_t sub = 0;
    if (sd >= 0 && sd < grid_ids) {
        const int32_t k = end_body(sj1, sj2, b.n, b.inv_mass, e, ssd, no_slot);
        if (k < b.n) {
            const double x[3] = {b.x[k], b.y[k], b.z[k]};
            uint32_t w = 1;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double u = (x[a] - bl.lo[a]) / bl.e[a];
                const int32_t q = (int32_t)((u - floor(u)) * (double)grids);
                sub += w * (uint32_t)max(0, min(q, grids - 1));
                w *= (uint32_t)grids;
            }
        }
    }
    keys[i] = ((uint32_t)sd << sb) | sub;
}

// First end of every (subdomain, dynamic body) group, ends sorted by (subdomain, body).
__global__ void __launch_bounds__(kBlock) k_slot_flags(const uint32_t *vals, int64_t n, const int32_t *sj1,
                                                       const int32_t *sj2, const int32_t *ssd, int32_t nb,
                                                       const double *inv_mass, int32_t *flags, int32_t no_slot) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t e = vals[i];
    const int32_t b = end_body(sj1, sj2, nb, inv_mass, e, ssd, no_slot);
    int f = 0;
    if (b < nb) {
        if (i == 0) {
            f = 1;
        } else {
            const uint32_t e0 = vals[i - 1];
            f = (ssd[e0 >> 1] != ssd[e >> 1] || end_body(sj1, sj2, nb, inv_mass, e0, ssd, no_slot) != b) ? 1 : 0;
        }
    }
    flags[i] = f;
}

__global__ void __launch_bounds__(kBlock) k_slot_write(const uint32_t *vals, int64_t n, const int32_t *sj1,
                                                       const int32_t *sj2, const int32_t *ssd, int32_t nb,
                                                       const double *inv_mass, const int32_t *flags,
                                                       const int32_t *ex, int32_t *slot_body, int32_t *slot_sdom,
                                                       int32_t no_slot) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n || !flags[i]) return;
    const uint32_t e = vals[i];
    slot_body[ex[i]] = end_body(sj1, sj2, nb, inv_mass, e, ssd, no_slot);
    slot_sdom[ex[i]] = ssd[e >> 1];
}

// Local slot of every contact end: -1 for a static body and for every end of
// a contact that takes no slot, -2 for a wall.
__global__ void __launch_bounds__(kBlock) k_end_slots(const uint32_t *vals, int64_t n, const int32_t *sj1,
                                                      const int32_t *sj2, const int32_t *ssd, int32_t nb,
                                                      const double *inv_mass, const int32_t *flags,
                                                      const int32_t *ex, const int32_t *tile_slot_off,
                                                      int16_t *ls, int32_t no_slot) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t e = vals[i];
    const int32_t b = end_body(sj1, sj2, nb, inv_mass, e, ssd, no_slot);
    const int32_t raw = (e & 1u) ? sj2[e >> 1] : sj1[e >> 1];
    ls[e] = (int16_t)(b < nb ? ex[i] + flags[i] - 1 - tile_slot_off[ssd[e >> 1]] : (raw < nb ? -1 : -2));
}

__global__ void __launch_bounds__(kBlock) k_fill64(int64_t *p, int64_t n, int64_t v) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}

// first[k] = first position of the run of key k in the sorted keys (untouched for absent keys)
__global__ void __launch_bounds__(kBlock) k_first_of_runs(const int32_t *key, int64_t n, int64_t *first) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= n) return;
    if (p == 0 || key[p - 1] != key[p]) first[key[p]] = p;
}
__global__ void __launch_bounds__(kBlock) k_first_of_runs32(const uint32_t *key, int64_t n, int32_t *first) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= n) return;
    if (p == 0 || key[p - 1] != key[p]) first[key[p]] = (int32_t)p;
}

// Sort keys of the bodies: the block of a dynamic body, nblocks for a static one.
__global__ void __launch_bounds__(kBlock) k_body_blocks(BodiesView b, Blocks bl, int32_t nblocks, uint32_t *keys,
                                                        uint32_t *vals) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= b.n) return;
    keys[i] = (uint32_t)(b.inv_mass[i] > 0.0 ? block_of(b, bl, i) : nblocks);
    vals[i] = (uint32_t)i;
}

// The same keys kept for the next step, and the number of bodies whose key differs from the last step's.
__global__ void __launch_bounds__(kBlock) k_body_blocks_cmp(BodiesView b, Blocks bl, int32_t nblocks, uint32_t *cur,
                                                            const uint32_t *prev, int compare, int32_t *changed) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    bool diff = false;
    if (i < b.n) {
        const uint32_t k = (uint32_t)(b.inv_mass[i] > 0.0 ? block_of(b, bl, i) : nblocks);
        cur[i] = k;
        diff = compare && prev[i] != k;
    }
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

__global__ void __launch_bounds__(kBlock) k_slot_of(const uint32_t *sorted_body, int32_t n, int32_t *slot) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p < n) slot[sorted_body[p]] = p;
}

// Slot (local to the contact's block) of both ends of a local contact; -1 for
// a static body and every end of a contact between blocks, -2 for a wall.
__global__ void __launch_bounds__(kBlock) k_block_ends(const int32_t *sj1, const int32_t *sj2, const int32_t *ssd,
                                                       int64_t nc, int32_t nblocks, int32_t nb,
                                                       const double *inv_mass, const int32_t *slot,
                                                       const int32_t *first_slot, int16_t *ls) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= nc) return;
    const int32_t id = ssd[p];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int32_t b = k ? sj2[p] : sj1[p];
        ls[2 * p + k] = (int16_t)((id < nblocks && b < nb && inv_mass[b] > 0.0) ? slot[b] - first_slot[id]
                                                                                  : (b < nb ? -1 : -2));
    }
}

// Colour ranges of positions begin .. end of the sweep record (sorted by
// colour): cstart[c] = first position of colour c, *ncol = last colour + 1;
// cstart must hold end in every entry beforehand.
__global__ void __launch_bounds__(kBlock) k_range_colours(const int32_t *col, int64_t begin, int64_t end,
                                                          int64_t *cstart, int32_t *ncol) {
    const int64_t p = begin + (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= end) return;
    const int c = col[p];
    if (p == begin || col[p - 1] != c) cstart[c] = p;
    if (p == end - 1) *ncol = c + 1;
}

// Dynamic contact ends per colour over positions begin .. end.
__global__ void __launch_bounds__(kBlock) k_range_dyn(const int32_t *sj1, const int32_t *sj2, const int32_t *col,
                                                      int64_t begin, int64_t end, int32_t nb, const double *inv_mass,
                                                      unsigned long long *cnt) {
    __shared__ unsigned int h[kMaxCol];
    for (int c = threadIdx.x; c < kMaxCol; c += kBlock) h[c] = 0u;
    __syncthreads();
    const int64_t p = begin + (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p < end) {
        const int32_t b1 = sj1[p], b2 = sj2[p];
        const unsigned d = (inv_mass[b1] > 0.0 ? 1u : 0u) + ((b2 < nb && inv_mass[b2] > 0.0) ? 1u : 0u);
        if (d) atomicAdd(&h[col[p]], d);
    }
    __syncthreads();
    for (int c = threadIdx.x; c < kMaxCol; c += kBlock)
        if (h[c]) atomicAdd(&cnt[c], (unsigned long long)h[c]);
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


// Block-local order, local part: one workgroup per block.  Its slots (the
// dynamic bodies of its local contacts, all inside the block and touched by
// no other block's local contact) are copied into LDS, the local contacts are
// taken colour by colour (no two contacts of a colour share a slot), each
// reading and updating the slot records in place -- the sequential
// Gauss-Seidel order of the block -- and the slots are written back.  mode 0
// applies the initial impulses in the same order, mode 1 relaxes (relax_contact,
// the arithmetic of every sweep kernel) and writes the impulses and the block's
// residual sums.  A static partner's record is read from the accumulators (it
// never changes), a wall is zero.
constexpr int kBlkThreads = 64;         // the held form (k_blk_pass) and k_blk_colour_runs
constexpr int kBlkStreamThreads = 128;  // the streamed form (k_blk_pass_stream)

// Colour runs of every block's local contacts, once per step.  A block's
// contacts are in (colour, key) order, so every colour present in it is one
// run: cs[tile_off[s] + s + r] = start of run r relative to the block's first
// contact (r = 0 .. nrun[s], the last entry the block's contact count).  A
// block has at most as many runs as contacts, so block s's entries fit in its
// count + 1 places and the table in (local contacts + blocks) entries.
__global__ void __launch_bounds__(kBlkThreads) k_blk_colour_runs(const int32_t *col, const int64_t *tile_off,
                                                                 int32_t *cs, int32_t *nrun) {
    constexpr int kWaves = kBlkThreads / 64;
    const int s = blockIdx.x;
    const int64_t c0 = tile_off[s], c1 = tile_off[s + 1];
    int32_t *out = cs + c0 + s;
    __shared__ int wave_cnt[kWaves];
    __shared__ int base;
    if (threadIdx.x == 0) base = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int64_t q0 = c0; q0 < c1; q0 += kBlkThreads) {
        const int64_t p = q0 + threadIdx.x;
        const bool first = p < c1 && (p == c0 || col[p - 1] != col[p]);
        const unsigned long long m = __ballot(first);
        if (lane == 0) wave_cnt[wv] = __popcll(m);
        __syncthreads();
        int off = base + __popcll(m & ((1ull << lane) - 1ull));
        for (int w = 0; w < wv; ++w) off += wave_cnt[w];
        if (first) out[off] = (int32_t)(p - c0);
        __syncthreads();
        if (threadIdx.x == 0)
            for (int w = 0; w < kWaves; ++w) base += wave_cnt[w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[base] = (int32_t)(c1 - c0);
        nrun[s] = base;
    }
}

// Contacts of a block held in each thread's registers at once: a chunk of
// kBlkThreads * kBlkHeld positions is loaded before its colour runs are
// relaxed, so the chain of runs waits on LDS and barriers only, not on a
// global load per colour.  Thread t holds positions t, t + kBlkThreads, ...
// of the chunk (ascending, hence in colour order).
constexpr int kBlkHeld = 3;

// s_waitcnt immediate of gfx9-family targets: vector memory count 0 (bits 3:0 and 15:14), export and LDS counts
// left at their maxima (bits 6:4 = 7, 11:8 = 15).
constexpr int kWaitVmcnt0 = 0x0F70;

// A block's slot records staged into LDS ([8][ns]: v'x v'y v'z w'x w'y w'z
// 1/m 1/I) and written back (the first six) by the held form: kStage slots
// per thread at a time, their body indices loaded first and then their
// records as whole 16-byte pieces, so that a block waits on two memory round
// trips per kStage * NT slots instead of two per NT (the streamed FP32 form
// keeps one slot per step: measured faster there).
constexpr int kStage = 8;

__device__ inline void load_rec8(const double *p, double v[8]) {
    const double2 *q = reinterpret_cast<const double2 *>(p);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double2 x = q[k];
        v[2 * k] = x.x;
        v[2 * k + 1] = x.y;
    }
}

__device__ inline void load_rec8(const float *p, float v[8]) {
    const float4 *q = reinterpret_cast<const float4 *>(p);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const float4 x = q[k];
        v[4 * k] = x.x;
        v[4 * k + 1] = x.y;
        v[4 * k + 2] = x.z;
        v[4 * k + 3] = x.w;
    }
}

// The solver records in the block-local sweeps' order (block_records): the
// first grid's slots take records 0 .. s0 - 1 in slot order, every other body
// the next records in index order.
__global__ void __launch_bounds__(kBlock) k_rec_first(const int32_t *slots, int64_t s0, int32_t *rec_of) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s < s0) rec_of[slots[s]] = (int32_t)s;
}

__global__ void __launch_bounds__(kBlock) k_rec_flags(const int32_t *rec_of, int32_t n, int32_t *flags) {
    const int32_t i = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (i < n) flags[i] = rec_of[i] < 0 ? 1 : 0;
}

__global__ void __launch_bounds__(kBlock) k_rec_rest(const int32_t *ex, int32_t n, int32_t s0, int32_t *rec_of,
                                                     int32_t *body_of) {
    const int32_t i = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (i >= n) return;
    int32_t r = rec_of[i];
    if (r < 0) {
        r = s0 + ex[i];
        rec_of[i] = r;
    }
    if (r < n) body_of[r] = i;  // a permutation when no body is a slot of two of the first grid's blocks
}

__global__ void __launch_bounds__(kBlock) k_slot_rec(const int32_t *slots, int64_t ns, const int32_t *rec_of,
                                                     int32_t *slot_rec) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s < ns) slot_rec[s] = rec_of[slots[s]];
}

__global__ void __launch_bounds__(kBlock) k_ends_rec(const int32_t *j1, const int32_t *j2, int64_t m, int32_t n,
                                                     const int32_t *rec_of, int32_t *j1r, int32_t *j2r) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= m) return;
    j1r[p] = rec_of[j1[p]];
    const int32_t k = j2[p];
    j2r[p] = k < n ? rec_of[k] : k;  // walls keep their index
}

template <class T, int NT>
__device__ inline void blk_stage(T *Vs, int ns, const T *vel, const int32_t *slot_body, int s0, int t) {
    for (int i0 = 0; i0 < ns; i0 += kStage * NT) {
        int32_t bi[kStage];
#pragma unroll
        for (int k = 0; k < kStage; ++k) {
            const int i = i0 + t + k * NT;
            bi[k] = i < ns ? slot_body[s0 + i] : -1;
        }
        T rec[kStage][8];
#pragma unroll
        for (int k = 0; k < kStage; ++k)
            if (bi[k] >= 0) load_rec8(vel + 8 * (int64_t)bi[k], rec[k]);
#pragma unroll
        for (int k = 0; k < kStage; ++k) {
            const int i = i0 + t + k * NT;
            if (i < ns) {
#pragma unroll
                for (int a = 0; a < 8; ++a) Vs[a * ns + i] = rec[k][a];
            }
        }
    }
}

template <class T, int NT>
__device__ inline void blk_write_back(const T *Vs, int ns, T *vel, const int32_t *slot_body, int s0, int t) {
    for (int i0 = 0; i0 < ns; i0 += kStage * NT) {
        int32_t bi[kStage];
#pragma unroll
        for (int k = 0; k < kStage; ++k) {
            const int i = i0 + t + k * NT;
            bi[k] = i < ns ? slot_body[s0 + i] : -1;
        }
#pragma unroll
        for (int k = 0; k < kStage; ++k)
            if (bi[k] >= 0) {
                const int i = i0 + t + k * NT;
                T *r = vel + 8 * (int64_t)bi[k];
#pragma unroll
                for (int a = 0; a < 6; ++a) r[a] = Vs[a * ns + i];
            }
    }
}

// One local contact's data, loaded ahead of its colour run.
template <class T>
struct HeldContact {
    T n[3], a1, a2, P[3], bias;
    int32_t ls;  // the two int16 end slots (>= 0 slot, -1 static body, -2 wall)
};

template <class T, int MODE>
__device__ inline void blk_load(const SubView<T> &sv, int64_t p, HeldContact<T> &h) {
    h.n[0] = sv.nx[p];
    h.n[1] = sv.ny[p];
    h.n[2] = sv.nz[p];
    h.a1 = sv.a1[p];
    h.a2 = sv.a2[p];
    h.P[0] = sv.px[p];
    h.P[1] = sv.py[p];
    h.P[2] = sv.pz[p];
    h.bias = MODE == 1 ? sv.bias[p] : T(0);
    h.ls = reinterpret_cast<const int32_t *>(sv.ls)[p];  // ls[2 p], ls[2 p + 1] in one aligned word
}

template <class T>
__device__ inline void blk_end_rec(const T *Vs, int ns, const T *vel, int l, const int32_t *j, int64_t p,
                                   Rec<T> &r) {
    if (l >= 0) {
        r.v[0] = Vs[0 * ns + l];
        r.v[1] = Vs[1 * ns + l];
        r.v[2] = Vs[2 * ns + l];
        r.w[0] = Vs[3 * ns + l];
        r.w[1] = Vs[4 * ns + l];
        r.w[2] = Vs[5 * ns + l];
        r.im = Vs[6 * ns + l];
        r.ii = Vs[7 * ns + l];
    } else if (l == -1) {  // a static body: its record never changes
        const T *g = vel + 8 * (int64_t)j[p];
        r.v[0] = g[0];
        r.v[1] = g[1];
        r.v[2] = g[2];
        r.w[0] = g[3];
        r.w[1] = g[4];
        r.w[2] = g[5];
        r.im = g[6];
        r.ii = g[7];
        // Wait for these loads here, on this rare path: otherwise the merge with the LDS path above waits for every
        // outstanding vector memory operation (the impulse stores of the contacts before included) on every contact.
        __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    } else {  // a wall
        r = zero_rec<T>();
    }
}

template <class T>
__device__ inline void blk_store_rec(T *Vs, int ns, int l, const Rec<T> &r) {
    if (l >= 0 && r.im > T(0)) {
        Vs[0 * ns + l] = r.v[0];
        Vs[1 * ns + l] = r.v[1];
        Vs[2 * ns + l] = r.v[2];
        Vs[3 * ns + l] = r.w[0];
        Vs[4 * ns + l] = r.w[1];
        Vs[5 * ns + l] = r.w[2];
    }
}

// One pass over the local contacts of every block of one grid, one workgroup
// per block, the block's body records in LDS.  MODE 0 applies the initial
// impulses, MODE 1 relaxes (Alg. 1) and leaves the block's residual sums in
// partials[2 s], [2 s + 1].  Colour runs in order, a barrier after each.
template <class T, int MODE>
__global__ void __launch_bounds__(kBlkThreads) k_blk_pass(SubView<T> sv, int32_t nb, T *vel, T mu, T relax,
                                                          const int64_t *tile_off, const int32_t *tile_slot_off,
                                                          const int32_t *slot_body, const int32_t *blk_cs,
                                                          const int32_t *blk_nrun, double *partials,
                                                          const int32_t *ctrl, int32_t id0) {
    (void)nb;
    if (MODE == 1 && ctrl[0]) return;  // an earlier sweep met the target (uniform over the grid)
    extern __shared__ __align__(16) unsigned char smem[];
    const int s = id0 + (int)blockIdx.x;  // this launch's blocks: ids id0 .. id0 + gridDim.x - 1
    const int64_t c0 = tile_off[s];
    const int count = (int)(tile_off[s + 1] - c0);
    const int s0 = tile_slot_off[s], ns = tile_slot_off[s + 1] - s0;
    T *Vs = reinterpret_cast<T *>(smem);  // [8][ns]: v'x v'y v'z w'x w'y w'z 1/m 1/I
    __shared__ int32_t cstart[kMaxCol + 1];
    const int32_t *cs = blk_cs + c0 + s;  // the block's colour runs
    const int ncol = blk_nrun[s];
    constexpr int kHeld = kBlkHeld, kChunk = kBlkThreads * kHeld;
    const int t = threadIdx.x;
    HeldContact<T> held[kHeld];
    // the first chunk's loads and the colour runs' starts go out before the block's records are staged
#pragma unroll
    for (int k = 0; k < kHeld; ++k)
        if (t + k * kBlkThreads < count) blk_load<T, MODE>(sv, c0 + t + k * kBlkThreads, held[k]);
    const int32_t cs0 = t <= ncol ? cs[t] : 0;
    blk_stage<T, kBlkThreads>(Vs, ns, vel, slot_body, s0, t);
    if (t <= ncol) cstart[t] = cs0;
    for (int c = t + kBlkThreads; c <= ncol; c += kBlkThreads) cstart[c] = cs[c];
    __syncthreads();
    double sd = 0.0, sp = 0.0;
    int run = 0;  // the colour run being relaxed (uniform)
    for (int q0 = 0; q0 < count; q0 += kChunk) {
        const int qend = min(count, q0 + kChunk);
        if (q0 > 0) {
#pragma unroll
            for (int k = 0; k < kHeld; ++k)
                if (q0 + t + k * kBlkThreads < qend) blk_load<T, MODE>(sv, c0 + q0 + t + k * kBlkThreads, held[k]);
        }
        while (run < ncol && cstart[run] < qend) {
            const int qa = max(cstart[run], q0), qb = min(cstart[run + 1], qend);
#pragma unroll
            for (int k = 0; k < kHeld; ++k) {
                const int q = q0 + t + k * kBlkThreads;
                if (q < qa || q >= qb) continue;
                const HeldContact<T> &h = held[k];
                if (MODE == 0 && h.P[0] == T(0) && h.P[1] == T(0) && h.P[2] == T(0)) continue;
                const int64_t p = c0 + q;
                const int l1 = (int)(int16_t)(h.ls & 0xffff), l2 = (int)(int16_t)((uint32_t)h.ls >> 16);
                Rec<T> r1, r2;
                blk_end_rec(Vs, ns, vel, l1, sv.j1, p, r1);
                blk_end_rec(Vs, ns, vel, l2, sv.j2, p, r2);
                if (MODE == 0) {
                    apply(r1, r2, h.n, h.a1, h.a2, h.P);
                } else {
                    T Pnew[3], dP[3];
                    relax_contact(h.n, h.bias, h.a1, h.a2, h.P, mu, relax, r1, r2, Pnew, dP);
                    sv.px[p] = Pnew[0];
                    sv.py[p] = Pnew[1];
                    sv.pz[p] = Pnew[2];
                    const double d0 = dP[0], d1 = dP[1], d2 = dP[2];
                    const double e0 = Pnew[0], e1 = Pnew[1], e2 = Pnew[2];
                    sd += d0 * d0 + d1 * d1 + d2 * d2;
                    sp += e0 * e0 + e1 * e1 + e2 * e2;
                }
                blk_store_rec(Vs, ns, l1, r1);
                blk_store_rec(Vs, ns, l2, r2);
            }
            __syncthreads();
            if (cstart[run + 1] > qend) break;  // the run goes on in the next chunk
            ++run;
        }
    }
    blk_write_back<T, kBlkThreads>(Vs, ns, vel, slot_body, s0, (int)threadIdx.x);
    if (MODE == 1) {
        __shared__ double red[2][kBlkThreads / 64];
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
            for (int w = 0; w < kBlkThreads / 64; ++w) {
                a += red[0][w];
                c += red[1][w];
            }
            partials[2 * s + 0] = a;
            partials[2 * s + 1] = c;
        }
    }
}

// The same pass with each colour run's contacts loaded when the run starts
// (one thread per contact of the run, 128 threads): fewer registers, so more
// workgroups per CU hide the load of each run; the faster form for FP32 records.
template <class T, int MODE>
__global__ void __launch_bounds__(kBlkStreamThreads) k_blk_pass_stream(SubView<T> sv, int32_t nb, T *vel, T mu, T relax,
                                                          const int64_t *tile_off, const int32_t *tile_slot_off,
                                                          const int32_t *slot_body, const int32_t *blk_cs,
                                                          const int32_t *blk_nrun, double *partials,
                                                          const int32_t *ctrl, int32_t id0) {
    if (MODE == 1 && ctrl[0]) return;  // an earlier sweep met the target (uniform over the grid)
    extern __shared__ __align__(16) unsigned char smem[];
    const int s = id0 + (int)blockIdx.x;  // this launch's blocks: ids id0 .. id0 + gridDim.x - 1
    const int64_t c0 = tile_off[s];
    const int s0 = tile_slot_off[s], ns = tile_slot_off[s + 1] - s0;
    T *Vs = reinterpret_cast<T *>(smem);  // [8][ns]: v'x v'y v'z w'x w'y w'z 1/m 1/I
    __shared__ int32_t cstart[kMaxCol + 1];
    const int32_t *cs = blk_cs + c0 + s;  // the block's colour runs
    const int ncol = blk_nrun[s];
    for (int i = threadIdx.x; i < ns; i += kBlkStreamThreads) {
        const T *r = vel + 8 * (int64_t)slot_body[s0 + i];
#pragma unroll
        for (int a = 0; a < 8; ++a) Vs[a * ns + i] = r[a];
    }
    for (int c = threadIdx.x; c <= ncol; c += kBlkStreamThreads) cstart[c] = cs[c];
    __syncthreads();
    double sd = 0.0, sp = 0.0;
    for (int c = 0; c < ncol; ++c) {
        const int64_t pa = c0 + cstart[c], pb = c0 + cstart[c + 1];
        for (int64_t p = pa + threadIdx.x; p < pb; p += kBlkStreamThreads) {
            const int l1 = sv.ls[2 * p], l2 = sv.ls[2 * p + 1];
            // body indices are read only for ends outside the block's slots (walls and static bodies)
            const int b1 = l1 >= 0 ? 0 : sv.j1[p], b2 = l2 >= 0 ? 0 : sv.j2[p];
            const T n[3] = {sv.nx[p], sv.ny[p], sv.nz[p]};
            const T a1 = sv.a1[p], a2 = sv.a2[p];
            const T P[3] = {sv.px[p], sv.py[p], sv.pz[p]};
            if (MODE == 0 && P[0] == T(0) && P[1] == T(0) && P[2] == T(0)) continue;
            Rec<T> r1, r2;
            if (l1 >= 0) {
                r1.v[0] = Vs[0 * ns + l1];
                r1.v[1] = Vs[1 * ns + l1];
                r1.v[2] = Vs[2 * ns + l1];
                r1.w[0] = Vs[3 * ns + l1];
                r1.w[1] = Vs[4 * ns + l1];
                r1.w[2] = Vs[5 * ns + l1];
                r1.im = Vs[6 * ns + l1];
                r1.ii = Vs[7 * ns + l1];
            } else {
                const T *r = vel + 8 * (int64_t)b1;
                r1.v[0] = r[0];
                r1.v[1] = r[1];
                r1.v[2] = r[2];
                r1.w[0] = r[3];
                r1.w[1] = r[4];
                r1.w[2] = r[5];
                r1.im = r[6];
                r1.ii = r[7];
            }
            if (l2 >= 0) {
                r2.v[0] = Vs[0 * ns + l2];
                r2.v[1] = Vs[1 * ns + l2];
                r2.v[2] = Vs[2 * ns + l2];
                r2.w[0] = Vs[3 * ns + l2];
                r2.w[1] = Vs[4 * ns + l2];
                r2.w[2] = Vs[5 * ns + l2];
                r2.im = Vs[6 * ns + l2];
                r2.ii = Vs[7 * ns + l2];
            } else if (b2 < nb) {
                const T *r = vel + 8 * (int64_t)b2;
                r2.v[0] = r[0];
                r2.v[1] = r[1];
                r2.v[2] = r[2];
                r2.w[0] = r[3];
                r2.w[1] = r[4];
                r2.w[2] = r[5];
                r2.im = r[6];
                r2.ii = r[7];
            } else {
                r2 = zero_rec<T>();
            }
            if (MODE == 0) {
                apply(r1, r2, n, a1, a2, P);
            } else {
                T Pnew[3], dP[3];
                relax_contact(n, sv.bias[p], a1, a2, P, mu, relax, r1, r2, Pnew, dP);
                sv.px[p] = Pnew[0];
                sv.py[p] = Pnew[1];
                sv.pz[p] = Pnew[2];
                const double d0 = dP[0], d1 = dP[1], d2 = dP[2];
                const double q0 = Pnew[0], q1 = Pnew[1], q2 = Pnew[2];
                sd += d0 * d0 + d1 * d1 + d2 * d2;
                sp += q0 * q0 + q1 * q1 + q2 * q2;
            }
            if (l1 >= 0 && r1.im > T(0)) {
                Vs[0 * ns + l1] = r1.v[0];
                Vs[1 * ns + l1] = r1.v[1];
                Vs[2 * ns + l1] = r1.v[2];
                Vs[3 * ns + l1] = r1.w[0];
                Vs[4 * ns + l1] = r1.w[1];
                Vs[5 * ns + l1] = r1.w[2];
            }
            if (l2 >= 0 && r2.im > T(0)) {
                Vs[0 * ns + l2] = r2.v[0];
                Vs[1 * ns + l2] = r2.v[1];
                Vs[2 * ns + l2] = r2.v[2];
                Vs[3 * ns + l2] = r2.w[0];
                Vs[4 * ns + l2] = r2.w[1];
                Vs[5 * ns + l2] = r2.w[2];
            }
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < ns; i += kBlkStreamThreads) {
        T *r = vel + 8 * (int64_t)slot_body[s0 + i];
#pragma unroll
        for (int a = 0; a < 6; ++a) r[a] = Vs[a * ns + i];
    }
    if (MODE == 1) {
        __shared__ double red[2][kBlkStreamThreads / 64];
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
            for (int w = 0; w < kBlkStreamThreads / 64; ++w) {
                a += red[0][w];
                c += red[1][w];
            }
            partials[2 * s + 0] = a;
            partials[2 * s + 1] = c;
        }
    }
}

}  // namespace

// The box cut into max(1, floor(L_a / edge)) blocks of edge L_a / that count per axis.
static nbgs_status make_blocks(nbgs_scene_t sc, double edge, Blocks &bl, int64_t &nblocks) {
    nblocks = 1;
    for (int a = 0; a < 3; ++a) {
        const double L = sc->hi[a] - sc->lo[a];
        double c = std::floor(L / edge);
        if (!(c >= 1.0)) c = 1.0;
        if (c > 4096.0) {
            set_error("%g blocks along an axis are too many: use a larger edge", c);
            return NBGS_ERR_INVALID_ARG;
        }
        bl.lo[a] = sc->lo[a];
        bl.nb[a] = (int32_t)c;
        bl.e[a] = L / c;
        nblocks *= (int64_t)c;
    }
    if (nblocks > (1 << 23) - 1) {
        set_error("%lld blocks are too many: use a larger edge", (long long)nblocks);
        return NBGS_ERR_INVALID_ARG;
    }
    return NBGS_OK;
}

// Ids of the scene's sweep order: the subdomains, or the blocks of the
// block-local order over all its grids plus the id of the contacts between
// blocks; 0 in the classic order.  Host arithmetic only (the tables sized by
// it count towards the workspace a detection needs).
nbgs_status order_ids(nbgs_scene_t sc, int64_t *ids) {
    *ids = 0;
    Blocks bl;
    int64_t nblocks = 1;
    if (sc->sub_edge > 0.0) {
        NBGS_TRY(make_blocks(sc, sc->sub_edge, bl, nblocks));
        *ids = nblocks;
    } else if (sc->blk_edge > 0.0) {
        NBGS_TRY(make_blocks(sc, sc->blk_edge, bl, nblocks));
        if (sc->blk_grids > 1) {
            int64_t B = 1;  // a shifted grid has one more block along a non-periodic axis
            for (int a = 0; a < 3; ++a) B *= bl.nb[a] + (sc->periodic[a] ? 0 : 1);
            nblocks = (int64_t)sc->blk_grids * B;
        }
        *ids = nblocks + 1;
    }
    return NBGS_OK;
}

// Subdomains of the contacts and, when the colouring is done, the tile and slot tables.
nbgs_status subdomain_assign(nbgs_scene_t sc) {
    hipStream_t s = sc->s;
    Blocks bl;
    int64_t nsub = 1;
    NBGS_TRY(make_blocks(sc, sc->sub_edge, bl, nsub));
    sc->n_sub = (int32_t)nsub;
    const int64_t nc = sc->nc;
    NBGS_TRY(sc->sdom.reserve((size_t)nc + 1));
    k_subdomain<<<grid_for(nc), kBlock, 0, s>>>(sc->b, sc->cb[sc->cur].j1.p, nc, bl, sc->sdom.p);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

// Groups of the contacts that no grid's block holds (k_cross_flags): with
// several grids their clusters are packed into *groups ids n_blk .. n_blk +
// *groups - 1, swept by the block pass, when the labelling settles within its
// round limit and every group fits a workgroup's LDS (kGroupMaxContacts);
// otherwise they keep the id n_blk and *groups = 0 (the colour launches).
// The id after the groups, n_blk + *groups, is that of the contacts swept by
// colour, which then holds none.
constexpr int32_t kGroupTarget = 1536;       // about six groups per compute unit
constexpr int32_t kGroupMaxContacts = 448;   // at most 896 slots: 56 KB of FP64 records
constexpr int kGroupMaxRounds = 48;

static nbgs_status cross_groups(nbgs_scene_t sc, int32_t *groups) {
    hipStream_t s = sc->s;
    *groups = 0;
    const int64_t nc = sc->nc;
    const int32_t N = sc->b.n, cross = sc->n_blk;
    if (nc <= 0 || nc >= (int64_t)0x3fffffff) return NBGS_OK;
    // scratch: tables the step's later set-up reserves at these sizes anyway
    const int64_t ne = 2 * nc;
    for (DevBuf<int32_t> *b : {&sc->eflags, &sc->eex}) NBGS_TRY(b->reserve((size_t)ne + 1));
    for (DevBuf<uint32_t> *b : {&sc->ekeys, &sc->evals}) NBGS_TRY(b->reserve((size_t)ne + 1));
    NBGS_TRY(sc->cursor.reserve((size_t)N + 1));
    NBGS_TRY(sc->xg_ctl.reserve(64, 1.0));
    const size_t need_tmp = exclusive_scan_tmp_bytes(nc + 2);
    if (need_tmp > sc->scan_tmp.cap) NBGS_TRY(sc->scan_tmp.reserve(need_tmp));
    int32_t *flag = sc->eflags.p, *pos = sc->eex.p, *blab = sc->cursor.p;
    int32_t *xl = reinterpret_cast<int32_t *>(sc->ekeys.p), *lab = reinterpret_cast<int32_t *>(sc->evals.p);
    const int32_t *j1 = sc->cb[sc->cur].j1.p, *j2 = sc->cb[sc->cur].j2.p;
    k_cross_flags<<<grid_for(nc), kBlock, 0, s>>>(sc->sdom.p, nc, cross, flag);
    NBGS_HIP(hipGetLastError());
    NBGS_TRY(exclusive_scan_i32(flag, pos, nc, sc->total(), sc->scan_tmp.p, sc->scan_tmp.cap, s));
    NBGS_TRY(scene_sync_small(sc, 0, 1));
    const int32_t nx = sc->pinned[0];
    if (nx <= 0) return NBGS_OK;
    k_cross_list<<<grid_for(nc), kBlock, 0, s>>>(sc->sdom.p, pos, nc, cross, xl, lab);
    k_fill<<<grid_for(N), kBlock, 0, s>>>(blab, N, 0x7fffffff);
    k_fill<<<1, kBlock, 0, s>>>(sc->xg_ctl.p, 64, 0);
    NBGS_HIP(hipGetLastError());
    const unsigned gx = grid_for(nx);
    int rounds = 0;
    bool settled = false;
    for (int batch = 4; rounds < kGroupMaxRounds && !settled; batch *= 2) {
        for (int r = 0; r < batch && rounds < kGroupMaxRounds; ++r, ++rounds) {
            k_cc_push<<<gx, kBlock, 0, s>>>(xl, nx, j1, j2, N, sc->b.inv_mass, lab, blab);
            k_cc_pull<<<gx, kBlock, 0, s>>>(xl, nx, j1, j2, N, sc->b.inv_mass, lab, blab, sc->xg_ctl.p + rounds);
        }
        NBGS_HIP(hipGetLastError());
        NBGS_HIP(hipMemcpyAsync(sc->pinned + 96, sc->xg_ctl.p + rounds - 1, sizeof(int32_t), hipMemcpyDeviceToHost,
                                s));
        NBGS_HIP(hipStreamSynchronize(s));
        settled = sc->pinned[96] == 0;  // the last round moved no label
    }
    if (!settled) return NBGS_OK;
    const int32_t per = std::max<int32_t>(16, (nx + kGroupTarget - 1) / kGroupTarget);
    const int32_t ng = (nx + per - 1) / per;
    NBGS_TRY(sc->xg_cnt.reserve((size_t)ng + 1));
    k_fill<<<grid_for(ng), kBlock, 0, s>>>(sc->xg_cnt.p, ng, 0);
    k_cc_ids<<<gx, kBlock, 0, s>>>(xl, nx, lab, cross, per, sc->sdom.p, sc->xg_cnt.p);
    k_max_i32<<<grid_for(ng), kBlock, 0, s>>>(sc->xg_cnt.p, ng, sc->xg_ctl.p + 63);
    NBGS_HIP(hipGetLastError());
    NBGS_HIP(hipMemcpyAsync(sc->pinned + 96, sc->xg_ctl.p + 63, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    NBGS_HIP(hipStreamSynchronize(s));
    if (sc->pinned[96] > kGroupMaxContacts) {  // a group too large for LDS: back to the colour launches
        k_cc_reset<<<gx, kBlock, 0, s>>>(xl, nx, cross, sc->sdom.p);
        NBGS_HIP(hipGetLastError());
        return NBGS_OK;
    }
    *groups = ng;
    return NBGS_OK;
}

// Block-local ids of the contacts: ids 0 .. n_blk - 1 local, n_blk between blocks.
// maybe_reuse: every pair of this step is one of the last step's (as far as the match has counted: small[4]), the
// dynamic bits are known (small[7] counts their changes) and the last step used this order; then, when no pair's
// grid id changed either, the clusters of the contacts local in no grid and their groups are the last step's.
nbgs_status block_assign(nbgs_scene_t sc, int32_t *changed, bool maybe_reuse) {
    hipStream_t s = sc->s;
    Blocks bl;
    int64_t nblocks = 1;
    NBGS_TRY(make_blocks(sc, sc->blk_edge, bl, nblocks));
    const int64_t nc = sc->nc;
    NBGS_TRY(sc->sdom.reserve((size_t)nc + 1));
    const ContactsView c = sc->cb[sc->cur].view();
    if (sc->blk_grids <= 1) {
        sc->n_blk = (int32_t)nblocks;
        sc->blk_grid_ids = (int32_t)nblocks;
        k_block_local<<<grid_for(nc), kBlock, 0, s>>>(sc->b, c.j1, c.j2, nc, bl, (int32_t)nblocks, sc->sdom.p);
    } else {
        // a shifted grid has one more block along a non-periodic axis
        int32_t M[3];
        int64_t B = 1;
        for (int a = 0; a < 3; ++a) {
            M[a] = bl.nb[a] + (sc->periodic[a] ? 0 : 1);
            B *= M[a];
        }
        if ((int64_t)sc->blk_grids * B > (1 << 23) - 1) {
            set_error("%lld blocks in %d grids are too many: use a larger edge", (long long)B, sc->blk_grids);
            return NBGS_ERR_INVALID_ARG;
        }
        sc->n_blk = sc->blk_grids * (int32_t)B;
        sc->blk_grid_ids = (int32_t)B;
        k_block_local_grids<<<grid_for(nc), kBlock, 0, s>>>(sc->b, c.j1, c.j2, nc, bl, sc->blk_grids, M[0], M[1], M[2],
                                                            sc->periodic[0], sc->periodic[1], sc->periodic[2],
                                                            sc->sdom.p);
    }
    const int32_t prev_groups = sc->blk_groups;
    sc->blk_groups = 0;
    if (sc->blk_grids > 1 && sc->blk_group_cross) {
        bool reused = false;
        if (maybe_reuse && sc->xg_prev_valid && sc->xg_prev_nblk == sc->n_blk && sc->prev_sdom.p && nc > 0) {
            NBGS_TRY(sc->xg_ctl.reserve(64, 1.0));
            k_fill<<<1, kBlock, 0, s>>>(sc->xg_ctl.p + 60, 1, 0);
            k_raw_ids_changed<<<grid_for(nc), kBlock, 0, s>>>(sc->sdom.p, sc->prev_sdom.p, c.matched, nc, sc->n_blk,
                                                             sc->xg_ctl.p + 60);
            NBGS_HIP(hipGetLastError());
            NBGS_HIP(hipMemcpyAsync(sc->pinned + 96, sc->xg_ctl.p + 60, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            NBGS_TRY(scene_sync_small(sc, 4, 4));
            if (sc->pinned[96] == 0 && sc->pinned[4] == 0 && sc->pinned[7] == 0) {
                k_ids_from_prev<<<grid_for(nc), kBlock, 0, s>>>(sc->prev_sdom.p, c.matched, nc, sc->sdom.p);
                NBGS_HIP(hipGetLastError());
                sc->blk_groups = prev_groups;
                reused = true;
            }
        }
        if (!reused) NBGS_TRY(cross_groups(sc, &sc->blk_groups));
        sc->xg_prev_valid = true;
        sc->xg_prev_nblk = sc->n_blk;
    } else {
        sc->xg_prev_valid = false;
    }
    sc->n_sub = sc->n_blk + sc->blk_groups + 1;
    NBGS_HIP(hipGetLastError());
    // every body's block, compared with the last step's (bodies without local contacts count too: they decide the
    // slots); the number of changes is added to changed
    const int32_t N = sc->b.n;
    NBGS_TRY(sc->bblk[0].reserve((size_t)N + 1));
    NBGS_TRY(sc->bblk[1].reserve((size_t)N + 1));
    const int k = sc->bblk_cur;
    const int compare = sc->bblk_valid && sc->bblk_nblocks == nblocks ? 1 : 0;
    k_body_blocks_cmp<<<grid_for(N), kBlock, 0, s>>>(sc->b, bl, (int32_t)nblocks, sc->bblk[k].p, sc->bblk[1 - k].p,
                                                     compare, changed);
    NBGS_HIP(hipGetLastError());
    sc->bblk_compared = compare != 0;
    sc->bblk_nblocks = nblocks;
    return NBGS_OK;
}

static nbgs_status cross_colours(nbgs_scene_t sc, const int32_t *col, const int32_t *sj1, const int32_t *sj2,
                                 int64_t xb, int64_t xe);
template <class T>
static nbgs_status prepare_impl(nbgs_scene_t sc, int32_t no_slot = -1, int values_per_slot = 14,
                                bool body_lists = true);

// Block-local order, per step: contact ranges of the ids (the sweep record
// is sorted by id), the slots -- every dynamic body of a block, bodies sorted
// by block (index order inside a block) -- and each local contact end's slot,
// the LDS limit, and the colour ranges and dynamic ends of the contacts
// between blocks.
template <class T>
static nbgs_status block_prepare_impl(nbgs_scene_t sc) {
    hipStream_t s = sc->s;
    const int64_t nc = sc->nc;
    const int32_t N = sc->b.n;
    const int32_t nsub = sc->n_sub, nblk = sc->n_blk;
    SweepBuf<T> &sw = sc->precision_used == NBGS_FP32_SWEEP ? *reinterpret_cast<SweepBuf<T> *>(&sc->sw32)
                                                            : *reinterpret_cast<SweepBuf<T> *>(&sc->sw64);
    const int32_t *ssd = sw.sdom.p;
    // first sweep position of every id
    NBGS_TRY(sc->tile_off.reserve((size_t)nsub + 1));
    k_fill64<<<grid_for((int64_t)nsub + 1), kBlock, 0, s>>>(sc->tile_off.p, (int64_t)nsub + 1, -1);
    k_first_of_runs<<<grid_for(nc), kBlock, 0, s>>>(ssd, nc, sc->tile_off.p);
    NBGS_HIP(hipGetLastError());
    // bodies sorted by block (static bodies last), the slot of every body, the first slot of every block
    Blocks bl;
    int64_t nblocks = 1;
    NBGS_TRY(make_blocks(sc, sc->blk_edge, bl, nblocks));
    for (DevBuf<uint32_t> *b : {&sc->bkeys, &sc->bvals, &sc->bkeys2, &sc->bvals2}) NBGS_TRY(b->reserve((size_t)N + 1));
    NBGS_TRY(sc->body_cnt.reserve((size_t)N + 1));  // the slot of every body
    NBGS_TRY(sc->tile_slot_off.reserve((size_t)nblk + 2));
    k_body_blocks<<<grid_for(N), kBlock, 0, s>>>(sc->b, bl, nblk, sc->bkeys.p, sc->bvals.p);
    NBGS_HIP(hipGetLastError());
    if ((size_t)radix_hist_entries(N) > sc->radix_hist.cap) NBGS_TRY(sc->radix_hist.reserve(radix_hist_entries(N)));
    const size_t need_tmp = exclusive_scan_tmp_bytes((int64_t)radix_hist_entries(N));
    if (need_tmp > sc->scan_tmp.cap) NBGS_TRY(sc->scan_tmp.reserve(need_tmp));
    int bits = 1;
    while (((int64_t)1 << bits) < (int64_t)nblk + 1) ++bits;
    bool alt = false;
    NBGS_TRY(radix_sort_pairs(sc->bkeys.p, sc->bvals.p, sc->bkeys2.p, sc->bvals2.p, N, bits, sc->radix_hist.p,
                              sc->scan_tmp.p, sc->scan_tmp.cap, &alt, s));
    const uint32_t *skeys = alt ? sc->bkeys2.p : sc->bkeys.p;
    const uint32_t *sbody = alt ? sc->bvals2.p : sc->bvals.p;
    if (N == 1) {
        skeys = sc->bkeys.p;
        sbody = sc->bvals.p;
    }
    sc->body_slots = sbody;
    k_slot_of<<<grid_for(N), kBlock, 0, s>>>(sbody, N, sc->body_cnt.p);
    k_fill<<<grid_for((int64_t)nblk + 2), kBlock, 0, s>>>(sc->tile_slot_off.p, (int64_t)nblk + 2, -1);
    k_first_of_runs32<<<grid_for(N), kBlock, 0, s>>>(skeys, N, sc->tile_slot_off.p);
    NBGS_HIP(hipGetLastError());
    // empty ids and blocks start where the next one does (host, small tables)
    std::vector<int64_t> toff((size_t)nsub + 1);
    std::vector<int32_t> soff((size_t)nblk + 2);
    NBGS_HIP(hipMemcpyAsync(toff.data(), sc->tile_off.p, sizeof(int64_t) * (nsub + 1), hipMemcpyDeviceToHost, s));
    NBGS_HIP(hipMemcpyAsync(soff.data(), sc->tile_slot_off.p, sizeof(int32_t) * (nblk + 2), hipMemcpyDeviceToHost, s));
    NBGS_HIP(hipStreamSynchronize(s));
    toff[(size_t)nsub] = nc;
    for (int32_t t = nsub - 1; t >= 0; --t)
        if (toff[(size_t)t] < 0) toff[(size_t)t] = toff[(size_t)t + 1];
    soff[(size_t)nblk + 1] = N;
    for (int32_t t = nblk; t >= 0; --t)
        if (soff[(size_t)t] < 0) soff[(size_t)t] = soff[(size_t)t + 1];
    int32_t max_slots = 0;
    for (int32_t t = 0; t < nblk; ++t) max_slots = std::max(max_slots, soff[(size_t)t + 1] - soff[(size_t)t]);
    const size_t lds = (size_t)max_slots * 8 * sizeof(T);
    if (lds > 60 * 1024) {
        set_error("a block holds %d bodies (%zu bytes of LDS); use a smaller block edge", max_slots, lds);
        return NBGS_ERR_CAPACITY;
    }
    sc->max_slots = max_slots;
    sc->launch_id0.assign(1, 0);
    sc->launch_n.assign(1, nblk);
    sc->launch_slots.assign(1, max_slots);
    sc->slot_s0 = N;  // one grid: every body has a slot (static bodies last)
    sc->n_slots = soff[(size_t)nblk];
    NBGS_HIP(hipMemcpyAsync(sc->tile_off.p, toff.data(), sizeof(int64_t) * (nsub + 1), hipMemcpyHostToDevice, s));
    NBGS_HIP(hipMemcpyAsync(sc->tile_slot_off.p, soff.data(), sizeof(int32_t) * (nblk + 2), hipMemcpyHostToDevice, s));
    // slot of every local contact end
    NBGS_TRY(sw.ls.reserve(2 * (size_t)nc + 1));
    k_block_ends<<<grid_for(nc), kBlock, 0, s>>>(sw.j1.p, sw.j2.p, ssd, nc, nblk, N, sc->b.inv_mass, sc->body_cnt.p,
                                                  sc->tile_slot_off.p, sw.ls.p);
    NBGS_HIP(hipGetLastError());
    // colour runs of every block's local contacts
    NBGS_TRY(sc->blk_cs.reserve((size_t)nc + nblk + 1));
    NBGS_TRY(sc->blk_nrun.reserve((size_t)nblk + 1));
    k_blk_colour_runs<<<(unsigned)nblk, kBlkThreads, 0, s>>>(sw.col.p, sc->tile_off.p, sc->blk_cs.p,
                                                             sc->blk_nrun.p);
    NBGS_HIP(hipGetLastError());
    // colours of the contacts between blocks (the last id's range)
    NBGS_TRY(cross_colours(sc, sw.col.p, sw.j1.p, sw.j2.p, toff[(size_t)nblk], toff[(size_t)nsub]));
    sc->blk_dyn_local = sc->n_slots;
    sc->blk_n_local = toff[(size_t)nblk];
    return NBGS_OK;
}

// Colour ranges and dynamic ends of the contacts between blocks, sweep positions [xb, xe), to the host.
static nbgs_status cross_colours(nbgs_scene_t sc, const int32_t *col, const int32_t *sj1, const int32_t *sj2,
                                 int64_t xb, int64_t xe) {
    hipStream_t s = sc->s;
    const int32_t N = sc->b.n;
    NBGS_TRY(sc->xcol_d.reserve(kMaxCol + 1 + kMaxCol));
    NBGS_TRY(sc->xncol_d.reserve(1));
    std::vector<int64_t> init((size_t)kMaxCol + 1, xe);
    NBGS_HIP(hipMemcpyAsync(sc->xcol_d.p, init.data(), sizeof(int64_t) * (kMaxCol + 1), hipMemcpyHostToDevice, s));
    NBGS_HIP(hipMemsetAsync(sc->xcol_d.p + kMaxCol + 1, 0, sizeof(int64_t) * kMaxCol, s));
    NBGS_HIP(hipMemsetAsync(sc->xncol_d.p, 0, sizeof(int32_t), s));
    if (xe > xb) {
        const unsigned g = grid_for(xe - xb);
        k_range_colours<<<g, kBlock, 0, s>>>(col, xb, xe, sc->xcol_d.p, sc->xncol_d.p);
        k_range_dyn<<<g, kBlock, 0, s>>>(sj1, sj2, col, xb, xe, N, sc->b.inv_mass,
                                          reinterpret_cast<unsigned long long *>(sc->xcol_d.p + kMaxCol + 1));
        NBGS_HIP(hipGetLastError());
    }
    std::vector<int64_t> xc((size_t)2 * kMaxCol + 1);
    int32_t ncol = 0;
    NBGS_HIP(hipMemcpyAsync(xc.data(), sc->xcol_d.p, sizeof(int64_t) * (2 * kMaxCol + 1), hipMemcpyDeviceToHost, s));
    NBGS_HIP(hipMemcpyAsync(&ncol, sc->xncol_d.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    NBGS_HIP(hipStreamSynchronize(s));  // the host vectors above are temporaries
    for (int c = ncol - 1; c >= 0; --c)  // empty colours start where the next one does
        if (xc[(size_t)c] == xe) xc[(size_t)c] = c + 1 < ncol ? xc[(size_t)c + 1] : xe;
    sc->xcol.assign(xc.begin(), xc.begin() + ncol);
    sc->xcol.push_back(xe);
    sc->xdyn.assign(xc.begin() + kMaxCol + 1, xc.begin() + kMaxCol + 1 + ncol);
    return NBGS_OK;
}

// Block-local order over several grids, per step: the slot tables built from
// the ends of the local contacts (every dynamic body a block's local contacts
// touch; the contacts between blocks take none), each block's colour
// boundaries, and the colour ranges of the contacts between blocks.
template <class T>
static nbgs_status block_grids_prepare_impl(nbgs_scene_t sc) {
    hipStream_t s = sc->s;
    const int32_t nblk = sc->n_blk;
    SweepBuf<T> &sw = sc->precision_used == NBGS_FP32_SWEEP ? *reinterpret_cast<SweepBuf<T> *>(&sc->sw32)
                                                            : *reinterpret_cast<SweepBuf<T> *>(&sc->sw64);
    // the last id's contacts (between blocks, swept by colour) take no slot; blocks and groups do
    const int32_t nids = sc->n_sub - 1;
    (void)nblk;
    NBGS_TRY(prepare_impl<T>(sc, nids, 8, false));
    NBGS_TRY(sc->blk_cs.reserve((size_t)sc->nc + nids + 1));
    NBGS_TRY(sc->blk_nrun.reserve((size_t)nids + 1));
    k_blk_colour_runs<<<(unsigned)nids, kBlkThreads, 0, s>>>(sw.col.p, sc->tile_off.p, sc->blk_cs.p,
                                                             sc->blk_nrun.p);
    NBGS_HIP(hipGetLastError());
    NBGS_TRY(cross_colours(sc, sw.col.p, sw.j1.p, sw.j2.p, sc->blk_first_cross, sc->nc));
    sc->blk_dyn_local = sc->n_slots;
    sc->blk_n_local = sc->blk_first_cross;
    return NBGS_OK;
}

static nbgs_status body_slot_lists(nbgs_scene_t sc, int64_t nslots);

// Slot tables of the subdomain solver (no_slot = -1, 14 values per slot in
// LDS, per-body slot lists for the correction reduction), also used for the
// block-local order over several grids (no_slot = the id of the contacts
// between blocks, 8 values per slot, no per-body lists): per id its contact
// range, per slot its body and id, per id its slot range, per contact end its
// local slot.
template <class T>
static nbgs_status prepare_impl(nbgs_scene_t sc, int32_t no_slot, int values_per_slot, bool body_lists) {
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
    // (scans over contact ends, bodies and the ids' tables)
    const size_t need_tmp = exclusive_scan_tmp_bytes(std::max<int64_t>(std::max<int64_t>(2 * nc, N), nsub) + 2);
    if (need_tmp > sc->scan_tmp.cap) NBGS_TRY(sc->scan_tmp.reserve(need_tmp));
    // contact ends sorted by body, then stably by subdomain
    const int64_t ne = 2 * nc;
    for (DevBuf<uint32_t> *b : {&sc->ekeys, &sc->evals, &sc->ekeys2, &sc->evals2}) NBGS_TRY(b->reserve((size_t)ne + 1));
    if ((size_t)radix_hist_entries(ne) > sc->radix_hist.cap) NBGS_TRY(sc->radix_hist.reserve(radix_hist_entries(ne)));
    const size_t need_tmp2 = exclusive_scan_tmp_bytes((int64_t)radix_hist_entries(ne));
    if (need_tmp2 > sc->scan_tmp.cap) NBGS_TRY(sc->scan_tmp.reserve(need_tmp2));
    k_ends<<<grid_for(ne), kBlock, 0, s>>>(sj1, sj2, ne, N, sc->b.inv_mass, sc->ekeys.p, sc->evals.p, ssd, no_slot);
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
    // block-local order over several grids: the first grid's slots sub-ordered by cell (k_end_tiles_sub)
    int32_t sb = 0;
    if (!body_lists && sc->blk_grids > 1 && sc->blk_grid_ids > 0) {
        sb = 3 * bits_for(sc->blk_grids);
        if (bits_for(nsub) + sb > 32) sb = 0;
    }
    if (sb > 0) {
        Blocks bl;
        int64_t nblocks = 1;
        NBGS_TRY(make_blocks(sc, sc->blk_edge, bl, nblocks));
        k_end_tiles_sub<<<grid_for(ne), kBlock, 0, s>>>(vals, ne, ssd, sj1, sj2, sc->b, bl, sc->blk_grids,
                                                        sc->blk_grid_ids, no_slot, sb, keys);
    } else {
        k_end_tiles<<<grid_for(ne), kBlock, 0, s>>>(vals, ne, ssd, keys);
    }
    NBGS_HIP(hipGetLastError());
    bool alt2 = false;
    NBGS_TRY(radix_sort_pairs(keys, vals, keys_o, vals_o, ne, std::max(1, bits_for(nsub) + sb), sc->radix_hist.p,
                              sc->scan_tmp.p, sc->scan_tmp.cap, &alt2, s));
    const uint32_t *svals = alt2 ? vals_o : vals;
    // slots
    NBGS_TRY(sc->eflags.reserve((size_t)ne + 1));
    NBGS_TRY(sc->eex.reserve((size_t)ne + 1));
    k_slot_flags<<<grid_for(ne), kBlock, 0, s>>>(svals, ne, sj1, sj2, ssd, N, sc->b.inv_mass, sc->eflags.p, no_slot);
    NBGS_HIP(hipGetLastError());
    NBGS_TRY(exclusive_scan_i32(sc->eflags.p, sc->eex.p, ne, sc->total(), sc->scan_tmp.p, sc->scan_tmp.cap, s));
    NBGS_TRY(scene_sync_small(sc, 0, 1));
    const int64_t nslots = sc->pinned[0];
    sc->n_slots = nslots;
    NBGS_TRY(sc->slot_body.reserve((size_t)nslots + 1));
    NBGS_TRY(sc->slot_sdom.reserve((size_t)nslots + 1));
    k_slot_write<<<grid_for(ne), kBlock, 0, s>>>(svals, ne, sj1, sj2, ssd, N, sc->b.inv_mass, sc->eflags.p, sc->eex.p,
                                                 sc->slot_body.p, sc->slot_sdom.p, no_slot);
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
                                                sc->tile_slot_off.p, sw.ls.p, no_slot);
    NBGS_HIP(hipGetLastError());
    if (nslots == 0 && body_lists) {
        set_error("no dynamic body in any subdomain");
        return NBGS_ERR_STATE;
    }
    if (body_lists) NBGS_TRY(body_slot_lists(sc, nslots));
    // tile sizes against the kernel's limits
    std::vector<int32_t> cnt((size_t)nsub), scnt((size_t)nsub);
    NBGS_HIP(hipMemcpyAsync(cnt.data(), sc->tile_cnt.p, sizeof(int32_t) * nsub, hipMemcpyDeviceToHost, s));
    NBGS_HIP(hipMemcpyAsync(scnt.data(), sc->tile_scnt.p, sizeof(int32_t) * nsub, hipMemcpyDeviceToHost, s));
    NBGS_HIP(hipStreamSynchronize(s));
    int32_t max_slots = 0;
    for (int32_t t = 0; t < nsub; ++t) max_slots = std::max(max_slots, scnt[(size_t)t]);
    const size_t lds = (size_t)max_slots * values_per_slot * sizeof(T);
    if (lds > 60 * 1024) {
        set_error("a %s touches %d bodies (%zu bytes of LDS); use a smaller %s edge", body_lists ? "subdomain" : "block",
                  max_slots, lds, body_lists ? "subdomain" : "block");
        return NBGS_ERR_CAPACITY;
    }
    sc->max_slots = max_slots;
    // the block-local order launches one grid at a time: each launch takes the local memory of its largest block
    // (the later grids' blocks hold only the contacts the earlier grids cut, so they need less and more of them
    // share a compute unit)
    sc->launch_id0.clear();
    sc->launch_n.clear();
    sc->launch_slots.clear();
    if (!body_lists && sc->blk_grid_ids > 0) {
        auto group = [&](int32_t id0, int32_t n) {
            int32_t m = 0;
            for (int32_t t = id0; t < id0 + n; ++t) m = std::max(m, scnt[(size_t)t]);
            sc->launch_id0.push_back(id0);
            sc->launch_n.push_back(n);
            sc->launch_slots.push_back(m);
        };
        for (int32_t id0 = 0; id0 < sc->n_blk; id0 += sc->blk_grid_ids)
            group(id0, std::min(sc->blk_grid_ids, sc->n_blk - id0));
        if (sc->blk_groups > 0) group(sc->n_blk, sc->blk_groups);  // the clusters no grid holds
        int64_t s0 = 0;
        for (int32_t t = 0; t < std::min(sc->blk_grid_ids, sc->n_blk); ++t) s0 += scnt[(size_t)t];
        sc->slot_s0 = s0;
    }
    // 64-bit contact offsets of the tiles
    std::vector<int64_t> toff((size_t)nsub + 1, 0);
    for (int32_t t = 0; t < nsub; ++t) toff[(size_t)t + 1] = toff[(size_t)t] + cnt[(size_t)t];
    NBGS_HIP(hipMemcpyAsync(sc->tile_off.p, toff.data(), sizeof(int64_t) * (nsub + 1), hipMemcpyHostToDevice, s));
    NBGS_HIP(hipStreamSynchronize(s));  // toff is a host temporary
    sc->blk_first_cross = toff[(size_t)nsub - 1];
    return NBGS_OK;
}

// Per body its slots in ascending subdomain (slots are numbered in (subdomain,
// body) order), for the subdomain solver's correction reduction.
static nbgs_status body_slot_lists(nbgs_scene_t sc, int64_t nslots) {
    hipStream_t s = sc->s;
    const int32_t N = sc->b.n;
    auto bits_for = [](int64_t n) {
        int b = 0;
        while (((int64_t)1 << b) < n) ++b;
        return b;
    };
    for (DevBuf<uint32_t> *b : {&sc->bkeys, &sc->bvals, &sc->bkeys2, &sc->bvals2})
        NBGS_TRY(b->reserve((size_t)nslots + 1));
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
    return NBGS_OK;
}

nbgs_status subdomain_prepare(nbgs_scene_t sc) {
    if (sc->precision_used == NBGS_FP32_SWEEP) return prepare_impl<float>(sc);
    return prepare_impl<double>(sc);
}

nbgs_status block_prepare(nbgs_scene_t sc) {
    sc->rec_valid = false;  // new slot tables
    if (sc->blk_grids > 1) {
        if (sc->precision_used == NBGS_FP32_SWEEP) return block_grids_prepare_impl<float>(sc);
        return block_grids_prepare_impl<double>(sc);
    }
    if (sc->precision_used == NBGS_FP32_SWEEP) return block_prepare_impl<float>(sc);
    return block_prepare_impl<double>(sc);
}

template <class T>
nbgs_status block_pass(nbgs_scene_t sc, int mode, T *vel) {
    if (sc->n_blk <= 0) return NBGS_OK;
    hipStream_t s = sc->s;
    SweepBuf<T> &sw = sc->precision_used == NBGS_FP32_SWEEP ? *reinterpret_cast<SweepBuf<T> *>(&sc->sw32)
                                                            : *reinterpret_cast<SweepBuf<T> *>(&sc->sw64);
    SubView<T> v;
    // with the records in the first grid's slot order (rec_on) the ends and slots are record indices
    v.j1 = sc->rec_on ? sc->j1r.p : sw.j1.p;
    v.j2 = sc->rec_on ? sc->j2r.p : sw.j2.p;
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
    const T mu = (T)sc->p.mu, relax = (T)sc->p.relax;
    // one grid: every dynamic body of a block, sorted by block; several: the bodies the local contacts touch
    const int32_t *slot_body = sc->rec_on ? sc->slot_rec.p
                               : sc->blk_grids > 1 ? sc->slot_body.p
                                                   : reinterpret_cast<const int32_t *>(sc->body_slots);
    // one launch per grid (a grid's blocks share no dynamic body, the next grid sees their results), then the
    // groups of the clusters no grid holds
    for (size_t li = 0; li < sc->launch_id0.size(); ++li) {
        const int32_t id0 = sc->launch_id0[li];
        const unsigned grid = (unsigned)sc->launch_n[li];
        if (grid == 0) continue;
        const size_t lds = (size_t)std::max(sc->launch_slots[li], 1) * 8 * sizeof(T);
        // FP64 records: the held form; FP32 records: the streamed form (the faster of the two for each)
        if constexpr (sizeof(T) == 8) {
            if (mode == 0)
                k_blk_pass<T, 0><<<grid, kBlkThreads, lds, s>>>(v, sc->b.n, vel, mu, relax, sc->tile_off.p,
                                                                 sc->tile_slot_off.p, slot_body, sc->blk_cs.p,
                                                                 sc->blk_nrun.p, sc->partials.p, sc->ctrl(), id0);
            else
                k_blk_pass<T, 1><<<grid, kBlkThreads, lds, s>>>(v, sc->b.n, vel, mu, relax, sc->tile_off.p,
                                                                 sc->tile_slot_off.p, slot_body, sc->blk_cs.p,
                                                                 sc->blk_nrun.p, sc->partials.p, sc->ctrl(), id0);
        } else {
            if (mode == 0)
                k_blk_pass_stream<T, 0><<<grid, kBlkStreamThreads, lds, s>>>(
                    v, sc->b.n, vel, mu, relax, sc->tile_off.p, sc->tile_slot_off.p, slot_body, sc->blk_cs.p,
                    sc->blk_nrun.p, sc->partials.p, sc->ctrl(), id0);
            else
                k_blk_pass_stream<T, 1><<<grid, kBlkStreamThreads, lds, s>>>(
                    v, sc->b.n, vel, mu, relax, sc->tile_off.p, sc->tile_slot_off.p, slot_body, sc->blk_cs.p,
                    sc->blk_nrun.p, sc->partials.p, sc->ctrl(), id0);
        }
        NBGS_HIP(hipGetLastError());
    }
    return NBGS_OK;
}

template nbgs_status block_pass<double>(nbgs_scene_t, int, double *);
template nbgs_status block_pass<float>(nbgs_scene_t, int, float *);

nbgs_status block_records(nbgs_scene_t sc) {
    sc->rec_on = false;
    // few contacts keep records for the touched bodies only: nothing to gain from a copy of every record
    if (!sc->blk_active || sc->sparse_bodies || sc->nc <= 0 || sc->n_blk <= 0) return NBGS_OK;
    if (sc->rec_valid) {
        sc->rec_on = true;
        return NBGS_OK;
    }
    hipStream_t s = sc->s;
    const int32_t N = sc->b.n;
    const int64_t nc = sc->nc;
    const bool multi = sc->blk_grids > 1;
    const int32_t *slots = multi ? sc->slot_body.p : reinterpret_cast<const int32_t *>(sc->body_slots);
    const int64_t nslots = multi ? sc->n_slots : (int64_t)N;  // one grid: every body, in block order
    const int64_t s0 = std::min<int64_t>(multi ? sc->slot_s0 : (int64_t)N, nslots);
    const int32_t *j1 = sc->precision_used == NBGS_FP32_SWEEP ? sc->sw32.j1.p : sc->sw64.j1.p;
    const int32_t *j2 = sc->precision_used == NBGS_FP32_SWEEP ? sc->sw32.j2.p : sc->sw64.j2.p;
    // the tables are part of the block-local order's workspace bound; without room the records stay in body order
    const size_t need_tmp = exclusive_scan_tmp_bytes((int64_t)N + 1);
    if (sc->rec_of.reserve((size_t)N + 1, 1.0) != NBGS_OK || sc->body_of.reserve((size_t)N + 1, 1.0) != NBGS_OK ||
        sc->rec_tmp.reserve((size_t)N + 1, 1.0) != NBGS_OK ||
        sc->slot_rec.reserve((size_t)(nslots > 0 ? nslots : 1)) != NBGS_OK ||
        sc->j1r.reserve((size_t)nc) != NBGS_OK || sc->j2r.reserve((size_t)nc) != NBGS_OK ||
        (need_tmp > sc->scan_tmp.cap && sc->scan_tmp.reserve(need_tmp) != NBGS_OK))
        return NBGS_OK;
    k_fill<<<grid_for(N), kBlock, 0, s>>>(sc->rec_of.p, N, -1);
    if (s0 > 0) k_rec_first<<<grid_for(s0), kBlock, 0, s>>>(slots, s0, sc->rec_of.p);
    k_rec_flags<<<grid_for(N), kBlock, 0, s>>>(sc->rec_of.p, N, sc->body_of.p);
    NBGS_HIP(hipGetLastError());
    NBGS_TRY(exclusive_scan_i32(sc->body_of.p, sc->rec_tmp.p, N, nullptr, sc->scan_tmp.p, sc->scan_tmp.cap, s));
    k_rec_rest<<<grid_for(N), kBlock, 0, s>>>(sc->rec_tmp.p, N, (int32_t)s0, sc->rec_of.p, sc->body_of.p);
    if (nslots > 0) k_slot_rec<<<grid_for(nslots), kBlock, 0, s>>>(slots, nslots, sc->rec_of.p, sc->slot_rec.p);
    k_ends_rec<<<grid_for(nc), kBlock, 0, s>>>(j1, j2, nc, N, sc->rec_of.p, sc->j1r.p, sc->j2r.p);
    NBGS_HIP(hipGetLastError());
    sc->rec_valid = true;
    sc->rec_on = true;
    return NBGS_OK;
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
