// Colouring of the contact conflict graph and the colour-major sweep order.
//
// On one GPU the subdomain affinity s_c(j) of Alg. 1 is replaced by a colour:
// no two contacts of a colour share a dynamic body, so every colour is one
// data-parallel stage of a Gauss-Seidel sweep whose result does not depend on
// the order inside the colour.
//
// Jones-Plassmann rounds with fixed priorities pi_j = splitmix64(key_j ^ seed)
// (ties: smaller key first): an uncoloured contact whose uncoloured conflicting
// contacts all have lower priority takes the smallest colour not used by its
// coloured conflicting contacts.  Every contact is thus coloured after all of
// its higher-priority neighbours and before its lower-priority ones, which is
// exactly the sequential greedy colouring in priority order.  A neighbour seen
// as uncoloured because its colour is not visible yet only delays a contact by
// a round; it never changes the colour chosen.
//
// Between time steps the contact graph changes little, so a step starts from
// the previous step's colours (matched by pair key) and repeats the greedy
// rule  colour(j) = smallest colour not held by a higher-priority neighbour
// over all contacts until a pass changes nothing.  The rule's fixed point is
// unique -- by induction over the longest chain of decreasing priority ending
// at j, after pass r every contact whose chain is at most r long holds its
// greedy colour and keeps it -- so the result is again the greedy colouring;
// only the number of passes depends on the start.
#include "nbgs_internal.h"

namespace nbgs {

namespace {

constexpr int kBlock = 256;
constexpr int kMaxColours = 256;

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// splitmix64 (Steele, Lea, Flood 2014): add the golden-ratio increment, then
// the published xor-shift-multiply finaliser.
__device__ inline uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__global__ void __launch_bounds__(kBlock) k_j2_degree(const int32_t *j2, int64_t nc, int32_t nb,
                                                      const double *inv_mass, int32_t *deg2) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nc) return;
    const int k = j2[j];
    if (k < nb && inv_mass[k] > 0.0) atomicAdd(&deg2[k], 1);
}

__global__ void __launch_bounds__(kBlock) k_j2_fill(const int32_t *j2, int64_t nc, int32_t nb,
                                                    const double *inv_mass, int32_t *cursor, int32_t *inc2) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nc) return;
    const int k = j2[j];
    if (k < nb && inv_mass[k] > 0.0) inc2[atomicAdd(&cursor[k], 1)] = (int32_t)j;
}

struct Probe {
    uint64_t key, prio;
    uint64_t used[kMaxColours / 64];
    bool blocked;
};

// l precedes j in the greedy order (higher priority, ties: smaller key)
__device__ inline bool precedes(uint64_t pl, uint64_t kl, uint64_t pj, uint64_t kj) {
    return pl > pj || (pl == pj && kl < kj);
}

__device__ inline void probe(Probe &pr, const ContactsView &c, const uint64_t *prio, int64_t l) {
    const int cl = __hip_atomic_load(&c.colour[l], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (cl >= 0) {
        pr.used[cl >> 6] |= 1ull << (cl & 63);
        return;
    }
    if (precedes(prio[l], c.key[l], pr.prio, pr.key)) pr.blocked = true;
}

// Priority from the pair key in the numbering of the contact's own scene
// (body i -> i - body_off[s], wall w of the scene -> n_s + w) and the scene's
// seed: a batched scene gets the priorities it would have alone.
__global__ void __launch_bounds__(kBlock) k_prio(const uint64_t *key, int64_t nc, uint64_t seed, SceneTable st,
                                                 int32_t nb, uint64_t *prio) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nc) return;
    uint64_t k = key[j];
    uint64_t sd = seed;
    if (st.body_scene) {
        const uint32_t i1 = (uint32_t)(k >> 32), i2 = (uint32_t)k;
        const int sc = st.body_scene[i1];
        const uint32_t b0 = (uint32_t)st.body_off[sc], ns = (uint32_t)st.body_off[sc + 1] - b0;
        const uint32_t l2 = i2 < (uint32_t)nb ? i2 - b0 : ns + (i2 - (uint32_t)nb - (uint32_t)st.wall_off[sc]);
        k = ((uint64_t)(i1 - b0) << 32) | (uint64_t)l2;
        sd = st.seed[sc];
    }
    prio[j] = splitmix64(k ^ sd);
}

// sdom (may be null): subdomain of every contact; contacts of different
// subdomains do not conflict.
__global__ void __launch_bounds__(kBlock) k_jp_round(ContactsView c, const uint64_t *prio, int64_t nc, int32_t nb,
                                                     const double *inv_mass, const int32_t *off1,
                                                     const int32_t *cnt1, const int32_t *off2, const int32_t *inc2,
                                                     const int32_t *sdom, int32_t *remaining, int32_t *overflow) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nc || c.colour[j] >= 0) return;
    const int32_t sj = sdom ? sdom[j] : 0;
    Probe pr;
    pr.key = c.key[j];
    pr.prio = prio[j];
    pr.blocked = false;
#pragma unroll
    for (int w = 0; w < kMaxColours / 64; ++w) pr.used[w] = 0;
    const int ends[2] = {c.j1[j], c.j2[j]};
    for (int e = 0; e < 2 && !pr.blocked; ++e) {
        const int b = ends[e];
        if (b >= nb || !(inv_mass[b] > 0.0)) continue;
        const int a0 = off1[b], a1 = a0 + cnt1[b];
        for (int l = a0; l < a1 && !pr.blocked; ++l)
            if (l != j && (!sdom || sdom[l] == sj)) probe(pr, c, prio, l);
        const int q1 = off2[b + 1];
        for (int q = off2[b]; q < q1 && !pr.blocked; ++q) {
            const int l = inc2[q];
            if (l != j && (!sdom || sdom[l] == sj)) probe(pr, c, prio, l);
        }
    }
    if (pr.blocked) return;
    int col = -1;
#pragma unroll
    for (int w = 0; w < kMaxColours / 64; ++w) {
        if (col < 0 && pr.used[w] != ~0ull) col = 64 * w + __ffsll((long long)~pr.used[w]) - 1;
    }
    if (col < 0) {
        atomicExch(overflow, 1);
        col = kMaxColours - 1;
    }
    __hip_atomic_store(&c.colour[j], col, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    atomicSub(remaining, 1);
}

// hist[c]: contacts of colour c; hist[256 + c]: dynamic bodies they touch
// (the body records a sweep launch of colour c reads and writes).
// One pass of colour(j) <- smallest colour not held by a higher-priority
// neighbour; *changed counts the contacts whose colour moved.  With dirty_in
// given, only the contacts it marks are evaluated: a contact's rule reads only
// its higher-priority neighbours, so it can change only after one of them
// did, and every contact that changes marks its lower-priority neighbours in
// dirty_out (also those it had already been read by in this pass).  The
// passes then touch the few contacts a change still reaches, and end at the
// same fixed point.
__global__ void __launch_bounds__(kBlock) k_colour_fix(ContactsView c, const uint64_t *prio, int64_t nc, int32_t nb,
                                                       const double *inv_mass, const int32_t *off1,
                                                       const int32_t *cnt1, const int32_t *off2,
                                                       const int32_t *inc2, const int32_t *sdom,
                                                       uint8_t *dirty_in, uint8_t *dirty_out, int32_t *changed,
                                                       int32_t *overflow) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nc || (dirty_in && !dirty_in[j])) return;
    if (dirty_in) dirty_in[j] = 0;  // left clear for the pass after next, which writes its marks there
    const int32_t sj = sdom ? sdom[j] : 0;
    const uint64_t kj = c.key[j], pj = prio[j];
    uint64_t used[kMaxColours / 64] = {0, 0, 0, 0};
    const int ends[2] = {c.j1[j], c.j2[j]};
    for (int e = 0; e < 2; ++e) {
        const int b = ends[e];
        if (b >= nb || !(inv_mass[b] > 0.0)) continue;
        const int a0 = off1[b], a1 = a0 + cnt1[b];
        for (int l = a0; l < a1; ++l) {
            if (l == j || (sdom && sdom[l] != sj) || !precedes(prio[l], c.key[l], pj, kj)) continue;
            const int cl = __hip_atomic_load(&c.colour[l], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            used[(cl >> 6) & 3] |= 1ull << (cl & 63);
        }
        const int q1 = off2[b + 1];
        for (int q = off2[b]; q < q1; ++q) {
            const int l = inc2[q];
            if (l == j || (sdom && sdom[l] != sj) || !precedes(prio[l], c.key[l], pj, kj)) continue;
            const int cl = __hip_atomic_load(&c.colour[l], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            used[(cl >> 6) & 3] |= 1ull << (cl & 63);
        }
    }
    int col = -1;
#pragma unroll
    for (int w = 0; w < kMaxColours / 64; ++w) {
        if (col < 0 && used[w] != ~0ull) col = 64 * w + __ffsll((long long)~used[w]) - 1;
    }
    if (col < 0) {
        atomicExch(overflow, 1);
        col = kMaxColours - 1;
    }
    if (col != c.colour[j]) {
        __hip_atomic_store(&c.colour[j], col, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        atomicAdd(changed, 1);
        if (dirty_out) {  // the lower-priority neighbours read this colour
            for (int e = 0; e < 2; ++e) {
                const int b = ends[e];
                if (b >= nb || !(inv_mass[b] > 0.0)) continue;
                const int a0 = off1[b], a1 = a0 + cnt1[b];
                for (int l = a0; l < a1; ++l)
                    if (l != j && (!sdom || sdom[l] == sj) && precedes(pj, kj, prio[l], c.key[l])) dirty_out[l] = 1;
                const int q1 = off2[b + 1];
                for (int q = off2[b]; q < q1; ++q) {
                    const int l = inc2[q];
                    if (l != j && (!sdom || sdom[l] == sj) && precedes(pj, kj, prio[l], c.key[l])) dirty_out[l] = 1;
                }
            }
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_fill_u8(uint8_t *p, int64_t n, uint8_t v) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void __launch_bounds__(kBlock) k_colour_hist(ContactsView c, int64_t nc, int32_t nb,
                                                        const double *inv_mass, int32_t *hist) {
    __shared__ int cnt[2 * kMaxColours];
    for (int d = threadIdx.x; d < 2 * kMaxColours; d += kBlock) cnt[d] = 0;
    __syncthreads();
    // a bounded grid walks the contacts, so that few workgroups meet at the global counters
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < nc; j += (int64_t)gridDim.x * kBlock) {
        const int col = c.colour[j] & (kMaxColours - 1);
        atomicAdd(&cnt[col], 1);
        const int b1 = c.j1[j], b2 = c.j2[j];
        const int dyn = (inv_mass[b1] > 0.0 ? 1 : 0) + (b2 < nb && inv_mass[b2] > 0.0 ? 1 : 0);
        atomicAdd(&cnt[kMaxColours + col], dyn);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < 2 * kMaxColours; d += kBlock)
        if (cnt[d]) atomicAdd(&hist[d], cnt[d]);
}

// Sort key of the sweep order: colour, or (subdomain, colour) with sdom.
__global__ void __launch_bounds__(kBlock) k_colour_keys(const int32_t *colour, const int32_t *sdom, int64_t nc,
                                                        uint32_t *keys, uint32_t *ids) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nc) return;
    keys[j] = sdom ? ((uint32_t)sdom[j] << 8) | (uint32_t)colour[j] : (uint32_t)colour[j];
    ids[j] = (uint32_t)j;
}

// Sweep position of every canonical contact (inverse of the colour sort's permutation).
__global__ void __launch_bounds__(kBlock) k_invert(const uint32_t *perm, int64_t nc, int32_t *pos) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p < nc) pos[perm[p]] = (int32_t)p;
}

// Sweep position p <- canonical record perm[p].  One thread per sweep
// position: the writes stream, and the reads of neighbouring positions (one
// colour of one region of the box) fall on a few canonical segments.
// indices = 0: the record's ends, order, colours, ids and friction
// coefficients are those of the last gather (same pairs in the same order);
// only geometry and impulses are written.
template <class T>
__global__ void __launch_bounds__(kBlock) k_gather_sweep(ContactsView c, const uint32_t *perm, const int32_t *sdom,
                                                         int64_t nc, double dt, double erp, SceneTable st,
                                                         SweepView<T> sv, int indices) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= nc) return;
    const int64_t j = perm[p];
    if (indices) {
        sv.perm[p] = (int32_t)j;
        if (sv.col) sv.col[p] = c.colour[j];
        if (sv.sdom) sv.sdom[p] = sdom[j];
        if (sv.mu) sv.mu[p] = (T)st.mu[st.body_scene[c.j1[j]]];
        sv.j1[p] = c.j1[j];
        sv.j2[p] = c.j2[j];
    }
    sv.nx[p] = (T)c.nx[j];
    sv.ny[p] = (T)c.ny[j];
    sv.nz[p] = (T)c.nz[j];
    const double xi = c.xi[j];
    const double corr = xi < 0.0 ? erp * xi : xi;  // scaled-down penetration correction (Sect. 3)
    sv.bias[p] = (T)(corr / dt);
    sv.a1[p] = (T)c.a1[j];
    sv.a2[p] = (T)c.a2[j];
    sv.px[p] = (T)c.px[j];
    sv.py[p] = (T)c.py[j];
    sv.pz[p] = (T)c.pz[j];
}

}  // namespace

nbgs_status launch_j2_degree(const ContactsView &c, int64_t nc, int32_t nb, const double *inv_mass, int32_t *deg2,
                             hipStream_t s) {
    NBGS_HIP(hipMemsetAsync(deg2, 0, sizeof(int32_t) * ((size_t)nb + 1), s));
    if (nc == 0) return NBGS_OK;
    k_j2_degree<<<grid_for(nc), kBlock, 0, s>>>(c.j2, nc, nb, inv_mass, deg2);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

nbgs_status launch_j2_fill(const ContactsView &c, int64_t nc, int32_t nb, const double *inv_mass, int32_t *cursor,
                           int32_t *inc2, hipStream_t s) {
    if (nc == 0) return NBGS_OK;
    k_j2_fill<<<grid_for(nc), kBlock, 0, s>>>(c.j2, nc, nb, inv_mass, cursor, inc2);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

nbgs_status launch_prio(const ContactsView &c, int64_t nc, uint64_t seed, const SceneTable &st, int32_t nb,
                        uint64_t *prio, hipStream_t s) {
    if (nc == 0) return NBGS_OK;
    k_prio<<<grid_for(nc), kBlock, 0, s>>>(c.key, nc, seed, st, nb, prio);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

nbgs_status launch_jp_round(const ContactsView &c, const uint64_t *prio, int64_t nc, int32_t nb,
                            const double *inv_mass, const int32_t *off1, const int32_t *cnt1, const int32_t *off2,
                            const int32_t *inc2, const int32_t *sdom, int32_t *remaining, int32_t *overflow,
                            hipStream_t s) {
    if (nc == 0) return NBGS_OK;
    k_jp_round<<<grid_for(nc), kBlock, 0, s>>>(c, prio, nc, nb, inv_mass, off1, cnt1, off2, inc2, sdom, remaining,
                                               overflow);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

nbgs_status launch_fill_u8(uint8_t *p, int64_t n, uint8_t v, hipStream_t s) {
    if (n <= 0) return NBGS_OK;
    k_fill_u8<<<grid_for(n), kBlock, 0, s>>>(p, n, v);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

nbgs_status launch_colour_fix(const ContactsView &c, const uint64_t *prio, int64_t nc, int32_t nb,
                              const double *inv_mass, const int32_t *off1, const int32_t *cnt1, const int32_t *off2,
                              const int32_t *inc2, const int32_t *sdom, uint8_t *dirty_in, uint8_t *dirty_out,
                              int32_t *changed, int32_t *overflow, bool clear_out, hipStream_t s) {
    if (nc == 0) return NBGS_OK;
    if (dirty_out && clear_out) {
        NBGS_TRY(launch_fill_u8(dirty_out, nc, 0, s));
    }
    k_colour_fix<<<grid_for(nc), kBlock, 0, s>>>(c, prio, nc, nb, inv_mass, off1, cnt1, off2, inc2, sdom, dirty_in,
                                                 dirty_out, changed, overflow);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

nbgs_status launch_colour_hist(const ContactsView &c, int64_t nc, int32_t nb, const double *inv_mass, int32_t *hist,
                               hipStream_t s) {
    NBGS_HIP(hipMemsetAsync(hist, 0, sizeof(int32_t) * 2 * kMaxColours, s));
    if (nc == 0) return NBGS_OK;
    const unsigned g = grid_for(nc);
    k_colour_hist<<<g < 1024u ? g : 1024u, kBlock, 0, s>>>(c, nc, nb, inv_mass, hist);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

nbgs_status launch_colour_keys(const ContactsView &c, const int32_t *sdom, int64_t nc, uint32_t *keys, uint32_t *ids,
                               hipStream_t s) {
    if (nc == 0) return NBGS_OK;
    k_colour_keys<<<grid_for(nc), kBlock, 0, s>>>(c.colour, sdom, nc, keys, ids);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

nbgs_status launch_invert(const uint32_t *perm, int64_t nc, int32_t *pos, hipStream_t s) {
    if (nc == 0) return NBGS_OK;
    k_invert<<<grid_for(nc), kBlock, 0, s>>>(perm, nc, pos);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

template <class T>
nbgs_status launch_gather_sweep(const ContactsView &c, const uint32_t *perm, const int32_t *sdom, int64_t nc,
                                double dt, double erp, const SceneTable &st, SweepView<T> sv, bool indices,
                                hipStream_t s) {
    if (nc == 0) return NBGS_OK;
    k_gather_sweep<T><<<grid_for(nc), kBlock, 0, s>>>(c, perm, sdom, nc, dt, erp, st, sv, indices ? 1 : 0);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

template nbgs_status launch_gather_sweep<double>(const ContactsView &, const uint32_t *, const int32_t *, int64_t,
                                                 double, double, const SceneTable &, SweepView<double>, bool,
                                                 hipStream_t);
template nbgs_status launch_gather_sweep<float>(const ContactsView &, const uint32_t *, const int32_t *, int64_t,
                                                double, double, const SceneTable &, SweepView<float>, bool,
                                                hipStream_t);

}  // namespace nbgs
