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

__device__ inline void probe(Probe &pr, const ContactsView &c, int64_t l, uint64_t seed) {
    const int cl = __hip_atomic_load(&c.colour[l], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (cl >= 0) {
        pr.used[cl >> 6] |= 1ull << (cl & 63);
        return;
    }
    const uint64_t kl = c.key[l];
    const uint64_t pl = splitmix64(kl ^ seed);
    if (pl > pr.prio || (pl == pr.prio && kl < pr.key)) pr.blocked = true;
}

__global__ void __launch_bounds__(kBlock) k_jp_round(ContactsView c, int64_t nc, int32_t nb,
                                                     const double *inv_mass, const int32_t *off1,
                                                     const int32_t *cnt1, const int32_t *off2, const int32_t *inc2,
                                                     uint64_t seed, int32_t *remaining, int32_t *overflow) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nc || c.colour[j] >= 0) return;
    Probe pr;
    pr.key = c.key[j];
    pr.prio = splitmix64(pr.key ^ seed);
    pr.blocked = false;
#pragma unroll
    for (int w = 0; w < kMaxColours / 64; ++w) pr.used[w] = 0;
    const int ends[2] = {c.j1[j], c.j2[j]};
    for (int e = 0; e < 2 && !pr.blocked; ++e) {
        const int b = ends[e];
        if (b >= nb || !(inv_mass[b] > 0.0)) continue;
        const int a0 = off1[b], a1 = a0 + cnt1[b];
        for (int l = a0; l < a1 && !pr.blocked; ++l)
            if (l != j) probe(pr, c, l, seed);
        const int q1 = off2[b + 1];
        for (int q = off2[b]; q < q1 && !pr.blocked; ++q) {
            const int l = inc2[q];
            if (l != j) probe(pr, c, l, seed);
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

__global__ void __launch_bounds__(kBlock) k_colour_hist(const int32_t *colour, int64_t nc, int32_t *hist) {
    __shared__ int cnt[kMaxColours];
    for (int d = threadIdx.x; d < kMaxColours; d += kBlock) cnt[d] = 0;
    __syncthreads();
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j < nc) atomicAdd(&cnt[colour[j] & (kMaxColours - 1)], 1);
    __syncthreads();
    for (int d = threadIdx.x; d < kMaxColours; d += kBlock)
        if (cnt[d]) atomicAdd(&hist[d], cnt[d]);
}

__global__ void __launch_bounds__(kBlock) k_colour_keys(const int32_t *colour, int64_t nc, uint32_t *keys,
                                                        uint32_t *ids) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nc) return;
    keys[j] = (uint32_t)colour[j];
    ids[j] = (uint32_t)j;
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_gather_sweep(ContactsView c, const uint32_t *perm, int64_t nc, double dt,
                                                         double erp, SweepView<T> sv) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= nc) return;
    const int64_t j = perm[p];
    sv.perm[p] = (int32_t)j;
    sv.j1[p] = c.j1[j];
    sv.j2[p] = c.j2[j];
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

nbgs_status launch_jp_round(const ContactsView &c, int64_t nc, int32_t nb, const double *inv_mass,
                            const int32_t *off1, const int32_t *cnt1, const int32_t *off2, const int32_t *inc2,
                            uint64_t seed, int32_t *remaining, int32_t *overflow, hipStream_t s) {
    if (nc == 0) return NBGS_OK;
    k_jp_round<<<grid_for(nc), kBlock, 0, s>>>(c, nc, nb, inv_mass, off1, cnt1, off2, inc2, seed, remaining,
                                               overflow);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

nbgs_status launch_colour_hist(const ContactsView &c, int64_t nc, int32_t *hist, hipStream_t s) {
    NBGS_HIP(hipMemsetAsync(hist, 0, sizeof(int32_t) * kMaxColours, s));
    if (nc == 0) return NBGS_OK;
    k_colour_hist<<<grid_for(nc), kBlock, 0, s>>>(c.colour, nc, hist);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

nbgs_status launch_colour_keys(const ContactsView &c, int64_t nc, uint32_t *keys, uint32_t *ids, hipStream_t s) {
    if (nc == 0) return NBGS_OK;
    k_colour_keys<<<grid_for(nc), kBlock, 0, s>>>(c.colour, nc, keys, ids);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

template <class T>
nbgs_status launch_gather_sweep(const ContactsView &c, const uint32_t *perm, int64_t nc, double dt, double erp,
                                SweepView<T> sv, hipStream_t s) {
    if (nc == 0) return NBGS_OK;
    k_gather_sweep<T><<<grid_for(nc), kBlock, 0, s>>>(c, perm, nc, dt, erp, sv);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

template nbgs_status launch_gather_sweep<double>(const ContactsView &, const uint32_t *, int64_t, double, double,
                                                 SweepView<double>, hipStream_t);
template nbgs_status launch_gather_sweep<float>(const ContactsView &, const uint32_t *, int64_t, double, double,
                                                SweepView<float>, hipStream_t);

}  // namespace nbgs
