// Nonlinear block Gauss-Seidel sweeps, accumulator init and integration.
//
// Velocity accumulators (Sect. 6.3, velocity form): each body holds v', w' of
// the current iterate in one 8-element record {v'x, v'y, v'z, w'x, w'y, w'z,
// 1/m, 1/I} -- 64 B in FP64, 32 B in FP32 -- so a contact gathers a body with
// one aligned 64 B (or 32 B) access.  Contacts are stored colour-major as a
// structure of arrays; one thread relaxes one contact.  Within a colour no
// two contacts share a dynamic body, so the read-modify-write of the two body
// records needs no atomics, and the per-body update order across colours is
// the colour order: the sweep is the sequential Gauss-Seidel in (colour, key)
// order, bit for bit.  The relaxation of one contact is relax_contact
// (contact_math.h), shared with the block-local pass.
#include <algorithm>

#include "contact_math.h"
#include "nbgs_internal.h"

namespace nbgs {

namespace {

constexpr int kBlock = kSweepBlock;

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

__device__ inline Rec<double> load_rec(const double *vel, int b) {
    const double2 *p = reinterpret_cast<const double2 *>(vel + 8 * (int64_t)b);
    const double2 a = p[0], c = p[1], d = p[2], e = p[3];
    Rec<double> r;
    r.v[0] = a.x;
    r.v[1] = a.y;
    r.v[2] = c.x;
    r.w[0] = c.y;
    r.w[1] = d.x;
    r.w[2] = d.y;
    r.im = e.x;
    r.ii = e.y;
    return r;
}

__device__ inline Rec<float> load_rec(const float *vel, int b) {
    const float4 *p = reinterpret_cast<const float4 *>(vel + 8 * (int64_t)b);
    const float4 a = p[0], c = p[1];
    Rec<float> r;
    r.v[0] = a.x;
    r.v[1] = a.y;
    r.v[2] = a.z;
    r.w[0] = a.w;
    r.w[1] = c.x;
    r.w[2] = c.y;
    r.im = c.z;
    r.ii = c.w;
    return r;
}

// Store v', w'.  With FULL the whole record is written back (the constants
// unchanged), so the write covers the record's aligned 64 B (32 B) instead of
// leaving a partially written memory burst.
template <bool FULL = false>
__device__ inline void store_vel(double *vel, int b, const Rec<double> &r) {
    double2 *p = reinterpret_cast<double2 *>(vel + 8 * (int64_t)b);
    p[0] = make_double2(r.v[0], r.v[1]);
    p[1] = make_double2(r.v[2], r.w[0]);
    p[2] = make_double2(r.w[1], r.w[2]);
    if (FULL) p[3] = make_double2(r.im, r.ii);
}

template <bool FULL = false>
__device__ inline void store_vel(float *vel, int b, const Rec<float> &r) {
    float4 *p = reinterpret_cast<float4 *>(vel + 8 * (int64_t)b);
    p[0] = make_float4(r.v[0], r.v[1], r.v[2], r.w[0]);
    if (FULL) {
        p[1] = make_float4(r.w[1], r.w[2], r.im, r.ii);
    } else {
        float2 *q = reinterpret_cast<float2 *>(vel + 8 * (int64_t)b + 4);
        q[0] = make_float2(r.w[1], r.w[2]);
    }
}

// Row length of the LDS stage of a workgroup's body records (8 rows, one per
// record value): 32 bytes of padding put the 8 rows that a transposed access
// of neighbouring lanes touches in distinct banks.
template <class T>
constexpr int kStageRow = kBlock + 32 / (int)sizeof(T);

// The solver's record of a body that no contact touches: what k_init_bodies
// writes, and what the sweeps leave unchanged.
template <class T>
__device__ inline void free_record(const BodiesView &b, int64_t i, double gx, double gy, double gz, double dt,
                                   T r[8]) {
    const double im = b.inv_mass[i];
    const bool dyn = im > 0.0;
    r[0] = (T)(dyn ? b.vx[i] + dt * gx : b.vx[i]);
    r[1] = (T)(dyn ? b.vy[i] + dt * gy : b.vy[i]);
    r[2] = (T)(dyn ? b.vz[i] + dt * gz : b.vz[i]);
    r[3] = (T)b.wx[i];
    r[4] = (T)b.wy[i];
    r[5] = (T)b.wz[i];
    r[6] = (T)im;
    r[7] = (T)b.inv_inertia[i];
}

// rec (or null: body order): the record of body i is record rec[i] (the block-local sweeps' order).
template <class T>
__global__ void __launch_bounds__(kBlock) k_init_bodies(BodiesView b, double gx, double gy, double gz, double dt,
                                                        T *vel, const int32_t *rec) {
    // the workgroup's records are staged in LDS (value-major) and written as one contiguous run, so that
    // neighbouring lanes store neighbouring words
    constexpr int S = kStageRow<T>;
    __shared__ T stage[8 * S];
    const int i0 = blockIdx.x * kBlock;
    const int t = threadIdx.x, i = i0 + t;
    if (rec) {  // each record whole at its own place
        if (i >= b.n) return;
        T r[8];
        free_record<T>(b, i, gx, gy, gz, dt, r);
        T *out = vel + 8 * (int64_t)rec[i];
#pragma unroll
        for (int a = 0; a < 8; ++a) out[a] = r[a];
        return;
    }
    if (i < b.n) {
        const double im = b.inv_mass[i];
        const bool dyn = im > 0.0;
        stage[0 * S + t] = (T)(dyn ? b.vx[i] + dt * gx : b.vx[i]);
        stage[1 * S + t] = (T)(dyn ? b.vy[i] + dt * gy : b.vy[i]);
        stage[2 * S + t] = (T)(dyn ? b.vz[i] + dt * gz : b.vz[i]);
        stage[3 * S + t] = (T)b.wx[i];
        stage[4 * S + t] = (T)b.wy[i];
        stage[5 * S + t] = (T)b.wz[i];
        stage[6 * S + t] = (T)im;
        stage[7 * S + t] = (T)b.inv_inertia[i];
    }
    __syncthreads();
    const int nvalid = b.n - i0 < kBlock ? b.n - i0 : kBlock;
    T *out = vel + 8 * (int64_t)i0;
    for (int q = t; q < 8 * nvalid; q += kBlock) out[q] = stage[(q & 7) * S + (q >> 3)];
}


// Bodies that some contact of the step touches (either end, walls excepted).
__global__ void __launch_bounds__(kBlock) k_mark_touched(const int32_t *j1, const int32_t *j2, int64_t nc, int32_t nb,
                                                         uint8_t *touched) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= nc) return;
    touched[j1[j]] = 1;
    const int32_t k = j2[j];
    if (k < nb) touched[k] = 1;
}

// k_init_bodies for the touched bodies only (few contacts: the other records are never read).
template <class T>
__global__ void __launch_bounds__(kBlock) k_init_touched(BodiesView b, double gx, double gy, double gz, double dt,
                                                         const uint8_t *touched, T *vel) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < b.n; i += (int64_t)gridDim.x * kBlock) {
        if (!touched[i]) continue;
        T r[8];
        free_record<T>(b, i, gx, gy, gz, dt, r);
        T *out = vel + 8 * i;
#pragma unroll
        for (int a = 0; a < 8; ++a) out[a] = r[a];
    }
}

// Initial impulses applied in colour order (one launch per colour), so every
// body receives them in the same order as in the sweeps.
template <class T>
__global__ void __launch_bounds__(kBlock) k_warm_scatter(SweepView<T> sv, int64_t begin, int64_t end, int32_t nb,
                                                         T *vel) {
    const int64_t p = begin + (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= end) return;
    const T P[3] = {sv.px[p], sv.py[p], sv.pz[p]};
    if (P[0] == T(0) && P[1] == T(0) && P[2] == T(0)) return;
    const int b1 = sv.j1[p], b2 = sv.j2[p];
    const T n[3] = {sv.nx[p], sv.ny[p], sv.nz[p]};
    Rec<T> r1 = load_rec(vel, b1);
    Rec<T> r2 = b2 < nb ? load_rec(vel, b2) : zero_rec<T>();
    apply(r1, r2, n, sv.a1[p], sv.a2[p], P);
    if (r1.im > T(0)) store_vel(vel, b1, r1);
    if (b2 < nb && r2.im > T(0)) store_vel(vel, b2, r2);
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Streamed contact arrays are read once and written once per sweep; with NT
// the accesses carry the non-temporal hint so that they do not evict the body
// records, which every colour of the sweep touches again.
template <bool NT, class V>
__device__ inline V ld(const V *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT, class V>
__device__ inline void st(V *p, V v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Workgroups -> contact tiles.  Without xcd_remap, workgroup b relaxes tiles
// b, b + P, b + 2P, ... (P = gridDim.x).  With xcd_remap the G tiles are cut
// into 8 contiguous ranges, one per XCD (the dispatcher deals consecutive
// workgroups round-robin over the 8 XCDs), and the workgroups of XCD x walk
// range x: neighbouring contacts, and the body records they share, stay in the
// L2 of one XCD.  P == G gives one tile per workgroup; P < G (a persistent
// grid) must then be a multiple of 8 so that every XCD has a workgroup.
struct TileWalk {
    unsigned t, end, step;
};

__device__ inline TileWalk tile_walk(unsigned b, unsigned P, unsigned G, int xcd_remap) {
    if (!xcd_remap) return {b, G, P};
    const unsigned x = b & 7u, i = b >> 3;
    const unsigned q = G >> 3, r = G & 7u;
    const unsigned lo = x * q + (x < r ? x : r);
    const unsigned hi = lo + q + (x < r ? 1u : 0u);
    const unsigned nx = (P >> 3) + ((x < (P & 7u)) ? 1u : 0u);
    return {lo + i, hi, nx};
}

// One tile of one colour: each thread relaxes CPT contacts (strided by the
// block size, all contact loads issued before any arithmetic) and adds
// |dP|^2 and |P|^2 to sd, sp.  Returns true when ctrl[0] != 0, i.e. an earlier
// sweep already met the residual target (the flag is read after the contact
// loads are in flight, so its latency hides behind them; it is the same for
// the whole grid and does not change during a launch).
template <class T, int BLOCK, int CPT, bool NT, bool FULL>
__device__ inline bool sweep_tile_body(const SweepView<T> &sv, int64_t begin, int64_t end, int32_t nb, T *vel, T mu,
                                       T relax, const int32_t *ctrl, unsigned tile, double &sd, double &sp) {
    const int64_t p0 = begin + (int64_t)tile * (BLOCK * CPT) + threadIdx.x;
    int b1[CPT], b2[CPT];
    bool ok[CPT];
    T n[CPT][3], bias[CPT], a1[CPT], a2[CPT], P[CPT][3], muk[CPT];
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        const int64_t p = p0 + (int64_t)k * BLOCK;
        ok[k] = p < end;
        const int64_t q = ok[k] ? p : begin;
        b1[k] = ld<NT>(sv.j1 + q);
        b2[k] = ld<NT>(sv.j2 + q);
        n[k][0] = ld<NT>(sv.nx + q);
        n[k][1] = ld<NT>(sv.ny + q);
        n[k][2] = ld<NT>(sv.nz + q);
        bias[k] = ld<NT>(sv.bias + q);
        a1[k] = ld<NT>(sv.a1 + q);
        a2[k] = ld<NT>(sv.a2 + q);
        P[k][0] = ld<NT>(sv.px + q);
        P[k][1] = ld<NT>(sv.py + q);
        P[k][2] = ld<NT>(sv.pz + q);
        muk[k] = sv.mu ? ld<NT>(sv.mu + q) : mu;
    }
    if (ctrl[0]) return true;
    Rec<T> r1[CPT], r2[CPT];
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        r1[k] = load_rec(vel, b1[k]);
        r2[k] = b2[k] < nb ? load_rec(vel, b2[k]) : zero_rec<T>();
    }
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        if (!ok[k]) continue;
        const T *nk = n[k];
        const T *Pk = P[k];
        T Pnew[3], dP[3];
        relax_contact(nk, bias[k], a1[k], a2[k], Pk, muk[k], relax, r1[k], r2[k], Pnew, dP);
        if (r1[k].im > T(0)) store_vel<FULL>(vel, b1[k], r1[k]);
        if (b2[k] < nb && r2[k].im > T(0)) store_vel<FULL>(vel, b2[k], r2[k]);
        const int64_t p = p0 + (int64_t)k * BLOCK;
        st<NT>(sv.px + p, Pnew[0]);
        st<NT>(sv.py + p, Pnew[1]);
        st<NT>(sv.pz + p, Pnew[2]);
        const double d0 = dP[0], d1 = dP[1], d2 = dP[2];
        const double q0 = Pnew[0], q1 = Pnew[1], q2 = Pnew[2];
        sd += d0 * d0 + d1 * d1 + d2 * d2;
        sp += q0 * q0 + q1 * q1 + q2 * q2;
    }
    return false;
}

// Workgroup sums of sd, sp (waves, then the waves in a fixed order) into out[0], out[1].
template <int BLOCK>
__device__ inline void block_partials(double sd, double sp, double (*red)[BLOCK / 64], double *out) {
    sd = wave_sum(sd);
    sp = wave_sum(sp);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][wave] = sd;
        red[1][wave] = sp;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, c = 0.0;
#pragma unroll
        for (int w = 0; w < BLOCK / 64; ++w) {
            a += red[0][w];
            c += red[1][w];
        }
        out[0] = a;
        out[1] = c;
    }
    __syncthreads();  // red is reused by the workgroup's next tile
}

// One colour of one sweep over G tiles by gridDim.x workgroups; partial sums per tile.
template <class T, int BLOCK, int CPT, bool NT, bool FULL>
__global__ void __launch_bounds__(BLOCK) k_sweep(SweepView<T> sv, int64_t begin, int64_t end, int32_t nb, T *vel,
                                                 T mu, T relax, double *partials, const int32_t *ctrl, unsigned G,
                                                 int xcd_remap) {
    __shared__ double red[2][BLOCK / 64];
    const TileWalk w = tile_walk(blockIdx.x, gridDim.x, G, xcd_remap);
    for (unsigned t = w.t; t < w.end; t += w.step) {
        double sd = 0.0, sp = 0.0;
        if (sweep_tile_body<T, BLOCK, CPT, NT, FULL>(sv, begin, end, nb, vel, mu, relax, ctrl, t, sd, sp)) return;
        block_partials<BLOCK>(sd, sp, red, partials + 2 * t);
    }
}

// Colour c with its range read from col[c], col[c + 1] (so that a captured
// graph serves every step); partial sums per workgroup, zero for a workgroup
// without tiles.
template <class T, int BLOCK, int CPT, bool NT, bool FULL>
__global__ void __launch_bounds__(BLOCK) k_sweep_dev(SweepView<T> sv, const int64_t *col, int c, int32_t nb, T *vel,
                                                     T mu, T relax, double *partials, const int32_t *ctrl,
                                                     int xcd_remap) {
    __shared__ double red[2][BLOCK / 64];
    const int64_t begin = col[c], end = col[c + 1];
    const unsigned G = (unsigned)((end - begin + BLOCK * CPT - 1) / (BLOCK * CPT));
    const TileWalk w = tile_walk(blockIdx.x, gridDim.x, G, xcd_remap);
    double sd = 0.0, sp = 0.0;
    for (unsigned t = w.t; t < w.end; t += w.step)
        if (sweep_tile_body<T, BLOCK, CPT, NT, FULL>(sv, begin, end, nb, vel, mu, relax, ctrl, t, sd, sp)) return;
    block_partials<BLOCK>(sd, sp, red, partials + 2 * blockIdx.x);
}


// Lane groups.  The L lanes of a group relax one contact together (L = 4 in
// FP64, 2 in FP32: the 16 B chunks of a body record).  Lane q loads chunk q of
// both body records, so that one load instruction reads each record as one
// contiguous piece (one memory request per record instead of one per chunk);
// DPP broadcasts inside the group hand every lane the whole records, every
// lane evaluates the contact (the same values by the same operations), lane q
// writes chunk q back (whole records) and lane 0 the impulse and the residual
// sums.
template <class T>
struct Chunks;
template <>
struct Chunks<double> {
    using V = double2;
    static constexpr int L = 4;
};
template <>
struct Chunks<float> {
    using V = float4;
    static constexpr int L = 2;
};

// Lane K of every group of L consecutive lanes, to each lane of that group
// (quad_perm selections: all four lanes of a quad read lane K; for pairs, lanes
// 0, 1 read lane K and lanes 2, 3 read lane 2 + K).
template <int L, int K>
__device__ inline int group_bcast_i32(int x) {
    if constexpr (L == 4) return __builtin_amdgcn_mov_dpp(x, K * 0x55, 0xf, 0xf, true);
    else return __builtin_amdgcn_mov_dpp(x, K == 0 ? 0xa0 : 0xf5, 0xf, 0xf, true);
}
template <int L, int K>
__device__ inline double group_bcast(double x) {
    const long long u = __double_as_longlong(x);
    const unsigned lo = (unsigned)group_bcast_i32<L, K>((int)(unsigned)(u & 0xffffffffll));
    const unsigned hi = (unsigned)group_bcast_i32<L, K>((int)(u >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <int L, int K>
__device__ inline float group_bcast(float x) {
    return __int_as_float(group_bcast_i32<L, K>(__float_as_int(x)));
}

__device__ inline Rec<double> group_rec(const double2 c) {
    Rec<double> r;
    r.v[0] = group_bcast<4, 0>(c.x);
    r.v[1] = group_bcast<4, 0>(c.y);
    r.v[2] = group_bcast<4, 1>(c.x);
    r.w[0] = group_bcast<4, 1>(c.y);
    r.w[1] = group_bcast<4, 2>(c.x);
    r.w[2] = group_bcast<4, 2>(c.y);
    r.im = group_bcast<4, 3>(c.x);
    r.ii = group_bcast<4, 3>(c.y);
    return r;
}

__device__ inline Rec<float> group_rec(const float4 c) {
    Rec<float> r;
    r.v[0] = group_bcast<2, 0>(c.x);
    r.v[1] = group_bcast<2, 0>(c.y);
    r.v[2] = group_bcast<2, 0>(c.z);
    r.w[0] = group_bcast<2, 0>(c.w);
    r.w[1] = group_bcast<2, 1>(c.x);
    r.w[2] = group_bcast<2, 1>(c.y);
    r.im = group_bcast<2, 1>(c.z);
    r.ii = group_bcast<2, 1>(c.w);
    return r;
}

// Chunk q of a record {v'x, v'y, v'z, w'x, w'y, w'z, 1/m, 1/I}.
__device__ inline double2 rec_chunk(const Rec<double> &r, int q) {
    return q == 0 ? make_double2(r.v[0], r.v[1])
                  : q == 1 ? make_double2(r.v[2], r.w[0]) : q == 2 ? make_double2(r.w[1], r.w[2]) : make_double2(r.im, r.ii);
}
__device__ inline float4 rec_chunk(const Rec<float> &r, int q) {
    return q == 0 ? make_float4(r.v[0], r.v[1], r.v[2], r.w[0]) : make_float4(r.w[1], r.w[2], r.im, r.ii);
}

// One tile of BLOCK / L contacts.  A group past the end relaxes the colour's
// first contact on copies and writes nothing; groups never straddle a wave.
template <class T, int BLOCK, bool NT>
__device__ inline bool sweep_group_body(const SweepView<T> &sv, int64_t begin, int64_t end, int32_t nb, T *vel, T mu,
                                        T relax, const int32_t *ctrl, unsigned tile, double &sd, double &sp) {
    using V = typename Chunks<T>::V;
    constexpr int L = Chunks<T>::L;
    const int q = (int)(threadIdx.x & (L - 1));
    const int64_t p = begin + (int64_t)tile * (BLOCK / L) + (int64_t)(threadIdx.x / L);
    const bool ok = p < end;
    const int64_t r = ok ? p : begin;
    const int b1 = ld<NT>(sv.j1 + r), b2 = ld<NT>(sv.j2 + r);
    const T n[3] = {ld<NT>(sv.nx + r), ld<NT>(sv.ny + r), ld<NT>(sv.nz + r)};
    const T bias = ld<NT>(sv.bias + r), a1 = ld<NT>(sv.a1 + r), a2 = ld<NT>(sv.a2 + r);
    const T P[3] = {ld<NT>(sv.px + r), ld<NT>(sv.py + r), ld<NT>(sv.pz + r)};
    const T muk = sv.mu ? ld<NT>(sv.mu + r) : mu;
    if (ctrl[0]) return true;
    const bool sphere2 = b2 < nb;
    const V c1 = reinterpret_cast<const V *>(vel + 8 * (int64_t)b1)[q];
    const V c2 = reinterpret_cast<const V *>(vel + 8 * (int64_t)(sphere2 ? b2 : b1))[q];  // a wall: replaced below
    Rec<T> r1 = group_rec(c1);
    const Rec<T> r2g = group_rec(c2);
    Rec<T> r2 = sphere2 ? r2g : zero_rec<T>();
    T Pnew[3], dP[3];
    relax_contact(n, bias, a1, a2, P, muk, relax, r1, r2, Pnew, dP);
    if (ok) {
        if (r1.im > T(0)) reinterpret_cast<V *>(vel + 8 * (int64_t)b1)[q] = rec_chunk(r1, q);
        if (sphere2 && r2.im > T(0)) reinterpret_cast<V *>(vel + 8 * (int64_t)b2)[q] = rec_chunk(r2, q);
        if (q == 0) {
            st<NT>(sv.px + p, Pnew[0]);
            st<NT>(sv.py + p, Pnew[1]);
            st<NT>(sv.pz + p, Pnew[2]);
            const double d0 = dP[0], d1 = dP[1], d2 = dP[2];
            const double q0 = Pnew[0], q1 = Pnew[1], q2 = Pnew[2];
            sd += d0 * d0 + d1 * d1 + d2 * d2;
            sp += q0 * q0 + q1 * q1 + q2 * q2;
        }
    }
    return false;
}

template <class T, int BLOCK, bool NT>
__global__ void __launch_bounds__(BLOCK) k_sweep_grp(SweepView<T> sv, int64_t begin, int64_t end, int32_t nb, T *vel,
                                                     T mu, T relax, double *partials, const int32_t *ctrl, unsigned G,
                                                     int xcd_remap) {
    __shared__ double red[2][BLOCK / 64];
    const TileWalk w = tile_walk(blockIdx.x, gridDim.x, G, xcd_remap);
    for (unsigned t = w.t; t < w.end; t += w.step) {
        double sd = 0.0, sp = 0.0;
        if (sweep_group_body<T, BLOCK, NT>(sv, begin, end, nb, vel, mu, relax, ctrl, t, sd, sp)) return;
        block_partials<BLOCK>(sd, sp, red, partials + 2 * t);
    }
}

template <class T, int BLOCK, bool NT>
__global__ void __launch_bounds__(BLOCK) k_sweep_grp_dev(SweepView<T> sv, const int64_t *col, int c, int32_t nb,
                                                         T *vel, T mu, T relax, double *partials, const int32_t *ctrl,
                                                         int xcd_remap) {
    __shared__ double red[2][BLOCK / 64];
    constexpr int PER = BLOCK / Chunks<T>::L;
    const int64_t begin = col[c], end = col[c + 1];
    const unsigned G = (unsigned)((end - begin + PER - 1) / PER);
    const TileWalk w = tile_walk(blockIdx.x, gridDim.x, G, xcd_remap);
    double sd = 0.0, sp = 0.0;
    for (unsigned t = w.t; t < w.end; t += w.step)
        if (sweep_group_body<T, BLOCK, NT>(sv, begin, end, nb, vel, mu, relax, ctrl, t, sd, sp)) return;
    block_partials<BLOCK>(sd, sp, red, partials + 2 * blockIdx.x);
}

// R_k = sqrt(sum |dP|^2) / max(sqrt(sum |P|^2), 1e-300), summed in a fixed
// order.  ctrl = {done, sweeps completed, numeric error}.
constexpr int kResBlock = 1024;

// at >= 0: this is sweep `at` (0-based) of the solve, the earlier sweeps were
// not summed; at < 0: the sweep after the last one counted in ctrl[1].
__global__ void __launch_bounds__(kResBlock) k_residual(const double *partials, int32_t n_partials, double target,
                                                        int32_t *ctrl, double *hist, int32_t at) {
    if (ctrl[0]) return;
    double a = 0.0, c = 0.0;
    const double2 *pp = reinterpret_cast<const double2 *>(partials);
    for (int q = threadIdx.x; q < n_partials; q += kResBlock) {
        const double2 v = pp[q];
        a += v.x;
        c += v.y;
    }
    __shared__ double red[2][kResBlock];
    red[0][threadIdx.x] = a;
    red[1][threadIdx.x] = c;
    __syncthreads();
    for (int s = kResBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double den = sqrt(red[1][0]);
        const double R = sqrt(red[0][0]) / (den > 1e-300 ? den : 1e-300);
        const int k = at >= 0 ? at : ctrl[1];
        hist[k] = R;
        ctrl[1] = k + 1;
        if (!(R == R) || R > 1.0e300) {
            ctrl[2] = 1;
            ctrl[0] = 1;
        } else if (target > 0.0 && R <= target) {
            ctrl[0] = 1;
        }
    }
}

// eq. (integrationscheme) with quaternion renormalisation; periodic wrap.
// SPARSE (few contacts): only the touched bodies' records are read; every
// other body takes the record k_init_bodies would have written.
template <class T, bool SPARSE>
__global__ void __launch_bounds__(kBlock) k_integrate(BodiesView b, Grid g0, SceneTable st, double dt, const T *vel,
                                                      const uint8_t *touched, double gx, double gy, double gz,
                                                      const int32_t *recmap) {
    // the workgroup's records are read as one contiguous run into LDS (neighbouring lanes load neighbouring words)
    constexpr int S = kStageRow<T>;
    __shared__ T stage[SPARSE ? 1 : 8 * S];
    const int i0 = blockIdx.x * kBlock;
    const int t = threadIdx.x, i = i0 + t;
    T rec[6];
    bool untouched = false;  // a body no contact touched (SPARSE): only the changed velocity words are written
    double old[6];
    if constexpr (SPARSE) {
        if (i >= b.n) return;
        if (touched[i]) {
            const T *r = vel + 8 * (int64_t)i;
#pragma unroll
            for (int a = 0; a < 6; ++a) rec[a] = r[a];
        } else {
            untouched = true;
            old[0] = b.vx[i];
            old[1] = b.vy[i];
            old[2] = b.vz[i];
            old[3] = b.wx[i];
            old[4] = b.wy[i];
            old[5] = b.wz[i];
            const bool dyn = b.inv_mass[i] > 0.0;
            rec[0] = (T)(dyn ? old[0] + dt * gx : old[0]);
            rec[1] = (T)(dyn ? old[1] + dt * gy : old[1]);
            rec[2] = (T)(dyn ? old[2] + dt * gz : old[2]);
#pragma unroll
            for (int a = 3; a < 6; ++a) rec[a] = (T)old[a];
        }
    } else {
        (void)touched;
        (void)gx;
        (void)gy;
        (void)gz;
        if (recmap) {  // records in the block-local sweeps' order: each read whole from its own place
            if (i >= b.n) return;
            const T *r = vel + 8 * (int64_t)recmap[i];
#pragma unroll
            for (int a = 0; a < 6; ++a) rec[a] = r[a];
        } else {
            const int nvalid = b.n - i0 < kBlock ? b.n - i0 : kBlock;
            const T *in = vel + 8 * (int64_t)i0;
            for (int q = t; q < 8 * nvalid; q += kBlock) stage[(q & 7) * S + (q >> 3)] = in[q];
            __syncthreads();
            if (i >= b.n) return;
#pragma unroll
            for (int a = 0; a < 6; ++a) rec[a] = stage[a * S + t];
        }
    }
    const Grid &g = st.body_scene ? st.grids[st.body_scene[i]] : g0;
    const double vx = (double)rec[0], vy = (double)rec[1], vz = (double)rec[2];
    const double ox = (double)rec[3], oy = (double)rec[4], oz = (double)rec[5];
    if (untouched) {  // the same words as the full write, without storing an unchanged one
        const double nv[6] = {vx, vy, vz, ox, oy, oz};
        double *dst[6] = {b.vx, b.vy, b.vz, b.wx, b.wy, b.wz};
#pragma unroll
        for (int a = 0; a < 6; ++a)
            if (__double_as_longlong(nv[a]) != __double_as_longlong(old[a])) dst[a][i] = nv[a];
    } else {
        b.vx[i] = vx;
        b.vy[i] = vy;
        b.vz[i] = vz;
        b.wx[i] = ox;
        b.wy[i] = oy;
        b.wz[i] = oz;
    }
    double pos[3] = {b.x[i] + dt * vx, b.y[i] + dt * vy, b.z[i] + dt * vz};
    double qw = b.qw[i], qx = b.qx[i], qy = b.qy[i], qz = b.qz[i];
    const double dw = 0.5 * (-qx * ox - qy * oy - qz * oz);
    const double dx = 0.5 * (qw * ox + qz * oy - qy * oz);
    const double dy = 0.5 * (-qz * ox + qw * oy + qx * oz);
    const double dz = 0.5 * (qy * ox - qx * oy + qw * oz);
    qw = qw + dt * dw;
    qx = qx + dt * dx;
    qy = qy + dt * dy;
    qz = qz + dt * dz;
    const double len = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    b.qw[i] = qw / len;
    b.qx[i] = qx / len;
    b.qy[i] = qy / len;
    b.qz[i] = qz / len;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (!g.periodic[a]) continue;
        if (pos[a] >= g.hi[a]) pos[a] = pos[a] - g.L[a];
        else if (pos[a] < g.lo[a]) pos[a] = pos[a] + g.L[a];
    }
    b.x[i] = pos[0];
    b.y[i] = pos[1];
    b.z[i] = pos[2];
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_save_impulses(SweepView<T> sv, int64_t nc, ContactsView c) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= nc) return;
    const int j = sv.perm[p];
    c.px[j] = (double)sv.px[p];
    c.py[j] = (double)sv.py[p];
    c.pz[j] = (double)sv.pz[p];
}

// touched (few contacts): an untouched body's record is the one k_init_bodies would have written (before the
// integration) or, after it, the body's velocities (which the integration took from that record).
template <class T>
__global__ void __launch_bounds__(kBlock) k_export(const T *vel, int32_t nb, double *v, double *w, BodiesView b,
                                                   const uint8_t *touched, int pending, double gx, double gy,
                                                   double gz, double dt, const int32_t *rec) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= nb) return;
    T fr[8];
    const T *r = vel + 8 * (int64_t)(rec ? rec[i] : i);
    if (touched && !touched[i]) {
        if (pending) {
            free_record<T>(b, i, gx, gy, gz, dt, fr);
        } else {
            fr[0] = (T)b.vx[i];
            fr[1] = (T)b.vy[i];
            fr[2] = (T)b.vz[i];
            fr[3] = (T)b.wx[i];
            fr[4] = (T)b.wy[i];
            fr[5] = (T)b.wz[i];
        }
        r = fr;
    }
    v[i] = (double)r[0];
    v[nb + i] = (double)r[1];
    v[2 * (int64_t)nb + i] = (double)r[2];
    w[i] = (double)r[3];
    w[nb + i] = (double)r[4];
    w[2 * (int64_t)nb + i] = (double)r[5];
}

}  // namespace

template <class T>
nbgs_status launch_init_bodies(const BodiesView &b, const double g[3], double dt, T *vel, const int32_t *rec,
                               hipStream_t s) {
    k_init_bodies<T><<<grid_for(b.n), kBlock, 0, s>>>(b, g[0], g[1], g[2], dt, vel, rec);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

template <class T>
nbgs_status launch_warm_scatter(SweepView<T> sv, int64_t begin, int64_t end, int32_t nb, T *vel, hipStream_t s) {
    if (end <= begin) return NBGS_OK;
    k_warm_scatter<T><<<grid_for(end - begin), kBlock, 0, s>>>(sv, begin, end, nb, vel);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

template <class T>
int64_t sweep_tile(const SweepTune &t) {
    return t.lanes ? (int64_t)t.block / Chunks<T>::L : (int64_t)t.block * t.cpt;
}
template int64_t sweep_tile<double>(const SweepTune &);
template int64_t sweep_tile<float>(const SweepTune &);

bool sweep_tune_supported(const SweepTune &t) {
    const bool blk = t.block == 64 || t.block == 128 || t.block == 256 || t.block == 512;
    return blk && (t.cpt == 1 || t.cpt == 2 || t.cpt == 4) && (t.xcd_remap == 0 || t.xcd_remap == 1) &&
           (t.nontemporal == 0 || t.nontemporal == 1) && (t.full_store == 0 || t.full_store == 1) &&
           (t.persistent == 0 || t.persistent == 1 || (t.persistent >= 8 && t.persistent % 8 == 0)) &&
           (t.graph == 0 || t.graph == 1) && (t.lanes == 0 || (t.lanes == 1 && t.cpt == 1));
}

// Workgroups of a persistent sweep grid: what the device holds resident at
// once (blocks per CU at this kernel's register use, times the CU count),
// rounded down to a multiple of 8.
template <class K>
unsigned persistent_cap(K kernel, int block) {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess || per_cu <= 0) per_cu = 1;
    const unsigned cap = (unsigned)per_cu * (unsigned)cus;
    return cap < 8 ? 8u : cap & ~7u;
}

template <class T>
nbgs_status launch_sweep_colour(SweepView<T> sv, int64_t begin, int64_t end, int32_t nb, T *vel, SweepParams sp,
                                const SweepTune &t, double *partials, const int32_t *ctrl, hipStream_t s) {
    if (end <= begin) return NBGS_OK;
    const int64_t tile = sweep_tile<T>(t);
    const unsigned G = (unsigned)((end - begin + tile - 1) / tile);
    const T mu = (T)sp.mu, relax = (T)sp.relax;
    if (t.lanes) {
#define NBGS_GRP_LAUNCH(B, NT)                                                                                     \
    do {                                                                                                           \
        auto kern = k_sweep_grp<T, B, NT>;                                                                         \
        unsigned grid = G;                                                                                         \
        if (t.persistent == 1) {                                                                                   \
            static const unsigned cap = persistent_cap(kern, B);                                                   \
            if (cap < grid) grid = cap;                                                                            \
        } else if (t.persistent > 1 && (unsigned)t.persistent < grid) {                                            \
            grid = (unsigned)t.persistent;                                                                         \
        }                                                                                                          \
        kern<<<grid, B, 0, s>>>(sv, begin, end, nb, vel, mu, relax, partials, ctrl, G, t.xcd_remap);               \
        NBGS_HIP(hipGetLastError());                                                                               \
        return NBGS_OK;                                                                                            \
    } while (0)
#define NBGS_GRP_CASE(B)                                                                                           \
    if (t.block == B) {                                                                                            \
        if (t.nontemporal) NBGS_GRP_LAUNCH(B, true);                                                               \
        else NBGS_GRP_LAUNCH(B, false);                                                                            \
    }
        NBGS_GRP_CASE(64)
        NBGS_GRP_CASE(128)
        NBGS_GRP_CASE(256)
        NBGS_GRP_CASE(512)
#undef NBGS_GRP_CASE
#undef NBGS_GRP_LAUNCH
        set_error("unsupported sweep tuning block=%d with lane groups", t.block);
        return NBGS_ERR_INVALID_ARG;
    }
#define NBGS_SWEEP_LAUNCH(B, C, NT, FULL)                                                                          \
    do {                                                                                                           \
        auto kern = k_sweep<T, B, C, NT, FULL>;                                                                    \
        unsigned grid = G;                                                                                         \
        if (t.persistent == 1) {                                                                                   \
            static const unsigned cap = persistent_cap(kern, B);                                                   \
            if (cap < grid) grid = cap;                                                                            \
        } else if (t.persistent > 1 && (unsigned)t.persistent < grid) {                                            \
            grid = (unsigned)t.persistent;                                                                         \
        }                                                                                                          \
        kern<<<grid, B, 0, s>>>(sv, begin, end, nb, vel, mu, relax, partials, ctrl, G, t.xcd_remap);               \
    } while (0)
#define NBGS_SWEEP_CASE(B, C)                                                                                      \
    if (t.block == B && t.cpt == C) {                                                                              \
        if (t.nontemporal && t.full_store) NBGS_SWEEP_LAUNCH(B, C, true, true);                                    \
        else if (t.nontemporal) NBGS_SWEEP_LAUNCH(B, C, true, false);                                              \
        else if (t.full_store) NBGS_SWEEP_LAUNCH(B, C, false, true);                                               \
        else NBGS_SWEEP_LAUNCH(B, C, false, false);                                                                \
        NBGS_HIP(hipGetLastError());                                                                               \
        return NBGS_OK;                                                                                            \
    }
    NBGS_SWEEP_CASE(64, 1)
    NBGS_SWEEP_CASE(64, 2)
    NBGS_SWEEP_CASE(64, 4)
    NBGS_SWEEP_CASE(128, 1)
    NBGS_SWEEP_CASE(128, 2)
    NBGS_SWEEP_CASE(128, 4)
    NBGS_SWEEP_CASE(256, 1)
    NBGS_SWEEP_CASE(256, 2)
    NBGS_SWEEP_CASE(256, 4)
    NBGS_SWEEP_CASE(512, 1)
    NBGS_SWEEP_CASE(512, 2)
    NBGS_SWEEP_CASE(512, 4)
#undef NBGS_SWEEP_CASE
#undef NBGS_SWEEP_LAUNCH
    set_error("unsupported sweep tuning block=%d cpt=%d", t.block, t.cpt);
    return NBGS_ERR_INVALID_ARG;
}

// Workgroups of a device-range sweep launch: the explicit cap, else what the
// device holds resident at once.
template <class T, int B, int C, bool NT, bool FULL>
unsigned dev_grid(const SweepTune &t) {
    if (t.persistent > 1) return (unsigned)t.persistent;
    static const unsigned cap = persistent_cap(k_sweep_dev<T, B, C, NT, FULL>, B);
    return cap;
}

#define NBGS_SWEEP_DEV_DISPATCH(ACTION)                                                                            \
    do {                                                                                                           \
        NBGS_SWEEP_DEV_CASE(64, 1, ACTION)                                                                         \
        NBGS_SWEEP_DEV_CASE(64, 2, ACTION)                                                                         \
        NBGS_SWEEP_DEV_CASE(64, 4, ACTION)                                                                         \
        NBGS_SWEEP_DEV_CASE(128, 1, ACTION)                                                                        \
        NBGS_SWEEP_DEV_CASE(128, 2, ACTION)                                                                        \
        NBGS_SWEEP_DEV_CASE(128, 4, ACTION)                                                                        \
        NBGS_SWEEP_DEV_CASE(256, 1, ACTION)                                                                        \
        NBGS_SWEEP_DEV_CASE(256, 2, ACTION)                                                                        \
        NBGS_SWEEP_DEV_CASE(256, 4, ACTION)                                                                        \
        NBGS_SWEEP_DEV_CASE(512, 1, ACTION)                                                                        \
        NBGS_SWEEP_DEV_CASE(512, 2, ACTION)                                                                        \
        NBGS_SWEEP_DEV_CASE(512, 4, ACTION)                                                                        \
    } while (0)
#define NBGS_SWEEP_DEV_CASE(B, C, ACTION)                                                                          \
    if (t.block == B && t.cpt == C) {                                                                              \
        if (t.nontemporal && t.full_store) ACTION(B, C, true, true);                                               \
        else if (t.nontemporal) ACTION(B, C, true, false);                                                         \
        else if (t.full_store) ACTION(B, C, false, true);                                                          \
        else ACTION(B, C, false, false);                                                                           \
    }

template <class T, int B, bool NT>
unsigned dev_grid_grp(const SweepTune &t) {
    if (t.persistent > 1) return (unsigned)t.persistent;
    static const unsigned cap = persistent_cap(k_sweep_grp_dev<T, B, NT>, B);
    return cap;
}

#define NBGS_GRP_DEV_DISPATCH(ACTION)                                                                              \
    do {                                                                                                           \
        if (t.block == 64) { if (t.nontemporal) ACTION(64, true); else ACTION(64, false); }                        \
        if (t.block == 128) { if (t.nontemporal) ACTION(128, true); else ACTION(128, false); }                     \
        if (t.block == 256) { if (t.nontemporal) ACTION(256, true); else ACTION(256, false); }                     \
        if (t.block == 512) { if (t.nontemporal) ACTION(512, true); else ACTION(512, false); }                     \
    } while (0)

template <class T>
unsigned sweep_graph_grid(const SweepTune &t) {
    if (t.lanes) {
#define NBGS_GRID_OF_GRP(B, NT) return dev_grid_grp<T, B, NT>(t)
        NBGS_GRP_DEV_DISPATCH(NBGS_GRID_OF_GRP);
#undef NBGS_GRID_OF_GRP
        return 0;
    }
#define NBGS_GRID_OF(B, C, NT, FULL) return dev_grid<T, B, C, NT, FULL>(t)
    NBGS_SWEEP_DEV_DISPATCH(NBGS_GRID_OF);
#undef NBGS_GRID_OF
    return 0;
}

template <class T>
nbgs_status launch_sweep_colour_dev(SweepView<T> sv, const int64_t *col, int32_t c, int32_t nb, T *vel, SweepParams sp,
                                    const SweepTune &t, double *partials, const int32_t *ctrl, hipStream_t s) {
    const T mu = (T)sp.mu, relax = (T)sp.relax;
    if (t.lanes) {
#define NBGS_LAUNCH_GRP_DEV(B, NT)                                                                                 \
    do {                                                                                                           \
        k_sweep_grp_dev<T, B, NT><<<dev_grid_grp<T, B, NT>(t), B, 0, s>>>(sv, col, c, nb, vel, mu, relax, partials, \
                                                                         ctrl, t.xcd_remap);                      \
        NBGS_HIP(hipGetLastError());                                                                               \
        return NBGS_OK;                                                                                            \
    } while (0)
        NBGS_GRP_DEV_DISPATCH(NBGS_LAUNCH_GRP_DEV);
#undef NBGS_LAUNCH_GRP_DEV
        set_error("unsupported sweep tuning block=%d with lane groups", t.block);
        return NBGS_ERR_INVALID_ARG;
    }
#define NBGS_LAUNCH_DEV(B, C, NT, FULL)                                                                            \
    do {                                                                                                           \
        k_sweep_dev<T, B, C, NT, FULL><<<dev_grid<T, B, C, NT, FULL>(t), B, 0, s>>>(sv, col, c, nb, vel, mu, relax, \
                                                                                   partials, ctrl, t.xcd_remap);  \
        NBGS_HIP(hipGetLastError());                                                                               \
        return NBGS_OK;                                                                                            \
    } while (0)
    NBGS_SWEEP_DEV_DISPATCH(NBGS_LAUNCH_DEV);
#undef NBGS_LAUNCH_DEV
    set_error("unsupported sweep tuning block=%d cpt=%d", t.block, t.cpt);
    return NBGS_ERR_INVALID_ARG;
}
#undef NBGS_SWEEP_DEV_CASE
#undef NBGS_SWEEP_DEV_DISPATCH
#undef NBGS_GRP_DEV_DISPATCH

nbgs_status launch_residual(const double *partials, int32_t n_partials, double target, int32_t *ctrl, double *hist,
                            hipStream_t s, int32_t at) {
    k_residual<<<1, kResBlock, 0, s>>>(partials, n_partials, target, ctrl, hist, at);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

template <class T>
nbgs_status launch_integrate(const BodiesView &b, const Grid &g, const SceneTable &st, double dt, const T *vel,
                             const uint8_t *touched, const double grav[3], const int32_t *rec, hipStream_t s) {
    if (touched)
        k_integrate<T, true><<<grid_for(b.n), kBlock, 0, s>>>(b, g, st, dt, vel, touched, grav[0], grav[1], grav[2],
                                                               nullptr);
    else
        k_integrate<T, false><<<grid_for(b.n), kBlock, 0, s>>>(b, g, st, dt, vel, nullptr, 0.0, 0.0, 0.0, rec);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

nbgs_status launch_mark_touched(const int32_t *j1, const int32_t *j2, int64_t nc, int32_t nb, uint8_t *touched,
                                hipStream_t s) {
    NBGS_HIP(hipMemsetAsync(touched, 0, (size_t)nb + 1, s));
    if (nc <= 0) return NBGS_OK;
    k_mark_touched<<<grid_for(nc), kBlock, 0, s>>>(j1, j2, nc, nb, touched);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

template <class T>
nbgs_status launch_init_touched(const BodiesView &b, const double g[3], double dt, const uint8_t *touched, T *vel,
                                hipStream_t s) {
    if (b.n <= 0) return NBGS_OK;
    const unsigned blocks = std::min<unsigned>(grid_for(b.n), 4096u);
    k_init_touched<T><<<blocks, kBlock, 0, s>>>(b, g[0], g[1], g[2], dt, touched, vel);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

template <class T>
nbgs_status launch_save_impulses(SweepView<T> sv, int64_t nc, ContactsView c, hipStream_t s) {
    if (nc == 0) return NBGS_OK;
    k_save_impulses<T><<<grid_for(nc), kBlock, 0, s>>>(sv, nc, c);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

template <class T>
nbgs_status launch_export_accumulators(const T *vel, int32_t nb, double *v, double *w, const BodiesView &b,
                                       const uint8_t *touched, bool pending, const double g[3], double dt,
                                       const int32_t *rec, hipStream_t s) {
    k_export<T><<<grid_for(nb), kBlock, 0, s>>>(vel, nb, v, w, b, touched, pending ? 1 : 0, g[0], g[1], g[2], dt,
                                                rec);
    NBGS_HIP(hipGetLastError());
    return NBGS_OK;
}

#define NBGS_INSTANTIATE(T)                                                                                       \
    template nbgs_status launch_init_bodies<T>(const BodiesView &, const double[3], double, T *, const int32_t *, \
                                               hipStream_t);                                                      \
    template nbgs_status launch_warm_scatter<T>(SweepView<T>, int64_t, int64_t, int32_t, T *, hipStream_t);      \
    template nbgs_status launch_sweep_colour<T>(SweepView<T>, int64_t, int64_t, int32_t, T *, SweepParams,       \
                                                const SweepTune &, double *, const int32_t *, hipStream_t);       \
    template nbgs_status launch_integrate<T>(const BodiesView &, const Grid &, const SceneTable &, double, const T *, \
                                             const uint8_t *, const double[3], const int32_t *, hipStream_t);    \
    template nbgs_status launch_init_touched<T>(const BodiesView &, const double[3], double, const uint8_t *, T *, \
                                                hipStream_t);                                                     \
    template unsigned sweep_graph_grid<T>(const SweepTune &);                                                     \
    template nbgs_status launch_sweep_colour_dev<T>(SweepView<T>, const int64_t *, int32_t, int32_t, T *,         \
                                                    SweepParams, const SweepTune &, double *, const int32_t *,    \
                                                    hipStream_t);                                                 \
    template nbgs_status launch_save_impulses<T>(SweepView<T>, int64_t, ContactsView, hipStream_t);              \
    template nbgs_status launch_export_accumulators<T>(const T *, int32_t, double *, double *, const BodiesView &, \
                                                       const uint8_t *, bool, const double[3], double,            \
                                                       const int32_t *, hipStream_t);

NBGS_INSTANTIATE(double)
NBGS_INSTANTIATE(float)

}  // namespace nbgs
