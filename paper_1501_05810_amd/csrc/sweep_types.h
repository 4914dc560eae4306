// The sweep record and launch-shape types the sweep kernels are compiled
// from (kept apart from the other internal declarations).
#pragma once

#include <cstdint>

namespace nbgs {

// Sweep-ordered (colour-major) per-contact record.
template <class T>
struct SweepView {
    int32_t *j1, *j2;
    int32_t *perm;  // sweep position -> canonical index
    T *nx, *ny, *nz, *bias, *a1, *a2, *px, *py, *pz;
    T *mu;  // friction coefficient per contact (batched scenes), null: one coefficient for all
    int32_t *col, *sdom;  // colour and subdomain per sweep position (subdomain solver), else null
};

// The sweep record as the subdomain solver reads it: ls holds, for end k of
// the contact at sweep position p, the body's slot local to the contact's
// subdomain at ls[2 p + k] (-1: wall or static body).
template <class T>
struct SubView {
    const int32_t *j1, *j2, *col;
    const int16_t *ls;  // slots stay below the LDS limit (at most a few thousand)
    const T *nx, *ny, *nz, *bias, *a1, *a2;
    T *px, *py, *pz;
};

struct SweepParams {
    double mu, relax;
};

struct SweepTune {
    int32_t block = 256;   // threads per workgroup
    int32_t cpt = 1;       // contacts per thread
    int32_t xcd_remap = 1; // contiguous tile runs per XCD
    int32_t nontemporal = 0; // non-temporal hint on the streamed contact arrays
    int32_t full_store = 0;  // write whole body records back
    int32_t persistent = 0;  // at most one resident round of workgroups, each walking several tiles
    int32_t graph = 0;       // sweeps replayed from a captured HIP graph (colour ranges read on the device)
    int32_t lanes = 0;       // 1: a group of lanes per contact, one lane per 16 B chunk of a body record
};

}  // namespace nbgs
