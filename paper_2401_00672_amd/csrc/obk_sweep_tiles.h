// Device bodies of the two sweep phases over one tile, shared by the
// per-group kernels and the batched team kernel.  T is the arithmetic type
// (double, or float in the inner sweeps of iterative refinement).
//
// phase R (one group): for each row a of the tile, from the same x,
//   w_a = (f_a - sum_k a_ak x_k) * inv_a
// phase S (one group): for each touched column c of the tile,
//   x_c = x_c + sum over the group's rows a holding c of w_a a_ac
// Entries are staged through LDS in chunks of kTileEntries; each row (column)
// is then reduced by one thread in ascending entry order.  Written in
// predicated form: every load is issued at an in-range index.
#pragma once

#include "obk_internal.h"

namespace obk {

template <class T>
__device__ __forceinline__ void tile_phase_r(const Tile& t, T* prod, const int64_t* __restrict__ rptr,
                                             const int32_t* __restrict__ rcol, const T* __restrict__ rval,
                                             const T* __restrict__ rf, const T* __restrict__ rinv,
                                             const T* __restrict__ x, T* __restrict__ w) {
    const int nseg = t.seg_end - t.seg_begin;
    const int me = threadIdx.x;
    const bool owner = me < nseg;
    const int64_t a = t.seg_begin + (owner ? me : 0);
    const int64_t k0 = rptr[a], k1 = rptr[a + 1];
    T acc = T(0);
    for (int64_t base = t.ent_begin; base < t.ent_end; base += kTileEntries) {
        const int len = (int)min<int64_t>(kTileEntries, t.ent_end - base);
        for (int q = me; q < len; q += kTileThreads) prod[q] = rval[base + q] * x[rcol[base + q]];
        __syncthreads();
        const int64_t lo = max(k0, base), hi = owner ? min(k1, base + len) : lo;
        for (int64_t k = lo; k < hi; k++) acc = acc + prod[k - base];
        __syncthreads();
    }
    const T fa = rf[a], ia = rinv[a];
    if (owner) w[a] = (fa - acc) * ia;
}

template <class T>
__device__ __forceinline__ void tile_phase_s(const Tile& t, T* prod, const int64_t* __restrict__ sptr,
                                             const int32_t* __restrict__ srow, const T* __restrict__ sval,
                                             const int32_t* __restrict__ tcol, const T* __restrict__ w,
                                             T* __restrict__ x) {
    const int nseg = t.seg_end - t.seg_begin;
    const int me = threadIdx.x;
    const bool owner = me < nseg;
    const int64_t sg = t.seg_begin + (owner ? me : 0);
    const int64_t k0 = sptr[sg], k1 = sptr[sg + 1];
    T acc = T(0);
    for (int64_t base = t.ent_begin; base < t.ent_end; base += kTileEntries) {
        const int len = (int)min<int64_t>(kTileEntries, t.ent_end - base);
        for (int q = me; q < len; q += kTileThreads) prod[q] = w[srow[base + q]] * sval[base + q];
        __syncthreads();
        const int64_t lo = max(k0, base), hi = owner ? min(k1, base + len) : lo;
        for (int64_t k = lo; k < hi; k++) acc = acc + prod[k - base];
        __syncthreads();
    }
    const int32_t c = tcol[sg];
    const T xc = x[c];
    if (owner) x[c] = xc + acc;
}

}  // namespace obk
