// Stop test and absorption decision of the iteration (device code shared by
// the control kernel and the resident 2D kernel).
#pragma once

#include <math.h>

#include "jko_internal.h"

namespace jko {

// Stop test and absorption decision of one check, run by the 64 lanes of one
// wave.  Each lane sums a fixed strided subset of the per-block partials and a
// fixed xor-butterfly combines the lanes, so the result is the same bits on
// every call (the resident kernel's blocks rely on this to agree).
//   done      when the violation is <= tol (tol > 0) or not finite; the step
//             returns the p of iteration iter - 1;
//   absorb_pending  set when max |log a| or max |log b| exceeds absorb (with
//             a_only: max |log a| alone): the scalings are carried as logs from
//             the end of this iteration on.
// COH: the partials are read with device-scope loads (written by other
// blocks of the same launch); at most 256 of them (one per resident block).
template <bool COH = false>
__device__ __forceinline__ double part_ld(const double* p) {
    return COH ? __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : *p;
}

template <bool COH = false>
__device__ __forceinline__ void ctl_update(Ctl* c, const Partials& part, int nparts, int iter, double tol,
                                           int check_mass, double absorb, int a_only) {
    const int lane = threadIdx.x & 63;
    double err = 0.0, mlb = 0.0, mass = 0.0, mla = 0.0;
    if (COH) {
        // at most 4 partials per lane (256 blocks): all loads in flight at
        // once, then the same sums in the same order as the loop below
        double ve[4], vb[4], vm[4], va[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int i = lane + 64 * j;
            const bool in = i < nparts;
            ve[j] = in ? part_ld<COH>(part.err + i) : 0.0;
            vb[j] = in ? part_ld<COH>(part.maxlogb + i) : 0.0;
            vm[j] = (in && check_mass) ? part_ld<COH>(part.mass + i) : 0.0;
            va[j] = (in && check_mass) ? part_ld<COH>(part.maxloga + i) : 0.0;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (lane + 64 * j >= nparts) break;
            err += ve[j];
            mlb = fmax(mlb, vb[j]);
            if (check_mass) {
                mass += vm[j];
                mla = fmax(mla, va[j]);
            }
        }
    } else {
        for (int i = lane; i < nparts; i += 64) {
            err += part_ld<COH>(part.err + i);
            mlb = fmax(mlb, part_ld<COH>(part.maxlogb + i));
            if (check_mass) {
                mass += part_ld<COH>(part.mass + i);
                mla = fmax(mla, part_ld<COH>(part.maxloga + i));
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        err += __shfl_xor(err, o, 64);
        mlb = fmax(mlb, __shfl_xor(mlb, o, 64));
        mass += __shfl_xor(mass, o, 64);
        mla = fmax(mla, __shfl_xor(mla, o, 64));
    }
    if (lane == 0) {
        c->err = err;
        c->maxlogb = mlb;
        if (check_mass) {
            c->mass = mass;
            c->maxloga = mla;
        }
        const bool finite = isfinite(err) && (!check_mass || isfinite(mass));
        if (!finite) {
            c->nonfinite = 1;
            c->done = 1;
            c->stop_iter = iter - 1;
        } else if (tol > 0.0 && err <= tol) {
            c->done = 1;
            c->stop_iter = iter - 1;
        }
        // the switch itself happens after this iteration's proximal
        // half-step (the scalings are converted, then logmode is set)
        c->absorb_pending = 0;
        if (!c->done && !c->logmode && absorb > 0.0 &&
            ((!a_only && mlb > absorb) || (check_mass && mla > absorb))) {
            c->absorb_pending = 1;
            c->absorptions += 1;
        }
    }
}

}  // namespace jko
