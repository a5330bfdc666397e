// Device helpers shared by the 2-D step kernels (single step, step pair,
// batched): vector loads, row registers, the stress-divergence stencil and
// the compensated accumulation.
#pragma once
#include "elwh_internal.h"
#include "lanes.h"
#include "xcd.h"

namespace elwh {

template <typename T, int V>
struct alignas(sizeof(T) * V) VecT {
    T x[V];
};

template <typename S, typename T, int V>
__device__ __forceinline__ void vload(const S* __restrict__ p, T (&o)[V]) {
    const VecT<S, V> v = *reinterpret_cast<const VecT<S, V>*>(p);
#pragma unroll
    for (int k = 0; k < V; ++k) o[k] = (T)v.x[k];
}

template <typename T, int V>
__device__ __forceinline__ void vzero(T (&o)[V]) {
#pragma unroll
    for (int k = 0; k < V; ++k) o[k] = (T)0;
}

template <typename T, int V>
struct RawRow {
    T u[V], v[V], l[V], m[V];
};

template <typename T, int V>
struct Row {
    T u[V], v[V], l[V], m[V];
    T uL, uR, vL, vR;   // neighbours of node 0 (left) and node V-1 (right)
};

// Stencil values of one node in one row.
template <typename T>
struct Nb {
    T u, v, uL, uR, vL, vR, l, m;
};

template <typename T, int V>
__device__ __forceinline__ Nb<T> node_of(const Row<T, V>& r, int k) {
    Nb<T> n;
    n.u = r.u[k];
    n.v = r.v[k];
    n.uL = k > 0 ? r.u[k > 0 ? k - 1 : 0] : r.uL;
    n.uR = k < V - 1 ? r.u[k < V - 1 ? k + 1 : 0] : r.uR;
    n.vL = k > 0 ? r.v[k > 0 ? k - 1 : 0] : r.vL;
    n.vR = k < V - 1 ? r.v[k < V - 1 ? k + 1 : 0] : r.vR;
    n.l = r.l[k];
    n.m = r.m[k];
    return n;
}

__device__ __forceinline__ void acc_add(double& hi, double& lo, double x, bool comp) {
    if (comp) {
        // Knuth's TwoSum: hi + x = t + e exactly; e goes to the compensation.
        // Between launches the compensation is stored in FP32: it holds only
        // rounding errors, below 2^-53 of the accumulator per term, so its
        // own rounding is near 2^-77 of the accumulator and the word costs 4
        // instead of 8 bytes per component and pass.
        const double t = hi + x;
        const double z = t - hi;
        const double e = (hi - (t - z)) + (x - z);
        hi = t;
        lo += e;
    } else {
        hi += x;
    }
}

// kind 0: interior row; 1: traction-free top row (S below); 2: traction-free bottom row (N above)
template <typename T>
__device__ __forceinline__ void stencil2d(int kind, const Nb<T>& S, const Nb<T>& C, const Nb<T>& N, T lamL, T lamR,
                                          T muL, T muR, T cxx2, T cyy2, T cxy, T cyyf, T cfx, T& Lu, T& Lv) {
    const T two = (T)2;
    const T AL = lamL + two * muL, AC = C.l + two * C.m, AR = lamR + two * muR;
    const T xu = cxx2 * ((AR + AC) * (C.uR - C.u) - (AC + AL) * (C.u - C.uL));
    const T xv = cxx2 * ((muR + C.m) * (C.vR - C.v) - (C.m + muL) * (C.v - C.vL));
    if (kind == 1) {
        const T AS = S.l + two * S.m;
        Lu = xu - cyyf * (C.m + S.m) * (C.u - S.u) - cfx * (C.m * (C.vR - C.vL) + S.m * (S.vR - S.vL)) +
             cfx * (lamR * (C.vR - S.vR) - lamL * (C.vL - S.vL));
        Lv = xv - cyyf * (AC + AS) * (C.v - S.v) - cfx * (C.l * (C.uR - C.uL) + S.l * (S.uR - S.uL)) +
             cfx * (muR * (C.uR - S.uR) - muL * (C.uL - S.uL));
    } else if (kind == 2) {
        const T AN = N.l + two * N.m;
        Lu = xu + cyyf * (C.m + N.m) * (N.u - C.u) + cfx * (C.m * (C.vR - C.vL) + N.m * (N.vR - N.vL)) +
             cfx * (lamR * (N.vR - C.vR) - lamL * (N.vL - C.vL));
        Lv = xv + cyyf * (AC + AN) * (N.v - C.v) + cfx * (C.l * (C.uR - C.uL) + N.l * (N.uR - N.uL)) +
             cfx * (muR * (N.uR - C.uR) - muL * (N.uL - C.uL));
    } else {
        const T AN = N.l + two * N.m, AS = S.l + two * S.m;
        Lu = xu + cyy2 * ((N.m + C.m) * (N.u - C.u) - (C.m + S.m) * (C.u - S.u)) +
             cxy * (lamR * (N.vR - S.vR) - lamL * (N.vL - S.vL) + N.m * (N.vR - N.vL) - S.m * (S.vR - S.vL));
        Lv = xv + cyy2 * ((AN + AC) * (N.v - C.v) - (AC + AS) * (C.v - S.v)) +
             cxy * (muR * (N.uR - S.uR) - muL * (N.uL - S.uL) + N.l * (N.uR - N.uL) - S.l * (S.uR - S.uL));
    }
}

// ---- ragged batch: problem lookup and per-tick step kinds -----------------

// Problem of tile b of the concatenated tiling: binary search for the last
// problem whose first tile is at or before b (offsets ascend; a problem with
// no tiles shares its successor's offset).
__device__ __forceinline__ int batch_problem_of(const BProb2D* __restrict__ pr, int np, int b, bool two) {
    int lo = 0, hi = np - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((two ? pr[mid].off2 : pr[mid].off) <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Whether problem p takes a kb-step launch at this tick (neff: steps done in
// its application): it has taken the half step and has kb or more steps
// left; otherwise it takes a single step.
__host__ __device__ __forceinline__ bool batch_multi_step(int neff, int nsteps, int kb) {
    return kb >= 2 && neff >= 1 && nsteps - neff >= kb;
}

// The first two state buffers other than ic and ip (ip may be -1).
__host__ __device__ __forceinline__ void batch_free_two(int ic, int ip, int& x1, int& x2) {
    x1 = -1;
    x2 = -1;
    for (int i = 0; i < 4; ++i) {
        if (i == ic || i == ip) continue;
        if (x1 < 0) x1 = i;
        else if (x2 < 0) x2 = i;
    }
}

// Target of a single step: over u^{n-1} in place when that is a state
// buffer, else the first free one.
__host__ __device__ __forceinline__ int batch_single_target(int ic, int ip) {
    if (ip >= 0) return ip;
    int x1, x2;
    batch_free_two(ic, ip, x1, x2);
    return x1;
}

template <int V>
struct Cols {
    static constexpr int W = V == 4 ? 252 : 64 * V - 2;   // computed columns per wavefront
};

}  // namespace elwh
