// common.hpp -- device helpers shared by the step and patch kernels:
// wavefront lane exchange, boundary index map, an edge's update terms
// (fluctuations with the limited correction flux folded in) and the
// y-pipeline slot.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "solvers.hpp"

namespace mc {

constexpr int WAVE = 64;
constexpr int TXO = WAVE - 4;  // output columns per work item

// ------------------------------------------------------------ lane exchange
// value of lane (lane + delta) mod 64, via the LDS crossbar (ds_bpermute)
__device__ __forceinline__ float xlane(int addr, float v)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}
__device__ __forceinline__ double xlane(int addr, double v)
{
    const long long x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)(x & 0xffffffffll));
    const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(x >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Neighbour exchange of the strip walkers: the value lane - 1 holds
// (from_left) and lane + 1 holds (from_right).  64-bit values use the DPP
// wave shifts (wave_shr:1 / wave_shl:1) with bound control, so every lane
// is written and no copy of the source is needed: two VALU moves, no LDS
// round trip.  The end lanes receive 0 (lane 0 from the left, lane 63 from
// the right); what they and the next lane inward compute from it belongs
// to halo lanes 0, 1, 62 and 63, whose results are discarded.  32-bit values
// use one ds_bpermute, which costs no VALU slot; measured on the 4096^2
// step, this split is the faster one for both types.
__device__ __forceinline__ int dpp_from_left(int v)
{
    return __builtin_amdgcn_mov_dpp(v, 0x138, 0xF, 0xF, true);  // wave_shr:1
}
__device__ __forceinline__ int dpp_from_right(int v)
{
    return __builtin_amdgcn_mov_dpp(v, 0x130, 0xF, 0xF, true);  // wave_shl:1
}
__device__ __forceinline__ float from_left(int up, float v) { return xlane(up, v); }
__device__ __forceinline__ float from_right(int dn, float v) { return xlane(dn, v); }
__device__ __forceinline__ double from_left(int, double v)
{
    const long long x = __double_as_longlong(v);
    const int lo = dpp_from_left((int)(x & 0xffffffffll)), hi = dpp_from_left((int)(x >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double from_right(int, double v)
{
    const long long x = __double_as_longlong(v);
    const int lo = dpp_from_right((int)(x & 0xffffffffll)), hi = dpp_from_right((int)(x >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const int lane = threadIdx.x & 63;
        const double o = xlane(((lane ^ off) & 63) << 2, v);
        v = o > v ? o : v;
    }
    return v;
}

// A value every lane holds alike (read from LDS, say) made a scalar: the
// branch it controls is then uniform for the compiler too.  Cross-lane
// reads (ds_bpermute) must only happen in uniform control flow: where the
// compiler sees a divergent branch it may run the lanes of one wavefront
// through different iterations of a loop, and a lane read from a lane that
// is not active returns 0.
__device__ __forceinline__ bool uniform_flag(bool b)
{
    return __builtin_amdgcn_readfirstlane(b ? 1 : 0) != 0;
}

__device__ __forceinline__ int bc_map(int i, int n, int bc)
{
    if (bc == 0) {  // periodic
        int r = i % n;
        return r < 0 ? r + n : r;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// bc_map of an index every lane holds alike (a row of a strip walker),
// both rules evaluated on the scalar unit and selected, so no branch
__device__ __forceinline__ int row_map(int j, int n, int bc)
{
    j = __builtin_amdgcn_readfirstlane(j);
    int r = j % n;
    r = r < 0 ? r + n : r;
    const int c = j < 0 ? 0 : (j >= n ? n - 1 : j);
    return bc == 0 ? r : c;
}

// a pointer every lane holds alike, made a scalar for the compiler (buffer
// resources built from it then need no per-lane loop)
template <typename P>
__device__ __forceinline__ P* uniform_ptr(P* p)
{
    const unsigned long long v = (unsigned long long)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return (P*)(((unsigned long long)hi << 32) | lo);
}

// ------------------------------------------------------------- fused step
// The two quantities the conservative update takes from one edge:
// lf = A-dQ + F (it updates the cell on the left) and rg = A+dQ - F (the
// cell on the right), F being the edge's correction flux.  dl and dr are
// what the limiter takes from the left and right neighbour edges (pair());
// solvers with a limiter of their own (SLOPE) take these in lterms().
template <class S, int LIM, typename T>
__device__ __forceinline__ void edge_terms(const DevParams& P, const typename S::E& e, const T* dl,
                                           const T* dr, T nu, T* lf, T* rg)
{
    if constexpr (S::SLOPE) {
        S::template lterms<LIM>(P, e, dl, dr, nu, lf, rg);
    } else {
        T coef[S::MWAVES];
#pragma unroll
        for (int p = 0; p < S::MWAVES; ++p) {
            if (LIM == LIM_FIRST_ORDER) {
                coef[p] = T(0);
            } else {
                const T nrm = S::norm2(P, e, p);
                const T s = S::speed(P, e, p);
                const T as = fabs(s);
                const T phi = limiter_phi<LIM, T>(s > T(0) ? dl[p] : dr[p], nrm);
                coef[p] = (T(0.5) * as) * fma(-nu, as, T(1)) * phi;
            }
        }
        S::terms(P, e, coef, lf, rg);
    }
}

// state of the y-sweep pipeline for one row parity (two alternate, so no
// register copies are needed from one row to the next)
template <class SY, typename T>
struct YSlot {
    typename SY::C c;                       // Q* of the row, prepared for the y-solve
    typename SY::E e;                       // y-edge between this row and the row above
    T d[SY::MWAVES];                        // its wave products with the edge above it
    T araw[SY::MAUX > 0 ? SY::MAUX : 1];    // the row's aux values as loaded (before prep)
};

}  // namespace mc
