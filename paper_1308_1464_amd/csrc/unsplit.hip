// unsplit.hip -- the unsplit 2D step with transverse Riemann solves on
// gfx950: both directions' edge solves from the one state q^n in a single
// pass (the paper found computing both directions at once its simplest and
// fastest form, section 2).  The method is the corner-transport form of the
// wave-propagation method (LeVeque 2002, chapters 20-21) with first-order
// transverse propagation and limited normal corrections:
//
//   Q' = Q - nux (A+dQ_{i-1/2} + A-dQ_{i+1/2}) - nuy (B+dQ_{j-1/2} + B-dQ_{j+1/2})
//          - nux (F_{i+1/2} - F_{i-1/2}) - nuy (G_{j+1/2} - G_{j-1/2}),
//
// F, G the limited normal corrections, each corrected by the transverse
// parts of the fluctuations of the other direction that enter the cells
// next to it: G_{i,j+1/2} -= nux/2 (B+A+dQ_{i-1/2,j} + B+A-dQ_{i+1/2,j}),
// G_{i,j-1/2} -= nux/2 (B-A+dQ_{i-1/2,j} + B-A-dQ_{i+1/2,j}), and the same
// with x and y exchanged for F.
//
// Layout: the strip walker of the split step.  Lane k of a wavefront owns
// column i0 - 2 + k and walks rows j0 - 2 .. j1 + 1 of q^n.  For row jj it
//   1. solves the x-edge left of its cell (lane exchange), limits it with
//      its neighbours and forms the normal x contribution to its cell, and
//      splits the two fluctuations of that edge transversally: the parts
//      entering its cell going up (U) and down (D);
//   2. solves the y-edge between rows jj - 1 and jj, splits its two
//      fluctuations transversally (right- and left-going parts, combined
//      across lanes into the F corrections of rows jj and jj - 1), and
//      completes the limited y-correction of the edge below row jj - 1;
//   3. finishes row jj - 2, whose every term is now known.
// Two slots alternate between rows (as in the split walker), each holding a
// row's prepared cell, its y-edge, and its partial sums.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "../../include/manyclaw.h"
#include "common.hpp"

namespace mc {
namespace uns {

constexpr int UBLOCK = 256;

// ------------------------------------------------------------ transverse splits
// Split d at an edge of normal direction IXY (record e, prepared cells L, R)
// into the parts moving down and up (IXY = 1) or left and right (IXY = 2) in
// the other direction.

// advection: the transverse velocity's sign
template <typename T, int IXY>
__device__ __forceinline__ void tsplit(const Componentwise<AdvectionC<T, IXY>>*, const DevParams& P,
                                       const typename Componentwise<AdvectionC<T, IXY>>::E&,
                                       const typename Componentwise<AdvectionC<T, IXY>>::C&,
                                       const typename Componentwise<AdvectionC<T, IXY>>::C&, const T* d,
                                       T* bm, T* bp)
{
    const T w = T(IXY == 1 ? P.v : P.u);
    const T wm = w < T(0) ? w : T(0), wp = w > T(0) ? w : T(0);
    bm[0] = wm * d[0];
    bp[0] = wp * d[0];
}

// constant-coefficient acoustics, q = (p, u, v): the two acoustic waves of
// the transverse direction, r = (-+Z, e_t) at speeds -+c
template <typename T, int IXY>
__device__ __forceinline__ void tsplit(const Componentwise<AcousticsC<T, IXY>>*, const DevParams& P,
                                       const typename Componentwise<AcousticsC<T, IXY>>::E&,
                                       const typename Componentwise<AcousticsC<T, IXY>>::C&,
                                       const typename Componentwise<AcousticsC<T, IXY>>::C&, const T* d,
                                       T* bm, T* bp)
{
    constexpr int t = IXY == 1 ? 2 : 1, o = IXY == 1 ? 1 : 2;
    const T Z = T(sqrt(P.K * P.rho)), c = T(sqrt(P.K / P.rho));
    const T b1 = (-d[0] + Z * d[t]) / (T(2) * Z);
    const T b3 = (d[0] + Z * d[t]) / (T(2) * Z);
    bm[0] = (c * b1) * Z;
    bm[t] = -(c * b1);
    bm[o] = T(0);
    bp[0] = (c * b3) * Z;
    bp[t] = c * b3;
    bp[o] = T(0);
}

// shallow water: eigenvectors of the transverse direction at the Roe
// average (vn, vt: averaged normal and transverse velocities, c = sqrt(g
// hbar)).  A dry edge passes c = 0 with d = 0 (its normal solve has no waves
// and no fluctuations): both parts are then 0.
template <typename T, int n, int t>
__device__ __forceinline__ void sw_tsplit(T vn, T vt, T c, const T* d, T* bm, T* bp)
{
    const T r2c = c > T(0) ? T(0.5) / c : T(0);
    const T b1 = ((vt + c) * d[0] - d[t]) * r2c;
    const T b2 = d[n] - vn * d[0];
    const T b3 = (d[t] - (vt - c) * d[0]) * r2c;
    const T l1 = vt - c, l2 = vt, l3 = vt + c;
    const T m1 = l1 < T(0) ? l1 : T(0), m2 = l2 < T(0) ? l2 : T(0), m3 = l3 < T(0) ? l3 : T(0);
    const T p1 = l1 - m1, p2 = l2 - m2, p3 = l3 - m3;
    const T a1 = m1 * b1, a2 = m2 * b2, a3 = m3 * b3;
    bm[0] = a1 + a3;
    bm[n] = (a1 + a3) * vn + a2;
    bm[t] = a1 * l1 + a3 * l3;
    const T c1 = p1 * b1, c2 = p2 * b2, c3 = p3 * b3;
    bp[0] = c1 + c3;
    bp[n] = (c1 + c3) * vn + c2;
    bp[t] = c1 * l1 + c3 * l3;
}

// shallow water, Roe: the edge's own Roe average (record: v[3] = s1, v[4] =
// s3, v[5] = transverse velocity, v[6] = normal velocity; all 0 on a dry edge)
template <typename T, int IXY>
__device__ __forceinline__ void tsplit(const SwRoe<T, IXY>*, const DevParams&, const typename SwRoe<T, IXY>::E& e,
                                       const typename SwRoe<T, IXY>::C&, const typename SwRoe<T, IXY>::C&,
                                       const T* d, T* bm, T* bp)
{
    sw_tsplit<T, SwRoe<T, IXY>::MU, SwRoe<T, IXY>::MV>(e.v[6], e.v[5], T(0.5) * (e.v[4] - e.v[3]), d, bm, bp);
}

// shallow water, HLLE: the Roe average of the edge's two cells (cell v[3],
// v[4] = normal and transverse velocity, v[5] = sqrt(h)); none on a dry edge
template <typename T, int IXY>
__device__ __forceinline__ void tsplit(const Componentwise<SwHlleC<T, IXY>>*, const DevParams& P,
                                       const typename Componentwise<SwHlleC<T, IXY>>::E&,
                                       const typename Componentwise<SwHlleC<T, IXY>>::C& L,
                                       const typename Componentwise<SwHlleC<T, IXY>>::C& R, const T* d, T* bm, T* bp)
{
    const bool wet = L.v[0] > T(0) && R.v[0] > T(0);
    const T sl = L.v[5], sr = R.v[5];
    const T w = sl + sr;
    T vn = (sl * L.v[3] + sr * R.v[3]) / w;
    T vt = (sl * L.v[4] + sr * R.v[4]) / w;
    T c = sqrt(T(P.g) * (T(0.5) * (L.v[0] + R.v[0])));
    if (!wet) { vn = T(0); vt = T(0); c = T(0); }
    sw_tsplit<T, SwHlleC<T, IXY>::MU, SwHlleC<T, IXY>::MV>(vn, vt, c, d, bm, bp);
}

// Euler, Roe: eigenvectors of the transverse direction at the Roe average
// of the two cells (cell v[4], v[5] = normal and transverse velocity, v[6] =
// H, v[7] = sqrt(rho)); no transverse part where the average's c^2 <= 0
template <typename T, int IXY>
__device__ __forceinline__ void tsplit(const Componentwise<EulerRoeC<T, IXY>>*, const DevParams& P,
                                       const typename Componentwise<EulerRoeC<T, IXY>>::E&,
                                       const typename Componentwise<EulerRoeC<T, IXY>>::C& L,
                                       const typename Componentwise<EulerRoeC<T, IXY>>::C& R, const T* d,
                                       T* bm, T* bp)
{
    constexpr int n = EulerRoeC<T, IXY>::MU, t = EulerRoeC<T, IXY>::MV;
    const T gm1 = T(P.gamma - 1.0);
    const T w = L.v[7] + R.v[7];
    const T un = (L.v[7] * L.v[4] + R.v[7] * R.v[4]) / w;
    const T ut = (L.v[7] * L.v[5] + R.v[7] * R.v[5]) / w;
    const T H = (L.v[7] * L.v[6] + R.v[7] * R.v[6]) / w;
    const T q2 = un * un + ut * ut;
    const T c2 = gm1 * (H - T(0.5) * q2);
#pragma unroll
    for (int m = 0; m < 4; ++m) { bm[m] = T(0); bp[m] = T(0); }
    if (!(c2 > T(0))) return;
    const T c = sqrt(c2);
    const T b2 = gm1 / c2 * ((H - q2) * d[0] + un * d[n] + ut * d[t] - d[3]);
    const T b3 = d[n] - un * d[0];
    const T b1 = ((ut + c) * d[0] - d[t] - c * b2) / (T(2) * c);
    const T b4 = d[0] - b1 - b2;
    const T lam[4] = {ut - c, ut, ut, ut + c};
    const T b[4] = {b1, b2, b3, b4};
    T r[4][4];
    r[0][0] = T(1); r[0][n] = un; r[0][t] = ut - c; r[0][3] = H - ut * c;
    r[1][0] = T(1); r[1][n] = un; r[1][t] = ut; r[1][3] = T(0.5) * q2;
    r[2][0] = T(0); r[2][n] = T(1); r[2][t] = T(0); r[2][3] = un;
    r[3][0] = T(1); r[3][n] = un; r[3][t] = ut + c; r[3][3] = H + ut * c;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const T lm = lam[p] < T(0) ? lam[p] : T(0), lp = lam[p] - lm;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            bm[m] = bm[m] + (lm * b[p]) * r[p][m];
            bp[m] = bp[m] + (lp * b[p]) * r[p][m];
        }
    }
}

// variable-coefficient acoustics (LeVeque 2002, ch. 21): the split of d entering cell m uses the
// impedances Z = rho c and speeds of m and of its neighbours across the
// transverse direction, b (below / left) and a (above / right): the down-
// (left-) going wave of the problem between b and m and the up- (right-)
// going wave of the problem between m and a.  T is the transverse velocity
// component (2 for x-edges, 1 for y-edges).
template <int TC, typename T>
__device__ __forceinline__ void tsplit_vc(const T* d, T Zb, T cb, T Zm, T Za, T ca, T* bm, T* bp)
{
    constexpr int o = 3 - TC;
    const T g1 = (-d[0] + Zm * d[TC]) / (Zb + Zm);
    const T g2 = (d[0] + Zm * d[TC]) / (Zm + Za);
    bm[0] = (cb * g1) * Zb;
    bm[TC] = -(cb * g1);
    bm[o] = T(0);
    bp[0] = (ca * g2) * Za;
    bp[TC] = ca * g2;
    bp[o] = T(0);
}

// ------------------------------------------------------------ the walker
template <class SY, typename T>
struct USlot {
    typename SY::C c;          // q^n of the row, prepared for the y-solve
    typename SY::E e;          // y-edge between this row and the one below
    T d[SY::MWAVES];           // its wave products with the edge below it
    T acc[SY::MEQN];           // the row's new value, terms added as they become known
    T u[SY::MEQN];             // up-going transverse parts entering the cell (for the G sum above it)
};

struct UArgs {
    const void* q;
    const void* aux;      // [maux][ny][nx] or null
    void* qo;
    DevParams P;
    int nx, ny, bc;
    double nux, nuy;
    int rows, nstrips, nitems;
    unsigned long long* smax_bits;  // [2]
    unsigned int* status;
};

template <typename T, template <typename, int> class SOL, int LIM>
struct UWalker {
    using SX = SOL<T, 1>;
    using SY = SOL<T, 2>;
    static constexpr int M = SX::MEQN, NW = SX::MWAVES, NC = SX::NC, NX = SX::NX, NA = SX::MAUX;
    using Slot = USlot<SY, T>;

    const T* __restrict__ q;
    const T* __restrict__ aux;
    T* __restrict__ qo;
    DevParams P;
    int64_t plane;
    int nx, ny, bc;
    int up, dn;
    int i, im, j0, nrows;
    bool outcol, xcount;
    T nux, nuy, hx, hy;
    T nq[M + NA];
    T outv[M];          // the row finished last, stored at the start of the next
    int64_t outoff;
    bool outpend;
    T smx, smy;
    unsigned st;

    // stores of the finished row go out after a wait for all vector memory
    // operations at the start of the next row, so that the wait covers
    // loads and stores issued a row earlier
    __device__ __forceinline__ void flush()
    {
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), expcnt and lgkmcnt untouched
        if (outpend) {
#pragma unroll
            for (int m = 0; m < M; ++m) qo[outoff + m * plane] = outv[m];
            outpend = false;
        }
    }

    __device__ __forceinline__ void fetch(int rel)
    {
        const int64_t off = (int64_t)bc_map(j0 + rel, ny, bc) * nx + im;
#pragma unroll
        for (int m = 0; m < M; ++m) nq[m] = q[off + m * plane];
#pragma unroll
        for (int k = 0; k < NA; ++k) nq[M + k] = aux[off + k * plane];
    }

    // row rel: N holds row rel - 2 (finished here) and takes row rel; O
    // holds row rel - 1.  A row's accumulator starts as q - nux X (its normal
    // x terms) and receives, as they become known: the G sums of the y-edges
    // below (this row) and above (next row) it, the F corrections of the
    // transverse parts of the same two y-edges, and the limited normal y
    // terms of the edges below (next row) and above (the row after)
    __device__ __forceinline__ void row(int rel, Slot& N, Slot& O)
    {
        flush();
        T raw[M + NA];
#pragma unroll
        for (int m = 0; m < M + NA; ++m) raw[m] = nq[m];
        if (rel + 1 < nrows + 2) fetch(rel + 1);
        // ---- 1. x-edge left of the cell: normal terms and transverse parts
        typename SX::C c;
#pragma unroll
        for (int m = 0; m < M; ++m) c.v[m] = raw[m];
#pragma unroll
        for (int k = 0; k < NA; ++k) c.v[NC - NA + k] = raw[M + k];
        SX::prep(P, c);
        typename SX::C l;
#pragma unroll
        for (int k = 0; k < NC; ++k) l.v[k] = from_left(up, c.v[k]);
        typename SX::E ex;
        const unsigned sx_st = SX::solve(P, l, c, ex);
        typename SX::E el;
#pragma unroll
        for (int k = 0; k < NX; ++k) el.v[k] = from_left(up, ex.v[k]);
        T d[NW], dr[NW], trl[NW];  // trl: what the edge on the left takes from this one
        SX::pair(P, ex, el, d, trl);
#pragma unroll
        for (int p = 0; p < NW; ++p) dr[p] = from_right(dn, trl[p]);
        T acc[M];
        {
            T lf[M], rg[M];
            edge_terms<SX, LIM>(P, ex, d, dr, nux, lf, rg);
#pragma unroll
            for (int m = 0; m < M; ++m) acc[m] = fma(-nux, rg[m] + from_right(dn, lf[m]), raw[m]);
        }
        T U[M], D[M];
        if constexpr (NA > 0) {
            // variable coefficients: the split depends on the receiving cell
            // only, so split the whole x-fluctuation entering this cell (A+
            // of the left edge, A- of the right edge) with the materials of
            // this cell and of the cells below (slot O) and above (prefetched)
            T am[M], ap[M], din[M];
            SX::fluct(P, ex, am, ap);
#pragma unroll
            for (int m = 0; m < M; ++m) din[m] = ap[m] + from_right(dn, am[m]);
            tsplit_vc<2, T>(din, O.c.v[3], O.c.v[4], c.v[3], nq[M] * nq[M + 1], nq[M + 1], D, U);
        } else {
            T am[M], ap[M], bm[M], bp[M];
            SX::fluct(P, ex, am, ap);
            tsplit((const SX*)nullptr, P, ex, l, c, am, bm, bp);
#pragma unroll
            for (int m = 0; m < M; ++m) { U[m] = from_right(dn, bp[m]); D[m] = from_right(dn, bm[m]); }
            tsplit((const SX*)nullptr, P, ex, l, c, ap, bm, bp);
#pragma unroll
            for (int m = 0; m < M; ++m) { U[m] = U[m] + bp[m]; D[m] = D[m] + bm[m]; }
        }
        if (rel >= 0 && rel < nrows && xcount) {
            smx = fmax(smx, SX::smax(P, ex));
            st |= sx_st;
        }
        // G sum of the y-edge below this row: U of the row below + D of this row
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const T gt = hx * (O.u[m] + D[m]);
            acc[m] = fma(-nuy, gt, acc[m]);
            O.acc[m] = fma(nuy, gt, O.acc[m]);
        }
        // ---- 2. y-edge between rows rel - 1 and rel
#pragma unroll
        for (int m = 0; m < M; ++m) N.c.v[m] = raw[m];
#pragma unroll
        for (int k = 0; k < NA; ++k) N.c.v[NC - NA + k] = raw[M + k];
        SY::prep(P, N.c);
        if (rel >= -1) {
            const unsigned sy_st = SY::solve(P, O.c, N.c, N.e);
            T tro[NW];  // what the limiter of the edge above (slot O) takes from N.e
            if (rel >= 0) SY::pair(P, N.e, O.e, N.d, tro);
            if (rel >= 0 && rel <= nrows && outcol) {
                smy = fmax(smy, SY::smax(P, N.e));
                st |= sy_st;
            }
            {
                // transverse parts: B+dQ enters this row's cell, B-dQ the cell
                // below; the right-going part of lane i and the left-going
                // part of lane i + 1 make the F correction right of cell i
                T bmq[M], bpq[M], lA[M], rA[M];
                SY::fluct(P, N.e, bmq, bpq);
                if constexpr (NA > 0) {
                    // materials of the receiving cell's left and right neighbours
                    tsplit_vc<1, T>(bpq, from_left(up, N.c.v[3]), from_left(up, N.c.v[4]), N.c.v[3],
                                    from_right(dn, N.c.v[3]), from_right(dn, N.c.v[4]), lA, rA);
                } else {
                    tsplit((const SY*)nullptr, P, N.e, O.c, N.c, bpq, lA, rA);
                }
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    const T f = rA[m] + from_right(dn, lA[m]);
                    acc[m] = fma(nux * hy, f - from_left(up, f), acc[m]);
                }
                if constexpr (NA > 0) {
                    tsplit_vc<1, T>(bmq, from_left(up, O.c.v[3]), from_left(up, O.c.v[4]), O.c.v[3],
                                    from_right(dn, O.c.v[3]), from_right(dn, O.c.v[4]), lA, rA);
                } else {
                    tsplit((const SY*)nullptr, P, N.e, O.c, N.c, bmq, lA, rA);
                }
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    const T f = rA[m] + from_right(dn, lA[m]);
                    O.acc[m] = fma(nux * hy, f - from_left(up, f), O.acc[m]);
                }
            }
            if (rel >= 1) {
                // the limited y-edge between rows rel - 2 and rel - 1
                T lfy[M], rgy[M];
                edge_terms<SY, LIM>(P, O.e, O.d, tro, nuy, lfy, rgy);
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    N.acc[m] = fma(-nuy, lfy[m], N.acc[m]);
                    O.acc[m] = fma(-nuy, rgy[m], O.acc[m]);
                }
            }
        }
        // ---- 3. row rel - 2 is complete
        const int ro = rel - 2;
        if (ro >= 0 && ro < nrows && outcol) {
            outoff = (int64_t)(j0 + ro) * nx + i;
            outpend = true;
#pragma unroll
            for (int m = 0; m < M; ++m) outv[m] = N.acc[m];
        }
        // ---- the slot takes row rel
#pragma unroll
        for (int m = 0; m < M; ++m) {
            N.acc[m] = acc[m];
            N.u[m] = U[m];
        }
    }
};

template <typename T, template <typename, int> class SOL, int LIM>
__global__ __launch_bounds__(UBLOCK) void unsplit_kernel(UArgs a)
{
    using W = UWalker<T, SOL, LIM>;
    using Slot = typename W::Slot;
    constexpr int M = W::M, NW = W::NW, NC = W::NC;
    const int lane = threadIdx.x & 63;
    W w;
    w.smx = T(0);
    w.smy = T(0);
    w.st = 0u;
    const int item = blockIdx.x * (UBLOCK / WAVE) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (item < a.nitems) {
        w.q = (const T*)a.q;
        w.aux = (const T*)a.aux;
        w.qo = (T*)a.qo;
        w.P = a.P;
        w.nx = a.nx;
        w.ny = a.ny;
        w.bc = a.bc;
        w.plane = (int64_t)a.nx * a.ny;
        w.up = ((lane + 63) & 63) << 2;
        w.dn = ((lane + 1) & 63) << 2;
        w.nux = T(a.nux);
        w.nuy = T(a.nuy);
        w.hx = T(0.5) * w.nux;
        w.hy = T(0.5) * w.nuy;
        const int strip = item % a.nstrips, chunk = item / a.nstrips;
        w.i = strip * TXO - 2 + lane;
        w.im = bc_map(w.i, a.nx, a.bc);
        w.j0 = chunk * a.rows;
        w.nrows = min(a.rows, a.ny - w.j0);
        w.outcol = lane >= 2 && lane < 2 + TXO && w.i < a.nx;
        w.xcount = lane >= 2 && lane <= 2 + TXO && w.i <= a.nx;
        Slot s0, s1;
#pragma unroll
        for (int k = 0; k < NC; ++k) { s0.c.v[k] = T(0); s1.c.v[k] = T(0); }
#pragma unroll
        for (int k = 0; k < W::SY::NE; ++k) { s0.e.v[k] = T(0); s1.e.v[k] = T(0); }
#pragma unroll
        for (int p = 0; p < NW; ++p) s0.d[p] = s1.d[p] = T(0);
#pragma unroll
        for (int m = 0; m < M; ++m) {
            s0.acc[m] = s0.u[m] = T(0);
            s1.acc[m] = s1.u[m] = T(0);
        }
        w.outpend = false;
        w.outoff = 0;
#pragma unroll
        for (int m = 0; m < M; ++m) w.outv[m] = T(0);
        w.fetch(-2);
        int rel = -2;
        const int rend = w.nrows + 2;
        for (; rel + 1 < rend; rel += 2) {
            w.row(rel, s0, s1);
            w.row(rel + 1, s1, s0);
        }
        if (rel < rend) w.row(rel, s0, s1);
        w.flush();
    }
    const double mx = wave_max((double)w.smx), my = wave_max((double)w.smy);
    unsigned stw = 0u;
    if (__ballot(w.st != 0u)) {
        for (unsigned b = 1; b <= 2; b <<= 1)
            if (__ballot((w.st & b) != 0u)) stw |= b;
    }
    if (lane == 0) {
        atomicMax(&a.smax_bits[0], (unsigned long long)__double_as_longlong(mx));
        atomicMax(&a.smax_bits[1], (unsigned long long)__double_as_longlong(my));
        if (stw) atomicOr(a.status, stw);
    }
}

struct UFinArgs {
    unsigned long long* bits;
    mc_cfl* cfl;
    double dx, dy, dt;
};
__global__ void unsplit_finish_kernel(UFinArgs a)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double sx = __longlong_as_double((long long)a.bits[0]) / a.dx;
    const double sy = __longlong_as_double((long long)a.bits[1]) / a.dy;
    const double sm = sx > sy ? sx : sy;
    if (a.cfl) {
        a.cfl->smax = sm;
        a.cfl->cfl = a.dt * sm;
    }
    atomicExch(&a.bits[0], 0ull);
    atomicExch(&a.bits[1], 0ull);
}

}  // namespace uns
}  // namespace mc

using namespace mc;
using namespace mc::uns;

extern "C" int mc__ctx_info(const mc_ctx* c, int* solver, int* dtype, mc_params* prm, int* cus, void** stream);
extern "C" int mc__ctx_grid(const mc_ctx* c, int* nx, int* ny, double* dx, double* dy, unsigned int** status);

namespace {

// per-context maxima [2]; the map is shared by every thread, each context's
// entry is used by the thread that owns the context
std::map<const mc_ctx*, unsigned long long*> g_bits;
std::mutex g_bits_mu;

int hip_check(hipError_t e)
{
    if (e != hipSuccess) {
        fprintf(stderr, "manyclaw: HIP error %s\n", hipGetErrorString(e));
        return MC_EHIP;
    }
    return MC_OK;
}

template <typename T, template <typename, int> class SOL, int LIM>
int launch(UArgs a, int cus, hipStream_t s)
{
    auto kfn = unsplit_kernel<T, SOL, LIM>;
    static const int occ = [kfn]() {  // thread-safe one-time query
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(kfn), UBLOCK, 0) !=
                hipSuccess ||
            nb < 1)
            nb = 1;
        return nb;
    }();
    // rows per item: fewest serial rows, rounds x (R + 4), over the resident wavefronts
    const int64_t W = (int64_t)occ * cus * (UBLOCK / WAVE);
    a.nstrips = (a.nx + TXO - 1) / TXO;
    int best = 8;
    int64_t best_cost = -1;
    for (int R = 8; R <= 1024; ++R) {
        if (R > a.ny && R != 8) break;
        const int64_t items = (int64_t)a.nstrips * ((a.ny + R - 1) / R);
        const int64_t cost = ((items + W - 1) / W) * (int64_t)(std::min(R, a.ny) + 4);
        if (best_cost < 0 || cost < best_cost || (cost == best_cost && R > best)) {
            best_cost = cost;
            best = R;
        }
    }
    a.rows = best;
    a.nitems = a.nstrips * ((a.ny + a.rows - 1) / a.rows);
    const int nblk = (a.nitems + UBLOCK / WAVE - 1) / (UBLOCK / WAVE);
    hipLaunchKernelGGL(kfn, dim3(nblk), dim3(UBLOCK), 0, s, a);
    return hip_check(hipGetLastError());
}

template <typename T, template <typename, int> class SOL>
int by_limiter(const UArgs& a, int lim, int cus, hipStream_t s)
{
    switch (lim) {
    case LIM_NONE: return launch<T, SOL, LIM_NONE>(a, cus, s);
    case LIM_MINMOD: return launch<T, SOL, LIM_MINMOD>(a, cus, s);
    case LIM_SUPERBEE: return launch<T, SOL, LIM_SUPERBEE>(a, cus, s);
    case LIM_VANLEER: return launch<T, SOL, LIM_VANLEER>(a, cus, s);
    case LIM_MC: return launch<T, SOL, LIM_MC>(a, cus, s);
    case LIM_FIRST_ORDER: return launch<T, SOL, LIM_FIRST_ORDER>(a, cus, s);
    default: return MC_EINVAL;
    }
}

template <typename T>
int by_solver(int solver, const UArgs& a, int lim, int cus, hipStream_t s)
{
    switch (solver) {
    case MC_ADVECTION: return by_limiter<T, AdvectionW>(a, lim, cus, s);
    case MC_ACOUSTICS: return by_limiter<T, AcousticsW>(a, lim, cus, s);
    case MC_SW_ROE: return by_limiter<T, SwRoe>(a, lim, cus, s);
    case MC_SW_HLLE: return by_limiter<T, SwHlle>(a, lim, cus, s);
    case MC_EULER_ROE: return by_limiter<T, EulerRoe>(a, lim, cus, s);
    case MC_ACOUSTICS_VC: return by_limiter<T, AcousticsVCW>(a, lim, cus, s);
    default: return MC_EUNSUPPORTED;
    }
}

}  // namespace

extern "C" {

void mc__unsplit_release_ctx(const mc_ctx* c)
{
    std::lock_guard<std::mutex> lk(g_bits_mu);
    auto it = g_bits.find(c);
    if (it == g_bits.end()) return;
    (void)hipFree(it->second);
    g_bits.erase(it);
}

int mc_step2d_unsplit(mc_ctx* c, mc_state* st, const void* aux, double dt, int limiter, int bc, mc_cfl* cfl_out)
{
    if (!c || !st || !st->q[0] || !st->q[1] || st->q[0] == st->q[1]) return MC_EINVAL;
    if (st->cur != 0 && st->cur != 1) return MC_EINVAL;
    if (!(dt >= 0.0) || limiter < MC_LIM_NONE || limiter > MC_LIM_FIRST_ORDER) return MC_EINVAL;
    if (bc != MC_BC_PERIODIC && bc != MC_BC_EXTRAP) return MC_EINVAL;
    int solver, dtype, cus;
    mc_params prm;
    void* stream;
    mc__ctx_info(c, &solver, &dtype, &prm, &cus, &stream);
    if (solver != MC_ADVECTION && solver != MC_ACOUSTICS && solver != MC_SW_ROE && solver != MC_SW_HLLE &&
        solver != MC_EULER_ROE && solver != MC_ACOUSTICS_VC)
        return MC_EUNSUPPORTED;
    if (solver == MC_ACOUSTICS_VC && !aux) return MC_EINVAL;
    int nx, ny;
    double dx, dy;
    unsigned int* status;
    mc__ctx_grid(c, &nx, &ny, &dx, &dy, &status);
    unsigned long long* bits = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_bits_mu);
        auto it = g_bits.find(c);
        if (it != g_bits.end()) bits = it->second;
    }
    if (!bits) {
        if (hipMalloc((void**)&bits, 2 * sizeof(unsigned long long)) != hipSuccess) return MC_ENOMEM;
        if (hip_check(hipMemset(bits, 0, 2 * sizeof(unsigned long long))) != MC_OK) {
            (void)hipFree(bits);
            return MC_EHIP;
        }
        std::lock_guard<std::mutex> lk(g_bits_mu);
        g_bits[c] = bits;
    }
    UArgs a;
    memset(&a, 0, sizeof(a));
    a.q = st->q[st->cur];
    a.aux = aux;
    a.qo = st->q[st->cur ^ 1];
    a.P.g = prm.g; a.P.gamma = prm.gamma; a.P.rho = prm.rho; a.P.K = prm.K; a.P.u = prm.u; a.P.v = prm.v;
    a.nx = nx;
    a.ny = ny;
    a.bc = bc;
    a.nux = dt / dx;
    a.nuy = dt / dy;
    a.smax_bits = bits;
    a.status = status;
    hipStream_t s = (hipStream_t)stream;
    int r = dtype == MC_F64 ? by_solver<double>(solver, a, limiter, cus, s) : by_solver<float>(solver, a, limiter, cus, s);
    if (r != MC_OK) return r;
    UFinArgs f;
    f.bits = bits;
    f.cfl = cfl_out;
    f.dx = dx;
    f.dy = dy;
    f.dt = dt;
    hipLaunchKernelGGL(unsplit_finish_kernel, dim3(1), dim3(64), 0, s, f);
    if ((r = hip_check(hipGetLastError())) != MC_OK) return r;
    st->cur ^= 1;
    return MC_OK;
}

}  // extern "C"
