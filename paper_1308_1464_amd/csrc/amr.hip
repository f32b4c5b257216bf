// amr.hip -- two-level refinement coupling of the split step on gfx950:
// refined patches that take r steps of dt / r per coarse step, their ghost
// cells from neighbouring patches or from the coarse level interpolated in
// space and time, and the conservative fix-up at coarse-fine edges.
//
// The paper's kernel table (section 1.2, Table 1) lists "dynamic time
// stepping" (input: the time step of the adjacent grid; output: updated
// values at grid boundaries), and the text asks that each refined grid
// manage its own time step with an update procedure on refinement
// boundaries built from spatial and temporal interpolation.  The procedure
// here is the standard one for the method: subcycling with interpolated
// ghost cells (Berger and Oliger 1984) and refluxing (Berger and Colella
// 1989); the refined patches are given (choosing them is grid management).
//
// Every grid of the hierarchy (the coarse grid and each patch) is stored
// ghost-padded, [meqn][ny + 4][nx + 4], so one walker serves both levels:
// it reads the padded array as it is (no index mapping) and x-sweeps the
// ghost rows too, so that the y-sweep reads x-swept ghost values.  The
// walker is the strip walker of the single-grid step (lane k of a wavefront
// owns column i0 - 2 + k; rows walk down a register pipeline) with two
// additions:
// The solvers are those whose fluctuations sum to a physical flux
// difference f(Q_r) - f(Q_l) (shallow water Roe and HLLE, Euler, acoustics,
// advection): the stored effective fluxes need f.
//   coarse grid  at the coarse edges listed in a per-edge map (an uncovered
//                cell on one side, a covered one on the other) it stores the
//                effective flux seen by the uncovered cell,
//                F = f(Q_u) + (A-dQ + Ftilde) or f(Q_u) - (A+dQ - Ftilde);
//   fine patch   at every boundary edge it stores (first substep) or adds
//                (later substeps) the effective flux seen by the inside cell.
// One coarse step (mc_amr_step):
//   coarse ghosts (boundary rule) -> coarse walker (dt) -> coarse ghosts of
//   the new state -> r x { fine ghosts at t + k dt / r -> fine walker (dt / r)
//   } -> reflux + average down -> smax / cfl.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <utility>
#include <vector>

#include "../../include/manyclaw.h"
#include "common.hpp"

namespace mc {
namespace amr {

constexpr int ABLOCK = 256;

struct GridDev {
    int32_t nx, ny;       // interior cells
    int64_t off;          // element offset of the padded array in its pool
    int32_t rows;         // rows per work item
    int32_t nstrips;
    int32_t ci0, cj0;     // footprint origin in coarse cells (patches)
    int64_t roff;         // fine register offset (elements)
};

struct ItemDev {
    int32_t grid, strip, chunk, pad;
};

struct WalkArgs {
    const GridDev* grids;
    const ItemDev* items;
    int nitems;
    const void* in;       // pool of padded inputs
    void* out;            // pool of padded outputs (interior written)
    DevParams P;
    double nux, nuy;
    const int32_t* xmap;  // coarse: [ny][nx + 1], slot * 2 + side or -1
    const int32_t* ymap;  // coarse: [ny + 1][nx]
    void* creg;           // coarse register [slots][meqn]
    void* freg;           // fine registers: per patch L [ny], R [ny], B [nx], T [nx] x [meqn]
    int accum;            // fine: add to the registers
    unsigned long long* smax_bits;  // [2] max |s| over counted x- and y-edges (IEEE bits)
    unsigned int* status;
};

// physical shallow-water flux in direction IXY of the raw state v[0..2]
template <typename T, int IXY>
__device__ __forceinline__ void sw_flux(T g, const T* v, T* f)
{
    const T h = v[0], hu = v[1], hv = v[2];
    if (IXY == 1) {
        const T u = hu / h;
        f[0] = hu;
        f[1] = hu * u + (T(0.5) * g) * (h * h);
        f[2] = hv * u;
    } else {
        const T w = hv / h;
        f[0] = hv;
        f[1] = hu * w;
        f[2] = hv * w + (T(0.5) * g) * (h * h);
    }
}

// physical flux in direction IXY of the raw state v (solver KIND: its
// MC_* code); the refluxing needs it for every solver whose fluctuations sum
// to a flux difference
template <typename T, int IXY, int KIND>
__device__ __forceinline__ void phys_flux(const DevParams& P, const T* v, T* f)
{
    if constexpr (KIND == MC_SW_ROE || KIND == MC_SW_HLLE) {
        sw_flux<T, IXY>(T(P.g), v, f);
    } else if constexpr (KIND == MC_EULER_ROE) {
        const T r = v[0], m1 = v[1], m2 = v[2], E = v[3];
        const T p = T(P.gamma - 1.0) * (E - T(0.5) * (m1 * m1 + m2 * m2) / r);
        const T w = (IXY == 1 ? m1 : m2) / r;
        f[0] = r * w;
        f[1] = m1 * w;
        f[2] = m2 * w;
        f[3] = (E + p) * w;
        f[IXY] = f[IXY] + p;
    } else if constexpr (KIND == MC_ACOUSTICS) {
        f[0] = T(P.K) * v[IXY];
        f[IXY] = v[0] / T(P.rho);
        f[3 - IXY] = T(0);
    } else {  // advection
        f[0] = T(IXY == 1 ? P.u : P.v) * v[0];
    }
}

template <typename T, template <typename, int> class SOL, int LIM, bool COARSE, int KIND>
struct PadWalker {
    using SX = SOL<T, 1>;
    using SY = SOL<T, 2>;
    static constexpr int M = SX::MEQN, NW = SX::MWAVES, NC = SX::NC, NX = SX::NX;
    using CX = typename SX::C;
    using EX = typename SX::E;
    using Slot = YSlot<SY, T>;

    const T* q;           // padded input of this grid
    T* qo;                // padded output of this grid
    DevParams P;
    int64_t plane;
    int nx, ny, pw;       // interior size, padded row width
    int up, dn;
    int i, ip;            // true column of this lane and its (clamped) padded column
    int j0, nrows;
    bool outcol, xcount, xown;
    T nux, nuy;
    T nq[M];
    T pend[M];
    T outv[M];            // the row finished last, stored at the start of the next
    int64_t outoff;
    bool outpend;
    T smx, smy;
    unsigned st;
    // records
    const int32_t* xmap;
    const int32_t* ymap;
    T* creg;
    T* freg;              // this patch's registers
    bool accum;

    __device__ __forceinline__ void fetch(int rel)
    {
        const T* rp = q + (int64_t)(j0 + rel + 2) * pw + ip;
#pragma unroll
        for (int m = 0; m < M; ++m) nq[m] = rp[m * plane];
    }

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

    __device__ __forceinline__ void put(T* dst, const T* F)
    {
#pragma unroll
        for (int m = 0; m < M; ++m) dst[m] = accum ? dst[m] + F[m] : F[m];
    }

    __device__ __forceinline__ void row(int rel, Slot& N, Slot& O)
    {
        flush();
        CX c;
#pragma unroll
        for (int m = 0; m < M; ++m) c.v[m] = nq[m];
        if (rel + 1 < nrows + 2) fetch(rel + 1);
        SX::prep(P, c);
        CX l;
#pragma unroll
        for (int k = 0; k < NC; ++k) l.v[k] = from_left(up, c.v[k]);
        EX e;
        const unsigned sx_st = SX::solve(P, l, c, e);
        EX el;
#pragma unroll
        for (int k = 0; k < NX; ++k) el.v[k] = from_left(up, e.v[k]);
        T d[NW], dr[NW], trl[NW];  // trl: what the edge on the left takes from this one
        SX::pair(P, e, el, d, trl);
#pragma unroll
        for (int p = 0; p < NW; ++p) dr[p] = from_right(dn, trl[p]);
        T lf[M], rg[M];
        edge_terms<SX, LIM>(P, e, d, dr, nux, lf, rg);
        T qs[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const T fr = from_right(dn, lf[m]);
            qs[m] = fma(-nux, fr, fma(-nux, rg[m], c.v[m]));
        }
        const bool inrow = rel >= 0 && rel < nrows;
        if (inrow && xcount) {
            smx = fmax(smx, SX::smax(P, e));
            st |= sx_st;
        }
        // x-edge records (edge left of this lane's cell, row j0 + rel)
        if (inrow && xown) {
            const int j = j0 + rel;
            T F[M];
            if (COARSE) {
                const int code = xmap[(int64_t)j * (nx + 1) + i];
                if (code >= 0) {
                    if ((code & 1) == 0) {          // uncovered cell on the left
                        phys_flux<T, 1, KIND>(P, l.v, F);
#pragma unroll
                        for (int m = 0; m < M; ++m) F[m] = F[m] + lf[m];
                    } else {
                        phys_flux<T, 1, KIND>(P, c.v, F);
#pragma unroll
                        for (int m = 0; m < M; ++m) F[m] = F[m] - rg[m];
                    }
                    T* dst = creg + (int64_t)(code >> 1) * M;
#pragma unroll
                    for (int m = 0; m < M; ++m) dst[m] = F[m];
                }
            } else if (i == 0) {
                phys_flux<T, 1, KIND>(P, c.v, F);
#pragma unroll
                for (int m = 0; m < M; ++m) F[m] = F[m] - rg[m];
                put(freg + (int64_t)j * M, F);
            } else if (i == nx) {
                phys_flux<T, 1, KIND>(P, l.v, F);
#pragma unroll
                for (int m = 0; m < M; ++m) F[m] = F[m] + lf[m];
                put(freg + (int64_t)(ny + j) * M, F);
            }
        }

        T q2n[M];
#pragma unroll
        for (int m = 0; m < M; ++m) { q2n[m] = N.c.v[m]; N.c.v[m] = qs[m]; }
        SY::prep(P, N.c);
        if (rel >= -1) {
            const unsigned sy_st = SY::solve(P, O.c, N.c, N.e);
            T tro[NW];  // what the limiter of the edge above (slot O) takes from N.e
            if (rel >= 0) SY::pair(P, N.e, O.e, N.d, tro);
            if (rel >= 0 && rel <= nrows && outcol) {
                smy = fmax(smy, SY::smax(P, N.e));
                st |= sy_st;
            }
            if (rel >= 1) {
                T lf[M], rg[M];
                edge_terms<SY, LIM>(P, O.e, O.d, tro, nuy, lf, rg);
                const int ro = rel - 2;
                if (ro >= 0 && ro < nrows && outcol) {
                    outoff = (int64_t)(j0 + ro + 2) * pw + (i + 2);
                    outpend = true;
#pragma unroll
                    for (int m = 0; m < M; ++m) outv[m] = fma(-nuy, lf[m], fma(-nuy, pend[m], q2n[m]));
                }
                // y-edge records: edge e between rows e - 1 (Q* = q2n) and e (O.c)
                const int ey = j0 + ro + 1;
                if (outcol && (ro + 1 < nrows || ey == ny)) {
                    T F[M];
                    if (COARSE) {
                        const int code = ymap[(int64_t)ey * nx + i];
                        if (code >= 0) {
                            if ((code & 1) == 0) {  // uncovered cell below
                                phys_flux<T, 2, KIND>(P, q2n, F);
#pragma unroll
                                for (int m = 0; m < M; ++m) F[m] = F[m] + lf[m];
                            } else {
                                phys_flux<T, 2, KIND>(P, O.c.v, F);
#pragma unroll
                                for (int m = 0; m < M; ++m) F[m] = F[m] - rg[m];
                            }
                            T* dst = creg + (int64_t)(code >> 1) * M;
#pragma unroll
                            for (int m = 0; m < M; ++m) dst[m] = F[m];
                        }
                    } else if (ey == 0) {
                        phys_flux<T, 2, KIND>(P, O.c.v, F);
#pragma unroll
                        for (int m = 0; m < M; ++m) F[m] = F[m] - rg[m];
                        put(freg + (int64_t)(2 * ny + i) * M, F);
                    } else if (ey == ny) {
                        phys_flux<T, 2, KIND>(P, q2n, F);
#pragma unroll
                        for (int m = 0; m < M; ++m) F[m] = F[m] + lf[m];
                        put(freg + (int64_t)(2 * ny + nx + i) * M, F);
                    }
                }
#pragma unroll
                for (int m = 0; m < M; ++m) pend[m] = rg[m];
            }
        }
    }
};

template <typename T, template <typename, int> class SOL, int LIM, bool COARSE, int KIND>
__global__ __launch_bounds__(ABLOCK) void walk_kernel(WalkArgs a)
{
    using W = PadWalker<T, SOL, LIM, COARSE, KIND>;
    using Slot = typename W::Slot;
    constexpr int M = W::M, NW = W::NW, NC = W::NC;
    const int lane = threadIdx.x & 63;
    const int item = blockIdx.x * (ABLOCK / WAVE) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    W w;
    w.smx = T(0);
    w.smy = T(0);
    w.st = 0u;
    if (item < a.nitems) {
        const ItemDev it = a.items[item];
        const GridDev gd = a.grids[it.grid];
        w.P = a.P;
        w.nx = gd.nx;
        w.ny = gd.ny;
        w.pw = gd.nx + 4;
        w.plane = (int64_t)(gd.nx + 4) * (gd.ny + 4);
        w.q = (const T*)a.in + gd.off;
        w.qo = (T*)a.out + gd.off;
        w.up = ((lane + 63) & 63) << 2;
        w.dn = ((lane + 1) & 63) << 2;
        w.nux = T(a.nux);
        w.nuy = T(a.nuy);
        w.i = it.strip * TXO - 2 + lane;
        w.ip = min(w.i + 2, gd.nx + 3);
        w.j0 = it.chunk * gd.rows;
        w.nrows = min(gd.rows, gd.ny - w.j0);
        w.outcol = lane >= 2 && lane < 2 + TXO && w.i < gd.nx;
        w.xcount = lane >= 2 && lane <= 2 + TXO && w.i <= gd.nx;
        // x-edge records: the edges left of the strip's own cells, and the
        // grid's last edge when the strip's last cell is the grid's (lane
        // 2 + TXO); lane 63 never owns one (its right neighbour is outside
        // the wavefront, and edge i = nx then belongs to the next strip)
        w.xown = lane >= 2 && w.i <= gd.nx && (lane < 2 + TXO || (lane == 2 + TXO && w.i == gd.nx));
        w.xmap = a.xmap;
        w.ymap = a.ymap;
        w.creg = (T*)a.creg;
        w.freg = COARSE ? nullptr : (T*)a.freg + gd.roff;
        w.accum = a.accum != 0;
#pragma unroll
        for (int m = 0; m < M; ++m) w.pend[m] = T(0);
        Slot s0, s1;
#pragma unroll
        for (int k = 0; k < NC; ++k) { s0.c.v[k] = T(0); s1.c.v[k] = T(0); }
#pragma unroll
        for (int k = 0; k < W::SY::NE; ++k) { s0.e.v[k] = T(0); s1.e.v[k] = T(0); }
#pragma unroll
        for (int p = 0; p < NW; ++p) s0.d[p] = s1.d[p] = T(0);
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
    // reductions: one atomic per wavefront and quantity
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

// ------------------------------------------------------------ ghost cells
// padded-cell index of ghost number g of a grid nx x ny (bottom two rows,
// top two rows, then the left and right two columns of the interior rows);
// returns (i, j) in interior coordinates (-2 .. n + 1)
__device__ __forceinline__ void ghost_ij(int64_t g, int nx, int ny, int& i, int& j)
{
    const int64_t wr = (int64_t)(nx + 4) * 2;
    if (g < wr) { j = (int)(g / (nx + 4)) - 2; i = (int)(g % (nx + 4)) - 2; return; }
    g -= wr;
    if (g < wr) { j = ny + (int)(g / (nx + 4)); i = (int)(g % (nx + 4)) - 2; return; }
    g -= wr;
    const int r = (int)(g / 4), c = (int)(g % 4);
    j = r;
    i = c < 2 ? c - 2 : nx + (c - 2);
}

__host__ __device__ __forceinline__ int64_t nghost(int nx, int ny) { return (int64_t)(nx + 4) * 4 + (int64_t)ny * 4; }

// coarse ghost cells by the boundary rule (in place)
template <typename T>
__global__ void coarse_ghost_kernel(T* G, int nx, int ny, int bc, int meqn)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nghost(nx, ny)) return;
    int i, j;
    ghost_ij(g, nx, ny, i, j);
    const int im = bc_map(i, nx, bc), jm = bc_map(j, ny, bc);
    const int64_t plane = (int64_t)(nx + 4) * (ny + 4);
    const int64_t dst = (int64_t)(j + 2) * (nx + 4) + (i + 2), src = (int64_t)(jm + 2) * (nx + 4) + (im + 2);
    for (int m = 0; m < meqn; ++m) G[m * plane + dst] = G[m * plane + src];
}

template <typename T>
__device__ __forceinline__ T minmod(T a, T b)
{
    return (a > T(0) && b > T(0)) ? (a < b ? a : b) : ((a < T(0) && b < T(0)) ? (a > b ? a : b) : T(0));
}

// limited linear interpolation of the padded coarse array G at fine cell (I, J)
template <typename T>
__device__ __forceinline__ T interp(const T* G, int pwc, int r, int I, int J, T xi, T eta)
{
    const int Ic = I / r, Jc = J / r;
    const T* c = G + (int64_t)(Jc + 2) * pwc + (Ic + 2);
    const T Q = c[0];
    const T sx = minmod(c[1] - Q, Q - c[-1]);
    const T sy = minmod(c[pwc] - Q, Q - c[-pwc]);
    return (Q + xi * sx) + eta * sy;
}

struct FillArgs {
    const GridDev* grids;
    int npatch;
    void* fine;              // current fine pool (ghosts written, interiors read)
    const void* gn;          // padded coarse at t
    const void* gn1;         // padded coarse at t + dt
    const int32_t* owner;    // [nyc][nxc] patch or -1
    int nxc, nyc, r, bc, meqn;
    double alpha;
};

template <typename T>
__global__ void fine_ghost_kernel(FillArgs a)
{
    const int p = blockIdx.y;
    const GridDev gd = a.grids[p];
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nghost(gd.nx, gd.ny)) return;
    int i, j;
    ghost_ij(g, gd.nx, gd.ny, i, j);
    const int NX = a.nxc * a.r, NY = a.nyc * a.r;
    int I = gd.ci0 * a.r + i, J = gd.cj0 * a.r + j;
    I = bc_map(I, NX, a.bc);
    J = bc_map(J, NY, a.bc);
    const int o = a.owner[(int64_t)(J / a.r) * a.nxc + (I / a.r)];
    T* dst = (T*)a.fine + gd.off + (int64_t)(j + 2) * (gd.nx + 4) + (i + 2);
    const int64_t plane = (int64_t)(gd.nx + 4) * (gd.ny + 4);
    if (o >= 0) {
        const GridDev go = a.grids[o];
        const int li = I - go.ci0 * a.r, lj = J - go.cj0 * a.r;
        const T* src = (const T*)a.fine + go.off + (int64_t)(lj + 2) * (go.nx + 4) + (li + 2);
        const int64_t po = (int64_t)(go.nx + 4) * (go.ny + 4);
        for (int m = 0; m < a.meqn; ++m) dst[m * plane] = src[m * po];
    } else {
        const int pwc = a.nxc + 4;
        const int64_t pc = (int64_t)(a.nxc + 4) * (a.nyc + 4);
        const T xi = T(((double)(I % a.r) + 0.5) / a.r - 0.5);
        const T eta = T(((double)(J % a.r) + 0.5) / a.r - 0.5);
        const T al = T(a.alpha);
        for (int m = 0; m < a.meqn; ++m) {
            const T va = interp<T>((const T*)a.gn + m * pc, pwc, a.r, I, J, xi, eta);
            const T vb = interp<T>((const T*)a.gn1 + m * pc, pwc, a.r, I, J, xi, eta);
            dst[m * plane] = (T(1) - al) * va + al * vb;
        }
    }
}

// ------------------------------------------------------------ fix-up
struct RefluxCell {
    int32_t i, j;
    int32_t slot[4];      // coarse register slot of the left, right, bottom, top edge, or -1
    int64_t fbase[4];     // fine register element index of the first of its r fine edges
};

struct FixArgs {
    const RefluxCell* cells;
    int ncells;
    const GridDev* grids;
    int npatch;
    void* coarse;         // padded coarse at t + dt (interior updated)
    const void* fine;     // final fine pool
    const void* creg;
    const void* freg;
    int nxc, nyc, r, meqn;
    double nux, nuy;
};

template <typename T>
__global__ void reflux_kernel(FixArgs a)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.ncells) return;
    const RefluxCell c = a.cells[k];
    const int64_t plane = (int64_t)(a.nxc + 4) * (a.nyc + 4);
    T* q = (T*)a.coarse + (int64_t)(c.j + 2) * (a.nxc + 4) + (c.i + 2);
    const T* cr = (const T*)a.creg;
    const T* fr = (const T*)a.freg;
    const T rr = T(a.r * a.r);
    for (int m = 0; m < a.meqn; ++m) {
        T v = q[m * plane];
        for (int d = 0; d < 4; ++d) {
            if (c.slot[d] < 0) continue;
            T s = fr[c.fbase[d] + m];
            for (int l = 1; l < a.r; ++l) s = s + fr[c.fbase[d] + (int64_t)l * a.meqn + m];
            const T Fbar = s / rr;
            const T Fc = cr[(int64_t)c.slot[d] * a.meqn + m];
            const T nu = T(d < 2 ? a.nux : a.nuy);
            v = v + nu * ((d & 1) ? (Fc - Fbar) : (Fbar - Fc));
        }
        q[m * plane] = v;
    }
}

template <typename T>
__global__ void average_kernel(FixArgs a)
{
    const int p = blockIdx.y;
    const GridDev gd = a.grids[p];
    const int cw = gd.nx / a.r, ch = gd.ny / a.r;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= cw * ch) return;
    const int bj = k / cw, bi = k % cw;
    const int64_t plane = (int64_t)(a.nxc + 4) * (a.nyc + 4);
    const int64_t fplane = (int64_t)(gd.nx + 4) * (gd.ny + 4);
    T* q = (T*)a.coarse + (int64_t)(gd.cj0 + bj + 2) * (a.nxc + 4) + (gd.ci0 + bi + 2);
    const T* f = (const T*)a.fine + gd.off;
    const T rr = T(a.r * a.r);
    for (int m = 0; m < a.meqn; ++m) {
        T s = T(0);
        for (int aa = 0; aa < a.r; ++aa)
            for (int b = 0; b < a.r; ++b)
                s = s + f[m * fplane + (int64_t)(bj * a.r + aa + 2) * (gd.nx + 4) + (bi * a.r + b + 2)];
        q[m * plane] = s / rr;
    }
}

// smax of the step in coarse units and the cfl; clears the maxima
struct AFinArgs {
    unsigned long long* bits;  // [4]: coarse x, coarse y, fine x, fine y
    mc_cfl* cfl;
    double dx, dy, r, dt;
};
__global__ void amr_finish_kernel(AFinArgs a)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double cx = __longlong_as_double((long long)a.bits[0]) / a.dx;
    const double cy = __longlong_as_double((long long)a.bits[1]) / a.dy;
    // fine speeds over fine cells, per coarse step of r fine steps: |s| r / (d / r) / r
    const double fx = __longlong_as_double((long long)a.bits[2]) / a.dx;
    const double fy = __longlong_as_double((long long)a.bits[3]) / a.dy;
    double sm = cx > cy ? cx : cy;
    sm = fx > sm ? fx : sm;
    sm = fy > sm ? fy : sm;
    if (a.cfl) {
        a.cfl->smax = sm;
        a.cfl->cfl = a.dt * sm;
    }
    for (int k = 0; k < 4; ++k) atomicExch(&a.bits[k], 0ull);
}

}  // namespace amr
}  // namespace mc

using namespace mc;
using namespace mc::amr;

// ------------------------------------------------------------------ host side
struct mc_amr {
    mc_ctx* ctx;
    int solver, dtype, esz, meqn;
    mc_params prm;
    int cus;
    hipStream_t stream;
    int nxc, nyc, r, bc, npatch;
    double dx, dy;
    unsigned int* status;
    std::vector<mc_amr_box> boxes;
    std::vector<GridDev> hgrids;       // [0] coarse, [1..] patches (pool offsets of their own pools)
    GridDev* grids = nullptr;          // device copy of the patch descriptors
    GridDev* cgrid = nullptr;          // device copy of the coarse descriptor
    ItemDev* citems = nullptr;
    ItemDev* fitems = nullptr;
    int ncitems = 0, nfitems = 0;
    void* cpool[2] = {nullptr, nullptr};   // padded coarse, current and next
    void* fpool[2] = {nullptr, nullptr};   // padded patches
    int ccur = 0, fcur = 0;
    int64_t fpool_elems = 0;
    int32_t* owner = nullptr;
    int32_t* xmap = nullptr;
    int32_t* ymap = nullptr;
    void* creg = nullptr;
    void* freg = nullptr;
    int64_t nslots = 0, freg_elems = 0;
    RefluxCell* rcells = nullptr;
    int nrcells = 0;
    int max_cov = 0;
    int64_t max_ghost = 0;
    unsigned long long* bits = nullptr;  // [4]
    std::vector<void*> owned;
};

extern "C" int mc__ctx_info(const mc_ctx* c, int* solver, int* dtype, mc_params* prm, int* cus, void** stream);
extern "C" int mc__ctx_grid(const mc_ctx* c, int* nx, int* ny, double* dx, double* dy, unsigned int** status);

namespace {

int hip_check(hipError_t e)
{
    if (e != hipSuccess) {
        fprintf(stderr, "manyclaw: HIP error %s\n", hipGetErrorString(e));
        return MC_EHIP;
    }
    return MC_OK;
}

int amr_alloc(mc_amr* a, void** p, size_t bytes)
{
    *p = nullptr;
    const hipError_t e = hipMalloc(p, bytes < 16 ? 16 : bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return e == hipErrorOutOfMemory ? MC_ENOMEM : MC_EHIP;
    }
    a->owned.push_back(*p);
    return MC_OK;
}

// rows per work item for a set of grids launched together: with W
// wavefronts resident at once a launch takes ceil(items / W) rounds of up to
// R + 4 rows each; take the R with the fewest serial rows (larger R on ties)
int choose_rows(const std::vector<std::pair<int, int>>& dims, int64_t W)
{
    int maxny = 1;
    for (auto& d : dims) maxny = std::max(maxny, d.second);
    int best = 8;
    int64_t best_cost = -1;
    for (int R = 8; R <= 1024; ++R) {
        if (R > maxny && R != 8) break;
        int64_t items = 0;
        for (auto& d : dims) items += (int64_t)((d.first + TXO - 1) / TXO) * ((d.second + R - 1) / R);
        const int64_t rounds = (items + W - 1) / W;
        const int64_t cost = rounds * (int64_t)(std::min(R, maxny) + 4);
        if (best_cost < 0 || cost < best_cost || (cost == best_cost && R > best)) {
            best_cost = cost;
            best = R;
        }
    }
    return best;
}

// resident wavefronts of the fine walker (its MC-limiter instance) on the device
template <typename T, template <typename, int> class SOL, int KIND>
int64_t resident_waves(int cus)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, reinterpret_cast<const void*>(walk_kernel<T, SOL, LIM_MC, false, KIND>), ABLOCK, 0) !=
            hipSuccess ||
        nb < 1)
        nb = 1;
    return (int64_t)nb * cus * (ABLOCK / WAVE);
}

template <typename T>
int64_t resident_waves_of(int solver, int cus)
{
    switch (solver) {
    case MC_SW_HLLE: return resident_waves<T, SwHlle, MC_SW_HLLE>(cus);
    case MC_EULER_ROE: return resident_waves<T, EulerRoe, MC_EULER_ROE>(cus);
    case MC_ACOUSTICS: return resident_waves<T, Acoustics, MC_ACOUSTICS>(cus);
    case MC_ADVECTION: return resident_waves<T, Advection, MC_ADVECTION>(cus);
    default: return resident_waves<T, SwRoe, MC_SW_ROE>(cus);
    }
}

// fields per cell of the solvers the coupling takes (those whose
// fluctuations sum to a physical flux difference), 0 for the others
static int amr_meqn(int solver)
{
    switch (solver) {
    case MC_SW_ROE: case MC_SW_HLLE: case MC_ACOUSTICS: return 3;
    case MC_EULER_ROE: return 4;
    case MC_ADVECTION: return 1;
    default: return 0;
    }
}

void items_for(const GridDev& g, int grid, std::vector<ItemDev>& out)
{
    const int nch = (g.ny + g.rows - 1) / g.rows;
    for (int c = 0; c < nch; ++c)
        for (int s = 0; s < g.nstrips; ++s) out.push_back(ItemDev{grid, s, c, 0});
}

template <typename T>
struct WalkLaunch {
    template <template <typename, int> class SOL, int LIM, int KIND>
    static int go(const WalkArgs& a, bool coarse, hipStream_t s)
    {
        if (a.nitems < 1) return MC_OK;
        const int nblk = (a.nitems + ABLOCK / WAVE - 1) / (ABLOCK / WAVE);
        if (coarse) hipLaunchKernelGGL((walk_kernel<T, SOL, LIM, true, KIND>), dim3(nblk), dim3(ABLOCK), 0, s, a);
        else hipLaunchKernelGGL((walk_kernel<T, SOL, LIM, false, KIND>), dim3(nblk), dim3(ABLOCK), 0, s, a);
        return hip_check(hipGetLastError());
    }
    template <template <typename, int> class SOL, int KIND>
    static int run(const WalkArgs& a, int lim, bool coarse, hipStream_t s)
    {
        switch (lim) {
        case LIM_NONE: return go<SOL, LIM_NONE, KIND>(a, coarse, s);
        case LIM_MINMOD: return go<SOL, LIM_MINMOD, KIND>(a, coarse, s);
        case LIM_SUPERBEE: return go<SOL, LIM_SUPERBEE, KIND>(a, coarse, s);
        case LIM_VANLEER: return go<SOL, LIM_VANLEER, KIND>(a, coarse, s);
        case LIM_MC: return go<SOL, LIM_MC, KIND>(a, coarse, s);
        case LIM_FIRST_ORDER: return go<SOL, LIM_FIRST_ORDER, KIND>(a, coarse, s);
        default: return MC_EINVAL;
        }
    }
    static int walk(const mc_amr* h, const WalkArgs& a, int lim, bool coarse)
    {
        switch (h->solver) {
        case MC_SW_ROE: return run<SwRoe, MC_SW_ROE>(a, lim, coarse, h->stream);
        case MC_SW_HLLE: return run<SwHlle, MC_SW_HLLE>(a, lim, coarse, h->stream);
        case MC_EULER_ROE: return run<EulerRoe, MC_EULER_ROE>(a, lim, coarse, h->stream);
        case MC_ACOUSTICS: return run<Acoustics, MC_ACOUSTICS>(a, lim, coarse, h->stream);
        case MC_ADVECTION: return run<Advection, MC_ADVECTION>(a, lim, coarse, h->stream);
        default: return MC_EUNSUPPORTED;
        }
    }
};

int walk(const mc_amr* h, const WalkArgs& a, int lim, bool coarse)
{
    return h->dtype == MC_F64 ? WalkLaunch<double>::walk(h, a, lim, coarse)
                              : WalkLaunch<float>::walk(h, a, lim, coarse);
}

template <typename T>
int step_t(mc_amr* h, double dt, int limiter, mc_cfl* cfl_out)
{
    hipStream_t st = h->stream;
    const int M = h->meqn;
    const GridDev& cg = h->hgrids[0];
    const int64_t ncg = nghost(cg.nx, cg.ny);
    T* cn = (T*)h->cpool[h->ccur];
    T* cn1 = (T*)h->cpool[h->ccur ^ 1];
    // 1. coarse ghosts, coarse step with the coarse-fine flux records
    hipLaunchKernelGGL(coarse_ghost_kernel<T>, dim3((unsigned)((ncg + 255) / 256)), dim3(256), 0, st, cn, cg.nx,
                       cg.ny, h->bc, M);
    WalkArgs w;
    memset(&w, 0, sizeof(w));
    w.P.g = h->prm.g;
    w.P.gamma = h->prm.gamma;
    w.P.rho = h->prm.rho;
    w.P.K = h->prm.K;
    w.P.u = h->prm.u;
    w.P.v = h->prm.v;
    w.grids = h->cgrid;
    w.items = h->citems;
    w.nitems = h->ncitems;
    w.in = cn;
    w.out = cn1;
    w.nux = dt / h->dx;
    w.nuy = dt / h->dy;
    w.xmap = h->xmap;
    w.ymap = h->ymap;
    w.creg = h->creg;
    w.smax_bits = h->bits;
    w.status = h->status;
    int r = walk(h, w, limiter, true);
    if (r != MC_OK) return r;
    hipLaunchKernelGGL(coarse_ghost_kernel<T>, dim3((unsigned)((ncg + 255) / 256)), dim3(256), 0, st, cn1, cg.nx,
                       cg.ny, h->bc, M);
    if ((r = hip_check(hipGetLastError())) != MC_OK) return r;
    // 2. subcycled patches
    if (h->npatch > 0) {
        const double dtf = dt / h->r, dxf = h->dx / h->r, dyf = h->dy / h->r;
        for (int k = 0; k < h->r; ++k) {
            FillArgs f;
            f.grids = h->grids;
            f.npatch = h->npatch;
            f.fine = h->fpool[h->fcur];
            f.gn = cn;
            f.gn1 = cn1;
            f.owner = h->owner;
            f.nxc = h->nxc;
            f.nyc = h->nyc;
            f.r = h->r;
            f.bc = h->bc;
            f.meqn = M;
            f.alpha = (double)k / (double)h->r;
            hipLaunchKernelGGL(fine_ghost_kernel<T>, dim3((unsigned)((h->max_ghost + 255) / 256), h->npatch),
                               dim3(256), 0, st, f);
            if ((r = hip_check(hipGetLastError())) != MC_OK) return r;
            WalkArgs v = w;
            v.grids = h->grids;
            v.items = h->fitems;
            v.nitems = h->nfitems;
            v.in = h->fpool[h->fcur];
            v.out = h->fpool[h->fcur ^ 1];
            v.nux = dtf / dxf;
            v.nuy = dtf / dyf;
            v.xmap = nullptr;
            v.ymap = nullptr;
            v.freg = h->freg;
            v.accum = k > 0;
            v.smax_bits = h->bits + 2;
            if ((r = walk(h, v, limiter, false)) != MC_OK) return r;
            h->fcur ^= 1;
        }
    }
    // 3. fix-up at coarse-fine edges, 4. averaging down
    FixArgs x;
    x.cells = h->rcells;
    x.ncells = h->nrcells;
    x.grids = h->grids;
    x.npatch = h->npatch;
    x.coarse = cn1;
    x.fine = h->fpool[h->fcur];
    x.creg = h->creg;
    x.freg = h->freg;
    x.nxc = h->nxc;
    x.nyc = h->nyc;
    x.r = h->r;
    x.meqn = M;
    x.nux = dt / h->dx;
    x.nuy = dt / h->dy;
    if (h->nrcells > 0)
        hipLaunchKernelGGL(reflux_kernel<T>, dim3((h->nrcells + 255) / 256), dim3(256), 0, st, x);
    if (h->npatch > 0)
        hipLaunchKernelGGL(average_kernel<T>, dim3((h->max_cov + 255) / 256, h->npatch), dim3(256), 0, st, x);
    AFinArgs fa;
    fa.bits = h->bits;
    fa.cfl = cfl_out;
    fa.dx = h->dx;
    fa.dy = h->dy;
    fa.r = h->r;
    fa.dt = dt;
    hipLaunchKernelGGL(amr_finish_kernel, dim3(1), dim3(64), 0, st, fa);
    if ((r = hip_check(hipGetLastError())) != MC_OK) return r;
    h->ccur ^= 1;
    return MC_OK;
}

// neighbour of coarse cell (i, j) under the boundary rule, false when it is
// outside the domain (extrapolation)
bool nb_cell(const mc_amr* h, int i, int j, int di, int dj, int& a, int& b)
{
    a = i + di;
    b = j + dj;
    if (h->bc == MC_BC_PERIODIC) {
        a = (a % h->nxc + h->nxc) % h->nxc;
        b = (b % h->nyc + h->nyc) % h->nyc;
        return true;
    }
    return a >= 0 && a < h->nxc && b >= 0 && b < h->nyc;
}

}  // namespace

extern "C" {

int mc_amr_create(mc_amr** out, mc_ctx* ctx, int32_t ratio, int32_t npatch, const mc_amr_box* boxes,
                  int32_t bc)
{
    if (!out || !ctx || ratio < 1 || ratio > 16 || npatch < 0 || (npatch > 0 && !boxes)) return MC_EINVAL;
    if (bc != MC_BC_PERIODIC && bc != MC_BC_EXTRAP) return MC_EINVAL;
    *out = nullptr;
    int solver, dtype, cus;
    mc_params prm;
    void* stream;
    mc__ctx_info(ctx, &solver, &dtype, &prm, &cus, &stream);
    if (amr_meqn(solver) == 0) return MC_EUNSUPPORTED;
    int nx, ny;
    double dx, dy;
    unsigned int* status;
    mc__ctx_grid(ctx, &nx, &ny, &dx, &dy, &status);
    // footprints: inside the grid, no overlap
    std::vector<int32_t> own((size_t)nx * ny, -1);
    for (int p = 0; p < npatch; ++p) {
        const mc_amr_box& b = boxes[p];
        if (b.cw < 1 || b.ch < 1 || b.ci0 < 0 || b.cj0 < 0 || b.ci0 + b.cw > nx || b.cj0 + b.ch > ny)
            return MC_EINVAL;
        if ((int64_t)b.cw * ratio > (1 << 20) || (int64_t)b.ch * ratio > (1 << 20)) return MC_EINVAL;
        for (int j = b.cj0; j < b.cj0 + b.ch; ++j)
            for (int i = b.ci0; i < b.ci0 + b.cw; ++i) {
                if (own[(size_t)j * nx + i] >= 0) return MC_EINVAL;
                own[(size_t)j * nx + i] = p;
            }
    }
    mc_amr* h = new mc_amr();
    h->ctx = ctx;
    h->solver = solver;
    h->dtype = dtype;
    h->esz = dtype == MC_F64 ? 8 : 4;
    h->meqn = amr_meqn(solver);
    h->prm = prm;
    h->cus = cus;
    h->stream = (hipStream_t)stream;
    h->nxc = nx;
    h->nyc = ny;
    h->r = ratio;
    h->bc = bc;
    h->npatch = npatch;
    h->dx = dx;
    h->dy = dy;
    h->status = status;
    h->boxes.assign(boxes, boxes + npatch);
    const int M = h->meqn;
    // descriptors and item lists
    const int64_t W = dtype == MC_F64 ? resident_waves_of<double>(solver, cus) : resident_waves_of<float>(solver, cus);
    std::vector<std::pair<int, int>> fdims;
    for (int p = 0; p < npatch; ++p) fdims.push_back({boxes[p].cw * ratio, boxes[p].ch * ratio});
    const int crows = choose_rows({{nx, ny}}, W);
    const int frows = npatch > 0 ? choose_rows(fdims, W) : 8;
    GridDev cgd;
    memset(&cgd, 0, sizeof(cgd));
    cgd.nx = nx;
    cgd.ny = ny;
    cgd.rows = std::min(crows, ny);
    cgd.nstrips = (nx + TXO - 1) / TXO;
    h->hgrids.push_back(cgd);
    std::vector<ItemDev> ci, fi;
    items_for(cgd, 0, ci);
    std::vector<GridDev> pg;
    int64_t off = 0, roff = 0;
    for (int p = 0; p < npatch; ++p) {
        GridDev g;
        memset(&g, 0, sizeof(g));
        g.nx = boxes[p].cw * ratio;
        g.ny = boxes[p].ch * ratio;
        g.off = off;
        g.rows = std::min(frows, g.ny);
        g.nstrips = (g.nx + TXO - 1) / TXO;
        g.ci0 = boxes[p].ci0;
        g.cj0 = boxes[p].cj0;
        g.roff = roff;
        off += (int64_t)M * (g.nx + 4) * (g.ny + 4);
        roff += (int64_t)M * (2 * g.nx + 2 * g.ny);
        pg.push_back(g);
        h->hgrids.push_back(g);
        items_for(g, p, fi);
        h->max_ghost = std::max<int64_t>(h->max_ghost, (int64_t)(g.nx + 4) * 4 + (int64_t)g.ny * 4);
        h->max_cov = std::max(h->max_cov, boxes[p].cw * boxes[p].ch);
    }
    h->fpool_elems = off;
    h->freg_elems = roff;
    h->ncitems = (int)ci.size();
    h->nfitems = (int)fi.size();
    // coarse-fine edges: maps for the coarse walker and the reflux cell list
    std::vector<int32_t> xmap((size_t)ny * (nx + 1), -1), ymap((size_t)(ny + 1) * nx, -1);
    std::vector<RefluxCell> rc;
    int64_t slot = 0;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            if (own[(size_t)j * nx + i] >= 0) continue;
            RefluxCell c;
            c.i = i;
            c.j = j;
            bool any = false;
            const int dirs[4][2] = {{-1, 0}, {1, 0}, {0, -1}, {0, 1}};
            for (int d = 0; d < 4; ++d) {
                c.slot[d] = -1;
                c.fbase[d] = 0;
                int a, b;
                if (!nb_cell(h, i, j, dirs[d][0], dirs[d][1], a, b)) continue;
                const int p = own[(size_t)b * nx + a];
                if (p < 0) continue;
                const GridDev& g = pg[p];
                int64_t side_base, pos;
                if (d == 0) { side_base = g.ny; pos = b - boxes[p].cj0; }            // patch's right side
                else if (d == 1) { side_base = 0; pos = b - boxes[p].cj0; }          // left side
                else if (d == 2) { side_base = 2 * g.ny + g.nx; pos = a - boxes[p].ci0; }  // top side
                else { side_base = 2 * g.ny; pos = a - boxes[p].ci0; }               // bottom side
                c.slot[d] = (int32_t)slot;
                c.fbase[d] = g.roff + (side_base + pos * ratio) * M;
                // the coarse edge, as the uncovered cell sees it
                if (d == 0) xmap[(size_t)j * (nx + 1) + i] = (int32_t)(slot * 2 + 1);
                else if (d == 1) xmap[(size_t)j * (nx + 1) + i + 1] = (int32_t)(slot * 2);
                else if (d == 2) ymap[(size_t)j * nx + i] = (int32_t)(slot * 2 + 1);
                else ymap[(size_t)(j + 1) * nx + i] = (int32_t)(slot * 2);
                ++slot;
                any = true;
            }
            if (any) rc.push_back(c);
        }
    h->nslots = slot;
    h->nrcells = (int)rc.size();
    // device buffers
    const int64_t cpl = (int64_t)M * (nx + 4) * (ny + 4);
    int r = MC_OK;
    r = r ? r : amr_alloc(h, &h->cpool[0], cpl * h->esz);
    r = r ? r : amr_alloc(h, &h->cpool[1], cpl * h->esz);
    r = r ? r : amr_alloc(h, &h->fpool[0], h->fpool_elems * h->esz);
    r = r ? r : amr_alloc(h, &h->fpool[1], h->fpool_elems * h->esz);
    r = r ? r : amr_alloc(h, (void**)&h->owner, own.size() * sizeof(int32_t));
    r = r ? r : amr_alloc(h, (void**)&h->xmap, xmap.size() * sizeof(int32_t));
    r = r ? r : amr_alloc(h, (void**)&h->ymap, ymap.size() * sizeof(int32_t));
    r = r ? r : amr_alloc(h, &h->creg, (size_t)(h->nslots * M) * h->esz);
    r = r ? r : amr_alloc(h, &h->freg, (size_t)h->freg_elems * h->esz);
    r = r ? r : amr_alloc(h, (void**)&h->rcells, rc.size() * sizeof(RefluxCell));
    r = r ? r : amr_alloc(h, (void**)&h->grids, pg.size() * sizeof(GridDev));
    r = r ? r : amr_alloc(h, (void**)&h->cgrid, sizeof(GridDev));
    r = r ? r : amr_alloc(h, (void**)&h->citems, ci.size() * sizeof(ItemDev));
    r = r ? r : amr_alloc(h, (void**)&h->fitems, fi.size() * sizeof(ItemDev));
    r = r ? r : amr_alloc(h, (void**)&h->bits, 4 * sizeof(unsigned long long));
    auto up = [&](void* d, const void* s, size_t n) {
        if (r == MC_OK && n > 0) r = hip_check(hipMemcpy(d, s, n, hipMemcpyHostToDevice));
    };
    up(h->owner, own.data(), own.size() * sizeof(int32_t));
    up(h->xmap, xmap.data(), xmap.size() * sizeof(int32_t));
    up(h->ymap, ymap.data(), ymap.size() * sizeof(int32_t));
    up(h->rcells, rc.data(), rc.size() * sizeof(RefluxCell));
    up(h->grids, pg.data(), pg.size() * sizeof(GridDev));
    up(h->cgrid, &cgd, sizeof(GridDev));
    up(h->citems, ci.data(), ci.size() * sizeof(ItemDev));
    up(h->fitems, fi.data(), fi.size() * sizeof(ItemDev));
    if (r == MC_OK) r = hip_check(hipMemset(h->bits, 0, 4 * sizeof(unsigned long long)));
    if (r == MC_OK) r = hip_check(hipMemset(h->cpool[0], 0, cpl * h->esz));
    if (r == MC_OK) r = hip_check(hipMemset(h->cpool[1], 0, cpl * h->esz));
    if (r == MC_OK && h->fpool_elems) r = hip_check(hipMemset(h->fpool[0], 0, h->fpool_elems * h->esz));
    if (r == MC_OK && h->fpool_elems) r = hip_check(hipMemset(h->fpool[1], 0, h->fpool_elems * h->esz));
    if (r != MC_OK) {
        mc_amr_destroy(h);
        return r;
    }
    *out = h;
    return MC_OK;
}

void mc_amr_destroy(mc_amr* h)
{
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    for (void* p : h->owned) (void)hipFree(p);
    delete h;
}

int mc_amr_dims(const mc_amr* h, int32_t which, int32_t* nx, int32_t* ny)
{
    if (!h || !nx || !ny || which < -1 || which >= h->npatch) return MC_EINVAL;
    const GridDev& g = h->hgrids[which + 1];
    *nx = g.nx;
    *ny = g.ny;
    return MC_OK;
}

// copies between a grid's interior [meqn][ny][nx] and its padded storage
static int copy_grid(mc_amr* h, int32_t which, void* q, bool to_amr)
{
    if (!h || !q || which < -1 || which >= h->npatch) return MC_EINVAL;
    const GridDev& g = h->hgrids[which + 1];
    char* base = (char*)(which < 0 ? h->cpool[h->ccur] : h->fpool[h->fcur]) + (which < 0 ? 0 : g.off * h->esz);
    const size_t pitch = (size_t)(g.nx + 4) * h->esz, row = (size_t)g.nx * h->esz;
    for (int m = 0; m < h->meqn; ++m) {
        char* pad = base + ((size_t)m * (g.ny + 4) * (g.nx + 4) + 2 * (g.nx + 4) + 2) * h->esz;
        char* dense = (char*)q + (size_t)m * g.ny * row;
        const hipError_t e = to_amr ? hipMemcpy2DAsync(pad, pitch, dense, row, row, g.ny, hipMemcpyDeviceToDevice,
                                                       h->stream)
                                    : hipMemcpy2DAsync(dense, row, pad, pitch, row, g.ny, hipMemcpyDeviceToDevice,
                                                       h->stream);
        if (hip_check(e) != MC_OK) return MC_EHIP;
    }
    return MC_OK;
}

int mc_amr_set(mc_amr* h, int32_t which, const void* q) { return copy_grid(h, which, (void*)q, true); }
int mc_amr_get(mc_amr* h, int32_t which, void* q) { return copy_grid(h, which, q, false); }

int mc_amr_step(mc_amr* h, double dt, int32_t limiter, mc_cfl* cfl_out)
{
    if (!h || !(dt >= 0.0) || limiter < MC_LIM_NONE || limiter > MC_LIM_FIRST_ORDER) return MC_EINVAL;
    return h->dtype == MC_F64 ? step_t<double>(h, dt, limiter, cfl_out) : step_t<float>(h, dt, limiter, cfl_out);
}

}  // extern "C"
