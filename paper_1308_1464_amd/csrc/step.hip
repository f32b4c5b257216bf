// step.hip -- gfx950 kernels of the 2D wave-propagation step and the C ABI.
//
// Kernels
//   rp2_kernel          one thread per edge; the method's per-edge work
//                       arrays (waves, speeds, fluctuations) written as SoA
//                       (paper, section 2)
//   step_kernel         the fused dimensionally split step (x-sweep, then
//                       y-sweep of its result; limiter, correction flux,
//                       update and CFL reduction fused; LeVeque 2002 ch. 6
//                       and ch. 19); with STRANG, the Strang-split step
//                       x(dt/2) y(dt) x(dt/2) in the same single pass
//   max_speed_kernel    dt_0 pre-pass
//
// The library is built with -ffp-contract=off: every multiply-add is an
// explicit fma(), so the unrolled copies of the row body, the row variant
// without row conditions and every tile shape evaluate bitwise the same
// operations.
//
// Layout of the fused step (one wavefront = one work item):
//   A work item is a strip of 60 output columns and R output rows.  Lane k
//   of the wavefront owns grid column i0 - 2 + k (k = 0..63), so lanes
//   2..61 are output columns and lanes 0, 1, 62, 63 hold the two ghost /
//   halo columns on each side.  The wavefront walks the rows j0-2 .. j1+1
//   top to bottom.  For every row it
//     1. loads q^n of its column (coalesced, ghost cells by index mapping,
//        never stored in memory),
//     2. solves the x-edge Riemann problem between its cell and the cell of
//        lane k-1 (cross-lane exchange), limits the waves with the
//        neighbouring edges' waves and forms the x-swept value Q* of its
//        cell -- exactly the x-sweep of that row;
//     3. feeds Q* of the row into a register pipeline that marches down its
//        column: the y-edge between this row and the previous one is
//        solved, the y-edge before it is limited and completed, and the row
//        two above is finished and stored.
//   Rows j0-2, j0-1, j1, j1+1 are x-swept again by the neighbouring items
//   (halo recompute), so no intermediate array ever reaches memory: one
//   read of q^n and one write of q^{n+1} per cell.  Re-applying the
//   boundary rule before the y-sweep is the same index mapping applied to
//   the row index.
//   With STRANG the halo is 4 lanes per side (56 output columns): each row
//   that the y pipeline finishes takes its closing x half-sweep at once,
//   which needs two more columns of the intermediate state on each side.
//   The rows of an item's interior ([j0 + 2, j1)) run a variant of the row
//   body without row conditions; the walkers with little arithmetic per
//   cell keep several rows in flight and store through buffer stores, so
//   a group of their rows is one block.  Rows per item come from the
//   occupancy rule or from mc_tune_rows, which times them on the grid.
//   The CFL reduction takes the wavefront maximum of |s| per direction,
//   one atomic per workgroup, and the last workgroup to finish turns the
//   maxima into smax = max(max|s_x|/dx, max|s_y|/dy), cfl = dt * smax and,
//   with a device clock, applies the time-step rule.
#include <hip/hip_runtime.h>

#include <limits.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <tuple>
#include <vector>

#include "../../include/manyclaw.h"
#include "common.hpp"

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

namespace mc {

constexpr int BLOCK = 256;     // 4 independent wavefronts per workgroup
// word 3 of a buffer resource for untyped (raw) access on this GPU family:
// a non-zero data format (32 bit), no swizzle, no index or thread-id adds
constexpr int BUF_WORD3 = 0x00020000;

// scratch shared by the kernels of one context (device memory)
struct Scratch {
    unsigned long long smax_bits[2];  // x and y max |s| as IEEE bits (values >= 0)
    unsigned int counter;             // workgroups finished in the current launch
    unsigned int status;              // OR of ST_* bits
    unsigned int pad[4];
};

struct DevClock {  // same layout as mc_clock
    double t, dt, cfl, smax;
    int32_t cur, n_acc, n_rej, status;
    double cfl_target, cfl_max;
    int32_t rej_run, reserved;
};
static_assert(sizeof(DevClock) == sizeof(mc_clock), "clock layout");

struct StepArgs {
    void* buf[2];          // ping-pong buffers
    const void* aux;
    DevClock* clk;         // device clock or null
    mc_cfl* cfl_out;       // or null
    Scratch* scr;
    DevParams P;
    double cfl_target, cfl_max;  // copied into the clock by the init pass
    double dt_host;        // used when clk is null
    int src_host;          // used when clk is null
    int nx, ny, bc, lim;
    double dx, dy;
    int rows;              // rows per work item
    int nstrips, nitems;
    int init_only;         // clock-init mode of the max-speed kernel
};

// last workgroup of a launch: fold the maxima into smax/cfl, apply the
// time-step rule to the clock, and reset the scratch for the next launch
__device__ void finish_launch(const StepArgs& a, double smx, double smy, unsigned st,
                              bool is_step, double dt)
{
    __shared__ unsigned int s_last;
    __shared__ double s_mx[BLOCK / WAVE], s_my[BLOCK / WAVE];
    __shared__ unsigned s_st[BLOCK / WAVE];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    smx = wave_max(smx);
    smy = wave_max(smy);
    // OR of the status bits across the wavefront
    unsigned long long anyst = __ballot(st != 0u);
    unsigned stw = 0u;
    if (anyst) {
        for (int b = 1; b <= 2; b <<= 1)
            if (__ballot((st & (unsigned)b) != 0u)) stw |= (unsigned)b;
    }
    if (lane == 0) { s_mx[wv] = smx; s_my[wv] = smy; s_st[wv] = stw; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double mx = 0.0, my = 0.0;
        unsigned sw = 0u;
        for (int w = 0; w < BLOCK / WAVE; ++w) {
            mx = s_mx[w] > mx ? s_mx[w] : mx;
            my = s_my[w] > my ? s_my[w] : my;
            sw |= s_st[w];
        }
        // Only these atomics carry data between workgroups (the state the
        // next launch reads is ordered by the launch boundary), so no memory
        // fence is needed here, only that this workgroup's maxima are in
        // place before its count: the read-modify-writes return their old
        // values, and waiting for those returns (vmcnt(0)) means they have
        // been performed.  (A device-scope fence would write back and
        // invalidate the L2 cache in every workgroup.)
        const unsigned long long o0 = __hip_atomic_fetch_max(
            &a.scr->smax_bits[0], (unsigned long long)__double_as_longlong(mx), __ATOMIC_RELAXED,
            __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long o1 = __hip_atomic_fetch_max(
            &a.scr->smax_bits[1], (unsigned long long)__double_as_longlong(my), __ATOMIC_RELAXED,
            __HIP_MEMORY_SCOPE_AGENT);
        const unsigned o2 = sw ? __hip_atomic_fetch_or(&a.scr->status, sw, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT) : 0u;
        asm volatile("s_waitcnt vmcnt(0)" : : "v"(o0), "v"(o1), "v"(o2) : "memory");
        const unsigned prev = __hip_atomic_fetch_add(&a.scr->counter, 1u, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        s_last = (prev == gridDim.x - 1) ? 1u : 0u;
    }
    __syncthreads();
    if (s_last && threadIdx.x == 0) {
        __threadfence();
        const double mxs = __longlong_as_double((long long)atomicAdd(&a.scr->smax_bits[0], 0ull));
        const double mys = __longlong_as_double((long long)atomicAdd(&a.scr->smax_bits[1], 0ull));
        const double sx = mxs / a.dx, sy = mys / a.dy;
        const double smax = sx > sy ? sx : sy;
        if (a.cfl_out) {
            a.cfl_out->smax = smax;
            a.cfl_out->cfl = is_step ? dt * smax : 0.0;
        }
        if (a.clk) {
            DevClock* c = a.clk;
            if (is_step) {
                const double cfl = dt * smax;
                c->cfl = cfl;
                c->smax = smax;
                if (cfl <= c->cfl_max) {
                    c->cur = c->cur ^ 1;
                    c->t = c->t + dt;
                    c->n_acc = c->n_acc + 1;
                    c->rej_run = 0;
                } else {
                    c->n_rej = c->n_rej + 1;
                    c->rej_run = c->rej_run + 1;
                    if (c->rej_run > MC_MAX_RETRIES) {  // latched until the clock is re-initialised
                        c->status = c->status | (int32_t)ST_CFL;
                        atomicOr(&a.scr->status, ST_CFL);
                    }
                }
                c->dt = c->cfl_target / smax;
            } else if (a.init_only) {
                c->cfl_target = a.cfl_target;
                c->cfl_max = a.cfl_max;
                c->t = 0.0;
                c->dt = a.cfl_target / smax;
                c->cfl = 0.0;
                c->smax = smax;
                c->cur = 0;
                c->n_acc = 0;
                c->n_rej = 0;
                c->status = 0;
                c->rej_run = 0;
                c->reserved = 0;
            }
        }
        atomicExch(&a.scr->smax_bits[0], 0ull);
        atomicExch(&a.scr->smax_bits[1], 0ull);
        atomicExch(&a.scr->counter, 0u);
    }
}

// Rows of q^n a wavefront keeps in flight ahead of the row it works on.  A
// wavefront walks its rows one after another, so with one row in flight
// each row waits out a full memory latency unless the row's own arithmetic
// covers it: the solvers with little arithmetic per cell (advection,
// acoustics) prefetch four rows in FP32 and eight in FP64 (2-3 % faster at
// 4096^2 than four; in FP32 eight were 1-5 % slower), which their register
// budget allows; the shallow-water and Euler walkers, whose arithmetic
// covers the latency and whose registers set the occupancy, keep one.
template <typename T, template <typename, int> class SOL>
constexpr int prefetch_rows()
{
    return SOL<T, 1>::MWAVES <= 2 ? (sizeof(T) == 8 ? 8 : 4) : 1;
}

// STRANG: the Strang-split step x(dt/2) y(dt) x(dt/2) in one pass (nux is
// then the half step's): each finished row takes its closing x half-sweep
// before it is stored.  That sweep reads the y-swept row two cells beyond
// each output column, so the halo is 4 lanes a side (56 output columns).
template <typename T, template <typename, int> class SOL, int LIM, bool STRANG = false>
struct StripWalker {
    using SX = SOL<T, 1>;
    using SY = SOL<T, 2>;
    static constexpr int M = SX::MEQN, NW = SX::MWAVES, NA = SX::MAUX, NC = SX::NC;
    static constexpr int NE = SX::NE, NX = SX::NX;
    static constexpr int HALO = STRANG ? 4 : 2, OUTW = WAVE - 2 * HALO;
    static constexpr int PF = prefetch_rows<T, SOL>();    // rows in flight
    // rows per iteration of the row loop: a multiple of 2 (the y-pipeline
    // slots alternate) and of PF (each prefetch slot serves every PF-th row)
    static constexpr int UNROLL = PF % 2 == 0 ? PF : 2 * PF;
    // Rows without row conditions let the compiler schedule a group of rows
    // as one block (the light walkers: up to 16 % faster) or with fewer
    // branches (FP32 shallow water, Euler: 1-2 %).  FP64 shallow water
    // measured no faster with the longer code and keeps the plain loop.
    static constexpr bool STEADY_ROWS = !(sizeof(T) == 8 && NW == 3);
    using CX = typename SX::C;
    using EX = typename SX::E;
    using Slot = YSlot<SY, T>;

    const T* __restrict__ q;
    const T* __restrict__ aux;
    T* __restrict__ qo;
    DevParams P;
    int64_t plane;
    int nx, ny, bc;
    int up, dn;         // ds_bpermute addresses of lanes - 1 and + 1
    int im, i;          // mapped and true column of this lane
    int xsrc;           // ds_bpermute address of the lane holding column im (STRANG, extrapolation)
    bool xperm;         // STRANG: some lane of this strip lies outside the grid under extrapolation
    int j0, j1;
    bool outcol, xcount;
    T nux, nuy;
    T nq[PF][M + (NA > 0 ? NA : 0) + 1];  // prefetched rows (a ring, indexed by row mod PF)
    T pend[M];          // right-going contribution of the y-edge above row jj - 1
    T outv[M];          // the row finished last, stored at the start of the next
    int outrow;         // its row (the same for the whole wavefront), or -1
    T smx, smy;         // max |s| over counted x- and y-edges
    unsigned st;

    // values of the lane on the left (xleft) or right (xright)
    template <int N>
    __device__ __forceinline__ void xleft(const T* v, T* o)
    {
#pragma unroll
        for (int k = 0; k < N; ++k) o[k] = from_left(up, v[k]);
    }
    template <int N>
    __device__ __forceinline__ void xright(const T* v, T* o)
    {
#pragma unroll
        for (int k = 0; k < N; ++k) o[k] = from_right(dn, v[k]);
    }

    // The row finished by one call is stored at the start of the next.  With
    // one row in flight this follows a wait for all vector memory operations:
    // the wait then covers the loads prefetched and the stores issued a whole
    // row earlier, instead of stores issued just before it.  With more rows in
    // flight the compiler's own waits cover each prefetched row as it is used.
    // The light walkers (several rows in flight) store through buffer
    // stores over the output row: a lane that owns no output (a halo lane,
    // or no row finished) gives an offset beyond the row and the hardware
    // drops its store, so no branch splits the row body around them.  (The
    // shallow-water and Euler walkers keep the masked stores: without the
    // branch, FP64 shallow water's schedule needs registers beyond three
    // wavefronts per SIMD.)
    __device__ __forceinline__ void flush()
    {
        if constexpr (PF == 1) __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), expcnt and lgkmcnt untouched
        if constexpr (PF > 1) {
            const int r = __builtin_amdgcn_readfirstlane(outrow >= 0 ? outrow : 0);
            const int off = (outrow >= 0 && outcol) ? i * (int)sizeof(T) : INT_MIN;
            T* rowp = uniform_ptr(qo) + (int64_t)r * nx;
#pragma unroll
            for (int m = 0; m < M; ++m) store_row(rowp + m * plane, off, outv[m]);
        } else if (outrow >= 0 && outcol) {
            const int64_t o = (int64_t)outrow * nx + i;
#pragma unroll
            for (int m = 0; m < M; ++m) qo[o + m * plane] = outv[m];
        }
        outrow = -1;
    }
    __device__ __forceinline__ void store_row(T* base, int off, T v)
    {
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(base, 0, nx * (int)sizeof(T), BUF_WORD3);
        if constexpr (sizeof(T) == 8)
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), rs, off, 0, 0);
        else
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rs, off, 0, 0);
    }

    template <int RS>
    __device__ __forceinline__ void fetch(int jj)
    {
        const int jm = row_map(jj, ny, bc);
        const T* rp = q + (int64_t)jm * nx;
#pragma unroll
        for (int m = 0; m < M; ++m) nq[RS][m] = rp[m * plane + im];
        if (NA > 0) {
            const T* ap = aux + (int64_t)jm * nx;
#pragma unroll
            for (int k = 0; k < NA; ++k) nq[RS][M + k] = ap[k * plane + im];
        }
    }

    // STRANG: the closing x half-sweep of the y-swept row jo (ys, its aux
    // a2).  The boundary rule is applied to the intermediate state first: with
    // extrapolation a lane outside the grid takes the value of the edge
    // column it maps to (a lane of this wavefront); periodic halo lanes
    // already hold their mapped columns' values.
    __device__ __forceinline__ void closing_sweep(int jo, T (&ys)[M], const T (&a2)[NA > 0 ? NA : 1])
    {
        if (xperm) {
#pragma unroll
            for (int m = 0; m < M; ++m) ys[m] = xlane(xsrc, ys[m]);
        }
        CX c;
#pragma unroll
        for (int m = 0; m < M; ++m) c.v[m] = ys[m];
#pragma unroll
        for (int k = 0; k < NA; ++k) c.v[NC - NA + k] = a2[k];
        SX::prep(P, c);
        CX l;
        xleft<NC>(c.v, l.v);
        EX e;
        const unsigned sx_st = SX::solve(P, l, c, e);
        EX el;
        xleft<NX>(e.v, el.v);
        T d[NW], dr[NW], trl[NW];  // trl: what the edge on the left takes from this one
        SX::pair(P, e, el, d, trl);
        xright<NW>(trl, dr);
        T lf[M], rg[M], lfr[M];
        edge_terms<SX, LIM>(P, e, d, dr, nux, lf, rg);
        xright<M>(lf, lfr);
        T out[M];
#pragma unroll
        for (int m = 0; m < M; ++m) out[m] = fma(-nux, lfr[m], fma(-nux, rg[m], c.v[m]));
        if (xcount) {
            smx = fmax(smx, SX::smax(P, e));
            st |= sx_st;
        }
        outrow = jo;
#pragma unroll
        for (int m = 0; m < M; ++m) outv[m] = out[m];
    }

    // the first PF rows of the walk into the prefetch ring
    template <int K>
    __device__ __forceinline__ void prologue(int jj, int jend)
    {
        if (jj + K < jend) fetch<K>(jj + K);
        if constexpr (K + 1 < PF) prologue<K + 1>(jj, jend);
    }

    // rows jj + K .. jj + UNROLL - 1 of a group: row jj + K takes prefetch
    // slot K mod PF and the y-pipeline slots in the order of its parity.
    // STEADY: every row of the group lies in [j0 + 2, j1), where every
    // row-dependent condition of row() holds.
    template <int K, bool STEADY = false>
    __device__ __forceinline__ void group(int jj, Slot& s0, Slot& s1)
    {
        if constexpr (K % 2 == 0) row<K % PF, STEADY>(jj + K, s0, s1);
        else row<K % PF, STEADY>(jj + K, s1, s0);
        // A STEADY group is one block; left alone, the scheduler starts all
        // its rows' x-sweeps first, which needs every row's data at the top
        // of the group and issues the refills at its end.  Keeping the rows
        // in order keeps each refill a group ahead of its use.
        if constexpr (STEADY) __builtin_amdgcn_sched_barrier(0);
        if constexpr (K + 1 < UNROLL) group<K + 1, STEADY>(jj, s0, s1);
    }

    // the rows left after the whole groups (fewer than UNROLL), in the same
    // slot order
    template <int K>
    __device__ __forceinline__ void tail(int jj, int jend, Slot& s0, Slot& s1)
    {
        if constexpr (K + 1 < UNROLL) {
            if (jj + K < jend) {
                if constexpr (K % 2 == 0) row<K % PF>(jj + K, s0, s1);
                else row<K % PF>(jj + K, s1, s0);
                tail<K + 1>(jj, jend, s0, s1);
            }
        }
    }

    // one row: x-sweep of row jj, then one stage of the y pipeline.  N is
    // the slot of row jj (it held row jj - 2), O the slot of row jj - 1; RS
    // is the prefetch slot holding row jj, refilled with row jj + PF.
    template <int RS, bool STEADY = false>
    __device__ __forceinline__ void row(int jj, Slot& N, Slot& O)
    {
        flush();
        // ---------------- x-sweep of row jj
        CX c;
        T av[NA > 0 ? NA : 1];
#pragma unroll
        for (int m = 0; m < M; ++m) c.v[m] = nq[RS][m];
#pragma unroll
        for (int k = 0; k < NA; ++k) { av[k] = nq[RS][M + k]; c.v[NC - NA + k] = av[k]; }
        // With one row in flight its load is issued as early as possible.
        // With several, the slot is refilled after the last use of the
        // values it held (below): issued here, the new load would need
        // registers of its own while the old values are still in use, and
        // the ring would then be rotated by copies at the loop's back edge,
        // which wait for every load in flight.
        if constexpr (PF == 1) {
            fetch<RS>(min(jj + PF, j1 + 1));
        }
        SX::prep(P, c);
        CX l;
        xleft<NC>(c.v, l.v);
        EX e;
        const unsigned sx_st = SX::solve(P, l, c, e);
        // the limiter's parts from the edge on the left (its record from
        // lane - 1) and from the edge on the right (from lane + 1)
        EX el;
        xleft<NX>(e.v, el.v);
        T d[NW], dr[NW], trl[NW];  // trl: what the edge on the left takes from this one
        SX::pair(P, e, el, d, trl);
        xright<NW>(trl, dr);
        T lf[M], rg[M], lfr[M];
        edge_terms<SX, LIM>(P, e, d, dr, nux, lf, rg);
        xright<M>(lf, lfr);   // A-dQ + F of the edge on the right
        T qs[M];
#pragma unroll
        for (int m = 0; m < M; ++m) qs[m] = fma(-nux, lfr[m], fma(-nux, rg[m], c.v[m]));

        // lane conditions as selects, row conditions known in STEADY rows:
        // no branch splits the row body
        const bool xrow = STEADY || (jj >= j0 && jj < j1);
        smx = (xrow && xcount) ? cfl_max<SX>(smx, SX::smax(P, e)) : smx;
        st |= xcount ? sx_st : 0u;

        // ---------------- y pipeline
        T q2n[M];  // Q* of row jj - 2, the slot's previous content
        T a2n[NA > 0 ? NA : 1];  // its aux values
#pragma unroll
        for (int m = 0; m < M; ++m) { q2n[m] = N.c.v[m]; N.c.v[m] = qs[m]; }
#pragma unroll
        for (int k = 0; k < NA; ++k) { a2n[k] = N.araw[k]; N.araw[k] = av[k]; N.c.v[NC - NA + k] = av[k]; }
        if constexpr (PF > 1) fetch<RS>(min(jj + PF, j1 + 1));
        SY::prep(P, N.c);
        if (STEADY || jj >= j0 - 1) {
            const unsigned sy_st = SY::solve(P, O.c, N.c, N.e);  // edge between jj-1 and jj
            st |= outcol ? sy_st : 0u;
            T tro[NW];  // what the limiter of the edge above (slot O) takes from N.e
            if (STEADY || jj >= j0) SY::pair(P, N.e, O.e, N.d, tro);
            const bool yrow = STEADY || (jj >= j0 && jj <= j1);
            smy = (yrow && outcol) ? cfl_max<SY>(smy, SY::smax(P, N.e)) : smy;
            if (STEADY || jj >= j0 + 1) {
                // complete the edge between rows jj-2 and jj-1 (slot O) and
                // finish row jj-2
                T lf[M], rg[M];
                edge_terms<SY, LIM>(P, O.e, O.d, tro, nuy, lf, rg);
                const int jo = jj - 2;
                if constexpr (!STRANG) {
                    if (STEADY || (jo >= j0 && jo < j1)) {  // wave-uniform; the store keeps the output lanes
                        outrow = jo;
#pragma unroll
                        for (int m = 0; m < M; ++m) outv[m] = fma(-nuy, lf[m], fma(-nuy, pend[m], q2n[m]));
                    }
                } else if (STEADY || (jo >= j0 && jo < j1)) {  // wave-uniform: every lane takes part
                    T ys[M];
#pragma unroll
                    for (int m = 0; m < M; ++m) ys[m] = fma(-nuy, lf[m], fma(-nuy, pend[m], q2n[m]));
                    closing_sweep(jo, ys, a2n);
                }
#pragma unroll
                for (int m = 0; m < M; ++m) pend[m] = rg[m];
            }
        }
    }
};

// wavefronts per SIMD the compiler is asked to fit (its register budget):
// 4 for the FP32 Euler walker, which lands just above the 128 registers
// that allow four; the others as they compile
template <typename T, template <typename, int> class SOL, bool STRANG>
constexpr int step_min_waves()
{
    return (sizeof(T) == 4 && SOL<T, 1>::MWAVES == 4 && !STRANG) ? 4 : 1;
}

template <typename T, template <typename, int> class SOL, int LIM, bool STRANG = false>
__global__ __launch_bounds__(BLOCK, (step_min_waves<T, SOL, STRANG>())) void step_kernel(StepArgs a)
{
    using W = StripWalker<T, SOL, LIM, STRANG>;
    using Slot = typename W::Slot;
    constexpr int M = W::M, NW = W::NW, NC = W::NC;

    const int lane = threadIdx.x & 63;
    int cur;
    double dt;
    if (a.clk) { cur = a.clk->cur; dt = a.clk->dt; }
    else { cur = a.src_host; dt = a.dt_host; }

    W w;
    w.q = (const T*)a.buf[cur];
    w.qo = (T*)a.buf[cur ^ 1];
    w.aux = (const T*)a.aux;
    w.P = a.P;
    w.nx = a.nx; w.ny = a.ny; w.bc = a.bc;
    w.plane = (int64_t)a.nx * a.ny;
    w.up = ((lane + 63) & 63) << 2;
    w.dn = ((lane + 1) & 63) << 2;
    w.nux = T(dt / a.dx);
    w.nuy = T(dt / a.dy);
    w.smx = T(0); w.smy = T(0); w.st = 0u;

    // work item of this wavefront: workgroups are dealt round-robin to the
    // 8 XCDs, so give each XCD a contiguous band of items (shared halo rows
    // and columns stay in that XCD's L2)
    const int per_xcd = gridDim.x >> 3;
    const int b = blockIdx.x;
    const int lb = (b & 7) * per_xcd + (b >> 3);
    const int item = lb * (BLOCK / WAVE) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    if (item < a.nitems) {
        const int strip = item % a.nstrips;
        const int chunk = item / a.nstrips;
        w.i = strip * W::OUTW - W::HALO + lane;
        w.im = bc_map(w.i, a.nx, a.bc);
        w.xsrc = (lane + (w.im - w.i)) << 2;
        // the same for every lane of the wavefront: its first and last columns
        const int first = strip * W::OUTW - W::HALO;
        w.xperm = w.bc != 0 && (first < 0 || first + (WAVE - 1) >= w.nx);
        w.j0 = chunk * a.rows;
        w.j1 = min(w.j0 + a.rows, a.ny);
        w.outcol = lane >= W::HALO && lane < W::HALO + W::OUTW && w.i < a.nx;
        w.xcount = lane >= W::HALO && lane <= W::HALO + W::OUTW && w.i <= a.nx;
#pragma unroll
        for (int m = 0; m < M; ++m) w.pend[m] = T(0);
        Slot s0, s1;
#pragma unroll
        for (int k = 0; k < NC; ++k) { s0.c.v[k] = T(0); s1.c.v[k] = T(0); }
#pragma unroll
        for (int k = 0; k < W::NE; ++k) { s0.e.v[k] = T(0); s1.e.v[k] = T(0); }
#pragma unroll
        for (int p = 0; p < NW; ++p) s0.d[p] = s1.d[p] = T(0);
#pragma unroll
        for (int k = 0; k < (W::NA > 0 ? W::NA : 1); ++k) s0.araw[k] = s1.araw[k] = T(0);

        w.outrow = -1;
#pragma unroll
        for (int m = 0; m < M; ++m) w.outv[m] = T(0);
        int jj = w.j0 - 2;
        const int jend = w.j1 + 2;
        w.template prologue<0>(jj, jend);
        // rows in groups of UNROLL (y-pipeline slots alternate, prefetch
        // slots cycle): the four rows that fill the pipeline (every item has
        // them), the rows of [j0 + 2, j1) without row conditions, the rest
        // with them, then the remaining rows with the same slot order
        if constexpr (W::STEADY_ROWS) {
            // the groups that hold the four pipeline-filling rows
#pragma unroll
            for (int k = 0; k < (4 + W::UNROLL - 1) / W::UNROLL; ++k, jj += W::UNROLL) w.template group<0>(jj, s0, s1);
            for (; jj + W::UNROLL - 1 < w.j1; jj += W::UNROLL) w.template group<0, true>(jj, s0, s1);
        }
        for (; jj + W::UNROLL - 1 < jend; jj += W::UNROLL) w.template group<0>(jj, s0, s1);
        w.template tail<0>(jj, jend, s0, s1);
        w.flush();
    }
    finish_launch(a, (double)w.smx, (double)w.smy, w.st, true, dt);
}

// ------------------------------------------------------- max-speed pre-pass
// one thread per (i, j) with 0 <= i <= nx, 0 <= j <= ny: the x-edge e_i of
// row j (j < ny) and the y-edge f_j of column i (i < nx)
template <typename T, template <typename, int> class SOL>
__global__ __launch_bounds__(BLOCK) void max_speed_kernel(StepArgs a)
{
    using SX = SOL<T, 1>;
    using SY = SOL<T, 2>;
    constexpr int M = SX::MEQN, NW = SX::MWAVES, NA = SX::MAUX, NC = SX::NC;
    const T* q = (const T*)a.buf[0];
    const T* aux = (const T*)a.aux;
    const int nx = a.nx, ny = a.ny, bc = a.bc;
    const int64_t plane = (int64_t)nx * ny;
    const int64_t n = (int64_t)(nx + 1) * (ny + 1);
    double smx = 0.0, smy = 0.0;
    unsigned st = 0u;
    for (int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x; t < n; t += (int64_t)gridDim.x * BLOCK) {
        const int i = (int)(t % (nx + 1)), j = (int)(t / (nx + 1));
        if (j < ny) {
            typename SX::C L, R;
            const int64_t ol = (int64_t)j * nx + bc_map(i - 1, nx, bc);
            const int64_t orr = (int64_t)j * nx + bc_map(i, nx, bc);
#pragma unroll
            for (int m = 0; m < M; ++m) { L.v[m] = q[m * plane + ol]; R.v[m] = q[m * plane + orr]; }
#pragma unroll
            for (int k = 0; k < NA; ++k) { L.v[NC - NA + k] = aux[k * plane + ol]; R.v[NC - NA + k] = aux[k * plane + orr]; }
            SX::prep(a.P, L);
            SX::prep(a.P, R);
            typename SX::E e;
            st |= SX::solve(a.P, L, R, e);
            smx = fmax(smx, (double)SX::smax(a.P, e));
        }
        if (i < nx) {
            typename SY::C L, R;
            const int64_t ol = (int64_t)bc_map(j - 1, ny, bc) * nx + i;
            const int64_t orr = (int64_t)bc_map(j, ny, bc) * nx + i;
#pragma unroll
            for (int m = 0; m < M; ++m) { L.v[m] = q[m * plane + ol]; R.v[m] = q[m * plane + orr]; }
#pragma unroll
            for (int k = 0; k < NA; ++k) { L.v[NC - NA + k] = aux[k * plane + ol]; R.v[NC - NA + k] = aux[k * plane + orr]; }
            SY::prep(a.P, L);
            SY::prep(a.P, R);
            typename SY::E e;
            st |= SY::solve(a.P, L, R, e);
            smy = fmax(smy, (double)SY::smax(a.P, e));
        }
    }
    finish_launch(a, smx, smy, st, false, 0.0);
}

// ------------------------------------------------------------- rp2 batch
struct Rp2Args {
    const void* ql;
    const void* qr;
    const void* aux;
    void* waves;
    void* speeds;
    void* amdq;
    void* apdq;
    Scratch* scr;
    DevParams P;
    int64_t n;
};

template <typename T, template <typename, int> class SOL, int IXY>
__global__ __launch_bounds__(BLOCK) void rp2_kernel(Rp2Args a)
{
    using S = SOL<T, IXY>;
    constexpr int M = S::MEQN, NW = S::MWAVES, NA = S::MAUX, NC = S::NC;
    const T* ql = (const T*)a.ql;
    const T* qr = (const T*)a.qr;
    const T* aux = (const T*)a.aux;
    T* W = (T*)a.waves;
    T* s = (T*)a.speeds;
    T* am = (T*)a.amdq;
    T* ap = (T*)a.apdq;
    const int64_t n = a.n;
    unsigned st = 0u;
    for (int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x; k < n; k += (int64_t)gridDim.x * BLOCK) {
        typename S::C L, R;
#pragma unroll
        for (int m = 0; m < M; ++m) { L.v[m] = ql[m * n + k]; R.v[m] = qr[m * n + k]; }
#pragma unroll
        for (int j = 0; j < NA; ++j) { L.v[NC - NA + j] = aux[j * n + k]; R.v[NC - NA + j] = aux[(NA + j) * n + k]; }
        S::prep(a.P, L);
        S::prep(a.P, R);
        typename S::E e;
        st |= S::solve(a.P, L, R, e);
        T Wc[NW][M], em[M], ep[M];
        S::waves(a.P, e, Wc);
        S::fluct(a.P, e, em, ep);
#pragma unroll
        for (int p = 0; p < NW; ++p) {
            s[p * n + k] = S::speed(a.P, e, p);
#pragma unroll
            for (int m = 0; m < M; ++m) W[((int64_t)p * M + m) * n + k] = Wc[p][m];
        }
#pragma unroll
        for (int m = 0; m < M; ++m) { am[m * n + k] = em[m]; ap[m * n + k] = ep[m]; }
    }
    if (__ballot(st != 0u)) {
        unsigned stw = 0u;
        for (int b = 1; b <= 2; b <<= 1)
            if (__ballot((st & (unsigned)b) != 0u)) stw |= (unsigned)b;
        if ((threadIdx.x & 63) == 0) atomicOr(&a.scr->status, stw);
    }
}

// ---------------------------------------------------------- copy probe
// 16-byte copy with CP_U loads in flight per thread (each wavefront moves
// CP_U x 1 KiB per pass), non-temporal loads and stores (the data is not
// reused), grid-stride over passes: the achievable HBM ceiling and the
// calibration of the memory counters (bytes read = bytes written = n)
constexpr int CP_U = 4;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(BLOCK) void copy_probe_kernel(const u32x4* __restrict__ src,
                                                           u32x4* __restrict__ dst, int64_t n16)
{
    const int64_t step = (int64_t)gridDim.x * BLOCK * CP_U;
    for (int64_t b = (int64_t)blockIdx.x * BLOCK * CP_U + threadIdx.x; b < n16; b += step) {
        u32x4 v[CP_U];
#pragma unroll
        for (int u = 0; u < CP_U; ++u) {
            const int64_t k = b + (int64_t)u * BLOCK;
            if (k < n16) v[u] = __builtin_nontemporal_load(&src[k]);
        }
#pragma unroll
        for (int u = 0; u < CP_U; ++u) {
            const int64_t k = b + (int64_t)u * BLOCK;
            if (k < n16) __builtin_nontemporal_store(v[u], &dst[k]);
        }
    }
}

}  // namespace mc

// =================================================================== host
using namespace mc;

struct GraphKey {
    void* q0; void* q1; const void* aux; void* clk; int n, lim, bc;
    bool operator<(const GraphKey& o) const
    {
        return std::tie(q0, q1, aux, clk, n, lim, bc) < std::tie(o.q0, o.q1, o.aux, o.clk, o.n, o.lim, o.bc);
    }
};

struct mc_ctx {
    int solver, dtype;
    mc_params params;
    int nx, ny;
    double dx, dy;
    hipStream_t stream;
    hipStream_t cap_stream;  // private stream used only to record graphs
    Scratch* scr;
    int rows;
    int cus;
    std::map<GraphKey, hipGraphExec_t> graphs;
};

static bool is_surrogate(int solver) { return solver == MC_SW_SURROGATE || solver == MC_EULER_SURROGATE; }

static int solver_dims(int solver, int* m, int* w, int* a)
{
    switch (solver) {
    case MC_ADVECTION: *m = 1; *w = 1; *a = 0; return 0;
    case MC_ACOUSTICS: *m = 3; *w = 2; *a = 0; return 0;
    case MC_ACOUSTICS_VC: *m = 3; *w = 2; *a = 2; return 0;
    case MC_SW_ROE: *m = 3; *w = 3; *a = 0; return 0;
    case MC_EULER_ROE: *m = 4; *w = 4; *a = 0; return 0;
    case MC_SW_HLLE: *m = 3; *w = 3; *a = 0; return 0;
    case MC_SW_SURROGATE: *m = 3; *w = 3; *a = 0; return 0;
    case MC_EULER_SURROGATE: *m = 4; *w = 4; *a = 0; return 0;
    default: return -1;
    }
}

static DevParams dev_params(const mc_params& p)
{
    DevParams d;
    d.g = p.g; d.gamma = p.gamma; d.rho = p.rho; d.K = p.K; d.u = p.u; d.v = p.v;
    return d;
}

static int hip_ok(hipError_t e)
{
    if (e != hipSuccess) {
        fprintf(stderr, "manyclaw: HIP error %s\n", hipGetErrorString(e));
        return MC_EHIP;
    }
    return MC_OK;
}

// kernel dispatch by (solver, dtype)
template <template <typename> class Launch, typename... A>
static int dispatch(int solver, int dtype, A&&... args)
{
    // Launch<T>::template run<SOL>(args...)
    if (dtype == MC_F64) {
        switch (solver) {
        case MC_ADVECTION: return Launch<double>::template run<Advection>(args...);
        case MC_ACOUSTICS: return Launch<double>::template run<Acoustics>(args...);
        case MC_ACOUSTICS_VC: return Launch<double>::template run<AcousticsVC>(args...);
        case MC_SW_ROE: return Launch<double>::template run<SwRoe>(args...);
        case MC_EULER_ROE: return Launch<double>::template run<EulerRoeK>(args...);
        case MC_SW_HLLE: return Launch<double>::template run<SwHlle>(args...);
        default: return MC_EUNSUPPORTED;
        }
    } else {
        switch (solver) {
        case MC_ADVECTION: return Launch<float>::template run<Advection>(args...);
        case MC_ACOUSTICS: return Launch<float>::template run<Acoustics>(args...);
        case MC_ACOUSTICS_VC: return Launch<float>::template run<AcousticsVC>(args...);
        case MC_SW_ROE: return Launch<float>::template run<SwRoe>(args...);
        case MC_EULER_ROE: return Launch<float>::template run<EulerRoeK>(args...);
        case MC_SW_HLLE: return Launch<float>::template run<SwHlle>(args...);
        default: return MC_EUNSUPPORTED;
        }
    }
}

// rows per work item: with W wavefronts resident at once (occupancy of the
// kernel x CUs), a launch takes ceil(items / W) rounds of (R + 4) rows each;
// pick the R with the fewest serial rows (larger R on ties), at least rmin
static int auto_rows(int nx, int ny, int waves_resident, int outw = TXO, int rmin = 8)
{
    const int nstrips = (nx + outw - 1) / outw;
    int best = 64;
    long best_cost = -1;
    for (int R = rmin; R <= 1024; ++R) {
        const int nch = (ny + R - 1) / R;
        if (R > ny && R != rmin) break;
        const long items = (long)nstrips * nch;
        const long rounds = (items + waves_resident - 1) / waves_resident;
        const long cost = rounds * (long)(std::min(R, ny) + 4);
        if (best_cost < 0 || cost < best_cost || (cost == best_cost && R > best)) {
            best_cost = cost;
            best = R;
        }
    }
    return best;
}

template <typename T, bool STRANG>
struct StepLaunchT {
    template <template <typename, int> class SOL, int LIM>
    static int go(StepArgs a, int cus, hipStream_t s)
    {
        auto kfn = step_kernel<T, SOL, LIM, STRANG>;
        if (a.rows <= 0) {
            // resident workgroups per CU for this kernel (thread-safe one-time query)
            static const int occ = [kfn]() {
                int nb = 0;
                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(kfn),
                                                                 BLOCK, 0) != hipSuccess || nb < 1)
                    nb = 1;
                return nb;
            }();
            // A one-field walker does so little per row that below about 32
            // rows an item's fixed part (filling the prefetch ring, the four
            // halo rows, the epilogue) outweighs what more wavefronts buy:
            // on the 2048^2 advection step, 56 us at R = 9 against 42 us at
            // R = 32.  The other walkers are best at the occupancy-filling R.
            constexpr int RMIN = SOL<T, 1>::MEQN == 1 ? 32 : 8;
            a.rows = auto_rows(a.nx, a.ny, occ * cus * (BLOCK / WAVE), StripWalker<T, SOL, LIM, STRANG>::OUTW,
                               RMIN);
        }
        constexpr int OUTW = StripWalker<T, SOL, LIM, STRANG>::OUTW;
        a.nstrips = (a.nx + OUTW - 1) / OUTW;
        a.nitems = a.nstrips * ((a.ny + a.rows - 1) / a.rows);
        int nblk = (a.nitems + BLOCK / WAVE - 1) / (BLOCK / WAVE);
        nblk = (nblk + 7) / 8 * 8;  // whole XCD bands
        hipLaunchKernelGGL(kfn, dim3(nblk), dim3(BLOCK), 0, s, a);
        return hip_ok(hipGetLastError());
    }
    template <template <typename, int> class SOL>
    static int run(const StepArgs& a, int cus, hipStream_t s)
    {
        switch (a.lim) {
        case LIM_NONE: return go<SOL, LIM_NONE>(a, cus, s);
        case LIM_MINMOD: return go<SOL, LIM_MINMOD>(a, cus, s);
        case LIM_SUPERBEE: return go<SOL, LIM_SUPERBEE>(a, cus, s);
        case LIM_VANLEER: return go<SOL, LIM_VANLEER>(a, cus, s);
        case LIM_MC: return go<SOL, LIM_MC>(a, cus, s);
        case LIM_FIRST_ORDER: return go<SOL, LIM_FIRST_ORDER>(a, cus, s);
        default: return MC_EINVAL;
        }
    }
};

template <typename T> using StepLaunch = StepLaunchT<T, false>;
template <typename T> using StrangLaunch = StepLaunchT<T, true>;

template <typename T>
struct SpeedLaunch {
    template <template <typename, int> class SOL>
    static int run(const StepArgs& a, int nblk, hipStream_t s)
    {
        hipLaunchKernelGGL((max_speed_kernel<T, SOL>), dim3(nblk), dim3(BLOCK), 0, s, a);
        return hip_ok(hipGetLastError());
    }
};

template <typename T>
struct Rp2Launch {
    template <template <typename, int> class SOL>
    static int run(const Rp2Args& a, int ixy, int nblk, hipStream_t s)
    {
        if (ixy == 1) hipLaunchKernelGGL((rp2_kernel<T, SOL, 1>), dim3(nblk), dim3(BLOCK), 0, s, a);
        else hipLaunchKernelGGL((rp2_kernel<T, SOL, 2>), dim3(nblk), dim3(BLOCK), 0, s, a);
        return hip_ok(hipGetLastError());
    }
};

static StepArgs base_args(mc_ctx* c, int limiter, int bc)
{
    StepArgs a;
    memset(&a, 0, sizeof(a));
    a.scr = c->scr;
    a.P = dev_params(c->params);
    a.nx = c->nx; a.ny = c->ny; a.bc = bc; a.lim = limiter;
    a.dx = c->dx; a.dy = c->dy;
    a.cfl_target = c->params.cfl_target;
    a.cfl_max = c->params.cfl_max;
    a.rows = c->rows;  // 0: chosen per launch from the kernel's occupancy
    return a;
}

// the tune cache file (kept by the batched-patch code)
extern "C" int mc__tune_cache_lookup(const char* key, int32_t* vals, int nmax);
extern "C" void mc__tune_cache_store(const char* key, const int32_t* vals, int n);

extern "C" {

// context fields for the other translation units of the library (not in the header)
int mc__ctx_info(const mc_ctx* c, int* solver, int* dtype, mc_params* prm, int* cus, void** stream)
{
    *solver = c->solver;
    *dtype = c->dtype;
    *prm = c->params;
    *cus = c->cus;
    *stream = (void*)c->stream;
    return MC_OK;
}

int mc__ctx_grid(const mc_ctx* c, int* nx, int* ny, double* dx, double* dy, unsigned int** status)
{
    *nx = c->nx;
    *ny = c->ny;
    *dx = c->dx;
    *dy = c->dy;
    *status = &c->scr->status;
    return MC_OK;
}

void mc_patches_release_ctx(const mc_ctx* c);
void mc__sur_release_ctx(const mc_ctx* c);
void mc__unsplit_release_ctx(const mc_ctx* c);
int mc__sur_rp2(mc_ctx* c, int ixy, int64_t n, const void* ql, const void* qr, void* waves, void* speeds,
                void* amdq, void* apdq);
int mc__sur_step(mc_ctx* c, mc_state* stt, double dt, int limiter, int bc, mc_cfl* cfl_out);

int mc_solver_dims(int solver, int32_t* meqn, int32_t* mwaves, int32_t* maux)
{
    int m, w, a;
    if (solver_dims(solver, &m, &w, &a) != 0) return MC_EINVAL;
    if (meqn) *meqn = m;
    if (mwaves) *mwaves = w;
    if (maux) *maux = a;
    return MC_OK;
}

const char* mc_strerror(int code)
{
    switch (code) {
    case MC_OK: return "ok";
    case MC_EINVAL: return "invalid argument";
    case MC_ENOMEM: return "out of device memory";
    case MC_EHIP: return "HIP runtime error";
    case MC_ECFL: return "step rejected by the CFL rule";
    case MC_ENONPHYS: return "non-physical state";
    case MC_EUNSUPPORTED: return "unsupported";
    case MC_ESCRATCH: return "request exceeds the static device array";
    default: return "unknown error";
    }
}

int mc_ctx_create(mc_ctx** out, int solver, int dtype, const mc_params* params, int32_t nx,
                  int32_t ny, double dx, double dy, void* hip_stream)
{
    int m, w, a;
    if (!out || !params) return MC_EINVAL;
    *out = nullptr;
    if (solver_dims(solver, &m, &w, &a) != 0) return MC_EINVAL;
    if (dtype != MC_F64 && dtype != MC_F32) return MC_EINVAL;
    if (nx < 1 || ny < 1 || !(dx > 0.0) || !(dy > 0.0)) return MC_EINVAL;
    mc_ctx* c = new mc_ctx();
    c->solver = solver; c->dtype = dtype; c->params = *params;
    c->nx = nx; c->ny = ny; c->dx = dx; c->dy = dy;
    c->stream = (hipStream_t)hip_stream;
    c->rows = 0;
    c->cus = 256;
    c->scr = nullptr;
    c->cap_stream = nullptr;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
        c->cus = cus;
    hipError_t e = hipMalloc((void**)&c->scr, sizeof(Scratch));
    if (e != hipSuccess) {
        fprintf(stderr, "manyclaw: hipMalloc of the context scratch failed: %s\n", hipGetErrorString(e));
        delete c;
        return e == hipErrorOutOfMemory ? MC_ENOMEM : MC_EHIP;
    }
    if (hip_ok(hipMemset(c->scr, 0, sizeof(Scratch))) != MC_OK ||
        hip_ok(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking)) != MC_OK) {
        (void)hipFree(c->scr);
        delete c;
        return MC_EHIP;
    }
    *out = c;
    return MC_OK;
}

void mc_ctx_destroy(mc_ctx* c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    mc_patches_release_ctx(c);
    mc__sur_release_ctx(c);
    mc__unsplit_release_ctx(c);
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    (void)hipFree(c->scr);
    delete c;
}

int mc_ctx_set_tile(mc_ctx* c, int32_t rows)
{
    if (!c || (rows != 0 && (rows < 8 || rows > 1024))) return MC_EINVAL;
    c->rows = rows;
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
    return MC_OK;
}

int mc_rp2(mc_ctx* c, int32_t ixy, int64_t n, const void* ql, const void* qr, const void* aux,
           void* waves, void* speeds, void* amdq, void* apdq)
{
    int m, w, na;
    if (!c || n < 0 || (ixy != 1 && ixy != 2)) return MC_EINVAL;
    solver_dims(c->solver, &m, &w, &na);
    if (n == 0) return MC_OK;
    if (!ql || !qr || !waves || !speeds || !amdq || !apdq || (na > 0 && !aux)) return MC_EINVAL;
    if (is_surrogate(c->solver)) {
        if (c->dtype != MC_F32) return MC_EINVAL;
        return mc__sur_rp2(c, ixy, n, ql, qr, waves, speeds, amdq, apdq);
    }
    Rp2Args a;
    a.ql = ql; a.qr = qr; a.aux = aux; a.waves = waves; a.speeds = speeds; a.amdq = amdq; a.apdq = apdq;
    a.scr = c->scr; a.P = dev_params(c->params); a.n = n;
    int64_t nb = (n + BLOCK - 1) / BLOCK;
    const int64_t cap = (int64_t)c->cus * 16;
    if (nb > cap) nb = cap;
    return dispatch<Rp2Launch>(c->solver, c->dtype, a, (int)ixy, (int)nb, c->stream);
}

int mc_step2d(mc_ctx* c, mc_state* st, const void* aux, double dt, int limiter, int bc,
              mc_cfl* cfl_out)
{
    int m, w, na;
    if (!c || !st || !st->q[0] || !st->q[1] || st->q[0] == st->q[1]) return MC_EINVAL;
    if (st->cur != 0 && st->cur != 1) return MC_EINVAL;
    if (!(dt >= 0.0) || limiter < MC_LIM_NONE || limiter > MC_LIM_FIRST_ORDER) return MC_EINVAL;
    if (bc != MC_BC_PERIODIC && bc != MC_BC_EXTRAP) return MC_EINVAL;
    if (is_surrogate(c->solver)) {
        if (c->dtype != MC_F32) return MC_EINVAL;
        return mc__sur_step(c, st, dt, limiter, bc, cfl_out);
    }
    solver_dims(c->solver, &m, &w, &na);
    if (na > 0 && !aux) return MC_EINVAL;
    StepArgs a = base_args(c, limiter, bc);
    a.buf[0] = st->q[0]; a.buf[1] = st->q[1];
    a.aux = aux; a.clk = nullptr; a.cfl_out = cfl_out;
    a.dt_host = dt; a.src_host = st->cur;
    int r = dispatch<StepLaunch>(c->solver, c->dtype, a, c->cus, c->stream);
    if (r == MC_OK) st->cur ^= 1;
    return r;
}

int mc_step2d_strang(mc_ctx* c, mc_state* st, const void* aux, double dt, int limiter, int bc,
                     mc_cfl* cfl_out)
{
    int m, w, na;
    if (!c || !st || !st->q[0] || !st->q[1] || st->q[0] == st->q[1]) return MC_EINVAL;
    if (st->cur != 0 && st->cur != 1) return MC_EINVAL;
    if (!(dt >= 0.0) || limiter < MC_LIM_NONE || limiter > MC_LIM_FIRST_ORDER) return MC_EINVAL;
    if (bc != MC_BC_PERIODIC && bc != MC_BC_EXTRAP) return MC_EINVAL;
    if (is_surrogate(c->solver)) return MC_EUNSUPPORTED;
    solver_dims(c->solver, &m, &w, &na);
    if (na > 0 && !aux) return MC_EINVAL;
    // one pass: x (dt/2), y (dt) and the closing x (dt/2) of each finished
    // row; the x Courant factor and the x speeds are halved by handing the
    // kernel 2 dx, so its smax is max(|s_x| / (2 dx), |s_y| / dy) over the
    // three sweeps
    StepArgs a = base_args(c, limiter, bc);
    a.dx = 2.0 * c->dx;
    a.buf[0] = st->q[0]; a.buf[1] = st->q[1];
    a.aux = aux; a.clk = nullptr; a.cfl_out = cfl_out;
    a.dt_host = dt; a.src_host = st->cur;
    const int r = dispatch<StrangLaunch>(c->solver, c->dtype, a, c->cus, c->stream);
    if (r == MC_OK) st->cur ^= 1;
    return r;
}

int mc_tune_rows(mc_ctx* c, const mc_state* st, const void* aux, double dt, int limiter, int bc,
                 int32_t* rows_out)
{
    int m, w, na;
    if (!c || !st || !st->q[0] || !st->q[1] || st->q[0] == st->q[1]) return MC_EINVAL;
    if (st->cur != 0 && st->cur != 1) return MC_EINVAL;
    if (!(dt >= 0.0) || limiter < MC_LIM_NONE || limiter > MC_LIM_FIRST_ORDER) return MC_EINVAL;
    if (bc != MC_BC_PERIODIC && bc != MC_BC_EXTRAP) return MC_EINVAL;
    if (is_surrogate(c->solver)) return MC_EUNSUPPORTED;
    solver_dims(c->solver, &m, &w, &na);
    if (na > 0 && !aux) return MC_EINVAL;
    // a choice kept in the tune cache file for this launch shape and device
    char key[160];
    {
        hipDeviceProp_t prop;
        int dev = 0;
        char arch[64] = "gpu";
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
            snprintf(arch, sizeof arch, "%s", prop.gcnArchName);
            char* colon = strchr(arch, ':');
            if (colon) *colon = 0;
        }
        snprintf(key, sizeof key, "rows-%d-%d-%d-%d-%dx%d-%s-%d", c->solver, c->dtype, limiter, bc, c->nx, c->ny,
                 arch, c->cus);
    }
    int32_t cached = -1;
    if (mc__tune_cache_lookup(key, &cached, 1) == 1 && (cached == 0 || (cached >= 8 && cached <= 1024))) {
        const int rc = mc_ctx_set_tile(c, cached);
        if (rc == MC_OK && rows_out) *rows_out = cached;
        return rc;
    }
    // candidates: the occupancy rule (0) and fixed heights up to the grid's
    static const int cand[] = {0, 16, 24, 32, 40, 48, 64, 96, 128, 192, 256};
    std::vector<int> rs;
    for (int R : cand)
        if (R == 0 || R <= std::max(c->ny, 8)) rs.push_back(R);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return MC_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return MC_EHIP; }
    std::vector<float> best_ms(rs.size(), -1.0f);
    int r = MC_OK;
    // two passes over the candidates, each one launch to warm up and three
    // timed; every launch is the step of q[cur] into q[1 - cur]
    for (int pass = 0; pass < 2 && r == MC_OK; ++pass) {
        for (size_t k = 0; k < rs.size() && r == MC_OK; ++k) {
            StepArgs a = base_args(c, limiter, bc);
            a.rows = rs[k];
            a.buf[0] = st->q[0]; a.buf[1] = st->q[1];
            a.aux = aux; a.clk = nullptr; a.cfl_out = nullptr;
            a.dt_host = dt; a.src_host = st->cur;
            r = dispatch<StepLaunch>(c->solver, c->dtype, a, c->cus, c->stream);
            if (r != MC_OK) break;
            if (hipEventRecord(e0, c->stream) != hipSuccess) { r = MC_EHIP; break; }
            for (int i = 0; i < 3 && r == MC_OK; ++i) r = dispatch<StepLaunch>(c->solver, c->dtype, a, c->cus, c->stream);
            if (r != MC_OK) break;
            float ms = 0.0f;
            if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                r = MC_EHIP;
                break;
            }
            if (best_ms[k] < 0.0f || ms < best_ms[k]) best_ms[k] = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (r != MC_OK) return r;
    // the fastest, unless the occupancy rule (candidate 0) is within 3 % of
    // it: differences that small are run-to-run noise, and the rule then
    // keeps the choice stable from run to run
    size_t kb = 0;
    for (size_t k = 1; k < rs.size(); ++k)
        if (best_ms[k] < best_ms[kb]) kb = k;
    if (best_ms[0] <= 1.03f * best_ms[kb]) kb = 0;
    const int32_t chosen = rs[kb];
    mc__tune_cache_store(key, &chosen, 1);
    const int rc = mc_ctx_set_tile(c, rs[kb]);
    if (rc == MC_OK && rows_out) *rows_out = rs[kb];
    return rc;
}

static int launch_speed(mc_ctx* c, const void* q, const void* aux, int bc, mc_cfl* out,
                        mc_clock* clk, int init)
{
    int m, w, na;
    if (!c || !q || (bc != MC_BC_PERIODIC && bc != MC_BC_EXTRAP)) return MC_EINVAL;
    if (is_surrogate(c->solver)) return MC_EINVAL;
    solver_dims(c->solver, &m, &w, &na);
    if (na > 0 && !aux) return MC_EINVAL;
    StepArgs a = base_args(c, MC_LIM_NONE, bc);
    a.buf[0] = (void*)q; a.buf[1] = nullptr;
    a.aux = aux; a.cfl_out = out; a.clk = (DevClock*)clk; a.init_only = init;
    const int64_t n = (int64_t)(c->nx + 1) * (c->ny + 1);
    int64_t nb = (n + BLOCK - 1) / BLOCK;
    const int64_t cap = (int64_t)c->cus * 8;
    if (nb > cap) nb = cap;
    return dispatch<SpeedLaunch>(c->solver, c->dtype, a, (int)nb, c->stream);
}

int mc_max_speed(mc_ctx* c, const void* q, const void* aux, int bc, mc_cfl* out)
{
    if (!out) return MC_EINVAL;
    return launch_speed(c, q, aux, bc, out, nullptr, 0);
}

int mc_clock_init(mc_ctx* c, mc_clock* clk, const void* q, const void* aux, int bc)
{
    if (!clk) return MC_EINVAL;
    return launch_speed(c, q, aux, bc, nullptr, clk, 1);
}

static int enqueue_run(mc_ctx* c, const StepArgs& a, int nsteps, hipStream_t s)
{
    for (int k = 0; k < nsteps; ++k) {
        int r = dispatch<StepLaunch>(c->solver, c->dtype, a, c->cus, s);
        if (r != MC_OK) return r;
    }
    return MC_OK;
}

int mc_run2d(mc_ctx* c, void* q0, void* q1, const void* aux, mc_clock* clk, int32_t nsteps,
             int limiter, int bc, int use_graph)
{
    int m, w, na;
    if (!c || !q0 || !q1 || q0 == q1 || !clk || nsteps < 0) return MC_EINVAL;
    if (limiter < MC_LIM_NONE || limiter > MC_LIM_FIRST_ORDER) return MC_EINVAL;
    if (bc != MC_BC_PERIODIC && bc != MC_BC_EXTRAP) return MC_EINVAL;
    if (is_surrogate(c->solver)) return MC_EINVAL;
    solver_dims(c->solver, &m, &w, &na);
    if (na > 0 && !aux) return MC_EINVAL;
    if (nsteps == 0) return MC_OK;
    StepArgs a = base_args(c, limiter, bc);
    a.buf[0] = q0; a.buf[1] = q1; a.aux = aux; a.clk = (DevClock*)clk; a.cfl_out = nullptr;
    if (!use_graph) return enqueue_run(c, a, nsteps, c->stream);

    GraphKey key{q0, q1, aux, (void*)clk, nsteps, limiter, bc};
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        if (hip_ok(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal)) != MC_OK)
            return MC_EHIP;
        int r = enqueue_run(c, a, nsteps, c->cap_stream);
        hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
        if (r != MC_OK || hip_ok(e) != MC_OK) { if (g) (void)hipGraphDestroy(g); return MC_EHIP; }
        e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (hip_ok(e) != MC_OK) return MC_EHIP;
        it = c->graphs.emplace(key, ge).first;
    }
    return hip_ok(hipGraphLaunch(it->second, c->stream));
}

int mc_copy_probe(mc_ctx* c, void* dst, const void* src, int64_t nbytes)
{
    if (!c || !dst || !src || nbytes < 0 || (nbytes % 16) != 0) return MC_EINVAL;
    if ((((uintptr_t)dst) | ((uintptr_t)src)) % 16 != 0) return MC_EINVAL;
    if (nbytes == 0) return MC_OK;
    const int64_t n16 = nbytes / 16;
    int64_t nb = (n16 + (int64_t)BLOCK * CP_U - 1) / ((int64_t)BLOCK * CP_U);
    const int64_t cap = (int64_t)c->cus * 16;  // 16 workgroups (64 wavefronts) per CU
    if (nb > cap) nb = cap;
    hipLaunchKernelGGL(copy_probe_kernel, dim3((unsigned)nb), dim3(BLOCK), 0, c->stream,
                       (const u32x4*)src, (u32x4*)dst, n16);
    return hip_ok(hipGetLastError());
}

int mc_status_get(mc_ctx* c, int32_t* status)
{
    if (!c || !status) return MC_EINVAL;
    unsigned v = 0;
    if (hip_ok(hipStreamSynchronize(c->stream)) != MC_OK) return MC_EHIP;
    if (hip_ok(hipMemcpy(&v, &c->scr->status, sizeof(v), hipMemcpyDeviceToHost)) != MC_OK) return MC_EHIP;
    unsigned z = 0;
    if (hip_ok(hipMemcpy(&c->scr->status, &z, sizeof(z), hipMemcpyHostToDevice)) != MC_OK) return MC_EHIP;
    *status = (int32_t)v;
    return MC_OK;
}

}  // extern "C"
