// solvers.hpp -- pointwise normal Riemann solvers for the gfx950 kernels.
//
// Each solver is a struct template over the arithmetic type T and the edge
// direction IXY (1: x-normal, 2: y-normal).  It is unaware of any
// parallelism around it: it sees two cells and fills one Edge (paper,
// section 2: the solver is left as it would be in serial code and the
// threading lives outside it).  The formulas are those of the
// wave-propagation method (LeVeque, Finite Volume Methods for Hyperbolic
// Problems, 2002, ch. 3, 4, 9, 14, 15; Harten & Hyman 1983 for the entropy
// fix; Einfeldt 1988 for HLLE; Toro 2009 ch. 11 for the Euler Roe form).
//
// Interface of a solver S (as used by the kernels):
//   MEQN, MWAVES, MAUX        sizes
//   NC                        values per Cell (state, then per-cell
//                             precomputed quantities and aux values)
//   NE, NX                    values per edge record; the first NX of them
//                             are all that dot() reads from its second edge
//   prep(P, c)                fills c.v[MEQN..NC) from the state c.v[0..MEQN)
//                             and the aux values
//   solve(P, L, R, e)         edge record of the Riemann problem between
//                             cells L (left) and R (right); returns
//                             ST_NONPHYS / ST_FALLBACK bits
//   speed(P, e, p)            s_p
//   smax(P, e)                max_p |s_p| (the edge's part of the CFL number)
//   dot(P, a, b, p)           W_p(a) . W_p(b), the limiter's wave product
//   norm2(P, e, p)            W_p . W_p
//   SLOPE                     false: the limiter takes theta = dot / norm2;
//                             true: it takes the neighbour's strength t
//                             along the edge's own eigenvectors (lterms)
//   pair(P, e, el, tl, tr)    for an edge e and its left (or upper)
//                             neighbour el: what the limiter of e takes from
//                             el (tl) and what that of el takes from e (tr);
//                             both W_p(e) . W_p(el) unless SLOPE
//   combo(P, e, coef, out)    out = sum_p coef_p W_p
//   fluct(P, e, am, ap)       A-dQ and A+dQ
//   waves(P, e, W)            the waves as components (batch Riemann output)
// A record stores whatever determines the waves: for shallow-water Roe the
// strengths alpha_p and the eigenvector parameters (nine scalars instead of
// nine wave components, three speeds and six fluctuations), for the linear
// systems the strengths (with the impedances and sound speeds when they vary
// per cell), for Euler the strengths and Roe-average parameters or, on HLLE
// edges, the two waves (EulerRoeK); the other solvers store components
// (Componentwise below).
// Momentum/velocity slots: MU is the component normal to the edge, MV the
// transverse one, so the y-normal solve is the x-normal one with the two
// slots exchanged.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mc {

enum : unsigned { ST_NONPHYS = 1u, ST_FALLBACK = 2u, ST_CFL = 4u };

struct DevParams {
    double g, gamma, rho, K, u, v;
};

template <typename T, int NC>
struct Cell {
    T v[NC];
};

template <typename T, int NE>
struct Rec {
    T v[NE];
};

// component form used by the solvers without a compact record
template <typename T, int MW, int ME>
struct Edge {
    T w[MW][ME];  // waves
    T s[MW];      // speeds
    T am[ME];     // left-going fluctuation A-dQ
    T ap[ME];     // right-going fluctuation A+dQ
};

template <typename T>
__device__ __forceinline__ T tmin0(T s) { return s < T(0) ? s : T(0); }
template <typename T>
__device__ __forceinline__ T tmax0(T s) { return s > T(0) ? s : T(0); }

// FP64 minimum and maximum as single instructions, for the shallow-water
// walker.  The compiler, unable to prove that an operand reaching a min or
// max from another block or a lane exchange is not a signalling NaN,
// precedes each such operand with a quieting max(x, x); no value here is
// ever a signalling NaN (all come from arithmetic on finite data), so these
// issue v_min_f64 / v_max_f64 alone.  (In the other walkers the opaque
// instruction cost more in scheduling than it saved.)
__device__ __forceinline__ double dmin_abs(double a, double b)
{
    double r;
    asm("v_min_f64 %0, |%1|, |%2|" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ double dmax_abs(double a, double b)
{
    double r;
    asm("v_max_f64 %0, |%1|, |%2|" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ double dmin(double a, double b)
{
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ double dmax(double a, double b)
{
    double r;
    asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ double dmin0(double s)
{
    double r;
    asm("v_min_f64 %0, %1, 0" : "=v"(r) : "v"(s));
    return r;
}
// whether a solver asks for the single-instruction FP64 maximum in the
// walker's CFL reduction (QMINMAX)
template <class S, class = void>
struct qminmax { static constexpr bool value = false; };
template <class S>
struct qminmax<S, decltype((void)S::QMINMAX)> { static constexpr bool value = S::QMINMAX; };
template <class S, typename T>
__device__ __forceinline__ T cfl_max(T m, T s)
{
    if constexpr (sizeof(T) == 8 && qminmax<S>::value) return dmax(m, s);
    else return fmax(m, s);
}
template <typename T>
__device__ __forceinline__ T qmin0(T s)
{
    if constexpr (sizeof(T) == 8) return dmin0(s);
    else return tmin0(s);
}

// ------------------------------------------------------------ fast math
// Reciprocal and reciprocal square root from the hardware estimates.  The
// FP64 estimates (v_rcp_f64, v_rsq_f64) are good to about 2^-23.  One
// correction of third order brings them to within a couple of ulps (the
// remaining relative error is of the order of the estimate's cubed, about
// 2^-69, below the rounding of the last step), without the range scaling of
// the IEEE division/sqrt sequences (all operands here are normal positive
// numbers): with e = 1 - x r, 1/x = r (1 + e + e^2 + ...), and with
// e = 1 - x y^2, 1/sqrt(x) = y (1 + e/2 + 3 e^2/8 + ...).  The FP32
// estimates are within 1 ulp as they are.
__device__ __forceinline__ double frcp(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, r, 1.0);
    return fma(r, fma(e, e, e), r);
}
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

// one Newton-Raphson step only: about 2^-46, used for the limiter ratio
__device__ __forceinline__ double frcp1(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float frcp1(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ double frsq(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }

// sqrt(x) for x > 0 (x * rsqrt(x)); 0 otherwise
__device__ __forceinline__ double fsqrt(double x) { return x > 0.0 ? x * frsq(x) : 0.0; }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

template <typename T>
__device__ __forceinline__ T tsqrt(T x) { return fsqrt(x); }

// ---------------------------------------------------- component records
// Wraps a solver B that produces component waves (B::solve fills an Edge)
// into the record interface.  Record layout: the structurally non-zero
// wave components (B::nz), then the speeds, then A-dQ, then A+dQ.  Every
// sum is an explicit multiply-add chain (the library is built without
// implicit contraction, so every tile evaluates the same operations).
template <class B>
struct Componentwise {
    using T = typename B::value_type;
    static constexpr int MEQN = B::MEQN, MWAVES = B::MWAVES, MAUX = B::MAUX, NC = B::NC;
    static constexpr int count_nz()
    {
        int n = 0;
        for (int p = 0; p < MWAVES; ++p)
            for (int m = 0; m < MEQN; ++m)
                if (B::nz(p, m)) ++n;
        return n;
    }
    static constexpr int NX = count_nz();
    static constexpr int NE = NX + MWAVES + 2 * MEQN;
    static constexpr int widx(int p, int m)
    {
        int n = 0;
        for (int pp = 0; pp < MWAVES; ++pp)
            for (int mm = 0; mm < MEQN; ++mm) {
                if (!B::nz(pp, mm)) continue;
                if (pp == p && mm == m) return n;
                ++n;
            }
        return -1;
    }
    using C = typename B::C;
    using E = Rec<T, NE>;

    __device__ static void prep(const DevParams& P, C& c) { B::prep(P, c); }
    __device__ static unsigned solve(const DevParams& P, const C& L, const C& R, E& r)
    {
        typename B::E e;
        const unsigned st = B::solve(P, L, R, e);
#pragma unroll
        for (int p = 0; p < MWAVES; ++p) {
#pragma unroll
            for (int m = 0; m < MEQN; ++m)
                if (B::nz(p, m)) r.v[widx(p, m)] = e.w[p][m];
            r.v[NX + p] = e.s[p];
        }
#pragma unroll
        for (int m = 0; m < MEQN; ++m) {
            r.v[NX + MWAVES + m] = e.am[m];
            r.v[NX + MWAVES + MEQN + m] = e.ap[m];
        }
        return st;
    }
    __device__ static T speed(const DevParams&, const E& r, int p) { return r.v[NX + p]; }
    __device__ static T smax(const DevParams&, const E& r)
    {
        T m = fabs(r.v[NX]);
#pragma unroll
        for (int p = 1; p < MWAVES; ++p) m = fmax(m, fabs(r.v[NX + p]));
        return m;
    }
    __device__ static T dot(const DevParams&, const E& a, const E& b, int p)
    {
        T acc = T(0);
        bool first = true;
#pragma unroll
        for (int m = 0; m < MEQN; ++m) {
            if (!B::nz(p, m)) continue;
            const int k = widx(p, m);
            acc = first ? a.v[k] * b.v[k] : fma(a.v[k], b.v[k], acc);
            first = false;
        }
        return acc;
    }
    __device__ static T norm2(const DevParams& P, const E& r, int p) { return dot(P, r, r, p); }
    static constexpr bool SLOPE = false;
    __device__ static void pair(const DevParams& P, const E& e, const E& el, T* tl, T* tr)
    {
#pragma unroll
        for (int p = 0; p < MWAVES; ++p) tl[p] = tr[p] = dot(P, e, el, p);
    }
    __device__ static void combo(const DevParams&, const E& r, const T* coef, T* out)
    {
#pragma unroll
        for (int m = 0; m < MEQN; ++m) {
            T acc = T(0);
            bool first = true;
#pragma unroll
            for (int p = 0; p < MWAVES; ++p) {
                if (!B::nz(p, m)) continue;
                const T w = r.v[widx(p, m)];
                acc = first ? coef[p] * w : fma(coef[p], w, acc);
                first = false;
            }
            out[m] = acc;
        }
    }
    __device__ static void fluct(const DevParams&, const E& r, T* am, T* ap)
    {
#pragma unroll
        for (int m = 0; m < MEQN; ++m) {
            am[m] = r.v[NX + MWAVES + m];
            ap[m] = r.v[NX + MWAVES + MEQN + m];
        }
    }
    __device__ static void waves(const DevParams&, const E& r, T (*W)[MEQN])
    {
#pragma unroll
        for (int p = 0; p < MWAVES; ++p)
#pragma unroll
            for (int m = 0; m < MEQN; ++m) W[p][m] = B::nz(p, m) ? r.v[widx(p, m)] : T(0);
    }
    // the two quantities the update needs: A-dQ + F and A+dQ - F, with the
    // correction flux F = sum_p coef_p W_p
    __device__ static void terms(const DevParams& P, const E& r, const T* coef, T* lf, T* rg)
    {
        T F[MEQN], am[MEQN], ap[MEQN];
        combo(P, r, coef, F);
        fluct(P, r, am, ap);
#pragma unroll
        for (int m = 0; m < MEQN; ++m) {
            lf[m] = am[m] + F[m];
            rg[m] = ap[m] - F[m];
        }
    }
};

// sum_p coef[p] W_p[m] over the structurally non-zero components of a
// component Edge
template <class S, typename T, typename E>
__device__ __forceinline__ T lincomb(const T* coef, const E& e, int m)
{
    T acc = T(0);
    bool first = true;
#pragma unroll
    for (int p = 0; p < S::MWAVES; ++p) {
        if (!S::nz(p, m)) continue;
        acc = first ? coef[p] * e.w[p][m] : fma(coef[p], e.w[p][m], acc);
        first = false;
    }
    return acc;
}

// amdq = sum_p min(s_p,0) W_p, apdq = sum_p max(s_p,0) W_p
template <class S, typename T, typename E>
__device__ __forceinline__ void upwind_split(E& e)
{
    T sm[S::MWAVES], sp[S::MWAVES];
#pragma unroll
    for (int p = 0; p < S::MWAVES; ++p) { sm[p] = tmin0(e.s[p]); sp[p] = tmax0(e.s[p]); }
#pragma unroll
    for (int m = 0; m < S::MEQN; ++m) {
        e.am[m] = lincomb<S>(sm, e, m);
        e.ap[m] = lincomb<S>(sp, e, m);
    }
}

// amdq = sum_p f_p W_p with the entropy-fixed left-going speeds f_p, and
// apdq = sum_p s_p W_p - amdq (their sum keeps the Roe total)
template <class S, typename T, typename E>
__device__ __forceinline__ void fixed_split(E& e, const T* f)
{
#pragma unroll
    for (int m = 0; m < S::MEQN; ++m) {
        const T tot = lincomb<S>(e.s, e, m);
        e.am[m] = lincomb<S>(f, e, m);
        e.ap[m] = tot - e.am[m];
    }
}

template <class S, typename T, typename E>
__device__ __forceinline__ void zero_edge(E& e)
{
#pragma unroll
    for (int p = 0; p < S::MWAVES; ++p) {
        e.s[p] = T(0);
#pragma unroll
        for (int m = 0; m < S::MEQN; ++m) e.w[p][m] = T(0);
    }
#pragma unroll
    for (int m = 0; m < S::MEQN; ++m) { e.am[m] = T(0); e.ap[m] = T(0); }
}

// ------------------------------------------------------------- limiters
// phi(theta) with theta = a / b, b = W.W > 0 (FVMHP ch. 6).  theta <= 0
// gives 0 for every limiter except "none".
enum : int { LIM_NONE = 0, LIM_MINMOD = 1, LIM_SUPERBEE = 2, LIM_VANLEER = 3, LIM_MC = 4,
             LIM_FIRST_ORDER = 5 };

// phi for theta = a / b; callers pass a > 0 only through the select below
template <int LIM, typename T>
__device__ __forceinline__ T limiter_phi(T a, T b)
{
    if (LIM == LIM_NONE) return T(1);
    const T th = a * frcp1(b);
    T r;
    if (LIM == LIM_MC) {
        r = fma(T(0.5), th, T(0.5));
        r = r < T(2) ? r : T(2);
        r = (T(2) * th) < r ? T(2) * th : r;
    } else if (LIM == LIM_MINMOD) {
        r = th < T(1) ? th : T(1);
    } else if (LIM == LIM_SUPERBEE) {
        const T x = T(2) * th < T(1) ? T(2) * th : T(1);
        const T y = th < T(2) ? th : T(2);
        r = x > y ? x : y;
    } else {  // van Leer
        r = (th + th) * frcp(T(1) + th);
    }
    // a > 0 implies b = W.W > 0; a <= 0 (including W = 0) gives phi = 0
    return a > T(0) ? r : T(0);
}

// (1/2) phi(t / a) a, a the wave's strength and t its upwind neighbour's
// along the same eigenvector (SLOPE solvers).  theta = t / a <= 0, and a = 0
// (theta taken as 0), give 0 for every limiter except "none".  med0(x, y) is
// the median of 0, x and y: the one of x, y nearer to 0 when they have the
// same sign, else 0 (minmod).
template <typename T>
__device__ __forceinline__ T med0(T x, T y)
{
    return fmin(fmax(x, y), fmax(fmin(x, y), T(0)));
}
template <int LIM, typename T>
__device__ __forceinline__ T slope_half(T a, T t)
{
    if (LIM == LIM_NONE) return T(0.5) * a;
    if (LIM == LIM_MC) {
        // a phi = minmod(2a, 2t, (a + t)/2): for a t > 0 the sign of a times
        // 2 min(|a|, |t|, |a + t| / 4), else 0
        const T m = fmin(fmin(fabs(a), fabs(t)), T(0.25) * fabs(a + t));
        return a * t > T(0) ? copysign(m, a) : T(0);
    }
    if (LIM == LIM_MINMOD) return T(0.5) * med0(a, t);
    if (LIM == LIM_SUPERBEE) {
        // the larger in magnitude of minmod(a, 2t) and minmod(2a, t)
        const T x = med0(a, T(2) * t), y = med0(T(2) * a, t);
        return T(0.5) * (fabs(x) >= fabs(y) ? x : y);
    }
    // van Leer: a phi = 2 a t / (a + t) for a t > 0
    const T at = a * t;
    return at > T(0) ? at * frcp(a + t) : T(0);
}
// slope_half with the single-instruction FP64 minimum (MC limiter)
template <int LIM, typename T>
__device__ __forceinline__ T slope_half_q(T a, T t)
{
    if constexpr (LIM == LIM_MC && sizeof(T) == 8) {
        const T m = dmin(dmin_abs(a, t), T(0.25) * fabs(a + t));
        return a * t > T(0) ? copysign(m, a) : T(0);
    } else {
        return slope_half<LIM, T>(a, t);
    }
}

// ------------------------------------------------------------- advection
template <typename T, int IXY>
struct AdvectionC {
    using value_type = T;
    static constexpr int MEQN = 1, MWAVES = 1, MAUX = 0, NC = 1;
    using C = Cell<T, NC>;
    using E = Edge<T, MWAVES, MEQN>;
    __host__ __device__ static constexpr bool nz(int, int) { return true; }
    __device__ static void prep(const DevParams&, C&) {}
    __device__ static unsigned solve(const DevParams& P, const C& L, const C& R, E& e)
    {
        e.w[0][0] = R.v[0] - L.v[0];
        e.s[0] = T(IXY == 1 ? P.u : P.v);
        upwind_split<AdvectionC, T>(e);
        return 0u;
    }
};

// ---------------------------------------------- constant-coefficient acoustics
// q = (p, u, v); eigenvalues -c, +c (the zero-speed shear wave carries no
// fluctuation and is left out), eigenvectors (-Z, 1) and (Z, 1) in the
// (p, normal velocity) slots, Z = rho c, c = sqrt(K/rho).
template <typename T, int IXY>
struct AcousticsC {
    using value_type = T;
    static constexpr int MEQN = 3, MWAVES = 2, MAUX = 0, NC = 3;
    static constexpr int MU = IXY == 1 ? 1 : 2, MV = IXY == 1 ? 2 : 1;
    using C = Cell<T, NC>;
    using E = Edge<T, MWAVES, MEQN>;
    __host__ __device__ static constexpr bool nz(int, int m) { return m != MV; }
    __device__ static void prep(const DevParams&, C&) {}
    __device__ static unsigned solve(const DevParams& P, const C& L, const C& R, E& e)
    {
        const T c = T(sqrt(P.K / P.rho));
        const T Z = T(P.rho * sqrt(P.K / P.rho));
        const T rz2 = T(0.5 / (P.rho * sqrt(P.K / P.rho)));
        const T dp = R.v[0] - L.v[0];
        const T du = R.v[MU] - L.v[MU];
        const T a1 = fma(Z, du, -dp) * rz2;
        const T a2 = fma(Z, du, dp) * rz2;
        e.w[0][0] = -a1 * Z; e.w[0][MU] = a1; e.w[0][MV] = T(0);
        e.w[1][0] = a2 * Z;  e.w[1][MU] = a2; e.w[1][MV] = T(0);
        e.s[0] = -c;
        e.s[1] = c;
        upwind_split<AcousticsC, T>(e);
        return 0u;
    }
};

// ---------------------------------------------- variable-coefficient acoustics
// aux = (rho, c) per cell; W1 = a1 (-Z_L, 1) at -c_L, W2 = a2 (Z_R, 1) at +c_R,
// a1 = (-dp + Z_R du)/(Z_L + Z_R), a2 = (dp + Z_L du)/(Z_L + Z_R).
// Cell: v[0..2] = q, v[3] = Z, v[4] = c (v[3] holds rho until prep).
template <typename T, int IXY>
struct AcousticsVCC {
    using value_type = T;
    static constexpr int MEQN = 3, MWAVES = 2, MAUX = 2, NC = 5;
    static constexpr int MU = IXY == 1 ? 1 : 2, MV = IXY == 1 ? 2 : 1;
    using C = Cell<T, NC>;
    using E = Edge<T, MWAVES, MEQN>;
    __host__ __device__ static constexpr bool nz(int, int m) { return m != MV; }
    __device__ static void prep(const DevParams&, C& c) { c.v[3] = c.v[3] * c.v[4]; }
    __device__ static unsigned solve(const DevParams&, const C& L, const C& R, E& e)
    {
        const T zl = L.v[3], zr = R.v[3];
        const T dp = R.v[0] - L.v[0];
        const T du = R.v[MU] - L.v[MU];
        const T rz = frcp(zl + zr);
        const T a1 = fma(zr, du, -dp) * rz;
        const T a2 = fma(zl, du, dp) * rz;
        e.w[0][0] = -a1 * zl; e.w[0][MU] = a1; e.w[0][MV] = T(0);
        e.w[1][0] = a2 * zr;  e.w[1][MU] = a2; e.w[1][MV] = T(0);
        e.s[0] = -L.v[4];
        e.s[1] = R.v[4];
        upwind_split<AcousticsVCC, T>(e);
        return 0u;
    }
};

// ------------------------------------------ strength records, linear systems
// The linear systems' eigenvectors are known in closed form, so an edge
// record keeps only the wave strengths (with variable coefficients also the
// impedances and sound speeds that fix the eigenvectors and speeds), and
// the limiter works on strengths as for shallow-water Roe (SwRoe::lterms):
// t is the upwind neighbour's strength along this edge's eigenvector, and
// phi(t / alpha) alpha comes from slope_half without a division.  For
// advection and constant-coefficient acoustics every edge has the same
// eigenvectors, so t is the neighbour's strength itself.

// advection: one wave alpha = q_R - q_L at the uniform speed u (x) or v (y)
template <typename T, int IXY>
struct AdvectionK {
    static constexpr int MEQN = 1, MWAVES = 1, MAUX = 0, NC = 1, NE = 1, NX = 1;
    using C = Cell<T, NC>;
    using E = Rec<T, NE>;
    __device__ static T vel(const DevParams& P) { return T(IXY == 1 ? P.u : P.v); }
    __device__ static void prep(const DevParams&, C&) {}
    __device__ static unsigned solve(const DevParams&, const C& L, const C& R, E& e)
    {
        e.v[0] = R.v[0] - L.v[0];
        return 0u;
    }
    __device__ static T speed(const DevParams& P, const E&, int) { return vel(P); }
    __device__ static T smax(const DevParams& P, const E&) { return fabs(vel(P)); }
    static constexpr bool SLOPE = true;
    __device__ static void pair(const DevParams&, const E& e, const E& el, T* tl, T* tr)
    {
        tl[0] = el.v[0];
        tr[0] = e.v[0];
    }
    template <int LIM>
    __device__ static void lterms(const DevParams& P, const E& e, const T* tl, const T* tr, T nu, T* lf,
                                  T* rg)
    {
        const T s = vel(P), a = e.v[0];
        T L = tmin0(s) * a;
        if (LIM != LIM_FIRST_ORDER) {
            const T as = fabs(s);
            L = fma(tmin0(s), a, (as * fma(-nu, as, T(1))) * slope_half<LIM, T>(a, s > T(0) ? tl[0] : tr[0]));
        }
        lf[0] = L;
        rg[0] = fma(s, a, -L);
    }
    __device__ static void fluct(const DevParams& P, const E& e, T* am, T* ap)
    {
        const T s = vel(P);
        am[0] = tmin0(s) * e.v[0];
        ap[0] = tmax0(s) * e.v[0];
    }
    __device__ static void waves(const DevParams&, const E& e, T (*W)[1]) { W[0][0] = e.v[0]; }
};

// constant-coefficient acoustics: W_1 = alpha_1 (-Z, 1) at -c and
// W_2 = alpha_2 (Z, 1) at +c in the (p, normal velocity) slots
template <typename T, int IXY>
struct AcousticsK {
    static constexpr int MEQN = 3, MWAVES = 2, MAUX = 0, NC = 3, NE = 2, NX = 2;
    static constexpr int MU = IXY == 1 ? 1 : 2, MV = IXY == 1 ? 2 : 1;
    using C = Cell<T, NC>;
    using E = Rec<T, NE>;
    __device__ static T cs(const DevParams& P) { return T(sqrt(P.K / P.rho)); }
    __device__ static T zs(const DevParams& P) { return T(P.rho * sqrt(P.K / P.rho)); }
    __device__ static void prep(const DevParams&, C&) {}
    __device__ static unsigned solve(const DevParams& P, const C& L, const C& R, E& e)
    {
        const T Z = zs(P);
        const T rz2 = T(0.5 / (P.rho * sqrt(P.K / P.rho)));
        const T dp = R.v[0] - L.v[0];
        const T du = R.v[MU] - L.v[MU];
        e.v[0] = fma(Z, du, -dp) * rz2;
        e.v[1] = fma(Z, du, dp) * rz2;
        return 0u;
    }
    __device__ static T speed(const DevParams& P, const E&, int p) { return p == 0 ? -cs(P) : cs(P); }
    __device__ static T smax(const DevParams& P, const E&) { return cs(P); }
    static constexpr bool SLOPE = true;
    __device__ static void pair(const DevParams&, const E& e, const E& el, T* tl, T* tr)
    {
        tl[0] = el.v[0]; tl[1] = el.v[1];
        tr[0] = e.v[0];  tr[1] = e.v[1];
    }
    // A-dQ + F = L_1 r_1 + L_2 r_2 and A+dQ - F = R_1 r_1 + R_2 r_2
    __device__ static void out(const DevParams& P, T L1, T L2, T* o)
    {
        o[0] = zs(P) * (L2 - L1);
        o[MU] = L1 + L2;
        o[MV] = T(0);
    }
    template <int LIM>
    __device__ static void lterms(const DevParams& P, const E& e, const T* tl, const T* tr, T nu, T* lf,
                                  T* rg)
    {
        const T c = cs(P), a1 = e.v[0], a2 = e.v[1];
        T L1 = -c * a1, L2 = T(0);
        if (LIM != LIM_FIRST_ORDER) {
            const T k = c * fma(-nu, c, T(1));
            L1 = fma(-c, a1, k * slope_half<LIM, T>(a1, tr[0]));  // s_1 < 0: the right neighbour's
            L2 = k * slope_half<LIM, T>(a2, tl[1]);               // s_2 > 0: the left neighbour's
        }
        out(P, L1, L2, lf);
        out(P, fma(-c, a1, -L1), fma(c, a2, -L2), rg);
    }
    __device__ static void fluct(const DevParams& P, const E& e, T* am, T* ap)
    {
        const T c = cs(P);
        out(P, -c * e.v[0], T(0), am);
        out(P, T(0), c * e.v[1], ap);
    }
    __device__ static void waves(const DevParams& P, const E& e, T (*W)[3])
    {
        const T Z = zs(P);
        W[0][0] = -e.v[0] * Z; W[0][MU] = e.v[0]; W[0][MV] = T(0);
        W[1][0] = e.v[1] * Z;  W[1][MU] = e.v[1]; W[1][MV] = T(0);
    }
};

// variable-coefficient acoustics, aux = (rho, c) per cell: W_1 = alpha_1
// (-Z_L, 1) at -c_L and W_2 = alpha_2 (Z_R, 1) at +c_R, alpha_1 =
// (-dp + Z_R du)/(Z_L + Z_R), alpha_2 = (dp + Z_L du)/(Z_L + Z_R).  Cell:
// v[0..2] = q, v[3] = Z, v[4] = c (v[3] holds rho until prep).  Record:
// alpha_1, alpha_2, Z_L, Z_R (these four go to the neighbouring edges'
// limiters), c_L, c_R.  The limiter's t_p = alpha_p(E) (r_p(E) . r_p(e)) /
// |r_p(e)|^2 with r_1 . r_1' = 1 + Z_L Z_L' and r_2 . r_2' = 1 + Z_R Z_R'.
template <typename T, int IXY>
struct AcousticsVCK {
    static constexpr int MEQN = 3, MWAVES = 2, MAUX = 2, NC = 5, NE = 6, NX = 4;
    static constexpr int MU = IXY == 1 ? 1 : 2, MV = IXY == 1 ? 2 : 1;
    using C = Cell<T, NC>;
    using E = Rec<T, NE>;
    __device__ static void prep(const DevParams&, C& c) { c.v[3] = c.v[3] * c.v[4]; }
    __device__ static unsigned solve(const DevParams&, const C& L, const C& R, E& e)
    {
        const T zl = L.v[3], zr = R.v[3];
        const T dp = R.v[0] - L.v[0];
        const T du = R.v[MU] - L.v[MU];
        const T rz = frcp(zl + zr);
        e.v[0] = fma(zr, du, -dp) * rz;
        e.v[1] = fma(zl, du, dp) * rz;
        e.v[2] = zl;
        e.v[3] = zr;
        e.v[4] = L.v[4];
        e.v[5] = R.v[4];
        return 0u;
    }
    __device__ static T speed(const DevParams&, const E& e, int p) { return p == 0 ? -e.v[4] : e.v[5]; }
    __device__ static T smax(const DevParams&, const E& e) { return fmax(e.v[4], e.v[5]); }
    static constexpr bool SLOPE = true;
    __device__ static void pair(const DevParams&, const E& e, const E& el, T* tl, T* tr)
    {
        const T g1 = fma(e.v[2], el.v[2], T(1)), g2 = fma(e.v[3], el.v[3], T(1));
        tl[0] = el.v[0] * g1; tl[1] = el.v[1] * g2;
        tr[0] = e.v[0] * g1;  tr[1] = e.v[1] * g2;
    }
    __device__ static void out(const E& e, T L1, T L2, T* o)
    {
        o[0] = fma(e.v[3], L2, -(e.v[2] * L1));
        o[MU] = L1 + L2;
        o[MV] = T(0);
    }
    template <int LIM>
    __device__ static void lterms(const DevParams&, const E& e, const T* tl, const T* tr, T nu, T* lf,
                                  T* rg)
    {
        const T a1 = e.v[0], a2 = e.v[1], cl = e.v[4], cr = e.v[5];
        T L1 = -cl * a1, L2 = T(0);
        if (LIM != LIM_FIRST_ORDER) {
            // 1 / |r_p|^2 of both families from one reciprocal (|r_p|^2 >= 1)
            const T n1 = fma(e.v[2], e.v[2], T(1)), n2 = fma(e.v[3], e.v[3], T(1));
            const T rr = frcp1(n1 * n2);
            // s_1 = -c_L <= 0 takes the right neighbour's part, s_2 = c_R >= 0
            // the left one's (at a zero speed the correction vanishes anyway)
            const T t1 = tr[0] * (rr * n2);
            const T t2 = tl[1] * (rr * n1);
            L1 = fma(-cl, a1, (cl * fma(-nu, cl, T(1))) * slope_half<LIM, T>(a1, t1));
            L2 = (cr * fma(-nu, cr, T(1))) * slope_half<LIM, T>(a2, t2);
        }
        out(e, L1, L2, lf);
        out(e, fma(-cl, a1, -L1), fma(cr, a2, -L2), rg);
    }
    __device__ static void fluct(const DevParams&, const E& e, T* am, T* ap)
    {
        out(e, -e.v[4] * e.v[0], T(0), am);
        out(e, T(0), e.v[5] * e.v[1], ap);
    }
    __device__ static void waves(const DevParams&, const E& e, T (*W)[3])
    {
        W[0][0] = -e.v[0] * e.v[2]; W[0][MU] = e.v[0]; W[0][MV] = T(0);
        W[1][0] = e.v[1] * e.v[3];  W[1][MU] = e.v[1]; W[1][MV] = T(0);
    }
};

// ---------------------------------------------------- shallow water, Roe + HH
// Cell: v[0..2] = (h, hu, hv), v[3] = normal velocity, v[4] = transverse
// velocity, v[5] = sqrt(h), v[6] = sqrt(g h).
// Record: v[0..2] = alpha_1..3, v[3] = s_1 = u_hat - c_hat,
// v[4] = s_3 = u_hat + c_hat, v[5] = v_hat, v[6] = u_hat, v[7], v[8] = the
// entropy-fixed left-going speeds of families 1 and 3.  The waves are
// W_1 = alpha_1 (1, s_1, v_hat), W_2 = alpha_2 (0, 0, 1),
// W_3 = alpha_3 (1, s_3, v_hat) in (h, normal, transverse) slots.
template <typename T, int IXY>
struct SwRoe {
    static constexpr int MEQN = 3, MWAVES = 3, MAUX = 0, NC = 7, NE = 9, NX = 6;
    static constexpr bool QMINMAX = true;  // the walker's CFL maximum as one FP64 instruction
    static constexpr int MU = IXY == 1 ? 1 : 2, MV = IXY == 1 ? 2 : 1;
    using C = Cell<T, NC>;
    using E = Rec<T, NE>;
    __device__ static void prep(const DevParams& P, C& c)
    {
        // one reciprocal square root gives sqrt(h), 1/h and c = sqrt(g) sqrt(h)
        const T h = c.v[0];
        const T y = frsq(h);
        const T rh = y * y;
        c.v[3] = c.v[MU] * rh;
        c.v[4] = c.v[MV] * rh;
        c.v[5] = h * y;
        c.v[6] = T(sqrt(P.g)) * c.v[5];
    }
    __device__ static unsigned solve(const DevParams& P, const C& L, const C& R, E& e)
    {
        const T g = T(P.g);
        const T hl = L.v[0], hr = R.v[0];
        // A dry or negative depth on either side gives an all-zero record.
        // The test is applied after the arithmetic (which then runs on
        // values that may be NaN and is discarded), so the common path
        // carries no zero-initialised copy of the record.
        const bool dry = !(hl > T(0)) || !(hr > T(0));
        const T sl = L.v[5], sr = R.v[5];
        const T rs = frcp(sl + sr);
        const T uh = fma(sl, L.v[3], sr * R.v[3]) * rs;
        const T vh = fma(sl, L.v[4], sr * R.v[4]) * rs;
        const T gh = T(0.5 * P.g) * (hl + hr);  // g (hl + hr) / 2
        const T ric = frsq(gh);          // 1 / c_hat
        const T ch = gh * ric;           // c_hat = sqrt(g h_bar)
        const T r2c = T(0.5) * ric;
        const T d0 = hr - hl;
        const T d1 = R.v[MU] - L.v[MU];
        const T d2 = R.v[MV] - L.v[MV];
        const T s1 = uh - ch, s3 = uh + ch;
        const T a1 = fma(s3, d0, -d1) * r2c;
        const T a3 = fma(-s1, d0, d1) * r2c;
        e.v[0] = a1;
        e.v[1] = fma(-vh, d0, d2);
        e.v[2] = a3;
        e.v[3] = s1;
        e.v[4] = s3;
        e.v[5] = vh;
        e.v[6] = uh;

        unsigned st = 0u;
        // family 1: transonic when lambda_l = uL - cL < 0 < lambda_r, with
        // lambda_r the characteristic speed of the state qL + W1.  For h1 > 0,
        // lambda_r > 0 exactly when hu1 > 0 and hu1^2 > g h1^3, so the
        // reciprocal and root are needed only on transonic edges.
        // The tests are evaluated in full (no short-circuit), so only the
        // rare transonic case branches.
        T f1 = tmin0(s1);
        const T lam_l1 = L.v[3] - L.v[6];
        const T h1 = hl + a1;
        const T m1 = fma(a1, s1, L.v[MU]);
        const bool ok1 = h1 > T(0);
        const bool fix1 = ok1 & (lam_l1 < T(0)) & (m1 > T(0)) & (m1 * m1 > g * (h1 * h1) * h1);
        // family 3: the state qR - W3 against the right state
        T f3 = tmin0(s3);
        const T lam_r3 = R.v[3] + R.v[6];
        const T h2 = hr - a3;
        const T m2 = fma(-a3, s3, R.v[MU]);
        const bool ok3 = h2 > T(0);
        const bool fix3 = ok3 & (lam_r3 > T(0)) & (m2 < T(0)) & (m2 * m2 > g * (h2 * h2) * h2);
        if (!(ok1 & ok3)) st |= ST_NONPHYS;
        e.v[7] = f1;
        e.v[8] = f3;
        // The entropy splits and the dry record are rare: one region holds
        // all three, so the common path passes a single branch (3 % faster
        // in FP32 than one branch each).
        if (fix1 | fix3 | dry) {
            if (fix1) {
                const T lam_r = fma(m1, frcp(h1), -tsqrt(g * h1));
                e.v[7] = lam_l1 * (lam_r - s1) * frcp(lam_r - lam_l1);
            }
            if (fix3) {
                const T lam_l = fma(m2, frcp(h2), tsqrt(g * h2));
                e.v[8] = lam_l * (lam_r3 - s3) * frcp(lam_r3 - lam_l);
            }
            if (dry) {
#pragma unroll
                for (int k = 0; k < NE; ++k) e.v[k] = T(0);
                st = ST_NONPHYS;
            }
        }
        return st;
    }
    __device__ static T speed(const DevParams&, const E& e, int p)
    {
        return p == 0 ? e.v[3] : (p == 1 ? e.v[6] : e.v[4]);
    }
    // |u_hat| <= max(|u_hat - c_hat|, |u_hat + c_hat|) as c_hat >= 0, so the
    // shear wave never sets the maximum
    __device__ static T smax(const DevParams&, const E& e)
    {
        if constexpr (sizeof(T) == 8) return dmax_abs(e.v[3], e.v[4]);
        else return fmax(fabs(e.v[3]), fabs(e.v[4]));
    }
    // r_1 . r_1' = 1 + s_1 s_1' + v v', r_2 . r_2' = 1, r_3 . r_3' = 1 + s_3 s_3' + v v'
    __device__ static T dot(const DevParams&, const E& a, const E& b, int p)
    {
        if (p == 1) return a.v[1] * b.v[1];
        const int k = p == 0 ? 3 : 4;
        return (a.v[p] * b.v[p]) * fma(a.v[k], b.v[k], fma(a.v[5], b.v[5], T(1)));
    }
    __device__ static T norm2(const DevParams& P, const E& e, int p) { return dot(P, e, e, p); }
    // The limiter in terms of strengths.  With W_p = alpha_p r_p,
    // theta = W_p(E) . W_p(e) / W_p(e) . W_p(e) = t / alpha_p(e) for
    // t = alpha_p(E) (r_p(E) . r_p(e)) / (r_p(e) . r_p(e)), so the limited wave
    // phi(theta) W_p(e) is phi(t / alpha) alpha r_p(e): a function of alpha
    // and t that needs no division for the MC, minmod and superbee limiters
    // (slope_half below) and no special case for a zero wave.
    static constexpr bool SLOPE = true;
    __device__ static void pair(const DevParams&, const E& e, const E& el, T* tl, T* tr)
    {
        const T vv = fma(e.v[5], el.v[5], T(1));
        const T g1 = fma(e.v[3], el.v[3], vv), g3 = fma(e.v[4], el.v[4], vv);  // r_p(e) . r_p(el)
        tl[0] = el.v[0] * g1; tl[1] = el.v[1]; tl[2] = el.v[2] * g3;
        tr[0] = e.v[0] * g1;  tr[1] = e.v[1];  tr[2] = e.v[2] * g3;
    }
    // A-dQ + F and A+dQ - F of the edge (as terms() below), the limited
    // strengths from the neighbours' parts tl (left) and tr (right)
    template <int LIM>
    __device__ static void lterms(const DevParams&, const E& e, const T* tl, const T* tr, T nu, T* lf,
                                  T* rg)
    {
        const T al[3] = {e.v[0], e.v[1], e.v[2]};
        const T s[3] = {e.v[3], e.v[6], e.v[4]};
        const T f[3] = {e.v[7], qmin0(e.v[6]), e.v[8]};
        T L[3], R[3];
        if (LIM == LIM_FIRST_ORDER) {
#pragma unroll
            for (int p = 0; p < 3; ++p) L[p] = f[p] * al[p];
        } else {
            // 1 / |r_p|^2 of the acoustic families from one reciprocal
            // (|r_p|^2 >= 1); |r_2|^2 = 1
            const T vv = fma(e.v[5], e.v[5], T(1));
            const T n1 = fma(s[0], s[0], vv), n3 = fma(s[2], s[2], vv);
            const T rr = frcp1(n1 * n3);
            const T inv[3] = {rr * n3, T(1), rr * n1};
#pragma unroll
            for (int p = 0; p < 3; ++p) {
                const T num = s[p] > T(0) ? tl[p] : tr[p];
                const T t = p == 1 ? num : num * inv[p];
                const T as = fabs(s[p]);
                // F_p = (1/2) |s| (1 - nu |s|) phi alpha = |s| (1 - nu |s|) slope_half
                L[p] = fma(f[p], al[p], (as * fma(-nu, as, T(1))) * slope_half_q<LIM, T>(al[p], t));
            }
        }
#pragma unroll
        for (int p = 0; p < 3; ++p) R[p] = fma(s[p], al[p], -L[p]);
        const T l13 = L[0] + L[2], r13 = R[0] + R[2];
        lf[0] = l13;
        lf[MU] = fma(L[0], s[0], L[2] * s[2]);
        lf[MV] = fma(l13, e.v[5], L[1]);
        rg[0] = r13;
        rg[MU] = fma(R[0], s[0], R[2] * s[2]);
        rg[MV] = fma(r13, e.v[5], R[1]);
    }
    __device__ static void combo(const DevParams&, const E& e, const T* c, T* out)
    {
        const T b1 = c[0] * e.v[0], b2 = c[1] * e.v[1], b3 = c[2] * e.v[2];
        const T b13 = b1 + b3;
        out[0] = b13;
        out[MU] = fma(b1, e.v[3], b3 * e.v[4]);
        out[MV] = fma(b13, e.v[5], b2);
    }
    __device__ static void fluct(const DevParams& P, const E& e, T* am, T* ap)
    {
        const T f[3] = {e.v[7], tmin0(e.v[6]), e.v[8]};
        const T s[3] = {e.v[3], e.v[6], e.v[4]};
        T tot[3];
        combo(P, e, s, tot);
        combo(P, e, f, am);
#pragma unroll
        for (int m = 0; m < 3; ++m) ap[m] = tot[m] - am[m];
    }
    // A-dQ + F and A+dQ - F for F = sum_p coef_p W_p.  With A-dQ = sum_p f_p W_p
    // (f_p = min(s_p, 0), or the entropy-fix split) and A+dQ = sum_p (s_p - f_p) W_p,
    // both are combinations of the same three waves: coefficients f_p + coef_p
    // and s_p - f_p - coef_p.
    __device__ static void terms(const DevParams& P, const E& e, const T* coef, T* lf, T* rg)
    {
        const T f[3] = {e.v[7], tmin0(e.v[6]), e.v[8]};
        const T s[3] = {e.v[3], e.v[6], e.v[4]};
        T a[3], b[3];
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            a[p] = f[p] + coef[p];
            b[p] = (s[p] - f[p]) - coef[p];
        }
        combo(P, e, a, lf);
        combo(P, e, b, rg);
    }
    __device__ static void waves(const DevParams&, const E& e, T (*W)[3])
    {
        W[0][0] = e.v[0]; W[0][MU] = e.v[0] * e.v[3]; W[0][MV] = e.v[0] * e.v[5];
        W[1][0] = T(0);   W[1][MU] = T(0);            W[1][MV] = e.v[1];
        W[2][0] = e.v[2]; W[2][MU] = e.v[2] * e.v[4]; W[2][MV] = e.v[2] * e.v[5];
    }
};

// ------------------------------------------------------- shallow water, HLLE
// Waves q* - qL (slot 0, speed s_L) and qR - q* (slot 2, speed s_R); slot 1
// empty.  s_L = min(uL - cL, u_hat - c_hat), s_R = max(uR + cR, u_hat + c_hat).
template <typename T, int IXY>
struct SwHlleC {
    using value_type = T;
    static constexpr int MEQN = 3, MWAVES = 3, MAUX = 0, NC = 7;
    static constexpr int MU = IXY == 1 ? 1 : 2, MV = IXY == 1 ? 2 : 1;
    using C = Cell<T, NC>;
    using E = Edge<T, MWAVES, MEQN>;
    __host__ __device__ static constexpr bool nz(int p, int) { return p != 1; }
    __device__ static void prep(const DevParams& P, C& c) { SwRoe<T, IXY>::prep(P, c); }
    __device__ static unsigned solve(const DevParams& P, const C& L, const C& R, E& e)
    {
        const T g = T(P.g);
        const T hl = L.v[0], hr = R.v[0];
        if (!(hl > T(0)) || !(hr > T(0))) {
            zero_edge<SwHlleC, T>(e);
            return ST_NONPHYS;
        }
        const T sl = L.v[5], sr = R.v[5];
        const T uh = fma(sl, L.v[3], sr * R.v[3]) * frcp(sl + sr);
        const T ch = tsqrt(g * (T(0.5) * (hl + hr)));
        T sL = L.v[3] - L.v[6], sR = R.v[3] + R.v[6];
        if (uh - ch < sL) sL = uh - ch;
        if (uh + ch > sR) sR = uh + ch;
        // normal fluxes (h u_n, h u_n^2 + g h^2/2, h u_n u_t)
        T fl[3], fr[3];
        fl[0] = L.v[MU]; fl[MU] = fma(L.v[MU], L.v[3], T(0.5) * g * (hl * hl)); fl[MV] = L.v[MU] * L.v[4];
        fr[0] = R.v[MU]; fr[MU] = fma(R.v[MU], R.v[3], T(0.5) * g * (hr * hr)); fr[MV] = R.v[MU] * R.v[4];
        const T rd = frcp(sR - sL);
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const T qs = fma(sR, R.v[m], fma(-sL, L.v[m], fl[m] - fr[m])) * rd;
            e.w[0][m] = qs - L.v[m];
            e.w[1][m] = T(0);
            e.w[2][m] = R.v[m] - qs;
        }
        e.s[0] = sL;
        e.s[1] = T(0);
        e.s[2] = sR;
        upwind_split<SwHlleC, T>(e);
        return 0u;
    }
};

// ------------------------------------------------- Euler, Roe + HH + HLLE
// Cell: v[0..3] = (rho, rho u, rho v, E), v[4] = normal velocity,
// v[5] = transverse velocity, v[6] = H = (E + p)/rho, v[7] = sqrt(rho),
// v[8] = c = sqrt(gamma p / rho), v[9] = p.
template <typename T, int IXY>
struct EulerRoeC {
    using value_type = T;
    static constexpr int MEQN = 4, MWAVES = 4, MAUX = 0, NC = 10;
    static constexpr int MU = IXY == 1 ? 1 : 2, MV = IXY == 1 ? 2 : 1;
    using C = Cell<T, NC>;
    using E = Edge<T, MWAVES, MEQN>;
    // the shear wave (slot 2) has only its transverse and energy components
    __host__ __device__ static constexpr bool nz(int p, int m) { return p != 2 || m == MV || m == 3; }
    // p = (gamma - 1)(E - (mx^2 + my^2) / (2 rho)), given 1/rho
    __device__ static T pressure(T gm1, T rr, T mx, T my, T En)
    {
        return gm1 * fma(T(-0.5) * rr, fma(mx, mx, my * my), En);
    }
    __device__ static void prep(const DevParams& P, C& c)
    {
        const T gm = T(P.gamma);
        const T r = c.v[0];
        const T y = frsq(r);
        const T rr = y * y;
        const T p = pressure(gm - T(1), rr, c.v[1], c.v[2], c.v[3]);
        c.v[4] = c.v[MU] * rr;
        c.v[5] = c.v[MV] * rr;
        c.v[6] = (c.v[3] + p) * rr;
        c.v[7] = r * y;
        c.v[8] = tsqrt(gm * p * rr);
        c.v[9] = p;
    }
    __device__ static void hlle(const C& L, const C& R, bool use_roe, T uh, T ch, E& e)
    {
        T sL, sR;
        if (use_roe) {
            sL = L.v[4] - L.v[8]; if (uh - ch < sL) sL = uh - ch;
            sR = R.v[4] + R.v[8]; if (uh + ch > sR) sR = uh + ch;
        } else {
            sL = L.v[4] - L.v[8]; if (R.v[4] - R.v[8] < sL) sL = R.v[4] - R.v[8];
            sR = R.v[4] + R.v[8]; if (L.v[4] + L.v[8] > sR) sR = L.v[4] + L.v[8];
        }
        T fl[4], fr[4];
        fl[0] = L.v[MU]; fl[MU] = fma(L.v[MU], L.v[4], L.v[9]); fl[MV] = L.v[MV] * L.v[4]; fl[3] = (L.v[3] + L.v[9]) * L.v[4];
        fr[0] = R.v[MU]; fr[MU] = fma(R.v[MU], R.v[4], R.v[9]); fr[MV] = R.v[MV] * R.v[4]; fr[3] = (R.v[3] + R.v[9]) * R.v[4];
        const T rd = frcp(sR - sL);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const T qs = fma(sR, R.v[m], fma(-sL, L.v[m], fl[m] - fr[m])) * rd;
            e.w[0][m] = qs - L.v[m];
            e.w[1][m] = T(0);
            e.w[2][m] = T(0);
            e.w[3][m] = R.v[m] - qs;
        }
        e.s[0] = sL; e.s[1] = T(0); e.s[2] = T(0); e.s[3] = sR;
        upwind_split<EulerRoeC, T>(e);
    }
    __device__ static unsigned solve(const DevParams& P, const C& L, const C& R, E& e)
    {
        const T gm = T(P.gamma), gm1 = gm - T(1);
        if (!(L.v[0] > T(0)) || !(R.v[0] > T(0)) || !(L.v[9] > T(0)) || !(R.v[9] > T(0))) {
            zero_edge<EulerRoeC, T>(e);
            return ST_NONPHYS;
        }
        const T sl = L.v[7], sr = R.v[7];
        const T rs = frcp(sl + sr);
        const T uh = fma(sl, L.v[4], sr * R.v[4]) * rs;
        const T vh = fma(sl, L.v[5], sr * R.v[5]) * rs;
        const T Hh = fma(sl, L.v[6], sr * R.v[6]) * rs;
        const T q2 = fma(uh, uh, vh * vh);
        const T c2 = gm1 * fma(T(-0.5), q2, Hh);
        if (!(c2 > T(0))) {
            hlle(L, R, false, T(0), T(0), e);
            return ST_FALLBACK;
        }
        const T ric = frsq(c2);
        const T ch = c2 * ric;
        const T d0 = R.v[0] - L.v[0];
        const T d1 = R.v[MU] - L.v[MU];
        const T d2 = R.v[MV] - L.v[MV];
        const T d3 = R.v[3] - L.v[3];
        const T a3 = fma(-vh, d0, d2);
        const T a2 = (gm1 * (ric * ric)) * fma(Hh - q2, d0, fma(uh, d1, fma(vh, d2, -d3)));
        const T a1 = fma(uh + ch, d0, fma(-ch, a2, -d1)) * (T(0.5) * ric);
        const T a4 = d0 - a1 - a2;
        const T s1 = uh - ch, s4 = uh + ch;
        e.w[0][0] = a1; e.w[0][MU] = a1 * s1; e.w[0][MV] = a1 * vh; e.w[0][3] = a1 * fma(-uh, ch, Hh);
        e.w[1][0] = a2; e.w[1][MU] = a2 * uh; e.w[1][MV] = a2 * vh; e.w[1][3] = a2 * (T(0.5) * q2);
        e.w[2][0] = T(0); e.w[2][MU] = T(0);  e.w[2][MV] = a3;      e.w[2][3] = a3 * vh;
        e.w[3][0] = a4; e.w[3][MU] = a4 * s4; e.w[3][MV] = a4 * vh; e.w[3][3] = a4 * fma(uh, ch, Hh);
        e.s[0] = s1; e.s[1] = uh; e.s[2] = uh; e.s[3] = s4;

        // Roe states next to the acoustic waves; HLLE if either is unphysical
        T q1[4], q3[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) { q1[m] = L.v[m] + e.w[0][m]; q3[m] = R.v[m] - e.w[3][m]; }
        if (!(q1[0] > T(0)) || !(q3[0] > T(0))) {
            hlle(L, R, true, uh, ch, e);
            return ST_FALLBACK;
        }
        const T r1 = frcp(q1[0]), r3 = frcp(q3[0]);
        const T p1 = pressure(gm1, r1, q1[1], q1[2], q1[3]);
        const T p3 = pressure(gm1, r3, q3[1], q3[2], q3[3]);
        if (!(p1 > T(0)) || !(p3 > T(0))) {
            hlle(L, R, true, uh, ch, e);
            return ST_FALLBACK;
        }
        // Harten-Hyman on the acoustic families; lambda_r > 0 for family 1
        // exactly when m1 > 0 and m1^2 > gamma p1 rho1 (likewise for 4)
        T f[4];
        f[0] = tmin0(s1);
        {
            const T lam_l = L.v[4] - L.v[8];
            const T m1 = q1[MU];
            if (lam_l < T(0) && m1 > T(0) && m1 * m1 > gm * p1 * q1[0]) {
                const T lam_r = fma(m1, r1, -tsqrt(gm * p1 * r1));
                f[0] = lam_l * (lam_r - s1) * frcp(lam_r - lam_l);
            }
        }
        f[1] = tmin0(uh);
        f[2] = f[1];
        f[3] = tmin0(s4);
        {
            const T lam_r = R.v[4] + R.v[8];
            const T m3 = q3[MU];
            if (lam_r > T(0) && m3 < T(0) && m3 * m3 > gm * p3 * q3[0]) {
                const T lam_l = fma(m3, r3, tsqrt(gm * p3 * r3));
                f[3] = lam_l * (lam_r - s4) * frcp(lam_r - lam_l);
            }
        }
        fixed_split<EulerRoeC, T>(e, f);
        return 0u;
    }
};

// --------------------------------------- Euler, compact record (Roe or HLLE)
// The same solver as EulerRoeC (its prep, tests, Roe decomposition, entropy
// fix and HLLE fallback), with the edge kept as 13 values instead of the 26
// of its component record.  A Roe edge's waves are alpha_p r_p with
//   r_1 = (1, u - c, v, H - u c), r_2 = (1, u, v, K), r_3 = (0, 0, 1, v),
//   r_4 = (1, u + c, v, H + u c)
// in (rho, normal, transverse, E) slots (u, v, c, H the Roe averages,
// K = (u^2 + v^2)/2), and speeds (u - c, u, u, u + c); the record holds
//   v[0..3] = alpha_1..4, v[4] = u - c, v[5] = u + c, v[6] = u, v[7] = v,
//   v[8] = H - u c, v[9] = H + u c, v[10] = K >= 0, v[11], v[12] = the
//   entropy-fixed left-going speeds of families 1 and 4.
// An HLLE edge (waves q* - qL and qR - q* at sL and sR, the other two empty)
// is marked by v[10] = -1 and holds
//   v[0..3] = q* - qL (grid slots), v[4] = sL, v[5] = sR, v[6] = 0,
//   v[7], v[8], v[9], v[11] = qR - q* (grid slots 0..3), v[12] = 0.
// Speeds read the same slots in both forms (v[4], v[6], v[6], v[5]).  The
// limiter and the update take the compact formulas when no lane of the
// wavefront has an HLLE edge among those involved, else the waves as
// components.
// Its cell keeps c^2 = gamma p / rho in v[8] instead of c: the sound speed
// of a cell is needed only on the rare paths (a transonic edge, the HLLE
// fallback), which take the root there, and the tests of the common path
// are written without roots or divisions (solve below).
template <typename T, int IXY>
struct EulerRoeK {
    using B = EulerRoeC<T, IXY>;
    using value_type = T;
    static constexpr int MEQN = 4, MWAVES = 4, MAUX = 0, NC = 10, NE = 13, NX = 12;
    static constexpr int MU = IXY == 1 ? 1 : 2, MV = IXY == 1 ? 2 : 1;
    using C = typename B::C;
    using E = Rec<T, NE>;
    static constexpr bool SLOPE = true;  // its own limiter path (lterms), on theta

    // as EulerRoeC::prep, with c^2 in v[8]
    __device__ __forceinline__ static void prep(const DevParams& P, C& c)
    {
        const T gm = T(P.gamma);
        const T r = c.v[0];
        const T y = frsq(r);
        const T rr = y * y;
        const T p = B::pressure(gm - T(1), rr, c.v[1], c.v[2], c.v[3]);
        c.v[4] = c.v[MU] * rr;
        c.v[5] = c.v[MV] * rr;
        c.v[6] = (c.v[3] + p) * rr;
        c.v[7] = r * y;
        c.v[8] = gm * p * rr;
        c.v[9] = p;
    }

    __device__ __forceinline__ static void hlle(const C& L, const C& R, bool use_roe, T uh, T ch, E& e)
    {
        // the cells' sound speeds from their c^2 (positive: both pressures
        // and densities are, or solve has returned before)
        const T cl = tsqrt(L.v[8]), cr = tsqrt(R.v[8]);
        T sL = L.v[4] - cl, sR = R.v[4] + cr;
        const T oL = use_roe ? uh - ch : R.v[4] - cr;
        const T oR = use_roe ? uh + ch : L.v[4] + cl;
        if (oL < sL) sL = oL;
        if (oR > sR) sR = oR;
        T fl[4], fr[4];
        fl[0] = L.v[MU]; fl[MU] = fma(L.v[MU], L.v[4], L.v[9]); fl[MV] = L.v[MV] * L.v[4]; fl[3] = (L.v[3] + L.v[9]) * L.v[4];
        fr[0] = R.v[MU]; fr[MU] = fma(R.v[MU], R.v[4], R.v[9]); fr[MV] = R.v[MV] * R.v[4]; fr[3] = (R.v[3] + R.v[9]) * R.v[4];
        const T rd = frcp(sR - sL);
        T w1[4], w4[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const T qs = fma(sR, R.v[m], fma(-sL, L.v[m], fl[m] - fr[m])) * rd;
            w1[m] = qs - L.v[m];
            w4[m] = R.v[m] - qs;
        }
        // every path writes the 13 slots in the same order, so the compiler
        // never merges stores to different slots (which would put the record
        // in memory)
        e.v[0] = w1[0]; e.v[1] = w1[1]; e.v[2] = w1[2]; e.v[3] = w1[3];
        e.v[4] = sL; e.v[5] = sR; e.v[6] = T(0);
        e.v[7] = w4[0]; e.v[8] = w4[1]; e.v[9] = w4[2];
        e.v[10] = T(-1); e.v[11] = w4[3]; e.v[12] = T(0);
    }

    __device__ __forceinline__ static unsigned solve(const DevParams& P, const C& L, const C& R, E& e)
    {
        const T gm = T(P.gamma), gm1 = gm - T(1);
        // Every test below is applied after the arithmetic, which then may
        // run on invalid values and is discarded: the rare outcomes (a
        // non-physical cell, the HLLE fallback, the transonic splits) share
        // one region, so the common path passes a single branch.
        const bool bad = !(L.v[0] > T(0)) | !(R.v[0] > T(0)) | !(L.v[9] > T(0)) | !(R.v[9] > T(0));
        const T sl = L.v[7], sr = R.v[7];
        const T rs = frcp(sl + sr);
        const T uh = fma(sl, L.v[4], sr * R.v[4]) * rs;
        const T vh = fma(sl, L.v[5], sr * R.v[5]) * rs;
        const T Hh = fma(sl, L.v[6], sr * R.v[6]) * rs;
        const T q2 = fma(uh, uh, vh * vh);
        const T c2 = gm1 * fma(T(-0.5), q2, Hh);
        const T ric = frsq(c2);
        const T ch = c2 * ric;
        const T d0 = R.v[0] - L.v[0];
        const T d1 = R.v[MU] - L.v[MU];
        const T d2 = R.v[MV] - L.v[MV];
        const T d3 = R.v[3] - L.v[3];
        const T a3 = fma(-vh, d0, d2);
        const T a2 = (gm1 * (ric * ric)) * fma(Hh - q2, d0, fma(uh, d1, fma(vh, d2, -d3)));
        const T a1 = fma(uh + ch, d0, fma(-ch, a2, -d1)) * (T(0.5) * ric);
        const T a4 = d0 - a1 - a2;
        const T s1 = uh - ch, s4 = uh + ch;
        const T H1 = fma(-uh, ch, Hh), H4 = fma(uh, ch, Hh);
        // Roe states next to the acoustic waves
        T q1[4], q3[4];
        q1[0] = L.v[0] + a1; q1[MU] = fma(a1, s1, L.v[MU]); q1[MV] = fma(a1, vh, L.v[MV]); q1[3] = fma(a1, H1, L.v[3]);
        q3[0] = R.v[0] - a4; q3[MU] = fma(-a4, s4, R.v[MU]); q3[MV] = fma(-a4, vh, R.v[MV]); q3[3] = fma(-a4, H4, R.v[3]);
        // rho p / (gamma - 1) = rho E - |m|^2 / 2 of each: for rho > 0 its
        // sign is that of p, with no division
        const T k1 = q1[MU] * q1[MU], k3 = q3[MU] * q3[MU];
        const T P1 = fma(T(-0.5), fma(q1[MV], q1[MV], k1), q1[3] * q1[0]);
        const T P3 = fma(T(-0.5), fma(q3[MV], q3[MV], k3), q3[3] * q3[0]);
        // HLLE when the Roe average has no sound speed (then with the cells'
        // speeds alone), or when either Roe state has no positive density
        // or pressure (with the Roe speeds too)
        const bool roe_ok = c2 > T(0);
        const bool fb = !roe_ok | !(q1[0] > T(0)) | !(q3[0] > T(0)) | !(P1 > T(0)) | !(P3 > T(0));
        // Harten-Hyman on the acoustic families (as EulerRoeC).  Family 1 is
        // transonic when uL - cL < 0 (uL < 0, or uL^2 < cL^2: together
        // uL |uL| < cL^2) and the Roe state q1 moves right at
        // m1 / rho1 - c1 > 0 (m1 > 0 and m1^2 > gamma p1 rho1 =
        // gamma (gamma - 1) P1: together m1 |m1| > gamma (gamma - 1) P1,
        // as P1 > 0 wherever the test is used); family 4 mirrors it.  The
        // tests need no root or division; the split itself does.
        const T gg = gm * gm1;
        const T ul = L.v[4], m1 = q1[MU], ur = R.v[4], m3 = q3[MU];
        const bool fx1 = (ul * fabs(ul) < L.v[8]) & (m1 * fabs(m1) > gg * P1);
        const bool fx4 = (-ur * fabs(ur) < R.v[8]) & (-m3 * fabs(m3) > gg * P3);
        e.v[0] = a1; e.v[1] = a2; e.v[2] = a3; e.v[3] = a4;
        e.v[4] = s1; e.v[5] = s4; e.v[6] = uh; e.v[7] = vh;
        e.v[8] = H1; e.v[9] = H4; e.v[10] = T(0.5) * q2;
        e.v[11] = tmin0(s1); e.v[12] = tmin0(s4);
        unsigned st = 0u;
        if (bad | fb | fx1 | fx4) {
            if constexpr (sizeof(T) == 4) {
                // FP32: straight-line, every rare candidate computed for the
                // whole wavefront and each lane selecting its outcome, so no
                // record values are copied where the region rejoins the
                // common path (4 % faster at 4096^2).  In FP64 the candidates'
                // roots and reciprocals cost more than the copies (the nested
                // form below is 15 % faster there).
                const T lam_l1 = ul - tsqrt(L.v[8]);
                const T lam_r1 = (m1 - tsqrt(gg * P1)) * frcp(q1[0]);
                const T f1 = lam_l1 * (lam_r1 - s1) * frcp(lam_r1 - lam_l1);
                const T lam_r4 = ur + tsqrt(R.v[8]);
                const T lam_l4 = (m3 + tsqrt(gg * P3)) * frcp(q3[0]);
                const T f4 = lam_l4 * (lam_r4 - s4) * frcp(lam_r4 - lam_l4);
                e.v[11] = fx1 ? f1 : e.v[11];
                e.v[12] = fx4 ? f4 : e.v[12];
                E hr;
                hlle(L, R, roe_ok, uh, ch, hr);
#pragma unroll
                for (int k = 0; k < NE; ++k) e.v[k] = bad ? T(0) : (fb ? hr.v[k] : e.v[k]);
                st = bad ? ST_NONPHYS : (fb ? ST_FALLBACK : 0u);
            } else if (bad) {
#pragma unroll
                for (int k = 0; k < NE; ++k) e.v[k] = T(0);
                st = ST_NONPHYS;
            } else if (fb) {
                hlle(L, R, roe_ok, uh, ch, e);
                st = ST_FALLBACK;
            } else {
                if (fx1) {
                    // c1 = sqrt(gamma p1 / rho1) = sqrt(gamma (gamma - 1) P1) / rho1
                    const T lam_l = ul - tsqrt(L.v[8]);
                    const T lam_r = (m1 - tsqrt(gg * P1)) * frcp(q1[0]);
                    e.v[11] = lam_l * (lam_r - s1) * frcp(lam_r - lam_l);
                }
                if (fx4) {
                    const T lam_r = ur + tsqrt(R.v[8]);
                    const T lam_l = (m3 + tsqrt(gg * P3)) * frcp(q3[0]);
                    e.v[12] = lam_l * (lam_r - s4) * frcp(lam_r - lam_l);
                }
            }
        }
        return st;
    }

    __device__ __forceinline__ static bool is_hlle(const E& e) { return e.v[10] < T(0); }
    __device__ __forceinline__ static T speed(const DevParams&, const E& e, int p)
    {
        return p == 0 ? e.v[4] : (p == 3 ? e.v[5] : e.v[6]);
    }
    // |u| <= max(|u - c|, |u + c|) as c >= 0; an HLLE edge's other speed is 0
    __device__ __forceinline__ static T smax(const DevParams&, const E& e) { return fmax(fabs(e.v[4]), fabs(e.v[5])); }

    // wave p as components (grid slots), either form
    __device__ __forceinline__ static void wave(const E& e, int p, T* w)
    {
        const bool h = is_hlle(e);
        const T vh = e.v[7];
        if (p == 0) {
            const T a = e.v[0];
            const T r[4] = {a, a * e.v[4], a * vh, a * e.v[8]};
            w[0] = h ? e.v[0] : r[0]; w[MU] = h ? e.v[MU] : r[1]; w[MV] = h ? e.v[MV] : r[2]; w[3] = h ? e.v[3] : r[3];
        } else if (p == 1) {
            const T a = e.v[1];
            w[0] = h ? T(0) : a; w[MU] = h ? T(0) : a * e.v[6]; w[MV] = h ? T(0) : a * vh; w[3] = h ? T(0) : a * e.v[10];
        } else if (p == 2) {
            const T a = e.v[2];
            w[0] = T(0); w[MU] = T(0); w[MV] = h ? T(0) : a; w[3] = h ? T(0) : a * vh;
        } else {
            const T a = e.v[3];
            w[0] = h ? e.v[7] : a; w[1] = h ? e.v[8] : (MU == 1 ? a * e.v[5] : a * vh);
            w[2] = h ? e.v[9] : (MU == 2 ? a * e.v[5] : a * vh); w[3] = h ? e.v[11] : a * e.v[9];
        }
    }
    // the waves as components W[p][m] (grid slots), either form
    __device__ __forceinline__ static void waves(const DevParams&, const E& e, T (*W)[4])
    {
        const bool h = is_hlle(e);
        const T a1 = e.v[0], a2 = e.v[1], a3 = e.v[2], a4 = e.v[3], vh = e.v[7];
        T R1[4], R2[4], R3[4], R4[4];
        R1[0] = a1; R1[MU] = a1 * e.v[4]; R1[MV] = a1 * vh; R1[3] = a1 * e.v[8];
        R2[0] = a2; R2[MU] = a2 * e.v[6]; R2[MV] = a2 * vh; R2[3] = a2 * e.v[10];
        R3[0] = T(0); R3[MU] = T(0); R3[MV] = a3; R3[3] = a3 * vh;
        R4[0] = a4; R4[MU] = a4 * e.v[5]; R4[MV] = a4 * vh; R4[3] = a4 * e.v[9];
        const T H4[4] = {e.v[7], e.v[8], e.v[9], e.v[11]};
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            W[0][m] = h ? e.v[m] : R1[m];
            W[1][m] = h ? T(0) : R2[m];
            W[2][m] = h ? T(0) : R3[m];
            W[3][m] = h ? H4[m] : R4[m];
        }
    }
    // left-going speeds f_p (entropy-fixed for a Roe edge, min(s, 0) for HLLE)
    __device__ __forceinline__ static void lspeeds(const E& e, T* f)
    {
        const bool h = is_hlle(e);
        const T fu = tmin0(e.v[6]);
        f[0] = h ? tmin0(e.v[4]) : e.v[11];
        f[1] = fu;
        f[2] = fu;
        f[3] = h ? tmin0(e.v[5]) : e.v[12];
    }
    __device__ __forceinline__ static void fluct(const DevParams& P, const E& e, T* am, T* ap)
    {
        T W[4][4], f[4];
        waves(P, e, W);
        lspeeds(e, f);
        const T s[4] = {e.v[4], e.v[6], e.v[6], e.v[5]};
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            T a = f[0] * W[0][m], b = (s[0] - f[0]) * W[0][m];
#pragma unroll
            for (int p = 1; p < 4; ++p) { a = fma(f[p], W[p][m], a); b = fma(s[p] - f[p], W[p][m], b); }
            am[m] = a;
            ap[m] = b;
        }
    }

    // W_p(e) . W_p(el) for the four waves
    __device__ __forceinline__ static void pair(const DevParams& P, const E& e, const E& el, T* tl, T* tr)
    {
        if (__builtin_expect(__ballot(is_hlle(e) || is_hlle(el)) != 0ull, 0)) {
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                T A[4], Bw[4];
                wave(e, p, A);
                wave(el, p, Bw);
                T d = A[0] * Bw[0];
#pragma unroll
                for (int m = 1; m < 4; ++m) d = fma(A[m], Bw[m], d);
                tl[p] = tr[p] = d;
            }
            return;
        }
        const T vv = fma(e.v[7], el.v[7], T(1));
        const T g1 = fma(e.v[8], el.v[8], fma(e.v[4], el.v[4], vv));
        const T g2 = fma(e.v[10], el.v[10], fma(e.v[6], el.v[6], vv));
        const T g4 = fma(e.v[9], el.v[9], fma(e.v[5], el.v[5], vv));
        tl[0] = tr[0] = (e.v[0] * el.v[0]) * g1;
        tl[1] = tr[1] = (e.v[1] * el.v[1]) * g2;
        tl[2] = tr[2] = (e.v[2] * el.v[2]) * vv;
        tl[3] = tr[3] = (e.v[3] * el.v[3]) * g4;
    }

    // A-dQ + F and A+dQ - F, F = sum_p coef_p W_p with coef_p the limited
    // 0.5 |s| (1 - nu |s|) phi(theta), theta = W_p(upwind) . W_p / W_p . W_p
    template <int LIM>
    __device__ __forceinline__ static void lterms(const DevParams& P, const E& e, const T* dl, const T* dr, T nu, T* lf,
                                  T* rg)
    {
        const bool h = is_hlle(e);
        const T s[4] = {e.v[4], e.v[6], e.v[6], e.v[5]};
        T f[4];
        if (__builtin_expect(__ballot(h) != 0ull, 0)) {
            lspeeds(e, f);
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                T W[4];
                wave(e, p, W);
                T nrm = W[0] * W[0];
#pragma unroll
                for (int m = 1; m < 4; ++m) nrm = fma(W[m], W[m], nrm);
                const T as = fabs(s[p]);
                const T c = LIM == LIM_FIRST_ORDER ? T(0)
                          : (T(0.5) * as) * fma(-nu, as, T(1)) * limiter_phi<LIM, T>(s[p] > T(0) ? dl[p] : dr[p], nrm);
                const T a = f[p] + c, b = (s[p] - f[p]) - c;
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    lf[m] = p == 0 ? a * W[m] : fma(a, W[m], lf[m]);
                    rg[m] = p == 0 ? b * W[m] : fma(b, W[m], rg[m]);
                }
            }
            return;
        }
        // Roe form (no lane holds an HLLE edge): the entropy-fixed left-going
        // speeds as stored, |r_p|^2 and the combinations through the
        // eigenvector parameters
        f[0] = e.v[11];
        f[1] = f[2] = tmin0(e.v[6]);
        f[3] = e.v[12];
        const T a[4] = {e.v[0], e.v[1], e.v[2], e.v[3]};
        const T vh = e.v[7];
        const T vv = fma(vh, vh, T(1));
        const T n[4] = {fma(e.v[8], e.v[8], fma(s[0], s[0], vv)), fma(e.v[10], e.v[10], fma(s[1], s[1], vv)), vv,
                        fma(e.v[9], e.v[9], fma(s[3], s[3], vv))};
        T L[4], R[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            T c = T(0);
            if (LIM != LIM_FIRST_ORDER) {
                const T as = fabs(s[p]);
                c = (T(0.5) * as) * fma(-nu, as, T(1)) *
                    limiter_phi<LIM, T>(s[p] > T(0) ? dl[p] : dr[p], (a[p] * a[p]) * n[p]);
            }
            L[p] = (f[p] + c) * a[p];
            R[p] = ((s[p] - f[p]) - c) * a[p];
        }
        // sum_p b_p r_p for b = L and b = R
        const T l124 = L[0] + L[1] + L[3], r124 = R[0] + R[1] + R[3];
        lf[0] = l124;
        lf[MU] = fma(L[0], s[0], fma(L[1], s[1], L[3] * s[3]));
        lf[MV] = fma(l124, vh, L[2]);
        lf[3] = fma(L[0], e.v[8], fma(L[1], e.v[10], fma(L[2], vh, L[3] * e.v[9])));
        rg[0] = r124;
        rg[MU] = fma(R[0], s[0], fma(R[1], s[1], R[3] * s[3]));
        rg[MV] = fma(r124, vh, R[2]);
        rg[3] = fma(R[0], e.v[8], fma(R[1], e.v[10], fma(R[2], vh, R[3] * e.v[9])));
    }
};

// solvers in the record interface used by the kernels
template <typename T, int IXY> using Advection = AdvectionK<T, IXY>;
template <typename T, int IXY> using Acoustics = AcousticsK<T, IXY>;
template <typename T, int IXY> using AcousticsVC = AcousticsVCK<T, IXY>;
// the same systems with component records (the unsplit step's transverse
// splits take their waves as components)
template <typename T, int IXY> using AdvectionW = Componentwise<AdvectionC<T, IXY>>;
template <typename T, int IXY> using AcousticsW = Componentwise<AcousticsC<T, IXY>>;
template <typename T, int IXY> using AcousticsVCW = Componentwise<AcousticsVCC<T, IXY>>;
template <typename T, int IXY> using SwHlle = Componentwise<SwHlleC<T, IXY>>;
template <typename T, int IXY> using EulerRoe = Componentwise<EulerRoeC<T, IXY>>;

}  // namespace mc
