// surrogate.hip -- learned normal Riemann solvers (shallow water, Euler) on
// gfx950: training-pair generation, BF16 matrix-core training (forward,
// backward, Adam) and the fused inference kernel that the split step uses in
// place of the Roe solve.
//
// The paper's method needs, at every cell edge, the waves, speeds and
// fluctuations of a normal Riemann problem (section 2, "Threading the
// Riemann solver"); the limiter and update around it are unchanged
// (section 1.2, Table 1).  Here a network stands in for that solve.  Per
// edge, in the normal frame (density or depth, normal momentum, transverse
// momentum[, energy]):
//   inputs    the states scaled by a reference density (depth) and sound
//             speed c0 of the edge's mean state, as mean velocities and the
//             scaled conserved jump m e (|e| = 1)
//   network   NIN-128-128-128-128-NOUT, GELU (tanh form) after hidden layers
//   outputs   K speeds (units c0) and K waves (units m x the scales), then
//             projected so that the fluctuations add up to f(qR) - f(qL)
//             shallow water: K = 2 (slots 0, 2); Euler: K = 3 (slots 0, 1, 3:
//             acoustic, entropy + shear, acoustic)
//   fallback  the plain solver (Roe + Harten-Hyman; HLLE where Roe fails) on
//             flagged edges (outside the training box, not subsonic on a
//             side, degenerate projection)
//
// Matrix-core layout (v_mfma_f32_16x16x32_bf16, wave64): an operand
// fragment gives each lane 8 bf16 (lane l: row or column l % 16, k-slots
// 8 (l / 16) .. + 7), the 16x16 FP32 result gives lane l column l % 16,
// rows 4 (l / 16) .. + 3.  The inference kernel computes each layer
// transposed, Z^T = W X^T: samples are columns, so a layer's result already
// sits in the lanes that feed the next layer's B operand, once the k-slots
// of the next layer's weights are permuted to match (slot j of lane group g
// in k-block kb holds neuron 32 kb + 4 g + j for j < 4 and
// 32 kb + 16 + 4 g + j - 4 for j >= 4).  Activations never leave registers;
// weights sit in LDS as ready-made fragments.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <vector>

#include "../../include/manyclaw.h"
#include "common.hpp"

namespace mc {
namespace sur {

typedef __bf16 bf16;
typedef bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int WID = 128, NLAYER = 5;

// network dimensions and the flat parameter layout: per layer W [out][in]
// row-major, then b [out]; BF16 training copies [out][inpad] layer by layer
template <int NIN_, int NOUT_>
struct Net {
    static constexpr int NIN = NIN_, NOUT = NOUT_;
    static_assert(NIN <= 8 && NOUT <= 16, "one k-slot group in, one fragment row block out");
    __host__ __device__ static constexpr int l_in(int l) { return l == 0 ? NIN : WID; }
    __host__ __device__ static constexpr int l_out(int l) { return l == NLAYER - 1 ? NOUT : WID; }
    __host__ __device__ static constexpr int l_inpad(int l) { return l == 0 ? 8 : WID; }
    __host__ __device__ static constexpr int w_off(int l)
    {
        return l == 0 ? 0 : w_off(l - 1) + l_out(l - 1) * l_in(l - 1) + l_out(l - 1);
    }
    __host__ __device__ static constexpr int b_off(int l) { return w_off(l) + l_out(l) * l_in(l); }
    __host__ __device__ static constexpr int t_off(int l)
    {
        return l == 0 ? 0 : t_off(l - 1) + l_out(l - 1) * l_inpad(l - 1);
    }
    static constexpr int NPARAMS = b_off(NLAYER - 1) + NOUT;
    static constexpr int NTRAIN = t_off(NLAYER - 1) + NOUT * WID;
    static constexpr int YS = NOUT <= 8 ? 8 : 16;   // row stride of targets and outputs
};

// inference image (same shape for every model): fragments (64 lanes x 8
// bf16 each), then FP32 biases (4 x 128 hidden, 16 output)
constexpr int NFRAG = 8 + 3 * 32 + 4;
__host__ __device__ constexpr int f_base(int l) { return l == 0 ? 0 : 8 + 32 * (l - 1); }
constexpr int NBIAS = 4 * WID + 16;
constexpr size_t IMG_BYTES = (size_t)NFRAG * 64 * 16 + NBIAS * 4;

enum : unsigned { FL_OOD = 1u, FL_DRY = 2u, FL_NONSUB = 4u, FL_PROJ = 8u };

// GELU, tanh form: 0.5 x (1 + tanh(k (x + a x^3))) = x / (1 + exp(-2 k (x + a x^3)))
constexpr double GK = 0.7978845608028654;  // sqrt(2/pi)
constexpr double GA = 0.044715;
constexpr double LOG2E = 1.4426950408889634;

// (seven vector instructions: the cubic as mul, fma, mul; exp2; add;
// reciprocal; mul -- the library is built without contraction, so the fma is
// written out)
__device__ __forceinline__ float gelu(float x)
{
    const float c0 = (float)(-2.0 * GK * LOG2E), c1 = (float)(-2.0 * GK * GA * LOG2E);
    const float x2 = x * x;
    const float e = __builtin_amdgcn_exp2f(x * fmaf(c1, x2, c0));
    return x * __builtin_amdgcn_rcpf(1.0f + e);
}
// d/dx of the above: s + 2 x s (1 - s) k (1 + 3 a x^2), s = 1 / (1 + exp(-2 k (x + a x^3)))
__device__ __forceinline__ float gelu_grad(float x)
{
    const float c0 = (float)(-2.0 * GK * LOG2E), c1 = (float)(-2.0 * GK * GA * LOG2E);
    const float x2 = x * x;
    const float e = __builtin_amdgcn_exp2f(x * fmaf(c1, x2, c0));
    const float s = __builtin_amdgcn_rcpf(1.0f + e);
    const float dy = fmaf((float)(3.0 * GK * GA), x2, (float)GK);
    return fmaf(2.0f * x * s * (1.0f - s), dy, s);
}

__device__ __forceinline__ bf16x8 zero8()
{
    bf16x8 z;
#pragma unroll
    for (int j = 0; j < 8; ++j) z[j] = (bf16)0.0f;
    return z;
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// LDS traffic between lanes of one wavefront: order the accesses of the
// wavefront around this point
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------ inference MLP
// One wavefront evaluates the network on its 64 lanes' inputs x; lane l gets
// its NOUT outputs in o.  sF: fragment image, sBias: biases, scr: 1024
// floats of this wavefront's LDS.  Must be reached by all 64 lanes together.
template <int NOUT>
__device__ void mlp64(const bf16x8* __restrict__ sF, const float* __restrict__ sBias, float* scr,
                      const float (&x)[8], float (&o)[16])
{
    const int lane = threadIdx.x & 63, s = lane & 15, g = lane >> 4;
    bf16x8 xin;
#pragma unroll
    for (int j = 0; j < 8; ++j) xin[j] = (bf16)x[j];
    bf16x8* sx = reinterpret_cast<bf16x8*>(scr);
    wave_sync();
    sx[lane] = xin;
    wave_sync();
    bf16x8 b0[4];
#pragma unroll
    for (int sb = 0; sb < 4; ++sb) b0[sb] = g == 0 ? sx[16 * sb + s] : zero8();

    f32x4 acc[8][4];
    bf16x8 bop[4][4];
    // layer 0: the inputs in k-slots 0..7 of lane group 0
#pragma unroll
    for (int nb = 0; nb < 8; ++nb) {
        const f32x4 bias = *reinterpret_cast<const f32x4*>(sBias + 16 * nb + 4 * g);
        const bf16x8 a = sF[(f_base(0) + nb) * 64 + lane];
#pragma unroll
        for (int sb = 0; sb < 4; ++sb) acc[nb][sb] = mfma(a, b0[sb], bias);
    }
    for (int l = 1; l < NLAYER; ++l) {
        // activation of the previous layer, into the permuted k-slots
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
#pragma unroll
            for (int sb = 0; sb < 4; ++sb)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    bop[kb][sb][j] = (bf16)gelu(acc[2 * kb][sb][j]);
                    bop[kb][sb][4 + j] = (bf16)gelu(acc[2 * kb + 1][sb][j]);
                }
        if (l == NLAYER - 1) break;
        const int fb = f_base(l);
#pragma unroll
        for (int nb = 0; nb < 8; ++nb) {
            const f32x4 bias = *reinterpret_cast<const f32x4*>(sBias + l * WID + 16 * nb + 4 * g);
#pragma unroll
            for (int sb = 0; sb < 4; ++sb) acc[nb][sb] = bias;
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) {
                const bf16x8 a = sF[(fb + nb * 4 + kb) * 64 + lane];
#pragma unroll
                for (int sb = 0; sb < 4; ++sb) acc[nb][sb] = mfma(a, bop[kb][sb], acc[nb][sb]);
            }
        }
    }
    // output layer: 16 rows, NOUT of them real
    f32x4 out[4];
    {
        const f32x4 bias = *reinterpret_cast<const f32x4*>(sBias + 4 * WID + 4 * g);
#pragma unroll
        for (int sb = 0; sb < 4; ++sb) out[sb] = bias;
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            const bf16x8 a = sF[(f_base(NLAYER - 1) + kb) * 64 + lane];
#pragma unroll
            for (int sb = 0; sb < 4; ++sb) out[sb] = mfma(a, bop[kb][sb], out[sb]);
        }
    }
    wave_sync();
    if (4 * g < NOUT) {
#pragma unroll
        for (int sb = 0; sb < 4; ++sb)
            *reinterpret_cast<f32x4*>(scr + (16 * sb + s) * 16 + 4 * g) = out[sb];
    }
    wave_sync();
#pragma unroll
    for (int j = 0; j < 16; ++j) o[j] = j < NOUT ? scr[lane * 16 + j] : 0.0f;
}

// ------------------------------------------------------------ edge results
template <int ME, int MW>
struct ERes {
    float s[MW];
    float w[MW][ME];
    float am[ME], ap[ME];
};

// network outputs -> K waves projected onto the flux difference, placed in
// their record slots; returns false when the projection is degenerate
template <class M>
__device__ __forceinline__ bool project_into(const float (&sk)[M::K], float (&Wk)[M::K][M::MEQN],
                                             const float (&df)[M::MEQN], ERes<M::MEQN, M::MW>& r)
{
    constexpr int ME = M::MEQN, K = M::K;
    float D = sk[0] * sk[0];
#pragma unroll
    for (int k = 1; k < K; ++k) D = D + sk[k] * sk[k];
    const bool ok = D > 0.0f && D <= 3.0e38f;
    const float iD = ok ? __builtin_amdgcn_rcpf(D) : 0.0f;
#pragma unroll
    for (int m = 0; m < ME; ++m) {
        float res = df[m] - sk[0] * Wk[0][m];
#pragma unroll
        for (int k = 1; k < K; ++k) res = res - sk[k] * Wk[k][m];
#pragma unroll
        for (int k = 0; k < K; ++k) Wk[k][m] = Wk[k][m] + sk[k] * res * iD;
    }
#pragma unroll
    for (int p = 0; p < M::MW; ++p) {
        r.s[p] = 0.0f;
#pragma unroll
        for (int m = 0; m < ME; ++m) r.w[p][m] = 0.0f;
    }
#pragma unroll
    for (int m = 0; m < ME; ++m) { r.am[m] = 0.0f; r.ap[m] = 0.0f; }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int p = M::slot(k);
        const float neg = sk[k] < 0.0f ? sk[k] : 0.0f, pos = sk[k] > 0.0f ? sk[k] : 0.0f;
        r.s[p] = sk[k];
#pragma unroll
        for (int m = 0; m < ME; ++m) {
            r.w[p][m] = Wk[k][m];
            r.am[m] = r.am[m] + neg * Wk[k][m];
            r.ap[m] = r.ap[m] + pos * Wk[k][m];
        }
    }
    return ok;
}

// ------------------------------------------------------------ models
// Shallow water: (h, hu_n, hu_t); h0 = (hL + hR)/2, c0 = sqrt(g h0); inputs
// (ubar/c0, vbar/c0, m, e) with (dh/h0, d(hu)/(h0 c0), d(hv)/(h0 c0)) = m e;
// two waves (slots 0 and 2).  Box: h in [1e-3, 10], |u|, |v| <= 5; near-dry
// below min h = 1e-2.
struct SwModel {
    using N = Net<6, 8>;
    static constexpr int MEQN = 3, MW = 3, K = 2, NREC = MW + MW * MEQN + 2 * MEQN;
    __host__ __device__ static constexpr int slot(int k) { return k == 0 ? 0 : 2; }
    static constexpr float H_LO = 1e-3f, H_HI = 10.0f, U_MAX = 5.0f, H_DRY = 1e-2f;

    __device__ static unsigned side(float g, const float* q)
    {
        unsigned f = 0u;
        // negated comparisons: a NaN anywhere counts as outside the box
        if (!(q[0] >= H_LO) || !(q[0] <= H_HI) || !(fabsf(q[1]) <= U_MAX * q[0]) ||
            !(fabsf(q[2]) <= U_MAX * q[0]))
            f |= FL_OOD;
        if (q[1] * q[1] >= ((g * q[0]) * q[0]) * q[0]) f |= FL_NONSUB;  // |u| >= c
        return f;
    }
    __device__ static unsigned flags(const DevParams& P, const float* L, const float* R)
    {
        const float g = (float)P.g;
        unsigned f = side(g, L) | side(g, R);
        const float hm = L[0] < R[0] ? L[0] : R[0];
        if (hm < H_DRY) f |= FL_DRY;
        return f;
    }
    // inputs x[8] (6 used) and the decoding scales sc = (h0, c0, m)
    __device__ static void features(const DevParams& P, const float* L, const float* R, float (&x)[8],
                                    float (&sc)[3])
    {
        const float g = (float)P.g;
        const float h0 = 0.5f * (L[0] + R[0]);
        const float c0 = __builtin_amdgcn_sqrtf(g * h0);
        const float rl = __builtin_amdgcn_rcpf(L[0]), rr = __builtin_amdgcn_rcpf(R[0]);
        const float rc = __builtin_amdgcn_rcpf(c0);
        const float ub = 0.5f * (L[1] * rl + R[1] * rr);
        const float vb = 0.5f * (L[2] * rl + R[2] * rr);
        const float rh = __builtin_amdgcn_rcpf(h0);
        const float rhc = rh * rc;
        const float d0 = (R[0] - L[0]) * rh, d1 = (R[1] - L[1]) * rhc, d2 = (R[2] - L[2]) * rhc;
        const float m = __builtin_amdgcn_sqrtf(d0 * d0 + d1 * d1 + d2 * d2);
        const float rm = m > 0.0f ? __builtin_amdgcn_rcpf(m) : 0.0f;
        x[0] = ub * rc; x[1] = vb * rc; x[2] = m;
        x[3] = d0 * rm; x[4] = d1 * rm; x[5] = d2 * rm;
        x[6] = 0.0f; x[7] = 0.0f;
        sc[0] = h0; sc[1] = c0; sc[2] = m;
    }
    __device__ static void flux(const DevParams& P, const float* q, float (&f)[MEQN])
    {
        const float u = q[1] * __builtin_amdgcn_rcpf(q[0]);
        f[0] = q[1];
        f[1] = q[1] * u + 0.5f * (float)P.g * (q[0] * q[0]);
        f[2] = q[2] * u;
    }
    __device__ static void decode(const float (&o)[16], const float (&sc)[3], float (&sk)[K],
                                  float (&Wk)[K][MEQN])
    {
        const float hc = sc[0] * sc[1];
        const float S[3] = {sc[0], hc, hc};
        sk[0] = sc[1] * o[0];
        sk[1] = sc[1] * o[1];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            Wk[0][m] = sc[2] * S[m] * o[2 + m];
            Wk[1][m] = sc[2] * S[m] * o[5 + m];
        }
    }
    // Roe + Harten-Hyman; HLLE where Roe's middle depth hL + alpha_1 <= 0
    __device__ static unsigned fallback(const DevParams& P, const float* L, const float* R,
                                        ERes<MEQN, MW>& r)
    {
        using Roe = SwRoe<float, 1>;
        using Hll = SwHlleC<float, 1>;
        typename Roe::C cl, cr;
        cl.v[0] = L[0]; cl.v[1] = L[1]; cl.v[2] = L[2];
        cr.v[0] = R[0]; cr.v[1] = R[1]; cr.v[2] = R[2];
        if (!(L[0] > 0.0f) || !(R[0] > 0.0f)) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                r.s[k] = 0.0f; r.am[k] = 0.0f; r.ap[k] = 0.0f;
                r.w[0][k] = r.w[1][k] = r.w[2][k] = 0.0f;
            }
            return ST_NONPHYS;
        }
        Roe::prep(P, cl);
        Roe::prep(P, cr);
        typename Roe::E e;
        Roe::solve(P, cl, cr, e);
        if (L[0] + e.v[0] > 0.0f) {
            Roe::waves(P, e, r.w);
#pragma unroll
            for (int p = 0; p < 3; ++p) r.s[p] = Roe::speed(P, e, p);
            Roe::fluct(P, e, r.am, r.ap);
            return 0u;
        }
        typename Hll::E h;
        const unsigned st = Hll::solve(P, cl, cr, h);
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            r.s[p] = h.s[p];
#pragma unroll
            for (int k = 0; k < 3; ++k) r.w[p][k] = h.w[p][k];
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) { r.am[k] = h.am[k]; r.ap[k] = h.ap[k]; }
        return st;
    }
};

// Euler (gamma-law gas): (rho, rho u_n, rho u_t, E); rho0, p0 the means,
// c0 = sqrt(gamma p0/rho0); inputs (ubar/c0, vbar/c0, m, e) with the jump
// scaled by (rho0, rho0 c0, rho0 c0, rho0 c0^2); three waves (slots 0, 1, 3).
// Box: rho, p in [0.05, 10], |u|, |v| <= 2 (products only: p rho =
// (gamma - 1)(E rho - |rho u|^2 / 2)).
struct EulerModel {
    using N = Net<7, 15>;
    static constexpr int MEQN = 4, MW = 4, K = 3, NREC = MW + MW * MEQN + 2 * MEQN;
    __host__ __device__ static constexpr int slot(int k) { return k == 0 ? 0 : (k == 1 ? 1 : 3); }
    static constexpr float R_LO = 0.05f, R_HI = 10.0f, P_LO = 0.05f, P_HI = 10.0f, U_MAX = 2.0f;

    // gm1 = gamma - 1 rounded from double (not the FP32 difference)
    __device__ static unsigned side(float gm, float gm1, const float* q)
    {
        const float pr = gm1 * (q[3] * q[0] - 0.5f * (q[1] * q[1] + q[2] * q[2]));
        unsigned f = 0u;
        if (!(q[0] >= R_LO) || !(q[0] <= R_HI) || !(pr >= P_LO * q[0]) || !(pr <= P_HI * q[0]) ||
            !(fabsf(q[1]) <= U_MAX * q[0]) || !(fabsf(q[2]) <= U_MAX * q[0]))
            f |= FL_OOD;
        if (q[1] * q[1] >= gm * pr) f |= FL_NONSUB;   // u^2 >= c^2
        return f;
    }
    __device__ static unsigned flags(const DevParams& P, const float* L, const float* R)
    {
        const float gm = (float)P.gamma, gm1 = (float)(P.gamma - 1.0);
        return side(gm, gm1, L) | side(gm, gm1, R);
    }
    __device__ static float pressure(float gm1, const float* q)
    {
        return gm1 * (q[3] - 0.5f * (q[1] * q[1] + q[2] * q[2]) * __builtin_amdgcn_rcpf(q[0]));
    }
    // inputs x[8] (7 used) and the decoding scales sc = (rho0, c0, m)
    __device__ static void features(const DevParams& P, const float* L, const float* R, float (&x)[8],
                                    float (&sc)[3])
    {
        const float gm = (float)P.gamma, gm1 = (float)(P.gamma - 1.0);
        const float r0 = 0.5f * (L[0] + R[0]);
        const float p0 = 0.5f * (pressure(gm1, L) + pressure(gm1, R));
        const float rr0 = __builtin_amdgcn_rcpf(r0);
        const float c0 = __builtin_amdgcn_sqrtf(gm * p0 * rr0);
        const float rc = __builtin_amdgcn_rcpf(c0);
        const float ub = 0.5f * (L[1] * __builtin_amdgcn_rcpf(L[0]) + R[1] * __builtin_amdgcn_rcpf(R[0]));
        const float vb = 0.5f * (L[2] * __builtin_amdgcn_rcpf(L[0]) + R[2] * __builtin_amdgcn_rcpf(R[0]));
        const float d0 = (R[0] - L[0]) * rr0;
        const float d1 = (R[1] - L[1]) * rr0 * rc;
        const float d2 = (R[2] - L[2]) * rr0 * rc;
        const float d3 = (R[3] - L[3]) * rr0 * rc * rc;
        const float m = __builtin_amdgcn_sqrtf(d0 * d0 + d1 * d1 + d2 * d2 + d3 * d3);
        const float rm = m > 0.0f ? __builtin_amdgcn_rcpf(m) : 0.0f;
        x[0] = ub * rc; x[1] = vb * rc; x[2] = m;
        x[3] = d0 * rm; x[4] = d1 * rm; x[5] = d2 * rm; x[6] = d3 * rm;
        x[7] = 0.0f;
        sc[0] = r0; sc[1] = c0; sc[2] = m;
    }
    __device__ static void flux(const DevParams& P, const float* q, float (&f)[MEQN])
    {
        const float p = pressure((float)(P.gamma - 1.0), q);
        const float u = q[1] * __builtin_amdgcn_rcpf(q[0]);
        f[0] = q[1];
        f[1] = q[1] * u + p;
        f[2] = q[2] * u;
        f[3] = (q[3] + p) * u;
    }
    __device__ static void decode(const float (&o)[16], const float (&sc)[3], float (&sk)[K],
                                  float (&Wk)[K][MEQN])
    {
        const float rc = sc[0] * sc[1];
        const float S[4] = {sc[0], rc, rc, rc * sc[1]};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            sk[k] = sc[1] * o[k];
#pragma unroll
            for (int m = 0; m < 4; ++m) Wk[k][m] = sc[2] * S[m] * o[3 + 4 * k + m];
        }
    }
    // the plain Euler solver: Roe + HH, HLLE where Roe fails
    __device__ static unsigned fallback(const DevParams& P, const float* L, const float* R,
                                        ERes<MEQN, MW>& r)
    {
        using Eu = EulerRoeC<float, 1>;
        typename Eu::C cl, cr;
#pragma unroll
        for (int m = 0; m < 4; ++m) { cl.v[m] = L[m]; cr.v[m] = R[m]; }
        if (!(L[0] > 0.0f) || !(R[0] > 0.0f)) {
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                r.s[m] = 0.0f; r.am[m] = 0.0f; r.ap[m] = 0.0f;
#pragma unroll
                for (int p = 0; p < 4; ++p) r.w[p][m] = 0.0f;
            }
            return ST_NONPHYS;
        }
        Eu::prep(P, cl);
        Eu::prep(P, cr);
        typename Eu::E e;
        const unsigned st = Eu::solve(P, cl, cr, e);
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            r.s[p] = e.s[p];
#pragma unroll
            for (int m = 0; m < 4; ++m) r.w[p][m] = e.w[p][m];
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) { r.am[m] = e.am[m]; r.ap[m] = e.ap[m]; }
        return st & ST_NONPHYS;
    }
};

// ------------------------------------------------------------ edge kernel
enum { MODE_SWEEP = 0, MODE_ARRAYS = 1, MODE_NET = 2 };
constexpr int EWAVES = 8;                 // wavefronts per workgroup
constexpr int EBLOCK = EWAVES * WAVE;
constexpr size_t EDGE_LDS = IMG_BYTES + (size_t)EWAVES * 1024 * 4;

struct EdgeArgs {
    const uint4* img;        // inference image (global)
    DevParams P;
    int64_t n;               // edges (or rows)
    // MODE_SWEEP: grid state and the record array
    const float* q;          // [meqn][ny][nx]
    float* rec;              // [NREC][n]
    int nx, ny, bc;
    // MODE_ARRAYS: mc_rp2 layout
    const float* ql;
    const float* qr;
    float* waves;            // [mw][meqn][n]
    float* speeds;           // [mw][n]
    float* amdq;
    float* apdq;
    // MODE_NET
    const float* X;          // [n][8]
    float* out;              // [n][YS]
    // reductions
    unsigned int* smax_bits; // max |s| over counted edges (IEEE bits of a float >= 0)
    unsigned long long* counts;  // [0] edges solved, [1] fallbacks
    unsigned int* status;
};

template <class M, int MODE, int IXY>
__global__ __launch_bounds__(EBLOCK) void edge_kernel(EdgeArgs a)
{
    constexpr int ME = M::MEQN, MW = M::MW, NOUT = M::N::NOUT, YS = M::N::YS;
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    const bf16x8* sF = reinterpret_cast<const bf16x8*>(lds);
    const float* sBias = reinterpret_cast<const float*>(lds + (size_t)NFRAG * 64 * 16);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    float* scr = reinterpret_cast<float*>(lds + IMG_BYTES) + wv * 1024;
    {
        uint4* dst = reinterpret_cast<uint4*>(lds);
        for (int i = threadIdx.x; i < (int)(IMG_BYTES / 16); i += EBLOCK) dst[i] = a.img[i];
    }
    __syncthreads();

    // normal-frame slots: for y-normal edges the two momenta exchange roles
    constexpr int S1 = IXY == 1 ? 1 : 2, S2 = IXY == 1 ? 2 : 1;
    const int64_t ntiles = (a.n + 63) / 64;
    float smx = 0.0f;
    unsigned st = 0u;
    unsigned nfb = 0u, nsolved = 0u;
    for (int64_t tile = (int64_t)blockIdx.x * EWAVES + wv; tile < ntiles;
         tile += (int64_t)gridDim.x * EWAVES) {
        const int64_t e = tile * 64 + lane;
        const bool valid = e < a.n;
        float x[8];
        float o[16];
        float L[ME], R[ME];
        float sc[3] = {1.0f, 1.0f, 0.0f};
        unsigned fl = 0u;
        bool counted = false;
        if (MODE == MODE_NET) {
#pragma unroll
            for (int j = 0; j < 8; ++j) x[j] = (valid && j < M::N::NIN) ? a.X[e * 8 + j] : 0.0f;
#pragma unroll
            for (int m = 0; m < ME; ++m) { L[m] = 1.0f; R[m] = 1.0f; }
        } else {
            float ql[ME], qr[ME];
            if (MODE == MODE_SWEEP) {
                // edge k of line `line` lies between ghosted cells k and k + 1,
                // i.e. interior cells k - 2 and k - 1 along the sweep
                int il, ir, jl, jr;
                int64_t k, line;
                if (IXY == 1) {
                    const int64_t ne = a.nx + 3;
                    line = e / ne;
                    k = e - line * ne;
                    jl = jr = (int)line;
                    il = bc_map((int)k - 2, a.nx, a.bc);
                    ir = bc_map((int)k - 1, a.nx, a.bc);
                    counted = k >= 1 && k <= a.nx + 1;
                } else {
                    line = e % a.nx;   // column
                    k = e / a.nx;
                    il = ir = (int)line;
                    jl = bc_map((int)k - 2, a.ny, a.bc);
                    jr = bc_map((int)k - 1, a.ny, a.bc);
                    counted = k >= 1 && k <= a.ny + 1;
                }
                if (!valid) { il = ir = 0; jl = jr = 0; }
                const int64_t plane = (int64_t)a.nx * a.ny;
                const int64_t cl = (int64_t)jl * a.nx + il, cr = (int64_t)jr * a.nx + ir;
#pragma unroll
                for (int m = 0; m < ME; ++m) {
                    ql[m] = a.q[m * plane + cl];
                    qr[m] = a.q[m * plane + cr];
                }
            } else {
#pragma unroll
                for (int m = 0; m < ME; ++m) {
                    ql[m] = valid ? a.ql[m * a.n + e] : 1.0f;
                    qr[m] = valid ? a.qr[m * a.n + e] : 1.0f;
                }
                counted = true;
            }
#pragma unroll
            for (int m = 0; m < ME; ++m) {
                const int src = m == 1 ? S1 : (m == 2 ? S2 : m);
                L[m] = ql[src];
                R[m] = qr[src];
            }
            fl = M::flags(a.P, L, R);
            M::features(a.P, L, R, x, sc);
            if (fl != 0u) {
#pragma unroll
                for (int j = 0; j < 8; ++j) x[j] = 0.0f;
            }
        }
        mlp64<NOUT>(sF, sBias, scr, x, o);
        // everything below is per lane (no cross-lane operations)
        if (valid && MODE == MODE_NET) {
#pragma unroll
            for (int j = 0; j < YS; ++j) a.out[e * YS + j] = j < NOUT ? o[j] : 0.0f;
        }
        if (!valid || MODE == MODE_NET) continue;
        ERes<ME, MW> r;
        if (fl == 0u) {
            float sk[M::K], Wk[M::K][ME], fL[ME], fR[ME], df[ME];
            M::decode(o, sc, sk, Wk);
            M::flux(a.P, L, fL);
            M::flux(a.P, R, fR);
#pragma unroll
            for (int m = 0; m < ME; ++m) df[m] = fR[m] - fL[m];
            if (!project_into<M>(sk, Wk, df, r)) fl |= FL_PROJ;
        }
        if (fl != 0u) {
            st |= M::fallback(a.P, L, R, r) | ST_FALLBACK;
            ++nfb;
        }
        ++nsolved;
        if (counted) {
#pragma unroll
            for (int p = 0; p < MW; ++p) smx = fmaxf(smx, fabsf(r.s[p]));
        }
        // back to grid orientation: component m of the normal frame goes to
        // slot m, with the two momenta exchanged for y-normal edges
        if (MODE == MODE_SWEEP) {
            float* rc = a.rec + e;
            const int64_t n = a.n;
#pragma unroll
            for (int p = 0; p < MW; ++p) {
                rc[p * n] = r.s[p];
#pragma unroll
                for (int m = 0; m < ME; ++m) {
                    const int gm = m == 1 ? S1 : (m == 2 ? S2 : m);
                    rc[(MW + ME * p + gm) * n] = r.w[p][m];
                }
            }
#pragma unroll
            for (int m = 0; m < ME; ++m) {
                const int gm = m == 1 ? S1 : (m == 2 ? S2 : m);
                rc[(MW + MW * ME + gm) * n] = r.am[m];
                rc[(MW + MW * ME + ME + gm) * n] = r.ap[m];
            }
        } else {
            const int64_t n = a.n;
#pragma unroll
            for (int p = 0; p < MW; ++p) {
                a.speeds[p * n + e] = r.s[p];
#pragma unroll
                for (int m = 0; m < ME; ++m) {
                    const int gm = m == 1 ? S1 : (m == 2 ? S2 : m);
                    a.waves[(p * ME + gm) * n + e] = r.w[p][m];
                }
            }
#pragma unroll
            for (int m = 0; m < ME; ++m) {
                const int gm = m == 1 ? S1 : (m == 2 ? S2 : m);
                a.amdq[gm * n + e] = r.am[m];
                a.apdq[gm * n + e] = r.ap[m];
            }
        }
    }
    if (MODE == MODE_NET) return;
    // workgroup reductions: max speed, status bits, counts
    __shared__ float s_mx[EWAVES];
    __shared__ unsigned s_st[EWAVES], s_fb[EWAVES], s_ns[EWAVES];
    {
        float v = smx;
        unsigned u = st, f = nfb, c = nsolved;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const int src = ((lane ^ off) & 63) << 2;
            v = fmaxf(v, xlane(src, v));
            u |= (unsigned)__builtin_amdgcn_ds_bpermute(src, (int)u);
            f += (unsigned)__builtin_amdgcn_ds_bpermute(src, (int)f);
            c += (unsigned)__builtin_amdgcn_ds_bpermute(src, (int)c);
        }
        if (lane == 0) { s_mx[wv] = v; s_st[wv] = u; s_fb[wv] = f; s_ns[wv] = c; }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float v = 0.0f;
        unsigned u = 0u;
        unsigned long long f = 0, c = 0;
        for (int w = 0; w < EWAVES; ++w) {
            v = fmaxf(v, s_mx[w]);
            u |= s_st[w];
            f += s_fb[w];
            c += s_ns[w];
        }
        atomicMax(a.smax_bits, __float_as_uint(v));
        if (u) atomicOr(a.status, u);
        if (f) atomicAdd(&a.counts[1], f);
        if (c) atomicAdd(&a.counts[0], c);
    }
}

// ------------------------------------------------------------ update kernel
// One interior cell per thread: correction fluxes at its two edges from the
// records of those edges and their neighbours, then the conservative update.
// Record layout: speeds [MW], waves [MW][ME], A-dQ [ME], A+dQ [ME].
struct UpdArgs {
    const float* q;   // [meqn][ny][nx], the sweep's input state
    float* qo;
    const float* rec; // [NREC][n]
    int64_t n;        // edges in the record array
    int nx, ny;
    float nu;         // dt / d
};

template <int ME, int MW, int LIM>
__device__ __forceinline__ void ftil_at(const float* rec, int64_t n, int64_t e, int64_t el, int64_t er,
                                        float nu, float (&F)[ME])
{
#pragma unroll
    for (int m = 0; m < ME; ++m) F[m] = 0.0f;
    if (LIM == LIM_FIRST_ORDER) return;
#pragma unroll
    for (int p = 0; p < MW; ++p) {
        const float s = rec[p * n + e];
        const int64_t eu = s > 0.0f ? el : er;
        float w[ME], wu[ME];
#pragma unroll
        for (int m = 0; m < ME; ++m) {
            w[m] = rec[(MW + ME * p + m) * n + e];
            wu[m] = rec[(MW + ME * p + m) * n + eu];
        }
        float wn = w[0] * w[0], wd = wu[0] * w[0];
#pragma unroll
        for (int m = 1; m < ME; ++m) {
            wn = wn + w[m] * w[m];
            wd = wd + wu[m] * w[m];
        }
        const float phi = limiter_phi<LIM, float>(wd, wn);
        const float as = fabsf(s);
        const float c = 0.5f * as * (1.0f - nu * as);
#pragma unroll
        for (int m = 0; m < ME; ++m) F[m] += c * (phi * w[m]);
    }
}

template <int ME, int MW, int IXY, int LIM>
__global__ __launch_bounds__(256) void update_kernel(UpdArgs a)
{
    const int64_t plane = (int64_t)a.nx * a.ny;
    for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < plane;
         c += (int64_t)gridDim.x * 256) {
        const int j = (int)(c / a.nx), i = (int)(c - (int64_t)j * a.nx);
        // edges kl = pos + 1 and kr = pos + 2 of the cell's line
        int64_t e0, step;
        if (IXY == 1) {
            e0 = (int64_t)j * (a.nx + 3) + i;
            step = 1;
        } else {
            e0 = (int64_t)j * a.nx + i;
            step = a.nx;
        }
        const int64_t e1 = e0 + step, e2 = e1 + step, e3 = e2 + step;
        float Fl[ME], Fr[ME];
        ftil_at<ME, MW, LIM>(a.rec, a.n, e1, e0, e2, a.nu, Fl);
        ftil_at<ME, MW, LIM>(a.rec, a.n, e2, e1, e3, a.nu, Fr);
#pragma unroll
        for (int m = 0; m < ME; ++m) {
            const float qv = a.q[m * plane + c];
            const float ap = a.rec[(MW + MW * ME + ME + m) * a.n + e1];
            const float am = a.rec[(MW + MW * ME + m) * a.n + e2];
            a.qo[m * plane + c] = qv - a.nu * (ap + am) - a.nu * (Fr[m] - Fl[m]);
        }
    }
}

// smax and cfl of the step from the two sweeps' maxima; clears them
struct FinArgs {
    unsigned int* smax_bits;  // [2]
    mc_cfl* cfl;
    double dx, dy, dt;
};
__global__ void finish_kernel(FinArgs a)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const double sx = (double)__uint_as_float(a.smax_bits[0]) / a.dx;
        const double sy = (double)__uint_as_float(a.smax_bits[1]) / a.dy;
        const double sm = sx > sy ? sx : sy;
        if (a.cfl) {
            a.cfl->smax = sm;
            a.cfl->cfl = a.dt * sm;
        }
        atomicExch(&a.smax_bits[0], 0u);
        atomicExch(&a.smax_bits[1], 0u);
    }
}

// ------------------------------------------------------------ parameter packing
__device__ __forceinline__ uint16_t bf16_bits(float v)
{
    const bf16 b = (bf16)v;
    return *reinterpret_cast<const uint16_t*>(&b);
}

// inference image: fragment f, lane l, slot j -> weight of row 16 nb + l % 16
// and the input neuron the slot stands for; then the biases
template <class NT>
__global__ void pack_image_kernel(const float* __restrict__ p, uint16_t* __restrict__ img)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int nw = NFRAG * 64 * 8;
    if (idx < nw) {
        const int f = idx / 512, lane = (idx / 8) & 63, j = idx & 7;
        int l, nb, kb;
        if (f < 8) { l = 0; nb = f; kb = 0; }
        else if (f < NFRAG - 4) { l = 1 + (f - 8) / 32; nb = ((f - 8) % 32) / 4; kb = (f - 8) % 4; }
        else { l = NLAYER - 1; nb = 0; kb = f - (NFRAG - 4); }
        const int row = 16 * nb + (lane & 15), gq = lane >> 4;
        float v = 0.0f;
        if (l == 0) {
            const int col = 8 * gq + j;
            if (col < NT::NIN) v = p[NT::w_off(0) + row * NT::NIN + col];
        } else {
            const int col = 32 * kb + (j < 4 ? 4 * gq + j : 16 + 4 * gq + (j - 4));
            if (row < NT::l_out(l)) v = p[NT::w_off(l) + row * WID + col];
        }
        img[idx] = bf16_bits(v);
    } else if (idx < nw + NBIAS) {
        const int b = idx - nw;
        float v = 0.0f;
        if (b < 4 * WID) v = p[NT::b_off(b / WID) + (b % WID)];
        else if (b - 4 * WID < NT::NOUT) v = p[NT::b_off(NLAYER - 1) + (b - 4 * WID)];
        float* fb = reinterpret_cast<float*>(img + nw);
        fb[b] = v;
    }
}

// BF16 training copies: layer l as [out][inpad] row-major (pad columns 0)
template <class NT>
__global__ void pack_train_kernel(const float* __restrict__ p, bf16* __restrict__ wt)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= NT::NTRAIN) return;
    int l = 0;
    while (l < NLAYER - 1 && idx >= NT::t_off(l + 1)) ++l;
    const int r = idx - NT::t_off(l);
    const int o = r / NT::l_inpad(l), i = r % NT::l_inpad(l);
    wt[idx] = (bf16)(i < NT::l_in(l) ? p[NT::w_off(l) + o * NT::l_in(l) + i] : 0.0f);
}

template <class NT>
__global__ void init_params_kernel(const double* __restrict__ U, float* __restrict__ p)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= NT::NPARAMS) return;
    int l = 0;
    while (l < NLAYER - 1 && idx >= NT::w_off(l + 1)) ++l;
    if (idx >= NT::b_off(l)) { p[idx] = 0.0f; return; }
    const double lim = sqrt(6.0 / (double)(NT::l_in(l) + NT::l_out(l)));
    p[idx] = (float)(-lim + 2.0 * lim * U[idx]);
}

__global__ void adam_kernel(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ gr, int np, float lr, float b1, float b2, float eps,
                            float c1, float c2)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= np) return;
    const float g = gr[idx];
    const float mm = b1 * m[idx] + (1.0f - b1) * g;
    const float vv = b2 * v[idx] + (1.0f - b2) * (g * g);
    m[idx] = mm;
    v[idx] = vv;
    p[idx] = p[idx] - lr * (mm * c1) / (sqrtf(vv * c2) + eps);
}

// ------------------------------------------------------------ training pairs
// shallow water: uniforms [6][n] -> h log-uniform in [1e-3, 10], u, v in
// [-5, 5]; labels from Roe in FP64
__global__ void gen_sw_kernel(const double* __restrict__ U, int64_t n, double g, float* __restrict__ X,
                              float* __restrict__ Y, int32_t* __restrict__ keep)
{
    DevParams P;
    P.g = g;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double lo = log(1e-3), hi = log(10.0);
        double q[2][3];
        for (int s = 0; s < 2; ++s) {
            const double h = exp(lo + (hi - lo) * U[(3 * s) * n + i]);
            const double u = -5.0 + 10.0 * U[(3 * s + 1) * n + i];
            const double v = -5.0 + 10.0 * U[(3 * s + 2) * n + i];
            q[s][0] = h; q[s][1] = h * u; q[s][2] = h * v;
        }
        const double hl = q[0][0], hr = q[1][0];
        // inputs (FP64, stored as FP32)
        const double h0 = 0.5 * (hl + hr), c0 = sqrt(g * h0);
        const double ul = q[0][1] / hl, vl = q[0][2] / hl, ur = q[1][1] / hr, vr = q[1][2] / hr;
        const double d0 = (hr - hl) / h0, d1 = (q[1][1] - q[0][1]) / (h0 * c0),
                     d2 = (q[1][2] - q[0][2]) / (h0 * c0);
        const double m = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        float* xr = X + i * 8;
        xr[0] = (float)(0.5 * (ul + ur) / c0);
        xr[1] = (float)(0.5 * (vl + vr) / c0);
        xr[2] = (float)m;
        xr[3] = (float)(m > 0.0 ? d0 / m : 0.0);
        xr[4] = (float)(m > 0.0 ? d1 / m : 0.0);
        xr[5] = (float)(m > 0.0 ? d2 / m : 0.0);
        xr[6] = 0.0f;
        xr[7] = 0.0f;
        // flags in FP32 on the FP32-rounded states
        const float Lf[3] = {(float)q[0][0], (float)q[0][1], (float)q[0][2]};
        const float Rf[3] = {(float)q[1][0], (float)q[1][1], (float)q[1][2]};
        const unsigned fl = SwModel::flags(P, Lf, Rf);
        // Roe in FP64
        const double sl = sqrt(hl), sr = sqrt(hr);
        const double uh = (sl * ul + sr * ur) / (sl + sr), vh = (sl * vl + sr * vr) / (sl + sr);
        const double ch = sqrt(g * h0);
        const double e0 = hr - hl, e1 = q[1][1] - q[0][1], e2 = q[1][2] - q[0][2];
        const double a1 = ((uh + ch) * e0 - e1) / (2.0 * ch);
        const double a2 = e2 - vh * e0;
        const double a3 = (e1 - (uh - ch) * e0) / (2.0 * ch);
        const double s1 = uh - ch, s3 = uh + ch;
        // entropy-fix test of families 1 and 3 (transonic across the wave)
        const double h1 = hl + a1, m1 = q[0][1] + a1 * s1;
        const double h2 = hr - a3, m2 = q[1][1] - a3 * s3;
        bool fix = !(h1 > 0.0) || !(h2 > 0.0);
        if (!fix) {
            const double l1l = ul - sqrt(g * hl), l1r = m1 / h1 - sqrt(g * h1);
            const double l3l = m2 / h2 + sqrt(g * h2), l3r = ur + sqrt(g * hr);
            fix = (l1l < 0.0 && l1r > 0.0) || (l3l < 0.0 && l3r > 0.0);
        }
        const bool kp = fl == 0u && m > 0.0 && s1 < 0.0 && s3 > 0.0 && !fix;
        keep[i] = kp ? 1 : 0;
        float* yr = Y + i * 8;
        if (!kp) {
            for (int j = 0; j < 8; ++j) yr[j] = 0.0f;
            continue;
        }
        // W_a = A-dQ / s1 = W1 + (min(s2, 0) / s1) W2, W_b = W3 + (max(s2, 0) / s3) W2
        const double ra = (uh < 0.0 ? uh : 0.0) / s1, rb = (uh > 0.0 ? uh : 0.0) / s3;
        const double wa[3] = {a1, a1 * s1, a1 * vh + ra * a2};
        const double wb[3] = {a3, a3 * s3, a3 * vh + rb * a2};
        const double S[3] = {h0, h0 * c0, h0 * c0};
        yr[0] = (float)(s1 / c0);
        yr[1] = (float)(s3 / c0);
        for (int k = 0; k < 3; ++k) {
            yr[2 + k] = (float)(wa[k] / (m * S[k]));
            yr[5 + k] = (float)(wb[k] / (m * S[k]));
        }
    }
}

// Euler: uniforms [8][n] -> rho, p log-uniform in [0.05, 10], u, v in
// [-2, 2]; labels from Roe in FP64 (pairs where Roe's intermediate states
// are not physical or the entropy fix splits a wave are not kept)
__global__ void gen_euler_kernel(const double* __restrict__ U, int64_t n, double gm, float* __restrict__ X,
                                 float* __restrict__ Y, int32_t* __restrict__ keep)
{
    DevParams P;
    P.gamma = gm;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double lo = log(0.05), hi = log(10.0);
        double q[2][4], pp[2];
        for (int s = 0; s < 2; ++s) {
            const double r = exp(lo + (hi - lo) * U[(4 * s) * n + i]);
            const double u = -2.0 + 4.0 * U[(4 * s + 1) * n + i];
            const double v = -2.0 + 4.0 * U[(4 * s + 2) * n + i];
            const double p = exp(lo + (hi - lo) * U[(4 * s + 3) * n + i]);
            q[s][0] = r; q[s][1] = r * u; q[s][2] = r * v; q[s][3] = p / (gm - 1.0) + 0.5 * r * (u * u + v * v);
        }
        for (int s = 0; s < 2; ++s)
            pp[s] = (gm - 1.0) * (q[s][3] - 0.5 * (q[s][1] * q[s][1] + q[s][2] * q[s][2]) / q[s][0]);
        const double rl = q[0][0], rr = q[1][0];
        const double r0 = 0.5 * (rl + rr), p0 = 0.5 * (pp[0] + pp[1]);
        const double c0 = sqrt(gm * p0 / r0);
        const double ul = q[0][1] / rl, vl = q[0][2] / rl, ur = q[1][1] / rr, vr = q[1][2] / rr;
        const double S[4] = {r0, r0 * c0, r0 * c0, r0 * c0 * c0};
        double d[4];
        for (int k = 0; k < 4; ++k) d[k] = (q[1][k] - q[0][k]) / S[k];
        const double m = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + d[3] * d[3]);
        float* xr = X + i * 8;
        xr[0] = (float)(0.5 * (ul + ur) / c0);
        xr[1] = (float)(0.5 * (vl + vr) / c0);
        xr[2] = (float)m;
        for (int k = 0; k < 4; ++k) xr[3 + k] = (float)(m > 0.0 ? d[k] / m : 0.0);
        xr[7] = 0.0f;
        const float Lf[4] = {(float)q[0][0], (float)q[0][1], (float)q[0][2], (float)q[0][3]};
        const float Rf[4] = {(float)q[1][0], (float)q[1][1], (float)q[1][2], (float)q[1][3]};
        const unsigned fl = EulerModel::flags(P, Lf, Rf);
        // Roe in FP64 (normal frame: component 1 normal, 2 transverse)
        const double Hl = (q[0][3] + pp[0]) / rl, Hr = (q[1][3] + pp[1]) / rr;
        const double sl = sqrt(rl), sr = sqrt(rr);
        const double uh = (sl * ul + sr * ur) / (sl + sr), vh = (sl * vl + sr * vr) / (sl + sr);
        const double Hh = (sl * Hl + sr * Hr) / (sl + sr);
        const double q2 = uh * uh + vh * vh;
        const double c2 = (gm - 1.0) * (Hh - 0.5 * q2);
        bool kp = fl == 0u && m > 0.0 && c2 > 0.0;
        double w[4][4] = {};
        double sp[4] = {};
        if (kp) {
            const double ch = sqrt(c2);
            const double e0 = q[1][0] - q[0][0], e1 = q[1][1] - q[0][1], e2 = q[1][2] - q[0][2],
                         e3 = q[1][3] - q[0][3];
            const double a3 = e2 - vh * e0;
            const double a2 = (gm - 1.0) / c2 * ((Hh - q2) * e0 + uh * e1 + vh * e2 - e3);
            const double a1 = ((uh + ch) * e0 - e1 - ch * a2) / (2.0 * ch);
            const double a4 = e0 - a1 - a2;
            const double W1[4] = {a1, a1 * (uh - ch), a1 * vh, a1 * (Hh - uh * ch)};
            const double W2[4] = {a2, a2 * uh, a2 * vh, a2 * (0.5 * q2)};
            const double W3[4] = {0.0, 0.0, a3, a3 * vh};
            const double W4[4] = {a4, a4 * (uh + ch), a4 * vh, a4 * (Hh + uh * ch)};
            sp[0] = uh - ch; sp[1] = uh; sp[2] = uh; sp[3] = uh + ch;
            for (int k = 0; k < 4; ++k) { w[0][k] = W1[k]; w[1][k] = W2[k]; w[2][k] = W3[k]; w[3][k] = W4[k]; }
            // Roe intermediate states next to the acoustic waves, entropy-fix test
            double q1[4], q3[4];
            for (int k = 0; k < 4; ++k) { q1[k] = q[0][k] + W1[k]; q3[k] = q[1][k] - W4[k]; }
            const bool ok1 = q1[0] > 0.0 && q3[0] > 0.0;
            double p1 = -1.0, p3 = -1.0;
            if (ok1) {
                p1 = (gm - 1.0) * (q1[3] - 0.5 * (q1[1] * q1[1] + q1[2] * q1[2]) / q1[0]);
                p3 = (gm - 1.0) * (q3[3] - 0.5 * (q3[1] * q3[1] + q3[2] * q3[2]) / q3[0]);
            }
            if (!ok1 || !(p1 > 0.0) || !(p3 > 0.0)) {
                kp = false;
            } else {
                const double l1l = ul - sqrt(gm * pp[0] / rl), l1r = q1[1] / q1[0] - sqrt(gm * p1 / q1[0]);
                const double l4l = q3[1] / q3[0] + sqrt(gm * p3 / q3[0]), l4r = ur + sqrt(gm * pp[1] / rr);
                const bool fix = (l1l < 0.0 && l1r > 0.0) || (l4l < 0.0 && l4r > 0.0);
                kp = !fix && sp[0] < 0.0 && sp[3] > 0.0;
            }
        }
        keep[i] = kp ? 1 : 0;
        float* yr = Y + i * 16;
        if (!kp) {
            for (int j = 0; j < 16; ++j) yr[j] = 0.0f;
            continue;
        }
        yr[0] = (float)(sp[0] / c0);
        yr[1] = (float)(sp[1] / c0);
        yr[2] = (float)(sp[3] / c0);
        for (int k = 0; k < 4; ++k) {
            yr[3 + k] = (float)(w[0][k] / (m * S[k]));
            yr[7 + k] = (float)((w[1][k] + w[2][k]) / (m * S[k]));
            yr[11 + k] = (float)(w[3][k] / (m * S[k]));
        }
        yr[15] = 0.0f;
    }
}

// stable compaction: counts per chunk, scan, scatter
constexpr int CCHUNK = 4096;  // rows per workgroup (256 threads x 16)
__global__ void count_kernel(const int32_t* __restrict__ keep, int64_t n, int32_t* __restrict__ cnt)
{
    __shared__ int s[256];
    const int64_t b0 = (int64_t)blockIdx.x * CCHUNK + threadIdx.x * 16;
    int c = 0;
    for (int j = 0; j < 16; ++j)
        if (b0 + j < n && keep[b0 + j]) ++c;
    s[threadIdx.x] = c;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) cnt[blockIdx.x] = s[0];
}

// exclusive scan of nb counts in one workgroup; total into *tot
__global__ void scan_kernel(int32_t* __restrict__ cnt, int nb, long long* __restrict__ tot)
{
    __shared__ long long s[1024];
    long long carry = 0;
    for (int base = 0; base < nb; base += 1024) {
        const int i = base + threadIdx.x;
        const long long v = i < nb ? cnt[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const long long t = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nb) cnt[i] = (int32_t)(carry + s[threadIdx.x] - v);
        const long long last = s[1023];
        __syncthreads();
        carry += last;
    }
    if (threadIdx.x == 0) *tot = carry;
}

// X rows of 8 floats, Y rows of ys floats (8 or 16)
__global__ void scatter_kernel(const int32_t* __restrict__ keep, int64_t n, const int32_t* __restrict__ off,
                               const float* __restrict__ X, const float* __restrict__ Y, int ys,
                               float* __restrict__ Xc, float* __restrict__ Yc)
{
    __shared__ int s[256];
    const int64_t b0 = (int64_t)blockIdx.x * CCHUNK + threadIdx.x * 16;
    int c = 0;
    for (int j = 0; j < 16; ++j)
        if (b0 + j < n && keep[b0 + j]) ++c;
    s[threadIdx.x] = c;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const int t = (int)threadIdx.x >= o ? s[threadIdx.x - o] : 0;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    int64_t pos = (int64_t)off[blockIdx.x] + s[threadIdx.x] - c;
    for (int j = 0; j < 16; ++j) {
        const int64_t i = b0 + j;
        if (i < n && keep[i]) {
            const float4* xs = reinterpret_cast<const float4*>(X + i * 8);
            float4* xd = reinterpret_cast<float4*>(Xc + pos * 8);
            xd[0] = xs[0]; xd[1] = xs[1];
            const float4* yss = reinterpret_cast<const float4*>(Y + i * ys);
            float4* yd = reinterpret_cast<float4*>(Yc + pos * ys);
            for (int k = 0; k < ys / 4; ++k) yd[k] = yss[k];
            ++pos;
        }
    }
}

// ------------------------------------------------------------ training GEMM
// C[M][N] = sum_k A(m, k) B(k, n) on 64x64 tiles, 4 wavefronts of 32x32,
// k in steps of 32 through LDS; FP32 accumulation.  Operand modes:
//   AM 0: A(m, k) = A[m lda + k] (k contiguous); 1: A[k lda + m]
//   BM 0: B(k, n) = B[n ldb + k] (k contiguous); 1: B[k ldb + n]
// blockIdx.z picks the k-range [z kchunk, (z + 1) kchunk) (split-K).
constexpr int TROW = 40;  // bf16 per LDS tile row (32 + 8 padding)

template <int MODE>
__device__ __forceinline__ void load_tile(const bf16* __restrict__ X, int64_t ld, int r0, int k0, int R,
                                          int ke, bf16* __restrict__ s)
{
    const int t = threadIdx.x;
    if (MODE == 0) {
        const int row = t >> 2, kq = (t & 3) * 8;
        const int r = r0 + row, k = k0 + kq;
        bf16x8 v = zero8();
        if (r < R) {
            const bf16* src = X + (int64_t)r * ld + k;
            if (k + 8 <= ke) {
                v = *reinterpret_cast<const bf16x8*>(src);
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    if (k + j < ke) v[j] = src[j];
            }
        }
        *reinterpret_cast<bf16x8*>(s + row * TROW + kq) = v;
    } else {
        const int kk = t >> 3, rq = (t & 7) * 8;
        const int k = k0 + kk, r = r0 + rq;
        bf16x8 v = zero8();
        if (k < ke) {
            const bf16* src = X + (int64_t)k * ld + r;
            if (r + 8 <= R) {
                v = *reinterpret_cast<const bf16x8*>(src);
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    if (r + j < R) v[j] = src[j];
            }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) s[(rq + j) * TROW + kk] = v[j];
    }
}

template <int AM, int BM, class EPI>
__global__ __launch_bounds__(256) void gemm_kernel(const bf16* __restrict__ A, int64_t lda,
                                                   const bf16* __restrict__ B, int64_t ldb, int M, int N,
                                                   int K, int kchunk, EPI epi)
{
    __shared__ __attribute__((aligned(16))) bf16 sA[64 * TROW];
    __shared__ __attribute__((aligned(16))) bf16 sB[64 * TROW];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
    const int kb = blockIdx.z * kchunk;
    const int ke = min(K, kb + kchunk);
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = kb; k0 < ke; k0 += 32) {
        load_tile<AM>(A, lda, m0, k0, M, ke, sA);
        load_tile<BM>(B, ldb, n0, k0, N, ke, sB);
        __syncthreads();
        bf16x8 af[2], bfr[2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
            af[i] = *reinterpret_cast<const bf16x8*>(sA + (wm + 16 * i + (lane & 15)) * TROW + 8 * (lane >> 4));
#pragma unroll
        for (int j = 0; j < 2; ++j)
            bfr[j] = *reinterpret_cast<const bf16x8*>(sB + (wn + 16 * j + (lane & 15)) * TROW + 8 * (lane >> 4));
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = mfma(af[i], bfr[j], acc[i][j]);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
                const int n = n0 + wn + 16 * j + (lane & 15);
                if (m < M && n < N) epi(m, n, acc[i][j][r], (int)blockIdx.z);
            }
}

// hidden layer forward: Z = acc + b, A_next = bf16(gelu(Z))
struct EpiHidden {
    const float* bias;
    float* Z;
    bf16* An;
    int ld;
    __device__ void operator()(int m, int n, float v, int) const
    {
        const float z = v + bias[n];
        Z[(int64_t)m * ld + n] = z;
        An[(int64_t)m * ld + n] = (bf16)gelu(z);
    }
};
struct EpiOut {
    const float* bias;
    float* out;
    int ld;
    __device__ void operator()(int m, int n, float v, int) const { out[(int64_t)m * ld + n] = v + bias[n]; }
};
// backward through GELU: dZ_prev = acc * gelu'(Z_prev)
struct EpiBack {
    const float* Zp;
    float* dZf;
    bf16* dZb;
    int ld;
    __device__ void operator()(int m, int n, float v, int) const
    {
        const int64_t i = (int64_t)m * ld + n;
        const float dz = v * gelu_grad(Zp[i]);
        dZf[i] = dz;
        dZb[i] = (bf16)dz;
    }
};
struct EpiPart {
    float* part;
    int M, N;
    __device__ void operator()(int m, int n, float v, int z) const
    {
        part[((int64_t)z * M + m) * N + n] = v;
    }
};

__global__ void to_bf16_rows_kernel(const float* __restrict__ X, int64_t n, int nin, bf16* __restrict__ A0)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * 8) return;
    const int c = (int)(i & 7);
    A0[i] = (bf16)(c < nin ? X[i] : 0.0f);
}

// dOut = 2 (out - Y) / (nout n) on the nout real columns of rows of stride
// ys (the padding columns of dOut are written 0); partial sums of squared
// errors per workgroup
__global__ void loss_kernel(const float* __restrict__ out, const float* __restrict__ Y, int64_t n, int nout,
                            int ys, float* __restrict__ dZf, bf16* __restrict__ dZb, float* __restrict__ part)
{
    __shared__ float s[256];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    float acc = 0.0f;
    if (i < n * ys) {
        const int c = (int)(i % ys);
        float gz = 0.0f;
        if (c < nout) {
            const float d = out[i] - Y[i];
            acc = d * d;
            gz = d * (2.0f / ((float)nout * (float)n));
        }
        dZf[i] = gz;
        dZb[i] = (bf16)gz;
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// sums nb partials in a fixed order; loss = sum / (nout n), also added to *acc
__global__ void loss_final_kernel(const float* __restrict__ part, int nb, int64_t n, int nout,
                                  float* __restrict__ loss, double* __restrict__ acc)
{
    __shared__ double s[256];
    double v = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) v += part[i];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double L = s[0] / ((double)nout * (double)n);
        if (loss) *loss = (float)L;
        if (acc) *acc += L;
    }
}

// column sums of dZ (rows of stride ld, first W columns) over row chunks of
// 256: part[chunk][c]
__global__ void colsum_kernel(const float* __restrict__ dZ, int64_t n, int W, int ld, float* __restrict__ part)
{
    __shared__ float s[256];
    const int rstep = 256 / W;
    const int c = threadIdx.x % W, r = threadIdx.x / W;
    const int64_t r0 = (int64_t)blockIdx.x * 256;
    float v = 0.0f;
    if (r < rstep)
        for (int64_t i = r0 + r; i < r0 + 256 && i < n; i += rstep) v += dZ[i * ld + c];
    s[threadIdx.x] = v;
    __syncthreads();
    if ((int)threadIdx.x < W) {
        float t = 0.0f;
        for (int k = 0; k < rstep; ++k) t += s[k * W + threadIdx.x];
        part[(int64_t)blockIdx.x * W + threadIdx.x] = t;
    }
}

// gradient of layer l from split-K partials [nz][out][inpad] and bias
// partials [nbp][out]
template <class NT>
__global__ void grad_reduce_kernel(const float* __restrict__ wpart, int nz, const float* __restrict__ bpart,
                                   int nbp, int l, float* __restrict__ grad)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int no = NT::l_out(l), ni = NT::l_in(l), np = NT::l_inpad(l);
    if (idx < no * ni) {
        const int o = idx / ni, i = idx % ni;
        float v = 0.0f;
        for (int z = 0; z < nz; ++z) v += wpart[((int64_t)z * no + o) * np + i];
        grad[NT::w_off(l) + idx] = v;
    } else if (idx < no * ni + no) {
        const int o = idx - no * ni;
        float v = 0.0f;
        for (int z = 0; z < nbp; ++z) v += bpart[(int64_t)z * no + o];
        grad[NT::b_off(l) + o] = v;
    }
}

// squared error over the nout real columns of rows of stride ys, partial
// sums per workgroup (evaluation)
__global__ void sqerr_kernel(const float* __restrict__ out, const float* __restrict__ Y, int64_t n, int nout,
                             int ys, double* __restrict__ part)
{
    __shared__ double s[256];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n * ys; i += (int64_t)gridDim.x * 256) {
        if ((int)(i % ys) < nout) {
            const double d = (double)out[i] - (double)Y[i];
            acc += d * d;
        }
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

}  // namespace sur
}  // namespace mc

using namespace mc;
using namespace mc::sur;

// ------------------------------------------------------------------ host side
struct mc_sur {
    int model;          // MC_SW_SURROGATE or MC_EULER_SURROGATE
    int np, nin, nout, ys, ntrain;
    hipStream_t stream;
    int max_batch;
    int cus;
    float* params;      // np FP32 master
    float* madam;
    float* vadam;
    float* grad;
    int64_t t;          // Adam steps taken
    uint16_t* img;      // inference image (IMG_BYTES)
    bf16* wt;           // training copies (ntrain)
    // training workspace (max_batch rows)
    bf16* A[NLAYER];    // layer inputs: A[0] [B][8], A[1..4] [B][128]
    float* Z[NLAYER];   // pre-activations of hidden layers 0..3 [B][128]
    float* out;         // [B][ys]
    float* dZf[2];      // [B][128] ping-pong (output layer: rows of ys)
    bf16* dZb[2];
    float* wpart;       // split-K partials
    float* bpart;       // bias partials
    float* lpart;       // loss partials
    float* loss;        // device scalar
    double* lacc;       // device epoch accumulator
    std::vector<void*> owned;
};

namespace {

constexpr int KCHUNK = 256;  // rows per split of the weight-gradient products

int hip_check(hipError_t e)
{
    if (e != hipSuccess) {
        fprintf(stderr, "manyclaw: HIP error %s\n", hipGetErrorString(e));
        return MC_EHIP;
    }
    return MC_OK;
}

template <typename T>
int alloc(mc_sur* s, T** p, size_t count)
{
    void* v = nullptr;
    const hipError_t e = hipMalloc(&v, count * sizeof(T) + 16);
    if (e != hipSuccess) {
        *p = nullptr;
        return e == hipErrorOutOfMemory ? MC_ENOMEM : MC_EHIP;
    }
    s->owned.push_back(v);
    *p = (T*)v;
    return MC_OK;
}

int nsplit(int64_t n) { return (int)((n + KCHUNK - 1) / KCHUNK); }

template <class M>
int repack_t(mc_sur* s)
{
    using NT = typename M::N;
    const int nimg = NFRAG * 64 * 8 + NBIAS;
    hipLaunchKernelGGL((pack_image_kernel<NT>), dim3((nimg + 255) / 256), dim3(256), 0, s->stream, s->params,
                       s->img);
    hipLaunchKernelGGL((pack_train_kernel<NT>), dim3((NT::NTRAIN + 255) / 256), dim3(256), 0, s->stream,
                       s->params, s->wt);
    return hip_check(hipGetLastError());
}

int repack(mc_sur* s)
{
    return s->model == MC_EULER_SURROGATE ? repack_t<EulerModel>(s) : repack_t<SwModel>(s);
}

int reset_adam(mc_sur* s)
{
    s->t = 0;
    if (hip_check(hipMemsetAsync(s->madam, 0, s->np * sizeof(float), s->stream)) != MC_OK) return MC_EHIP;
    if (hip_check(hipMemsetAsync(s->vadam, 0, s->np * sizeof(float), s->stream)) != MC_OK) return MC_EHIP;
    return repack(s);
}

template <int AM, int BM, class EPI>
void gemm(hipStream_t st, const bf16* A, int64_t lda, const bf16* B, int64_t ldb, int M, int N, int K,
          int kchunk, EPI epi)
{
    const int nz = (K + kchunk - 1) / kchunk;
    dim3 grid((M + 63) / 64, (N + 63) / 64, nz > 0 ? nz : 1);
    hipLaunchKernelGGL((gemm_kernel<AM, BM, EPI>), grid, dim3(256), 0, st, A, lda, B, ldb, M, N, K, kchunk, epi);
}

// forward of n rows already in s->A[0], loss against Y (rows of YS), backward
// into s->grad
template <class M>
int loss_grad_t(mc_sur* s, int64_t n64, const float* Y, float* loss_out, double* lacc)
{
    using NT = typename M::N;
    const int n = (int)n64;
    hipStream_t st = s->stream;
    // forward
    for (int l = 0; l < NLAYER; ++l) {
        const bf16* W = s->wt + NT::t_off(l);
        const float* bias = s->params + NT::b_off(l);
        const int K = NT::l_inpad(l);
        if (l < NLAYER - 1) {
            EpiHidden e{bias, s->Z[l], s->A[l + 1], WID};
            gemm<0, 0>(st, s->A[l], K, W, K, n, WID, K, K, e);
        } else {
            EpiOut e{bias, s->out, NT::YS};
            gemm<0, 0>(st, s->A[l], K, W, K, n, NT::NOUT, K, K, e);
        }
    }
    // loss and its gradient w.r.t. the outputs
    const int nlb = (int)((n64 * NT::YS + 255) / 256);
    hipLaunchKernelGGL(loss_kernel, dim3(nlb), dim3(256), 0, st, s->out, Y, n64, NT::NOUT, NT::YS, s->dZf[0],
                       s->dZb[0], s->lpart);
    hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(256), 0, st, s->lpart, nlb, n64, NT::NOUT,
                       loss_out ? loss_out : s->loss, lacc);
    // backward
    int cur = 0;
    for (int l = NLAYER - 1; l >= 0; --l) {
        const int no = NT::l_out(l), np = NT::l_inpad(l);
        const int ld = l == NLAYER - 1 ? NT::YS : WID;   // row stride of dZ
        // dW = dZ^T A: M = out, N = inpad, K = n (split)
        EpiPart ep{s->wpart, no, np};
        gemm<1, 1>(st, s->dZb[cur], ld, s->A[l], np, no, np, n, KCHUNK, ep);
        const int ncb = (n + 255) / 256;
        hipLaunchKernelGGL(colsum_kernel, dim3(ncb), dim3(256), 0, st, s->dZf[cur], n64, no, ld, s->bpart);
        const int ng = no * NT::l_in(l) + no;
        hipLaunchKernelGGL((grad_reduce_kernel<NT>), dim3((ng + 255) / 256), dim3(256), 0, st, s->wpart,
                           nsplit(n), s->bpart, ncb, l, s->grad);
        if (l > 0) {
            // dA = dZ W: M = n, N = inpad(l) = 128, K = out; times gelu'(Z_{l-1})
            EpiBack eb{s->Z[l - 1], s->dZf[cur ^ 1], s->dZb[cur ^ 1], WID};
            gemm<0, 1>(st, s->dZb[cur], ld, s->wt + NT::t_off(l), np, n, np, no, no, eb);
            cur ^= 1;
        }
    }
    return hip_check(hipGetLastError());
}

int loss_grad_core(mc_sur* s, int64_t n, const float* Y, float* loss_out, double* lacc)
{
    return s->model == MC_EULER_SURROGATE ? loss_grad_t<EulerModel>(s, n, Y, loss_out, lacc)
                                          : loss_grad_t<SwModel>(s, n, Y, loss_out, lacc);
}

int launch_adam(mc_sur* s, float lr, float b1, float b2, float eps)
{
    s->t += 1;
    const double c1 = 1.0 / (1.0 - pow((double)b1, (double)s->t));
    const double c2 = 1.0 / (1.0 - pow((double)b2, (double)s->t));
    hipLaunchKernelGGL(adam_kernel, dim3((s->np + 255) / 256), dim3(256), 0, s->stream, s->params, s->madam,
                       s->vadam, s->grad, s->np, lr, b1, b2, eps, (float)c1, (float)c2);
    if (hip_check(hipGetLastError()) != MC_OK) return MC_EHIP;
    return repack(s);
}

int edge_blocks(int cus, int64_t n)
{
    const int64_t tiles = (n + 63) / 64;
    int64_t nb = (tiles + EWAVES - 1) / EWAVES;
    if (nb > cus) nb = cus;
    return nb < 1 ? 1 : (int)nb;
}

template <class M, int MODE, int IXY>
int launch_edges(const EdgeArgs& a, int cus, hipStream_t st)
{
    static bool attr = false;
    if (!attr) {
        if (hip_check(hipFuncSetAttribute((const void*)edge_kernel<M, MODE, IXY>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)EDGE_LDS)) != MC_OK)
            return MC_EHIP;
        attr = true;
    }
    hipLaunchKernelGGL((edge_kernel<M, MODE, IXY>), dim3(edge_blocks(cus, a.n)), dim3(EBLOCK), EDGE_LDS, st, a);
    return hip_check(hipGetLastError());
}

template <class M, int IXY>
void launch_update(const UpdArgs& u, int limiter, int64_t ub, hipStream_t st)
{
    constexpr int ME = M::MEQN, MW = M::MW;
    switch (limiter) {
    case MC_LIM_NONE: hipLaunchKernelGGL((update_kernel<ME, MW, IXY, LIM_NONE>), dim3(ub), dim3(256), 0, st, u); break;
    case MC_LIM_MINMOD: hipLaunchKernelGGL((update_kernel<ME, MW, IXY, LIM_MINMOD>), dim3(ub), dim3(256), 0, st, u); break;
    case MC_LIM_SUPERBEE: hipLaunchKernelGGL((update_kernel<ME, MW, IXY, LIM_SUPERBEE>), dim3(ub), dim3(256), 0, st, u); break;
    case MC_LIM_VANLEER: hipLaunchKernelGGL((update_kernel<ME, MW, IXY, LIM_VANLEER>), dim3(ub), dim3(256), 0, st, u); break;
    case MC_LIM_MC: hipLaunchKernelGGL((update_kernel<ME, MW, IXY, LIM_MC>), dim3(ub), dim3(256), 0, st, u); break;
    default: hipLaunchKernelGGL((update_kernel<ME, MW, IXY, LIM_FIRST_ORDER>), dim3(ub), dim3(256), 0, st, u); break;
    }
}

// per-context state of the surrogate step
struct SurCtx {
    mc_sur* net = nullptr;
    float* qs = nullptr;       // intermediate state after the x-sweep
    float* rec = nullptr;      // edge records
    size_t rec_elems = 0;
    unsigned int* red = nullptr;  // smax bits: [0] x-sweep, [1] y-sweep, [2] mc_rp2
    unsigned long long* counts = nullptr;  // [2]
};
// per-context surrogate state; the map is shared by every thread, each
// context's entry is used by the thread that owns the context
std::map<const mc_ctx*, SurCtx> g_ctx;
std::mutex g_ctx_mu;

// the entry of context c, or null
SurCtx* find_ctx(const mc_ctx* c)
{
    std::lock_guard<std::mutex> lk(g_ctx_mu);
    auto it = g_ctx.find(c);
    return it == g_ctx.end() ? nullptr : &it->second;
}

bool model_ok(int model) { return model == MC_SW_SURROGATE || model == MC_EULER_SURROGATE; }

template <class M>
int sur_rp2_t(SurCtx& sc, const mc_params& prm, int cus, hipStream_t st, unsigned int* status, int ixy,
              int64_t n, const void* ql, const void* qr, void* waves, void* speeds, void* amdq, void* apdq)
{
    EdgeArgs a;
    memset(&a, 0, sizeof(a));
    a.img = reinterpret_cast<const uint4*>(sc.net->img);
    a.P.g = prm.g;
    a.P.gamma = prm.gamma;
    a.n = n;
    a.ql = (const float*)ql;
    a.qr = (const float*)qr;
    a.waves = (float*)waves;
    a.speeds = (float*)speeds;
    a.amdq = (float*)amdq;
    a.apdq = (float*)apdq;
    a.smax_bits = sc.red + 2;
    a.counts = sc.counts;
    a.status = status;
    return ixy == 1 ? launch_edges<M, MODE_ARRAYS, 1>(a, cus, st) : launch_edges<M, MODE_ARRAYS, 2>(a, cus, st);
}

template <class M>
int sur_step_t(SurCtx& sc, const mc_params& prm, int cus, hipStream_t st, int nx, int ny, double dx, double dy,
               unsigned int* status, mc_state* stt, double dt, int limiter, int bc, mc_cfl* cfl_out)
{
    constexpr int ME = M::MEQN;
    const int64_t plane = (int64_t)nx * ny;
    const int64_t nex = (int64_t)(nx + 3) * ny, ney = (int64_t)(ny + 3) * nx;
    const size_t need = (size_t)M::NREC * (size_t)(nex > ney ? nex : ney);
    if (!sc.qs) {
        if (hipMalloc((void**)&sc.qs, ME * plane * sizeof(float)) != hipSuccess) return MC_ENOMEM;
    }
    if (sc.rec_elems < need) {
        (void)hipFree(sc.rec);
        sc.rec = nullptr;
        sc.rec_elems = 0;
        if (hipMalloc((void**)&sc.rec, need * sizeof(float)) != hipSuccess) return MC_ENOMEM;
        sc.rec_elems = need;
    }
    const float* q0 = (const float*)stt->q[stt->cur];
    float* q1 = (float*)stt->q[stt->cur ^ 1];

    EdgeArgs a;
    memset(&a, 0, sizeof(a));
    a.img = reinterpret_cast<const uint4*>(sc.net->img);
    a.P.g = prm.g;
    a.P.gamma = prm.gamma;
    a.nx = nx;
    a.ny = ny;
    a.bc = bc;
    a.rec = sc.rec;
    a.counts = sc.counts;
    a.status = status;
    UpdArgs u;
    u.rec = sc.rec;
    u.nx = nx;
    u.ny = ny;
    int64_t ub = (plane + 255) / 256;
    if (ub > (int64_t)cus * 32) ub = (int64_t)cus * 32;

    int r;
    // x-sweep
    a.q = q0;
    a.n = nex;
    a.smax_bits = sc.red + 0;
    r = launch_edges<M, MODE_SWEEP, 1>(a, cus, st);
    if (r != MC_OK) return r;
    u.q = q0; u.qo = sc.qs; u.n = nex; u.nu = (float)(dt / dx);
    launch_update<M, 1>(u, limiter, ub, st);
    if ((r = hip_check(hipGetLastError())) != MC_OK) return r;
    // y-sweep on the x-swept state
    a.q = sc.qs;
    a.n = ney;
    a.smax_bits = sc.red + 1;
    r = launch_edges<M, MODE_SWEEP, 2>(a, cus, st);
    if (r != MC_OK) return r;
    u.q = sc.qs; u.qo = q1; u.n = ney; u.nu = (float)(dt / dy);
    launch_update<M, 2>(u, limiter, ub, st);
    if ((r = hip_check(hipGetLastError())) != MC_OK) return r;
    FinArgs f;
    f.smax_bits = sc.red;
    f.cfl = cfl_out;
    f.dx = dx;
    f.dy = dy;
    f.dt = dt;
    hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(64), 0, st, f);
    if ((r = hip_check(hipGetLastError())) != MC_OK) return r;
    stt->cur ^= 1;
    return MC_OK;
}

}  // namespace

extern "C" {

int mc__ctx_info(const mc_ctx* c, int* solver, int* dtype, mc_params* prm, int* cus, void** stream);
int mc__ctx_grid(const mc_ctx* c, int* nx, int* ny, double* dx, double* dy, unsigned int** status);

int mc_sur_dims(int32_t model, int32_t* nparams, int32_t* nin, int32_t* nout, int32_t* ystride)
{
    if (!model_ok(model) || !nparams || !nin || !nout || !ystride) return MC_EINVAL;
    if (model == MC_EULER_SURROGATE) {
        using NT = EulerModel::N;
        *nparams = NT::NPARAMS; *nin = NT::NIN; *nout = NT::NOUT; *ystride = NT::YS;
    } else {
        using NT = SwModel::N;
        *nparams = NT::NPARAMS; *nin = NT::NIN; *nout = NT::NOUT; *ystride = NT::YS;
    }
    return MC_OK;
}

int mc_sur_create(mc_sur** out, int32_t model, int32_t max_batch, void* hip_stream)
{
    if (!out || !model_ok(model) || max_batch < 1 || max_batch > (1 << 20)) return MC_EINVAL;
    *out = nullptr;
    mc_sur* s = new mc_sur();
    s->model = model;
    if (model == MC_EULER_SURROGATE) {
        using NT = EulerModel::N;
        s->np = NT::NPARAMS; s->nin = NT::NIN; s->nout = NT::NOUT; s->ys = NT::YS; s->ntrain = NT::NTRAIN;
    } else {
        using NT = SwModel::N;
        s->np = NT::NPARAMS; s->nin = NT::NIN; s->nout = NT::NOUT; s->ys = NT::YS; s->ntrain = NT::NTRAIN;
    }
    s->stream = (hipStream_t)hip_stream;
    s->max_batch = max_batch;
    s->t = 0;
    s->cus = 256;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
        s->cus = cus;
    const size_t B = (size_t)max_batch;
    const int nz = nsplit(max_batch), ncb = (max_batch + 255) / 256, nlb = (int)((B * s->ys + 255) / 256);
    int r = MC_OK;
    r = r ? r : alloc(s, &s->params, s->np);
    r = r ? r : alloc(s, &s->madam, s->np);
    r = r ? r : alloc(s, &s->vadam, s->np);
    r = r ? r : alloc(s, &s->grad, s->np);
    r = r ? r : alloc(s, &s->img, IMG_BYTES / 2);
    r = r ? r : alloc(s, &s->wt, s->ntrain);
    r = r ? r : alloc(s, &s->A[0], B * 8);
    for (int l = 1; l < NLAYER; ++l) r = r ? r : alloc(s, &s->A[l], B * WID);
    for (int l = 0; l < NLAYER - 1; ++l) r = r ? r : alloc(s, &s->Z[l], B * WID);
    s->Z[NLAYER - 1] = nullptr;
    r = r ? r : alloc(s, &s->out, B * s->ys);
    for (int k = 0; k < 2; ++k) {
        r = r ? r : alloc(s, &s->dZf[k], B * WID);
        r = r ? r : alloc(s, &s->dZb[k], B * WID);
    }
    r = r ? r : alloc(s, &s->wpart, (size_t)nz * WID * WID);
    r = r ? r : alloc(s, &s->bpart, (size_t)ncb * WID);
    r = r ? r : alloc(s, &s->lpart, (size_t)nlb);
    r = r ? r : alloc(s, &s->loss, 1);
    r = r ? r : alloc(s, &s->lacc, 1);
    if (r == MC_OK) r = hip_check(hipMemsetAsync(s->params, 0, s->np * sizeof(float), s->stream));
    if (r == MC_OK) r = reset_adam(s);
    if (r == MC_OK) r = hip_check(hipStreamSynchronize(s->stream));
    if (r != MC_OK) {
        mc_sur_destroy(s);
        return r;
    }
    *out = s;
    return MC_OK;
}

void mc_sur_destroy(mc_sur* s)
{
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    {
        std::lock_guard<std::mutex> lk(g_ctx_mu);
        for (auto& kv : g_ctx)
            if (kv.second.net == s) kv.second.net = nullptr;
    }
    for (void* p : s->owned) (void)hipFree(p);
    delete s;
}

int mc_sur_set_params(mc_sur* s, const float* params)
{
    if (!s || !params) return MC_EINVAL;
    if (hip_check(hipMemcpyAsync(s->params, params, s->np * sizeof(float), hipMemcpyDeviceToDevice,
                                 s->stream)) != MC_OK)
        return MC_EHIP;
    return reset_adam(s);
}

int mc_sur_get_params(mc_sur* s, float* params)
{
    if (!s || !params) return MC_EINVAL;
    return hip_check(hipMemcpyAsync(params, s->params, s->np * sizeof(float), hipMemcpyDeviceToDevice,
                                    s->stream));
}

int mc_sur_init_params(mc_sur* s, const double* uniforms)
{
    if (!s || !uniforms) return MC_EINVAL;
    if (s->model == MC_EULER_SURROGATE)
        hipLaunchKernelGGL((init_params_kernel<EulerModel::N>), dim3((s->np + 255) / 256), dim3(256), 0,
                           s->stream, uniforms, s->params);
    else
        hipLaunchKernelGGL((init_params_kernel<SwModel::N>), dim3((s->np + 255) / 256), dim3(256), 0,
                           s->stream, uniforms, s->params);
    if (hip_check(hipGetLastError()) != MC_OK) return MC_EHIP;
    return reset_adam(s);
}

int mc_sur_gen(mc_sur* s, const mc_params* prm, int64_t n, const double* U, float* X, float* Y, int32_t* keep)
{
    if (!s || !prm || n < 0) return MC_EINVAL;
    const bool eu = s->model == MC_EULER_SURROGATE;
    if (eu ? !(prm->gamma > 1.0) : !(prm->g > 0.0)) return MC_EINVAL;
    if (n == 0) return MC_OK;
    if (!U || !X || !Y || !keep) return MC_EINVAL;
    int64_t nb = (n + 255) / 256;
    if (nb > (int64_t)s->cus * 64) nb = (int64_t)s->cus * 64;
    if (eu)
        hipLaunchKernelGGL(gen_euler_kernel, dim3((unsigned)nb), dim3(256), 0, s->stream, U, n, prm->gamma, X, Y,
                           keep);
    else
        hipLaunchKernelGGL(gen_sw_kernel, dim3((unsigned)nb), dim3(256), 0, s->stream, U, n, prm->g, X, Y, keep);
    return hip_check(hipGetLastError());
}

int mc_sur_compact(mc_sur* s, int64_t n, const float* X, const float* Y, const int32_t* keep, float* Xc,
                   float* Yc, int64_t* n_kept)
{
    if (!s || n < 0 || !n_kept) return MC_EINVAL;
    *n_kept = 0;
    if (n == 0) return MC_OK;
    if (!X || !Y || !keep || !Xc || !Yc) return MC_EINVAL;
    const int64_t nb = (n + CCHUNK - 1) / CCHUNK;
    if (nb > (1 << 24)) return MC_EINVAL;
    int32_t* cnt = nullptr;
    long long* tot = nullptr;
    if (hip_check(hipMalloc((void**)&cnt, nb * sizeof(int32_t))) != MC_OK) return MC_ENOMEM;
    if (hip_check(hipMalloc((void**)&tot, sizeof(long long))) != MC_OK) {
        (void)hipFree(cnt);
        return MC_ENOMEM;
    }
    hipLaunchKernelGGL(count_kernel, dim3((unsigned)nb), dim3(256), 0, s->stream, keep, n, cnt);
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s->stream, cnt, (int)nb, tot);
    hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)nb), dim3(256), 0, s->stream, keep, n, cnt, X, Y, s->ys, Xc,
                       Yc);
    int r = hip_check(hipGetLastError());
    long long t = 0;
    if (r == MC_OK) r = hip_check(hipMemcpyAsync(&t, tot, sizeof(t), hipMemcpyDeviceToHost, s->stream));
    if (r == MC_OK) r = hip_check(hipStreamSynchronize(s->stream));
    (void)hipFree(cnt);
    (void)hipFree(tot);
    *n_kept = t;
    return r;
}

int mc_sur_forward(mc_sur* s, int64_t n, const float* X, float* out)
{
    if (!s || n < 0) return MC_EINVAL;
    if (n == 0) return MC_OK;
    if (!X || !out) return MC_EINVAL;
    EdgeArgs a;
    memset(&a, 0, sizeof(a));
    a.img = reinterpret_cast<const uint4*>(s->img);
    a.n = n;
    a.X = X;
    a.out = out;
    return s->model == MC_EULER_SURROGATE ? launch_edges<EulerModel, MODE_NET, 1>(a, s->cus, s->stream)
                                          : launch_edges<SwModel, MODE_NET, 1>(a, s->cus, s->stream);
}

int mc_sur_loss_grad(mc_sur* s, int64_t n, const float* X, const float* Y, float* grad, float* loss)
{
    if (!s || n < 1 || n > s->max_batch || !X || !Y) return MC_EINVAL;
    hipLaunchKernelGGL(to_bf16_rows_kernel, dim3((unsigned)((n * 8 + 255) / 256)), dim3(256), 0, s->stream, X, n,
                       s->nin, s->A[0]);
    int r = loss_grad_core(s, n, Y, loss, nullptr);
    if (r == MC_OK && grad)
        r = hip_check(hipMemcpyAsync(grad, s->grad, s->np * sizeof(float), hipMemcpyDeviceToDevice, s->stream));
    return r;
}

int mc_sur_adam(mc_sur* s, float lr, float beta1, float beta2, float eps)
{
    if (!s || !(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !(eps > 0.0f))
        return MC_EINVAL;
    return launch_adam(s, lr, beta1, beta2, eps);
}

int mc_sur_train(mc_sur* s, int64_t n, const float* X, const float* Y, int32_t batch, int32_t epochs,
                 float lr0, const int32_t* order, float* loss_host)
{
    if (!s || !X || !Y || batch < 1 || batch > s->max_batch || epochs < 0 || !(lr0 >= 0.0f)) return MC_EINVAL;
    const int64_t nbat = n / batch;
    if (nbat < 1 || (epochs > 0 && !order)) return MC_EINVAL;
    for (int64_t i = 0; i < (int64_t)epochs * nbat; ++i)
        if (order[i] < 0 || order[i] >= nbat) return MC_EINVAL;
    const double total = (double)epochs * (double)nbat;
    int64_t it = 0;
    for (int e = 0; e < epochs; ++e) {
        if (hip_check(hipMemsetAsync(s->lacc, 0, sizeof(double), s->stream)) != MC_OK) return MC_EHIP;
        for (int64_t k = 0; k < nbat; ++k) {
            const int64_t b = order[(int64_t)e * nbat + k];
            const float* xb = X + b * batch * 8;
            const float* yb = Y + b * batch * s->ys;
            hipLaunchKernelGGL(to_bf16_rows_kernel, dim3((unsigned)(((int64_t)batch * 8 + 255) / 256)), dim3(256),
                               0, s->stream, xb, (int64_t)batch, s->nin, s->A[0]);
            int r = loss_grad_core(s, batch, yb, nullptr, s->lacc);
            if (r != MC_OK) return r;
            const float lr = (float)(0.5 * (double)lr0 * (1.0 + cos(M_PI * (double)it / total)));
            r = launch_adam(s, lr, 0.9f, 0.999f, 1e-8f);
            if (r != MC_OK) return r;
            ++it;
        }
        double acc = 0.0;
        if (hip_check(hipMemcpyAsync(&acc, s->lacc, sizeof(double), hipMemcpyDeviceToHost, s->stream)) != MC_OK)
            return MC_EHIP;
        if (hip_check(hipStreamSynchronize(s->stream)) != MC_OK) return MC_EHIP;
        if (loss_host) loss_host[e] = (float)(acc / (double)nbat);
    }
    return MC_OK;
}

int mc_sur_eval(mc_sur* s, int64_t n, const float* X, const float* Y, double* loss_host)
{
    if (!s || n < 1 || !X || !Y || !loss_host) return MC_EINVAL;
    // chunks of the training workspace's output buffer
    const int64_t chunk = s->max_batch;
    const int nb = 256;
    double* part = nullptr;
    if (hip_check(hipMalloc((void**)&part, nb * sizeof(double))) != MC_OK) return MC_ENOMEM;
    double total = 0.0;
    int r = MC_OK;
    std::vector<double> hp(nb);
    for (int64_t o = 0; o < n && r == MC_OK; o += chunk) {
        const int64_t m = (n - o) < chunk ? (n - o) : chunk;
        r = mc_sur_forward(s, m, X + o * 8, s->out);
        if (r != MC_OK) break;
        hipLaunchKernelGGL(sqerr_kernel, dim3(nb), dim3(256), 0, s->stream, s->out, Y + o * s->ys, m, s->nout,
                           s->ys, part);
        r = hip_check(hipGetLastError());
        if (r == MC_OK) r = hip_check(hipMemcpyAsync(hp.data(), part, nb * sizeof(double), hipMemcpyDeviceToHost,
                                                     s->stream));
        if (r == MC_OK) r = hip_check(hipStreamSynchronize(s->stream));
        for (int i = 0; i < nb && r == MC_OK; ++i) total += hp[i];
    }
    (void)hipFree(part);
    *loss_host = total / ((double)s->nout * (double)n);
    return r;
}

// ------------------------------------------------------------ contexts
int mc_ctx_set_surrogate(mc_ctx* c, mc_sur* s)
{
    if (!c) return MC_EINVAL;
    int solver, dtype, cus;
    mc_params prm;
    void* stream;
    mc__ctx_info(c, &solver, &dtype, &prm, &cus, &stream);
    if (!model_ok(solver) || dtype != MC_F32) return MC_EINVAL;
    if (s && s->model != solver) return MC_EINVAL;
    SurCtx* scp;
    {
        std::lock_guard<std::mutex> lk(g_ctx_mu);
        scp = &g_ctx[c];
    }
    SurCtx& sc = *scp;
    sc.net = s;
    if (!sc.red) {
        if (hip_check(hipMalloc((void**)&sc.red, 4 * sizeof(unsigned int))) != MC_OK) return MC_ENOMEM;
        if (hip_check(hipMalloc((void**)&sc.counts, 2 * sizeof(unsigned long long))) != MC_OK) return MC_ENOMEM;
        if (hip_check(hipMemset(sc.red, 0, 4 * sizeof(unsigned int))) != MC_OK) return MC_EHIP;
        if (hip_check(hipMemset(sc.counts, 0, 2 * sizeof(unsigned long long))) != MC_OK) return MC_EHIP;
    }
    return MC_OK;
}

int mc_sur_edge_stats(mc_ctx* c, int64_t* edges, int64_t* fallback)
{
    if (!c || !edges || !fallback) return MC_EINVAL;
    SurCtx* sc = find_ctx(c);
    *edges = 0;
    *fallback = 0;
    if (!sc || !sc->counts) return MC_OK;
    int solver, dtype, cus;
    mc_params prm;
    void* stream;
    mc__ctx_info(c, &solver, &dtype, &prm, &cus, &stream);
    unsigned long long h[2] = {0, 0};
    if (hip_check(hipStreamSynchronize((hipStream_t)stream)) != MC_OK) return MC_EHIP;
    if (hip_check(hipMemcpy(h, sc->counts, sizeof(h), hipMemcpyDeviceToHost)) != MC_OK) return MC_EHIP;
    if (hip_check(hipMemset(sc->counts, 0, sizeof(h))) != MC_OK) return MC_EHIP;
    *edges = (int64_t)h[0];
    *fallback = (int64_t)h[1];
    return MC_OK;
}

void mc__sur_release_ctx(const mc_ctx* c)
{
    std::lock_guard<std::mutex> lk(g_ctx_mu);
    auto it = g_ctx.find(c);
    if (it == g_ctx.end()) return;
    (void)hipFree(it->second.qs);
    (void)hipFree(it->second.rec);
    (void)hipFree(it->second.red);
    (void)hipFree(it->second.counts);
    g_ctx.erase(it);
}

// mc_rp2 on a surrogate context
int mc__sur_rp2(mc_ctx* c, int ixy, int64_t n, const void* ql, const void* qr, void* waves, void* speeds,
                void* amdq, void* apdq)
{
    SurCtx* sc = find_ctx(c);
    if (!sc || !sc->net) return MC_EINVAL;
    int solver, dtype, cus;
    mc_params prm;
    void* stream;
    mc__ctx_info(c, &solver, &dtype, &prm, &cus, &stream);
    int nx, ny;
    double dx, dy;
    unsigned int* status;
    mc__ctx_grid(c, &nx, &ny, &dx, &dy, &status);
    hipStream_t st = (hipStream_t)stream;
    if (solver == MC_EULER_SURROGATE)
        return sur_rp2_t<EulerModel>(*sc, prm, cus, st, status, ixy, n, ql, qr, waves, speeds, amdq, apdq);
    return sur_rp2_t<SwModel>(*sc, prm, cus, st, status, ixy, n, ql, qr, waves, speeds, amdq, apdq);
}

// one split step with the surrogate edge solve: edges x -> update x (into
// the intermediate state) -> edges y -> update y
int mc__sur_step(mc_ctx* c, mc_state* stt, double dt, int limiter, int bc, mc_cfl* cfl_out)
{
    SurCtx* sc = find_ctx(c);
    if (!sc || !sc->net) return MC_EINVAL;
    int solver, dtype, cus;
    mc_params prm;
    void* stream;
    mc__ctx_info(c, &solver, &dtype, &prm, &cus, &stream);
    int nx, ny;
    double dx, dy;
    unsigned int* status;
    mc__ctx_grid(c, &nx, &ny, &dx, &dy, &status);
    hipStream_t st = (hipStream_t)stream;
    if (solver == MC_EULER_SURROGATE)
        return sur_step_t<EulerModel>(*sc, prm, cus, st, nx, ny, dx, dy, status, stt, dt, limiter, bc,
                                      cfl_out);
    return sur_step_t<SwModel>(*sc, prm, cus, st, nx, ny, dx, dy, status, stt, dt, limiter, bc, cfl_out);
}

}  // extern "C"
