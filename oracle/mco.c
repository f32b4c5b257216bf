/*
 * mco.c -- plain FP64 CPU oracle of the 2D wave-propagation step.
 *
 * TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU-baseline timing).  It
 * shares no code with the HIP library.  Built with -O2 -ffp-contract=off so
 * that every expression is evaluated as written, with correctly rounded
 * division and square root.
 *
 * The paper (section 1.1) describes the method in words: cells hold averages,
 * a Riemann problem is solved at every cell edge, and the method is the
 * wave-propagation algorithm of the package it parallelises.  It states no
 * formula, so each routine below follows the standard statement of that
 * method, cited per routine (LeVeque, "Finite Volume Methods for Hyperbolic
 * Problems", 2002, abbreviated FVMHP).  Loops follow the paper's structure:
 * pointwise Riemann solves over every edge into ordinary work arrays
 * (section 2), then the limiter (Table 1), then the update.
 */
#include "mco.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXEQ 4
#define MAXW 4

int mco_dims(int solver, int* meqn, int* mwaves, int* maux)
{
    int m = 0, w = 0, a = 0;
    switch (solver) {
    case MCO_ADVECTION:    m = 1; w = 1; a = 0; break;
    case MCO_ACOUSTICS:    m = 3; w = 2; a = 0; break;
    case MCO_ACOUSTICS_VC: m = 3; w = 2; a = 2; break;
    case MCO_SW_ROE:       m = 3; w = 3; a = 0; break;
    case MCO_EULER_ROE:    m = 4; w = 4; a = 0; break;
    case MCO_SW_HLLE:      m = 3; w = 3; a = 0; break;
    default: return -1;
    }
    if (meqn) *meqn = m;
    if (mwaves) *mwaves = w;
    if (maux) *maux = a;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Riemann solvers.  Each writes mwaves waves, speeds and fluctuations.
 * The y-normal solve uses the same formulas with the roles of the two
 * velocity (momentum) components exchanged: mu is the normal component,
 * mv the transverse one. */

static void zero_out(int meqn, int mwaves, double* wave, double* s, double* amdq, double* apdq)
{
    for (int p = 0; p < mwaves; ++p) {
        s[p] = 0.0;
        for (int m = 0; m < meqn; ++m) wave[p * meqn + m] = 0.0;
    }
    for (int m = 0; m < meqn; ++m) { amdq[m] = 0.0; apdq[m] = 0.0; }
}

/* amdq = sum_p min(s_p,0) W_p ; apdq = sum_p max(s_p,0) W_p */
static void split_fluct(int meqn, int mwaves, const double* wave, const double* s,
                        double* amdq, double* apdq)
{
    for (int m = 0; m < meqn; ++m) { amdq[m] = 0.0; apdq[m] = 0.0; }
    for (int p = 0; p < mwaves; ++p) {
        double sm = s[p] < 0.0 ? s[p] : 0.0;
        double sp = s[p] > 0.0 ? s[p] : 0.0;
        for (int m = 0; m < meqn; ++m) {
            amdq[m] += sm * wave[p * meqn + m];
            apdq[m] += sp * wave[p * meqn + m];
        }
    }
}

/* Scalar advection q_t + u q_x + v q_y = 0 (FVMHP ch. 4, upwind waves):
 * one wave W = qR - qL moving at the normal velocity. */
static int rp_advection(const mco_params* P, int ixy, const double* ql, const double* qr,
                        double* wave, double* s, double* amdq, double* apdq)
{
    double a = (ixy == 1) ? P->u : P->v;
    wave[0] = qr[0] - ql[0];
    s[0] = a;
    split_fluct(1, 1, wave, s, amdq, apdq);
    return 0;
}

/* Constant-coefficient linear acoustics, q = (p, u, v) (FVMHP ch. 3 and
 * ch. 18): eigenvalues -c, 0, +c with c = sqrt(K/rho), impedance Z = rho c,
 * eigenvectors (-Z, 1, 0) and (Z, 1, 0) in (p, normal velocity, transverse
 * velocity) order.  The zero-speed shear wave carries no fluctuation and is
 * omitted, so mwaves = 2. */
static int rp_acoustics(const mco_params* P, int ixy, const double* ql, const double* qr,
                        double* wave, double* s, double* amdq, double* apdq)
{
    int mu = (ixy == 1) ? 1 : 2, mv = (ixy == 1) ? 2 : 1;
    double c = sqrt(P->K / P->rho);
    double Z = P->rho * c;
    double dp = qr[0] - ql[0];
    double du = qr[mu] - ql[mu];
    double a1 = (-dp + Z * du) / (2.0 * Z);
    double a2 = (dp + Z * du) / (2.0 * Z);
    wave[0 * 3 + 0] = -a1 * Z; wave[0 * 3 + mu] = a1; wave[0 * 3 + mv] = 0.0;
    wave[1 * 3 + 0] = a2 * Z;  wave[1 * 3 + mu] = a2; wave[1 * 3 + mv] = 0.0;
    s[0] = -c;
    s[1] = c;
    split_fluct(3, 2, wave, s, amdq, apdq);
    return 0;
}

/* Variable-coefficient acoustics, aux = (rho, c) per cell (FVMHP ch. 9):
 * W1 = a1 (-Z_L, 1, 0) at speed -c_L, W2 = a2 (Z_R, 1, 0) at speed +c_R with
 * a1 = (-dp + Z_R du)/(Z_L + Z_R), a2 = (dp + Z_L du)/(Z_L + Z_R). */
static int rp_acoustics_vc(int ixy, const double* ql, const double* qr,
                           const double* auxl, const double* auxr,
                           double* wave, double* s, double* amdq, double* apdq)
{
    int mu = (ixy == 1) ? 1 : 2, mv = (ixy == 1) ? 2 : 1;
    double cl = auxl[1], cr = auxr[1];
    double zl = auxl[0] * cl, zr = auxr[0] * cr;
    double dp = qr[0] - ql[0];
    double du = qr[mu] - ql[mu];
    double a1 = (-dp + zr * du) / (zl + zr);
    double a2 = (dp + zl * du) / (zl + zr);
    wave[0 * 3 + 0] = -a1 * zl; wave[0 * 3 + mu] = a1; wave[0 * 3 + mv] = 0.0;
    wave[1 * 3 + 0] = a2 * zr;  wave[1 * 3 + mu] = a2; wave[1 * 3 + mv] = 0.0;
    s[0] = -cl;
    s[1] = cr;
    split_fluct(3, 2, wave, s, amdq, apdq);
    return 0;
}

/* shallow-water normal flux, components (h, hu_n, hu_t) written in the
 * physical slots (0, mu, mv) */
static void sw_flux(double g, int mu, int mv, const double* q, double* f)
{
    double h = q[0], un = q[mu] / q[0], ut = q[mv] / q[0];
    f[0] = q[mu];
    f[mu] = q[mu] * un + 0.5 * g * h * h;
    f[mv] = q[mu] * ut;
}

/* Shallow water, Roe linearisation with the Harten-Hyman entropy fix
 * (FVMHP ch. 15: Roe averages h_bar = (hL+hR)/2, u_hat, v_hat weighted by
 * sqrt(h), c_hat = sqrt(g h_bar); eigenvectors (1, u-c, v), (0, 0, 1),
 * (1, u+c, v); the transonic split of a rarefaction family follows Harten
 * and Hyman (1983) as presented in FVMHP ch. 15). */
static int rp_sw_roe(const mco_params* P, int ixy, const double* ql, const double* qr,
                     double* wave, double* s, double* amdq, double* apdq)
{
    const double g = P->g;
    int mu = (ixy == 1) ? 1 : 2, mv = (ixy == 1) ? 2 : 1;
    double hl = ql[0], hr = qr[0];
    if (!(hl > 0.0) || !(hr > 0.0)) {
        zero_out(3, 3, wave, s, amdq, apdq);
        return MCO_ST_NONPHYS;
    }
    double ul = ql[mu] / hl, vl = ql[mv] / hl;
    double ur = qr[mu] / hr, vr = qr[mv] / hr;
    double sql = sqrt(hl), sqr = sqrt(hr);
    double hbar = 0.5 * (hl + hr);
    double uhat = (sql * ul + sqr * ur) / (sql + sqr);
    double vhat = (sql * vl + sqr * vr) / (sql + sqr);
    double chat = sqrt(g * hbar);

    double d0 = hr - hl;
    double d1 = qr[mu] - ql[mu];
    double d2 = qr[mv] - ql[mv];

    double a1 = ((uhat + chat) * d0 - d1) / (2.0 * chat);
    double a2 = d2 - vhat * d0;
    double a3 = (d1 - (uhat - chat) * d0) / (2.0 * chat);

    double* W1 = wave + 0;
    double* W2 = wave + 3;
    double* W3 = wave + 6;
    W1[0] = a1; W1[mu] = a1 * (uhat - chat); W1[mv] = a1 * vhat;
    W2[0] = 0.0; W2[mu] = 0.0; W2[mv] = a2;
    W3[0] = a3; W3[mu] = a3 * (uhat + chat); W3[mv] = a3 * vhat;
    s[0] = uhat - chat;
    s[1] = uhat;
    s[2] = uhat + chat;

    int st = 0;
    for (int m = 0; m < 3; ++m) amdq[m] = 0.0;

    /* family 1: left state and the state between waves 1 and 2 */
    {
        double lam_l = ul - sqrt(g * hl);
        double q1[3];
        for (int m = 0; m < 3; ++m) q1[m] = ql[m] + W1[m];
        int transonic = 0;
        double lam_r = 0.0;
        if (q1[0] > 0.0) {
            lam_r = q1[mu] / q1[0] - sqrt(g * q1[0]);
            transonic = (lam_l < 0.0) && (0.0 < lam_r);
        } else {
            st |= MCO_ST_NONPHYS;
        }
        if (transonic) {
            double f = lam_l * (lam_r - s[0]) / (lam_r - lam_l);
            for (int m = 0; m < 3; ++m) amdq[m] += f * W1[m];
        } else {
            double sm = s[0] < 0.0 ? s[0] : 0.0;
            for (int m = 0; m < 3; ++m) amdq[m] += sm * W1[m];
        }
    }
    /* family 2: linearly degenerate shear wave */
    {
        double sm = s[1] < 0.0 ? s[1] : 0.0;
        for (int m = 0; m < 3; ++m) amdq[m] += sm * W2[m];
    }
    /* family 3: the state between waves 2 and 3, and the right state */
    {
        double q2[3];
        for (int m = 0; m < 3; ++m) q2[m] = qr[m] - W3[m];
        double lam_r = ur + sqrt(g * hr);
        int transonic = 0;
        double lam_l = 0.0;
        if (q2[0] > 0.0) {
            lam_l = q2[mu] / q2[0] + sqrt(g * q2[0]);
            transonic = (lam_l < 0.0) && (0.0 < lam_r);
        } else {
            st |= MCO_ST_NONPHYS;
        }
        if (transonic) {
            double f = lam_l * (lam_r - s[2]) / (lam_r - lam_l);
            for (int m = 0; m < 3; ++m) amdq[m] += f * W3[m];
        } else {
            double sm = s[2] < 0.0 ? s[2] : 0.0;
            for (int m = 0; m < 3; ++m) amdq[m] += sm * W3[m];
        }
    }
    /* apdq = sum_p s_p W_p - amdq keeps amdq + apdq equal to the Roe total */
    for (int m = 0; m < 3; ++m) {
        double tot = s[0] * W1[m] + s[1] * W2[m] + s[2] * W3[m];
        apdq[m] = tot - amdq[m];
    }
    return st;
}

/* Shallow water HLLE (Einfeldt 1988): s_L = min(uL - cL, u_hat - c_hat),
 * s_R = max(uR + cR, u_hat + c_hat), middle state
 * q* = (s_R qR - s_L qL - (f(qR) - f(qL))) / (s_R - s_L); waves q* - qL
 * (slot 0, speed s_L) and qR - q* (slot 2, speed s_R); slot 1 is empty. */
static int rp_sw_hlle(const mco_params* P, int ixy, const double* ql, const double* qr,
                      double* wave, double* s, double* amdq, double* apdq)
{
    const double g = P->g;
    int mu = (ixy == 1) ? 1 : 2, mv = (ixy == 1) ? 2 : 1;
    double hl = ql[0], hr = qr[0];
    if (!(hl > 0.0) || !(hr > 0.0)) {
        zero_out(3, 3, wave, s, amdq, apdq);
        return MCO_ST_NONPHYS;
    }
    double ul = ql[mu] / hl, ur = qr[mu] / hr;
    double sql = sqrt(hl), sqr = sqrt(hr);
    double uhat = (sql * ul + sqr * ur) / (sql + sqr);
    double chat = sqrt(g * 0.5 * (hl + hr));
    double cl = sqrt(g * hl), cr = sqrt(g * hr);
    double sL = ul - cl, sR = ur + cr;
    if (uhat - chat < sL) sL = uhat - chat;
    if (uhat + chat > sR) sR = uhat + chat;
    double fl[3], fr[3], qs[3];
    sw_flux(g, mu, mv, ql, fl);
    sw_flux(g, mu, mv, qr, fr);
    for (int m = 0; m < 3; ++m)
        qs[m] = (sR * qr[m] - sL * ql[m] - (fr[m] - fl[m])) / (sR - sL);
    for (int m = 0; m < 3; ++m) {
        wave[0 * 3 + m] = qs[m] - ql[m];
        wave[1 * 3 + m] = 0.0;
        wave[2 * 3 + m] = qr[m] - qs[m];
    }
    s[0] = sL;
    s[1] = 0.0;
    s[2] = sR;
    split_fluct(3, 3, wave, s, amdq, apdq);
    (void)mv;
    return 0;
}

/* Euler pressure and flux, components (rho, m_n, m_t, E) in slots
 * (0, mu, mv, 3); p = (gamma-1)(E - (m_n^2 + m_t^2)/(2 rho)). */
static double eu_pressure(double gm, const double* q)
{
    return (gm - 1.0) * (q[3] - 0.5 * (q[1] * q[1] + q[2] * q[2]) / q[0]);
}

static void eu_flux(double gm, int mu, int mv, const double* q, double* f)
{
    double p = eu_pressure(gm, q);
    double un = q[mu] / q[0];
    f[0] = q[mu];
    f[mu] = q[mu] * un + p;
    f[mv] = q[mv] * un;
    f[3] = (q[3] + p) * un;
}

/* Euler HLLE with the same wave layout as the Roe solver: slot 0 = q* - qL
 * at s_L, slot 3 = qR - q* at s_R, slots 1 and 2 empty.  With use_roe the
 * speed bounds include the Roe speeds u_hat -+ c_hat (Einfeldt); without
 * (Roe averages unusable) they come from the two cell speeds only. */
static void eu_hlle(double gm, int mu, int mv, const double* ql, const double* qr,
                    int use_roe, double uhat, double chat,
                    double* wave, double* s, double* amdq, double* apdq)
{
    double ul = ql[mu] / ql[0], ur = qr[mu] / qr[0];
    double cl = sqrt(gm * eu_pressure(gm, ql) / ql[0]);
    double cr = sqrt(gm * eu_pressure(gm, qr) / qr[0]);
    double sL, sR;
    if (use_roe) {
        sL = ul - cl; if (uhat - chat < sL) sL = uhat - chat;
        sR = ur + cr; if (uhat + chat > sR) sR = uhat + chat;
    } else {
        sL = ul - cl; if (ur - cr < sL) sL = ur - cr;
        sR = ur + cr; if (ul + cl > sR) sR = ul + cl;
    }
    double fl[4], fr[4], qs[4];
    eu_flux(gm, mu, mv, ql, fl);
    eu_flux(gm, mu, mv, qr, fr);
    for (int m = 0; m < 4; ++m)
        qs[m] = (sR * qr[m] - sL * ql[m] - (fr[m] - fl[m])) / (sR - sL);
    for (int m = 0; m < 4; ++m) {
        wave[0 * 4 + m] = qs[m] - ql[m];
        wave[1 * 4 + m] = 0.0;
        wave[2 * 4 + m] = 0.0;
        wave[3 * 4 + m] = qr[m] - qs[m];
    }
    s[0] = sL; s[1] = 0.0; s[2] = 0.0; s[3] = sR;
    split_fluct(4, 4, wave, s, amdq, apdq);
}

/* Euler, Roe linearisation (Toro 2009 ch. 11; FVMHP ch. 14-15), four waves:
 * acoustic (u-c), entropy (u), shear (u), acoustic (u+c).  Harten-Hyman fix
 * on families 1 and 4 with lambda = u -+ sqrt(gamma p / rho).  HLLE
 * fallback when c_hat^2 <= 0 or a Roe intermediate state has rho <= 0 or
 * p <= 0. */
static int rp_euler_roe(const mco_params* P, int ixy, const double* ql, const double* qr,
                        double* wave, double* s, double* amdq, double* apdq)
{
    const double gm = P->gamma;
    int mu = (ixy == 1) ? 1 : 2, mv = (ixy == 1) ? 2 : 1;
    double rl = ql[0], rr = qr[0];
    if (!(rl > 0.0) || !(rr > 0.0)) {
        zero_out(4, 4, wave, s, amdq, apdq);
        return MCO_ST_NONPHYS;
    }
    double pl = eu_pressure(gm, ql), pr = eu_pressure(gm, qr);
    if (!(pl > 0.0) || !(pr > 0.0)) {
        zero_out(4, 4, wave, s, amdq, apdq);
        return MCO_ST_NONPHYS;
    }
    double ul = ql[mu] / rl, vl = ql[mv] / rl, Hl = (ql[3] + pl) / rl;
    double ur = qr[mu] / rr, vr = qr[mv] / rr, Hr = (qr[3] + pr) / rr;
    double sl = sqrt(rl), sr = sqrt(rr);
    double uhat = (sl * ul + sr * ur) / (sl + sr);
    double vhat = (sl * vl + sr * vr) / (sl + sr);
    double Hhat = (sl * Hl + sr * Hr) / (sl + sr);
    double q2hat = uhat * uhat + vhat * vhat;
    double c2hat = (gm - 1.0) * (Hhat - 0.5 * q2hat);
    if (!(c2hat > 0.0)) {
        eu_hlle(gm, mu, mv, ql, qr, 0, 0.0, 0.0, wave, s, amdq, apdq);
        return MCO_ST_FALLBACK;
    }
    double chat = sqrt(c2hat);

    double d0 = qr[0] - ql[0];
    double d1 = qr[mu] - ql[mu];
    double d2 = qr[mv] - ql[mv];
    double d3 = qr[3] - ql[3];

    double a3 = d2 - vhat * d0;
    double a2 = (gm - 1.0) / c2hat * ((Hhat - q2hat) * d0 + uhat * d1 + vhat * d2 - d3);
    double a1 = ((uhat + chat) * d0 - d1 - chat * a2) / (2.0 * chat);
    double a4 = d0 - a1 - a2;

    double* W1 = wave + 0;
    double* W2 = wave + 4;
    double* W3 = wave + 8;
    double* W4 = wave + 12;
    W1[0] = a1; W1[mu] = a1 * (uhat - chat); W1[mv] = a1 * vhat; W1[3] = a1 * (Hhat - uhat * chat);
    W2[0] = a2; W2[mu] = a2 * uhat;          W2[mv] = a2 * vhat; W2[3] = a2 * (0.5 * q2hat);
    W3[0] = 0.0; W3[mu] = 0.0;               W3[mv] = a3;        W3[3] = a3 * vhat;
    W4[0] = a4; W4[mu] = a4 * (uhat + chat); W4[mv] = a4 * vhat; W4[3] = a4 * (Hhat + uhat * chat);
    s[0] = uhat - chat;
    s[1] = uhat;
    s[2] = uhat;
    s[3] = uhat + chat;

    /* Roe intermediate states next to the acoustic waves */
    double q1[4], q3[4];
    for (int m = 0; m < 4; ++m) { q1[m] = ql[m] + W1[m]; q3[m] = qr[m] - W4[m]; }
    double p1 = (q1[0] > 0.0) ? eu_pressure(gm, q1) : -1.0;
    double p3 = (q3[0] > 0.0) ? eu_pressure(gm, q3) : -1.0;
    if (!(q1[0] > 0.0) || !(q3[0] > 0.0) || !(p1 > 0.0) || !(p3 > 0.0)) {
        eu_hlle(gm, mu, mv, ql, qr, 1, uhat, chat, wave, s, amdq, apdq);
        return MCO_ST_FALLBACK;
    }

    for (int m = 0; m < 4; ++m) amdq[m] = 0.0;
    /* family 1 */
    {
        double lam_l = ul - sqrt(gm * pl / rl);
        double lam_r = q1[mu] / q1[0] - sqrt(gm * p1 / q1[0]);
        if ((lam_l < 0.0) && (0.0 < lam_r)) {
            double f = lam_l * (lam_r - s[0]) / (lam_r - lam_l);
            for (int m = 0; m < 4; ++m) amdq[m] += f * W1[m];
        } else {
            double sm = s[0] < 0.0 ? s[0] : 0.0;
            for (int m = 0; m < 4; ++m) amdq[m] += sm * W1[m];
        }
    }
    /* families 2 and 3: linearly degenerate */
    {
        double sm = s[1] < 0.0 ? s[1] : 0.0;
        for (int m = 0; m < 4; ++m) amdq[m] += sm * W2[m];
        sm = s[2] < 0.0 ? s[2] : 0.0;
        for (int m = 0; m < 4; ++m) amdq[m] += sm * W3[m];
    }
    /* family 4 */
    {
        double lam_l = q3[mu] / q3[0] + sqrt(gm * p3 / q3[0]);
        double lam_r = ur + sqrt(gm * pr / rr);
        if ((lam_l < 0.0) && (0.0 < lam_r)) {
            double f = lam_l * (lam_r - s[3]) / (lam_r - lam_l);
            for (int m = 0; m < 4; ++m) amdq[m] += f * W4[m];
        } else {
            double sm = s[3] < 0.0 ? s[3] : 0.0;
            for (int m = 0; m < 4; ++m) amdq[m] += sm * W4[m];
        }
    }
    for (int m = 0; m < 4; ++m) {
        double tot = s[0] * W1[m] + s[1] * W2[m] + s[2] * W3[m] + s[3] * W4[m];
        apdq[m] = tot - amdq[m];
    }
    return 0;
}

int mco_rp1(int solver, const mco_params* P, int ixy,
            const double* ql, const double* qr,
            const double* auxl, const double* auxr,
            double* wave, double* s, double* amdq, double* apdq)
{
    switch (solver) {
    case MCO_ADVECTION:    return rp_advection(P, ixy, ql, qr, wave, s, amdq, apdq);
    case MCO_ACOUSTICS:    return rp_acoustics(P, ixy, ql, qr, wave, s, amdq, apdq);
    case MCO_ACOUSTICS_VC:
        if (!auxl || !auxr) return MCO_ST_BADARG;
        return rp_acoustics_vc(ixy, ql, qr, auxl, auxr, wave, s, amdq, apdq);
    case MCO_SW_ROE:       return rp_sw_roe(P, ixy, ql, qr, wave, s, amdq, apdq);
    case MCO_EULER_ROE:    return rp_euler_roe(P, ixy, ql, qr, wave, s, amdq, apdq);
    case MCO_SW_HLLE:      return rp_sw_hlle(P, ixy, ql, qr, wave, s, amdq, apdq);
    default: return MCO_ST_BADARG;
    }
}

int mco_rp2(int solver, const mco_params* P, int ixy, int64_t n,
            const double* ql, const double* qr, const double* aux,
            double* waves, double* speeds, double* amdq, double* apdq)
{
    int meqn, mwaves, maux;
    if (mco_dims(solver, &meqn, &mwaves, &maux) != 0) return MCO_ST_BADARG;
    if (maux > 0 && !aux) return MCO_ST_BADARG;
    int st = 0;
    for (int64_t e = 0; e < n; ++e) {
        double a[MAXEQ], b[MAXEQ], al[2], ar[2];
        double w[MAXW * MAXEQ], s[MAXW], am[MAXEQ], ap[MAXEQ];
        for (int m = 0; m < meqn; ++m) { a[m] = ql[m * n + e]; b[m] = qr[m * n + e]; }
        for (int k = 0; k < maux; ++k) { al[k] = aux[k * n + e]; ar[k] = aux[(maux + k) * n + e]; }
        st |= mco_rp1(solver, P, ixy, a, b, maux ? al : NULL, maux ? ar : NULL, w, s, am, ap);
        for (int p = 0; p < mwaves; ++p) {
            speeds[p * n + e] = s[p];
            for (int m = 0; m < meqn; ++m) waves[((int64_t)p * meqn + m) * n + e] = w[p * meqn + m];
        }
        for (int m = 0; m < meqn; ++m) { amdq[m * n + e] = am[m]; apdq[m * n + e] = ap[m]; }
    }
    return st;
}

/* ------------------------------------------------------------------ */
/* Wave limiters (FVMHP ch. 6): phi(theta) of the smoothness ratio. */
double mco_phi(int limiter, double theta)
{
    double r;
    switch (limiter) {
    case MCO_LIM_NONE:
        return 1.0;
    case MCO_LIM_MINMOD:
        r = theta < 1.0 ? theta : 1.0;
        return r > 0.0 ? r : 0.0;
    case MCO_LIM_SUPERBEE: {
        double a = 2.0 * theta < 1.0 ? 2.0 * theta : 1.0;
        double b = theta < 2.0 ? theta : 2.0;
        r = a > b ? a : b;
        return r > 0.0 ? r : 0.0;
    }
    case MCO_LIM_VANLEER:
        return (theta + fabs(theta)) / (1.0 + fabs(theta));
    case MCO_LIM_MC: {
        double c = 0.5 * (1.0 + theta);
        r = c;
        if (2.0 < r) r = 2.0;
        if (2.0 * theta < r) r = 2.0 * theta;
        return r > 0.0 ? r : 0.0;
    }
    default:
        return 0.0;
    }
}

/* ------------------------------------------------------------------ */
/* 1D high-resolution wave propagation along one grid line (FVMHP ch. 6):
 *   Q*_i = Q_i - nu (A+dQ_{i-1/2} + A-dQ_{i+1/2}) - nu (F~_{i+1/2} - F~_{i-1/2}),
 *   F~_{i-1/2} = 1/2 sum_p |s^p| (1 - nu |s^p|) phi(theta^p) W^p,
 *   theta^p_{i-1/2} = W^p_{I-1/2} . W^p_{i-1/2} / W^p_{i-1/2} . W^p_{i-1/2},
 *   I = i-1 if s^p > 0, i+1 otherwise, with unlimited neighbour waves.
 * qg holds n + 4 cells of the line including two ghost cells per side, with
 * component stride gs; edge k (0 <= k < n + 3) lies between ghosted cells k
 * and k + 1, so the edge between interior cells i-1 and i is k = i + 1.
 * Work arrays are the plain per-edge arrays of the method. */
typedef struct {
    double* wave;  /* [mwaves][meqn][n+3] */
    double* s;     /* [mwaves][n+3] */
    double* amdq;  /* [meqn][n+3] */
    double* apdq;  /* [meqn][n+3] */
    double* ftil;  /* [meqn][n+3] */
} work1d;

static int sweep1d(int solver, const mco_params* P, int ixy, int n,
                   const double* qg, int64_t gs, const double* auxg, int64_t as,
                   double nu, double d, int limiter,
                   double* qo, int64_t os, double* smax, work1d* W)
{
    int meqn, mwaves, maux;
    mco_dims(solver, &meqn, &mwaves, &maux);
    const int ne = n + 3;
    int st = 0;

    /* Riemann problem at every edge */
    for (int k = 0; k < ne; ++k) {
        double a[MAXEQ], b[MAXEQ], al[2], ar[2];
        double w[MAXW * MAXEQ], s[MAXW], am[MAXEQ], ap[MAXEQ];
        for (int m = 0; m < meqn; ++m) { a[m] = qg[m * gs + k]; b[m] = qg[m * gs + k + 1]; }
        for (int j = 0; j < maux; ++j) { al[j] = auxg[j * as + k]; ar[j] = auxg[j * as + k + 1]; }
        st |= mco_rp1(solver, P, ixy, a, b, maux ? al : NULL, maux ? ar : NULL, w, s, am, ap);
        for (int p = 0; p < mwaves; ++p) {
            W->s[p * ne + k] = s[p];
            for (int m = 0; m < meqn; ++m) W->wave[(p * meqn + m) * ne + k] = w[p * meqn + m];
        }
        for (int m = 0; m < meqn; ++m) { W->amdq[m * ne + k] = am[m]; W->apdq[m * ne + k] = ap[m]; }
    }

    /* CFL: counted edges are those bounding an interior cell, k = 1 .. n+1 */
    double sm = 0.0;
    for (int k = 1; k <= n + 1; ++k)
        for (int p = 0; p < mwaves; ++p) {
            double v = fabs(W->s[p * ne + k]) / d;
            if (v > sm) sm = v;
        }
    *smax = sm;

    /* limiter and correction flux on edges k = 1 .. n+1 */
    for (int m = 0; m < meqn; ++m)
        for (int k = 0; k < ne; ++k) W->ftil[m * ne + k] = 0.0;
    if (limiter != MCO_LIM_FIRST_ORDER) {
        for (int k = 1; k <= n + 1; ++k) {
            for (int p = 0; p < mwaves; ++p) {
                double sp = W->s[p * ne + k];
                double wn = 0.0, wd = 0.0;
                int kk = (sp > 0.0) ? k - 1 : k + 1;
                for (int m = 0; m < meqn; ++m) {
                    double wk = W->wave[(p * meqn + m) * ne + k];
                    wn += wk * wk;
                    wd += W->wave[(p * meqn + m) * ne + kk] * wk;
                }
                double phi;
                if (wn == 0.0) {
                    phi = 0.0;
                } else {
                    phi = mco_phi(limiter, wd / wn);
                }
                double c = 0.5 * fabs(sp) * (1.0 - nu * fabs(sp));
                for (int m = 0; m < meqn; ++m)
                    W->ftil[m * ne + k] += c * (phi * W->wave[(p * meqn + m) * ne + k]);
            }
        }
    }

    /* conservative update of interior cells i = 0 .. n-1 (ghosted i + 2) */
    for (int m = 0; m < meqn; ++m)
        for (int i = 0; i < n; ++i) {
            int kl = i + 1, kr = i + 2;
            double qi = qg[m * gs + i + 2];
            double v = qi - nu * (W->apdq[m * ne + kl] + W->amdq[m * ne + kr])
                          - nu * (W->ftil[m * ne + kr] - W->ftil[m * ne + kl]);
            qo[m * os + i] = v;
        }
    return st;
}

static int work_alloc(work1d* W, int meqn, int mwaves, int n)
{
    int64_t ne = n + 3;
    W->wave = (double*)malloc(sizeof(double) * mwaves * meqn * ne);
    W->s = (double*)malloc(sizeof(double) * mwaves * ne);
    W->amdq = (double*)malloc(sizeof(double) * meqn * ne);
    W->apdq = (double*)malloc(sizeof(double) * meqn * ne);
    W->ftil = (double*)malloc(sizeof(double) * meqn * ne);
    return (W->wave && W->s && W->amdq && W->apdq && W->ftil) ? 0 : -1;
}

static void work_free(work1d* W)
{
    free(W->wave); free(W->s); free(W->amdq); free(W->apdq); free(W->ftil);
}

/* ghost-cell index map (two ghost cells per side): periodic wraps,
 * zero-order extrapolation copies the nearest interior cell */
static int bc_index(int i, int n, int bc)
{
    if (bc == MCO_BC_PERIODIC) {
        int r = i % n;
        return r < 0 ? r + n : r;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

/* Fill a ghosted copy [nf][ny+4][nx+4] of a field array [nf][ny][nx]. */
static void fill_ghosts(int nf, int nx, int ny, const double* q, int bc, double* g)
{
    int gx = nx + 4, gy = ny + 4;
    for (int m = 0; m < nf; ++m)
        for (int j = -2; j < ny + 2; ++j)
            for (int i = -2; i < nx + 2; ++i) {
                int ii = bc_index(i, nx, bc), jj = bc_index(j, ny, bc);
                g[((int64_t)m * gy + (j + 2)) * gx + (i + 2)] = q[((int64_t)m * ny + jj) * nx + ii];
            }
}

static int check_args(int solver, int nx, int ny, double dx, double dy, int limiter, int bc)
{
    if (mco_dims(solver, NULL, NULL, NULL) != 0) return -1;
    if (nx < 1 || ny < 1 || !(dx > 0.0) || !(dy > 0.0)) return -1;
    if (limiter < MCO_LIM_NONE || limiter > MCO_LIM_FIRST_ORDER) return -1;
    if (bc != MCO_BC_PERIODIC && bc != MCO_BC_EXTRAP) return -1;
    return 0;
}

/* One x-sweep (ixy = 1) or y-sweep (ixy = 2) of the whole grid, from the
 * ghosted array g into out [meqn][ny][nx]. */
static int sweep2d(int solver, const mco_params* P, int ixy, int nx, int ny,
                   const double* g, const double* ga, double nu, double d, int limiter,
                   double* out, double* smax_out, int nthreads)
{
    int meqn, mwaves, maux;
    mco_dims(solver, &meqn, &mwaves, &maux);
    const int gx = nx + 4, gy = ny + 4;
    const int nlines = (ixy == 1) ? ny : nx;
    const int n = (ixy == 1) ? nx : ny;
    int st = 0, fail = 0;
    double smax = 0.0;
    if (nthreads < 1) nthreads = 1;
#ifdef _OPENMP
#pragma omp parallel num_threads(nthreads) reduction(|:st) reduction(max:smax) reduction(|:fail)
#endif
    {
        work1d W;
        double* line = (double*)malloc(sizeof(double) * meqn * (n + 4));
        double* aline = (double*)malloc(sizeof(double) * (maux ? maux : 1) * (n + 4));
        double* oline = (double*)malloc(sizeof(double) * meqn * n);
        if (work_alloc(&W, meqn, mwaves, n) != 0 || !line || !aline || !oline) {
            fail = 1;
        } else {
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
            for (int L = 0; L < nlines; ++L) {
                /* gather the line with its two ghost cells per side */
                for (int m = 0; m < meqn; ++m)
                    for (int k = 0; k < n + 4; ++k) {
                        int64_t idx = (ixy == 1)
                            ? ((int64_t)m * gy + (L + 2)) * gx + k
                            : ((int64_t)m * gy + k) * gx + (L + 2);
                        line[m * (n + 4) + k] = g[idx];
                    }
                for (int a = 0; a < maux; ++a)
                    for (int k = 0; k < n + 4; ++k) {
                        int64_t idx = (ixy == 1)
                            ? ((int64_t)a * gy + (L + 2)) * gx + k
                            : ((int64_t)a * gy + k) * gx + (L + 2);
                        aline[a * (n + 4) + k] = ga[idx];
                    }
                double sm = 0.0;
                st |= sweep1d(solver, P, ixy, n, line, n + 4, aline, n + 4, nu, d,
                              limiter, oline, n, &sm, &W);
                if (sm > smax) smax = sm;
                for (int m = 0; m < meqn; ++m)
                    for (int k = 0; k < n; ++k) {
                        int64_t idx = (ixy == 1)
                            ? ((int64_t)m * ny + L) * nx + k
                            : ((int64_t)m * ny + k) * nx + L;
                        out[idx] = oline[m * n + k];
                    }
            }
        }
        work_free(&W);
        free(line); free(aline); free(oline);
    }
    if (fail) return MCO_ST_BADARG;
    *smax_out = smax;
    return st;
}

int mco_step2d(int solver, const mco_params* P, int nx, int ny, double dx, double dy,
               const double* q, const double* aux, double dt, int limiter, int bc,
               double* qout, double* smax_out, int nthreads)
{
    if (check_args(solver, nx, ny, dx, dy, limiter, bc) != 0 || !q || !qout || !P)
        return MCO_ST_BADARG;
    int meqn, mwaves, maux;
    mco_dims(solver, &meqn, &mwaves, &maux);
    if (maux > 0 && !aux) return MCO_ST_BADARG;
    int64_t gsz = (int64_t)(nx + 4) * (ny + 4);
    double* g = (double*)malloc(sizeof(double) * meqn * gsz);
    double* ga = (double*)malloc(sizeof(double) * (maux ? maux : 1) * gsz);
    double* qs = (double*)malloc(sizeof(double) * meqn * (int64_t)nx * ny);
    if (!g || !ga || !qs) { free(g); free(ga); free(qs); return MCO_ST_BADARG; }
    if (maux > 0) fill_ghosts(maux, nx, ny, aux, bc, ga);

    int st = 0;
    double sx = 0.0, sy = 0.0;
    /* x-sweep: ghost cells of q^n, full dt */
    fill_ghosts(meqn, nx, ny, q, bc, g);
    st |= sweep2d(solver, P, 1, nx, ny, g, ga, dt / dx, dx, limiter, qs, &sx, nthreads);
    /* y-sweep on the x-swept state, boundary conditions re-applied */
    fill_ghosts(meqn, nx, ny, qs, bc, g);
    st |= sweep2d(solver, P, 2, nx, ny, g, ga, dt / dy, dy, limiter, qout, &sy, nthreads);

    if (smax_out) *smax_out = sx > sy ? sx : sy;
    free(g); free(ga); free(qs);
    return st;
}

int mco_max_speed(int solver, const mco_params* P, int nx, int ny, double dx, double dy,
                  const double* q, const double* aux, int bc, double* smax_out, int nthreads)
{
    if (check_args(solver, nx, ny, dx, dy, MCO_LIM_NONE, bc) != 0 || !q || !P || !smax_out)
        return MCO_ST_BADARG;
    int meqn, mwaves, maux;
    mco_dims(solver, &meqn, &mwaves, &maux);
    if (maux > 0 && !aux) return MCO_ST_BADARG;
    int64_t gsz = (int64_t)(nx + 4) * (ny + 4);
    double* g = (double*)malloc(sizeof(double) * meqn * gsz);
    double* ga = (double*)malloc(sizeof(double) * (maux ? maux : 1) * gsz);
    double* tmp = (double*)malloc(sizeof(double) * meqn * (int64_t)nx * ny);
    if (!g || !ga || !tmp) { free(g); free(ga); free(tmp); return MCO_ST_BADARG; }
    fill_ghosts(meqn, nx, ny, q, bc, g);
    if (maux > 0) fill_ghosts(maux, nx, ny, aux, bc, ga);
    /* speeds of both edge directions at the same state q: a zero-dt sweep
     * in each direction evaluates exactly the Riemann problems counted */
    double sx = 0.0, sy = 0.0;
    int st = 0;
    st |= sweep2d(solver, P, 1, nx, ny, g, ga, 0.0, dx, MCO_LIM_FIRST_ORDER, tmp, &sx, nthreads);
    st |= sweep2d(solver, P, 2, nx, ny, g, ga, 0.0, dy, MCO_LIM_FIRST_ORDER, tmp, &sy, nthreads);
    *smax_out = sx > sy ? sx : sy;
    free(g); free(ga); free(tmp);
    return st;
}

int mco_run2d(int solver, const mco_params* P, int nx, int ny, double dx, double dy,
              double* q, const double* aux, int limiter, int bc,
              double cfl_target, double cfl_max, int nsteps,
              double* dt_hist, double* t_out, int* nrej_out, int nthreads)
{
    if (check_args(solver, nx, ny, dx, dy, limiter, bc) != 0 || !q || !P || nsteps < 0)
        return MCO_ST_BADARG;
    int meqn;
    mco_dims(solver, &meqn, NULL, NULL);
    int64_t sz = (int64_t)meqn * nx * ny;
    double* qn = (double*)malloc(sizeof(double) * sz);
    if (!qn) return MCO_ST_BADARG;
    double smax = 0.0;
    int st = mco_max_speed(solver, P, nx, ny, dx, dy, q, aux, bc, &smax, nthreads);
    double dt = cfl_target / smax;
    double t = 0.0;
    int nrej = 0, n = 0, streak = 0;
    while (n < nsteps) {
        double sm = 0.0;
        st |= mco_step2d(solver, P, nx, ny, dx, dy, q, aux, dt, limiter, bc, qn, &sm, nthreads);
        double cfl = dt * sm;
        if (cfl > cfl_max) {
            ++nrej;
            dt = cfl_target / sm;
            if (++streak > 1000) { st |= MCO_ST_STALLED; break; }
            continue;
        }
        streak = 0;
        memcpy(q, qn, sizeof(double) * sz);
        t += dt;
        if (dt_hist) dt_hist[n] = dt;
        ++n;
        dt = cfl_target / sm;
    }
    free(qn);
    if (t_out) *t_out = t;
    if (nrej_out) *nrej_out = nrej;
    return st;
}
