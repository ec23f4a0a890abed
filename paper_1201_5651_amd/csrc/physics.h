// physics.h -- device-side physics of the photoionisation source-term step.
//
// Per-cell geometry of a vertex source, photon-conserving photoionisation and
// photoheating rates, hydrogen rate coefficients and cooling, and the
// micro-integrator of eq. (2) (neutral fraction x = 1 - y and internal energy
// E) of Mackey (A&A 2012).  Everything is templated on the arithmetic type R
// (double for PI_FP64, float for PI_FP32/PI_MIXED bulk work).
//
// Dimensionless geometry: distances are in cell units and the host folds the
// large dimensional constants into Q/dx^3 and sigma0*dx, so every quantity a
// kernel touches stays inside the float range (Q ~ 1e48 and r^2 ~ 1e40 do not).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// Host and device: the same code also builds into host-side unit harnesses.
#define PI_HD __host__ __device__

namespace pi {

constexpr double KB = 1.380649e-16;           // Boltzmann constant [erg/K]
constexpr double T_FLOOR = 10.0;              // temperature floor [K]
constexpr double THIN_CELL = 2e-2;            // table rates: quadrature below this absorbed fraction
constexpr double W_FLOOR = 0.6;               // Mellema weights: 1 / max(0.6, tau)
// (2/pi) * integral of dV/r^2 over a unit cube seen from one corner: the chord
// that lets the source-corner cell absorb its octant's Q/8 exactly in both the
// optically thin and the optically thick limit.
constexpr double CORNER_CHORD = 1.2213748039031678;
constexpr int NTAB = 64;
constexpr int MAX_SRC = 4;        // point sources of one grid
constexpr int NEWTON_MAXIT = 60;
constexpr int NEWTON_2D_MAXIT = 20;
constexpr int FALLBACK_MAXIT = 200;
constexpr double SUB_DX = 0.2;    // initial substeps: max x change at the initial rate
constexpr int SUB_MAX = 128;
constexpr int SUB_LEVELS = 6;     // substep halvings allowed
constexpr double REJ_DX = 0.3;    // reject a substep that moves x by more
constexpr double REJ_E = 3.0;     // ... or changes E by more than this factor
// A substep-control decision (initial substep count, rejection) whose deciding
// quantity lies within this relative distance of its threshold could go the
// other way under a change of precision; the mixed-precision path re-solves
// such cells in double.
constexpr double MIX_MARGIN = 1e-3;
// Ionisation-front cells of the mixed-precision path: a cell whose neutral
// fraction at the start of the micro-integration lies in [FRONT_X_LO,
// FRONT_X_HI] -- the transition layer between the ionised gas (x < 1e-3) and
// gas that is still mostly neutral (x > 1/2) -- is integrated in double only
// (the float pass skips it).  Gas ahead of the front that the hardest photons
// have only begun to ionise (1/2 < x < 1) is not part of the layer.
constexpr double FRONT_X_LO = 1e-3;
constexpr double FRONT_X_HI = 0.5;
template <typename R> PI_HD __forceinline__ bool front_cell(R x)
{
    return x >= R(FRONT_X_LO) && x <= R(FRONT_X_HI);
}

template <typename R> struct Tol;
template <> struct Tol<double> {
    static constexpr double half_ulp1 = 5.551115123125783e-17;   // half the spacing below 1
    static constexpr double rtol = 1e-13;   // Newton converged
    static constexpr double stall = 1e-11;  // correction stopped shrinking: rounding floor
    static constexpr double one_step = 0.0; // double always confirms convergence
};
template <> struct Tol<float> {
    static constexpr float half_ulp1 = 2.98023224e-8f;
    static constexpr float rtol = 4e-7f;
    static constexpr float stall = 1e-4f;
    // A first Newton step of relative size d from the stage's starting guess
    // leaves an error of order d^2 (quadratic convergence): when it is a plain
    // Newton step (no projection onto [0,1], no halving of E) and d is below
    // the square root of rtol, its result is accepted without one more
    // residual evaluation to confirm it.
    static constexpr float one_step = 3e-4f;
};

// Rate table as the kernels use it: values normalised by Q, and the log-Hermite
// form (the cubic Hermite interpolant of ln V/V_0 in ln tau between the
// log-spaced nodes, from the values and logarithmic slopes at the nodes) so
// that the interpolation is accurate in float too.  Each interval carries the
// cubic's coefficients in its local coordinate t in [0, 1),
// {a0, a1, a2, a3} for ln V/V_0 = a0 + a1 t + a2 t^2 + a3 t^3, and
// {b1, b2, b3} = {a1, 2 a2, 3 a3} / Delta for its derivative in ln tau.
template <typename R> struct DevTable {
    R p0, p1_0, h0, h1_0;    // P(0)/Q, -P'(0)/Q, H(0)/Q [erg], -H'(0)/Q [erg]
    R s1, inv_delta, delta;  // ln tau_1, 1/Delta, Delta (node spacing in ln tau)
    R tau1, tau_last;
    // interval j runs from node j + 1 to node j + 2 (node 0 is tau = 0):
    // {a0, a1, a2, a3, b1, b2, b3, 0}
    alignas(16) R cp[NTAB][8];
    alignas(16) R ch[NTAB][8];
};

// Per-grid constants, passed by value to every kernel.
template <typename R> struct Params {
    int nx, ny, nz;
    int sx, sy, sz;
    int64_t ncell;
    R QV;        // Q / dx^3 [photons s^-1 cm^-3]; plane-parallel source: flux / dx
    R sdx;       // sigma0 * dx               [cm^3] (times n_H x: optical depth per cell length)
    R eps;       // mono: heating per photoionisation [erg]
    R T_fixed, alpha_B;
    R K[4];
    int spectrum, thermal, recomb, collisional, cooling, weights, src_rule, n_sub;
    int plane;   // 1: plane-parallel source at x = -inf
    const DevTable<R>* tab;
};

// Float arithmetic uses the hardware transcendental instructions (a few ulp,
// far inside the 1e-4 float tolerance); double uses the correctly rounded
// library routines.  Every logarithm and square root taken here has a
// positive normal argument (T >= 10 K, tau >= 1e-4, squared distances >=
// 3/4 in cell units), so the bare instruction needs no denormal scaling.
#if defined(__HIP_DEVICE_COMPILE__)
#define PI_FEXP(v) __expf(v)
#define PI_FLOG(v) (__builtin_amdgcn_logf(v) * 0.693147181f)
#define PI_FPOW(a, b) __powf(a, b)
#define PI_FSQRT(v) __builtin_amdgcn_sqrtf(v)
#define PI_FPOW01(v) __builtin_amdgcn_exp2f(0.1f * __builtin_amdgcn_logf(v))
#else   // host-side unit harnesses
#define PI_FEXP(v) expf(v)
#define PI_FLOG(v) logf(v)
#define PI_FPOW(a, b) powf(a, b)
#define PI_FSQRT(v) sqrtf(v)
#define PI_FPOW01(v) powf(v, 0.1f)
#endif
template <typename R> PI_HD __forceinline__ R r_exp(R v);
template <> PI_HD __forceinline__ double r_exp<double>(double v) { return exp(v); }
template <> PI_HD __forceinline__ float r_exp<float>(float v) { return PI_FEXP(v); }
template <typename R> PI_HD __forceinline__ R r_expm1(R v);
template <> PI_HD __forceinline__ double r_expm1<double>(double v) { return expm1(v); }
template <> PI_HD __forceinline__ float r_expm1<float>(float v) { return expm1f(v); }
template <typename R> PI_HD __forceinline__ R r_log(R v);
template <> PI_HD __forceinline__ double r_log<double>(double v) { return log(v); }
template <> PI_HD __forceinline__ float r_log<float>(float v) { return PI_FLOG(v); }
template <typename R> PI_HD __forceinline__ R r_sqrt(R v);
template <> PI_HD __forceinline__ double r_sqrt<double>(double v) { return sqrt(v); }
template <> PI_HD __forceinline__ float r_sqrt<float>(float v) { return PI_FSQRT(v); }
template <typename R> PI_HD __forceinline__ R r_pow(R a, R b);
template <> PI_HD __forceinline__ double r_pow<double>(double a, double b) { return pow(a, b); }
template <> PI_HD __forceinline__ float r_pow<float>(float a, float b) { return PI_FPOW(a, b); }
// T^(1/10), from which the power laws of T are formed by products.
template <typename R> PI_HD __forceinline__ R r_pow01(R v);
template <> PI_HD __forceinline__ double r_pow01<double>(double v) { return exp(0.1 * log(v)); }
template <> PI_HD __forceinline__ float r_pow01<float>(float v) { return PI_FPOW01(v); }
// Reciprocal: correctly rounded in double, the hardware reciprocal (1 ulp) in
// float device code.
template <typename R> PI_HD __forceinline__ R r_rcp(R v);
template <> PI_HD __forceinline__ double r_rcp<double>(double v) { return 1.0 / v; }
#if defined(__HIP_DEVICE_COMPILE__)
template <> PI_HD __forceinline__ float r_rcp<float>(float v) { return __builtin_amdgcn_rcpf(v); }
#else
template <> PI_HD __forceinline__ float r_rcp<float>(float v) { return 1.0f / v; }
#endif
// Fused multiply-add with one rounding, wherever a value must come out the
// same from every code path that forms it.
template <typename R> PI_HD __forceinline__ R r_fma(R a, R b, R c);
template <> PI_HD __forceinline__ double r_fma<double>(double a, double b, double c)
{
    return fma(a, b, c);
}
template <> PI_HD __forceinline__ float r_fma<float>(float a, float b, float c)
{
    return fmaf(a, b, c);
}
template <typename R> PI_HD __forceinline__ R r_abs(R v) { return v < R(0) ? -v : v; }
template <typename R> PI_HD __forceinline__ R r_max(R a, R b) { return a > b ? a : b; }
template <typename R> PI_HD __forceinline__ R r_min(R a, R b) { return a < b ? a : b; }

// ------------------------------------------------------------------ geometry
// Cell (i,j,k) seen from the source vertex (Sect. 5): ad[d] = |centre - src|
// in cell units (half integers), dominant axis a (ties z > y > x), and the
// two factors of the photon-conserving rate: g = 1 / (4 pi r^2 ds) in cell
// units (the shell volume the entering photons spread over), ell = ds, the
// chord between successive planes of the dominant axis; the octant's corner
// cell instead takes g = 1/8 of the source over its own volume with the
// corner-cube mean chord.
template <typename R> struct CellGeom {
    R g, ell;
};

template <typename R>
PI_HD __forceinline__ CellGeom<R> cell_geom_at(const Params<R>& p, int sx, int sy, int sz, int i,
                                               int j, int k)
{
    if (p.plane) {
        // slab cell of its row: the flux (in QV) over one cell length
        CellGeom<R> c;
        c.g = R(1);
        c.ell = R(1);
        return c;
    }
    // exact half-integers: (2i + 1 - 2s) / 2
    const R ax = r_abs(R(2 * (i - sx) + 1)) * R(0.5);
    const R ay = r_abs(R(2 * (j - sy) + 1)) * R(0.5);
    const R az = r_abs(R(2 * (k - sz) + 1)) * R(0.5);
    const R rr = ax * ax + ay * ay + az * az;
    const R da = (az >= ax && az >= ay) ? az : (ay >= ax ? ay : ax);
    CellGeom<R> c;
    if (p.src_rule && da == R(0.5)) {
        c.g = R(0.125);
        c.ell = R(CORNER_CHORD);
    } else {
        const R ds = r_sqrt(rr) * r_rcp(da);
        c.g = r_rcp(R(4.0 * 3.14159265358979323846) * rr * ds);
        c.ell = ds;
    }
    return c;
}

// Geometry of cell (i,j,k) seen from source 0.
template <typename R>
PI_HD __forceinline__ CellGeom<R> cell_geom(const Params<R>& p, int i, int j, int k)
{
    return cell_geom_at(p, p.sx, p.sy, p.sz, i, j, k);
}

// -------------------------------------------------------------------- table
// Normalised table value and d/dtau at optical depth tau >= 0 for P (which=0)
// and H (which=1) together: first-order Taylor from tau = 0 below the first
// log node, cubic Hermite in (ln tau, ln V/V0) between nodes, zero beyond.
template <typename R>
PI_HD __forceinline__ void table_pair(const DevTable<R>* __restrict__ T, R tau, R& P, R& dP,
                                           R& H, R& dH)
{
    if (tau < T->tau1) {
        P = T->p0 - T->p1_0 * tau;
        dP = -T->p1_0;
        H = T->h0 - T->h1_0 * tau;
        dH = -T->h1_0;
        return;
    }
    if (tau >= T->tau_last) {
        P = dP = H = dH = R(0);
        return;
    }
    const R s = r_log(tau);
    const R f = (s - T->s1) * T->inv_delta;
    int j = (int)f;                     // f >= 0 here
    j = j < 0 ? 0 : (j > NTAB - 3 ? NTAB - 3 : j);
    const R t = f - R(j);
    const R itau = r_rcp(tau);
    {
        const R* c = T->cp[j];
        const R L = r_fma(r_fma(r_fma(c[3], t, c[2]), t, c[1]), t, c[0]);
        const R dL = r_fma(r_fma(c[6], t, c[5]), t, c[4]);   // d ln V / d ln tau
        P = T->p0 * r_exp(L);
        dP = P * dL * itau;
    }
    {
        const R* c = T->ch[j];
        const R L = r_fma(r_fma(r_fma(c[3], t, c[2]), t, c[1]), t, c[0]);
        const R dL = r_fma(r_fma(c[6], t, c[5]), t, c[4]);
        H = T->h0 * r_exp(L);
        dH = H * dL * itau;
    }
}

// d/dtau of the normalised P and H alone (the thin-cell quadrature needs no
// values): between nodes V'(tau) = V0 exp(L - ln tau) dL, which needs no
// reciprocal of tau.
template <typename R>
PI_HD __forceinline__ void table_dpair(const DevTable<R>* __restrict__ T, R tau, R& dP, R& dH)
{
    if (tau < T->tau1) {
        dP = -T->p1_0;
        dH = -T->h1_0;
        return;
    }
    if (tau >= T->tau_last) {
        dP = dH = R(0);
        return;
    }
    const R s = r_log(tau);
    const R f = (s - T->s1) * T->inv_delta;
    int j = (int)f;                     // f >= 0 here
    j = j < 0 ? 0 : (j > NTAB - 3 ? NTAB - 3 : j);
    const R t = f - R(j);
    {
        const R* c = T->cp[j];
        const R L = r_fma(r_fma(r_fma(c[3], t, c[2]), t, c[1]), t, c[0]);
        const R dL = r_fma(r_fma(c[6], t, c[5]), t, c[4]);
        dP = T->p0 * dL * r_exp(L - s);
    }
    {
        const R* c = T->ch[j];
        const R L = r_fma(r_fma(r_fma(c[3], t, c[2]), t, c[1]), t, c[0]);
        const R dL = r_fma(r_fma(c[6], t, c[5]), t, c[4]);
        dH = T->h0 * dL * r_exp(L - s);
    }
}

// ------------------------------------------------------ rates of one cell
// Environment of one cell for a micro-integration: density, geometry and the
// entering column, fixed over the interval.
template <typename R> struct Env {
    R n;        // n_H
    R inv_n;    // 1 / n_H
    R c3;       // 1 / (3 k_B n_H): T = 2 E c3 / (2 - x)
    R Qg;       // Q/dx^3 * g: photons entering per unit volume and time, unattenuated
    R k;        // cell optical depth per unit neutral fraction = n sigma0 dx ell
    R tau;      // entering column
    R att;      // mono: exp(-tau)
    R Pin, Hin; // table: normalised P, H at tau
    R lin;      // table: -d ln P / d tau at tau (fraction absorbed per unit depth)
};

// Environment of a cell lit by a source of QV photons per second per cell
// volume.
template <typename R>
PI_HD __forceinline__ Env<R> make_env_q(const Params<R>& p, R QV, R n, CellGeom<R> c, R tau)
{
    Env<R> e;
    e.n = n;
    e.inv_n = r_rcp(n);
    e.c3 = e.inv_n * R(1.0 / (3.0 * KB));
    e.Qg = QV * c.g;
    e.k = n * p.sdx * c.ell;
    e.tau = tau;
    e.att = R(0);
    e.Pin = e.Hin = e.lin = R(0);
    if (p.spectrum == 0) {
        e.att = r_exp(-tau);
    } else {
        R dP, dH;
        table_pair(p.tab, tau, e.Pin, dP, e.Hin, dH);
        e.lin = e.Pin > R(0) ? -dP * r_rcp(e.Pin) : R(0);
    }
    return e;
}

template <typename R>
PI_HD __forceinline__ Env<R> make_env(const Params<R>& p, R n, CellGeom<R> c, R tau)
{
    return make_env_q(p, p.QV, n, c, tau);
}

// Photoionisations A and photoheating G per unit volume and time, and their
// x-derivatives: what enters the cell minus what leaves it (photon-conserving
// form), with the entering column frozen and the cell's own depth k x.
template <typename R>
PI_HD __forceinline__ void photo(const Params<R>& p, const Env<R>& e, R x, R& A, R& dA, R& G,
                                      R& dG)
{
    const R u = e.k * x;
    if (p.spectrum == 0) {
        const R f = e.Qg * e.att;
        A = f * (-r_expm1(-u));
        dA = f * r_exp(-u) * e.k;
        G = A * p.eps;
        dG = dA * p.eps;
        return;
    }
    if (u * e.lin < R(THIN_CELL)) {
        // the cell absorbs a small fraction of what enters: P(tau) - P(tau + u)
        // as the integral of -dP/dtau over the cell by two-point Gauss-Legendre
        // (no cancellation); the x-derivative keeps only the leading term
        // k * mean(-dP/dtau)
        const R c2 = R(0.28867513459481288225);   // 1 / (2 sqrt 3)
        R dP1, dH1, dP2, dH2;
        table_dpair(p.tab, e.tau + (R(0.5) - c2) * u, dP1, dH1);
        table_dpair(p.tab, e.tau + (R(0.5) + c2) * u, dP2, dH2);
        const R mP = R(-0.5) * (dP1 + dP2), mH = R(-0.5) * (dH1 + dH2);
        A = e.Qg * mP * u;
        dA = e.Qg * mP * e.k;
        G = e.Qg * mH * u;
        dG = e.Qg * mH * e.k;
    } else {
        R P, dP, H, dH;
        table_pair(p.tab, e.tau + u, P, dP, H, dH);
        A = e.Qg * (e.Pin - P);
        dA = -e.Qg * dP * e.k;
        G = e.Qg * (e.Hin - H);
        dG = -e.Qg * dH * e.k;
    }
}

// Further point sources of a grid with several: source 0 is (sx, sy, sz) with
// QV of its Params, source q >= 1 sits at v[q - 1] with QV[q - 1].
template <typename R> struct Sources {
    int n;                    // point sources of the grid, >= 1
    int v[MAX_SRC - 1][3];
    R QV[MAX_SRC - 1];        // Q / dx^3
};

// Cell lit by up to MS point sources (a grid with several sources): one Env
// per source (its own geometry and entering column, common n_H); the rates of
// the ns sources add.  The solvers take either environment type.
template <typename R, int MS> struct EnvM {
    R n, inv_n, c3;
    int ns;
    Env<R> s[MS];
};

// Source q's environment, picked by selects over the sources (no indexed
// access, which would place the array in scratch memory).
template <typename R, int MS>
PI_HD __forceinline__ Env<R> env_of(const EnvM<R, MS>& e, int q)
{
    Env<R> r = e.s[0];
#pragma unroll
    for (int k = 1; k < MS; ++k) {
        const bool on = q == k;
        r.n = on ? e.s[k].n : r.n;
        r.inv_n = on ? e.s[k].inv_n : r.inv_n;
        r.c3 = on ? e.s[k].c3 : r.c3;
        r.Qg = on ? e.s[k].Qg : r.Qg;
        r.k = on ? e.s[k].k : r.k;
        r.tau = on ? e.s[k].tau : r.tau;
        r.att = on ? e.s[k].att : r.att;
        r.Pin = on ? e.s[k].Pin : r.Pin;
        r.Hin = on ? e.s[k].Hin : r.Hin;
        r.lin = on ? e.s[k].lin : r.lin;
    }
    return r;
}

// The sources' rates one after another (a loop, not unrolled: the lookups of
// all sources at once spill the integrator's registers).
template <typename R, int MS>
PI_HD __forceinline__ void photo(const Params<R>& p, const EnvM<R, MS>& e, R x, R& A, R& dA,
                                 R& G, R& dG)
{
    photo(p, e.s[0], x, A, dA, G, dG);
#pragma unroll 1
    for (int q = 1; q < MS; ++q) {
        if (q < e.ns) {
            R a, da, g, dg;
            photo(p, env_of(e, q), x, a, da, g, dg);
            A += a;
            dA += da;
            G += g;
            dG += dg;
        }
    }
}

// Temperature-dependent coefficients and their logarithmic T-derivatives:
// case-B recombination (constant or alpha_B (T/1e4)^-0.7), collisional
// ionisation and the cooling coefficients of Cen (1992): recombination and
// free-free (times n_e n_HII), collisional excitation and ionisation (times
// n_e n_HI).
template <typename R> struct Coef {
    R invT;        // 1 / T
    R alpha, dla;
    R aci, dlci;
    R cii, dcii;   // value and dT-derivative (not logarithmic)
    R cin, dcin;
};

// The power laws are products of one power u = T^(1/10):
//   T^1/2                 = u^5
//   (T/1e4)^-0.7          = 1e4^0.7 u^3 / T
//   (T/1e6)^0.7           = 1e6^-0.7 u^7
//   T^1/2 (T/1e3)^-0.2    = 10^0.6 u^3
// Without Cool the cooling coefficients are left at zero (for a caller that
// needs no dE/dt).
template <typename R, bool Cool = true>
PI_HD __forceinline__ Coef<R> coefs(const Params<R>& p, R T)
{
    Coef<R> c;
    const R invT = r_rcp(T);
    c.invT = invT;
    const bool pw = p.recomb != 0, cool = Cool && p.thermal == 1 && p.cooling != 0;
    const R u = r_pow01(T), u2 = u * u, u3 = u2 * u;
    if (!pw) {
        c.alpha = p.alpha_B;
        c.dla = R(0);
    } else {
        c.alpha = p.alpha_B * R(630.95734448019324) * u3 * invT;   // 1e4^0.7
        c.dla = R(-0.7) * invT;
    }
    const R sT = u3 * u2;
    const R s5 = sT * R(0.0031622776601683794);   // sqrt(T/1e5)
    const R invq = r_rcp(R(1) + s5);
    const R dlq = R(0.5) * s5 * invT * invq;       // d ln q / dT, q = 1 + sqrt(T/1e5)
    const R eci = (p.collisional || p.cooling) ? r_exp(R(-157809.1) * invT) : R(0);
    const R dle = R(157809.1) * invT * invT;       // d ln eci / dT
    c.aci = R(0);
    c.dlci = R(0);
    if (p.collisional) {
        c.aci = R(5.85e-11) * sT * invq * eci;
        c.dlci = R(0.5) * invT - dlq + dle;
    }
    c.cii = c.dcii = c.cin = c.dcin = R(0);
    if (cool) {
        const R t6 = R(6.3095734448019325e-05) * (sT * u2);                 // 1e6^-0.7
        const R i16 = r_rcp(R(1) + t6);
        const R crec = R(8.70e-27 * 3.9810717055349722) * u3 * i16;
        const R dlrec = (R(0.3) - R(0.7) * t6 * i16) * invT;
        const R cff = R(1.42e-27 * 1.3) * sT;
        const R cce = R(7.50e-19) * invq * r_exp(R(-118348.0) * invT);
        const R dlce = -dlq + R(118348.0) * invT * invT;
        R cci = R(0), dlci2 = R(0);
        if (p.collisional) {
            cci = R(1.27e-21) * sT * invq * eci;
            dlci2 = R(0.5) * invT - dlq + dle;
        }
        c.cii = crec + cff;
        c.dcii = crec * dlrec + cff * R(0.5) * invT;
        c.cin = cce + cci;
        c.dcin = cce * dlce + cci * dlci2;
    }
    return c;
}

// Right-hand side of eq. (2) in (x, E) and its Jacobian.
template <typename R> struct Rhs {
    R fx, fE, jxx, jxE, jEx, jEE;
    R A, rec, T;
};

template <typename R, typename EV>
PI_HD __forceinline__ void rhs_xT(const Params<R>& p, const EV& e, const Coef<R>& c, R x,
                                       R& fx, R& dfx)
{
    R A, dA, G, dG;
    photo(p, e, x, A, dA, G, dG);
    const R n = e.n, y = R(1) - x;
    fx = -A * e.inv_n - c.aci * n * x * y + c.alpha * n * y * y;
    dfx = -dA * e.inv_n - c.aci * n * (R(1) - R(2) * x) - R(2) * c.alpha * n * y;
}

// Temperature floor: the coefficients see max(T, T_FLOOR) and the cooling is
// tapered by max(0, 1 - T_FLOOR/T), so the floor is approached smoothly and
// never crossed by cooling.
// Without Cool only the x-rate and its Jacobian row, A, rec and T are formed
// (fE and its derivatives are zero): what the timestep needs when the energy
// criterion is off, bit for bit as with it.
template <typename R, typename EV, bool Cool = true>
PI_HD __forceinline__ void rhs_full(const Params<R>& p, const EV& e, R x, R E, Rhs<R>& r)
{
    const R n = e.n;
    R T, Tc, dTdx = R(0), dTdE = R(0), above = R(1);
    if (p.thermal == 0) {
        T = Tc = p.T_fixed;
    } else {
        const R i2mx = r_rcp(R(2) - x);
        dTdE = R(2) * e.c3 * i2mx;
        T = E * dTdE;
        dTdx = T * i2mx;
        above = T > R(T_FLOOR) ? R(1) : R(0);
        Tc = T > R(T_FLOOR) ? T : R(T_FLOOR);
    }
    Coef<R> c = coefs<R, Cool>(p, Tc);
    c.dla *= above;
    c.dlci *= above;
    R A, dA, G, dG;
    photo(p, e, x, A, dA, G, dG);
    const R y = R(1) - x;
    r.A = A;
    r.rec = c.alpha * n * n * y * y;
    r.T = Tc;
    r.fx = -A * e.inv_n - c.aci * n * x * y + c.alpha * n * y * y;
    const R dfx_dT = -c.aci * c.dlci * n * x * y + c.alpha * c.dla * n * y * y;
    r.jxx = -dA * e.inv_n - c.aci * n * (R(1) - R(2) * x) - R(2) * c.alpha * n * y + dfx_dT * dTdx;
    r.jxE = dfx_dT * dTdE;
    if (p.thermal == 0 || !Cool) {
        r.fE = r.jEx = r.jEE = R(0);
        return;
    }
    // 1/T where it is used (above the floor, where Tc is T)
    const R iT = c.invT;
    const R w = T > R(T_FLOOR) ? R(1) - R(T_FLOOR) * iT : R(0);
    const R dw = T > R(T_FLOOR) ? R(T_FLOOR) * iT * iT : R(0);
    const R n2 = n * n;
    const R lam0 = n2 * (y * y * c.cii + x * y * c.cin);
    const R dlam0_dx = n2 * (R(-2) * y * c.cii + (R(1) - R(2) * x) * c.cin);
    const R dlam0_dT = above * n2 * (y * y * c.dcii + x * y * c.dcin);
    const R dlam_dT = dlam0_dT * w + lam0 * dw;
    r.fE = G - lam0 * w;
    r.jEx = dG - dlam0_dx * w - dlam_dT * dTdx;
    r.jEE = -dlam_dT * dTdE;
}

template <typename R> PI_HD __forceinline__ R e_floor(R n, R x)
{
    return R(1.5 * KB * T_FLOOR) * n * (R(2) - x);
}

// Scalar stage solve x = xb + hg fx(x) at fixed temperature (coefficients c):
// Newton safeguarded by the bracket [0, 1] (the residual increases with x); a
// root outside [0, 1] is returned clamped.
template <typename R, typename EV>
PI_HD R solve_x(const Params<R>& p, const EV& e, const Coef<R>& c, R xb, R hg, R x, int& nit)
{
    x = r_min(r_max(x, R(0)), R(1));
    R lo = R(0), hi = R(1);
    R eprev = R(1e30);
    for (int it = 0; it < NEWTON_MAXIT; ++it) {
        ++nit;
        R fx, dfx;
        rhs_xT(p, e, c, x, fx, dfx);
        const R G = x - xb - hg * fx;
        const R dG = R(1) - hg * dfx;
        if (G > R(0)) hi = x; else lo = x;
        R xn = x - G / dG;
        if (xn <= R(0) && lo == R(0)) {
            R f0, d0;
            rhs_xT(p, e, c, R(0), f0, d0);
            if (-xb - hg * f0 >= R(0)) return R(0);
        }
        if (xn >= R(1) && hi == R(1)) {
            R f1, d1;
            rhs_xT(p, e, c, R(1), f1, d1);
            if (R(1) - xb - hg * f1 <= R(0)) return R(1);
        }
        if (!(xn >= lo && xn <= hi)) xn = R(0.5) * (lo + hi);
        const R err = r_abs(xn - x) / r_max(xn, R(1e-12));
        x = xn;
        if (err <= Tol<R>::rtol || (err >= eprev && err <= Tol<R>::stall)) break;
        eprev = err;
    }
    return x;
}

// Energy residual of the stage equation with T held, after solving x at that T.
template <typename R, typename EV>
PI_HD R t_residual(const Params<R>& p, const EV& e, R xb, R Eb, R hg, R T, R& xs)
{
    const Coef<R> c = coefs(p, T);
    int nit = 0;
    const R x = solve_x(p, e, c, xb, hg, r_min(r_max(xb, R(0)), R(1)), nit);
    const R E = R(1.5 * KB) * e.n * (R(2) - x) * T;
    Rhs<R> r;
    rhs_full(p, e, x, E, r);
    xs = x;
    return E - Eb - hg * r.fE;
}

// Fallback of the T-evolving stage solve (rarely taken): nested bracketed
// solve in (x, T) -- x at fixed T by the scalar solve, and the energy residual
// bracketed in ln T from the floor upwards and solved by the Illinois variant
// of regula falsi.
template <typename R, typename EV>
PI_HD void fallback_solve(const Params<R>& p, const EV& e, R xb, R Eb, R hg,
                                            R& x, R& E)
{
    R xs;
    R la = r_log(R(T_FLOOR));
    R ga = t_residual(p, e, xb, Eb, hg, R(T_FLOOR), xs);
    if (ga >= R(0)) {
        x = xs;
        E = R(1.5 * KB) * e.n * (R(2) - xs) * R(T_FLOOR);
        return;
    }
    const R Tg = r_max(R(2) * E / (R(3.0 * KB) * e.n * (R(2) - x)), R(2.0 * T_FLOOR));
    R lb = r_log(Tg);
    R gb = t_residual(p, e, xb, Eb, hg, Tg, xs);
    for (int k = 0; k < 60 && gb < R(0); ++k) {
        la = lb;
        ga = gb;
        lb += R(1);
        gb = t_residual(p, e, xb, Eb, hg, r_exp(lb), xs);
    }
    R lc = lb;
    int side = 0;
    for (int it = 0; it < FALLBACK_MAXIT; ++it) {
        lc = (la * gb - lb * ga) / (gb - ga);
        const R gc = t_residual(p, e, xb, Eb, hg, r_exp(lc), xs);
        if (gc == R(0) || r_abs(lb - la) <= Tol<R>::rtol * r_abs(lc)) break;
        if ((gc > R(0)) == (gb > R(0))) {
            lb = lc;
            gb = gc;
            if (side == -1) ga *= R(0.5);
            side = -1;
        } else {
            la = lc;
            ga = gc;
            if (side == 1) gb *= R(0.5);
            side = 1;
        }
    }
    const R T = r_exp(lc);
    t_residual(p, e, xb, Eb, hg, T, xs);
    x = xs;
    E = R(1.5 * KB) * e.n * (R(2) - xs) * T;
}


// Stage solve Y = base + hg f(Y); counts Newton iterations and fallbacks in w.
// T fixed: the scalar bracketed Newton.  T evolving: Newton on (x, E) with x
// projected onto [0,1] (E then takes the step of the linearisation with x on
// the bound) and E kept positive, at most NEWTON_2D_MAXIT iterations (in float,
// a small plain first step is accepted at once, see Tol<float>::one_step);
// if it has not settled, a nested bracketed solve in (x, T): x at fixed T by the
// scalar solve, and the energy residual bracketed in ln T from the floor
// upwards and solved by the Illinois variant of regula falsi.
// Work done by one micro-integration (accepted and rejected substeps, stage
// fallbacks), summed per launch for the performance counters.
struct Work {
    int accepted, rejected, fallbacks, newton;
    int close;   // substep-control decisions near their thresholds
    int fixed;   // cells re-solved in double (mixed precision)
};

template <typename R, typename EV>
PI_HD void stage_solve(const Params<R>& p, const EV& e, R xb, R Eb, R hg, R& x, R& E,
                       Work& w)
{
    if (p.thermal == 0) {
        const Coef<R> c = coefs(p, p.T_fixed);
        x = solve_x(p, e, c, xb, hg, x, w.newton);
        return;
    }
    x = r_min(r_max(x, R(0)), R(1));
    if (!(E > R(0))) E = e_floor(e.n, x);
    R eprev = R(1e30);
    for (int it = 0; it < NEWTON_2D_MAXIT; ++it) {
        ++w.newton;
        Rhs<R> r;
        rhs_full(p, e, x, E, r);
        const R Rx = x - xb - hg * r.fx;
        const R RE = E - Eb - hg * r.fE;
        const R a11 = R(1) - hg * r.jxx, a12 = -hg * r.jxE;
        const R a21 = -hg * r.jEx, a22 = R(1) - hg * r.jEE;
        const R idet = r_rcp(a11 * a22 - a12 * a21);
        R xn = x - (a22 * Rx - a12 * RE) * idet;
        R En = E - (a11 * RE - a21 * Rx) * idet;
        bool plain = true;   // an unmodified Newton step
        if (!(xn >= R(0)) || xn > R(1)) {
            plain = false;
            // x held on the bound; E takes the step of the linearisation there
            const R xbnd = xn > R(1) ? R(1) : R(0);
            En = E - (RE + a21 * (xbnd - x)) * r_rcp(a22);
            xn = xbnd;
        }
        if (!(En > R(0))) {
            En = R(0.5) * E;
            plain = false;
        }
        const R err = r_max(r_abs(xn - x) * r_rcp(r_max(xn, R(1e-12))), r_abs(En - E) * r_rcp(En));
        // x held on a bound while the residual puts the root inside [0, 1]
        // (a negative slope of the x-residual): not a solution -- unless at 1
        // the root lies within half a rounding step of 1
        const bool stuck = (xn >= R(1) && Rx > Tol<R>::half_ulp1 * r_abs(a11)) ||
                           (xn <= R(0) && Rx < R(0));
        x = xn;
        E = En;
        if (!stuck && (err <= Tol<R>::rtol || (err >= eprev && err <= Tol<R>::stall) ||
                       (plain && it == 0 && err <= Tol<R>::one_step))) {
            // x = 1 held although it is an unstable equilibrium (a11 < 0) and
            // the residual pushes x inside: the precision cannot resolve the
            // seed that would start the runaway
            if (xn >= R(1) && Rx > R(0) && a11 < R(0)) ++w.close;
            return;
        }
        eprev = err;
    }
    fallback_solve(p, e, xb, Eb, hg, x, E);
    ++w.fallbacks;
    ++w.close;   // (its tolerance follows the precision: re-solved in double when mixed)
}

// Initial substep count of one micro-integration: at least n_sub, and enough
// that at the initial rate no substep moves x by more than SUB_DX; at most
// SUB_MAX.
template <typename R, typename EV>
PI_HD __forceinline__ int substeps(const Params<R>& p, const EV& e, R x0, R E0, R h, Work& w,
                                  R& fx0, R& fE0)
{
    Rhs<R> r;
    rhs_full(p, e, x0, E0, r);
    fx0 = r.fx;
    fE0 = r.fE;
    const double s = (double)h * (double)r_abs(r.fx) / SUB_DX;
    int ns = p.n_sub > 0 ? p.n_sub : 1;
    if (s > (double)ns * (1.0 - MIX_MARGIN) && s < (double)SUB_MAX * (1.0 + MIX_MARGIN)) {
        const double fr = s - floor(s);   // ceil(s) changes at the integers
        if (fr < MIX_MARGIN * s || 1.0 - fr < MIX_MARGIN * s) ++w.close;
    }
    if (s > (double)ns) ns = s >= (double)SUB_MAX ? SUB_MAX : (int)ceil(s);
    return ns;
}

// A stage solve at its call in sdirk_step, and a float micro-integration at
// its call: inlined for float cells (out of line, the environment would be
// passed on the stack and read from scratch memory in every rate evaluation,
// and the compiler's inlining budget does not always take them whole); the
// compiler's choice for double.
template <typename R, typename EV> struct InlineFloat { static constexpr bool value = false; };
template <typename EV> struct InlineFloat<float, EV> { static constexpr bool value = true; };
template <typename R, typename EV>
PI_HD __forceinline__ void stage_solve_at(const Params<R>& p, const EV& e, R xb, R Eb, R hg, R& x,
                                          R& E, Work& w)
{
    if constexpr (InlineFloat<R, EV>::value) {
        [[clang::always_inline]] stage_solve(p, e, xb, Eb, hg, x, E, w);
    } else {
        stage_solve(p, e, xb, Eb, hg, x, E, w);
    }
}

// Starting guess of a stage solve: the stage's base advanced by hg times an
// estimate of the rate, unless that takes x out of [0, 1] or changes E by more
// than PRED_MAX of itself (a stiff component, for which the explicit estimate
// overshoots); then the base itself.  The guess only changes where Newton
// starts, not the root it converges to.
constexpr double PRED_MAX = 0.5;
template <typename R>
PI_HD __forceinline__ void stage_guess(R xb, R Eb, R hg, R fx, R fE, R& xg, R& Eg)
{
    const R dx = hg * fx, dE = hg * fE;
    const bool ok = xb + dx >= R(0) && xb + dx <= R(1) && r_abs(dE) <= R(PRED_MAX) * Eb;
    xg = ok ? xb + dx : xb;
    Eg = ok ? Eb + dE : Eb;
}

// One step of the two-stage, L-stable, stiffly accurate SDIRK method
// (gamma = 1 - 1/sqrt 2); the second stage starts from y + ((1-gamma)/gamma)(Y1 - y).
// (fx, fE) is the rate at (x, E) on entry and at the new (x, E) on return: a
// solved stage equation Y = base + hg f(Y) gives f(Y) = (Y - base)/hg without
// another evaluation.  Stage 1 starts from y + hg f(y), stage 2 from its base
// + hg f(Y1).
template <typename R, typename EV>
PI_HD __forceinline__ void sdirk_step(const Params<R>& p, const EV& e, R hs, R& x, R& E,
                                      R& fx, R& fE, Work& w, R& x_stage1)
{
    const R gam = R(0.29289321881345247560);          // 1 - 1/sqrt(2)
    const R cst = R(2.41421356237309504880);          // (1 - gamma)/gamma
    const R hg = gam * hs;
    R X1, F1;
    stage_guess(x, E, hg, fx, fE, X1, F1);
    stage_solve_at(p, e, x, E, hg, X1, F1, w);
    const R xb = x + cst * (X1 - x);
    const R Eb = E + cst * (F1 - E);
    R X2, F2;
    stage_guess(xb, Eb, R(1), X1 - x, F1 - E, X2, F2);   // hg f(Y1) = Y1 - y
    stage_solve_at(p, e, xb, Eb, hg, X2, F2, w);
    const R ihg = r_rcp(hg);
    fx = (X2 - xb) * ihg;
    fE = (F2 - Eb) * ihg;
    x_stage1 = X1;
    x = X2;
    E = F2;
}

// Integral of exp(-tau) terms held as S exp(-m), so that a very thick cell
// does not underflow (algorithm 1's time-averaged attenuation).
template <typename R> struct LseAcc {
    R m = R(0), S = R(0);
    PI_HD __forceinline__ void add(R w, R tau)
    {
        if (S == R(0)) {
            m = tau;
            S = w;
        } else if (tau >= m) {
            S += w * r_exp(-(tau - m));
        } else {
            S = S * r_exp(-(m - tau)) + w;
            m = tau;
        }
    }
};

// Micro-integration M(x0, E0; tau, h) with deterministic substep control: the
// interval is cut into U = ns 2^SUB_LEVELS units; a substep of s units is
// rejected and halved (while s > 1) if x moved by more than REJ_DX or E changed
// by more than a factor REJ_E, and doubled again after an accepted substep
// when the position allows.  E is held at or above
// the temperature floor between substeps.
// With AVG (algorithm 1, Sect. 2.1) the cell's attenuation exp(-k x(t)) is
// integrated over h with the same SDIRK stages (weights 1 - gamma and gamma at
// the two stage values of x of every accepted substep), and tau_avg returns
// the time-averaged optical depth -ln <exp(-k x)>.
template <typename R, bool AVG, typename EV>
PI_HD void micro_t(const Params<R>& p, const EV& e, R h, R& x, R& E, Work& w, R* tau_avg)
{
    if constexpr (AVG) *tau_avg = e.k * x;
    if (!(h > R(0))) return;
    LseAcc<R> acc;
    const bool evolve = p.thermal == 1;
    if (evolve && E < e_floor(e.n, x)) E = e_floor(e.n, x);
    R fx, fE;
    const int ns = substeps(p, e, x, E, h, w, fx, fE);
    const int top = 1 << SUB_LEVELS;
    const int U = ns * top;
    const double hU = (double)h / (double)U;   // one division; substeps are s units of it
    int pos = 0, s = top;
    while (pos < U) {
        const R hs = R(hU * (double)s);
        R xn = x, En = E, fxn = fx, fEn = fE, X1;
        sdirk_step(p, e, hs, xn, En, fxn, fEn, w, X1);
        const R dx = r_abs(xn - x);
        const bool bad = dx > R(REJ_DX) || (evolve && (En > R(REJ_E) * E || En * R(REJ_E) < E));
        if (r_abs(dx - R(REJ_DX)) < R(MIX_MARGIN * REJ_DX) ||
            (evolve && (r_abs(En - R(REJ_E) * E) < R(MIX_MARGIN * REJ_E) * E ||
                        r_abs(En * R(REJ_E) - E) < R(MIX_MARGIN) * E)))
            ++w.close;
        if (bad && s > 1) {
            s >>= 1;
            ++w.rejected;
            continue;
        }
        ++w.accepted;
        if constexpr (AVG) {
            const R gam = R(0.29289321881345247560);
            acc.add(hs * (R(1) - gam), e.k * X1);
            acc.add(hs * gam, e.k * xn);
        }
        x = xn;
        E = En;
        fx = fxn;
        fE = fEn;
        if (evolve && E < e_floor(e.n, x)) E = e_floor(e.n, x);
        pos += s;
        if (s < top && pos % (2 * s) == 0) s <<= 1;
    }
    if constexpr (AVG) *tau_avg = acc.m - r_log(acc.S / h);
}

template <typename R, typename EV>
PI_HD __forceinline__ void micro(const Params<R>& p, const EV& e, R h, R& x, R& E, Work& w)
{
    if constexpr (InlineFloat<R, EV>::value) {
        // inline, as stage_solve_at: its environment then stays in registers
        [[clang::always_inline]] micro_t<R, false>(p, e, h, x, E, w, nullptr);
    } else {
        micro_t<R, false>(p, e, h, x, E, w, nullptr);
    }
}

// Per-cell limit of eq. (4) at (x, E) with the entering column of t_n:
// min(K1 t_rec, K2 E/|dE/dt|, K3 max(0.05, x)/|dy/dt|, K4/|dy/dt|); a factor
// of +inf (or any value above 1e30) disables its criterion, and a zero rate
// does not limit.
template <typename R>
PI_HD __forceinline__ double cell_dt(const Params<R>& p, const Rhs<R>& r, R n, R x, R E)
{
    const R KOFF = R(1e30);
    double dt = __builtin_huge_val();
    const double ydot = (double)r_abs(r.fx);
    if (p.K[0] < KOFF) {
        const Coef<R> c = coefs(p, r.T);
        dt = fmin(dt, (double)p.K[0] / ((double)c.alpha * (double)n));
    }
    if (p.K[1] < KOFF && p.thermal == 1 && r.fE != R(0))
        dt = fmin(dt, (double)p.K[1] * (double)E / fabs((double)r.fE));
    if (p.K[2] < KOFF && ydot > 0.0) dt = fmin(dt, (double)p.K[2] * fmax(0.05, (double)x) / ydot);
    if (p.K[3] < KOFF && ydot > 0.0) dt = fmin(dt, (double)p.K[3] / ydot);
    return dt;
}

}  // namespace pi
