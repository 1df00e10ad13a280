// Sparse waveform stage on the GPU (Sec. II: the 11 parameters, harmonic
// modes h_lm = A_lm e^{i phi_lm} (Eq. amp_and_phase), the time-frequency map
// t_lm(f) = t_coal - (1/2pi) dphi_lm/df (Eq. t_f) and the cut t_lm < 0).
//
// The paper names PhenomHM without printing it; the model evaluated here is
// the project's PhenomHM-structured surrogate:
//   (2,2) phase: TaylorF2 (3.5PN point mass + 1.5PN spin-orbit + 2PN
//     spin-spin) for M f <= 0.008, continued C^2 by
//     b0 + b1 f - (3/5) cR f^{-5/3} - kRD fd F((f - fRD)/fd),
//     F(u) = u atan u - ln(1 + u^2)/2, kRD = 1/fd;
//   (2,2) amplitude: sqrt(2 eta/3) pi^{-1/6} M^2/D_L (M f)^{-7/6}
//     (1 + 2 L(f)) / (1 + e^{u}), L = 1/(1+u^2), u = (f - fRD)/fd;
//   remnant: a_f = x1^2 chi1 + x2^2 chi2 + 2 sqrt3 eta - 3.871 eta^2
//     + 4.028 eta^3 (clamped to +-0.99), E_rad quartic in eta, (2,2,0) QNM
//     from the Berti-Cardoso-Will fit form;
//   alignment: phase and slope vanish at f_peak = argmax f^2 A_22, so
//     t_22(f_peak) = t_coal;
//   mode (l,m): (2,2) functions at f~ = 2f/m, phase x m/2 plus the constant
//     of the stationary-phase transform, amplitude x sqrt(2/m) |H_lm/H_22|
//     (leading post-Newtonian order of the multipole radiation).
#include <hip/hip_runtime.h>

#include <cmath>

#include "mbh_internal.h"

namespace mbh {
namespace {

constexpr double kPi = 3.141592653589793238462643;
constexpr double kTwoPi = 6.283185307179586476925287;
constexpr double kMsunSec = 4.925490947e-6;          // G Msun / c^3
constexpr double kGpcSec = 3.0856775814913673e25 / 299792458.0;
constexpr double kEulerGamma = 0.5772156649015329;
constexpr double kMfJoin = 0.008;
constexpr double kMfCut = 0.2;
constexpr double kLorentzHeight = 2.0;

__device__ bool params_ok(const double *p)
{
    bool ok = true;
    for (int i = 0; i < 11; ++i) ok = ok && isfinite(p[i]);
    ok = ok && (p[0] > 0.0) && (p[1] > 0.0) && (p[1] <= 1.0);
    ok = ok && (fabs(p[2]) <= 0.99) && (fabs(p[3]) <= 0.99) && (p[4] > 0.0);
    return ok;
}

// TaylorF2 (2,2) phase phi_I = -Psi(v) and its first two f-derivatives.
__device__ void taylorf2(const Source &s, double f, double &ph, double &d1, double &d2)
{
    const double v = cbrt(kPi * s.M * f);
    const double iv = 1.0 / v;
    const double iv2 = iv * iv, iv3 = iv2 * iv, iv4 = iv2 * iv2, iv5 = iv4 * iv;
    const double iv6 = iv3 * iv3, iv7 = iv6 * iv;
    const double K = 3.0 / (128.0 * s.eta);
    const double lg4v = log(4.0 * v);
    const double lgv = log(v * 2.449489742783178098197284);  // v / v_lso, v_lso = 6^{-1/2}
    const double P = K * (iv5 + s.p2 * iv3 + s.p3 * iv2 + s.p4 * iv + s.p5 * (1.0 + 3.0 * lgv) +
                          (s.p6 + s.p6L * lg4v) * v + s.p7 * v * v);
    const double Pv = K * (-5.0 * iv6 - 3.0 * s.p2 * iv4 - 2.0 * s.p3 * iv3 - s.p4 * iv2 + 3.0 * s.p5 * iv +
                           s.p6 + s.p6L * (lg4v + 1.0) + 2.0 * s.p7 * v);
    const double Pvv = K * (30.0 * iv7 + 12.0 * s.p2 * iv5 + 6.0 * s.p3 * iv4 + 2.0 * s.p4 * iv3 -
                            3.0 * s.p5 * iv2 + s.p6L * iv + 2.0 * s.p7);
    const double piM = kPi * s.M;
    const double dv = piM * iv2 / 3.0;
    const double ddv = -2.0 * piM * piM * iv5 / 9.0;
    ph = -P;
    d1 = -Pv * dv;
    d2 = -(Pvv * dv * dv + Pv * ddv);
}

__device__ void ringdown_phase(const Source &s, double f, double &ph, double &d1, double &d2)
{
    const double u = (f - s.fRD) / s.fd;
    const double at = atan(u);
    const double fm53 = pow(f, -5.0 / 3.0);
    const double fm83 = fm53 / f;
    ph = s.b0 + s.b1 * f - 0.6 * s.cR * fm53 - s.kRD * s.fd * (u * at - 0.5 * log1p(u * u));
    d1 = s.b1 + s.cR * fm83 - s.kRD * at;
    d2 = -(8.0 / 3.0) * s.cR * fm83 / f - s.kRD / (s.fd * (1.0 + u * u));
}

__device__ void phase22_raw(const Source &s, double f, double &ph, double &d1, double &d2)
{
    if (f <= s.fJ) taylorf2(s, f, ph, d1, d2);
    else ringdown_phase(s, f, ph, d1, d2);
}

__device__ double amp22(const Source &s, double f)
{
    const double u = (f - s.fRD) / s.fd;
    const double lor = 1.0 / (1.0 + u * u);
    return s.A0 * pow(s.M * f, -7.0 / 6.0) * (1.0 + kLorentzHeight * lor) / (1.0 + exp(u));
}

// d/df ln(f^2 A_22)
__device__ double dlog_f2amp(const Source &s, double f)
{
    const double u = (f - s.fRD) / s.fd;
    const double lor = 1.0 / (1.0 + u * u);
    const double tail = 1.0 - 1.0 / (1.0 + exp(u));   // 1 - logistic cut-off
    const double dlor = -2.0 * u * lor * lor / s.fd;
    return 5.0 / (6.0 * f) + kLorentzHeight * dlor / (1.0 + kLorentzHeight * lor) - tail / s.fd;
}

// Leading-order coefficient of the time-domain mode h_lm ~ H_lm e^{-i m Phi}
// of a circular binary relative to H_22, at orbital velocity v: r = |H_lm/H_22|
// and the constant phase of the frequency-domain mode.  The positive
// frequencies carry h_{l,-m} = (-1)^l conj(h_lm); stationary phase of a
// harmonic m adds pi/4, i.e. (1 - m/2) pi/4 relative to (m/2) phi_22, so the
// constant is l pi - arg H_lm - (m - 2) pi/8 (not reduced modulo 2 pi), with
//   arg H = 0 (22, 32), -pi/2 (33, 43), pi (44), pi/2 (21).
__device__ void mode_factor(const Source &s, int l, int m, double v, double &r, double &off)
{
    const double e3 = 1.0 - 3.0 * s.eta;
    double argh;
    if (l == 2 && m == 2) { r = 1.0; argh = 0.0; }
    else if (l == 3 && m == 3) { r = 0.75 * sqrt(15.0 / 14.0) * s.delta * v; argh = -0.5 * kPi; }
    else if (l == 4 && m == 4) { r = (8.0 / 9.0) * sqrt(5.0 / 7.0) * e3 * v * v; argh = kPi; }
    else if (l == 2 && m == 1) { r = s.delta * v / 3.0; argh = 0.5 * kPi; }
    else if (l == 3 && m == 2) { r = (1.0 / 3.0) * sqrt(5.0 / 7.0) * e3 * v * v; argh = 0.0; }
    else { r = 9.0 / (4.0 * sqrt(70.0)) * s.delta * (1.0 - 2.0 * s.eta) * v * v * v; argh = -0.5 * kPi; }
    off = l * kPi - argh - (m - 2) * kPi / 8.0;
}

// Mode amplitude, phase and its derivative at f (aligned (2,2) at f~ = 2f/m).
__device__ void mode_at(const Source &s, int l, int m, double f, double &A, double &ph, double &dph)
{
    const double ft = 2.0 * f / m;
    double p, a, b;
    phase22_raw(s, ft, p, a, b);
    const double v = cbrt(kPi * s.M * ft);
    double r, off;
    mode_factor(s, l, m, v, r, off);
    A = sqrt(2.0 / m) * r * amp22(s, ft);
    ph = 0.5 * m * (p - s.al0 - s.al1 * (ft - s.fpeak)) + off;
    dph = a - s.al1;
}

__device__ double mode_time(const Source &s, int l, int m, double f)
{
    const double ft = 2.0 * f / m;
    double p, a, b;
    phase22_raw(s, ft, p, a, b);
    return s.tcoal - (a - s.al1) / kTwoPi;
}

// ---------------------------------------------------------------------------
// Root brackets refined by a group of kRootLanes lanes of one wavefront.  Each
// round places kRootLanes - 1 points evenly inside [lo, hi] (one per lane;
// the last lane holds hi), keeps the sub-bracket in which the predicate
// first holds, and stops once no double lies strictly inside, i.e. lo and hi
// are adjacent doubles.  pred must be false at lo and true at hi; for a
// predicate that switches once, the result is the smallest double at which
// it holds, the pair that repeated halving also ends on, in a fifth
// of the halving rounds (each round divides the bracket by kRootLanes, not 2).  All
// lanes of a group must call it together with the same lo and hi; the group
// is the aligned block of kRootLanes lanes containing the caller.
// ---------------------------------------------------------------------------
constexpr int kRootLanes = 32;
static_assert(kRootLanes >= 2 && kRootLanes <= 32 && (kRootLanes & (kRootLanes - 1)) == 0, "group of 2..32 lanes");

template <typename F>
__device__ void group_bracket(double &lo, double &hi, F pred)
{
    const int lane = threadIdx.x & 63;
    const int gl = lane & (kRootLanes - 1);
    const int base = lane - gl;
    const unsigned gmask = kRootLanes == 32 ? 0xffffffffu : (1u << (kRootLanes & 31)) - 1u;
    for (int round = 0; round < 80; ++round) {
        const double x = gl < kRootLanes - 1 ? fma(hi - lo, (double)(gl + 1) * (1.0 / kRootLanes), lo) : hi;
        const bool inside = x > lo && x < hi;
        const bool hit = inside && pred(x);
        const unsigned gi = (unsigned)(__ballot(inside) >> base) & gmask;
        const unsigned gh = (unsigned)(__ballot(hit) >> base) & gmask;
        if (gi == 0u) break;                       // lo and hi are adjacent
        if (gh != 0u) {
            const int j = __ffs(gh) - 1;           // first sample where pred holds
            const unsigned below = gi & ((1u << j) - 1u);
            const double xj = __shfl(x, base + j);
            const double xb = __shfl(x, base + (below ? 31 - __clz(below) : 0));
            if (below) lo = xb;
            hi = xj;
        } else {
            lo = __shfl(x, base + 31 - __clz(gi));  // pred false at every sample
        }
    }
}

// ---------------------------------------------------------------------------
// Kernel 1: per-walker constants, one group of kRootLanes lanes per walker
// (the lanes share the root search for f_peak; lane 0 of the group writes).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(128) void k_source(const double *__restrict__ params, int B, double t0, Source *__restrict__ out)
{
    const int w = (blockIdx.x * blockDim.x + threadIdx.x) / kRootLanes;
    const bool writer = (threadIdx.x & (kRootLanes - 1)) == 0;
    if (w >= B) return;                            // whole groups leave together
    const double *p = params + 11 * (size_t)w;
    Source s;
    for (int i = 0; i < (int)(sizeof(Source) / sizeof(double)); ++i) reinterpret_cast<double *>(&s)[i] = 0.0;
    s.valid = params_ok(p) ? 1 : 0;
    if (!s.valid) {
        if (writer) out[w] = s;
        return;
    }
    const double q = p[1];
    s.M = p[0] * kMsunSec;
    s.x1 = 1.0 / (1.0 + q);
    s.x2 = q / (1.0 + q);
    s.eta = s.x1 * s.x2;
    s.delta = s.x1 - s.x2;
    s.chi1 = p[2];
    s.chi2 = p[3];
    s.Dl = p[4] * kGpcSec;
    s.phiref = p[5];
    s.iota = p[6];
    s.lam = p[7];
    s.beta = p[8];
    s.psi = p[9];
    s.tcoal = t0 + p[10];

    const double eta = s.eta, eta2 = eta * eta, eta3 = eta2 * eta;
    const double so = (113.0 / 12.0 * s.x1 * s.x1 + 6.25 * eta) * s.chi1 + (113.0 / 12.0 * s.x2 * s.x2 + 6.25 * eta) * s.chi2;
    const double ss = 9.875 * eta * s.chi1 * s.chi2;
    s.p2 = 3715.0 / 756.0 + 55.0 / 9.0 * eta;
    s.p3 = -16.0 * kPi + 4.0 * so;
    s.p4 = 15293365.0 / 508032.0 + 27145.0 / 504.0 * eta + 3085.0 / 72.0 * eta2 - 10.0 * ss;
    s.p5 = kPi * (38645.0 / 756.0 - 65.0 / 9.0 * eta);
    s.p6 = 11583231236531.0 / 4694215680.0 - 640.0 / 3.0 * kPi * kPi - 6848.0 / 21.0 * kEulerGamma +
           (-15737765635.0 / 3048192.0 + 2255.0 / 12.0 * kPi * kPi) * eta + 76055.0 / 1728.0 * eta2 -
           127825.0 / 1296.0 * eta3;
    s.p6L = -6848.0 / 21.0;
    s.p7 = kPi * (77096675.0 / 254016.0 + 378515.0 / 1512.0 * eta - 74045.0 / 756.0 * eta2);

    double af = s.x1 * s.x1 * s.chi1 + s.x2 * s.x2 * s.chi2 + 3.464101615137754587 * eta - 3.871 * eta2 + 4.028 * eta3;
    af = fmin(0.99, fmax(-0.99, af));
    s.af = af;
    const double erad = 0.0559745 * eta + 0.580951 * eta2 - 0.960673 * eta3 + 3.35241 * eta2 * eta2;
    s.Mfin = s.M * (1.0 - erad);
    const double omega = 1.5251 - 1.1568 * pow(1.0 - af, 0.1292);
    const double Q = 0.7 + 1.4187 * pow(1.0 - af, -0.4990);
    s.fRD = omega / (kTwoPi * s.Mfin);
    s.fd = s.fRD / (2.0 * Q);

    s.fJ = kMfJoin / s.M;
    s.kRD = 1.0 / s.fd;
    double pj, d1j, d2j;
    taylorf2(s, s.fJ, pj, d1j, d2j);
    const double uj = (s.fJ - s.fRD) / s.fd;
    s.cR = -0.375 * pow(s.fJ, 11.0 / 3.0) * (d2j + s.kRD / (s.fd * (1.0 + uj * uj)));
    s.b1 = d1j - s.cR * pow(s.fJ, -8.0 / 3.0) + s.kRD * atan(uj);
    s.b0 = pj - s.b1 * s.fJ + 0.6 * s.cR * pow(s.fJ, -5.0 / 3.0) + s.kRD * s.fd * (uj * atan(uj) - 0.5 * log1p(uj * uj));

    // f_peak: bisection of d ln(f^2 A_22)/df on [f_J, f_RD]
    double lo = s.fJ, hi = s.fRD, fp;
    if (dlog_f2amp(s, lo) <= 0.0) {
        fp = lo;
    } else if (dlog_f2amp(s, hi) >= 0.0) {
        fp = hi;
    } else {
        group_bracket(lo, hi, [&](double x) { return dlog_f2amp(s, x) <= 0.0; });
        fp = 0.5 * (lo + hi);
    }
    s.fpeak = fp;
    double a, b, c;
    phase22_raw(s, fp, a, b, c);
    s.al0 = a;
    s.al1 = b;
    s.A0 = sqrt(2.0 * eta / 3.0) * pow(kPi, -1.0 / 6.0) * s.M * s.M / s.Dl;
    if (writer) out[w] = s;
}

// Spin-weight -2 spherical harmonic, l <= 4, via the Wigner small-d sum.
__device__ void swsh_m2(int l, int m, double th, double ph, double &re, double &im)
{
    const double fact[9] = {1.0, 1.0, 2.0, 6.0, 24.0, 120.0, 720.0, 5040.0, 40320.0};
    const double c = cos(0.5 * th), sn = sin(0.5 * th);
    double d = 0.0;
    for (int k = 0; k <= 2 * l; ++k) {
        const int a = l + m - k, b = l - 2 - k, e = k + 2 - m;
        if (a < 0 || b < 0 || e < 0) continue;
        const double pre = sqrt(fact[l + m] * fact[l - m] * fact[l + 2] * fact[l - 2]) / (fact[a] * fact[b] * fact[k] * fact[e]);
        double cp = 1.0, sp = 1.0;
        for (int i = 0; i < a + b; ++i) cp *= c;
        for (int i = 0; i < k + e; ++i) sp *= sn;
        d += ((k & 1) ? -pre : pre) * cp * sp;
    }
    const double amp = sqrt((2.0 * l + 1.0) / (4.0 * kPi)) * d;
    double sm, cm;
    sincos(m * ph, &sm, &cm);
    re = amp * cm;
    im = amp * sm;
}

// ---------------------------------------------------------------------------
// Kernel 2: frequency support and polarization weights, one group of
// kRootLanes lanes per (walker, mode).  f_start is the root of t_lm(f) = 0,
// bracketed to adjacent doubles; f_end = min(band end, (m/2) 0.2 / M).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_bands(int B, Modes md, GridDesc g, const Source *__restrict__ src, ModeBand *__restrict__ band)
{
    const int id = (blockIdx.x * blockDim.x + threadIdx.x) / kRootLanes;
    if (id >= B * md.nm) return;                   // whole groups leave together
    const int w = id / md.nm, im = id - w * md.nm;
    const int l = md.l[im], m = md.m[im];
    const Source s = src[w];
    ModeBand b;
    b.fs = 0.0;
    b.fe = 0.0;
    b.klo = 0;
    b.khi = -1;
    b.active = 0;
    b.pad = 0;
    b.kp[0] = b.kp[1] = b.kc[0] = b.kc[1] = 0.0;
    if (s.valid) {
        const double f_lo = (double)g.k0 * g.df;
        const double f_hi = (double)(g.k0 + g.n - 1) * g.df;
        const double fe = fmin(0.5 * m * kMfCut / s.M, f_hi);
        b.fs = f_lo;
        b.fe = fe;
        bool have = fe > f_lo;
        double fs = f_lo;
        if (have) {
            if (mode_time(s, l, m, f_lo) >= 0.0) {
                fs = f_lo;
            } else if (mode_time(s, l, m, fe) < 0.0) {
                have = false;
            } else {
                double lo = f_lo, hi = fe;
                group_bracket(lo, hi, [&](double x) { return mode_time(s, l, m, x) >= 0.0; });
                fs = hi;
            }
        }
        if (have) {
            b.fs = fs;
            long long klo = (long long)ceil(fs / g.df);
            long long khi = (long long)floor(fe / g.df);
            if (klo < g.k0) klo = g.k0;
            if (khi > g.k0 + g.n - 1) khi = g.k0 + g.n - 1;
            b.klo = (int)klo;
            b.khi = (int)khi;
            b.active = (khi >= klo + 3) ? 1 : 0;
        }
        // K+ = (Y_{l,-m} + (-1)^l conj Y_{lm}) / 2,  Kx = i (Y_{l,-m} - (-1)^l conj Y_{lm}) / 2
        double ar, ai, br, bi;
        swsh_m2(l, -m, s.iota, s.phiref, ar, ai);
        swsh_m2(l, m, s.iota, s.phiref, br, bi);
        bi = -bi;
        const double sg = (l & 1) ? -1.0 : 1.0;
        b.kp[0] = 0.5 * (ar + sg * br);
        b.kp[1] = 0.5 * (ai + sg * bi);
        const double dr = ar - sg * br, di = ai - sg * bi;
        b.kc[0] = -0.5 * di;
        b.kc[1] = 0.5 * dr;
    }
    if ((threadIdx.x & (kRootLanes - 1)) == 0) band[id] = b;
}

// ---------------------------------------------------------------------------
// Kernel 3: knots and A_lm, phi_lm, t_lm at every knot; one thread per
// (walker, mode, knot).  Knots are log-spaced on [f_start, f_end].
// ---------------------------------------------------------------------------
__global__ void k_knots(int B, Modes md, GridDesc g, const Source *__restrict__ src,
                        const ModeBand *__restrict__ band, double *__restrict__ kf, double *__restrict__ kt,
                        double *__restrict__ fn)
{
    const int ns = g.ns;
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (long long)B * md.nm * ns) return;
    const int j = (int)(id % ns);
    const int wm = (int)(id / ns);
    const int w = wm / md.nm, im = wm - w * md.nm;
    const ModeBand b = band[wm];
    double *fnm = fn + (size_t)wm * kNumFn * ns;
    if (!b.active) {
        kf[id] = 0.0;
        kt[id] = 0.0;
        for (int q = 0; q < kNumFn; ++q) fnm[q * ns + j] = 0.0;
        return;
    }
    double f;
    if (j == 0) f = b.fs;
    else if (j == ns - 1) f = b.fe;
    else {
        const double la = log(b.fs), lb = log(b.fe);
        f = exp(la + (lb - la) * ((double)j / (double)(ns - 1)));
    }
    const Source s = src[w];
    double A, ph, dph;
    mode_at(s, md.l[im], md.m[im], f, A, ph, dph);
    kf[id] = f;
    kt[id] = s.tcoal - dph / kTwoPi;
    fnm[0 * ns + j] = A;
    fnm[1 * ns + j] = ph;
}

}  // namespace

const void *source_kernel() { return reinterpret_cast<const void *>(&k_source); }

hipError_t launch_waveform(const double *params, int B, const Modes &md, const GridDesc &g, const Work &wk,
                           hipStream_t st)
{
    if (B <= 0) return hipSuccess;
    // kRootLanes lanes per walker and per (walker, mode)
    constexpr int kPerBlock = 64 / kRootLanes;
    k_source<<<(unsigned)((B + 2 * kPerBlock - 1) / (2 * kPerBlock)), 128, 0, st>>>(params, B, g.t0, wk.src);
    const int nb = B * md.nm;
    k_bands<<<(unsigned)((nb + kPerBlock - 1) / kPerBlock), 64, 0, st>>>(B, md, g, wk.src, wk.band);
    const long long nk = (long long)nb * g.ns;
    k_knots<<<(unsigned)((nk + 255) / 256), 256, 0, st>>>(B, md, g, wk.src, wk.band, wk.kf, wk.kt, wk.fn);
    return hipGetLastError();
}

}  // namespace mbh
