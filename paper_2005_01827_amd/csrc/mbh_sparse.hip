// Sparse stage on the GPU (rows a1-a5): per-walker constants, each mode's
// frequency band, its knots, the LISA response at the knots and the spline
// coefficients.  Each step is one device function; the staged entry points
// run them as separate kernels (k_source, k_bands, k_knots, k_response,
// k_spline), and k_sparse runs all of them for one (walker, mode) in one
// workgroup.  Both call the same functions, so they write the same bits.
//
// Waveform (Sec. II: the 11 parameters, harmonic
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
//
// Response (Sec. II, Eq. response; TDI A = (Z-X)/sqrt2, E = (X-2Y+Z)/sqrt6,
// T = (X+Y+Z)/sqrt3).  The paper cites Marsat & Baker (2018) for the
// transfer function; this is the project's first-principles version of it:
// a rigid equilateral triangle (arm L = 2.5e9 m, plane tilted 60 degrees)
// whose centre moves on a circular 1 AU orbit, evaluated at the mode's own
// time t_lm(f).  The link s -> r, unit vector n, responds to a plane wave of
// direction k and polarization tensor P with
//   G_rs = -i pi f L sinc(pi f L (1 - k.n)) exp(-i pi f (L + k.(x_s + x_r))) n.P.n
// (x_i: spacecraft offsets from the centre; the common delay
// exp(-2 pi i f k.p0) is moved into the phase so that the splined functions
// stay slowly varying).  First-generation Michelson combinations with the
// delay z = exp(-2 pi i f L):
//   X = (1 - z^2) [(y12 + z y21) - (y13 + z y31)],  Y, Z cyclically.
//
// Spline setup (Sec. II.A): not-a-knot cubic splines of the eight real
// functions of each mode (A, phi, Re/Im T^A, T^E, T^T) over the log-spaced
// knots, by parallel cyclic reduction of the second-derivative system.
#include <type_traits>
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
constexpr double kPiPowM16 = 0x1.a711c663294aap-1;   // pi^(-1/6), the double nearest

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

// d/df ln(f^2 A_22) in v and its own f-derivative in dv
__device__ void dlog_f2amp(const Source &s, double f, double &v, double &dv)
{
    const double u = (f - s.fRD) / s.fd;
    const double lor = 1.0 / (1.0 + u * u);
    const double lg = 1.0 / (1.0 + exp(u));          // logistic cut-off
    const double tail = 1.0 - lg;
    const double dlor = -2.0 * u * lor * lor / s.fd;
    const double den = 1.0 + kLorentzHeight * lor;
    v = 5.0 / (6.0 * f) + kLorentzHeight * dlor / den - tail / s.fd;
    const double ddlor = -2.0 / s.fd * (lor * lor / s.fd + 2.0 * u * lor * dlor);
    dv = -5.0 / (6.0 * f * f) + kLorentzHeight * (ddlor * den - kLorentzHeight * dlor * dlor) / (den * den) -
         tail * lg / (s.fd * s.fd);
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

// t_lm(f) and its f-derivative (the second phase derivative of the (2,2)
// mode at 2f/m, scaled); the value is formed exactly as the root search of
// f_start needs it.
__device__ void mode_time(const Source &s, int l, int m, double f, double &t, double &dt)
{
    const double ft = 2.0 * f / m;
    double p, a, b;
    phase22_raw(s, ft, p, a, b);
    t = s.tcoal - (a - s.al1) / kTwoPi;
    dt = -(2.0 / m) * b / kTwoPi;
}

// ---------------------------------------------------------------------------
// Roots by one whole wavefront.  g(x, v, d) sets v = g(x) and d = g'(x) of a
// function that rises through its root; the predicate is g >= 0.  Every lane
// of the wavefront calls wave_root together with the same lo and hi.
//
// The first round evaluates both ends (lanes 0 and 63) and 62 points between
// them, log-spaced over a range wider than a factor 2 and evenly spaced
// otherwise, and returns the end values in glo and ghi.  Only if
// g(lo) < 0 <= g(hi) does the search go on: each later round keeps the
// bracket [lo, hi] with the values and slopes at both ends, and samples
//   - 48 lanes evenly over a window about the two Newton steps from the ends,
//     twice as wide as their spread, when that window is under an eighth of
//     the bracket (near the root the steps straddle it and their spread
//     shrinks quadratically), with 16 lanes evenly over the bracket, the last
//     at hi;
//   - else 64 lanes evenly over the bracket, the last at hi.
// The new bracket is the smallest sample where the predicate holds and the
// largest sample below it where it does not.  The search stops once no
// sample lies strictly inside, i.e. lo and hi are adjacent doubles (the even
// lanes reach every gap of fewer than 16 doubles).  For a predicate that
// switches once this is the pair that repeated halving ends on.  Each round
// divides the bracket by at least 16; near the root the window cuts it by
// far more, so a root takes about 5 rounds where even sampling took 11.
// ---------------------------------------------------------------------------
constexpr int kRootLanes = 64;                 // a root search occupies one wavefront
constexpr int kRootWindow = 48;                // window lanes of a guided round

// v of lane j (j the same in every lane)
__device__ __forceinline__ double lane_value(double v, int j)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, j);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), j);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// The point of lane 'lane' in wave_root's first round over [lo, hi].
__device__ __forceinline__ double wave_root_point(double lo, double hi, int lane)
{
    const bool wide = lo > 0.0 && hi > 2.0 * lo;
    const double L = wide ? log(hi / lo) : 0.0;
    const double t = (double)lane * (1.0 / 63.0);
    return lane == 0 ? lo : lane == 63 ? hi : wide ? lo * exp(L * t) : fma(hi - lo, t, lo);
}

// g0 serves the first round (it may return values formed ahead of time for
// the points of wave_root_point), g every later one.
template <typename F, typename F0>
__device__ void wave_root(double &lo, double &hi, double &glo, double &ghi, F g, F0 g0)
{
    typedef unsigned long long lanes_t;
    const int lane = threadIdx.x & 63;
    double x = wave_root_point(lo, hi, lane), v = 0.0, d = 0.0;
    const bool in0 = lane == 0 || lane == 63 || (x > lo && x < hi);
    if (in0) g0(x, v, d);
    glo = lane_value(v, 0);
    ghi = lane_value(v, 63);
    if (!(glo < 0.0 && ghi >= 0.0)) return;
    // lanes are in increasing x: the first hit, and the last miss before it
    double gl, dl, gh, dh;
    {
        const bool hit = lane == 63 || (in0 && lane > 0 && v >= 0.0);
        const int jh = __ffsll((lanes_t)__ballot(hit)) - 1;
        const lanes_t miss = (lanes_t)__ballot(lane == 0 || (in0 && !(v >= 0.0))) & ((1ull << jh) - 1ull);
        const int jl = 63 - __clzll(miss);
        lo = lane_value(x, jl);
        gl = lane_value(v, jl);
        dl = lane_value(d, jl);
        hi = lane_value(x, jh);
        gh = lane_value(v, jh);
        dh = lane_value(d, jh);
    }
    for (int round = 0; round < 80; ++round) {
        const double W = hi - lo;
        const double xa = dl > 0.0 ? lo - gl / dl : hi;
        const double xb = dh > 0.0 ? hi - gh / dh : lo;
        const double a = fmin(xa, xb), b = fmax(xa, xb);
        const double c = 0.5 * (a + b);
        const double hw = 2.0 * (b - a) + 0x1p-50 * fabs(c);
        const bool win = hw < 0.125 * W && c > lo && c < hi;       // false for a NaN
        const lanes_t wmask = win ? (1ull << kRootWindow) - 1ull : 0ull;
        if (win && lane < kRootWindow) {
            x = fma(hw, (double)(2 * lane + 1 - kRootWindow) * (1.0 / (kRootWindow + 1)), c);
        } else {
            const int j = win ? lane - kRootWindow : lane;
            const int last = win ? 63 - kRootWindow : 63;
            x = j < last ? fma(W, (double)(j + 1) * (win ? 1.0 / (64 - kRootWindow) : 1.0 / 64), lo) : hi;
        }
        const bool inside = x > lo && x < hi;
        if ((lanes_t)__ballot(inside) == 0ull) break;               // lo and hi are adjacent
        v = 0.0;
        d = 0.0;
        if (inside) g(x, v, d);
        const bool hit = inside && v >= 0.0;
        // each part (window, even) is sorted: its first hit and last miss
        const lanes_t hm = (lanes_t)__ballot(hit);
        int jh = -1;
        double nh = hi;
        if (hm & wmask) {
            const int j = __ffsll(hm & wmask) - 1;
            const double xj = lane_value(x, j);
            if (xj < nh) { nh = xj; jh = j; }
        }
        if (hm & ~wmask) {
            const int j = __ffsll(hm & ~wmask) - 1;
            const double xj = lane_value(x, j);
            if (xj < nh) { nh = xj; jh = j; }
        }
        if (jh >= 0) {
            hi = nh;
            gh = lane_value(v, jh);
            dh = lane_value(d, jh);
        }
        const lanes_t mm = (lanes_t)__ballot(inside && !hit && x < hi);
        int jl = -1;
        double nl = lo;
        if (mm & wmask) {
            const int j = 63 - __clzll(mm & wmask);
            const double xj = lane_value(x, j);
            if (xj > nl) { nl = xj; jl = j; }
        }
        if (mm & ~wmask) {
            const int j = 63 - __clzll(mm & ~wmask);
            const double xj = lane_value(x, j);
            if (xj > nl) { nl = xj; jl = j; }
        }
        if (jl >= 0) {
            lo = nl;
            gl = lane_value(v, jl);
            dl = lane_value(d, jl);
        }
    }
}

template <typename F>
__device__ void wave_root(double &lo, double &hi, double &glo, double &ghi, F g)
{
    wave_root(lo, hi, glo, ghi, g, g);
}

// ---------------------------------------------------------------------------
// Per-walker constants (a1) from the 11 parameters at p, all but f_peak and
// the alignment there (source_of adds those).
// ---------------------------------------------------------------------------
__device__ __forceinline__ Source source_consts(const double *__restrict__ p, double t0)
{
    Source s;
    for (int i = 0; i < (int)(sizeof(Source) / sizeof(double)); ++i) reinterpret_cast<double *>(&s)[i] = 0.0;
    s.valid = params_ok(p) ? 1 : 0;
    if (!s.valid) return s;
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
    {
        // propagation direction and polarization basis of the response
        double sl, cl, sb, cb, sp, cp;
        sincos(s.lam, &sl, &cl);
        sincos(s.beta, &sb, &cb);
        sincos(s.psi, &sp, &cp);
        const double u[3] = {sl, -cl, 0.0};
        const double v[3] = {-sb * cl, -sb * sl, cb};
        s.kv[0] = -cb * cl;
        s.kv[1] = -cb * sl;
        s.kv[2] = -sb;
        for (int i = 0; i < 3; ++i) {
            s.ep[i] = cp * u[i] + sp * v[i];
            s.eq[i] = -sp * u[i] + cp * v[i];
        }
    }

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
    return s;
}

// ---------------------------------------------------------------------------
// Per-walker constants (a1 and the alignment at f_peak), from the 11
// parameters at p.  Called by a whole wavefront, whose lanes share
// the root search for f_peak; every lane returns the same value.
// ---------------------------------------------------------------------------
__device__ __forceinline__ Source source_of(const double *__restrict__ p, double t0)
{
    Source s = source_consts(p, t0);
    if (!s.valid) return s;
    const double eta = s.eta;
    // f_peak: root of d ln(f^2 A_22)/df on [f_J, f_RD], bracketed to adjacent
    // doubles (the root search takes g = -d ln(f^2 A_22)/df, which rises)
    double lo = s.fJ, hi = s.fRD, glo, ghi, fp;
    wave_root(lo, hi, glo, ghi, [&](double x, double &v, double &dv) {
        dlog_f2amp(s, x, v, dv);
        v = -v;
        dv = -dv;
    });
    if (glo >= 0.0) fp = s.fJ;                     // the slope is already <= 0 at f_J
    else if (ghi <= 0.0) fp = s.fRD;               // still >= 0 at f_RD
    else fp = 0.5 * (lo + hi);
    s.fpeak = fp;
    double a, b, c;
    phase22_raw(s, fp, a, b, c);
    s.al0 = a;
    s.al1 = b;
    s.A0 = sqrt(2.0 * eta / 3.0) * kPiPowM16 * s.M * s.M / s.Dl;
    return s;
}

// Kernel 1: one wavefront per walker (its lane 0 writes).
__global__ __launch_bounds__(128) void k_source(const double *__restrict__ params, int B, double t0, Source *__restrict__ out)
{
    const int w = (blockIdx.x * blockDim.x + threadIdx.x) / kRootLanes;
    const bool writer = (threadIdx.x & (kRootLanes - 1)) == 0;
    if (w >= B) return;                            // whole wavefronts leave together
    const Source s = source_of(params + 11 * (size_t)w, t0);
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
// Frequency support of mode (l, m) (a3), called by a whole wavefront; the
// weights are left zero.  f_start is the root of t_lm(f) = 0, bracketed to
// adjacent doubles; f_end = min(band end, (m/2) 0.2 / M).
// ---------------------------------------------------------------------------
__device__ __forceinline__ ModeBand band_support(const Source &s, int l, int m, const GridDesc &g,
                                                 const double *pre = nullptr)
{
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
            double lo = f_lo, hi = fe, glo, ghi;
            const auto g1 = [&](double x, double &t, double &dt) { mode_time(s, l, m, x, t, dt); };
            if (pre) {
                // first round from band_first_round: d phi_22/df and its
                // derivative at the round's points, aligned here as mode_time does
                const int lane = threadIdx.x & 63;
                wave_root(lo, hi, glo, ghi, g1, [&](double, double &t, double &dt) {
                    t = s.tcoal - (pre[lane] - s.al1) / kTwoPi;
                    dt = -(2.0 / m) * pre[kRootLanes + lane] / kTwoPi;
                });
            } else {
                wave_root(lo, hi, glo, ghi, g1);
            }
            if (glo >= 0.0) fs = f_lo;                 // the mode starts before the band
            else if (ghi < 0.0) have = false;          // ... or only after its end
            else fs = hi;
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
    }
    return b;
}

// The first round of band_support's f_start search for a mode of order m, ahead of
// the alignment at f_peak (which it does not need): d phi_22/df and its
// derivative at 2f/m for the round's points f, into pre[lane] and
// pre[kRootLanes + lane].  Called by a whole wavefront with the walker's
// constants (source_consts); the same bits as mode_time forms there.
__device__ __forceinline__ void band_first_round(const Source &s, int m, const GridDesc &g, double *pre)
{
    if (!s.valid) return;
    const double f_lo = (double)g.k0 * g.df;
    const double f_hi = (double)(g.k0 + g.n - 1) * g.df;
    const double fe = fmin(0.5 * m * kMfCut / s.M, f_hi);
    if (!(fe > f_lo)) return;
    const int lane = threadIdx.x & 63;
    const double x = wave_root_point(f_lo, fe, lane);
    double p = 0.0, a = 0.0, b = 0.0;
    if (lane == 0 || lane == 63 || (x > f_lo && x < fe)) phase22_raw(s, 2.0 * x / m, p, a, b);
    pre[lane] = a;
    pre[kRootLanes + lane] = b;
}

// Plus and cross weights of mode (l, m) (complex, re and im), which depend
// only on the inclination and phi_ref:
//   K+ = (Y_{l,-m} + (-1)^l conj Y_{lm}) / 2,  Kx = i (Y_{l,-m} - (-1)^l conj Y_{lm}) / 2.
__device__ void mode_weights(int l, int m, double iota, double phiref, double (&kp)[2], double (&kc)[2])
{
    double ar, ai, br, bi;
    swsh_m2(l, -m, iota, phiref, ar, ai);
    swsh_m2(l, m, iota, phiref, br, bi);
    bi = -bi;
    const double sg = (l & 1) ? -1.0 : 1.0;
    kp[0] = 0.5 * (ar + sg * br);
    kp[1] = 0.5 * (ai + sg * bi);
    const double dr = ar - sg * br, di = ai - sg * bi;
    kc[0] = -0.5 * di;
    kc[1] = 0.5 * dr;
}

// Band and weights of mode (l, m) (a3), by one wavefront.
__device__ __forceinline__ ModeBand band_of(const Source &s, int l, int m, const GridDesc &g)
{
    ModeBand b = band_support(s, l, m, g);
    if (s.valid) mode_weights(l, m, s.iota, s.phiref, b.kp, b.kc);
    return b;
}

// Kernel 2: one wavefront per (walker, mode).
__global__ __launch_bounds__(64) void k_bands(int B, Modes md, GridDesc g, const Source *__restrict__ src, ModeBand *__restrict__ band)
{
    const int id = (blockIdx.x * blockDim.x + threadIdx.x) / kRootLanes;
    if (id >= B * md.nm) return;                   // whole wavefronts leave together
    const int w = id / md.nm, im = id - w * md.nm;
    const Source s = src[w];
    const ModeBand b = band_of(s, md.l[im], md.m[im], g);
    if ((threadIdx.x & (kRootLanes - 1)) == 0) band[id] = b;
}

// ---------------------------------------------------------------------------
// Knot j of an active band (a2): knots are log-spaced on [f_start, f_end];
// A_lm, phi_lm and t_lm there.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void knot_of(const Source &s, const ModeBand &b, int l, int m, int j, int ns, double &f,
                                        double &t, double &A, double &ph)
{
    if (j == 0) f = b.fs;
    else if (j == ns - 1) f = b.fe;
    else {
        const double la = log(b.fs), lb = log(b.fe);
        f = exp(la + (lb - la) * ((double)j / (double)(ns - 1)));
    }
    double dph;
    mode_at(s, l, m, f, A, ph, dph);
    t = s.tcoal - dph / kTwoPi;
}

// Kernel 3: one thread per (walker, mode, knot).
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
    const Source s = src[w];
    double f, t, A, ph;
    knot_of(s, b, md.l[im], md.m[im], j, ns, f, t, A, ph);
    kf[id] = f;
    kt[id] = t;
    fnm[0 * ns + j] = A;
    fnm[1 * ns + j] = ph;
}

// ---------------------------------------------------------------------------
// Response (a4).
// ---------------------------------------------------------------------------

constexpr double kArmSec = 2.5e9 / 299792458.0;                 // L / c
constexpr double kAuSec = 1.495978707e11 / 299792458.0;         // 1 AU / c
constexpr double kYearSec = 3.15576e7;

struct Cplx {
    double re, im;
};
__device__ inline Cplx cmul(Cplx a, Cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline Cplx cadd(Cplx a, Cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ inline Cplx csub(Cplx a, Cplx b) { return {a.re - b.re, a.im - b.im}; }
__device__ inline Cplx cscale(Cplx a, double s) { return {a.re * s, a.im * s}; }

__device__ inline double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// T^{A,E,T} of mode band b at frequency f and time t, and the total phase:
// r[0] = ph - 2 pi f t_coal + (orbital delay phase), r[1..6] = Re/Im T^A,
// T^E, T^T.
__device__ __forceinline__ void response_at(const Source &s, const ModeBand &b, double f, double t, double ph,
                                            double (&r)[7])
{
    // propagation direction and polarization basis (per walker, from the source)
    const double *k = s.kv, *ep = s.ep, *eq = s.eq;

    // constellation at time t (light-seconds): spacecraft i at ring phase
    // b_i = 2 pi i / 3, whose cos(2 al - b_i), sin(2 al - b_i) and
    // cos(al - b_i) follow from al and 2 al by the addition formulas
    const double al = kTwoPi * t / kYearSec;
    double sa, ca;
    sincos(al, &sa, &ca);
    const double p0[3] = {kAuSec * ca, kAuSec * sa, 0.0};
    const double c2a = (ca - sa) * (ca + sa), s2a = 2.0 * sa * ca;
    const double eR = kArmSec / (2.0 * 1.7320508075688772935);   // e R = L / (2 sqrt3)
    const double cbv[3] = {1.0, -0.5, -0.5};
    const double sbv[3] = {0.0, 0.86602540378443864676, -0.86602540378443864676};
    double x[3][3];
    for (int i = 0; i < 3; ++i) {
        const double c2 = c2a * cbv[i] + s2a * sbv[i];
        const double s2 = s2a * cbv[i] - c2a * sbv[i];
        const double c1 = ca * cbv[i] + sa * sbv[i];
        x[i][0] = eR * (0.5 * c2 - 1.5 * cbv[i]);
        x[i][1] = eR * (0.5 * s2 - 1.5 * sbv[i]);
        x[i][2] = -eR * 1.7320508075688772935 * c1;
    }

    const Cplx kp = {b.kp[0], b.kp[1]}, kc = {b.kc[0], b.kc[1]};
    const double pfL = kPi * f * kArmSec;

    // y[r][s]: link s -> r
    Cplx y[3][3];
    for (int r = 0; r < 3; ++r) {
        y[r][r] = {0.0, 0.0};
        for (int q = 0; q < 3; ++q) {
            if (q == r) continue;
            double n[3], xs[3];
            for (int i = 0; i < 3; ++i) {
                n[i] = (x[r][i] - x[q][i]) / kArmSec;
                xs[i] = x[q][i] + x[r][i];
            }
            const double np = dot3(n, ep), nq = dot3(n, eq);
            const Cplx nPn = cadd(cscale(kp, np * np - nq * nq), cscale(kc, 2.0 * np * nq));
            const double arg = pfL * (1.0 - dot3(k, n));
            const double sinc = (arg == 0.0) ? 1.0 : sin(arg) / arg;
            double sph, cph;
            sincos(-kPi * f * (kArmSec + dot3(k, xs)), &sph, &cph);
            // -i pfL sinc e^{i ph}
            const Cplx pre = {pfL * sinc * sph, -pfL * sinc * cph};
            y[r][q] = cmul(pre, nPn);
        }
    }
    double sz, cz;
    sincos(-kTwoPi * f * kArmSec, &sz, &cz);
    const Cplx z = {cz, sz};
    const Cplx z2 = cmul(z, z);
    const Cplx omz2 = {1.0 - z2.re, -z2.im};
    Cplx xyz[3];
    for (int c = 0; c < 3; ++c) {
        const int a = c, bb = (c + 1) % 3, d = (c + 2) % 3;
        const Cplx arm1 = cadd(y[a][bb], cmul(z, y[bb][a]));
        const Cplx arm2 = cadd(y[a][d], cmul(z, y[d][a]));
        xyz[c] = cmul(omz2, csub(arm1, arm2));
    }
    const double r2 = 1.4142135623730950488, r6 = 2.4494897427831780982, r3 = 1.7320508075688772935;
    const Cplx TA = cscale(csub(xyz[2], xyz[0]), 1.0 / r2);
    const Cplx TE = cscale(cadd(csub(xyz[0], cscale(xyz[1], 2.0)), xyz[2]), 1.0 / r6);
    const Cplx TT = cscale(cadd(cadd(xyz[0], xyz[1]), xyz[2]), 1.0 / r3);
    const double phorb = -kTwoPi * f * dot3(k, p0);
    r[0] = ph - kTwoPi * f * s.tcoal + phorb;
    r[1] = TA.re;
    r[2] = TA.im;
    r[3] = TE.re;
    r[4] = TE.im;
    r[5] = TT.re;
    r[6] = TT.im;
}

// Kernel 4: one thread per (walker, mode, knot).
__global__ __launch_bounds__(128) void k_response(int B, Modes md, GridDesc g, const Source *__restrict__ src,
                           const ModeBand *__restrict__ band, const double *__restrict__ kf,
                           const double *__restrict__ kt, double *__restrict__ fn)
{
    const int ns = g.ns;
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (long long)B * md.nm * ns) return;
    const int j = (int)(id % ns);
    const int wm = (int)(id / ns);
    const int w = wm / md.nm;
    const ModeBand b = band[wm];
    if (!b.active) return;
    const Source s = src[w];
    double *fnm = fn + (size_t)wm * kNumFn * ns;
    double r[7];
    response_at(s, b, kf[id], kt[id], fnm[1 * ns + j], r);
    for (int q = 0; q < 7; ++q) fnm[(q + 1) * ns + j] = r[q];
}

// ---------------------------------------------------------------------------
// Spline setup (a5).
// ---------------------------------------------------------------------------

// First dense bin k with k df >= x (|x/df| < 2^31): the ceiling of the
// rounded quotient is within one of it, so one correction each way is exact.
__device__ __forceinline__ int first_bin(double x, double df)
{
    long long k = (long long)ceil(x / df);
    if ((double)k * df < x) ++k;
    if ((double)(k - 1) * df >= x) --k;
    return (int)max(-1LL, min(k, 0x7ffffffeLL));
}

constexpr int kSplineThreads = 256;
constexpr int kThomasRows = 16;    // rows per interleaved system left for the Thomas sweeps
constexpr int kSplineRows = 4;     // most rows per thread: ns - 2 <= 1024
constexpr int kCoefChunk = 8;      // coefficient items per thread whose loads are issued together

// LDS of one spline workgroup solving G functions together: the matrix
// (3 m) and the reciprocals of its diagonal (m), G right-hand sides, 2 G end
// values, the knots, the reciprocal interval widths and the knots' first
// dense bins.  Kept 1 KB under 64 KB, which leaves room for the fused
// kernel's static LDS (the walker constants, the band, the item-list band);
// G does not change the arithmetic of any function, only how many share a pass.
constexpr size_t kSplineLdsMax = 65536 - 1024;
__host__ __device__ inline size_t spline_lds_for(int ns, int G)
{
    const size_t m = (size_t)ns - 2;
    return sizeof(double) * ((4 + G) * m + 2 * G + ns + (ns - 1)) + sizeof(int) * ns;
}
// Functions solved together: the most of 8, 4, 2, 1 that fit in LDS (all
// eight up to 512 knots, one at 1024).
__host__ __device__ inline int spline_group(int ns)
{
    int G = kNumFn;
    while (G > 1 && spline_lds_for(ns, G) > kSplineLdsMax) G /= 2;
    return G;
}
inline size_t spline_lds_bytes(int ns) { return spline_lds_for(ns, spline_group(ns)); }
// Rows per thread of the cyclic reduction (1, 2 or kSplineRows): only as
// many as the ns - 2 rows need, since the rows of a round are held in
// registers across its barrier.
__host__ __device__ inline int spline_rows(int ns)
{
    const int m = ns - 2;
    return m <= kSplineThreads ? 1 : m <= 2 * kSplineThreads ? 2 : kSplineRows;
}

// Not-a-knot splines through (f_j, y_j) of (walker, mode) wm, by one workgroup
// of kSplineThreads threads with sm its dynamic LDS (spline_lds_for(ns, G)).
// Unknowns M_1..M_{ns-2} (second derivatives; row r <-> M_{r+1}); M_0 and
// M_{ns-1} follow from continuity of the third derivative at f_1 and
// f_{ns-2}.  The matrix depends only on the knots, so the eight functions of
// a mode share it; it is strictly diagonally dominant (also the two modified
// end rows), so parallel cyclic reduction is stable: in round k every row
// eliminates its neighbours at distance 2^k, and after ceil(log2(ns-2))
// rounds each row stands alone, M = d / b.  The workgroup also writes
// kbin[i], the first dense bin k with k df >= f_i, so that the dense stage
// finds intervals by integer comparison (bin k lies in interval i iff
// kbin[i] <= k < kbin[i+1], the same as f_i <= k df < f_{i+1}), and stores
// the cubic of interval i re-centred on fc = kbin[i+1] df, the first dense
// bin of the next interval: q(t) = p(t + fc - f_i), evaluated by the dense
// stage at t = f - fc.
template <int G, int R>
__device__ __forceinline__ void spline_solve(int wm, const GridDesc &g, bool act, const double *__restrict__ kf,
                                             const double *__restrict__ fn, double *__restrict__ coef,
                                             int *__restrict__ kbin, double *sm)
{
    const int ns = g.ns, m = ns - 2;
    const double *xg = kf + (size_t)wm * ns;
    double *out = coef + (size_t)wm * (ns - 1) * kCoefPerIv;
    double *A = sm, *Bm = sm + m, *C = sm + 2 * m, *D = sm + 3 * m;   // D[G][m]
    double *M0 = D + (size_t)G * m, *M1 = M0 + G;                       // M_0, M_{ns-1} per function
    double *x = M1 + G, *hinv = x + ns;                                 // knots, 1 / (x[i+1] - x[i])
    double *binv = hinv + (ns - 1);                                     // 1 / b of every row, per round
    int *kbl = reinterpret_cast<int *>(binv + m);                       // first dense bin of each knot
    {
        int *kb = kbin + (size_t)wm * ns;
        for (int i = threadIdx.x; i < ns; i += kSplineThreads) {
            const double xi = xg[i];
            const int k = act ? first_bin(xi, g.df) : 0;
            kb[i] = k;
            kbl[i] = k;
            x[i] = xi;
        }
    }
    if (!act) {
        for (int i = threadIdx.x; i < (ns - 1) * kCoefPerIv; i += kSplineThreads) out[i] = 0.0;
        return;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < ns - 1; i += kSplineThreads) hinv[i] = 1.0 / (x[i + 1] - x[i]);
    __syncthreads();
    for (int q0 = 0; q0 < kNumFn; q0 += G) {
        // the system: matrix rows and right-hand sides 6 (s_{i} - s_{i-1})
        for (int r = threadIdx.x; r < m; r += kSplineThreads) {
            const int i = r + 1;
            const double h0 = x[i] - x[i - 1], h1 = x[i + 1] - x[i];
            double sub = h0, dia = 2.0 * (h0 + h1), sup = h1;
            if (r == 0) {
                dia = (h0 + h1) * (h0 + 2.0 * h1) / h1;
                sup = (h1 * h1 - h0 * h0) / h1;
                sub = 0.0;
            }
            if (r == m - 1) {
                dia = (h0 + h1) * (2.0 * h0 + h1) / h0;
                sub = (h0 * h0 - h1 * h1) / h0;
                sup = 0.0;
            }
            A[r] = sub;
            Bm[r] = dia;
            binv[r] = 1.0 / dia;
            C[r] = sup;
            for (int q = 0; q < G; ++q) {
                const double *y = fn + ((size_t)wm * kNumFn + q0 + q) * ns;
                D[(size_t)q * m + r] = 6.0 * ((y[i + 1] - y[i]) * hinv[i] - (y[i] - y[i - 1]) * hinv[i - 1]);
            }
        }
        __syncthreads();
        // Parallel cyclic reduction until the rows fall into P interleaved
        // systems of at most kThomasRows rows (rows r = c, c + P, c + 2P, ...
        // for c < P; P = 1 solves the whole system by one sweep), then one
        // Thomas sweep per system: first the pivots and the modified upper
        // diagonal, shared by the G functions, then the right-hand sides.
        // Each row's new b is stored with its reciprocal (one division per
        // row instead of one per neighbour).
        int P = 1;
        while (P * kThomasRows < m) P *= 2;
        for (int s = 1; s < P; s *= 2) {
            double na[R], nb[R], nc[R], nd[R][G];
#pragma unroll
            for (int u = 0; u < R; ++u) {
                if (u * kSplineThreads < m) {
                    // neighbour indices clamped into the system, so that every
                    // load of the round is issued at once, with no branch; a
                    // missing neighbour gets a zero factor (rows past m repeat
                    // row m - 1 and are not stored)
                    const int r = min((int)threadIdx.x + u * kSplineThreads, m - 1);
                    const int rl = max(r - s, 0), rh = min(r + s, m - 1);
                    const double Ar = A[r], Cr = C[r], Br = Bm[r];
                    const double bl = binv[rl], bh = binv[rh];
                    const double Al = A[rl], Cl = C[rl], Ah = A[rh], Ch = C[rh];
                    double dr[G], dl[G], dh[G];
#pragma unroll
                    for (int q = 0; q < G; ++q) {
                        const double *dq = D + (size_t)q * m;
                        dr[q] = dq[r];
                        dl[q] = dq[rl];
                        dh[q] = dq[rh];
                    }
                    const double al = r - s >= 0 ? -Ar * bl : 0.0;
                    const double ga = r + s < m ? -Cr * bh : 0.0;
                    na[u] = al * Al;
                    nc[u] = ga * Ch;
                    nb[u] = Br + al * Cl + ga * Ah;
#pragma unroll
                    for (int q = 0; q < G; ++q) nd[u][q] = dr[q] + al * dl[q] + ga * dh[q];
                }
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < R; ++u) {
                const int r = threadIdx.x + u * kSplineThreads;
                if (r < m) {
                    A[r] = na[u];
                    Bm[r] = nb[u];
                    binv[r] = 1.0 / nb[u];
                    C[r] = nc[u];
#pragma unroll
                    for (int q = 0; q < G; ++q) D[(size_t)q * m + r] = nd[u][q];
                }
            }
            __syncthreads();
        }
        // After the rounds with s < P, row r couples only to r - P and r + P,
        // and A[r] = 0 for r < P, C[r] = 0 for r >= m - P.  Forward sweep of
        // system c: pivot 1 / (b - a c'_prev) into binv, c' into C.
        // Each system has at most kThomasRows rows (P kThomasRows >= m); its
        // rows are read into registers first, so that the sweeps wait on no
        // load.
        if ((int)threadIdx.x < P) {
            const int c = threadIdx.x;
            double bv[kThomasRows], av[kThomasRows], cv[kThomasRows];
#pragma unroll
            for (int k = 0; k < kThomasRows; ++k) {
                const int r = min(c + k * P, m - 1);
                bv[k] = Bm[r];
                av[k] = A[r];
                cv[k] = C[r];
            }
            double cp = 0.0;
#pragma unroll
            for (int k = 0; k < kThomasRows; ++k) {
                const int r = c + k * P;
                if (r < m) {
                    const double rd = 1.0 / (bv[k] - av[k] * cp);
                    cp = cv[k] * rd;
                    C[r] = cp;
                    binv[r] = rd;
                }
            }
        }
        __syncthreads();
        // right-hand sides forward, then back substitution: M_{r+1} in D
        for (int t = threadIdx.x; t < P * G; t += kSplineThreads) {
            const int c = t % P, q = t / P;
            double *dq = D + (size_t)q * m;
            const int nr = (m - c + P - 1) / P;            // rows of system c
            double dv[kThomasRows], av[kThomasRows], bi[kThomasRows], cv[kThomasRows];
#pragma unroll
            for (int k = 0; k < kThomasRows; ++k) {
                const int r = min(c + k * P, m - 1);
                dv[k] = dq[r];
                av[k] = A[r];
                bi[k] = binv[r];
                cv[k] = C[r];
            }
            double dp = 0.0;
#pragma unroll
            for (int k = 0; k < kThomasRows; ++k) {
                if (k < nr) {
                    dp = (dv[k] - av[k] * dp) * bi[k];
                    dv[k] = dp;
                }
            }
            double xv = 0.0;                               // the last row keeps its forward value
#pragma unroll
            for (int k = kThomasRows - 1; k >= 0; --k) {
                if (k < nr) {
                    xv = dv[k] - cv[k] * xv;
                    dq[c + k * P] = xv;
                }
            }
        }
        __syncthreads();
        // end values from the not-a-knot conditions
        if (threadIdx.x < G) {
            const double *Mq = D + (size_t)threadIdx.x * m;   // Mq[r] = M_{r+1}
            const double h0 = x[1] - x[0], h1 = x[2] - x[1];
            M0[threadIdx.x] = ((h0 + h1) * Mq[0] - h0 * Mq[1]) / h1;
            const double ha = x[ns - 2] - x[ns - 3], hb = x[ns - 1] - x[ns - 2];
            M1[threadIdx.x] = ((ha + hb) * Mq[m - 1] - hb * Mq[m - 2]) / ha;
        }
        __syncthreads();
        // coefficients of interval i from knots i, i+1, re-centred on fc, one
        // (interval, function) item per thread and pass (the function index
        // fastest, so that a wavefront's stores are contiguous); every load
        // of a thread's kCoefChunk items is issued before the first is used
        const int nt = (ns - 1) * G;
        for (int t0 = 0; t0 < nt; t0 += kCoefChunk * kSplineThreads) {
            double ya[kCoefChunk], yb[kCoefChunk], mi[kCoefChunk], mj[kCoefChunk];
            double xa[kCoefChunk], xb[kCoefChunk], hv[kCoefChunk];
            int kb[kCoefChunk];
#pragma unroll
            for (int k = 0; k < kCoefChunk; ++k) {
                const int t = min(t0 + (int)threadIdx.x + k * kSplineThreads, nt - 1);
                const int i = t / G, q = t % G;
                const double *y = fn + ((size_t)wm * kNumFn + q0 + q) * ns;
                const double *Mq = D + (size_t)q * m;
                ya[k] = y[i];
                yb[k] = y[i + 1];
                mi[k] = i == 0 ? M0[q] : Mq[max(i - 1, 0)];
                mj[k] = i + 1 == ns - 1 ? M1[q] : Mq[min(i, m - 1)];
                xa[k] = x[i];
                xb[k] = x[i + 1];
                hv[k] = hinv[i];
                kb[k] = kbl[i + 1];
            }
#pragma unroll
            for (int k = 0; k < kCoefChunk; ++k) {
                const int t = t0 + (int)threadIdx.x + k * kSplineThreads;
                if (t < nt) {
                    const int i = t / G, q = t % G;
                    const double h = xb[k] - xa[k], hi = hv[k];
                    const double sl = (yb[k] - ya[k]) * hi;
                    const double p0 = ya[k], p1 = sl - h * (1.0 / 6.0) * (2.0 * mi[k] + mj[k]), p2 = 0.5 * mi[k];
                    const double p3 = (mj[k] - mi[k]) * hi * (1.0 / 6.0);
                    const double dl = (double)kb[k] * g.df - xa[k];
                    double *o = out + (size_t)i * kCoefPerIv + (q0 + q) * 4;
                    o[0] = fma(fma(fma(p3, dl, p2), dl, p1), dl, p0);
                    o[1] = fma(fma(3.0 * p3, dl, 2.0 * p2), dl, p1);
                    o[2] = fma(3.0 * p3, dl, p2);
                    o[3] = p3;
                }
            }
        }
        __syncthreads();
    }
}

// Kernel 5: one workgroup per (walker, mode).
template <int G, int R>
__global__ __launch_bounds__(kSplineThreads) void k_spline(int B, Modes md, GridDesc g,
                                                           const ModeBand *__restrict__ band,
                                                           const double *__restrict__ kf,
                                                           const double *__restrict__ fn,
                                                           double *__restrict__ coef, int *__restrict__ kbin)
{
    extern __shared__ double sm[];
    const int wm = blockIdx.x;
    if (wm >= B * md.nm) return;
    spline_solve<G, R>(wm, g, band[wm].active != 0, kf, fn, coef, kbin, sm);
}

// ---------------------------------------------------------------------------
// The whole sparse stage of one (walker, mode) in one workgroup: the
// walker's constants (each of its mode workgroups computes them, wavefront
// 0) and the mode's weights (wavefront 1) at once, the mode's band
// (wavefront 0), its knots and the response there (one thread per knot, with
// no round trip through memory between the two) and the spline.  With
// a.ticket set, workgroup 0 also zeroes the dense stage's item counter.
// ---------------------------------------------------------------------------
template <int G, int R>
__global__ __launch_bounds__(kSplineThreads) void k_sparse(const double *__restrict__ params, int B, Modes md,
                                                           GridDesc g, SparseArgs a)
{
    extern __shared__ double sm[];
    __shared__ Source ss;
    __shared__ ModeBand sb;
    __shared__ double swt[4];                      // the mode's K+ and Kx
    __shared__ double spre[2 * kRootLanes];        // first round of the f_start search
    const int wm = blockIdx.x;
    if (wm >= B * md.nm) return;                   // whole workgroups leave together
    const int w = wm / md.nm, im = wm - w * md.nm;
    const int l = md.l[im], m = md.m[im], ns = g.ns;
    if (threadIdx.x < kRootLanes) {
        const Source s = source_of(params + 11 * (size_t)w, g.t0);
        if (threadIdx.x == 0) {
            ss = s;
            if (im == 0) a.src[w] = s;
        }
    } else if (threadIdx.x < 2 * kRootLanes) {
        // the mode's weights need only the inclination and phi_ref: the
        // second wavefront forms them while the first finds f_peak and f_start
        double kp[2], kc[2];
        mode_weights(l, m, params[11 * (size_t)w + 6], params[11 * (size_t)w + 5], kp, kc);
        if (threadIdx.x == kRootLanes) {
            swt[0] = kp[0];
            swt[1] = kp[1];
            swt[2] = kc[0];
            swt[3] = kc[1];
        }
        // then the first round of the mode's f_start search, which needs
        // every walker constant but the alignment at f_peak
        band_first_round(source_consts(params + 11 * (size_t)w, g.t0), m, g, spre);
    }
    __syncthreads();
    if (threadIdx.x < kRootLanes) {
        ModeBand b = band_support(ss, l, m, g, spre);
        if (ss.valid) {
            b.kp[0] = swt[0];
            b.kp[1] = swt[1];
            b.kc[0] = swt[2];
            b.kc[1] = swt[3];
        }
        if (threadIdx.x == 0) {
            sb = b;
            a.band[wm] = b;
        }
    }
    __syncthreads();
    if (a.ticket && wm == 0 && threadIdx.x == 0) *a.ticket = 0;
    // the knots read the walker's constants and the band from LDS as needed
    const ModeBand &b = sb;
    double *fnm = a.fn + (size_t)wm * kNumFn * ns;
    for (int j = threadIdx.x; j < ns; j += kSplineThreads) {
        const size_t id = (size_t)wm * ns + j;
        if (!b.active) {
            a.kf[id] = 0.0;
            a.kt[id] = 0.0;
            for (int q = 0; q < kNumFn; ++q) fnm[q * ns + j] = 0.0;
            continue;
        }
        double f, t, A, ph, r[7];
        knot_of(ss, b, l, m, j, ns, f, t, A, ph);
        response_at(ss, b, f, t, ph, r);
        a.kf[id] = f;
        a.kt[id] = t;
        fnm[0 * ns + j] = A;
        for (int q = 0; q < 7; ++q) fnm[(q + 1) * ns + j] = r[q];
    }
    __syncthreads();
    spline_solve<G, R>(wm, g, b.active != 0, a.kf, a.fn, a.coef, a.kbin, sm);
}

}  // namespace

const void *source_kernel() { return reinterpret_cast<const void *>(&k_source); }

// f(G, R) with G and R as compile-time constants, for the shapes the knot
// counts can take: all eight functions together whenever they fit (up to
// about 540 knots, so up to 4 rows per thread), fewer only with more than
// 512 rows (4 rows per thread).  Returns false for any other pair.
template <typename F>
bool with_spline_shape(int ns, F f)
{
    const int G = spline_group(ns), R = spline_rows(ns);
    using std::integral_constant;
    if (G == kNumFn && R == 1) return f(integral_constant<int, kNumFn>(), integral_constant<int, 1>()), true;
    if (G == kNumFn && R == 2) return f(integral_constant<int, kNumFn>(), integral_constant<int, 2>()), true;
    if (G == kNumFn && R == kSplineRows)
        return f(integral_constant<int, kNumFn>(), integral_constant<int, kSplineRows>()), true;
    if (G == kNumFn / 2 && R == kSplineRows)
        return f(integral_constant<int, kNumFn / 2>(), integral_constant<int, kSplineRows>()), true;
    if (G == kNumFn / 4 && R == kSplineRows)
        return f(integral_constant<int, kNumFn / 4>(), integral_constant<int, kSplineRows>()), true;
    if (G == 1 && R == kSplineRows) return f(integral_constant<int, 1>(), integral_constant<int, kSplineRows>()), true;
    return false;
}

const void *sparse_kernel(int ns)
{
    const void *k = nullptr;
    with_spline_shape(ns, [&](auto gc, auto rc) {
        k = reinterpret_cast<const void *>(&k_sparse<decltype(gc)::value, decltype(rc)::value>);
    });
    return k;
}

hipError_t launch_waveform(const double *params, int B, const Modes &md, const GridDesc &g, const Work &wk,
                           hipStream_t st)
{
    if (B <= 0) return hipSuccess;
    // one wavefront per walker and per (walker, mode)
    constexpr int kPerBlock = 64 / kRootLanes;
    k_source<<<(unsigned)((B + 2 * kPerBlock - 1) / (2 * kPerBlock)), 128, 0, st>>>(params, B, g.t0, wk.src);
    const int nb = B * md.nm;
    k_bands<<<(unsigned)((nb + kPerBlock - 1) / kPerBlock), 64, 0, st>>>(B, md, g, wk.src, wk.band);
    const long long nk = (long long)nb * g.ns;
    k_knots<<<(unsigned)((nk + 255) / 256), 256, 0, st>>>(B, md, g, wk.src, wk.band, wk.kf, wk.kt, wk.fn);
    return hipGetLastError();
}

hipError_t launch_response(int B, const Modes &md, const GridDesc &g, const Work &wk, hipStream_t st)
{
    if (B <= 0) return hipSuccess;
    const long long nk = (long long)B * md.nm * g.ns;
    k_response<<<(unsigned)((nk + 127) / 128), 128, 0, st>>>(B, md, g, wk.src, wk.band, wk.kf, wk.kt, wk.fn);
    return hipGetLastError();
}

hipError_t launch_spline(int B, const Modes &md, const GridDesc &g, const Work &wk, hipStream_t st)
{
    if (B <= 0) return hipSuccess;
    const size_t lds = spline_lds_bytes(g.ns);
    const unsigned grid = (unsigned)(B * md.nm);
    if (!with_spline_shape(g.ns, [&](auto gc, auto rc) {
            k_spline<decltype(gc)::value, decltype(rc)::value>
                <<<grid, kSplineThreads, lds, st>>>(B, md, g, wk.band, wk.kf, wk.fn, wk.coef, wk.kbin);
        }))
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_sparse(const double *params, int B, const Modes &md, const GridDesc &g, const Work &wk,
                         bool reset_ticket, hipStream_t st)
{
    if (B <= 0) return hipSuccess;
    SparseArgs a;
    a.src = wk.src;
    a.band = wk.band;
    a.kf = wk.kf;
    a.kt = wk.kt;
    a.fn = wk.fn;
    a.coef = wk.coef;
    a.kbin = wk.kbin;
    a.ticket = reset_ticket ? wk.ticket : nullptr;
    const size_t lds = spline_lds_bytes(g.ns);
    const unsigned grid = (unsigned)(B * md.nm);
    if (!with_spline_shape(g.ns, [&](auto gc, auto rc) {
            k_sparse<decltype(gc)::value, decltype(rc)::value><<<grid, kSplineThreads, lds, st>>>(params, B, md, g, a);
        }))
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace mbh
