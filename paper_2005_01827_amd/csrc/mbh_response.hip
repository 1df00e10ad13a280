// Fast Fourier-domain LISA response and spline setup on the GPU.
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
// knots, by a Thomas solve of the second-derivative system.
#include <hip/hip_runtime.h>

#include <cmath>

#include "mbh_internal.h"

namespace mbh {
namespace {

constexpr double kPi = 3.141592653589793238462643;
constexpr double kTwoPi = 6.283185307179586476925287;
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

// One thread per (walker, mode, knot): T^{A,E,T} and the total phase.
__global__ void k_response(int B, Modes md, GridDesc g, const Source *__restrict__ src,
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
    const double f = kf[id];
    const double t = kt[id];
    double *fnm = fn + (size_t)wm * kNumFn * ns;

    // propagation direction and polarization basis
    double sl, cl, sb, cb, sp, cp;
    sincos(s.lam, &sl, &cl);
    sincos(s.beta, &sb, &cb);
    sincos(s.psi, &sp, &cp);
    const double k[3] = {-cb * cl, -cb * sl, -sb};
    const double u[3] = {sl, -cl, 0.0};
    const double v[3] = {-sb * cl, -sb * sl, cb};
    double ep[3], eq[3];
    for (int i = 0; i < 3; ++i) {
        ep[i] = cp * u[i] + sp * v[i];
        eq[i] = -sp * u[i] + cp * v[i];
    }

    // constellation at time t (light-seconds)
    const double al = kTwoPi * t / kYearSec;
    double sa, ca;
    sincos(al, &sa, &ca);
    const double p0[3] = {kAuSec * ca, kAuSec * sa, 0.0};
    const double eR = kArmSec / (2.0 * 1.7320508075688772935);   // e R = L / (2 sqrt3)
    double x[3][3];
    for (int i = 0; i < 3; ++i) {
        const double bi = kTwoPi * i / 3.0;
        double s2, c2, s1, c1, sbi, cbi;
        sincos(2.0 * al - bi, &s2, &c2);
        sincos(al - bi, &s1, &c1);
        sincos(bi, &sbi, &cbi);
        x[i][0] = eR * (0.5 * c2 - 1.5 * cbi);
        x[i][1] = eR * (0.5 * s2 - 1.5 * sbi);
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
    fnm[1 * ns + j] = fnm[1 * ns + j] - kTwoPi * f * s.tcoal + phorb;
    fnm[2 * ns + j] = TA.re;
    fnm[3 * ns + j] = TA.im;
    fnm[4 * ns + j] = TE.re;
    fnm[5 * ns + j] = TE.im;
    fnm[6 * ns + j] = TT.re;
    fnm[7 * ns + j] = TT.im;
}

// One thread per (walker, mode, function): not-a-knot spline through
// (f_j, y_j).  Unknowns M_1..M_{ns-2} (second derivatives); M_0 and M_{ns-1}
// follow from continuity of the third derivative at f_1 and f_{ns-2}.
// The Thomas sweep keeps 2*ns doubles per thread in scratch, interleaved
// across threads (element r of thread id at r*nt + id) so that the 64 lanes
// of a wavefront touch consecutive addresses.  Each of the three serial
// sweeps loads kSplineU knots' operands at once and then runs kSplineU steps
// from registers, so a step waits on memory once per kSplineU steps rather
// than once per step.  The kNumFn threads of each (walker, mode) also write
// kbin[i] for i = q mod kNumFn: the first dense bin k with k df >= f_i, so
// that the dense stage can find intervals by integer comparison: bin k lies
// in interval i iff kbin[i] <= k < kbin[i+1], which is the same as
// f_i <= k df < f_{i+1} in double precision.
constexpr int kSplineU = 16;

// First dense bin k with k df >= x (|x/df| < 2^31): the ceiling of the
// rounded quotient is within one of it, so one correction each way is exact.
__device__ __forceinline__ int first_bin(double x, double df)
{
    long long k = (long long)ceil(x / df);
    if ((double)k * df < x) ++k;
    if ((double)(k - 1) * df >= x) --k;
    return (int)max(-1LL, min(k, 0x7ffffffeLL));
}

__global__ void k_spline(int B, Modes md, GridDesc g, const ModeBand *__restrict__ band,
                         const double *__restrict__ kf, const double *__restrict__ fn, double *__restrict__ coef,
                         double *__restrict__ scratch, int *__restrict__ kbin)
{
    constexpr int U = kSplineU;
    const int ns = g.ns;
    const int nt = B * md.nm * kNumFn;
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= nt) return;
    const int q = id % kNumFn;
    const int wm = id / kNumFn;
    double *out = coef + (size_t)wm * (ns - 1) * kCoefPerIv + q * 4;
    const double *x = kf + (size_t)wm * ns;
    const bool act = band[wm].active != 0;
    {
        int *kb = kbin + (size_t)wm * ns;
        for (int i0 = q; i0 < ns; i0 += U * kNumFn) {
            double xs[U];
#pragma unroll
            for (int u = 0; u < U; ++u) xs[u] = x[min(i0 + u * kNumFn, ns - 1)];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = i0 + u * kNumFn;
                if (i < ns) kb[i] = act ? first_bin(xs[u], g.df) : 0;
            }
        }
    }
    if (!act) {
        for (int i = 0; i < ns - 1; ++i)
            for (int c = 0; c < 4; ++c) out[(size_t)i * kCoefPerIv + c] = 0.0;
        return;
    }
    const double *y = fn + ((size_t)wm * kNumFn + q) * ns;
    double *cp = scratch + id;                    // cp[r]  -> cp[r * nt]
    double *Mv = scratch + (size_t)ns * nt + id;  // Mv[i]  -> Mv[i * nt]
    const int m = ns - 2;  // unknowns M_1..M_{ns-2}, row r <-> M_{r+1}

    // forward elimination; row r uses knots r, r+1, r+2
    double prev_c = 0.0, prev_d = 0.0;
    double xa = x[0], xb = x[1], ya = y[0], yb = y[1];
    for (int r0 = 0; r0 < m; r0 += U) {
        double xs[U], ys[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = min(r0 + u + 2, ns - 1);
            xs[u] = x[j];
            ys[u] = y[j];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = r0 + u;
            if (r >= m) continue;
            const double xc = xs[u], yc = ys[u];
            const double h0 = xb - xa, h1 = xc - xb;
            const double s0 = (yb - ya) / h0, s1 = (yc - yb) / h1;
            double sub = h0, dia = 2.0 * (h0 + h1), sup = h1;
            const double rhs = 6.0 * (s1 - s0);
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
            const double den = dia - sub * prev_c;
            const double c = sup / den;
            const double d = (rhs - sub * prev_d) / den;
            cp[(size_t)r * nt] = c;
            Mv[(size_t)(r + 1) * nt] = d;   // holds d_r until back substitution
            prev_c = c;
            prev_d = d;
            xa = xb; xb = xc; ya = yb; yb = yc;
        }
    }
    // back substitution: M_{m} = d_{m-1}; M_{r+1} = d_r - c_r M_{r+2} for r = m-2 .. 0
    double mn = prev_d;
    for (int r0 = m - 2; r0 >= 0; r0 -= U) {
        double ds[U], cs[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = max(r0 - u, 0);
            ds[u] = Mv[(size_t)(r + 1) * nt];
            cs[u] = cp[(size_t)r * nt];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = r0 - u;
            if (r < 0) continue;
            mn = ds[u] - cs[u] * mn;
            Mv[(size_t)(r + 1) * nt] = mn;
        }
    }
    {
        const double h0 = x[1] - x[0], h1 = x[2] - x[1];
        Mv[0] = ((h0 + h1) * Mv[(size_t)nt] - h0 * Mv[(size_t)2 * nt]) / h1;
        const double ha = x[ns - 2] - x[ns - 3], hb = x[ns - 1] - x[ns - 2];
        Mv[(size_t)(ns - 1) * nt] = ((ha + hb) * Mv[(size_t)(ns - 2) * nt] - hb * Mv[(size_t)(ns - 3) * nt]) / ha;
    }
    // coefficients of interval i from knots i, i+1, then re-centred on
    // fc = kbin[i+1] df, the first dense bin of the next interval: the dense
    // stage evaluates q(f - fc) = p(f - x_i) with q(t) = p(t + fc - x_i), and
    // takes fc from the interval bound it already holds
    double x0 = x[0], y0 = y[0], m0 = Mv[0];
    for (int i0 = 0; i0 < ns - 1; i0 += U) {
        double xs[U], ys[U], ms[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = min(i0 + u + 1, ns - 1);
            xs[u] = x[j];
            ys[u] = y[j];
            ms[u] = Mv[(size_t)j * nt];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u;
            if (i >= ns - 1) continue;
            const double x1 = xs[u], y1 = ys[u], m1 = ms[u];
            const double h = x1 - x0;
            const double sl = (y1 - y0) / h;
            const double p0 = y0, p1 = sl - h * (2.0 * m0 + m1) / 6.0, p2 = 0.5 * m0, p3 = (m1 - m0) / (6.0 * h);
            const double dl = (double)first_bin(x1, g.df) * g.df - x0;
            double *o = out + (size_t)i * kCoefPerIv;
            o[0] = fma(fma(fma(p3, dl, p2), dl, p1), dl, p0);
            o[1] = fma(fma(3.0 * p3, dl, 2.0 * p2), dl, p1);
            o[2] = fma(3.0 * p3, dl, p2);
            o[3] = p3;
            x0 = x1; y0 = y1; m0 = m1;
        }
    }
}

}  // namespace

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
    const int nt = B * md.nm * kNumFn;
    k_spline<<<(nt + 63) / 64, 64, 0, st>>>(B, md, g, wk.band, wk.kf, wk.fn, wk.coef, wk.spline_scratch, wk.kbin);
    return hipGetLastError();
}

}  // namespace mbh
