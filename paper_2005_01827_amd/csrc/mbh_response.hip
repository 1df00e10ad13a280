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
// knots, by parallel cyclic reduction of the second-derivative system.
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
constexpr int kSplineRows = 4;     // rows per thread: ns - 2 <= 1024

// LDS of one spline workgroup solving G functions together: the matrix
// (3 m) and the reciprocals of its diagonal (m), G right-hand sides, 2 G end
// values, the knots, the reciprocal interval widths and the knots' first
// dense bins.
constexpr size_t kSplineLdsMax = 65536;
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

// Not-a-knot splines through (f_j, y_j), one workgroup per (walker, mode).
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
template <int G>
__global__ __launch_bounds__(kSplineThreads) void k_spline(int B, Modes md, GridDesc g,
                                                           const ModeBand *__restrict__ band,
                                                           const double *__restrict__ kf,
                                                           const double *__restrict__ fn,
                                                           double *__restrict__ coef, int *__restrict__ kbin)
{
    extern __shared__ double sm[];
    const int ns = g.ns, m = ns - 2;
    const int wm = blockIdx.x;
    if (wm >= B * md.nm) return;
    const double *xg = kf + (size_t)wm * ns;
    double *out = coef + (size_t)wm * (ns - 1) * kCoefPerIv;
    const bool act = band[wm].active != 0;
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
            C[r] = sup;
            for (int q = 0; q < G; ++q) {
                const double *y = fn + ((size_t)wm * kNumFn + q0 + q) * ns;
                D[(size_t)q * m + r] = 6.0 * ((y[i + 1] - y[i]) * hinv[i] - (y[i] - y[i - 1]) * hinv[i - 1]);
            }
        }
        __syncthreads();
        // cyclic reduction rounds; each round first forms 1 / b of every
        // row, one division per row instead of one per neighbour
        for (int s = 1; s < m; s *= 2) {
            for (int r = threadIdx.x; r < m; r += kSplineThreads) binv[r] = 1.0 / Bm[r];
            __syncthreads();
            double na[kSplineRows], nb[kSplineRows], nc[kSplineRows], nd[kSplineRows][G];
#pragma unroll
            for (int u = 0; u < kSplineRows; ++u) {
                const int r = threadIdx.x + u * kSplineThreads;
                if (r >= m) continue;
                const bool lo = r - s >= 0, hi = r + s < m;
                const double al = lo ? -A[r] * binv[r - s] : 0.0;
                const double ga = hi ? -C[r] * binv[r + s] : 0.0;
                na[u] = lo ? al * A[r - s] : 0.0;
                nc[u] = hi ? ga * C[r + s] : 0.0;
                nb[u] = Bm[r] + (lo ? al * C[r - s] : 0.0) + (hi ? ga * A[r + s] : 0.0);
#pragma unroll
                for (int q = 0; q < G; ++q) {
                    const double *dq = D + (size_t)q * m;
                    nd[u][q] = dq[r] + (lo ? al * dq[r - s] : 0.0) + (hi ? ga * dq[r + s] : 0.0);
                }
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kSplineRows; ++u) {
                const int r = threadIdx.x + u * kSplineThreads;
                if (r >= m) continue;
                A[r] = na[u];
                Bm[r] = nb[u];
                C[r] = nc[u];
#pragma unroll
                for (int q = 0; q < G; ++q) D[(size_t)q * m + r] = nd[u][q];
            }
            __syncthreads();
        }
        // M_{r+1} = d_r / b_r, in place
        for (int t = threadIdx.x; t < G * m; t += kSplineThreads) D[t] /= Bm[t % m];
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
        // coefficients of interval i from knots i, i+1, re-centred on fc
        for (int t = threadIdx.x; t < (ns - 1) * G; t += kSplineThreads) {
            const int i = t / G, q = t % G;
            const double *Mq = D + (size_t)q * m;
            const double *y = fn + ((size_t)wm * kNumFn + q0 + q) * ns;
            const double mi = i == 0 ? M0[q] : Mq[i - 1];
            const double mj = i + 1 == ns - 1 ? M1[q] : Mq[i];
            const double x0 = x[i], h = x[i + 1] - x0, hi = hinv[i];
            const double sl = (y[i + 1] - y[i]) * hi;
            const double p0 = y[i], p1 = sl - h * (2.0 * mi + mj) / 6.0, p2 = 0.5 * mi, p3 = (mj - mi) * hi / 6.0;
            const double dl = (double)kbl[i + 1] * g.df - x0;
            double *o = out + (size_t)i * kCoefPerIv + (q0 + q) * 4;
            o[0] = fma(fma(fma(p3, dl, p2), dl, p1), dl, p0);
            o[1] = fma(fma(3.0 * p3, dl, 2.0 * p2), dl, p1);
            o[2] = fma(3.0 * p3, dl, p2);
            o[3] = p3;
        }
        __syncthreads();
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
    const size_t lds = spline_lds_bytes(g.ns);
    const unsigned grid = (unsigned)(B * md.nm);
    switch (spline_group(g.ns)) {
    case kNumFn:
        k_spline<kNumFn><<<grid, kSplineThreads, lds, st>>>(B, md, g, wk.band, wk.kf, wk.fn, wk.coef, wk.kbin);
        break;
    case kNumFn / 2:
        k_spline<kNumFn / 2><<<grid, kSplineThreads, lds, st>>>(B, md, g, wk.band, wk.kf, wk.fn, wk.coef, wk.kbin);
        break;
    case kNumFn / 4:
        k_spline<kNumFn / 4><<<grid, kSplineThreads, lds, st>>>(B, md, g, wk.band, wk.kf, wk.fn, wk.coef, wk.kbin);
        break;
    default:
        k_spline<1><<<grid, kSplineThreads, lds, st>>>(B, md, g, wk.band, wk.kf, wk.fn, wk.coef, wk.kbin);
        break;
    }
    return hipGetLastError();
}

}  // namespace mbh
