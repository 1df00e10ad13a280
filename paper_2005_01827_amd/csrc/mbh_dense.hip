// Dense stage on the GPU: interpolation of every mode onto the dense grid,
// the per-channel template h^c(f_k) = sum_lm T^c_lm A_lm e^{i phi_lm}
// (Sec. II.A) and the noise-weighted sums of Eqs. NLL/innerprod/innerprodsum:
//   R_c  = sum_k |d_k - h_k|^2 w_k,  DH_c = sum_k Re(d_k h_k^*) w_k,
//   HH_c = sum_k |h_k|^2 w_k,        w_k = 4 df / S_c(f_k),
// over each walker's union band, plus the data-only sum outside it from
// per-channel prefix sums, so that ln L = -(R + DD_out)/2.
//
// Work decomposition: the dense grid is cut into tiles of tile_bins bins;
// work items (walker, tile) cover each walker's union band and are listed
// tile-major (all walkers of tile 0, then tile 1, ...); workgroups take the
// next item from a counter, so that workgroups running together share a few
// data tiles in L2 and the batch ends evenly.
// Each item writes its 9 partial sums to a walker-major slot, and one
// wavefront per walker adds its slots in a fixed order, so results do not
// depend on the order or the launch shape (no floating-point atomics).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "mbh_internal.h"

namespace mbh {
namespace {


// ---------------------------------------------------------------------------
// Setup: w = 4 df / S and per-channel prefix sums of |d|^2 w.
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanPer = 8;
constexpr int kScanChunk = kScanThreads * kScanPer;

// one thread per (channel, padded bin); grid over 3 n_pad
__global__ void k_weights(const double *__restrict__ psd, const double2 *__restrict__ d_in,
                          double2 *__restrict__ d, double *__restrict__ w, double *__restrict__ e2,
                          float2 *__restrict__ dhi32, float2 *__restrict__ dlo32, float *__restrict__ sw32,
                          long long n, long long n_pad, double df4)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * n_pad) return;
    const int ch = (int)(t / n_pad);
    const long long k = t - ch * n_pad;
    const long long o = data_at(ch, k);
    if (k >= n) {
        d[o] = make_double2(0.0, 0.0);
        w[o] = 0.0;
        return;
    }
    const long long i = ch * n + k;
    const double wi = df4 / psd[i];
    const double2 di = d_in[i];
    w[o] = wi;
    d[o] = di;
    e2[i] = (di.x * di.x + di.y * di.y) * wi;
    if (dhi32) {
        // whitened data d sqrt(w) as an FP32 pair hi + lo (about 48 bits), so
        // that the residual d - h of the FP32 stage is formed without the
        // rounding of the data; sqrt(w) in FP32 stays inside the FP32 range
        // where w itself (up to ~1e44 near the arm-transfer nulls) would not
        const double sq = sqrt(wi);
        const double xr = di.x * sq, xi = di.y * sq;
        const float hr = (float)xr, hi = (float)xi;
        dhi32[i] = make_float2(hr, hi);
        dlo32[i] = make_float2((float)(xr - (double)hr), (float)(xi - (double)hi));
        sw32[i] = (float)sq;
    }
}

// Block-local inclusive scan of kScanChunk values, deterministic order.
__device__ double block_scan_sum(double *sh, double v)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const double a = (t >= off) ? sh[t - off] : 0.0;
        __syncthreads();
        sh[t] += a;
        __syncthreads();
    }
    return sh[t];
}

// pass 1: chunk sums; grid (nchunks, 3)
__global__ void k_scan_chunks(const double *__restrict__ e2, int n, double *__restrict__ chunk_sum, int nchunks)
{
    __shared__ double sh[kScanThreads];
    const int c = blockIdx.y, ch = blockIdx.x;
    const double *x = e2 + (size_t)c * n;
    const int base = ch * kScanChunk + threadIdx.x * kScanPer;
    double s = 0.0;
    for (int i = 0; i < kScanPer; ++i)
        if (base + i < n) s += x[base + i];
    const double incl = block_scan_sum(sh, s);
    if (threadIdx.x == kScanThreads - 1) chunk_sum[c * nchunks + ch] = incl;
}

// pass 2: exclusive scan of the chunk sums, one block per channel
__global__ void k_scan_offsets(double *__restrict__ chunk_sum, int nchunks)
{
    __shared__ double sh[kScanThreads];
    double *cs = chunk_sum + (size_t)blockIdx.x * nchunks;
    double carry = 0.0;
    for (int b0 = 0; b0 < nchunks; b0 += kScanThreads) {
        const int i = b0 + threadIdx.x;
        const double v = (i < nchunks) ? cs[i] : 0.0;
        const double incl = block_scan_sum(sh, v);
        if (i < nchunks) cs[i] = carry + incl - v;
        __syncthreads();
        carry += sh[kScanThreads - 1];
        __syncthreads();
    }
}

// pass 3: pre[c][i] = sum_{k < i} e2[c][k], i = 0..n
__global__ void k_scan_final(const double *__restrict__ e2, int n, const double *__restrict__ chunk_off, int nchunks,
                             double *__restrict__ pre)
{
    __shared__ double sh[kScanThreads];
    const int c = blockIdx.y, ch = blockIdx.x;
    const double *x = e2 + (size_t)c * n;
    double *p = pre + (size_t)c * (n + 1);
    const int base = ch * kScanChunk + threadIdx.x * kScanPer;
    double v[kScanPer];
    double s = 0.0;
    for (int i = 0; i < kScanPer; ++i) {
        v[i] = (base + i < n) ? x[base + i] : 0.0;
        s += v[i];
    }
    const double incl = block_scan_sum(sh, s);
    double run = chunk_off[c * nchunks + ch] + incl - s;
    for (int i = 0; i < kScanPer; ++i) {
        if (base + i < n) p[base + i] = run;
        run += v[i];
    }
    if (base + kScanPer >= n && base < n) p[n] = run;
}

// ---------------------------------------------------------------------------
// Work items.
// ---------------------------------------------------------------------------
__global__ void k_walker_bands(int B, int nm, GridDesc g, const Source *__restrict__ src,
                               const ModeBand *__restrict__ band, WalkerBand *__restrict__ wb)
{
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= B) return;
    wb[w] = walker_band(w, nm, g, src, band);
}

// A single walker's work-item list in one launch instead of five (items_one).
__global__ __launch_bounds__(256) void k_items_one(int nm, GridDesc g, const Source *__restrict__ src,
                                                   const ModeBand *__restrict__ band, WalkerBand *__restrict__ wb,
                                                   int *__restrict__ wbase, int *__restrict__ tile_off,
                                                   int *__restrict__ ticket, int *__restrict__ item_w,
                                                   int *__restrict__ item_t, int max_items)
{
    items_one(nm, g, src, band, wb, wbase, tile_off, ticket, item_w, item_t, max_items);
}

// exclusive scan of ntiles over walkers (single block)
__global__ void k_scan_walkers(int B, const WalkerBand *__restrict__ wb, int *__restrict__ wbase)
{
    __shared__ int sh[1024];
    int carry = 0;
    for (int b0 = 0; b0 < B; b0 += 1024) {
        const int i = b0 + threadIdx.x;
        const int v = (i < B) ? wb[i].ntiles : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int a = (threadIdx.x >= (unsigned)off) ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += a;
            __syncthreads();
        }
        if (i < B) wbase[i] = carry + sh[threadIdx.x] - v;
        const int tot = sh[1023];
        __syncthreads();
        carry += tot;
    }
    if (threadIdx.x == 0) wbase[B] = carry;
}

// Work items in tile-major order: all walkers whose band covers tile 0, in
// walker order, then tile 1, and so on.  Workgroups that run at the same time
// then share the same few data tiles, which stay in L2 instead of every
// walker streaming its whole band from memory.  Partial-sum slots stay
// walker-major (slot = wbase[w] + tile - tile_lo), so the reduction, and with
// it every bit of ln L, does not depend on the order.
__device__ __forceinline__ bool covers(const WalkerBand &b, int t)
{
    return t >= b.tile_lo && t < b.tile_lo + b.ntiles;
}

// count of walkers per tile; one workgroup per tile
__global__ __launch_bounds__(256) void k_tile_count(int B, const WalkerBand *__restrict__ wb,
                                                    int *__restrict__ tile_off)
{
    __shared__ int red[256];
    const int t = blockIdx.x;
    int c = 0;
    for (int w = threadIdx.x; w < B; w += 256) c += covers(wb[w], t) ? 1 : 0;
    red[threadIdx.x] = c;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) tile_off[t] = red[0];
}

// exclusive scan of the per-tile counts in place (single workgroup of 1024)
__global__ __launch_bounds__(1024) void k_tile_scan(int ntiles, int *__restrict__ tile_off, int *__restrict__ ticket)
{
    // the dense kernel that follows takes its items from this counter
    if (threadIdx.x == 0) ticket[0] = 0;
    __shared__ int sh[1024];
    int carry = 0;
    for (int b0 = 0; b0 < ntiles; b0 += 1024) {
        const int i = b0 + threadIdx.x;
        const int v = (i < ntiles) ? tile_off[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int a = (threadIdx.x >= (unsigned)off) ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += a;
            __syncthreads();
        }
        if (i < ntiles) tile_off[i] = carry + sh[threadIdx.x] - v;
        const int tot = sh[1023];
        __syncthreads();
        carry += tot;
    }
    if (threadIdx.x == 0) tile_off[ntiles] = carry;
}

// the walkers of each tile, compacted in walker order; one workgroup per tile
__global__ __launch_bounds__(256) void k_tile_fill(int B, const WalkerBand *__restrict__ wb,
                                                   const int *__restrict__ tile_off, int *__restrict__ item_w,
                                                   int *__restrict__ item_t, int max_items)
{
    __shared__ int sh[256];
    const int t = blockIdx.x;
    int run = tile_off[t];
    for (int w0 = 0; w0 < B; w0 += 256) {
        const int w = w0 + threadIdx.x;
        const int f = (w < B && covers(wb[w], t)) ? 1 : 0;
        sh[threadIdx.x] = f;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            const int a = (threadIdx.x >= (unsigned)off) ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += a;
            __syncthreads();
        }
        const int pos = run + sh[threadIdx.x] - f;
        if (f && pos < max_items) {
            item_w[pos] = w;
            item_t[pos] = t;
        }
        const int tot = sh[255];
        __syncthreads();
        run += tot;
    }
}

// ---------------------------------------------------------------------------
// Dense interpolation + inner products.
// ---------------------------------------------------------------------------
struct DenseArgs {
    int B, nm, ns, k0, n;
    int steps, tile_bins;
    double df;
    int max_items;
    int one_per_walker;
    int use_ticket;      // take items from *ticket instead of a fixed stride
    int *ticket;
    const ModeBand *band;
    const WalkerBand *wband;
    const int *wbase;
    const int *item_w;
    const int *item_t;
    const double *kf;
    const int *kbin;
    const double *coef;
    const double2 *d;
    const double *w;
    double *partial;
    double2 *h;          // template output (WriteH only)
    const double *cis_tab;
    // FP32 dense stage
    const float2 *dhi32;
    const float2 *dlo32;
    const float *sw32;
    const float *coef32;
    const float *cis32;
};

__device__ __forceinline__ int uni_i(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Interval of dense bin k among the knot bins kb[0..ns-1] of one (walker,
// mode): the largest iv in [c, ns-2] with kb[iv] <= k, for kb[c] <= k, and
// nb = kb[iv + 1].  win holds kb[min(c + 1 + lane, ns - 1)], the 64 knot bins
// after the step's first interval, one per lane: a binary search over that
// window by shuffles (seven probes, no memory access) replaces a walk with
// one dependent load per knot, which dominated steps that cross many knots.
// Every lane of the wavefront must take part (the shuffles read other
// lanes); beyond the window (more than 64 knots in one step) or at the last
// interval the walk over kb finishes the search.
__device__ __forceinline__ int lane_interval(const int *kb, int ns, int c, int win, int k, int &nb)
{
    int t = -1;   // largest t with win[t] <= k, -1 if none
#pragma unroll
    for (int s2 = 64; s2 >= 1; s2 >>= 1) {
        const int p = t + s2;
        const int v = __shfl(win, p < 63 ? p : 63, 64);
        if (p <= 63 && v <= k) t = p;
    }
    int iv = c + 1 + t;
    nb = __shfl(win, t < 62 ? t + 1 : 63, 64);
    if (t == 63 || iv > ns - 2) {
        iv = min(iv, ns - 2);
        while (iv < ns - 2 && kb[iv + 1] <= k) ++iv;
        nb = kb[iv + 1];
    }
    return iv;
}

// e^{i phi} = e^{i q pi/512} e^{i r}.  t = phi 512/pi is rounded to the
// integer q by adding and subtracting 1.5 2^52 (exact for |t| < 2^51), which
// leaves q mod 2^32 in the low word of the sum; r = phi - q pi/512 with a
// two-part pi/512 (two FMAs), so |r| <= pi/1024 up to rounding.  On that
// range sin r = r - r^3/6 truncates below 2.3e-15 and cos r = 1 - r^2/2 +
// r^4/24 below 1.2e-18, far under the rounding of phi itself (the phase of a
// mode reaches 2 pi f t_c, about 1e6 rad, whose last bit is 1e-10 rad);
// e^{i q pi/512} is entry q mod 1024 of a table of cos and sin of j pi/512,
// staged in LDS (16 KB): one per-lane LDS read replaces the quadrant logic
// and most of the polynomial of a reduction modulo pi/2.
//
// Device table layout (filled once per context): kCisN constants, then the
// kRotN (cos, sin) pairs.
constexpr int kRotN = 1024;
constexpr int kCisN = 8;
constexpr int kCisPoly = 5;      // constants used by cis(): 512/pi, pi/512 (two parts), -1/6, 1/24
constexpr int kTwoOverPi = 6;    // 2/pi, for the quarter-turn reduction of the FP32 stage
constexpr double kRoundShift = 6755399441055744.0;   // 1.5 * 2^52
static_assert(kCisN % 2 == 0 && kCisN + 2 * kRotN <= kCisTabDoubles, "rotation table must fit the device table");
const double kCisHost[kCisN] = {
    162.97466172610082383,                                    // 512/pi
    3.141592653589793116 / 512.0,                             // pi/512 rounded to double (exact scaling of pi)
    1.2246467991473532e-16 / 512.0,                           // pi/512 - the above
    -1.0 / 6.0,                                               // sin: r^3
    1.0 / 24.0,                                               // cos: r^4
    0.0,
    0.63661977236758134308,                                   // 2/pi
    0.0};

typedef const __attribute__((address_space(4))) double cdouble;
typedef const __attribute__((address_space(4))) int cint;

struct CisConst {
    double k[kCisPoly];
    double two_over_pi;
    const double2 *rot;   // kRotN entries in LDS
};

// A zero the compiler cannot prove wave-uniform: indexing with it turns a
// table read into per-lane vector loads, so the values live in VGPRs.
__device__ __forceinline__ int lane_zero()
{
    int z;
    asm volatile("v_mov_b32 %0, 0" : "=v"(z));
    return z;
}

// The polynomial and reduction constants are held in VGPRs: in
// scalar registers they pushed the per-mode interval state and the
// coefficient blocks into SGPR spills, whose reloads cost more VALU issue
// than the VGPRs cost occupancy.  The rotation table is copied to LDS by the
// workgroup (the caller synchronises before first use).
__device__ __forceinline__ void load_cis(CisConst &K, const double *tab, double2 *rot_lds)
{
    const double *t = tab + lane_zero();
#pragma unroll
    for (int i = 0; i < kCisPoly; ++i) K.k[i] = t[i];
    K.two_over_pi = t[kTwoOverPi];
    for (int i = threadIdx.x; i < kRotN; i += blockDim.x)
        rot_lds[i] = ((const double2 *)(tab + kCisN))[i];
    K.rot = rot_lds;
}

__device__ __forceinline__ void cis(const CisConst &K, double phi, double &sn, double &cs)
{
    const double y = fma(phi, K.k[0], kRoundShift);
    const double q = y - kRoundShift;
    const double2 e = K.rot[__double2loint(y) & (kRotN - 1)];
    double r = fma(-q, K.k[1], phi);
    r = fma(-q, K.k[2], r);
    const double r2 = r * r;
    const double sr = fma(r * r2, K.k[3], r);
    const double pc = fma(K.k[4], r2, -0.5);
    const double cr = fma(r2, pc, 1.0);
    cs = fma(e.x, cr, -(e.y * sr));
    sn = fma(e.y, cr, e.x * sr);
}

// Cubic c0 + c1 x + c2 x^2 + c3 x^3 from a wave-uniform table (scalar
// registers), by Horner's rule with alternating signs:
//   u = -(c3 x + c2),  v = u x - c1,  result = -v x + c0.
// Every FMA carries a negation modifier, which only the three-operand
// encoding can express, so each reads its scalar coefficient in place; the
// plain form is compiled to the two-operand accumulate FMA with every
// coefficient first copied to vector registers (6 moves per cubic).  Only c2
// (the first FMA has two scalar operands) is copied.  Starting instead with
// the product c3 * x from a scalar register was measured to drop the c3 x^3
// term on gfx950 when x had just been computed (reproduced by a one-wavefront
// test kernel), so that form is not used; the parity tests guard this.
// The copy of c2 is one 64-bit move (the compiler splits it into two 32-bit
// moves).
__device__ __forceinline__ double vcopy(double s)
{
    double v;
    asm("v_mov_b64 %0, %1" : "=v"(v) : "s"(s));
    return v;
}
__device__ __forceinline__ double cubic_s(cdouble *c, double x)
{
    const double u = fma(-c[3], x, -vcopy(c[2]));
    const double v = fma(u, x, -c[1]);
    return fma(-v, x, c[0]);
}
__device__ __forceinline__ double cubic_v(const double *c, double x)
{
    return fma(fma(fma(c[3], x, c[2]), x, c[1]), x, c[0]);
}

// One mode at one bin: h^c += T^c(dx) A(dx) e^{i phi(dx)}, with the 32
// coefficients of the bin's interval at c (A, phi, Re/Im T^A, T^E, T^T),
// either wave-uniform (cdouble*, scalar loads) or per lane.  The compiler
// barriers keep one group of eight coefficients in flight at a time, which
// bounds scalar-register pressure.
template <typename P>
__device__ __forceinline__ double cub(P c, double x);
template <>
__device__ __forceinline__ double cub<cdouble *>(cdouble *c, double x) { return cubic_s(c, x); }
template <>
__device__ __forceinline__ double cub<const double *>(const double *c, double x) { return cubic_v(c, x); }

template <typename P>
__device__ __forceinline__ void mode_bin(const CisConst &K, P c, double dx, double (&hr)[3], double (&hi)[3])
{
    const double amp = cub<P>(c + 0, dx);
    const double ph = cub<P>(c + 4, dx);
    asm volatile("" ::: "memory");
    double sn, cs;
    cis(K, ph, sn, cs);
    const double ar = amp * cs, ai = amp * sn;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        const double tr = cub<P>(c + 8 + 8 * ch, dx);
        const double ti = cub<P>(c + 12 + 8 * ch, dx);
        hr[ch] = fma(tr, ar, fma(-ti, ai, hr[ch]));
        hi[ch] = fma(tr, ai, fma(ti, ar, hi[ch]));
        asm volatile("" ::: "memory");
    }
}

// One mode at the NB bins of a lane in one step, all in one interval and
// inside the mode's band: the wave-uniform coefficients are read once and
// feed NB independent evaluations, with no per-bin test.
template <int NB>
__device__ __forceinline__ void mode_bins_u(const CisConst &K, cdouble *c, const double (&dx)[NB],
                                            double (&hr)[NB][3], double (&hi)[NB][3])
{
    double ar[NB], ai[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const double amp = cubic_s(c + 0, dx[b]);
        const double ph = cubic_s(c + 4, dx[b]);
        double sn, cs;
        cis(K, ph, sn, cs);
        ar[b] = amp * cs;
        ai[b] = amp * sn;
    }
    asm volatile("" ::: "memory");
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const double tr = cubic_s(c + 8 + 8 * ch, dx[b]);
            const double ti = cubic_s(c + 12 + 8 * ch, dx[b]);
            hr[b][ch] = fma(tr, ar[b], fma(-ti, ai[b], hr[b][ch]));
            hi[b][ch] = fma(tr, ai[b], fma(ti, ar[b], hi[b][ch]));
        }
        asm volatile("" ::: "memory");
    }
}

// ---- FP32 dense stage ---------------------------------------------------
// The phase polynomial is evaluated and reduced in FP64 (phases reach 1e7
// rad); the remainder of a quarter turn, |r| <= pi/4, goes to FP32 for the
// sine and cosine.  Amplitude and response cubics and the complex products
// run in FP32 from an FP32 copy of the coefficients.
constexpr int kCis32N = 10;
const float kCis32Host[kCis32N] = {
    1.5707963267948966f,                                                  // pi/2
    1.0f / 362880.0f, -1.0f / 5040.0f, 1.0f / 120.0f, -1.0f / 6.0f,          // sin: r^9 .. r^3
    -1.0f / 3628800.0f, 1.0f / 40320.0f, -1.0f / 720.0f, 1.0f / 24.0f, -0.5f  // cos: r^10 .. r^2
};
typedef const __attribute__((address_space(4))) float cfloat;

struct CisConst32 {
    float k[kCis32N];
};

__device__ __forceinline__ void load_cis32(CisConst32 &K, const float *tab)
{
    cfloat *t = (cfloat *)tab;
#pragma unroll
    for (int i = 0; i < kCis32N; ++i) K.k[i] = t[i];
}

// e^{i phi} for an FP64 phase: quarter turns t = phi 2/pi and q = rint(t) in
// FP64, r = (t - q) pi/2 in FP32, Taylor polynomials of sin r (to r^9) and
// cos r (to r^10), truncation below 2e-9 on |r| <= pi/4.
__device__ __forceinline__ void cis32(const CisConst &K, const CisConst32 &Kf, double phi, float &sn, float &cs)
{
    const double t = phi * K.two_over_pi;
    const double q = rint(t);
    const float r = (float)(t - q) * Kf.k[0];
    const float r2 = r * r;
    float ps = fmaf(Kf.k[1], r2, Kf.k[2]);
    ps = fmaf(ps, r2, Kf.k[3]);
    ps = fmaf(ps, r2, Kf.k[4]);
    const float sr = fmaf(r * r2, ps, r);
    float pc = fmaf(Kf.k[5], r2, Kf.k[6]);
    pc = fmaf(pc, r2, Kf.k[7]);
    pc = fmaf(pc, r2, Kf.k[8]);
    pc = fmaf(pc, r2, Kf.k[9]);
    const float cr = fmaf(r2, pc, 1.0f);
    const int iq = ((int)q) & 3;
    const float a = (iq & 1) ? cr : sr;
    const float b = (iq & 1) ? sr : cr;
    sn = (iq & 2) ? -a : a;
    cs = ((iq + 1) & 2) ? -b : b;
}

__device__ __forceinline__ float cubic32_s(cfloat *c, float x)
{
    return fmaf(fmaf(fmaf(c[3], x, c[2]), x, c[1]), x, c[0]);
}
__device__ __forceinline__ float cubic32_v(const float *c, float x)
{
    return fmaf(fmaf(fmaf(c[3], x, c[2]), x, c[1]), x, c[0]);
}
template <typename P>
__device__ __forceinline__ float cub32(P c, float x);
template <>
__device__ __forceinline__ float cub32<cfloat *>(cfloat *c, float x) { return cubic32_s(c, x); }
template <>
__device__ __forceinline__ float cub32<const float *>(const float *c, float x) { return cubic32_v(c, x); }

// One mode at one bin, FP32 stage: cd points at the FP64 coefficients of the
// interval (phase at +4), cf at their FP32 copy (amplitude at +0, response at
// +8).
template <typename PD, typename PF>
__device__ __forceinline__ void mode_bin32(const CisConst &K, const CisConst32 &Kf, PD cd, PF cf, double dx,
                                           float (&hr)[3], float (&hi)[3])
{
    const double ph = cub<PD>(cd + 4, dx);
    const float dxf = (float)dx;
    const float amp = cub32<PF>(cf + 0, dxf);
    asm volatile("" ::: "memory");
    float sn, cs;
    cis32(K, Kf, ph, sn, cs);
    const float ar = amp * cs, ai = amp * sn;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        const float tr = cub32<PF>(cf + 8 + 8 * ch, dxf);
        const float ti = cub32<PF>(cf + 12 + 8 * ch, dxf);
        hr[ch] = fmaf(tr, ar, fmaf(-ti, ai, hr[ch]));
        hi[ch] = fmaf(tr, ai, fmaf(ti, ar, hi[ch]));
    }
}

// FP32 stage, NB bins of a lane in one interval (see mode_bins_u).
template <int NB>
__device__ __forceinline__ void mode_bins32_u(const CisConst &K, const CisConst32 &Kf, cdouble *cd, cfloat *cf,
                                              const double (&dx)[NB], float (&hr)[NB][3], float (&hi)[NB][3])
{
    float ar[NB], ai[NB], dxf[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const double ph = cubic_s(cd + 4, dx[b]);
        dxf[b] = (float)dx[b];
        const float amp = cubic32_s(cf + 0, dxf[b]);
        float sn, cs;
        cis32(K, Kf, ph, sn, cs);
        ar[b] = amp * cs;
        ai[b] = amp * sn;
    }
    asm volatile("" ::: "memory");
#pragma unroll
    for (int ch = 0; ch < 3; ++ch)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const float tr = cubic32_s(cf + 8 + 8 * ch, dxf[b]);
            const float ti = cubic32_s(cf + 12 + 8 * ch, dxf[b]);
            hr[b][ch] = fmaf(tr, ar[b], fmaf(-ti, ai[b], hr[b][ch]));
            hi[b][ch] = fmaf(tr, ai[b], fmaf(ti, ar[b], hi[b][ch]));
        }
}

// Kahan-compensated FP32 sum: s - c carries the running total.
__device__ __forceinline__ void kahan_add(float &s, float &c, float x)
{
#pragma clang fp contract(off)
    const float y = x - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

// Residual square of the FP32 stage, one real component, in float-float:
// r = (dh + dl) - ht with the data as an FP32 pair and the whitened template
// ht in FP32.  TwoSum (Knuth) makes dh - ht exact as s + e, so r = s + rl
// with rl = e + dl; r^2 = s^2 + 2 s rl (+ rl^2, below 2^-48 r^2), with s^2
// split exactly by an FMA (TwoProd, Dekker / Ogita-Rump-Oishi).  The high
// part joins the running sum (hs, ls) by TwoSum and every low part goes to
// ls.  Contraction stays off here: fusing a product into the sums would
// break the error-free transformations.
__device__ __forceinline__ void ff_resid_add(float dh, float dl, float ht, float &hs, float &ls)
{
#pragma clang fp contract(off)
    const float s = dh - ht;
    const float bv = s - dh;
    const float e = (dh - (s - bv)) + (-ht - bv);
    const float rl = e + dl;
    const float p = s * s;
    const float pe = __builtin_fmaf(s, s, -p);
    const float q = __builtin_fmaf(s + s, rl, pe);
    const float t = hs + p;
    const float bt = t - hs;
    const float et = (hs - (t - bt)) + (p - bt);
    hs = t;
    ls = ls + (et + q);
}

// A work item is (walker, tile); each of the four wavefronts of a block takes
// 64*J consecutive bins in J/NB steps of 64*NB (lane l: bins s_j + 64 b + l,
// b < NB).  Per step the wavefront evaluates all modes at its bins; with
// NB = 2 each coefficient fetch of the uniform path serves two bins per lane,
// which halves the scalar loads and interval bookkeeping per bin and gives
// every wavefront two independent evaluation chains.  For every mode it keeps, in
// scalar registers, the sparse interval of its current step and the first
// bin of the next interval (integer bin bounds from kbin).  A step inside one
// interval (the common case: intervals span tens to tens of thousands of
// bins) reads the interval's 32 coefficients with scalar loads; a step that
// crosses knots falls back to a per-lane interval search and per-lane loads.
// Only the current bin's template lives in registers; the residual sums are
// accumulated per step.
//
// kF32 selects the FP32 stage: FP64 phase, FP32 template, whitened data as
// an FP32 pair, and the residual sums R_c in float-float (ff_resid_add), so
// that ln L keeps the residual form of Eq. NLL and only the template carries
// FP32 rounding; <d|h> and <h|h> (inner-product kernel only) are Kahan sums.
// kROnly: accumulate only the residual sums R_c (ln L needs nothing else);
// <d|h>_c and <h|h>_c are then left at zero.
// Occupancy: the FP64 likelihood kernel (kROnly) is held to 96 vector
// registers, five wavefronts per SIMD, which hides more of the scalar-load
// waits than four (measured 6 % faster; one 64-bit value is spilled, reloaded
// once per item); six would spill 32 values and ran 27 % slower.  The other
// instantiations keep three or four, where the tighter bound would spill more.
// kOne: one walker with no item list (launch_dense with walker_one); every
// workgroup forms the walker's band from its mode bands (an invalid walker
// has no active mode, so its band is empty) and takes the walker's tiles in
// order, and workgroup 0 stores the band and the scan over walkers for the
// reduction.
// One walker fills at most one workgroup per compute unit, so kOne takes
// two wavefronts per SIMD and the registers to spill nothing.
template <bool kWriteH, bool kF32, int NB, bool kROnly, bool kOne = false>
__global__ __launch_bounds__(kDenseThreads, kOne ? 2 : kROnly ? 5 : ((NB == 1 || kF32) ? 4 : 3)) void k_dense(DenseArgs a)
{
    static_assert(!kROnly || !kWriteH, "residual-only sums only on the likelihood paths");
    static_assert(!kOne || kROnly, "one-walker launches only on the likelihood paths");
    __shared__ double red[kDenseThreads / 64][kPartials];
    __shared__ double2 rot[kRotN];
    __shared__ int xcur[kDenseThreads / 64][kMaxModes];   // interval of a deferred mode, per wavefront
    __shared__ WalkerBand one;                            // kOne: the walker's band
    int total = kOne ? 0 : min(a.wbase[a.B], a.max_items);
    if (kOne && threadIdx.x == 0) {
        WalkerBand r;
        r.klo = 0;
        r.khi = -1;
        r.tile_lo = 0;
        r.ntiles = 0;
        int lo = 0x7fffffff, hi = -1;
        for (int m = 0; m < a.nm; ++m) {
            const ModeBand mb = a.band[m];
            if (!mb.active) continue;
            lo = min(lo, mb.klo);
            hi = max(hi, mb.khi);
        }
        if (hi >= lo) {
            r.klo = lo;
            r.khi = hi;
            r.tile_lo = (lo - a.k0) / a.tile_bins;
            r.ntiles = (hi - a.k0) / a.tile_bins - r.tile_lo + 1;
        }
        one = r;
        if (blockIdx.x == 0) {
            const_cast<WalkerBand *>(a.wband)[0] = r;
            const_cast<int *>(a.wbase)[0] = 0;
            const_cast<int *>(a.wbase)[1] = r.ntiles;
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ns = a.ns;
    CisConst K;
    load_cis(K, a.cis_tab, rot);
    __syncthreads();
    if (kOne) total = min(uni_i(one.ntiles), a.max_items);
    CisConst32 Kf;
    if (kF32) load_cis32(Kf, a.cis32);
    // Items: a fixed stride over the tile-major list, the items of one walker
    // (one_per_walker), or the next free item from a counter (tickets): a
    // workgroup that finishes early takes more, and workgroups running
    // together stay on neighbouring items of the list.  With tickets, the
    // first item of workgroup b is item b and the counter hands out items
    // gridDim.x and up (had every workgroup drawn its first item from the
    // counter, the first ones to start, which draw their second item as
    // they begin the first, could take two items while later ones found
    // none; with one walker's 245 items on 245 workgroups that doubled the
    // kernel).  The next ticket is taken when an item starts and read by
    // every thread after the item's last barrier, through two LDS slots used
    // in turn (a slot is rewritten only two items later, after a barrier
    // that every reader has passed), so no register holds it across the item.
    __shared__ int next_item[2];
    int par = 0;
    const bool tickets = !kWriteH && a.use_ticket && !a.one_per_walker;
    int item = blockIdx.x, end = total, step = gridDim.x;
    if (a.one_per_walker) {
        item = a.wbase[blockIdx.x];
        end = min(a.wbase[blockIdx.x + 1], total);
        step = 1;
    }
    while (item < end) {
        if (tickets && threadIdx.x == 0) next_item[par ^ 1] = (int)gridDim.x + atomicAdd(a.ticket, 1);
        // item values are wave-uniform: held in scalar registers, so that
        // none occupies a vector register across the item
        const int wk = a.one_per_walker ? (int)blockIdx.x : kOne ? 0 : uni_i(a.item_w[item]);
        WalkerBand wb = kOne ? one : a.wband[wk];
        wb.klo = uni_i(wb.klo);
        wb.khi = uni_i(wb.khi);
        wb.tile_lo = uni_i(wb.tile_lo);
        const int base = kOne ? 0 : uni_i(a.wbase[wk]);
        const int tile = a.one_per_walker || kOne ? wb.tile_lo + (item - base) : uni_i(a.item_t[item]);
        const int slot = uni_i(base + (tile - wb.tile_lo));
        const int kw = uni_i(a.k0 + tile * a.tile_bins + wave * (64 * a.steps));
        const int kwl = kw + 64 * a.steps - 1;

        // per-mode wave-uniform state: band, current interval, next bound
        int mlo[kMaxModes], mhi[kMaxModes], cur[kMaxModes], nxt[kMaxModes];
#pragma unroll
        for (int m = 0; m < kMaxModes; ++m) {
            mlo[m] = 1;
            mhi[m] = 0;
            cur[m] = 0;
            nxt[m] = 0x7fffffff;
            if (m < a.nm) {
                const ModeBand mb = a.band[wk * a.nm + m];
                if (mb.active && mb.khi >= kw && mb.klo <= kwl) {
                    const int kbo = (wk * a.nm + m) * ns;
                    cint *kb = (cint *)(a.kbin + kbo);
                    const int kfirst = uni_i(max(kw, mb.klo));
                    // largest i in [0, ns-2] with kb[i] <= kfirst, i.e. the
                    // number of such entries less one (kb is nondecreasing):
                    // every lane tests ns/64 entries and the wavefront counts
                    // the hits, one round of independent loads instead of a
                    // chain of log2(ns) dependent ones
                    int cnt = 0;
                    for (int j0 = 0; j0 < ns - 1; j0 += 256) {
                        int v[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int j = j0 + 64 * u + lane;
                            v[u] = j < ns - 1 ? a.kbin[kbo + j] : 0x7fffffff;
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u) cnt += __popcll(__ballot(v[u] <= kfirst));
                    }
                    const int i = uni_i(max(cnt - 1, 0));
                    mlo[m] = uni_i(mb.klo);
                    mhi[m] = uni_i(mb.khi);
                    cur[m] = i;
                    nxt[m] = uni_i(kb[i + 1]);
                }
            }
        }

        double acc[kPartials];
#pragma unroll
        for (int q = 0; q < kPartials; ++q) acc[q] = 0.0;
        float rh[3], rl[3];   // FP32 stage: float-float residual sums R_c
        float ks[6], kc[6];   // FP32 stage: Kahan sums of DH_c, HH_c
#pragma unroll
        for (int q = 0; q < 3; ++q) rh[q] = rl[q] = 0.0f;
#pragma unroll
        for (int q = 0; q < 6; ++q) ks[q] = kc[q] = 0.0f;

        // a step covers 64*NB bins; lane l takes bins s0 + 64 b + l
        for (int j = 0; j < a.steps; j += NB) {
            const int s0 = kw + 64 * j;
            int k[NB], idx[NB];
            bool inw[NB];
            double f[NB];
            double2 dv[NB][3];
            double wv[NB][3];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                k[b] = s0 + 64 * b + lane;
                inw[b] = (k[b] >= wb.klo) && (k[b] <= wb.khi);
                idx[b] = inw[b] ? k[b] - a.k0 : 0;
                f[b] = (double)k[b] * a.df;
            }
            unsigned xmask = 0u;   // modes whose step crosses a knot (wave-uniform)
            double hr[NB][3], hi[NB][3];
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) hr[b][ch] = hi[b][ch] = 0.0;
            float hr32[NB][3], hi32[NB][3];
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) hr32[b][ch] = hi32[b][ch] = 0.0f;
#pragma unroll
            for (int m = 0; m < kMaxModes; ++m) {
                const int lo = max(s0, mlo[m]), hi_ = min(s0 + 64 * NB - 1, mhi[m]);
                if (lo > hi_) continue;
                // knots and bin bounds of (walker, mode) start at kbo, its
                // intervals at ivo = kbo - wm; one shared base pointer per
                // table keeps the per-mode state to two 32-bit offsets
                const int wm = wk * a.nm + m;
                const int kbo = uni_i(wm * ns);
                const int ivo = kbo - wm;
                while (cur[m] < ns - 2 && nxt[m] <= lo) {
                    cur[m] = uni_i(cur[m] + 1);
                    nxt[m] = uni_i(((cint *)a.kbin)[kbo + cur[m] + 1]);
                }
                // the wave-uniform path takes a step that lies wholly inside
                // the mode's band and inside one interval; a step at a band
                // edge (once or twice per mode and walker) or across a knot
                // goes to the per-lane code
                const bool whole = s0 >= mlo[m] && s0 + 64 * NB - 1 <= mhi[m];
                if (whole && hi_ < nxt[m]) {
                    // the cubics of interval i are centred on the first bin of
                    // the next interval, kbin[i+1] = nxt: no knot load needed
                    const int iv = cur[m];
                    const double x0 = (double)nxt[m] * a.df;
                    const size_t c0 = (size_t)(ivo + iv) * kCoefPerIv;
                    if (NB > 1) {
                        double dx[NB];
#pragma unroll
                        for (int b = 0; b < NB; ++b) dx[b] = f[b] - x0;
                        if (kF32)
                            mode_bins32_u<NB>(K, Kf, (cdouble *)a.coef + c0, (cfloat *)a.coef32 + c0, dx, hr32, hi32);
                        else
                            mode_bins_u<NB>(K, (cdouble *)a.coef + c0, dx, hr, hi);
                    } else {
                        if (kF32)
                            mode_bin32<cdouble *, cfloat *>(K, Kf, (cdouble *)a.coef + c0, (cfloat *)a.coef32 + c0,
                                                            f[0] - x0, hr32[0], hi32[0]);
                        else
                            mode_bin<cdouble *>(K, (cdouble *)a.coef + c0, f[0] - x0, hr[0], hi[0]);
                    }
                } else if (!kF32) {
                    // defer the mode to the per-lane pass below, which then
                    // exists once instead of once per unrolled mode (3-5 %
                    // faster on the FP64 paths)
                    xmask |= 1u << m;
                    if (lane == 0) xcur[wave][m] = cur[m];
                } else {
                    // FP32 stage: per-lane evaluation in place (deferring did
                    // not pay there)
                    const int win = a.kbin[kbo + min(cur[m] + 1 + lane, ns - 1)];
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        int nb;
                        const int iv = lane_interval(a.kbin + kbo, ns, cur[m], win, k[b], nb);
                        if (k[b] < mlo[m] || k[b] > mhi[m]) continue;
                        const size_t c0 = (size_t)(ivo + iv) * kCoefPerIv;
                        const double xc = (double)nb * a.df;
                        mode_bin32<const double *, const float *>(K, Kf, a.coef + c0, a.coef32 + c0, f[b] - xc,
                                                                  hr32[b], hi32[b]);
                    }
                }
            }
            // per-lane pass over the modes whose step crosses a knot or a
            // band edge: each lane skips bins outside the band and finds its
            // own interval from the one of the step's start
#pragma nounroll
            for (unsigned mm = xmask; mm != 0u; mm &= mm - 1u) {
                const int m = uni_i(__builtin_ctz(mm));
                const int wm = wk * a.nm + m;
                const int kbo = uni_i(wm * ns);
                const int ivo = kbo - wm;
                const ModeBand mb = a.band[wm];
                const int c = uni_i(xcur[wave][m]);
                const int win = a.kbin[kbo + min(c + 1 + lane, ns - 1)];
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    int nb;
                    const int iv = lane_interval(a.kbin + kbo, ns, c, win, k[b], nb);
                    if (k[b] < mb.klo || k[b] > mb.khi) continue;
                    const size_t c0 = (size_t)(ivo + iv) * kCoefPerIv;
                    const double xc = (double)nb * a.df;
                    mode_bin<const double *>(K, a.coef + c0, f[b] - xc, hr[b], hi[b]);
                }
            }
            if (kWriteH) {
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    if (inw[b])
#pragma unroll
                        for (int ch = 0; ch < 3; ++ch)
                            a.h[(size_t)ch * a.n + idx[b]] = make_double2(hr[b][ch], hi[b][ch]);
            } else if (kF32) {
                // the data are loaded after the modes, as on the FP64 path
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    if (!inw[b]) continue;
#pragma unroll
                    for (int ch = 0; ch < 3; ++ch) {
                        const size_t o = (size_t)ch * a.n + idx[b];
                        const float2 dh = a.dhi32[o], dl = a.dlo32[o];
                        const float sw = a.sw32[o];
                        // whitened template h sqrt(w)
                        const float wr = hr32[b][ch] * sw, wi = hi32[b][ch] * sw;
                        ff_resid_add(dh.x, dl.x, wr, rh[ch], rl[ch]);
                        ff_resid_add(dh.y, dl.y, wi, rh[ch], rl[ch]);
                        if (!kROnly) {
                            kahan_add(ks[ch], kc[ch], fmaf(dh.x, wr, dh.y * wi));
                            kahan_add(ks[3 + ch], kc[3 + ch], fmaf(wr, wr, wi * wi));
                        }
                    }
                }
            } else {
                // d and w are loaded here, after the modes: holding them across
                // the mode loop took registers the mode evaluation needs
                // (measured: 9 % slower).  Bins s0 + 64 b + lane form block
                // (s0 - k0)/64 + b of the blocked layout: one wave-uniform
                // block address, the lane's element, and the channel as an
                // immediate offset.  Lanes outside the walker's band read
                // real (or padding) values that the sums below skip.
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const long long blk = uni_i((s0 - a.k0) / kDataBlk + b);
                    const char *db = (const char *)(a.d + blk * (3 * kDataBlk));
                    const char *wb = (const char *)(a.w + blk * (3 * kDataBlk));
#pragma unroll
                    for (int ch = 0; ch < 3; ++ch) {
                        dv[b][ch] = *(const double2 *)(db + ((unsigned)lane * 16u + ch * kDataBlk * 16u));
                        wv[b][ch] = *(const double *)(wb + ((unsigned)lane * 8u + ch * kDataBlk * 8u));
                    }
                }
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    if (!inw[b]) continue;
#pragma unroll
                    for (int ch = 0; ch < 3; ++ch) {
                        const double rr = dv[b][ch].x - hr[b][ch], ri = dv[b][ch].y - hi[b][ch];
                        acc[ch] = fma(fma(rr, rr, ri * ri), wv[b][ch], acc[ch]);
                        if (!kROnly) {
                            acc[3 + ch] =
                                fma(fma(dv[b][ch].x, hr[b][ch], dv[b][ch].y * hi[b][ch]), wv[b][ch], acc[3 + ch]);
                            acc[6 + ch] = fma(fma(hr[b][ch], hr[b][ch], hi[b][ch] * hi[b][ch]), wv[b][ch], acc[6 + ch]);
                        }
                    }
                }
            }
        }
        if (kWriteH) {
            item += step;
            continue;
        }
        if (kF32) {
#pragma unroll
            for (int q = 0; q < 3; ++q) acc[q] = (double)rh[q] + (double)rl[q];
            if (!kROnly)
#pragma unroll
                for (int q = 0; q < 6; ++q) acc[3 + q] = (double)ks[q] - (double)kc[q];
        }

        // wavefront butterfly, then the four wavefronts in order
#pragma unroll
        for (int q = 0; q < kPartials; ++q) {
            double v = acc[q];
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
            acc[q] = v;
        }
        if (lane == 0)
#pragma unroll
            for (int q = 0; q < kPartials; ++q) red[wave][q] = acc[q];
        __syncthreads();
        if (threadIdx.x < kPartials) {
            double s = 0.0;
#pragma unroll
            for (int wv = 0; wv < kDenseThreads / 64; ++wv) s += red[wv][threadIdx.x];
            a.partial[(size_t)slot * kPartials + threadIdx.x] = s;
        }
        __syncthreads();
        if (tickets) {
            par ^= 1;
            item = uni_i(next_item[par]);
        } else {
            item += step;
        }
    }
}

// One wavefront per walker: fixed-order sum of its item partials plus the
// data-only contribution outside its band.
__global__ void k_reduce(int B, GridDesc g, const Source *__restrict__ src, const WalkerBand *__restrict__ wband,
                         const int *__restrict__ wbase, const double *__restrict__ partial,
                         const double *__restrict__ pre, double *__restrict__ out7, double *__restrict__ logL)
{
    const int w = blockIdx.x;
    const int lane = threadIdx.x;
    if (w >= B) return;
    // the walker's band, validity and prefix sums are read while the
    // partials are summed (independent loads, one round trip for both)
    const WalkerBand wb = wband[w];
    const bool valid = src[w].valid != 0;
    double p_lo[3], p_hi[3], p_n[3];
    for (int c = 0; c < 3; ++c) {
        const double *p = pre + (size_t)c * (g.n + 1);
        p_n[c] = p[g.n];
        p_lo[c] = wb.ntiles > 0 ? p[wb.klo - g.k0] : 0.0;
        p_hi[c] = wb.ntiles > 0 ? p[wb.khi - g.k0 + 1] : 0.0;
    }
    double acc[kPartials];
    for (int q = 0; q < kPartials; ++q) acc[q] = 0.0;
    // each lane adds its items in increasing order; the partials of four
    // of them are loaded (at clamped indices) before any is added
    const int b0 = wbase[w], b1 = wbase[w + 1];
    for (int it0 = b0; it0 < b1; it0 += 4 * 64) {
        double v[4][kPartials];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const size_t it = (size_t)min(it0 + lane + 64 * u, b1 - 1);
#pragma unroll
            for (int q = 0; q < kPartials; ++q) v[u][q] = partial[it * kPartials + q];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (it0 + lane + 64 * u < b1)
#pragma unroll
                for (int q = 0; q < kPartials; ++q) acc[q] += v[u][q];
    }
    for (int q = 0; q < kPartials; ++q) {
        double v = acc[q];
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        acc[q] = v;
    }
    if (lane != 0) return;
    double o[7];
    if (!valid) {
        o[0] = -INFINITY;
        for (int q = 1; q < 7; ++q) o[q] = 0.0;
    } else {
        // residual form over the band (both precisions), data-only sum
        // outside it
        double dd_out = 0.0;
        for (int c = 0; c < 3; ++c) {
            if (wb.ntiles > 0) dd_out += p_lo[c] + (p_n[c] - p_hi[c]);
            else dd_out += p_n[c];
        }
        o[0] = -0.5 * (acc[0] + acc[1] + acc[2] + dd_out);
        for (int c = 0; c < 3; ++c) {
            o[1 + c] = acc[3 + c];
            o[4 + c] = acc[6 + c];
        }
    }
    if (out7)
        for (int q = 0; q < 7; ++q) out7[(size_t)w * 7 + q] = o[q];
    if (logL) logL[w] = o[0];
}

DenseArgs make_args(int B, const Modes &md, const GridDesc &g, const Work &wk, const Data &dt, int max_items)
{
    DenseArgs a;
    a.B = B;
    a.nm = md.nm;
    a.ns = g.ns;
    a.k0 = g.k0;
    a.n = g.n;
    a.steps = g.steps;
    a.tile_bins = g.tile_bins;
    a.df = g.df;
    a.max_items = max_items;
    a.one_per_walker = 0;
    a.use_ticket = 0;
    a.ticket = wk.ticket;
    a.band = wk.band;
    a.wband = wk.wband;
    a.wbase = wk.wbase;
    a.item_w = wk.item_w;
    a.item_t = wk.item_t;
    a.kf = wk.kf;
    a.kbin = wk.kbin;
    a.coef = wk.coef;
    a.d = dt.d;
    a.w = dt.w;
    a.partial = wk.partial;
    a.h = nullptr;
    a.cis_tab = wk.cis_tab;
    a.dhi32 = dt.dhi32;
    a.dlo32 = dt.dlo32;
    a.sw32 = dt.sw32;
    a.coef32 = wk.coef32;
    a.cis32 = wk.cis32;
    return a;
}

int num_cus()
{
    static int cus = 0;
    if (cus == 0) {
        int dev = 0, c = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
            c = 256;
        cus = c;
    }
    return cus;
}

// Workgroups of a dense launch: blocks_per_cu per compute unit, but never
// more than the batch can have items (B walkers of at most ceil(n / tile)
// tiles each): a workgroup past the last item would still stage the rotation
// table and take a ticket before leaving, which for a single walker cost
// more than its items.
int dense_grid(int B, const GridDesc &g, const Schedule &sch)
{
    if (sch.one_per_walker) return B;
    const long long most = (long long)B * ((g.n + g.tile_bins - 1) / g.tile_bins);
    const long long grid = (long long)num_cus() * sch.blocks_per_cu;
    return (int)std::max(1LL, std::min(grid, most));
}

// FP32 copy of the spline coefficient table
__global__ void k_coef32(const double *__restrict__ coef, float *__restrict__ coef32, long long total)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < total) coef32[i] = (float)coef[i];
}

}  // namespace

const double *cis_table_host(int *n)
{
    // cos and sin of j pi/512 from long double, rounded once to double;
    // built on first use (thread-safe static initialisation)
    struct Tab {
        double v[kCisN + 2 * kRotN];
        Tab()
        {
            const long double pi = 3.141592653589793238462643383279502884L;
            for (int i = 0; i < kCisN; ++i) v[i] = kCisHost[i];
            for (int j = 0; j < kRotN; ++j) {
                v[kCisN + 2 * j] = (double)cosl(pi * j / (kRotN / 2));
                v[kCisN + 2 * j + 1] = (double)sinl(pi * j / (kRotN / 2));
            }
        }
    };
    static const Tab tab;
    *n = kCisN + 2 * kRotN;
    return tab.v;
}

const float *cis32_table_host(int *n)
{
    *n = kCis32N;
    return kCis32Host;
}

hipError_t launch_coef32(int B, const Modes &md, const GridDesc &g, const Work &wk, hipStream_t st)
{
    if (B <= 0 || g.precision == 0) return hipSuccess;
    const long long total = (long long)B * md.nm * (g.ns - 1) * kCoefPerIv;
    k_coef32<<<(unsigned)((total + 255) / 256), 256, 0, st>>>(wk.coef, wk.coef32, total);
    return hipGetLastError();
}

hipError_t launch_setup_data(const double *psd, const double2 *d_in, double2 *d, double *w, double *pre,
                             double *scratch, float2 *dhi32, float2 *dlo32, float *sw32, const GridDesc &g,
                             double df4, hipStream_t st)
{
    const long long total = 3LL * g.n;
    const long long n_pad = data_padded(g.n);
    double *e2 = scratch;                  // [3][n]
    const int nchunks = (g.n + kScanChunk - 1) / kScanChunk;
    double *chunk = scratch + total;       // [3][nchunks]
    k_weights<<<(unsigned)((3 * n_pad + 255) / 256), 256, 0, st>>>(psd, d_in, d, w, e2, dhi32, dlo32, sw32, g.n,
                                                                   n_pad, df4);
    k_scan_chunks<<<dim3(nchunks, 3), kScanThreads, 0, st>>>(e2, g.n, chunk, nchunks);
    k_scan_offsets<<<3, kScanThreads, 0, st>>>(chunk, nchunks);
    k_scan_final<<<dim3(nchunks, 3), kScanThreads, 0, st>>>(e2, g.n, chunk, nchunks, pre);
    return hipGetLastError();
}

hipError_t launch_walker_bands(int B, const Modes &md, const GridDesc &g, const Work &wk, hipStream_t st)
{
    // a single walker's band is built with its items (launch_items), which
    // a dense launch runs first, or by the dense kernel itself (walker_one)
    if (B <= 1) return hipSuccess;
    k_walker_bands<<<(B + 127) / 128, 128, 0, st>>>(B, md.nm, g, wk.src, wk.band, wk.wband);
    k_scan_walkers<<<1, 1024, 0, st>>>(B, wk.wband, wk.wbase);
    return hipGetLastError();
}

void launch_items(int B, int nm, const GridDesc &g, const Work &wk, int max_items, hipStream_t st)
{
    if (B == 1) {
        k_items_one<<<1, 256, 0, st>>>(nm, g, wk.src, wk.band, wk.wband, wk.wbase, wk.tile_off, wk.ticket, wk.item_w,
                                       wk.item_t, max_items);
        return;
    }
    const int ntiles = (g.n + g.tile_bins - 1) / g.tile_bins;
    k_tile_count<<<ntiles, 256, 0, st>>>(B, wk.wband, wk.tile_off);
    k_tile_scan<<<1, 1024, 0, st>>>(ntiles, wk.tile_off, wk.ticket);
    k_tile_fill<<<ntiles, 256, 0, st>>>(B, wk.wband, wk.tile_off, wk.item_w, wk.item_t, max_items);
}

hipError_t launch_dense(int B, const Modes &md, const GridDesc &g, const Work &wk, const Data &dt, int max_items,
                        const Schedule &sch, bool inner, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1,
                        bool walker_one)
{
    if (B <= 0) return hipSuccess;
    walker_one = walker_one && B == 1 && !sch.one_per_walker && !inner;
    if (!walker_one) launch_items(B, md.nm, g, wk, max_items, st);
    DenseArgs a = make_args(B, md, g, wk, dt, max_items);
    a.one_per_walker = sch.one_per_walker;
    a.use_ticket = sch.one_per_walker ? 0 : 1;
    const int grid = dense_grid(B, g, sch);
    hipError_t e;
    if (ev0 && (e = hipEventRecord(ev0, st)) != hipSuccess) return e;
    if (walker_one && g.precision != 0)
        k_dense<false, true, kBinsPerLane, true, true><<<grid, kDenseThreads, 0, st>>>(a);
    else if (walker_one)
        k_dense<false, false, kBinsPerLane, true, true><<<grid, kDenseThreads, 0, st>>>(a);
    else if (g.precision != 0 && inner)
        k_dense<false, true, kBinsPerLane, false><<<grid, kDenseThreads, 0, st>>>(a);
    else if (g.precision != 0)
        k_dense<false, true, kBinsPerLane, true><<<grid, kDenseThreads, 0, st>>>(a);
    else if (inner)
        k_dense<false, false, kBinsPerLane, false><<<grid, kDenseThreads, 0, st>>>(a);
    else
        k_dense<false, false, kBinsPerLane, true><<<grid, kDenseThreads, 0, st>>>(a);
    if (ev1 && (e = hipEventRecord(ev1, st)) != hipSuccess) return e;
    return hipGetLastError();
}

const void *reduce_kernel() { return reinterpret_cast<const void *>(&k_reduce); }

hipError_t launch_reduce(int B, const GridDesc &g, const Work &wk, const Data &dt, double *out7, double *logL,
                         hipStream_t st)
{
    if (B <= 0) return hipSuccess;
    k_reduce<<<B, 64, 0, st>>>(B, g, wk.src, wk.wband, wk.wbase, wk.partial, dt.pre, out7, logL);
    return hipGetLastError();
}

// Zero fill by a kernel rather than a memset node, so that a caller may
// capture the template launch in a graph.
__global__ void k_zero2(double2 *__restrict__ h, long long count)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) h[i] = make_double2(0.0, 0.0);
}

hipError_t launch_template(const Modes &md, const GridDesc &g, const Work &wk, double2 *h, hipStream_t st)
{
    Data none = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    const long long nh = 3LL * g.n;
    k_zero2<<<(unsigned)((nh + 255) / 256), 256, 0, st>>>(h, nh);
    const int max_items = (g.n + g.tile_bins - 1) / g.tile_bins + 1;
    launch_items(1, md.nm, g, wk, max_items, st);
    DenseArgs a = make_args(1, md, g, wk, none, max_items);
    a.h = h;
    // the same step structure as the FP64 likelihood (two bins per lane, knot
    // crossings deferred alike), so each bin's modes are summed in the same
    // order and a likelihood on this template is exactly zero at its source
    k_dense<true, false, kBinsPerLane, false><<<dense_grid(1, g, Schedule()), kDenseThreads, 0, st>>>(a);
    return hipGetLastError();
}

}  // namespace mbh
