// Dense stage on the GPU: interpolation of every mode onto the dense grid,
// the per-channel template h^c(f_k) = sum_lm T^c_lm A_lm e^{i phi_lm}
// (Sec. II.A) and the noise-weighted sums of Eqs. NLL/innerprod/innerprodsum:
//   R_c  = sum_k |d_k - h_k|^2 w_k,  DH_c = sum_k Re(d_k h_k^*) w_k,
//   HH_c = sum_k |h_k|^2 w_k,        w_k = 4 df / S_c(f_k),
// over each walker's union band, plus the data-only sum outside it from
// per-channel prefix sums, so that ln L = -(R + DD_out)/2.
//
// Work decomposition: a walker's union band is cut into tiles of kTileBins
// bins; work items (walker, tile) are numbered walker-major and processed by
// a grid-stride loop.  Each item writes its 9 partial sums to its own slot,
// and one wavefront per walker adds its slots in a fixed order, so results do
// not depend on scheduling (no floating-point atomics).
#include <hip/hip_runtime.h>

#include <cmath>

#include "mbh_internal.h"

namespace mbh {
namespace {

constexpr double kInvTwoPi = 0.15915494309189533576888;
// 2 pi = kTwoPiHi + kTwoPiLo (kTwoPiHi = 2 pi rounded to double).  With
// fused multiply-adds, phi - n kTwoPiHi - n kTwoPiLo is accurate to a few
// 1e-16 rad for the |n| < 2^23 of phases below ~5e7 rad.
constexpr double kTwoPiHi = 6.283185307179586232;
constexpr double kTwoPiLo = 2.4492935982947064e-16;

// ---------------------------------------------------------------------------
// Setup: w = 4 df / S and per-channel prefix sums of |d|^2 w.
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanPer = 8;
constexpr int kScanChunk = kScanThreads * kScanPer;

__global__ void k_weights(const double *__restrict__ psd, const double2 *__restrict__ d, double *__restrict__ w,
                          double *__restrict__ e2, long long total, double df4)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const double wi = df4 / psd[i];
    w[i] = wi;
    const double2 di = d[i];
    e2[i] = (di.x * di.x + di.y * di.y) * wi;
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
    WalkerBand r;
    r.klo = 0;
    r.khi = -1;
    r.tile_lo = 0;
    r.ntiles = 0;
    if (src[w].valid) {
        int lo = 0x7fffffff, hi = -1;
        for (int im = 0; im < nm; ++im) {
            const ModeBand b = band[w * nm + im];
            if (!b.active) continue;
            lo = min(lo, b.klo);
            hi = max(hi, b.khi);
        }
        if (hi >= lo) {
            r.klo = lo;
            r.khi = hi;
            r.tile_lo = (lo - g.k0) / kTileBins;
            r.ntiles = (hi - g.k0) / kTileBins - r.tile_lo + 1;
        }
    }
    wb[w] = r;
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

__global__ void k_fill_items(int B, const WalkerBand *__restrict__ wb, const int *__restrict__ wbase,
                             int *__restrict__ item_w, int max_items)
{
    const int w = blockIdx.x;
    if (w >= B) return;
    const int base = wbase[w], nt = wb[w].ntiles;
    for (int j = threadIdx.x; j < nt; j += blockDim.x)
        if (base + j < max_items) item_w[base + j] = w;
}

// ---------------------------------------------------------------------------
// Dense interpolation + inner products.
// ---------------------------------------------------------------------------
struct DenseArgs {
    int B, nm, ns, k0, n;
    double df;
    int max_items;
    const ModeBand *band;
    const WalkerBand *wband;
    const int *wbase;
    const int *item_w;
    const double *kf;
    const double *coef;
    const double2 *d;
    const double *w;
    double *partial;
    double2 *h;          // template output (WriteH only)
};

// Largest knot index i with kf[i] <= f (clamped to [0, ns-2]), starting from
// the log-spacing estimate.
__device__ inline int locate(const double *kf, int ns, double fs, double fe, double f)
{
    int i = (int)floor(log(f / fs) / log(fe / fs) * (double)(ns - 1));
    i = max(0, min(ns - 2, i));
    while (i > 0 && kf[i] > f) --i;
    while (i < ns - 2 && kf[i + 1] <= f) ++i;
    return i;
}

__device__ inline double horner(const double *c, double x) { return c[0] + x * (c[1] + x * (c[2] + x * c[3])); }

// e^{i phi} with the phase first reduced to [-pi, pi].
__device__ inline void cis_reduced(double phi, double &s, double &c)
{
    const double nq = rint(phi * kInvTwoPi);
    double r = fma(-nq, kTwoPiHi, phi);
    r = fma(-nq, kTwoPiLo, r);
    sincos(r, &s, &c);
}

template <bool kWriteH>
__global__ __launch_bounds__(kDenseThreads) void k_dense(DenseArgs a)
{
    __shared__ double red[kDenseThreads / 64][kPartials];
    const int total = min(a.wbase[a.B], a.max_items);
    const int tid = threadIdx.x;
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int wk = a.item_w[item];
        const WalkerBand wb = a.wband[wk];
        const int tile = wb.tile_lo + (item - a.wbase[wk]);
        const int kb = a.k0 + tile * kTileBins;

        double hr[kDenseJ][3], hi[kDenseJ][3];
#pragma unroll
        for (int j = 0; j < kDenseJ; ++j)
#pragma unroll
            for (int c = 0; c < 3; ++c) hr[j][c] = hi[j][c] = 0.0;

        for (int im = 0; im < a.nm; ++im) {
            const ModeBand mb = a.band[wk * a.nm + im];
            if (!mb.active || mb.khi < kb || mb.klo >= kb + kTileBins) continue;
            const double *kf = a.kf + (size_t)(wk * a.nm + im) * a.ns;
            const double *cf = a.coef + (size_t)(wk * a.nm + im) * (a.ns - 1) * kCoefPerIv;
            int iv = -1;
#pragma unroll
            for (int j = 0; j < kDenseJ; ++j) {
                const int k = kb + tid + kDenseThreads * j;
                if (k < mb.klo || k > mb.khi) continue;
                const double f = (double)k * a.df;
                if (iv < 0) iv = locate(kf, a.ns, mb.fs, mb.fe, f);
                else while (iv < a.ns - 2 && kf[iv + 1] <= f) ++iv;
                const double dx = f - kf[iv];
                const double *c = cf + (size_t)iv * kCoefPerIv;
                const double amp = horner(c + 0, dx);
                const double ph = horner(c + 4, dx);
                double sn, cs;
                cis_reduced(ph, sn, cs);
                const double ar = amp * cs, ai = amp * sn;
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    const double tr = horner(c + 8 + 8 * ch, dx);
                    const double ti = horner(c + 12 + 8 * ch, dx);
                    hr[j][ch] += tr * ar - ti * ai;
                    hi[j][ch] += tr * ai + ti * ar;
                }
            }
        }

        if (kWriteH) {
#pragma unroll
            for (int j = 0; j < kDenseJ; ++j) {
                const int k = kb + tid + kDenseThreads * j;
                if (k < wb.klo || k > wb.khi) continue;
                const int idx = k - a.k0;
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) a.h[(size_t)ch * a.n + idx] = make_double2(hr[j][ch], hi[j][ch]);
            }
            continue;
        }

        double acc[kPartials];
#pragma unroll
        for (int q = 0; q < kPartials; ++q) acc[q] = 0.0;
#pragma unroll
        for (int j = 0; j < kDenseJ; ++j) {
            const int k = kb + tid + kDenseThreads * j;
            if (k < wb.klo || k > wb.khi) continue;
            const int idx = k - a.k0;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                const double2 dv = a.d[(size_t)ch * a.n + idx];
                const double wv = a.w[(size_t)ch * a.n + idx];
                const double rr = dv.x - hr[j][ch], ri = dv.y - hi[j][ch];
                acc[ch] += (rr * rr + ri * ri) * wv;
                acc[3 + ch] += (dv.x * hr[j][ch] + dv.y * hi[j][ch]) * wv;
                acc[6 + ch] += (hr[j][ch] * hr[j][ch] + hi[j][ch] * hi[j][ch]) * wv;
            }
        }
        // wavefront butterfly, then the four wavefronts in order
#pragma unroll
        for (int q = 0; q < kPartials; ++q) {
            double v = acc[q];
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
            acc[q] = v;
        }
        const int wave = tid >> 6, lane = tid & 63;
        if (lane == 0)
#pragma unroll
            for (int q = 0; q < kPartials; ++q) red[wave][q] = acc[q];
        __syncthreads();
        if (tid < kPartials) {
            double s = 0.0;
#pragma unroll
            for (int wv = 0; wv < kDenseThreads / 64; ++wv) s += red[wv][tid];
            a.partial[(size_t)item * kPartials + tid] = s;
        }
        __syncthreads();
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
    double acc[kPartials];
    for (int q = 0; q < kPartials; ++q) acc[q] = 0.0;
    const int b0 = wbase[w], b1 = wbase[w + 1];
    for (int it = b0 + lane; it < b1; it += 64)
        for (int q = 0; q < kPartials; ++q) acc[q] += partial[(size_t)it * kPartials + q];
    for (int q = 0; q < kPartials; ++q) {
        double v = acc[q];
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        acc[q] = v;
    }
    if (lane != 0) return;
    double o[7];
    if (!src[w].valid) {
        o[0] = -INFINITY;
        for (int q = 1; q < 7; ++q) o[q] = 0.0;
    } else {
        const WalkerBand wb = wband[w];
        double dd_out = 0.0;
        for (int c = 0; c < 3; ++c) {
            const double *p = pre + (size_t)c * (g.n + 1);
            if (wb.ntiles > 0) dd_out += p[wb.klo - g.k0] + (p[g.n] - p[wb.khi - g.k0 + 1]);
            else dd_out += p[g.n];
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
    a.df = g.df;
    a.max_items = max_items;
    a.band = wk.band;
    a.wband = wk.wband;
    a.wbase = wk.wbase;
    a.item_w = wk.item_w;
    a.kf = wk.kf;
    a.coef = wk.coef;
    a.d = dt.d;
    a.w = dt.w;
    a.partial = wk.partial;
    a.h = nullptr;
    return a;
}

int dense_grid()
{
    static int grid = 0;
    if (grid == 0) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        grid = cus * 8;
    }
    return grid;
}

}  // namespace

hipError_t launch_setup_data(const double *psd, const double2 *d, double *w, double *pre, double *scratch,
                             const GridDesc &g, double df4, hipStream_t st)
{
    const long long total = 3LL * g.n;
    double *e2 = scratch;                  // [3][n]
    const int nchunks = (g.n + kScanChunk - 1) / kScanChunk;
    double *chunk = scratch + total;       // [3][nchunks]
    k_weights<<<(unsigned)((total + 255) / 256), 256, 0, st>>>(psd, d, w, e2, total, df4);
    k_scan_chunks<<<dim3(nchunks, 3), kScanThreads, 0, st>>>(e2, g.n, chunk, nchunks);
    k_scan_offsets<<<3, kScanThreads, 0, st>>>(chunk, nchunks);
    k_scan_final<<<dim3(nchunks, 3), kScanThreads, 0, st>>>(e2, g.n, chunk, nchunks, pre);
    return hipGetLastError();
}

hipError_t launch_walker_bands(int B, const Modes &md, const GridDesc &g, const Work &wk, hipStream_t st)
{
    if (B <= 0) return hipSuccess;
    k_walker_bands<<<(B + 127) / 128, 128, 0, st>>>(B, md.nm, g, wk.src, wk.band, wk.wband);
    k_scan_walkers<<<1, 1024, 0, st>>>(B, wk.wband, wk.wbase);
    return hipGetLastError();
}

hipError_t launch_dense(int B, const Modes &md, const GridDesc &g, const Work &wk, const Data &dt, int max_items,
                        hipStream_t st, hipEvent_t ev0, hipEvent_t ev1)
{
    if (B <= 0) return hipSuccess;
    k_fill_items<<<B, 256, 0, st>>>(B, wk.wband, wk.wbase, wk.item_w, max_items);
    DenseArgs a = make_args(B, md, g, wk, dt, max_items);
    hipError_t e;
    if (ev0 && (e = hipEventRecord(ev0, st)) != hipSuccess) return e;
    k_dense<false><<<dense_grid(), kDenseThreads, 0, st>>>(a);
    if (ev1 && (e = hipEventRecord(ev1, st)) != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t launch_reduce(int B, const GridDesc &g, const Work &wk, const Data &dt, double *out7, double *logL,
                         hipStream_t st)
{
    if (B <= 0) return hipSuccess;
    k_reduce<<<B, 64, 0, st>>>(B, g, wk.src, wk.wband, wk.wbase, wk.partial, dt.pre, out7, logL);
    return hipGetLastError();
}

hipError_t launch_template(const Modes &md, const GridDesc &g, const Work &wk, double2 *h, hipStream_t st)
{
    Data none = {nullptr, nullptr, nullptr};
    const int max_items = (g.n + kTileBins - 1) / kTileBins + 1;
    k_fill_items<<<1, 256, 0, st>>>(1, wk.wband, wk.wbase, wk.item_w, max_items);
    DenseArgs a = make_args(1, md, g, wk, none, max_items);
    a.h = h;
    k_dense<true><<<dense_grid(), kDenseThreads, 0, st>>>(a);
    return hipGetLastError();
}

}  // namespace mbh
