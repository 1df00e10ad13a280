// Learned proposal: an affine-coupling normalizing flow with hand-written
// forward, inverse, backward and Adam kernels (the C ABI is in include/mbh.h).
//
// The flow gives the sampler an independence proposal that it can both draw
// from and evaluate; the ensemble stretch move with parallel tempering
// (Sec. III.A) stays the workhorse and the flow is mixed in as an extra
// Metropolis-Hastings move.  Each coupling layer keeps nc coordinates and
// maps the other nt = dim - nc as y = x exp(s) + t, with (s, t) from a
// two-hidden-layer tanh MLP of the kept coordinates, so the log-Jacobian is
// the sum of s.
//
// Kernel layout.  Rows (samples) are processed kS = 16 at a time per
// workgroup; the MLP of a layer then runs as small matrix products in which
// thread j owns hidden unit j for all 16 rows: weights are stored
// input-major so that thread j reads W[i][j] coalesced, and the activations
// of the 16 rows sit in LDS transposed ([unit][row]) so that one 16-byte LDS
// broadcast feeds four FMAs.  Training stores, per layer, the layer input,
// both hidden activations and s; the backward kernel turns them into
// per-row gradients of the pre-activations, and the parameter gradient is a
// sum over rows computed in fixed-size row chunks (partials in FP64) that
// are then summed in chunk order, so every result is bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mbh.h"

namespace {

constexpr int kS = 16;            // rows per workgroup
constexpr int kMaxDim = 32;
constexpr int kMaxNt = kMaxDim / 2;
constexpr int kMaxO = 2 * kMaxNt;
constexpr int kMaxH = 256;
constexpr int kMaxLayers = 32;
constexpr int kMaxBatch = 1 << 20;
constexpr int kMaxChunks = 64;    // parameter-gradient row chunks
constexpr int kMinChunk = 256;
constexpr float kHalfLog2Pi = 0.91893853320467274178f;

struct FlowArgs {
    int dim, L, H, n, ntmax;
    const int *perm;         // [L][dim]
    const int *nc;           // [L]
    const long long *off;    // [L+1] first parameter of each layer
    const float *params;
};

struct LayerW {
    int nc, nt, no;
    const int *p;
    const float *W1, *b1, *W2, *b2, *W3, *b3;
};

__device__ __forceinline__ LayerW layer_w(const FlowArgs &a, int l)
{
    LayerW w;
    w.nc = a.nc[l];
    w.nt = a.dim - w.nc;
    w.no = 2 * w.nt;
    w.p = a.perm + l * a.dim;
    w.W1 = a.params + a.off[l];
    w.b1 = w.W1 + w.nc * a.H;
    w.W2 = w.b1 + a.H;
    w.b2 = w.W2 + a.H * a.H;
    w.W3 = w.b2 + a.H;
    w.b3 = w.W3 + a.H * w.no;
    return w;
}

// The backward kernel reads rows of W1, W2 and W3 kU at a time into
// registers, the next batch issued before the current one is used, so that a
// thread has up to 2 kU loads in flight instead of one dependent load per
// multiply-add.  The order of the multiply-adds is unchanged.
constexpr int kU = 16;
static_assert(kMaxO <= 2 * kU, "a row of the output map must fit two weight batches");

// w[q] = row[j0 + q]; entries at or past jmax (>= 1) load entry jmax - 1
// instead, so a batch is kU loads with no branch or select that would wait
// for them (the caller skips those entries).
__device__ __forceinline__ void load_run(float (&w)[kU], const float *__restrict__ row, int j0, int jmax)
{
#pragma unroll
    for (int q = 0; q < kU; ++q) w[q] = row[min(j0 + q, jmax - 1)];
}

// acc[s] += w * v[s] for the 16 rows of one LDS column v (16-byte aligned).
__device__ __forceinline__ void fma16(float (&acc)[kS], float w, const float *v)
{
    const float4 *v4 = reinterpret_cast<const float4 *>(v);
#pragma unroll
    for (int q = 0; q < kS / 4; ++q) {
        const float4 x = v4[q];
        acc[4 * q + 0] = fmaf(w, x.x, acc[4 * q + 0]);
        acc[4 * q + 1] = fmaf(w, x.y, acc[4 * q + 1]);
        acc[4 * q + 2] = fmaf(w, x.z, acc[4 * q + 2]);
        acc[4 * q + 3] = fmaf(w, x.w, acc[4 * q + 3]);
    }
}

// Weights of one layer staged in LDS by the pass kernel: W1 [nc][H] and b1,
// then b2, W3 [H][no] and b3 (two contiguous runs of the parameter array).
// W2 [H][H] stays in global memory and is read column by column in batches.
__host__ __device__ inline int stage_floats(int nc, int H, int no) { return nc * H + 2 * H + H * no + no; }
constexpr int kPassThreads = 256;
constexpr size_t kPassStaticLds = 8192;   // bound on the pass kernel's static LDS
constexpr int kStageBatch = 16;           // staged floats per thread per round of loads
// The second hidden layer, h2 = tanh(h1 W2 + b2) for the workgroup's 16 rows,
// is a [16 x H] x [H x H] product: it runs on the matrix cores as 16 x 16
// output tiles (v_mfma_f32_16x16x4f32, FP32 in and out), K in items of
// kKSteps steps of 4.  Lane l of a wavefront supplies A[i][k] = h1 of row
// l % 16, unit k0 + l / 16, and B[k][j] = W2[k0 + l / 16][j0 + l % 16], and
// receives D[4 (l / 16) + v][j0 + l % 16], v = 0..3.
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kKSteps = 32;
constexpr int kKItem = 4 * kKSteps;   // rows of W2 per item
constexpr int kWaves = kPassThreads / 64;
__host__ __device__ inline int h_padded(int H) { return (H + kKItem - 1) / kKItem * kKItem; }

// B operand of item (tile t, K block kb): rows and columns past H repeat
// row / column H - 1; the rows meet zero padding of h1, the columns are
// never written.
__device__ __forceinline__ void load_w2_item(float (&b)[kKSteps], const float *__restrict__ W2, int H, int t,
                                             int kb, int ln)
{
    const int col = min(t * 16 + (ln & 15), H - 1);
    const int r0 = kb * kKItem + (ln >> 4);
#pragma unroll
    for (int q = 0; q < kKSteps; ++q) b[q] = W2[(size_t)min(r0 + 4 * q, H - 1) * H + col];
}

// acc += h1[rows][kb block] x W2[kb block][tile] (h1t is [unit][row], zero past H)
__device__ __forceinline__ void mfma_item(f32x4 &acc, const float (&b)[kKSteps], const float *h1t, int kb, int ln)
{
    const float *a = h1t + (size_t)(kb * kKItem + (ln >> 4)) * kS + (ln & 15);
#pragma unroll
    for (int q = 0; q < kKSteps; ++q) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[4 * q * kS], b[q], acc, 0, 0, 0);
}

// One pass through all layers for kS rows: forward (u -> z) or inverse
// (z -> u).  With kStore (forward only) the per-layer inputs X[l], hidden
// activations H1[l], H2[l] and scales SV[l] are written for the backward
// pass, X[L] = z, and logq goes to 'logq'.
//
// A pass over a few hundred rows runs a handful of workgroups, so its time
// is the chain of dependent steps through the layers, and every global read
// waits for memory beyond L2 (the L2 does not keep the weights from one
// launch to the next).  Hence, per layer: one burst of loads stages the
// small weights (W1, W3, biases, the permutation) in LDS and loads each
// wavefront's first two W2 items into registers.  For the first hidden
// layer the kS rows are split between kS / kR groups of H threads, thread
// (group g, unit j) computing unit j for rows g kR .. g kR + kR - 1 (the
// results do not depend on kR).  The second hidden layer runs on the matrix
// cores (above), the four wavefronts taking every fourth output tile, with
// the next W2 item in flight while one is multiplied.
template <bool kInv, bool kStore, int kR>
__global__ __launch_bounds__(kPassThreads) void k_flow_pass(FlowArgs a, const float *__restrict__ in,
                                                            float *__restrict__ out, float *__restrict__ logq,
                                                            float *__restrict__ X, float *__restrict__ H1,
                                                            float *__restrict__ H2, float *__restrict__ SV)
{
    static_assert(kS % kR == 0 && kR % 4 == 0, "row groups of whole float4 columns");
    constexpr int kG = kS / kR;
    __shared__ float xs[kS][kMaxDim];
    __shared__ float ob[kS][kMaxO];
    __shared__ float ld[kS];
    __shared__ float sq[kS];
    __shared__ int lnc[kMaxLayers];
    __shared__ long long loff[kMaxLayers];
    __shared__ int lperm[kMaxDim];
    extern __shared__ float4 dyn4[];
    const int tid = threadIdx.x;
    const int row0 = blockIdx.x * kS;
    const int dim = a.dim, H = a.H, n = a.n, Hp = h_padded(H);
    float *h1t = reinterpret_cast<float *>(dyn4);   // [Hp][kS], rows H.. Hp-1 zero
    float *h2t = h1t + Hp * kS;                      // [H][kS]
    float *wsm = h2t + H * kS;                       // staged weights of the current layer
    // thread -> (row group, hidden unit); threads beyond kG H only help with the staging
    const int grp = tid / H, j = tid - grp * H;
    const bool unit = grp < kG;
    const int rg = grp * kR;
    // wavefront -> output tiles wv, wv + kWaves, ... of the second hidden layer
    const int wv = tid >> 6, ln = tid & 63;
    const int ntile = (H + 15) / 16, nkb = h_padded(H) / kKItem;
    const int nit = (wv < ntile ? (ntile - wv + kWaves - 1) / kWaves : 0) * nkb;

    for (int e = tid; e < kS * dim; e += kPassThreads) {
        const int s = e / dim, c = e - s * dim, r = row0 + s;
        xs[s][c] = r < n ? in[(size_t)r * dim + c] : 0.f;
    }
    if (tid < a.L) {
        lnc[tid] = a.nc[tid];
        loff[tid] = a.off[tid];
    }
    for (int e = H * kS + tid; e < Hp * kS; e += kPassThreads) h1t[e] = 0.f;
    if (tid < kS) ld[tid] = 0.f;
    __syncthreads();
    if (kInv && tid < kS) {
        float q = 0.f;
        for (int c = 0; c < dim; ++c) q = fmaf(xs[tid][c], xs[tid][c], q);
        sq[tid] = q;
    }

    for (int li = 0; li < a.L; ++li) {
        const int l = kInv ? a.L - 1 - li : li;
        const int nc = lnc[l], nt = dim - nc, no = 2 * nt;
        const float *gw = a.params + loff[l];
        const float *W2 = gw + nc * H + H;
        const int len1 = nc * H + H, len2 = H + H * no + no, tot = len1 + len2;
        // burst: the permutation, the first two W2 items and the staged weights
        const int pv = tid < dim ? a.perm[l * dim + tid] : 0;
        float bA[kKSteps], bB[kKSteps];
        if (nit > 0) load_w2_item(bA, W2, H, wv, 0, ln);
        if (nit > 1) load_w2_item(bB, W2, H, wv + kWaves * (1 / nkb), 1 % nkb, ln);
        for (int e0 = tid; e0 < tot; e0 += kStageBatch * kPassThreads) {
            float v[kStageBatch];
#pragma unroll
            for (int q = 0; q < kStageBatch; ++q) {
                const int e = min(e0 + q * kPassThreads, tot - 1);
                v[q] = *(e < len1 ? gw + e : W2 + (size_t)H * H + (e - len1));
            }
#pragma unroll
            for (int q = 0; q < kStageBatch; ++q) {
                const int e = e0 + q * kPassThreads;
                if (e < tot) wsm[e] = v[q];
            }
        }
        if (tid < dim) lperm[tid] = pv;
        if (kStore) {
            for (int e = tid; e < kS * dim; e += kPassThreads) {
                const int s = e / dim, c = e - s * dim, r = row0 + s;
                if (r < n) X[((size_t)l * n + r) * dim + c] = xs[s][c];
            }
        }
        __syncthreads();
        const float *W1s = wsm, *b1s = wsm + nc * H, *b2s = wsm + len1, *W3s = b2s + H, *b3s = W3s + H * no;
        // h1 = tanh(x_c W1 + b1)
        if (unit) {
            float acc[kR];
            const float bj = b1s[j];
#pragma unroll
            for (int r = 0; r < kR; ++r) acc[r] = bj;
            for (int i = 0; i < nc; ++i) {
                const float wij = W1s[i * H + j];
                const int c = lperm[i];
#pragma unroll
                for (int r = 0; r < kR; ++r) acc[r] = fmaf(wij, xs[rg + r][c], acc[r]);
            }
#pragma unroll
            for (int r = 0; r < kR; ++r) {
                const float h = tanhf(acc[r]);
                h1t[j * kS + rg + r] = h;
                if (kStore && row0 + rg + r < n) H1[((size_t)l * n + row0 + rg + r) * H + j] = h;
            }
        }
        __syncthreads();
        // h2 = tanh(h1 W2 + b2): items (tile wv + kWaves m, K block kb) in order
        {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            auto item = [&](int it, const float(&b)[kKSteps]) {
                const int t = wv + kWaves * (it / nkb), kb = it % nkb;
                const int col = t * 16 + (ln & 15);
                if (kb == 0) {
                    const float bj = b2s[min(col, H - 1)];
                    acc = f32x4{bj, bj, bj, bj};
                }
                mfma_item(acc, b, h1t, kb, ln);
                if (kb == nkb - 1 && col < H) {
                    const int r4 = 4 * (ln >> 4);
                    float4 h;
                    h.x = tanhf(acc[0]);
                    h.y = tanhf(acc[1]);
                    h.z = tanhf(acc[2]);
                    h.w = tanhf(acc[3]);
                    *reinterpret_cast<float4 *>(&h2t[col * kS + r4]) = h;
                    if (kStore) {
                        const float hv[4] = {h.x, h.y, h.z, h.w};
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            if (row0 + r4 + v < n) H2[((size_t)l * n + row0 + r4 + v) * H + col] = hv[v];
                    }
                }
            };
            for (int it = 0; it < nit; it += 2) {
                item(it, bA);
                if (it + 2 < nit) load_w2_item(bA, W2, H, wv + kWaves * ((it + 2) / nkb), (it + 2) % nkb, ln);
                if (it + 1 < nit) {
                    item(it + 1, bB);
                    if (it + 3 < nit) load_w2_item(bB, W2, H, wv + kWaves * ((it + 3) / nkb), (it + 3) % nkb, ln);
                }
            }
        }
        __syncthreads();
        // o = h2 W3 + b3
        for (int e = tid; e < kS * no; e += kPassThreads) {
            const int s = e / no, k = e - s * no;
            float acc = b3s[k];
            for (int i = 0; i < H; ++i) acc = fmaf(h2t[i * kS + s], W3s[i * no + k], acc);
            ob[s][k] = acc;
        }
        __syncthreads();
        // y_t = x_t exp(s) + t  (inverse: x_t = (y_t - t) exp(-s)); ob[s][j] <- s
        for (int e = tid; e < kS * nt; e += kPassThreads) {
            const int s = e / nt, jj = e - s * nt;
            const float sv = tanhf(ob[s][jj]);
            const float t = ob[s][nt + jj];
            const int c = lperm[nc + jj];
            const float x = xs[s][c];
            xs[s][c] = kInv ? (x - t) * expf(-sv) : fmaf(x, expf(sv), t);
            ob[s][jj] = sv;
            if (kStore && row0 + s < n) SV[((size_t)l * n + row0 + s) * a.ntmax + jj] = sv;
        }
        __syncthreads();
        if (tid < kS) {
            float acc = ld[tid];
            for (int jj = 0; jj < nt; ++jj) acc += ob[tid][jj];
            ld[tid] = acc;
        }
        __syncthreads();
    }

    for (int e = tid; e < kS * dim; e += kPassThreads) {
        const int s = e / dim, c = e - s * dim, r = row0 + s;
        if (r < n) {
            if (out) out[(size_t)r * dim + c] = xs[s][c];
            if (kStore) X[((size_t)a.L * n + r) * dim + c] = xs[s][c];
        }
    }
    if (tid < kS && row0 + tid < n && logq) {
        float q;
        if (kInv) {
            q = sq[tid];
        } else {
            q = 0.f;
            for (int c = 0; c < dim; ++c) q = fmaf(xs[tid][c], xs[tid][c], q);
        }
        logq[row0 + tid] = -0.5f * q - dim * kHalfLog2Pi + ld[tid];
    }
}

// Launch of the pass kernel for H hidden units: row groups of 8 when two
// groups of H threads fit the workgroup, else one group of 16.
template <bool kInv, bool kStore>
hipError_t launch_pass(const FlowArgs &a, int H, size_t lds, const float *in, float *out, float *logq, float *X,
                       float *H1, float *H2, float *SV, hipStream_t st)
{
    const unsigned blocks = (unsigned)((a.n + kS - 1) / kS);
    if (2 * H <= kPassThreads)
        k_flow_pass<kInv, kStore, kS / 2><<<blocks, kPassThreads, lds, st>>>(a, in, out, logq, X, H1, H2, SV);
    else
        k_flow_pass<kInv, kStore, kS><<<blocks, kPassThreads, lds, st>>>(a, in, out, logq, X, H1, H2, SV);
    return hipGetLastError();
}

// Per-row backward pass of loss = -(1/n) sum log q: writes the gradients of
// the loss with respect to the MLP outputs (Go), and the pre-activations of
// both hidden layers (Gp2, Gp1), layer by layer from the last.
__global__ __launch_bounds__(256) void k_flow_back(FlowArgs a, const float *__restrict__ X,
                                                   const float *__restrict__ H1, const float *__restrict__ H2,
                                                   const float *__restrict__ SV, float *__restrict__ Go,
                                                   float *__restrict__ Gp1, float *__restrict__ Gp2, float inv_n)
{
    __shared__ float xin[kS][kMaxDim];
    __shared__ float gx[kS][kMaxDim];
    __shared__ float sv[kS][kMaxNt];
    __shared__ float gob[kS][kMaxO];
    __shared__ __align__(16) float h1t[kMaxH * kS];   // h1, then d loss / d pre1
    __shared__ __align__(16) float h2t[kMaxH * kS];   // h2, then d loss / d pre2

    const int tid = threadIdx.x, nth = blockDim.x;
    const int row0 = blockIdx.x * kS;
    const int dim = a.dim, H = a.H, n = a.n, omax = 2 * a.ntmax;
    // d loss / d z = z / n
    for (int e = tid; e < kS * dim; e += nth) {
        const int s = e / dim, c = e - s * dim, r = row0 + s;
        gx[s][c] = r < n ? X[((size_t)a.L * n + r) * dim + c] * inv_n : 0.f;
    }
    for (int l = a.L - 1; l >= 0; --l) {
        const LayerW w = layer_w(a, l);
        for (int e = tid; e < kS * dim; e += nth) {
            const int s = e / dim, c = e - s * dim, r = row0 + s;
            xin[s][c] = r < n ? X[((size_t)l * n + r) * dim + c] : 0.f;
        }
        for (int e = tid; e < kS * w.nt; e += nth) {
            const int s = e / w.nt, j = e - s * w.nt, r = row0 + s;
            sv[s][j] = r < n ? SV[((size_t)l * n + r) * a.ntmax + j] : 0.f;
        }
        for (int j = tid; j < H; j += nth) {
#pragma unroll
            for (int s = 0; s < kS; ++s) {
                const bool ok = row0 + s < n;
                const size_t idx = ((size_t)l * n + row0 + s) * H + j;
                h1t[j * kS + s] = ok ? H1[idx] : 0.f;
                h2t[j * kS + s] = ok ? H2[idx] : 0.f;
            }
        }
        __syncthreads();
        // Coupling: y = x e^s + t, s = tanh(o_s), t = o_t; the log-det term
        // contributes -1/n to every d loss / d s.
        for (int e = tid; e < kS * w.nt; e += nth) {
            const int s = e / w.nt, j = e - s * w.nt, r = row0 + s;
            const int c = w.p[w.nc + j];
            const float sj = sv[s][j];
            const float ex = expf(sj);
            const float gy = gx[s][c];
            const float gs = r < n ? fmaf(gy * xin[s][c], ex, -inv_n) : 0.f;
            const float go_s = gs * (1.f - sj * sj);
            gob[s][j] = go_s;
            gob[s][w.nt + j] = gy;
            gx[s][c] = gy * ex;
            if (r < n) {
                Go[((size_t)l * n + r) * omax + j] = go_s;
                Go[((size_t)l * n + r) * omax + w.nt + j] = gy;
            }
        }
        __syncthreads();
        // d loss / d pre2 = (W3 go) * (1 - h2^2), in place over h2
        for (int j = tid; j < H; j += nth) {
            const float *w3 = w.W3 + j * w.no;
            float wa[kU], wb[kU];
            load_run(wa, w3, 0, w.no);
            load_run(wb, w3, kU, w.no);
#pragma unroll
            for (int s = 0; s < kS; ++s) {
                float acc = 0.f;
#pragma unroll
                for (int k = 0; k < kU; ++k)
                    if (k < w.no) acc = fmaf(wa[k], gob[s][k], acc);
#pragma unroll
                for (int k = 0; k < kU; ++k)
                    if (kU + k < w.no) acc = fmaf(wb[k], gob[s][kU + k], acc);
                const float h = h2t[j * kS + s];
                const float g = acc * (1.f - h * h);
                h2t[j * kS + s] = g;
                if (row0 + s < n) Gp2[((size_t)l * n + row0 + s) * H + j] = g;
            }
        }
        __syncthreads();
        // d loss / d pre1 = (W2 gp2) * (1 - h1^2), in place over h1
        for (int i = tid; i < H; i += nth) {
            float acc[kS];
#pragma unroll
            for (int s = 0; s < kS; ++s) acc[s] = 0.f;
            const float *w2 = w.W2 + (size_t)i * H;
            float wa[kU], wb[kU];
            load_run(wa, w2, 0, H);
            for (int j0 = 0; j0 < H; j0 += 2 * kU) {
                load_run(wb, w2, j0 + kU, H);
#pragma unroll
                for (int q = 0; q < kU; ++q)
                    if (j0 + q < H) fma16(acc, wa[q], &h2t[(j0 + q) * kS]);
                load_run(wa, w2, j0 + 2 * kU, H);
#pragma unroll
                for (int q = 0; q < kU; ++q)
                    if (j0 + kU + q < H) fma16(acc, wb[q], &h2t[(j0 + kU + q) * kS]);
            }
#pragma unroll
            for (int s = 0; s < kS; ++s) {
                const float h = h1t[i * kS + s];
                const float g = acc[s] * (1.f - h * h);
                h1t[i * kS + s] = g;
                if (row0 + s < n) Gp1[((size_t)l * n + row0 + s) * H + i] = g;
            }
        }
        __syncthreads();
        // Kept coordinates: pass-through gradient plus W1 gp1.
        for (int e = tid; e < kS * w.nc; e += nth) {
            const int s = e / w.nc, i = e - s * w.nc;
            const float *w1 = w.W1 + (size_t)i * H;
            float acc = 0.f;
            float wa[kU], wb[kU];
            load_run(wa, w1, 0, H);
            for (int j0 = 0; j0 < H; j0 += 2 * kU) {
                load_run(wb, w1, j0 + kU, H);
#pragma unroll
                for (int q = 0; q < kU; ++q)
                    if (j0 + q < H) acc = fmaf(wa[q], h1t[(j0 + q) * kS + s], acc);
                load_run(wa, w1, j0 + 2 * kU, H);
#pragma unroll
                for (int q = 0; q < kU; ++q)
                    if (j0 + kU + q < H) acc = fmaf(wb[q], h1t[(j0 + kU + q) * kS + s], acc);
            }
            gx[s][w.p[i]] += acc;
        }
        __syncthreads();
    }
}

// Parameter gradient: for parameter q and row chunk blockIdx.y, the FP64 sum
// over the chunk's rows (in row order) of activation x upstream gradient.
__global__ __launch_bounds__(256) void k_flow_wgrad(FlowArgs a, const float *__restrict__ X,
                                                    const float *__restrict__ H1, const float *__restrict__ H2,
                                                    const float *__restrict__ Go, const float *__restrict__ Gp1,
                                                    const float *__restrict__ Gp2, int chunk, long long P,
                                                    double *__restrict__ partial)
{
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= P) return;
    const int n = a.n, H = a.H, dim = a.dim, omax = 2 * a.ntmax;
    const int r0 = blockIdx.y * chunk;
    const int r1 = min(n, r0 + chunk);
    int l = 0;
    while (l + 1 < a.L && q >= a.off[l + 1]) ++l;
    const int nc = a.nc[l], no = 2 * (dim - nc);
    long long k = q - a.off[l];
    const size_t lrow = (size_t)l * n;
    double acc = 0.0;
    if (k < (long long)nc * H) {                       // W1[i][j]
        const int i = (int)(k / H), j = (int)(k % H);
        const int c = a.perm[l * dim + i];
        for (int r = r0; r < r1; ++r)
            acc += (double)X[(lrow + r) * dim + c] * (double)Gp1[(lrow + r) * H + j];
    } else if ((k -= (long long)nc * H) < H) {          // b1[j]
        for (int r = r0; r < r1; ++r) acc += (double)Gp1[(lrow + r) * H + k];
    } else if ((k -= H) < (long long)H * H) {           // W2[i][j]
        const int i = (int)(k / H), j = (int)(k % H);
        for (int r = r0; r < r1; ++r)
            acc += (double)H1[(lrow + r) * H + i] * (double)Gp2[(lrow + r) * H + j];
    } else if ((k -= (long long)H * H) < H) {           // b2[j]
        for (int r = r0; r < r1; ++r) acc += (double)Gp2[(lrow + r) * H + k];
    } else if ((k -= H) < (long long)H * no) {          // W3[i][k]
        const int i = (int)(k / no), o = (int)(k % no);
        for (int r = r0; r < r1; ++r)
            acc += (double)H2[(lrow + r) * H + i] * (double)Go[(lrow + r) * omax + o];
    } else {                                            // b3[k]
        k -= (long long)H * no;
        for (int r = r0; r < r1; ++r) acc += (double)Go[(lrow + r) * omax + k];
    }
    partial[(size_t)blockIdx.y * P + q] = acc;
}

__global__ void k_flow_gsum(const double *__restrict__ partial, int nchunk, long long P, float *__restrict__ grad)
{
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= P) return;
    double g = 0.0;
    for (int c = 0; c < nchunk; ++c) g += partial[(size_t)c * P + q];
    grad[q] = (float)g;
}

// loss = -(1/n) sum logq, one workgroup, fixed summation tree.
__global__ __launch_bounds__(256) void k_flow_loss(const float *__restrict__ logq, int n, double *__restrict__ loss)
{
    __shared__ double red[256];
    double acc = 0.0;
    for (int r = threadIdx.x; r < n; r += 256) acc += (double)logq[r];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = -red[0] / n;
}

__global__ void k_flow_adam(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                            const float *__restrict__ g, long long P, float lr, float c1, float c2)
{
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= P) return;
    const float gq = g[q];
    const float mq = fmaf(0.9f, m[q], 0.1f * gq);
    const float vq = fmaf(0.999f, v[q], 0.001f * gq * gq);
    m[q] = mq;
    v[q] = vq;
    p[q] -= lr * (mq * c1) / (sqrtf(vq * c2) + 1e-8f);
}

// splitmix64: the seeded generator of the default permutations and initial
// weights (host only).
uint64_t splitmix64(uint64_t &s)
{
    uint64_t z = (s += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

double uniform01(uint64_t &s) { return (splitmix64(s) >> 11) * (1.0 / 9007199254740992.0); }

}  // namespace

struct mbh_flow {
    int dim = 0, L = 0, H = 0, max_batch = 0, ntmax = 0;
    long long P = 0;
    size_t pass_lds = 0;   // dynamic LDS bytes of the pass kernel
    std::vector<int> perm, nc;
    std::vector<long long> off;
    int *d_perm = nullptr, *d_nc = nullptr;
    long long *d_off = nullptr;
    float *params = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    double *partial = nullptr, *loss = nullptr;
    float *X = nullptr, *H1 = nullptr, *H2 = nullptr, *SV = nullptr, *Go = nullptr, *Gp1 = nullptr, *Gp2 = nullptr;
    float *logq = nullptr;
    std::vector<void *> allocs;
    long long adam_step = 0;
    bool have_grad = false;
    std::string err;
};

namespace {

const char *kNoFlow = "mbh: null flow";

mbh_status ffail(mbh_flow *f, mbh_status st, const char *fmt, ...)
{
    if (f) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        f->err = buf;
    }
    return st;
}

mbh_status fhip(mbh_flow *f, hipError_t e, const char *where)
{
    return ffail(f, MBH_EHIP, "mbh: %s failed: %s", where, hipGetErrorString(e));
}

template <typename T>
mbh_status falloc(mbh_flow *f, T **p, size_t count)
{
    *p = nullptr;
    void *raw = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(&raw, count * sizeof(T));
    if (e != hipSuccess || raw == nullptr) {
        (void)hipGetLastError();
        return ffail(f, MBH_ENOMEM, "mbh: hipMalloc of %zu bytes failed", count * sizeof(T));
    }
    f->allocs.push_back(raw);
    *p = static_cast<T *>(raw);
    return MBH_OK;
}

void free_all(mbh_flow *f)
{
    for (void *p : f->allocs) (void)hipFree(p);
    f->allocs.clear();
}

FlowArgs args(const mbh_flow *f, int n)
{
    FlowArgs a;
    a.dim = f->dim;
    a.L = f->L;
    a.H = f->H;
    a.n = n;
    a.ntmax = f->ntmax;
    a.perm = f->d_perm;
    a.nc = f->d_nc;
    a.off = f->d_off;
    a.params = f->params;
    return a;
}

int pass_threads(int H) { return H >= 256 ? 256 : ((H + 63) / 64) * 64; }

mbh_status check_rows(mbh_flow *f, const void *a, const void *b, int n)
{
    if (n < 0 || n > f->max_batch) return ffail(f, MBH_EBATCH, "mbh: n = %d outside [0, max_batch = %d]", n, f->max_batch);
    if (n > 0 && (!a || !b)) return ffail(f, MBH_EINVAL, "mbh: null row buffer");
    if (a == b && n > 0) return ffail(f, MBH_EINVAL, "mbh: input and output rows must not alias");
    return MBH_OK;
}

}  // namespace

extern "C" {

mbh_status mbh_flow_create(int dim, int n_layers, int hidden, int max_batch, const int *perm_host, uint64_t seed,
                           mbh_flow **out)
{
    if (!out) return MBH_EINVAL;
    *out = nullptr;
    if (dim < 2 || dim > kMaxDim || n_layers < 1 || n_layers > kMaxLayers || hidden < 16 || hidden > kMaxH ||
        max_batch < 1 || max_batch > kMaxBatch)
        return MBH_EINVAL;
    mbh_flow *f = new mbh_flow();
    f->dim = dim;
    f->L = n_layers;
    f->H = hidden;
    f->max_batch = max_batch;
    f->ntmax = (dim + 1) / 2;
    uint64_t st = seed;
    f->perm.resize((size_t)n_layers * dim);
    for (int l = 0; l < n_layers; ++l) {
        int *row = &f->perm[(size_t)l * dim];
        if (perm_host) {
            std::vector<int> seen(dim, 0);
            for (int c = 0; c < dim; ++c) {
                const int v = perm_host[(size_t)l * dim + c];
                if (v < 0 || v >= dim || seen[v]++) {
                    delete f;
                    return MBH_EINVAL;
                }
                row[c] = v;
            }
        } else {
            for (int c = 0; c < dim; ++c) row[c] = c;
            for (int c = dim - 1; c > 0; --c) {
                const int r = (int)(splitmix64(st) % (uint64_t)(c + 1));
                std::swap(row[c], row[r]);
            }
        }
    }
    f->nc.resize(n_layers);
    f->off.resize(n_layers + 1);
    long long P = 0;
    for (int l = 0; l < n_layers; ++l) {
        const int nc = (l % 2 == 0) ? (dim + 1) / 2 : dim / 2;
        const int no = 2 * (dim - nc);
        f->nc[l] = nc;
        f->off[l] = P;
        P += (long long)nc * hidden + hidden + (long long)hidden * hidden + hidden + (long long)hidden * no + no;
    }
    f->off[n_layers] = P;
    f->P = P;
    int stage = 0;
    for (int l = 0; l < n_layers; ++l) stage = std::max(stage, stage_floats(f->nc[l], hidden, 2 * (dim - f->nc[l])));
    f->pass_lds = sizeof(float) * ((size_t)(h_padded(hidden) + hidden) * kS + (size_t)stage);
    {
        int dev = 0, lds_max = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
            f->pass_lds + kPassStaticLds > (size_t)lds_max) {
            (void)hipGetLastError();
            delete f;
            return MBH_EINVAL;
        }
    }

    // Initial weights: U(-1/sqrt(fan_in), 1/sqrt(fan_in)); the output map is zero.
    std::vector<float> p0((size_t)P, 0.f);
    for (int l = 0; l < n_layers; ++l) {
        float *w = &p0[(size_t)f->off[l]];
        const int nc = f->nc[l];
        const double a1 = 1.0 / std::sqrt((double)nc), a2 = 1.0 / std::sqrt((double)hidden);
        for (long long i = 0; i < (long long)nc * hidden + hidden; ++i) w[i] = (float)(a1 * (2 * uniform01(st) - 1));
        w += (long long)nc * hidden + hidden;
        for (long long i = 0; i < (long long)hidden * hidden + hidden; ++i) w[i] = (float)(a2 * (2 * uniform01(st) - 1));
    }

    const size_t mb = (size_t)max_batch;
    mbh_status s = MBH_OK;
    if ((s = falloc(f, &f->d_perm, f->perm.size())) || (s = falloc(f, &f->d_nc, (size_t)n_layers)) ||
        (s = falloc(f, &f->d_off, (size_t)n_layers + 1)) || (s = falloc(f, &f->params, (size_t)P)) ||
        (s = falloc(f, &f->m, (size_t)P)) || (s = falloc(f, &f->v, (size_t)P)) ||
        (s = falloc(f, &f->grad, (size_t)P)) || (s = falloc(f, &f->partial, (size_t)kMaxChunks * P)) ||
        (s = falloc(f, &f->loss, 1)) || (s = falloc(f, &f->X, (n_layers + 1) * mb * dim)) ||
        (s = falloc(f, &f->H1, n_layers * mb * hidden)) || (s = falloc(f, &f->H2, n_layers * mb * hidden)) ||
        (s = falloc(f, &f->Gp1, n_layers * mb * hidden)) || (s = falloc(f, &f->Gp2, n_layers * mb * hidden)) ||
        (s = falloc(f, &f->SV, n_layers * mb * f->ntmax)) || (s = falloc(f, &f->Go, n_layers * mb * 2 * f->ntmax)) ||
        (s = falloc(f, &f->logq, mb))) {
        free_all(f);
        delete f;
        return s;
    }
    hipError_t e;
    if ((e = hipMemcpy(f->d_perm, f->perm.data(), f->perm.size() * sizeof(int), hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(f->d_nc, f->nc.data(), f->nc.size() * sizeof(int), hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(f->d_off, f->off.data(), f->off.size() * sizeof(long long), hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(f->params, p0.data(), (size_t)P * sizeof(float), hipMemcpyHostToDevice)) ||
        (e = hipMemset(f->m, 0, (size_t)P * sizeof(float))) || (e = hipMemset(f->v, 0, (size_t)P * sizeof(float)))) {
        (void)hipGetLastError();
        free_all(f);
        delete f;
        return MBH_EHIP;
    }
    *out = f;
    return MBH_OK;
}

void mbh_flow_destroy(mbh_flow *f)
{
    if (!f) return;
    (void)hipDeviceSynchronize();
    free_all(f);
    delete f;
}

const char *mbh_flow_last_error(const mbh_flow *f) { return f ? f->err.c_str() : kNoFlow; }

int64_t mbh_flow_num_params(const mbh_flow *f) { return f ? (int64_t)f->P : -1; }

mbh_status mbh_flow_get_layout(const mbh_flow *f, int *perm_host, int *nc_host)
{
    if (!f) return MBH_EINVAL;
    if (perm_host) memcpy(perm_host, f->perm.data(), f->perm.size() * sizeof(int));
    if (nc_host) memcpy(nc_host, f->nc.data(), f->nc.size() * sizeof(int));
    return MBH_OK;
}

mbh_status mbh_flow_get_params(mbh_flow *f, float *params_host)
{
    if (!f) return MBH_EINVAL;
    if (!params_host) return ffail(f, MBH_EINVAL, "mbh: null parameter buffer");
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(params_host, f->params, (size_t)f->P * sizeof(float), hipMemcpyDeviceToHost);
    return e == hipSuccess ? MBH_OK : fhip(f, e, "hipMemcpy (flow parameters)");
}

mbh_status mbh_flow_set_params(mbh_flow *f, const float *params_host)
{
    if (!f) return MBH_EINVAL;
    if (!params_host) return ffail(f, MBH_EINVAL, "mbh: null parameter buffer");
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(f->params, params_host, (size_t)f->P * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(f->m, 0, (size_t)f->P * sizeof(float));
    if (e == hipSuccess) e = hipMemset(f->v, 0, (size_t)f->P * sizeof(float));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return fhip(f, e, "flow parameter upload");
    f->adam_step = 0;
    f->have_grad = false;
    return MBH_OK;
}

mbh_status mbh_flow_forward(mbh_flow *f, const float *u_dev, int n, float *z_dev, float *logq_dev, void *stream)
{
    if (!f) return MBH_EINVAL;
    if (mbh_status s = check_rows(f, u_dev, z_dev, n)) return s;
    if (n == 0) return MBH_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = launch_pass<false, false>(args(f, n), f->H, f->pass_lds, u_dev, z_dev, logq_dev, nullptr, nullptr,
                                             nullptr, nullptr, st);
    return e == hipSuccess ? MBH_OK : fhip(f, e, "k_flow_pass launch");
}

mbh_status mbh_flow_inverse(mbh_flow *f, const float *z_dev, int n, float *u_dev, float *logq_dev, void *stream)
{
    if (!f) return MBH_EINVAL;
    if (mbh_status s = check_rows(f, z_dev, u_dev, n)) return s;
    if (n == 0) return MBH_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = launch_pass<true, false>(args(f, n), f->H, f->pass_lds, z_dev, u_dev, logq_dev, nullptr, nullptr,
                                            nullptr, nullptr, st);
    return e == hipSuccess ? MBH_OK : fhip(f, e, "k_flow_pass launch");
}

mbh_status mbh_flow_loss_grad(mbh_flow *f, const float *u_dev, int n, double *loss_host, float *grad_host,
                              void *stream)
{
    if (!f) return MBH_EINVAL;
    if (n < 1 || n > f->max_batch)
        return ffail(f, MBH_EBATCH, "mbh: n = %d outside [1, max_batch = %d]", n, f->max_batch);
    if (!u_dev) return ffail(f, MBH_EINVAL, "mbh: null row buffer");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const FlowArgs a = args(f, n);
    const int blocks = (n + kS - 1) / kS, th = pass_threads(f->H);
    hipError_t e = launch_pass<false, true>(a, f->H, f->pass_lds, u_dev, nullptr, f->logq, f->X, f->H1, f->H2, f->SV,
                                            st);
    if (e != hipSuccess) return fhip(f, e, "k_flow_pass launch");
    k_flow_back<<<blocks, th, 0, st>>>(a, f->X, f->H1, f->H2, f->SV, f->Go, f->Gp1, f->Gp2, 1.0f / n);
    int chunk = (n + kMaxChunks - 1) / kMaxChunks;
    if (chunk < kMinChunk) chunk = kMinChunk;
    const int nchunk = (n + chunk - 1) / chunk;
    const unsigned gq = (unsigned)((f->P + 255) / 256);
    k_flow_wgrad<<<dim3(gq, nchunk), 256, 0, st>>>(a, f->X, f->H1, f->H2, f->Go, f->Gp1, f->Gp2, chunk, f->P,
                                                   f->partial);
    k_flow_gsum<<<gq, 256, 0, st>>>(f->partial, nchunk, f->P, f->grad);
    k_flow_loss<<<1, 256, 0, st>>>(f->logq, n, f->loss);
    e = hipGetLastError();
    if (e != hipSuccess) return fhip(f, e, "flow training launch");
    if (loss_host) e = hipMemcpyAsync(loss_host, f->loss, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && grad_host)
        e = hipMemcpyAsync(grad_host, f->grad, (size_t)f->P * sizeof(float), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fhip(f, e, "flow gradient");
    f->have_grad = true;
    return MBH_OK;
}

mbh_status mbh_flow_adam(mbh_flow *f, float lr, void *stream)
{
    if (!f) return MBH_EINVAL;
    if (!f->have_grad) return ffail(f, MBH_EINVAL, "mbh: mbh_flow_adam without a preceding mbh_flow_loss_grad");
    if (!(lr > 0.f) || !std::isfinite(lr)) return ffail(f, MBH_EINVAL, "mbh: learning rate must be positive");
    const long long t = ++f->adam_step;
    const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)t)));
    hipStream_t st = static_cast<hipStream_t>(stream);
    k_flow_adam<<<(unsigned)((f->P + 255) / 256), 256, 0, st>>>(f->params, f->m, f->v, f->grad, f->P, lr, c1, c2);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MBH_OK : fhip(f, e, "k_flow_adam launch");
}

}  // extern "C"
