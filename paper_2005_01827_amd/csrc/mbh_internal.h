// Device-side data structures and kernel launchers shared by the HIP
// translation units of libmbh.  Everything here is GPU-path code; the CPU
// oracle neither includes nor links it.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mbh {

constexpr int kMaxModes = 6;
constexpr int kNumFn = 8;          // A, phi, Re/Im T^A, Re/Im T^E, Re/Im T^T
constexpr int kCoefPerIv = kNumFn * 4;  // 32 doubles per sparse interval

// Dense tiling of the frequency axis: a work item is (walker, tile) with
// GridDesc::tile_bins = kDenseThreads * GridDesc::steps consecutive bins,
// processed by kDenseThreads threads; each wavefront takes 64*steps
// consecutive bins in 'steps' steps of 64 (coalesced loads of d and w).
// Long tiles let a wavefront reuse each interval's coefficients from the
// scalar cache over many steps (measured on a 1024-walker sweep of the
// 2^25-s grid: 8 steps 18.1 ms, 16 steps 16.8 ms, 32 steps 16.3 ms, 64 steps
// 16.8 ms, where coarser items balance worse); small problems need shorter
// tiles to keep enough work items in flight, so a context picks 'steps' from
// its grid and batch size (dense_steps()).
constexpr int kDenseThreads = 256;
constexpr int kMaxDenseSteps = 32;
constexpr int kMinDenseSteps = 2;
constexpr int kBinsPerLane = 2;   // bins per lane per step of the FP64 dense kernel
static_assert(kMinDenseSteps % kBinsPerLane == 0, "steps per wavefront must be a multiple of the bins per lane");
constexpr int kCisTabDoubles = 2064;  // device table of the dense-stage sin/cos constants and rotations
constexpr int kPartials = 9;       // R_c, DH_c, HH_c for c = A, E, T

// Per-walker constants of the waveform model (built by the source kernel).
struct Source {
    double M, eta, delta, x1, x2, chi1, chi2, Dl;
    double phiref, iota, lam, beta, psi, tcoal;
    double p2, p3, p4, p5, p6, p6L, p7;     // TaylorF2 coefficients
    double af, Mfin, fRD, fd;               // remnant spin, mass, (2,2,0) QNM
    double fJ, kRD, cR, b1, b0;             // merger-ringdown phase piece
    double fpeak, al0, al1;                 // alignment at max f^2 A_22
    double A0;                              // amplitude scale
    double kv[3], ep[3], eq[3];             // propagation direction, polarization basis (lambda, beta, psi)
    int valid;
    int pad;
};

// Frequency support of one (walker, mode).
struct ModeBand {
    double fs, fe;      // [f_start, f_end]
    int klo, khi;       // covered dense bins, inclusive
    int active;         // >= 4 covered bins
    int pad;
    double kp[2], kc[2];  // plus/cross weights of the mode (complex)
};

// Union band of one walker and its work-item range.
struct WalkerBand {
    int klo, khi;       // union of the active mode bands, inclusive
    int tile_lo;        // first tile index (tiles counted from bin k0)
    int ntiles;         // 0 if the walker has no active mode or is invalid
};

struct Modes {
    int nm;
    int l[kMaxModes];
    int m[kMaxModes];
};

struct GridDesc {
    double df;
    double t0;
    int k0;
    int n;
    int ns;             // sparse knots per mode
    int precision;      // 0: FP64 dense stage; 1: FP32 with compensated sums
    int steps;          // 64-bin steps per wavefront in the dense stage
    int tile_bins;      // kDenseThreads * steps
};

// Steps per wavefront for a grid of n bins and batches up to max_batch: the
// longest tile (up to kMaxDenseSteps) that still gives about 4096 work items
// for a full batch, at least kMinDenseSteps.
inline int dense_steps(long long n, int max_batch)
{
    int s = kMaxDenseSteps;
    while (s > kMinDenseSteps && (long long)max_batch * n < 4096LL * kDenseThreads * s) s /= 2;
    return s;
}

// Device workspace of a context (all pointers device memory).
struct Work {
    Source *src;            // [B]
    ModeBand *band;         // [B][nm]
    WalkerBand *wband;      // [B]
    double *kf;             // [B][nm][ns]        knots
    double *kt;             // [B][nm][ns]        t_lm at the knots
    double *fn;             // [B][nm][8][ns]     function values at the knots
    double *coef;           // [B][nm][ns-1][8][4] spline coefficients
    int *kbin;              // [B][nm][ns] first dense bin k with k df >= knot
    int *item_w;            // [max items] walker of each work item (tile-major order)
    int *item_t;            // [max items] tile of each work item
    int *tile_off;          // [tiles + 1] first item of each tile
    int *ticket;            // next work item of the dense kernel (zeroed by the tile scan)
    int *wbase;             // [B+1]  exclusive scan of ntiles; wbase[B] = total
    double *partial;        // [max items][9]
    double *out7;           // [B][7] default output
    double *cis_tab;        // constants of the dense-stage sin/cos
    float *cis32;           // the same for the FP32 dense stage
    float *coef32;          // [B][nm][ns-1][32] FP32 copy of coef (FP32 dense stage)
};

// Outputs of the fused sparse kernel (the Work arrays it writes).
struct SparseArgs {
    Source *src;
    ModeBand *band;
    double *kf, *kt, *fn, *coef;
    int *kbin;
    int *ticket;            // if not null: zeroed, for a dense launch with walker_one
};

// Union band of walker w's active modes and its range of tiles.
__device__ inline WalkerBand walker_band(int w, int nm, const GridDesc &g, const Source *__restrict__ src,
                                         const ModeBand *__restrict__ band)
{
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
            r.tile_lo = (lo - g.k0) / g.tile_bins;
            r.ntiles = (hi - g.k0) / g.tile_bins - r.tile_lo + 1;
        }
    }
    return r;
}

// The work-item list of a single walker, built by one whole workgroup: its
// band, the exclusive scan over walkers, the per-tile offsets, the items
// (its own tiles, in order) and the zeroed counter, the lists the general
// kernels build for B = 1.
__device__ inline void items_one(int nm, const GridDesc &g, const Source *__restrict__ src,
                                 const ModeBand *__restrict__ band, WalkerBand *__restrict__ wb,
                                 int *__restrict__ wbase, int *__restrict__ tile_off, int *__restrict__ ticket,
                                 int *__restrict__ item_w, int *__restrict__ item_t, int max_items)
{
    __shared__ WalkerBand r;
    if (threadIdx.x == 0) {
        r = walker_band(0, nm, g, src, band);
        wb[0] = r;
        wbase[0] = 0;
        wbase[1] = r.ntiles;
        ticket[0] = 0;
    }
    __syncthreads();
    const int ntiles = (g.n + g.tile_bins - 1) / g.tile_bins;
    for (int t = threadIdx.x; t <= ntiles; t += blockDim.x) tile_off[t] = min(max(t - r.tile_lo, 0), r.ntiles);
    for (int i = threadIdx.x; i < r.ntiles && i < max_items; i += blockDim.x) {
        item_w[i] = 0;
        item_t[i] = r.tile_lo + i;
    }
}

// Blocked layout of the data and weights read by the dense stage: bins in
// blocks of 64, each block holding the 64 values of channel A, then E, then
// T, so that a wavefront's 64 consecutive bins of all three channels are one
// wave-uniform block address plus lane * element size and an immediate
// channel offset.  The arrays are padded with zeros to a multiple of
// kDataPad bins, past the end of the last tile a dense launch can touch.
constexpr int kDataBlk = 64;
constexpr int kDataPad = 16384;
__host__ __device__ inline long long data_padded(long long n) { return (n + kDataPad - 1) / kDataPad * kDataPad; }
__host__ __device__ inline long long data_at(int ch, long long i)
{
    return ((i / kDataBlk) * 3 + ch) * kDataBlk + (i % kDataBlk);
}

// Data resident for the life of a context.
struct Data {
    const double2 *d;       // blocked [n_pad/64][3][64] A, E, T data (data_at)
    const double *w;        // blocked [n_pad/64][3][64] 4 df / S_n, 0 in the padding
    const double *pre;      // [3][n+1] prefix sums of |d|^2 w
    const float2 *dhi32;    // [3][n]   d sqrt(w), FP32 high part (FP32 dense stage)
    const float2 *dlo32;    // [3][n]   d sqrt(w) - dhi32, FP32 low part
    const float *sw32;      // [3][n]   sqrt(w) in FP32
};

// ---- launchers (each defined next to its kernels) ----
// host copies of the dense-stage sin/cos constants (uploaded to Work::cis_tab
// and Work::cis32)
const double *cis_table_host(int *n);
const float *cis32_table_host(int *n);

// d_in [3][n] and psd [3][n] as uploaded; writes the blocked d and w, the
// prefix sums and (if not null: FP32C contexts) dhi32 / dlo32 / sw32 [3][n]
hipError_t launch_setup_data(const double *psd, const double2 *d_in, double2 *d, double *w, double *pre,
                             double *scratch, float2 *dhi32, float2 *dlo32, float *sw32, const GridDesc &g,
                             double df4, hipStream_t st);

// FP32 copy of the spline coefficients for the FP32 dense stage
hipError_t launch_coef32(int B, const Modes &md, const GridDesc &g, const Work &wk, hipStream_t st);

hipError_t launch_waveform(const double *params, int B, const Modes &md, const GridDesc &g, const Work &wk,
                           hipStream_t st);

hipError_t launch_response(int B, const Modes &md, const GridDesc &g, const Work &wk, hipStream_t st);

hipError_t launch_spline(int B, const Modes &md, const GridDesc &g, const Work &wk, hipStream_t st);

// launch_waveform + launch_response + launch_spline as one kernel, one
// workgroup per (walker, mode), writing the same bits; with reset_ticket it
// also zeroes the dense stage's work-item counter, for a launch_dense with
// walker_one (one walker: no item list to build).
hipError_t launch_sparse(const double *params, int B, const Modes &md, const GridDesc &g, const Work &wk,
                         bool reset_ticket, hipStream_t st);

// Batches up to this size take the fused sparse kernel on the graph path
// (measured on the 2^22-s grid: 8-10 % less time per call than the chain of
// five kernels from 2 to 32 walkers, 6 % more at 64).
constexpr int kFusedSparseMaxBatch = 32;

hipError_t launch_walker_bands(int B, const Modes &md, const GridDesc &g, const Work &wk, hipStream_t st);

// Launch shape of the dense kernel: blocks_per_cu workgroups per compute unit
// taking (walker, tile) items from a counter, or, with one_per_walker, one
// workgroup per walker walking its own tiles (the unbalanced reference
// schedule).
struct Schedule {
    int blocks_per_cu = 8;
    int one_per_walker = 0;
};

int num_cus();

// ev0/ev1 (optional) are recorded on st right before and after the dense
// kernel.  inner = false: the FP64 path accumulates only the residual sums
// (enough for ln L); <d|h>_c and <h|h>_c of the output are then zero.
// walker_one (B = 1, the item counter already zero, as launch_sparse with
// reset_ticket leaves it; not with one_per_walker): no item list is built;
// every workgroup forms the walker's band from its mode bands and takes the
// walker's tiles in order from the counter, and workgroup 0 stores the band
// and the scan over walkers for the reduction.  Otherwise the launch builds
// the work-item list first.
hipError_t launch_dense(int B, const Modes &md, const GridDesc &g, const Work &wk, const Data &dt,
                        int max_items, const Schedule &sch, bool inner, hipStream_t st, hipEvent_t ev0 = nullptr,
                        hipEvent_t ev1 = nullptr, bool walker_one = false);

hipError_t launch_reduce(int B, const GridDesc &g, const Work &wk, const Data &dt, double *out7,
                         double *logL, hipStream_t st);

// Host handles of the first and last kernels of a likelihood sweep (the one
// that reads the walker parameters, the one that writes ln L), by which the
// context finds their nodes in a captured graph and points them at the
// caller's buffers for each launch.
const void *source_kernel();
const void *sparse_kernel(int ns);   // the fused sparse kernel launch_sparse uses for ns knots
const void *reduce_kernel();

hipError_t launch_template(const Modes &md, const GridDesc &g, const Work &wk, double2 *h, hipStream_t st);

}  // namespace mbh
