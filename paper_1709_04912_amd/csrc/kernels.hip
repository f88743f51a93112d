// gfx950 kernels of libscg: the matrix-free projector and backprojector, TV
// and its subgradient, the perturbation trials, the CG vector updates and the
// preconditioning filter.
//
// Every reduction is deterministic: per-thread partial sums, a fixed 64-lane
// butterfly, per-block partials in FP64 and a fixed-order final sum done by
// the last block to finish (a counter decides which block is last; there are
// no floating-point atomics), so results are bitwise reproducible.
#include "scg_internal.h"

namespace scg {

namespace {

constexpr int kBlock = 256;
constexpr int kMaxVecBlocks = 512;

__device__ __forceinline__ float sat(float v) { return __builtin_amdgcn_fmed3f(v, 0.0f, 1.0f); }
__device__ __forceinline__ double sat(double v) { return fmin(fmax(v, 0.0), 1.0); }

// floor() converted to int in one instruction (float); two for double.
__device__ __forceinline__ int flr(float v)
{
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(v));
    return r;
}
__device__ __forceinline__ int flr(double v) { return (int)floor(v); }

__device__ __forceinline__ float frc(float v) { return __builtin_amdgcn_fractf(v); }
__device__ __forceinline__ double frc(double v) { return v - floor(v); }

// Square root of a TV term: the hardware instruction for FP32 (within 1 ulp;
// both sides of every TV comparison use it), IEEE sqrt for FP64.
__device__ __forceinline__ float tsqrt(float v) { return __builtin_amdgcn_sqrtf(v); }
__device__ __forceinline__ double tsqrt(double v) { return sqrt(v); }

template <typename T> __device__ __forceinline__ T pK(const ProjAngle &a);
template <> __device__ __forceinline__ float pK<float>(const ProjAngle &a) { return a.Kf; }
template <> __device__ __forceinline__ double pK<double>(const ProjAngle &a) { return a.K; }
template <typename T> __device__ __forceinline__ T pC(const ProjAngle &a);
template <> __device__ __forceinline__ float pC<float>(const ProjAngle &a) { return a.Cf; }
template <> __device__ __forceinline__ double pC<double>(const ProjAngle &a) { return a.C; }
template <typename T> __device__ __forceinline__ T pM(const ProjAngle &a);
template <> __device__ __forceinline__ float pM<float>(const ProjAngle &a) { return a.inv_mf; }
template <> __device__ __forceinline__ double pM<double>(const ProjAngle &a) { return a.inv_m; }

template <typename T> struct BpW { T K, C, CK, M, c, s; };
template <typename T> __device__ __forceinline__ BpW<T> bpw(const BpAngle &a);
template <> __device__ __forceinline__ BpW<float> bpw<float>(const BpAngle &a)
{
    return {a.Kf, a.Cf, a.CKf, a.inv_mf, a.cf, a.sf};
}
template <> __device__ __forceinline__ BpW<double> bpw<double>(const BpAngle &a)
{
    return {a.K, a.C, a.C - a.K, a.inv_m, a.c, a.s};
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double load_relaxed(const double *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Block partial sums of NV values; the last block to finish sums all partials
// in a fixed order. Returns true in every thread of the last block; `tot` is
// valid in its thread 0. Every thread of the block must call this.
//
// Arrivals are counted in two levels (kRedGroups counters, 256 bytes apart,
// then one top counter) so that no single counter takes more than
// max(blocks / kRedGroups, kRedGroups) atomic increments; a single shared
// counter serialises every block's increment.
template <int NV, typename A>
__device__ bool reduce_finish(const A (&v)[NV], double *partials, unsigned *counter,
                              double *tot)
{
    __shared__ double sh[NV][16];   // up to 1024 threads
    __shared__ int s_last;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    const unsigned nblk = gridDim.x * gridDim.y * gridDim.z;
    const unsigned bid = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = wave_sum((double)v[k]);
        if (lane == 0) sh[k][wid] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += sh[threadIdx.x][w];
        partials[(size_t)bid * NV + threadIdx.x] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned g = bid % kRedGroups;
        const unsigned members = (nblk - g + kRedGroups - 1) / kRedGroups;
        int last = 0;
        if (atomicAdd(&counter[g * kRedStride], 1u) == members - 1) {
            __hip_atomic_store(&counter[g * kRedStride], 0u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            __threadfence();
            const unsigned groups = nblk < kRedGroups ? nblk : kRedGroups;
            last = atomicAdd(&counter[kRedGroups * kRedStride], 1u) == groups - 1;
            if (last)
                __hip_atomic_store(&counter[kRedGroups * kRedStride], 0u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        s_last = last;
    }
    __syncthreads();
    if (!s_last) return false;
    __threadfence();
    for (int k = 0; k < NV; ++k) {
        double acc = 0.0;
        for (unsigned b = threadIdx.x; b < nblk; b += blockDim.x)
            acc += load_relaxed(&partials[(size_t)b * NV + k]);
        acc = wave_sum(acc);
        __syncthreads();
        if (lane == 0) sh[0][wid] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int w = 0; w < nw; ++w) s += sh[0][w];
            tot[k] = s;
        }
    }
    return true;
}

__device__ __forceinline__ bool stopped(const DevState *st) { return st != nullptr && st->done; }

__device__ __forceinline__ scg_trace_entry *trace_at(DevState *st, scg_trace_entry *trace, int k)
{
    if (trace == nullptr || k < 1 || k > st->trace_cap) return nullptr;
    return &trace[k - 1];
}

__device__ __forceinline__ void set_done(DevState *st, int status)
{
    st->done = 1;
    st->status = status;
}

// gamma_l = gamma0 a^l for the next kTrialsPerPass trials (threads 0..15 of a
// block, one power each).
__device__ __forceinline__ void fill_gammas(DevState *st, int ell)
{
    if (threadIdx.x < kTrialsPerPass) {
        double g = st->gamma0 * pow(st->a, (double)(ell + (int)threadIdx.x));
        st->gam[threadIdx.x] = st->is_f32 ? (double)(float)g : g;
    }
}

inline int vec_blocks(size_t n)
{
    size_t b = (n + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > (size_t)kMaxVecBlocks) b = kMaxVecBlocks;
    return (int)b;
}

}  // namespace

// ---------------------------------------------------------------------------
// Elementwise helpers
// ---------------------------------------------------------------------------

template <typename T>
__global__ void k_fill(T *p, size_t n, T v)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <typename T>
__global__ void k_copy(T *dst, const T *src, size_t n, const DevState *st)
{
    if (stopped(st)) return;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

template <typename T> void launch_fill(T *p, size_t n, T v, hipStream_t s)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_fill<T>, dim3(vec_blocks(n)), dim3(kBlock), 0, s, p, n, v);
}

template <typename T>
void launch_copy(T *dst, const T *src, size_t n, const DevState *st, hipStream_t s)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_copy<T>, dim3(vec_blocks(n)), dim3(kBlock), 0, s, dst, src, n, st);
}

// ---------------------------------------------------------------------------
// Image staging: the transposed copy that angles stepping over columns read
// (32x32 tiles through LDS so both the read and the write are coalesced).
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void k_stage(const T *__restrict__ x, T *__restrict__ xt,
                                                Geo G, const DevState *st)
{
    if (stopped(st)) return;
    __shared__ T tile[32][33];
    const int n = G.n;
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const int i = by + r, j = bx + tx;
        tile[r][tx] = (i < n && j < n) ? x[(size_t)i * n + j] : T(0);
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int j = bx + r, i = by + tx;
        if (i < n && j < n) xt[(size_t)j * n + i] = tile[tx][r];
    }
}

template <typename T>
void launch_stage(const T *x, T *xt, const Geo &G, const DevState *st, hipStream_t s)
{
    dim3 grid((G.n + 31) / 32, (G.n + 31) / 32);
    hipLaunchKernelGGL(k_stage<T>, grid, dim3(256), 0, s, x, xt, G, st);
}

// ---------------------------------------------------------------------------
// Forward projector A (ray-driven, banded). Block (bin chunk, angle group):
// thread t owns bin b = chunk*kPjBins + (t & 127) for the group's angles
// (t >> 7) + 2m, m = 0..3 (each wavefront has one angle per slot). The block
// walks bands of kPjBand steps along the group's major axis (rows of x, or
// rows of x^T for angles stepping over columns), staging kPjWin columns of
// each band in LDS, column-major with a stride of kPjBand + 1 elements so
// neighbouring columns fall in different banks; the next band is prefetched
// into registers while the current one is consumed. Within a band a ray's
// crossing coordinate is an integer anchor plus an FP32 fraction (the anchor
// from FP64), so the split weights stay accurate near the axes where the
// chord ramp is steep. Per step: the crossing, its floor and fraction, one
// clamped FMA for the split weight, two LDS reads and three FMAs/adds.
// ---------------------------------------------------------------------------

template <typename T, int NQ>
__global__ __launch_bounds__(kPjBins * NQ) void k_project(const T *__restrict__ x,
                                                          const T *__restrict__ xt, Geo G,
                                                          ProjTables P, const T *__restrict__ y,
                                                          int y_stride, T *__restrict__ out,
                                                          int out_stride, int out_off,
                                                          double *partials, unsigned *counter,
                                                          DevState *st, int mode,
                                                          scg_trace_entry *trace)
{
    if (stopped(st)) return;
    // NQ groups of kPjBins threads; group q traces angles q, q + NQ, ... of
    // the block's angle group for one bin each.
    constexpr int NT = kPjBins * NQ;
    constexpr int LS = kPjBand + 1;               // LDS column stride (elements)
    constexpr int SLOTS = kPjGroup / NQ;
    constexpr int RPT = kPjWin * kPjBand / NT;    // staged rows per thread
    static_assert(kPjGroup % NQ == 0 && NT % kPjWin == 0 && kPjBand % RPT == 0,
                  "projector tiling");
    __shared__ T lds[kPjWin * LS];
    const int t = threadIdx.x;
    const int chunk = blockIdx.x, gi = blockIdx.y;
    const PjGroup grp = P.groups[gi];
    const int quarter = __builtin_amdgcn_readfirstlane(t / kPjBins);
    const int b_raw = chunk * kPjBins + (t & (kPjBins - 1));
    const bool bin_ok = b_raw < G.nb;
    const int b = bin_ok ? b_raw : G.nb - 1;   // idle lanes trace the chunk's last ray
    const int n = G.n;
    const T *img = grp.major ? xt : x;
    const int *win = P.win + ((size_t)gi * P.n_chunks + chunk) * P.n_bands;
    const int scol = t % kPjWin, srow = (t / kPjWin) * RPT;

    double u0[SLOTS];
    T acc[SLOTS], accr[SLOTS];
#pragma unroll
    for (int m = 0; m < SLOTS; ++m) {
        const int slot = quarter + NQ * m;
        acc[m] = T(0);
        accr[m] = T(0);
        u0[m] = 0.0;
        if (slot < grp.count) {
            const ProjAngle &A = P.ang[grp.a0 + slot];
            u0[m] = fma((double)b, A.u0_step, A.u0_base);
        }
    }

    T pre[RPT];
    auto prefetch = [&](int band) {
        const int jw = win[band];
        const int i0 = band * kPjBand + srow;
        const int col = jw + scol;
        const bool cok = col >= 0 && col < n;
        const T *src = img + (size_t)i0 * n + (cok ? col : 0);
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            T v = T(0);
            if (i0 + r < n) v = src[(size_t)r * n];
            pre[r] = cok ? v : T(0);
        }
    };

    int band = 0;
    while (band < P.n_bands && win[band] == kWinSkip) ++band;
    if (band < P.n_bands) prefetch(band);
    while (band < P.n_bands) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RPT; ++r) lds[scol * LS + srow + r] = pre[r];
        __syncthreads();
        const int jw = win[band];
        const int i0 = band * kPjBand;
        int nxt = band + 1;
        while (nxt < P.n_bands && win[nxt] == kWinSkip) ++nxt;
        if (nxt < P.n_bands) prefetch(nxt);
#pragma unroll
        for (int m = 0; m < SLOTS; ++m) {
            const int slot = quarter + NQ * m;
            if (slot < grp.count) {
                const ProjAngle &A = P.ang[grp.a0 + slot];
                const double us = fma((double)i0, A.slope, u0[m]);
                const double fu = floor(us);
                const T *col0 = lds + ((int)fu - jw) * LS;
                const T F0 = (T)(us - fu);
                const T slope = (T)A.slope, K = pK<T>(A), C = pC<T>(A);
                T a_ = acc[m], ar = accr[m];
#pragma unroll
                for (int k = 0; k < kPjBand; ++k) {
                    const T v = fma((T)k, slope, F0);
                    const int jl = flr(v);
                    const T wl = sat(fma(frc(v), -K, C));
                    const T *col = col0 + jl * LS;
                    const T xl = col[k], xr = col[LS + k];
                    a_ = fma(wl, xl - xr, a_);
                    ar += xr;
                }
                acc[m] = a_;
                accr[m] = ar;
            }
        }
        band = nxt;
    }

    double sq = 0.0;
#pragma unroll
    for (int m = 0; m < SLOTS; ++m) {
        const int slot = quarter + NQ * m;
        if (slot < grp.count && bin_ok) {
            const int a = grp.a0 + slot;
            T val = (acc[m] + accr[m]) * pM<T>(P.ang[a]);
            if (y != nullptr) val -= y[(size_t)a * y_stride + b];
            out[(size_t)a * out_stride + out_off + b] = val;
            sq += (double)val * (double)val;
        }
    }
    if (mode == kRedNone) return;
    double v[1] = {sq}, tot[1];
    if (!reduce_finish(v, partials, counter, tot) || threadIdx.x != 0) return;
    const double s = tot[0];
    if (mode == kRedResidual || mode == kRedResidualStep) {
        const double f = 0.5 * s;
        st->f_half = f;
        if (mode == kRedResidualStep)
            if (scg_trace_entry *tr = trace_at(st, trace, st->k)) tr->f_half = f;
        if (!isfinite(f)) {
            set_done(st, SCG_ENAN);
        } else if (f <= st->eps) {
            // Inside a step, the next loop test f(x_{k+1/2}) <= eps ends the
            // solve at k+1 with output x_{k+1/2}; the rest of the step is not
            // needed for the output and is skipped.
            if (mode == kRedResidualStep) {
                st->steps += 1;
                st->k += 1;
            }
            set_done(st, SCG_OK);
        }
    } else if (mode == kRedNormQ || mode == kRedInitNormQ || mode == kRedNormQCG) {
        st->qq = s;
        if (!isfinite(s)) {
            set_done(st, SCG_ENAN);
        } else if (s == 0.0) {
            set_done(st, SCG_EBREAKDOWN);
        } else {
            st->alpha = (mode == kRedNormQCG) ? st->delta / s : -st->gp / s;
            if (scg_trace_entry *tr = trace_at(st, trace, st->k)) tr->alpha = st->alpha;
        }
    }
}

template <typename T>
void launch_project(const T *x, const T *xt, const Geo &G, const ProjTables &P, const T *y,
                    int y_stride, T *out, int out_stride, int out_off, double *partials,
                    unsigned *counter, DevState *st, int mode, scg_trace_entry *trace,
                    int nq, hipStream_t s)
{
    dim3 grid(P.n_chunks, P.n_groups);
    if (nq == 4)
        hipLaunchKernelGGL((k_project<T, 4>), grid, dim3(kPjBins * 4), 0, s, x, xt, G, P, y,
                           y_stride, out, out_stride, out_off, partials, counter, st, mode, trace);
    else
        hipLaunchKernelGGL((k_project<T, 2>), grid, dim3(kPjBins * 2), 0, s, x, xt, G, P, y,
                           y_stride, out, out_stride, out_off, partials, counter, st, mode, trace);
}

// Copies an unpadded sinogram into the padded layout (pads stay zero).
template <typename T>
__global__ void k_pad_sino(const T *__restrict__ y, T *__restrict__ rpad, Geo G)
{
    const size_t L = (size_t)G.na * G.nb;
    for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < L;
         q += (size_t)gridDim.x * blockDim.x) {
        const size_t a = q / G.nb, b = q % G.nb;
        rpad[a * G.rs + kSinoPadL + b] = y[q];
    }
}

template <typename T> void launch_pad_sino(const T *y, T *rpad, const Geo &G, hipStream_t s)
{
    hipLaunchKernelGGL(k_pad_sino<T>, dim3(vec_blocks((size_t)G.na * G.nb)), dim3(kBlock), 0, s,
                       y, rpad, G);
}

// ---------------------------------------------------------------------------
// Backprojector A^T (pixel-driven, tiled). A block owns a 16 x 16 pixel tile;
// thread t owns the pixels (t >> 3, 2(t & 7)) and (t >> 3, 2(t & 7) + 1).
// Angles are processed in chunks of kBpChunk: for each angle the kBpWin bins
// around the tile centre's projection are staged in LDS, already scaled by
// 1/m, next to the angle's parameters (cos, sin, the two weight constants and
// the centre's fractional position); the next chunk is prefetched into
// registers while the current one is consumed. A pixel's footprint centre is
// an FP32 offset from the tile centre (it stays in (4, 27) bins), its two
// bins are one paired LDS read and its two weights two clamped FMAs. DUAL
// backprojects a second sinogram with the same weights (S-PCG: g' and z').
// ---------------------------------------------------------------------------

constexpr int kBpPrm = 8;   // per-angle parameters staged in LDS

template <typename T, bool DUAL, int NS>
__global__ __launch_bounds__(kBpThreads * NS) void k_backproject(const T *__restrict__ r,
                                                                  const T *__restrict__ r2, Geo G,
                                                                  const BpAngle *__restrict__ ang,
                                                                  T *__restrict__ out,
                                                                  T *__restrict__ out2,
                                                                  const T *__restrict__ dotv,
                                                                  double *partials,
                                                                  unsigned *counter, DevState *st,
                                                                  int mode)
{
    if (stopped(st)) return;
    // NS groups of kBpThreads threads share one tile; group gs takes angle
    // chunks gs, gs + NS, ... and the groups' sums are added in a fixed order
    // at the end.
    constexpr int NW = DUAL ? 2 : 1;
    constexpr int NE = kBpChunk * kBpWin / kBpThreads;   // staged bins per thread and sinogram
    __shared__ T win[NS][NW][kBpChunk * kBpWin];
    __shared__ T prm[NS][kBpChunk * kBpPrm];
    static_assert(NS * NW * kBpChunk * kBpWin >= (NS - 1) * kBpThreads * 2 * NW,
                  "combine buffer fits in the windows");
    const int gs = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kBpThreads);
    const int t = threadIdx.x % kBpThreads;
    const int ty = t >> 3, tx = (t & 7) * 2;
    const int i0 = blockIdx.y * kBpTile, j0 = blockIdx.x * kBpTile;
    const double xc = ((double)j0 + 7.5) - G.h, yc = G.h - ((double)i0 + 7.5);
    const T dx = (T)((double)tx - 7.5), dy = (T)(7.5 - (double)ty);
    T acc0 = T(0), acc1 = T(0), bcc0 = T(0), bcc1 = T(0);
    const int nchunks = (G.na + kBpChunk - 1) / kBpChunk;

    T pre[NW][NE];
    T ppr[kBpPrm];
    auto prefetch = [&](int ch) {
        const int a0 = ch * kBpChunk;
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            const int q = t + e * kBpThreads;
            const int al = q / kBpWin, k = q % kBpWin;
            const int a = a0 + al;
            T v = T(0), v2 = T(0);
            if (a < G.na) {
                const BpAngle &A = ang[a];
                const double pc = fma(xc, A.c, fma(yc, A.s, G.hb));
                const int bb = (int)floor(pc) - kBpHalf + k;
                if (bb >= 0 && bb < G.nb) {
                    const T m = (T)A.inv_m;
                    const size_t off = (size_t)a * G.rs + kSinoPadL + bb;
                    v = r[off] * m;
                    if (DUAL) v2 = r2[off] * m;
                }
            }
            pre[0][e] = v;
            if (DUAL) pre[NW - 1][e] = v2;
        }
        if (t < kBpChunk) {
            const int a = a0 + t;
#pragma unroll
            for (int k = 0; k < kBpPrm; ++k) ppr[k] = T(0);
            if (a < G.na) {
                const BpAngle &A = ang[a];
                const BpW<T> W = bpw<T>(A);
                const double pc = fma(xc, A.c, fma(yc, A.s, G.hb));
                ppr[0] = W.c;
                ppr[1] = W.s;
                ppr[2] = W.K;
                ppr[3] = W.C;
                ppr[4] = W.CK;
                ppr[5] = (T)(pc - (floor(pc) - kBpHalf));
            }
        }
    };

    if (gs < nchunks) prefetch(gs);
    for (int c0 = 0; c0 < nchunks; c0 += NS) {
        const int ch = c0 + gs;
        const bool live = ch < nchunks;
        __syncthreads();
        if (live) {
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                win[gs][0][t + e * kBpThreads] = pre[0][e];
                if (DUAL) win[gs][NW - 1][t + e * kBpThreads] = pre[NW - 1][e];
            }
            if (t < kBpChunk) {
#pragma unroll
                for (int k = 0; k < kBpPrm; ++k) prm[gs][t * kBpPrm + k] = ppr[k];
            }
        }
        __syncthreads();
        if (ch + NS < nchunks) prefetch(ch + NS);
        const int na = live ? min(kBpChunk, G.na - ch * kBpChunk) : 0;
#pragma unroll 2
        for (int al = 0; al < na; ++al) {
            const T *pr = &prm[gs][al * kBpPrm];
            const T c = pr[0], s = pr[1], K = pr[2], C = pr[3], CK = pr[4];
            const T u0 = fma(dx, c, fma(dy, s, pr[5]));
            const T u1 = u0 + c;
            const T *row = &win[gs][0][al * kBpWin];
            const int b0 = (int)u0, b1 = (int)u1;   // u > 0: truncation is floor
            const T f0 = frc(u0), f1 = frc(u1);
            const T w00 = sat(fma(f0, -K, C)), w01 = sat(fma(f0, K, CK));
            const T w10 = sat(fma(f1, -K, C)), w11 = sat(fma(f1, K, CK));
            acc0 = fma(w00, row[b0], acc0);
            acc0 = fma(w01, row[b0 + 1], acc0);
            acc1 = fma(w10, row[b1], acc1);
            acc1 = fma(w11, row[b1 + 1], acc1);
            if (DUAL) {
                const T *row2 = &win[gs][NW - 1][al * kBpWin];
                bcc0 = fma(w00, row2[b0], bcc0);
                bcc0 = fma(w01, row2[b0 + 1], bcc0);
                bcc1 = fma(w10, row2[b1], bcc1);
                bcc1 = fma(w11, row2[b1 + 1], bcc1);
            }
        }
    }

    if (NS > 1) {
        // groups 1..NS-1 hand their sums to group 0 through the windows
        T *red = &win[0][0][0];
        __syncthreads();
        if (gs > 0) {
            T *d = red + ((gs - 1) * kBpThreads + t) * 2 * NW;
            d[0] = acc0;
            d[1] = acc1;
            if (DUAL) {
                d[2] = bcc0;
                d[3] = bcc1;
            }
        }
        __syncthreads();
        if (gs == 0) {
            for (int g = 1; g < NS; ++g) {
                const T *d = red + ((g - 1) * kBpThreads + t) * 2 * NW;
                acc0 += d[0];
                acc1 += d[1];
                if (DUAL) {
                    bcc0 += d[2];
                    bcc1 += d[3];
                }
            }
        }
    }

    const int i = i0 + ty, j = j0 + tx;
    double d = 0.0;
    if (gs == 0 && i < G.n) {
        const size_t p = (size_t)i * G.n + j;
        if (j < G.n) {
            out[p] = acc0;
            if (DUAL) out2[p] = bcc0;
            if (mode == kRedDotGH) d += (double)(DUAL ? bcc0 : acc0) * (double)dotv[p];
            else if (mode == kRedDotGG) d += (double)acc0 * (double)acc0;
        }
        if (j + 1 < G.n) {
            out[p + 1] = acc1;
            if (DUAL) out2[p + 1] = bcc1;
            if (mode == kRedDotGH) d += (double)(DUAL ? bcc1 : acc1) * (double)dotv[p + 1];
            else if (mode == kRedDotGG) d += (double)acc1 * (double)acc1;
        }
    }
    if (mode == kRedNone) return;
    double v[1] = {d}, tot[1];
    if (!reduce_finish(v, partials, counter, tot) || threadIdx.x != 0) return;
    if (mode == kRedDotGH) st->gh = tot[0];
    else st->gg = tot[0];
}

template <typename T, bool DUAL>
void launch_bp_split(const T *r, const T *r2, const Geo &G, const BpAngle *ang, T *out, T *out2,
                     const T *dotv, double *partials, unsigned *counter, DevState *st, int mode,
                     int split, hipStream_t s)
{
    dim3 grid((G.n + kBpTile - 1) / kBpTile, (G.n + kBpTile - 1) / kBpTile);
    if (split >= 4)
        hipLaunchKernelGGL((k_backproject<T, DUAL, 4>), grid, dim3(kBpThreads * 4), 0, s, r, r2, G,
                           ang, out, out2, dotv, partials, counter, st, mode);
    else if (split == 2)
        hipLaunchKernelGGL((k_backproject<T, DUAL, 2>), grid, dim3(kBpThreads * 2), 0, s, r, r2, G,
                           ang, out, out2, dotv, partials, counter, st, mode);
    else
        hipLaunchKernelGGL((k_backproject<T, DUAL, 1>), grid, dim3(kBpThreads), 0, s, r, r2, G,
                           ang, out, out2, dotv, partials, counter, st, mode);
}

template <typename T>
void launch_backproject(const T *r, const T *r2, const Geo &G, const BpAngle *ang, T *out,
                        T *out2, const T *dotv, double *partials, unsigned *counter,
                        DevState *st, int mode, int split, hipStream_t s)
{
    if (r2 != nullptr)
        launch_bp_split<T, true>(r, r2, G, ang, out, out2, dotv, partials, counter, st, mode,
                                 split, s);
    else
        launch_bp_split<T, false>(r, r2, G, ang, out, out2, dotv, partials, counter, st, mode,
                                  split, s);
}

// ---------------------------------------------------------------------------
// Total variation: t_ij = sqrt(a^2 + b^2 + kappa^2) over the (N-1)^2 interior
// forward differences a = x[i+1][j] - x[i][j], b = x[i][j+1] - x[i][j], and
// the subgradient s = sum over terms of d t / d x (a term with t = 0 adds 0).
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ T tv_term(T a, T b, T k2)
{
    return tsqrt(fma(a, a, fma(b, b, k2)));
}

// Subgradient entry and own TV term of pixel (i, j) from its 3 x 3
// neighbourhood X[di][dj] (di, dj in 0..2, centre at [1][1]).
template <typename T>
__device__ __forceinline__ T tv_pixel(const T (&X)[3][3], int i, int j, int n, T k2, T &own)
{
    const T xc = X[1][1];
    T sg = T(0);
    own = T(0);
    if (i + 1 < n && j + 1 < n) {          // own term (i, j)
        const T a = X[2][1] - xc, b = X[1][2] - xc;
        const T t = tv_term(a, b, k2);
        own = t;
        if (t != T(0)) sg -= (a + b) / t;
    }
    if (i >= 1 && j + 1 < n) {             // term (i-1, j): x is its lower neighbour
        const T base = X[0][1];
        const T a = xc - base, b = X[0][2] - base;
        const T t = tv_term(a, b, k2);
        if (t != T(0)) sg += a / t;
    }
    if (j >= 1 && i + 1 < n) {             // term (i, j-1): x is its right neighbour
        const T base = X[1][0];
        const T a = X[2][0] - base, b = xc - base;
        const T t = tv_term(a, b, k2);
        if (t != T(0)) sg += b / t;
    }
    return sg;
}

// TV(x) into *tv_dst and optionally the subgradient (scg_tv, solver output).
template <typename T>
__global__ __launch_bounds__(256) void k_tv(const T *__restrict__ x, T *__restrict__ s_out,
                                             Geo G, double kappa, double *partials,
                                             unsigned *counter, double *tv_dst)
{
    const int n = G.n;
    const T k2 = (T)(kappa * kappa);
    double tv = 0.0;
    const size_t J = (size_t)n * n;
    for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < J;
         p += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(p / n), j = (int)(p % n);
        T X[3][3];
#pragma unroll
        for (int di = 0; di < 3; ++di)
#pragma unroll
            for (int dj = 0; dj < 3; ++dj) {
                const int ii = i + di - 1, jj = j + dj - 1;
                X[di][dj] = (ii >= 0 && ii < n && jj >= 0 && jj < n) ? x[(size_t)ii * n + jj] : T(0);
            }
        T own;
        const T sg = tv_pixel(X, i, j, n, k2, own);
        tv += (double)own;
        if (s_out != nullptr) s_out[p] = sg;
    }
    double v[1] = {tv}, tot[1];
    if (!reduce_finish(v, partials, counter, tot) || threadIdx.x != 0) return;
    *tv_dst = tot[0];
}

template <typename T>
void launch_tv(const T *x, T *s_out, const Geo &G, double kappa, double *partials,
               unsigned *counter, double *tv_dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_tv<T>, dim3(vec_blocks((size_t)G.n * G.n)), dim3(kBlock), 0, s, x, s_out,
                       G, kappa, partials, counter, tv_dst);
}

// ---------------------------------------------------------------------------
// Step boundary of the superiorized solvers, fused with the TV work that opens
// the next step: x_{k+1} = x_{k+1/2} + alpha p' (the last line of the previous
// step) on a 32 x 8 tile plus a one-pixel halo held in LDS, then the TV
// subgradient s at x_{k+1}, ||s||^2 and TV(x_{k+1}). The last block closes the
// previous step (k, the carried ||A p||^2 and g^T p), applies the iteration
// cap, opens the new step (replayed decisions, trace) and prepares the first
// pass of trials (v = -s/||s||, gamma0 a^(l+m)).
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void k_xtv(const T *__restrict__ xh, const T *__restrict__ p,
                                              T *__restrict__ x, T *__restrict__ s_out, Geo G,
                                              double *partials, unsigned *counter, DevState *st,
                                              const int32_t *forced, scg_trace_entry *trace)
{
    if (st->done) return;
    constexpr int TW = 32, TH = 8;
    __shared__ T tile[TH + 2][TW + 2];
    const int n = G.n;
    const int i0 = blockIdx.y * TH, j0 = blockIdx.x * TW;
    const T al = (T)st->alpha;
    const T k2 = (T)(st->kappa * st->kappa);
    for (int e = threadIdx.x; e < (TH + 2) * (TW + 2); e += blockDim.x) {
        const int ii = i0 - 1 + e / (TW + 2), jj = j0 - 1 + e % (TW + 2);
        T v = T(0);
        if (ii >= 0 && ii < n && jj >= 0 && jj < n) {
            const size_t q = (size_t)ii * n + jj;
            v = fma(al, p[q], xh[q]);
        }
        tile[e / (TW + 2)][e % (TW + 2)] = v;
    }
    __syncthreads();
    const int ty = threadIdx.x / TW, tx = threadIdx.x % TW;
    const int i = i0 + ty, j = j0 + tx;
    double tv = 0.0, ss = 0.0;
    if (i < n && j < n) {
        T X[3][3];
#pragma unroll
        for (int di = 0; di < 3; ++di)
#pragma unroll
            for (int dj = 0; dj < 3; ++dj) X[di][dj] = tile[ty + di][tx + dj];
        T own;
        const T sg = tv_pixel(X, i, j, n, k2, own);
        const size_t q = (size_t)i * n + j;
        x[q] = X[1][1];
        s_out[q] = sg;
        tv = (double)own;
        ss = (double)sg * (double)sg;
    }
    double v[2] = {tv, ss}, tot[2];
    if (!reduce_finish(v, partials, counter, tot)) return;
    __shared__ int s_go, s_ell;
    if (threadIdx.x == 0) {
        // close the previous step
        st->qq_prev = st->qq;
        st->gp_prev = st->gp;
        st->k += 1;
        st->steps += 1;
        s_go = 0;
        if (st->steps >= st->max_iter) {
            set_done(st, SCG_ENOCONV);
        } else {
            // open step k: perturbed(x_k) starts here
            const int k = st->k;
            st->trials_step = 0;
            st->accepted = -1;
            st->gamma = 0.0;
            st->search_done = (st->flags & SCG_FLAG_NO_PERTURB) ? 1 : 0;
            st->tv_x = tot[0];
            st->s_norm2 = tot[1];
            const bool dir = tot[1] > 0.0 && isfinite(tot[1]);
            st->inv_snorm = dir ? 1.0 / sqrt(tot[1]) : 0.0;
            if (scg_trace_entry *tr = trace_at(st, trace, k)) {
                tr->k = k;
                tr->accepted = -1;
                tr->trials = 0;
                tr->ell = st->ell;
                tr->gamma = 0.0;
                tr->beta = 0.0;
                tr->alpha = 0.0;
                tr->tv_x = tot[0];
                tr->f_half = 0.0;
            }
            if (!st->search_done && forced != nullptr && k - 1 < st->forced_len) {
                const int nt = forced[2 * (k - 1)], am = forced[2 * (k - 1) + 1];
                const int l0 = st->ell;
                double g = 0.0;
                if (am >= 0 && dir) {
                    g = st->gamma0 * pow(st->a, (double)(l0 + am));
                    g = st->is_f32 ? (double)(float)g : g;
                }
                st->ell = l0 + nt;
                st->trials_step = nt;
                st->trials_total += nt;
                st->accepted = dir ? am : -1;
                st->gamma = g;
                st->search_done = 1;
                if (scg_trace_entry *tr = trace_at(st, trace, k)) {
                    tr->accepted = st->accepted;
                    tr->trials = nt;
                    tr->ell = st->ell;
                    tr->gamma = g;
                }
            }
            if (!st->search_done && !dir) {
                // No nonascending direction: x_{k+1/2} = x_k and l is unchanged.
                st->search_done = 1;
            }
            s_go = !st->search_done;
            s_ell = st->ell;
        }
    }
    __syncthreads();
    if (s_go) fill_gammas(st, s_ell);
}

template <typename T>
void launch_xtv(const T *xh, const T *p, T *x, T *s_out, const Geo &G, double *partials,
                unsigned *counter, DevState *st, const int32_t *forced, scg_trace_entry *trace,
                hipStream_t s)
{
    dim3 grid((G.n + 31) / 32, (G.n + 7) / 8);
    hipLaunchKernelGGL(k_xtv<T>, grid, dim3(256), 0, s, xh, p, x, s_out, G, partials, counter, st,
                       forced, trace);
}

// ---------------------------------------------------------------------------
// perturbed(): one pass evaluates TV(x + gamma_m v) for kTrialsPerPass
// successive values gamma_m = gamma0 a^(l+m), v = -s/||s||, together with
// TV(x) summed in the same order; the last block takes the first m with
// TV(x + gamma_m v) <= TV(x), exactly as trying them one after another.
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void k_trials(const T *__restrict__ x, const T *__restrict__ s,
                                                 Geo G, double *partials, unsigned *counter,
                                                 DevState *st, scg_trace_entry *trace)
{
    if (st->done || st->search_done) return;
    constexpr int M = kTrialsPerPass;
    T gam[M];
#pragma unroll
    for (int m = 0; m < M; ++m) gam[m] = (T)st->gam[m];
    const T inv = (T)st->inv_snorm;
    const T k2 = (T)(st->kappa * st->kappa);
    const int n = G.n, m1 = n - 1;
    T acc[M + 1];
#pragma unroll
    for (int m = 0; m <= M; ++m) acc[m] = T(0);
    const size_t terms = (size_t)m1 * m1;
    for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < terms;
         q += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(q / m1), j = (int)(q % m1);
        const size_t c = (size_t)i * n + j;
        const T xc = x[c], xd = x[c + n], xr = x[c + 1];
        const T vc = -s[c] * inv, vd = -s[c + n] * inv, vr = -s[c + 1] * inv;
        acc[M] += tv_term(xd - xc, xr - xc, k2);
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const T g = gam[m];
            const T zc = fma(g, vc, xc), zd = fma(g, vd, xd), zr = fma(g, vr, xr);
            acc[m] += tv_term(zd - zc, zr - zc, k2);
        }
    }
    __shared__ double tot[M + 1];
    if (!reduce_finish(acc, partials, counter, tot)) return;
    __shared__ int s_more, s_ell;
    if (threadIdx.x == 0) {
        const double tvx = tot[M];
        st->tv_x = tvx;
        const int left = st->max_trials - st->trials_step;
        const int nv = left < M ? left : M;
        int hit = -1;
        for (int m = 0; m < nv; ++m)
            if (tot[m] <= tvx) {
                hit = m;
                break;
            }
        const int used = hit >= 0 ? hit + 1 : nv;
        const int first = st->trials_step;
        st->ell += used;
        st->trials_step += used;
        st->trials_total += used;
        if (hit >= 0) {
            st->accepted = first + hit;
            st->gamma = (double)gam[hit];
            st->search_done = 1;
        } else if (st->trials_step >= st->max_trials) {
            st->accepted = -1;
            st->gamma = 0.0;
            st->search_done = 1;
        }
        if (st->search_done) {
            if (scg_trace_entry *tr = trace_at(st, trace, st->k)) {
                tr->accepted = st->accepted;
                tr->trials = st->trials_step;
                tr->ell = st->ell;
                tr->gamma = st->gamma;
                tr->tv_x = tvx;
            }
        }
        s_more = !st->search_done;
        s_ell = st->ell;
    }
    __syncthreads();
    if (s_more) fill_gammas(st, s_ell);
}

template <typename T>
void launch_trials(const T *x, const T *s, const Geo &G, double *partials, unsigned *counter,
                   DevState *st, scg_trace_entry *trace, hipStream_t stream)
{
    size_t terms = (size_t)(G.n - 1) * (G.n - 1);
    hipLaunchKernelGGL(k_trials<T>, dim3(vec_blocks(terms)), dim3(kBlock), 0, stream, x, s, G,
                       partials, counter, st, trace);
}

// ---------------------------------------------------------------------------
// 32 x 32 tile kernels that write an image and its transpose (the forward
// projector reads both): x_{k+1/2} = x_k + gamma v (computed exactly as in the
// trials), and the direction update p' = -src + beta p with the partial
// g'^T p'.
//   rule 0 (CG-PR-STEP):  beta = g'^T h / p^T h   (p^T h evaluated as ||A p||^2)
//   rule 1 (CG-CD-STEP):  beta = -||g'||^2 / g^T p
//   rule 2 (PCG-PR-STEP): beta = z'^T h / p^T h, src = z'
//   rule 3 (CG-STEP):     beta = delta' / delta, delta' = ||g'||^2
// init != 0: beta = 0 (the initial p0 = -g0 or -z0).
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void k_perturb(const T *__restrict__ x, const T *__restrict__ s,
                                                  T *__restrict__ xh, T *__restrict__ xht, Geo G,
                                                  DevState *st)
{
    if (st->done) return;
    __shared__ T tile[32][33];
    const bool move = st->accepted >= 0 && st->gamma != 0.0;
    const T g = (T)st->gamma, inv = (T)st->inv_snorm;
    const int n = G.n;
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const int i = by + r, j = bx + tx;
        T v = T(0);
        if (i < n && j < n) {
            const size_t q = (size_t)i * n + j;
            const T xc = x[q];
            v = move ? fma(g, -s[q] * inv, xc) : xc;
            xh[q] = v;
        }
        tile[r][tx] = v;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int j = bx + r, i = by + tx;
        if (i < n && j < n) xht[(size_t)j * n + i] = tile[tx][r];
    }
}

template <typename T>
void launch_perturb(const T *x, const T *s, T *xh, T *xht, const Geo &G, DevState *st,
                    hipStream_t stream)
{
    dim3 grid((G.n + 31) / 32, (G.n + 31) / 32);
    hipLaunchKernelGGL(k_perturb<T>, grid, dim3(256), 0, stream, x, s, xh, xht, G, st);
}

template <typename T>
__global__ __launch_bounds__(256) void k_p_update(const T *__restrict__ g, const T *__restrict__ z,
                                                   T *__restrict__ p, T *__restrict__ pt, Geo G,
                                                   double *partials, unsigned *counter,
                                                   DevState *st, int rule, int init,
                                                   scg_trace_entry *trace)
{
    if (st->done) return;
    __shared__ T tile[32][33];
    double beta = 0.0;
    if (!init) {
        if (rule == 0 || rule == 2) beta = st->gh / st->qq_prev;
        else if (rule == 1) beta = -st->gg / st->gp_prev;
        else beta = st->gg / st->delta;
    }
    const T bt = (T)beta;
    const T *src = (rule == 2) ? z : g;
    const int n = G.n;
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    double acc = 0.0;
    for (int r = ty; r < 32; r += 8) {
        const int i = by + r, j = bx + tx;
        T pn = T(0);
        if (i < n && j < n) {
            const size_t q = (size_t)i * n + j;
            pn = init ? -src[q] : fma(bt, p[q], -src[q]);
            p[q] = pn;
            acc += (double)g[q] * (double)pn;
        }
        tile[r][tx] = pn;
    }
    __syncthreads();
    if (pt != nullptr) {
        for (int r = ty; r < 32; r += 8) {
            const int j = bx + r, i = by + tx;
            if (i < n && j < n) pt[(size_t)j * n + i] = tile[tx][r];
        }
    }
    double v[1] = {acc}, tot[1];
    if (!reduce_finish(v, partials, counter, tot) || threadIdx.x != 0) return;
    st->beta = beta;
    st->gp = tot[0];
    if (rule == 3) st->delta = st->gg;
    if (!isfinite(beta) || !isfinite(tot[0])) set_done(st, SCG_ENAN);
    if (!init)
        if (scg_trace_entry *tr = trace_at(st, trace, st->k)) tr->beta = beta;
}

template <typename T>
void launch_p_update(const T *g, const T *z, T *p, T *pt, const Geo &G, double *partials,
                     unsigned *counter, DevState *st, int rule, int init,
                     scg_trace_entry *trace, hipStream_t s)
{
    dim3 grid((G.n + 31) / 32, (G.n + 31) / 32);
    hipLaunchKernelGGL(k_p_update<T>, grid, dim3(256), 0, s, g, z, p, pt, G, partials, counter,
                       st, rule, init, trace);
}

// Plain CG (Alg. CG, CG-STEP): x' = x + alpha p and the recursive gradient
// g' = g + alpha h with ||g'||^2; closes the step.
template <typename T>
__global__ __launch_bounds__(256) void k_x_update_cg(T *__restrict__ x, const T *__restrict__ p,
                                                      const T *__restrict__ h, T *__restrict__ g,
                                                      size_t J, DevState *st, double *partials,
                                                      unsigned *counter)
{
    if (st->done) return;
    const T al = (T)st->alpha;
    double acc = 0.0;
    for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < J;
         q += (size_t)gridDim.x * blockDim.x) {
        x[q] = fma(al, p[q], x[q]);
        const T gn = fma(al, h[q], g[q]);
        g[q] = gn;
        acc += (double)gn * (double)gn;
    }
    double v[1] = {acc}, tot[1];
    if (!reduce_finish(v, partials, counter, tot) || threadIdx.x != 0) return;
    st->gg = tot[0];
    st->qq_prev = st->qq;
    st->k += 1;
    st->steps += 1;
}

template <typename T>
void launch_x_update_cg(T *x, const T *p, const T *h, T *g, const Geo &G, DevState *st,
                        double *partials, unsigned *counter, hipStream_t s)
{
    size_t J = (size_t)G.n * G.n;
    hipLaunchKernelGGL(k_x_update_cg<T>, dim3(vec_blocks(J)), dim3(kBlock), 0, s, x, p, h, g, J,
                       st, partials, counter);
}

// Plain CG: the iteration cap at the top of the loop.
__global__ void k_iter_begin(DevState *st)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (st->done) return;
    if (st->steps >= st->max_iter) set_done(st, SCG_ENOCONV);
}

void launch_iter_begin(DevState *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_iter_begin, dim3(1), dim3(64), 0, s, st);
}

// ---------------------------------------------------------------------------
// Preconditioning filter F^T C F per projection, as the linear convolution
// with k[d] = (1/P) sum_m c(w_m) cos(w_m d) (|d| < n_bins) that the
// zero-padded DFT product equals. One block per angle; the projection and
// the kernel are staged in LDS and each thread produces four neighbouring
// outputs from a sliding window of kernel taps.
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void k_filter(const T *__restrict__ r, T *__restrict__ out,
                                                 const T *__restrict__ kern, Geo G,
                                                 int out_padded, const DevState *st)
{
    if (stopped(st)) return;
    extern __shared__ unsigned char smem[];
    T *row = reinterpret_cast<T *>(smem);
    T *kk = row + G.nb;                  // kk[d + nb - 1] = k[|d|], d in (-nb, nb)
    const int a = blockIdx.x, nb = G.nb;
    const T *ra = r + (size_t)a * G.rs + kSinoPadL;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) row[b] = ra[b];
    for (int d = threadIdx.x; d < 2 * nb - 1; d += blockDim.x) {
        const int dd = d - (nb - 1);
        kk[d] = kern[dd < 0 ? -dd : dd];
    }
    __syncthreads();
    for (int b0 = threadIdx.x * 4; b0 < nb; b0 += blockDim.x * 4) {
        // out[b0+t] = sum_bp k[b0 + t - bp] row[bp]
        T acc0 = 0, acc1 = 0, acc2 = 0, acc3 = 0;
        for (int bp = 0; bp < nb; ++bp) {
            const T rv = row[bp];
            const int base = b0 - bp + nb - 1;
            acc0 = fma(kk[base], rv, acc0);
            if (b0 + 1 < nb) acc1 = fma(kk[base + 1], rv, acc1);
            if (b0 + 2 < nb) acc2 = fma(kk[base + 2], rv, acc2);
            if (b0 + 3 < nb) acc3 = fma(kk[base + 3], rv, acc3);
        }
        T *oa = out + (size_t)a * (out_padded ? G.rs : nb) + (out_padded ? kSinoPadL : 0);
        oa[b0] = acc0;
        if (b0 + 1 < nb) oa[b0 + 1] = acc1;
        if (b0 + 2 < nb) oa[b0 + 2] = acc2;
        if (b0 + 3 < nb) oa[b0 + 3] = acc3;
    }
}

template <typename T>
void launch_filter(const T *r, T *out, const T *kernel, const Geo &G, int out_padded,
                   const DevState *st, hipStream_t s)
{
    size_t shm = (size_t)(3 * G.nb) * sizeof(T);
    hipLaunchKernelGGL(k_filter<T>, dim3(G.na), dim3(256), shm, s, r, out, kernel, G, out_padded,
                       st);
}

// ---- explicit instantiations ----------------------------------------------
#define SCG_INST(T)                                                                            \
    template void launch_fill<T>(T *, size_t, T, hipStream_t);                                 \
    template void launch_copy<T>(T *, const T *, size_t, const DevState *, hipStream_t);       \
    template void launch_stage<T>(const T *, T *, const Geo &, const DevState *, hipStream_t); \
    template void launch_project<T>(const T *, const T *, const Geo &, const ProjTables &,      \
                                    const T *, int, T *, int, int, double *, unsigned *,        \
                                    DevState *, int, scg_trace_entry *, int, hipStream_t);      \
    template void launch_pad_sino<T>(const T *, T *, const Geo &, hipStream_t);                \
    template void launch_backproject<T>(const T *, const T *, const Geo &, const BpAngle *,    \
                                        T *, T *, const T *, double *, unsigned *, DevState *, \
                                        int, int, hipStream_t);                                 \
    template void launch_tv<T>(const T *, T *, const Geo &, double, double *, unsigned *,      \
                               double *, hipStream_t);                                          \
    template void launch_xtv<T>(const T *, const T *, T *, T *, const Geo &, double *,         \
                                unsigned *, DevState *, const int32_t *, scg_trace_entry *,     \
                                hipStream_t);                                                   \
    template void launch_trials<T>(const T *, const T *, const Geo &, double *, unsigned *,    \
                                   DevState *, scg_trace_entry *, hipStream_t);                 \
    template void launch_perturb<T>(const T *, const T *, T *, T *, const Geo &, DevState *,   \
                                    hipStream_t);                                               \
    template void launch_p_update<T>(const T *, const T *, T *, T *, const Geo &, double *,    \
                                     unsigned *, DevState *, int, int, scg_trace_entry *,      \
                                     hipStream_t);                                              \
    template void launch_x_update_cg<T>(T *, const T *, const T *, T *, const Geo &,           \
                                        DevState *, double *, unsigned *, hipStream_t);        \
    template void launch_filter<T>(const T *, T *, const T *, const Geo &, int,                \
                                   const DevState *, hipStream_t);

SCG_INST(float)
SCG_INST(double)

}  // namespace scg
