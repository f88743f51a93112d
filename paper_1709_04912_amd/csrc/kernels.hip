// gfx950 kernels of libscg: the matrix-free projector and backprojector, TV
// and its subgradient, the perturbation trials, the CG vector updates and the
// preconditioning filter.
//
// Solver kernels are written as block bodies and launched two ways: for one
// solve, or batched, where one launch covers a phase of many solves and a
// block map gives each block its solve and local block index. Scalars come
// from reductions that are deterministic and free of atomics: every block
// stores its partial sums (fixed 64-lane butterflies, FP64), and a finisher
// launch (one block per solve) sums them in a fixed order and applies the
// scalar logic of the algorithm to the solve's device state.
#include "scg_internal.h"

namespace scg {

namespace {

// Pointers read from a descriptor in memory are generic to the compiler,
// whose flat loads also count as LDS operations and so make every LDS wait
// wait for the global loads in flight. The kernel bodies access memory
// through these global-qualified views instead.
template <typename P> __device__ __forceinline__ auto gl(P *p)
{
#if defined(__HIP_DEVICE_COMPILE__)
    using G = __attribute__((address_space(1))) P;
    return (G *)p;
#else
    return p;   // host pass of the single-source compile: never executed
#endif
}

// Read-only data that a kernel indexes uniformly across a wavefront (per-angle
// constants): constant-qualified views, which the compiler reads through the
// scalar cache into scalar registers.
template <typename P> __device__ __forceinline__ auto cst(const P *p)
{
#if defined(__HIP_DEVICE_COMPILE__)
    using C = const __attribute__((address_space(4))) P;
    return (C *)p;
#else
    return p;
#endif
}

constexpr int kBlock = 256;
constexpr int kXtvRows = 16;   // tile height of the step-boundary TV pass (two rows per thread)
constexpr int kMaxVecBlocks = 512;

// Raw buffer views. A load through the buffer unit whose per-lane byte
// offset is at or past the view's size returns zero without touching memory;
// kernels use that for the zero padding around an image and pass kBufOob as
// the offset of an element that lies outside it. The per-lane offset alone
// is range-checked, so a uniform (scalar) offset is only added where every
// element it reaches exists.
#if defined(__HIP_DEVICE_COMPILE__)
using Rsrc = __amdgpu_buffer_rsrc_t;
#else
struct Rsrc {
    int w[4];
};
#endif
constexpr uint32_t kBufOob = 0x80000000u;

// Projector steps whose LDS reads are in flight together.
constexpr int kPjGroupSteps = 8;

__device__ __forceinline__ Rsrc buf_rsrc(const void *p, uint32_t bytes)
{
#if defined(__HIP_DEVICE_COMPILE__)
    // word 3: raw (unswizzled) dword-addressed buffer on gfx9-family parts
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes,
                                             0x00020000);
#else
    return Rsrc{};
#endif
}

template <typename T> __device__ __forceinline__ T buf_load(Rsrc r, uint32_t voff, uint32_t soff);
template <> __device__ __forceinline__ float buf_load<float>(Rsrc r, uint32_t voff, uint32_t soff)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_bit_cast(float,
                              __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
#else
    return 0.0f;
#endif
}
template <>
__device__ __forceinline__ double buf_load<double>(Rsrc r, uint32_t voff, uint32_t soff)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_bit_cast(double,
                              __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
#else
    return 0.0;
#endif
}

__device__ __forceinline__ float sat(float v) { return __builtin_amdgcn_fmed3f(v, 0.0f, 1.0f); }
__device__ __forceinline__ double sat(double v) { return fmin(fmax(v, 0.0), 1.0); }

__device__ __forceinline__ float frc(float v) { return __builtin_amdgcn_fractf(v); }
__device__ __forceinline__ double frc(double v) { return v - floor(v); }

// Square root of a TV term: the hardware instruction for FP32 (within 1 ulp;
// both sides of every TV comparison use it), IEEE sqrt for FP64.
__device__ __forceinline__ float tsqrt(float v) { return __builtin_amdgcn_sqrtf(v); }
__device__ __forceinline__ double tsqrt(double v) { return sqrt(v); }

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

// Block sum of NV values into dst[0..NV) (thread k < NV writes dst[k]).
// Every thread of the block must call this.
template <int NV, typename A>
__device__ void block_store(const A (&v)[NV], double *dst)
{
    __shared__ double sh[NV][16];   // up to 1024 threads
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = wave_sum((double)v[k]);
        if (lane == 0) sh[k][wid] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += sh[threadIdx.x][w];
        gl(dst)[threadIdx.x] = s;
    }
    __syncthreads();
}

// Block sums of NV values of a kBlock-thread block into dst[k] for
// first <= k < NV, through LDS: one row per value, eight lanes per row, each
// lane summing a fixed stride-8 subset in order and a three-step butterfly
// joining the eight (many values cost a few LDS passes instead of a shuffle
// tree each). Every thread of the block must call this.
template <int NV, typename A>
__device__ void block_store_rows(const A (&v)[NV], double *dst, int first)
{
    static_assert(NV * 8 <= kBlock, "eight lanes per value");
    constexpr int S = kBlock + 8;   // row stride: the next row's lanes start 8 banks on
    __shared__ A sh[NV * S];
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[k * S + threadIdx.x] = v[k];
    __syncthreads();
    const int k = threadIdx.x >> 3, p = threadIdx.x & 7;
    double acc = 0.0;
    if (k < NV) {
        for (int i = 0; i < kBlock / 8; ++i) acc += (double)sh[k * S + p + 8 * i];
    }
    acc += __shfl_xor(acc, 1, 64);
    acc += __shfl_xor(acc, 2, 64);
    acc += __shfl_xor(acc, 4, 64);
    if (k < NV && k >= first && p == 0) gl(dst)[k] = acc;
    __syncthreads();
}

// tot[k] = sum over blocks b of partials[b * stride + k], k < nv: lane-strided
// runs, then a fixed butterfly; one wave per value so that all loads are in
// flight together. tot is in shared memory and valid in every thread after.
__device__ void final_sums(const double *partials, int nblk, int stride, int nv, double *tot)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    constexpr int U = 8;   // loads in flight per lane
    for (int k = wid; k < nv; k += nw) {
        double acc = 0.0;
        const auto *pg = gl(partials);
        for (int b0 = lane; b0 < nblk; b0 += 64 * U) {
            double v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int b = b0 + 64 * u;
                v[u] = b < nblk ? pg[(size_t)b * stride + k] : 0.0;
            }
            // the lane's running sum in block order, as one load at a time
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (b0 + 64 * u < nblk) acc += v[u];
        }
        acc = wave_sum(acc);
        if (lane == 0) tot[k] = acc;
    }
    __syncthreads();
}

// Sum over b < nblk of partials[b], formed by every thread of a kBlock-thread
// block (b strided by the block, four loads in flight, then fixed butterflies
// and the waves' sums in order) and returned to all of them. Every block that
// calls it on the same data gets the same bits: a kernel that needs a scalar
// of the previous launch forms it itself, and the finisher that records it
// forms the same value.
__device__ double block_sum1(const double *partials, int nblk)
{
    __shared__ double wsum[kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    constexpr int U = 8;
    const auto *pg = gl(partials);
    double acc = 0.0;
    for (int b0 = threadIdx.x; b0 < nblk; b0 += kBlock * U) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int b = b0 + kBlock * u;
            v[u] = b < nblk ? pg[b] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (b0 + kBlock * u < nblk) acc += v[u];
    }
    acc = wave_sum(acc);
    __syncthreads();   // a previous call's readers are done with wsum
    if (lane == 0) wsum[wid] = acc;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) t += wsum[w];
    return t;
}

// block_sum1 of two arrays (element b at pa[b * as], pb[b * bs]) with the
// loads of both in flight together; each result has the bits block_sum1
// gives for its array. The first kBlock threads take part, so a wider block
// forms the same bits; every thread of the block must call it.
__device__ void block_sum2(const double *pa, int na, const double *pb, int nb, double &sa,
                           double &sb, int as = 1, int bs = 1)
{
    __shared__ double wsum[2][kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    constexpr int U = 8;
    const auto *ga = gl(pa);
    const auto *gb = gl(pb);
    const int n = threadIdx.x < kBlock ? (na > nb ? na : nb) : 0;
    double acc_a = 0.0, acc_b = 0.0;
    for (int b0 = threadIdx.x; b0 < n; b0 += kBlock * U) {
        double va[U], vb[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int b = b0 + kBlock * u;
            va[u] = b < na ? ga[(size_t)b * as] : 0.0;
            vb[u] = b < nb ? gb[(size_t)b * bs] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (b0 + kBlock * u < na) acc_a += va[u];
            if (b0 + kBlock * u < nb) acc_b += vb[u];
        }
    }
    acc_a = wave_sum(acc_a);
    acc_b = wave_sum(acc_b);
    __syncthreads();   // a previous call's readers are done with wsum
    if (lane == 0 && wid < kBlock / 64) {
        wsum[0][wid] = acc_a;
        wsum[1][wid] = acc_b;
    }
    __syncthreads();
    sa = 0.0;
    sb = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
        sa += wsum[0][w];
        sb += wsum[1][w];
    }
}

// Variants whose step size alpha = -g'^T p' / ||A p'||^2 is formed by the TV
// pass that uses it (and recorded by that pass's finisher) instead of by a
// finisher launch of its own.
__device__ __forceinline__ bool local_alpha(int variant)
{
    return variant == SCG_S_CG || variant == SCG_S_CG_CD || variant == SCG_S_PCG;
}

__device__ __forceinline__ bool stopped(const DevState *st)
{
    return st != nullptr && gl(st)->done;
}

// Trace entry of the open step: k + kofs (entries count from 1).
template <typename S> __device__ __forceinline__ auto trace_at(S *st, scg_trace_entry *trace)
{
    using R = decltype(gl(trace));
    const int k = st->k + st->kofs;
    if (trace == nullptr || k < 1 || k > st->trace_cap) return (R) nullptr;
    return gl(trace) + (k - 1);
}

template <typename S> __device__ __forceinline__ void set_done(S *st, int status)
{
    st->done = 1;
    st->status = status;
}

// gtab[m] = gamma0 a^(l+m), m < max_trials: the step sizes of the trials of
// the step that starts with counter value l (rounded to the image precision,
// the value the trials and the accepted perturbation use). All threads of
// the block take part.
// gamma_{l+m} = gamma0 a^(l+m) (eq. of the gamma sequence), in the solve's
// precision: every kernel that needs one forms it with this formula, so all
// get the same bits.
template <typename S> __device__ __forceinline__ double gamma_at(const S *st, int ell, int m)
{
    const double g = st->gamma0 * pow(st->a, (double)(ell + m));
    return st->is_f32 ? (double)(float)g : g;
}

template <typename S> __device__ __forceinline__ void fill_gtab(double *gtab, S *st, int ell)
{
    const int mt = st->max_trials;
    auto *gt = gl(gtab);
    for (int m = threadIdx.x; m < mt; m += blockDim.x) gt[m] = gamma_at(st, ell, m);
}

// The first trial launch's entries of the table, gamma_{l+m} for m <
// kTrialsPerPass and the current l (the threads below kTrialsPerPass).
template <typename S> __device__ __forceinline__ void fill_first_gammas(double *gtab, S *st)
{
    const int m = threadIdx.x;
    if (m < kTrialsPerPass && m < st->max_trials) gl(gtab)[m] = gamma_at(st, st->ell, m);
}

inline int vec_blocks(size_t n)
{
    size_t b = (n + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > (size_t)kMaxVecBlocks) b = kMaxVecBlocks;
    return (int)b;
}

// Block coordinates of a body: (x, y) in an (nx, ny) grid.
struct VBlk {
    int x, y, nx, ny;
    __device__ int id() const { return y * nx + x; }
    __device__ int count() const { return nx * ny; }
};

__device__ __forceinline__ VBlk vblk_of(int local, int nx, int ny)
{
    return VBlk{local % nx, local / nx, nx, ny};
}

__device__ __forceinline__ VBlk grid_vblk()
{
    return VBlk{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, (int)gridDim.y};
}

// Launch-order block index. With swz, consecutive indices go to the same
// XCD: the hardware hands workgroup b to XCD b mod 8, so the blocks the
// hardware places on one XCD get one contiguous range of indices and share
// that XCD's L2 for the data neighbouring blocks read.
__device__ __forceinline__ int launch_index(int swz)
{
    const int b = blockIdx.x, n = gridDim.x;
    if (!swz) return b;
    const int per = n / kXcds, rem = n % kXcds;
    const int xcd = b % kXcds, idx = b / kXcds;
    return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

// A solve's descriptor (a copy: the bodies' stores cannot alias it).
template <typename T> __device__ __forceinline__ Solve<T> load_solve(const Solve<T> *S, int i)
{
    return gl(S)[i];
}

// The solve and the local block index of a batched launch's block. The
// streaming kernels take the XCD-contiguous order (the default): a tile and
// the neighbours whose edge rows it reads then sit on one XCD, and the rows
// they share are fetched into one L2 instead of several. The operators pass
// their tuned order.
__device__ __forceinline__ BlkMap locate(const BlkMap *map, int swz = 1)
{
    const int b = launch_index(swz);
    if (map == nullptr) return BlkMap{0, b};
    return map[b];
}

}  // namespace

int blocks_xtv(const Geo &G) { return ((G.n + 31) / 32) * ((G.n + kXtvRows - 1) / kXtvRows); }
int blocks_t32(const Geo &G) { return ((G.n + 31) / 32) * ((G.n + 31) / 32); }
int blocks_vec(size_t n) { return vec_blocks(n); }
int blocks_sv(const Geo &G) { return G.na; }
int blocks_bp(const Geo &G, bool mirror)
{
    const int t = (G.n + kBpTile - 1) / kBpTile;
    return t * (mirror ? bp_mirror_cols(G.n) : t);
}
int blocks_trials(const Geo &G, int nchunks)
{
    const int b = vec_blocks((size_t)(G.n - 1) * (G.n - 1));
    const int cap = kMaxPartials / (1 + kTrialsPerPass * nchunks);
    return b < cap ? b : cap;
}

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

// Output copy of every solve of a batch (x_{k+1/2} for the S- variants, x
// for CG), run after the loop whether or not the solve stopped.
template <typename T>
__global__ __launch_bounds__(256) void kb_copy_out(const Solve<T> *S, const BlkMap *map,
                                                    int from_xh)
{
    const BlkMap m = locate(map);
    const Solve<T> d = load_solve(S, m.solve);
    const auto *src = gl(from_xh ? d.xh : d.x);
    auto *dst = gl(d.xout);
    const size_t J = (size_t)d.G.n * d.G.n;
    for (size_t i = m.local * (size_t)blockDim.x + threadIdx.x; i < J;
         i += (size_t)d.nb_vec * blockDim.x)
        dst[i] = src[i];
}

template <typename T>
void launch_b_copy_out(const Solve<T> *S, const BlkMap *map, int nblocks, int from_xh,
                       hipStream_t s)
{
    hipLaunchKernelGGL(kb_copy_out<T>, dim3(nblocks), dim3(kBlock), 0, s, S, map, from_xh);
}

// ---------------------------------------------------------------------------
// Image staging: the transposed copy that angles stepping over columns read
// (32x32 tiles through LDS so both the read and the write are coalesced).
// ---------------------------------------------------------------------------

template <typename T>
__device__ void stage_body(const T *__restrict__ x_, T *__restrict__ xt_, const Geo &G, VBlk vb)
{
    const auto *x = gl(x_);
    auto *xt = gl(xt_);
    __shared__ T tile[32][33];
    const int n = G.n;
    const int bx = vb.x * 32, by = vb.y * 32;
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
__global__ __launch_bounds__(256) void k_stage(const T *__restrict__ x, T *__restrict__ xt, Geo G)
{
    stage_body(x, xt, G, grid_vblk());
}

template <typename T> void launch_stage(const T *x, T *xt, const Geo &G, hipStream_t s)
{
    dim3 grid((G.n + 31) / 32, (G.n + 31) / 32);
    hipLaunchKernelGGL(k_stage<T>, grid, dim3(256), 0, s, x, xt, G);
}

template <typename T>
__global__ __launch_bounds__(256) void kb_stage(const Solve<T> *S, const BlkMap *map, int phase)
{
    const BlkMap m = locate(map);
    const Solve<T> d = load_solve(S, m.solve);
    if (stopped(d.st)) return;
    const int nt = (d.G.n + 31) / 32;
    stage_body(phase == kStageX ? d.x : d.xh, d.xs, d.G, vblk_of(m.local, nt, nt));
}

template <typename T>
void launch_b_stage(const Solve<T> *S, const BlkMap *map, int nblocks, int phase, hipStream_t s)
{
    hipLaunchKernelGGL(kb_stage<T>, dim3(nblocks), dim3(256), 0, s, S, map, phase);
}

// ---------------------------------------------------------------------------
// Forward projector A (ray-driven, banded). Block (bin chunk, angle group):
// NQ groups of kPjBins threads; thread t owns bin b = chunk*kPjBins +
// (t mod 2 kPjBins) / 2 for the group's angles 2 (t / 2 kPjBins) + (t mod 2)
// + NQ m (each wavefront traces 32 bins of two neighbouring angles, lanes
// alternating between them). The block walks bands of kPjBand steps along the
// group's major axis (rows of x, or rows of x^T for angles stepping over
// columns), staging kPjWin columns of each band in LDS, column-major with a
// stride of kPjBand + 1 elements (the two split columns of a step are one
// paired read); the next band is prefetched into registers while the
// current one is consumed. Within a band a ray's crossing coordinate is an integer anchor
// plus an FP32 fraction (the anchor from FP64), so the split weights stay
// accurate near the axes where the chord ramp is steep. Per step: the
// crossing, its integer part and fraction, one clamped FMA for the split weight, two
// LDS reads and three FMAs/adds. With y given, out = A x - y. With partials
// given, the block stores its sum of out^2, or of out * dotv with dotv given
// (same layout as out).
//
// Mirrored form (MIR, tables over the angles a <= n_a / 2): mirroring the
// image about its vertical axis maps ray (a, b) onto ray (n_a - a, b), so a
// ray's crossings, split weights and LDS addresses also serve that second
// ray, read from a second window of the band that holds the mirrored image
// (columns reversed for angles stepping over rows; for angles stepping over
// columns, the rows of x^T reversed). Each LDS column then holds the band's
// kPjBand rows followed by the same rows of the mirrored window, so both
// paired reads of a step come from one address with immediate offsets.
// Angle 0 and angle n_a / 2 are their own mirrors: their slots form one ray.
// A pair of rays is half the threads of the plain form, so the block has two
// halves that trace the same rays over the first and the second half of each
// band's rows, and the second half's sums join the first's at the end.
// ---------------------------------------------------------------------------

// Waves per SIMD a projector instance is compiled for: the FP32 mirrored
// form's 1024-thread blocks need two per CU (8 waves per SIMD, at most 64
// VGPRs) to match the plain form's occupancy; the others keep the default.
template <typename T, int NQ, bool MIR> constexpr int pj_min_waves()
{
    return (MIR && NQ == 4 && sizeof(T) == 4) ? 8 : 1;
}

// Block id of the projector's local block index: heaviest first in launch
// order (the XCD-contiguous order keeps neighbouring blocks together instead).
__device__ __forceinline__ int pj_block(const ProjTables &P, int local, int swz)
{
    return (swz || P.order == nullptr) ? local : gl(P.order)[local];
}

template <typename T, int NQ, int GA, bool MIR>
__device__ void project_body(const T *__restrict__ x, const T *__restrict__ xt, const Geo &G,
                             const ProjTables &P, const T *__restrict__ y, int y_stride,
                             T *__restrict__ out, int out_stride, int out_off,
                             const T *__restrict__ dotv, double *partials, VBlk vb)
{
    constexpr int NH = MIR ? 2 : 1;               // halves of a band's rows
    constexpr int NTQ = kPjBins * NQ;             // threads of one half
    constexpr int NT = NTQ * NH;
    constexpr int KH = kPjBand / NH;              // rows of a band per half
    // steps whose LDS reads are in flight together (two in the mirrored
    // form, which holds four reads per step within its 64 VGPRs)
    constexpr int GS = MIR ? 2 : kPjGroupSteps;
    // LDS column stride (elements): the band's rows, then (MIR) the mirrored
    // window's from one element past them; odd, so a half-wavefront's reads
    // at one step stay in distinct banks, and a step's four reads pair into
    // two-address reads (k, MO + k) and (LS + k, LS + MO + k) whose two
    // addresses lie in different banks
    constexpr int LS = (MIR ? 2 : 1) * kPjBand + 1;
    constexpr int MO = kPjBand + 1;               // offset of the mirrored rows
    constexpr int LSZ = kPjWin * LS;
    constexpr int SLOTS = GA / NQ;
    constexpr int RPT = kPjWin * kPjBand / NT;    // staged rows per thread
    static_assert(GA % NQ == 0 && GA <= kPjGroup && NT % kPjWin == 0 && kPjBand % RPT == 0,
                  "projector tiling");
    __shared__ T lds[LSZ];
    const int t = threadIdx.x;
    const int chunk = vb.x, gi = vb.y;
    const PjGroup grp = gl(P.groups)[gi];
    const auto *pang = gl(P.ang);
    // Each wavefront traces 32 bins of two neighbouring angles, the angles
    // alternating lane by lane: the rays of a half-wavefront then cross at
    // most about 24 columns of a row (16 bins at up to sqrt(2) columns
    // apart), so their paired LDS reads fall in distinct banks; 64 bins of
    // one angle would span up to 90 columns and collide.
    const int th = MIR ? t % NTQ : t;             // thread within its half
    const int half = MIR ? t / NTQ : 0;
    const int quarter = 2 * (th / (2 * kPjBins)) + (th & 1);
    const int b_raw = chunk * kPjBins + ((th & (2 * kPjBins - 1)) >> 1);
    const bool bin_ok = b_raw < G.nb;
    const int b = bin_ok ? b_raw : G.nb - 1;   // idle lanes trace the chunk's last ray
    const int n = G.n;
    const Rsrc img = buf_rsrc(grp.major ? xt : x, (uint32_t)((size_t)n * n * sizeof(T)));
    const uint32_t rowb = (uint32_t)n * (uint32_t)sizeof(T);   // bytes per image row
    const auto *win = gl(P.win) + ((size_t)gi * P.n_chunks + chunk) * P.n_bands;
    const int scol = t % kPjWin, srow = (t / kPjWin) * RPT;

    double u0[SLOTS];
    T acc[SLOTS], accr[SLOTS], macc[SLOTS], maccr[SLOTS];
#pragma unroll
    for (int m = 0; m < SLOTS; ++m) {
        const int slot = quarter + NQ * m;
        acc[m] = T(0);
        accr[m] = T(0);
        macc[m] = T(0);
        maccr[m] = T(0);
        u0[m] = 0.0;
        if (slot < grp.count) {
            const auto &A = pang[grp.a0 + slot];
            u0[m] = fma((double)b, A.u0_step, A.u0_base);
        }
    }

    // the group's angle parameters, read by every band from LDS (each lane's
    // angle is its own, so a global load per band would stall the band)
    __shared__ double s_slope[kPjGroup];
    __shared__ T s_K[kPjGroup], s_C[kPjGroup];
    if (t < grp.count) {
        const auto &A = pang[grp.a0 + t];
        s_slope[t] = A.slope;
        s_K[t] = sizeof(T) == 4 ? (T)A.Kf : (T)A.K;
        s_C[t] = sizeof(T) == 4 ? (T)A.Cf : (T)A.C;
    }

    // staging loads: one per row, columns outside the image read as zero
    T pre[RPT], mpre[MIR ? RPT : 1];
    auto prefetch = [&](int band) {
        const int jw = win[band];
        const int i0 = band * kPjBand + srow;
        const int col = jw + scol;
        const bool cok = col >= 0 && col < n;
        const uint32_t vo = cok ? (uint32_t)(i0 * n + col) * (uint32_t)sizeof(T) : kBufOob;
        const bool full = (band + 1) * kPjBand <= n;
        if (full) {
            // every row of the band exists: the row step is a scalar offset
#pragma unroll
            for (int r = 0; r < RPT; ++r) pre[r] = buf_load<T>(img, vo, (uint32_t)r * rowb);
        } else {
            // last band of a ragged image: rows past the end read as zero
#pragma unroll
            for (int r = 0; r < RPT; ++r) pre[r] = buf_load<T>(img, vo + (uint32_t)r * rowb, 0u);
        }
        if constexpr (MIR) {
            if (!grp.major) {
                // rows of x: the mirrored window is column n - 1 - col of
                // the same rows (inside the image exactly when col is)
                const uint32_t mvo =
                    cok ? (uint32_t)(i0 * n + (n - 1 - col)) * (uint32_t)sizeof(T) : kBufOob;
                if (full) {
#pragma unroll
                    for (int r = 0; r < RPT; ++r)
                        mpre[r] = buf_load<T>(img, mvo, (uint32_t)r * rowb);
                } else {
#pragma unroll
                    for (int r = 0; r < RPT; ++r)
                        mpre[r] = buf_load<T>(img, mvo + (uint32_t)r * rowb, 0u);
                }
            } else {
                // rows of x^T: band row i0 + r mirrors to row n - 1 - i0 - r;
                // load them upwards from the lowest, mpre[r] holding band row
                // srow + RPT - 1 - r. Rows above the image (a ragged last
                // band) have a negative index: as an unsigned offset it lies
                // past the view and reads zero.
                const int lo = n - i0 - RPT;
                if (full) {
                    const uint32_t mvo =
                        cok ? (uint32_t)(lo * n + col) * (uint32_t)sizeof(T) : kBufOob;
#pragma unroll
                    for (int r = 0; r < RPT; ++r)
                        mpre[r] = buf_load<T>(img, mvo, (uint32_t)r * rowb);
                } else {
#pragma unroll
                    for (int r = 0; r < RPT; ++r)
                        mpre[r] = buf_load<T>(
                            img, cok ? (uint32_t)((lo + r) * n + col) * (uint32_t)sizeof(T) : kBufOob,
                            0u);
                }
            }
        }
    };

    // The plain form loads the next band into registers while it works on
    // the current one. The mirrored form issues a band's loads just before
    // the barrier that precedes its LDS stores: holding them through the
    // band's steps would take 16 more VGPRs than its 64 allow, and with two
    // blocks per CU one block's steps cover the other's loads.
    constexpr bool PRE = !MIR;
    int band = 0;
    while (band < P.n_bands && win[band] == kWinSkip) ++band;
    if (PRE && band < P.n_bands) prefetch(band);
    while (band < P.n_bands) {
        if (!PRE) prefetch(band);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RPT; ++r) lds[scol * LS + srow + r] = pre[r];
        if constexpr (MIR) {
            if (!grp.major) {
#pragma unroll
                for (int r = 0; r < RPT; ++r) lds[scol * LS + MO + srow + r] = mpre[r];
            } else {
#pragma unroll
                for (int r = 0; r < RPT; ++r) lds[scol * LS + MO + srow + RPT - 1 - r] = mpre[r];
            }
        }
        __syncthreads();
        const int jw = win[band];
        const int i0 = band * kPjBand;
        int nxt = band + 1;
        while (nxt < P.n_bands && win[nxt] == kWinSkip) ++nxt;
        if (PRE && nxt < P.n_bands) prefetch(nxt);
#pragma unroll
        for (int m = 0; m < SLOTS; ++m) {
            const int slot = quarter + NQ * m;
            if (slot < grp.count) {
                const double slope64 = s_slope[slot];
                const double us = fma((double)i0, slope64, u0[m]);
                // The band adds exactly zero for a ray whose crossings stay
                // left of column -1 or right of column n over its rows (both
                // split columns are zero padding); skip it when that holds
                // for the whole wavefront.
                const double ue = fma((double)(kPjBand - 1), slope64, us);
                const bool miss = fmax(us, ue) < -1.0 || fmin(us, ue) > (double)n;
                if (__all(miss)) continue;
                // anchor one column left of the ray's leftmost crossing in the
                // band: every step's offset from it is at least 1, so the
                // column is the truncation of the offset
                const double fu = floor(fmin(us, ue)) - 1.0;
                // byte offset in LDS of the anchor column at the half's
                // first row; a step's column adds a 24-bit multiple of the
                // column stride
                const int kb = half * KH;
                const int cb = ((int)fu - jw) * (LS * (int)sizeof(T)) + kb * (int)sizeof(T);
                const T slope = (T)slope64;
                const T F0 = MIR ? fma((T)kb, slope, (T)(us - fu)) : (T)(us - fu);
                const T K = s_K[slot];
                const T C = s_C[slot];
                // the band's terms are summed apart and then added to the
                // ray's sum: rounding grows with the band plus the band count,
                // not with N
                T a_ = T(0), ar = T(0), ma = T(0), mar = T(0);
                // steps in groups of kPjGroupSteps: the group's LDS reads are
                // issued before its terms are summed (in step order)
#pragma unroll
                for (int k0 = 0; k0 < KH; k0 += GS) {
                    T xl[GS], xr[GS], wl[GS];
                    T ml[MIR ? GS : 1], mr[MIR ? GS : 1];
#pragma unroll
                    for (int j = 0; j < GS; ++j) {
                        const int k = k0 + j;
                        const T v = fma((T)k, slope, F0);
                        const int jl = (int)v;
                        wl[j] = sat(fma(frc(v), -K, C));
                        const T *col = reinterpret_cast<const T *>(
                            reinterpret_cast<const char *>(lds) +
                            __mul24(jl, LS * (int)sizeof(T)) + cb);
                        xl[j] = col[k];
                        xr[j] = col[LS + k];
                        if constexpr (MIR) {
                            ml[j] = col[MO + k];
                            mr[j] = col[LS + MO + k];
                        }
                    }
#pragma unroll
                    for (int j = 0; j < GS; ++j) {
                        a_ = fma(wl[j], xl[j] - xr[j], a_);
                        ar += xr[j];
                        if constexpr (MIR) {
                            ma = fma(wl[j], ml[j] - mr[j], ma);
                            mar += mr[j];
                        }
                    }
                }
                acc[m] += a_;
                accr[m] += ar;
                if constexpr (MIR) {
                    macc[m] += ma;
                    maccr[m] += mar;
                }
            }
        }
        band = nxt;
    }

    if constexpr (MIR) {
        // the second half's sums join the first half's (LDS reused once
        // every band's reads are done)
        static_assert(4 * SLOTS * NTQ <= LSZ, "projector half sums");
        __syncthreads();
        if (half == 1) {
#pragma unroll
            for (int m = 0; m < SLOTS; ++m) {
                lds[(4 * m + 0) * NTQ + th] = acc[m];
                lds[(4 * m + 1) * NTQ + th] = accr[m];
                lds[(4 * m + 2) * NTQ + th] = macc[m];
                lds[(4 * m + 3) * NTQ + th] = maccr[m];
            }
        }
        __syncthreads();
        if (half == 0) {
#pragma unroll
            for (int m = 0; m < SLOTS; ++m) {
                acc[m] += lds[(4 * m + 0) * NTQ + th];
                accr[m] += lds[(4 * m + 1) * NTQ + th];
                macc[m] += lds[(4 * m + 2) * NTQ + th];
                maccr[m] += lds[(4 * m + 3) * NTQ + th];
            }
        }
    }
    double sq = 0.0;
#pragma unroll
    for (int m = 0; m < SLOTS; ++m) {
        const int slot = quarter + NQ * m;
        if (slot < grp.count && bin_ok && half == 0) {
            const int a = grp.a0 + slot;
            const T im = sizeof(T) == 4 ? (T)pang[a].inv_mf : (T)pang[a].inv_m;
            T val = (acc[m] + accr[m]) * im;
            if (y != nullptr) val -= gl(y)[(size_t)a * y_stride + b];
            const size_t o = (size_t)a * out_stride + out_off + b;
            gl(out)[o] = val;
            const T w = dotv != nullptr ? gl(dotv)[o] : val;
            sq += (double)val * (double)w;
            if constexpr (MIR) {
                // the mirrored ray n_a - a (angles 0 and n_a / 2 have none)
                const int am = G.na - a;
                if (a > 0 && am != a) {
                    T mv = (macc[m] + maccr[m]) * im;
                    if (y != nullptr) mv -= gl(y)[(size_t)am * y_stride + b];
                    const size_t mo = (size_t)am * out_stride + out_off + b;
                    gl(out)[mo] = mv;
                    const T mw = dotv != nullptr ? gl(dotv)[mo] : mv;
                    sq += (double)mv * (double)mw;
                }
            }
        }
    }
    if (partials == nullptr) return;
    double v[1] = {sq};
    block_store(v, partials + vb.id());
}

template <typename T, int NQ, int GA, bool MIR>
__global__ __launch_bounds__(kPjBins * NQ * (MIR ? 2 : 1), (pj_min_waves<T, NQ, MIR>())) void k_project(const T *__restrict__ x,
                                                          const T *__restrict__ xt, Geo G,
                                                          ProjTables P, T *__restrict__ out,
                                                          int out_stride, int out_off, int swz)
{
    project_body<T, NQ, GA, MIR>(x, xt, G, P, nullptr, 0, out, out_stride, out_off, nullptr,
                                 nullptr,
                                 vblk_of(pj_block(P, launch_index(swz), swz), P.n_chunks,
                                         P.n_groups));
}

template <typename T>
void launch_project(const T *x, const T *xt, const Geo &G, const ProjTables &P, T *out,
                    int out_stride, int out_off, int nq, int swz, hipStream_t s)
{
    dim3 grid(P.n_chunks * P.n_groups);
    auto go = [&](auto kern, int nthreads) {
        hipLaunchKernelGGL(kern, grid, dim3(nthreads), 0, s, x, xt, G, P, out, out_stride,
                           out_off, swz);
    };
    const bool g8 = P.group_max > 4;
    if (P.mirror) {
        if (nq == 4)
            g8 ? go(k_project<T, 4, 8, true>, kPjBins * 8) : go(k_project<T, 4, 4, true>, kPjBins * 8);
        else
            g8 ? go(k_project<T, 2, 8, true>, kPjBins * 4) : go(k_project<T, 2, 4, true>, kPjBins * 4);
    } else {
        if (nq == 4)
            g8 ? go(k_project<T, 4, 8, false>, kPjBins * 4)
               : go(k_project<T, 4, 4, false>, kPjBins * 4);
        else
            g8 ? go(k_project<T, 2, 8, false>, kPjBins * 2)
               : go(k_project<T, 2, 4, false>, kPjBins * 2);
    }
}

template <typename T, int NQ, int GA, bool MIR>
__global__ __launch_bounds__(kPjBins * NQ * (MIR ? 2 : 1), (pj_min_waves<T, NQ, MIR>())) void kb_project(const Solve<T> *S, const BlkMap *map,
                                                           int phase, int swz)
{
    const BlkMap m = locate(map, swz);
    const Solve<T> d = load_solve(S, m.solve);
    if (stopped(d.st)) return;
    // descriptor fields into registers: the body's stores cannot alias them
    const Geo G = d.G;
    const ProjTables P = d.P;
    const VBlk vb = vblk_of(pj_block(P, m.local, swz), P.n_chunks, P.n_groups);
    // one body instance: pick the phase's vectors first (kPjU: u = A g'
    // into rt with the partials of u^T q)
    const bool q = phase == kPjQ, u = phase == kPjU;
    const T *img = q ? d.p : (u ? d.g : (phase == kPjResX ? d.x : d.xh));
    const T *imgt = q ? d.pt : d.xs;
    const T *y = (q || u) ? nullptr : d.y;
    T *out = q ? d.q : (u ? d.rt : d.r);
    const T *dv = u ? d.q : nullptr;
    double *part = phase == kPjResXhF ? d.partials2 : d.partials;
    project_body<T, NQ, GA, MIR>(img, imgt, G, P, y, G.nb, out, G.rs, kSinoPadL, dv, part, vb);
}

template <typename T>
void launch_b_project(const Solve<T> *S, const BlkMap *map, int nblocks, int phase, int nq,
                      int ga, int mir, int swz, hipStream_t s)
{
    auto go = [&](auto kern, int nthreads) {
        hipLaunchKernelGGL(kern, dim3(nblocks), dim3(nthreads), 0, s, S, map, phase, swz);
    };
    const bool g8 = ga > 4;
    if (mir) {
        if (nq == 4)
            g8 ? go(kb_project<T, 4, 8, true>, kPjBins * 8) : go(kb_project<T, 4, 4, true>, kPjBins * 8);
        else
            g8 ? go(kb_project<T, 2, 8, true>, kPjBins * 4) : go(kb_project<T, 2, 4, true>, kPjBins * 4);
    } else {
        if (nq == 4)
            g8 ? go(kb_project<T, 4, 8, false>, kPjBins * 4)
               : go(kb_project<T, 4, 4, false>, kPjBins * 4);
        else
            g8 ? go(kb_project<T, 2, 8, false>, kPjBins * 2)
               : go(kb_project<T, 2, 4, false>, kPjBins * 2);
    }
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
// Backprojector A^T (pixel-driven, tiled). A tile of 16 x 16 pixels is owned
// by NS groups of 128 threads; thread t of a group owns the pixels (t >> 3,
// 2(t & 7)) and (t >> 3, 2(t & 7) + 1), and group gs takes the angle chunks
// gs, gs + NS, ... (the groups' sums are added in a fixed order at the end).
// Angles are processed in chunks of kBpChunk (half that in the mirrored form
// below): for each angle the kBpWin bins
// around the tile centre's projection are staged in LDS, already scaled by
// 1/m, next to the angle's parameters (cos and the weight constants) and,
// for each of the tile's 16 rows, the row's part of the footprint position
// (the centre's fractional position plus the row offset times sin, shared
// by the 8 threads of a row); the next chunk is prefetched into registers
// while the current one is consumed. A pixel's footprint centre is an FP32
// offset from the tile centre (it stays in (4, 27) bins) and takes one FMA
// per angle, its two bins are two LDS reads and its two weights two clamped
// FMAs. DUAL
// backprojects a second sinogram with the same weights (S-PCG: g' and z').
// MIR uses the image's mirror symmetry about its vertical axis: the pixel
// (i, n-1-j) at angle pi - theta lies at the same detector position as
// (i, j) at theta (and at angle 0 at the mirrored position), so one
// footprint position and its two weights serve both pixels. The launch then
// covers the tiles of the left ceil(n/2) columns; each thread reads a second
// staged window, taken from the mirror angle's row (row 0 reversed for angle
// 0), and also writes the mirror pixels. This uses angle theta's parameters
// for pi - theta, i.e. a trig table made exactly symmetric, which moves A^T
// by about 1e-13 relative in FP64 (the table's asymmetry is a few units in
// the last place). With partials given, the block stores its part of a dot
// product: dot = 1, out (or out2 when DUAL) against dotv; dot = 2, out
// against itself; dot = 3 (DUAL), out against out2.
// ---------------------------------------------------------------------------

constexpr int kBpPrm = 4;   // per-angle parameters staged in LDS
// Waves per SIMD the FP32 backprojector is held to: eight (at most 64
// VGPRs) for one sinogram and for the mirrored form's 1024-thread blocks (two
// fit a CU's LDS), six for its smaller blocks; the others are left to the
// compiler.
template <typename T, bool DUAL, bool MIR, int NS>
constexpr int kBpWaves = sizeof(T) != 4 || DUAL ? 1 : (MIR && NS < 8 ? 6 : 8);
constexpr int kBpRt = kBpTile / (kBpThreads / kBpChunk);   // row terms per thread
static_assert(kBpThreads % kBpChunk == 0 && kBpRt * (kBpThreads / kBpChunk) == kBpTile,
              "the threads of an angle cover the tile's rows");

template <typename T, bool DUAL, int NS, bool MIR = false>
__device__ void backproject_body(const T *__restrict__ r, const T *__restrict__ r2, const Geo &G,
                                 const BpAngle *__restrict__ ang, T *__restrict__ out,
                                 T *__restrict__ out2, T *__restrict__ outT,
                                 const T *__restrict__ dotv, int dot, double *partials, VBlk vb)
{
    static_assert(!(DUAL && MIR), "the mirrored form backprojects one sinogram");
    constexpr int NW = DUAL || MIR ? 2 : 1;
    // the mirrored form stages half as many angles per chunk, so that two
    // 1024-thread blocks (eight angle groups) fit a CU's LDS
    constexpr int CH = MIR ? kBpChunk / 2 : kBpChunk;
    constexpr int RT = kBpTile / (kBpThreads / CH);   // row terms per thread
    static_assert(kBpThreads % CH == 0 && RT * (kBpThreads / CH) == kBpTile, "row terms");
    constexpr int NE = CH * kBpWin / kBpThreads;   // staged bins per thread and sinogram
    // an angle's windows side by side (the second one's reads take the
    // first one's address plus an immediate offset)
    __shared__ T win[NS][CH][NW][kBpWin];
    // angle parameters and row terms, two buffers: the next chunk's are
    // written while the current chunk's are read
    __shared__ T prm[2][NS][CH * kBpPrm];
    __shared__ T rowt[2][NS][CH * kBpTile];
    static_assert(NS * CH * NW * kBpWin >= (NS - 1) * kBpThreads * 2 * NW,
                  "combine buffer fits in the windows");
    const int gs = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kBpThreads);
    const int t = threadIdx.x % kBpThreads;
    const int ty = t >> 3, tx = (t & 7) * 2;
    const int i0 = vb.y * kBpTile, j0 = vb.x * kBpTile;
    const double xc = ((double)j0 + 7.5) - G.h, yc = G.h - ((double)i0 + 7.5);
    const T dx = (T)((double)tx - 7.5);
    T acc0 = T(0), acc1 = T(0), bcc0 = T(0), bcc1 = T(0);
    const int nchunks = (G.na + CH - 1) / CH;

    // Window of each angle of a chunk: first bin and 1/m, from the FP64
    // frame computed once per angle by the params step.
    struct WinRef {
        int base;
        T m;
    };
    __shared__ WinRef wref[NS][CH];
    const Rsrc sino = buf_rsrc(r, (uint32_t)((size_t)G.na * G.rs * sizeof(T)));
    const Rsrc sino2 = buf_rsrc(DUAL ? r2 : r, (uint32_t)((size_t)G.na * G.rs * sizeof(T)));

    T pre[NW][NE];
    // FP64 frame of the chunk's angles (kBpThreads / CH threads per
    // angle, each computing it): the per-pixel parameters and RT of the
    // row terms, written to LDS buffer `buf`, and the window reference the
    // staging loads read.
    auto params = [&](int ch, int buf) {
        const int al = t * RT / kBpTile, r0 = t * RT % kBpTile;
        const int a = ch * CH + al;
        T pp[kBpPrm], rt[RT];
#pragma unroll
        for (int k = 0; k < kBpPrm; ++k) pp[k] = T(0);
#pragma unroll
        for (int k = 0; k < RT; ++k) rt[k] = T(0);
        WinRef w{0, T(0)};
        if (a < G.na) {
            const BpAngle A = gl(ang)[a];
            const BpW<T> W = bpw<T>(A);
            const double pc = fma(xc, A.c, fma(yc, A.s, G.hb));
            const double fb = floor(pc) - kBpHalf;
            const T fr = (T)(pc - fb);
            pp[0] = W.c;
            pp[1] = W.K;
            pp[2] = W.C;
            pp[3] = W.CK;
#pragma unroll
            for (int k = 0; k < RT; ++k) rt[k] = fma((T)(7.5 - (double)(r0 + k)), W.s, fr);
            w.base = (int)fb;
            w.m = (T)A.inv_m;
        }
#pragma unroll
        for (int k = 0; k < RT; ++k) rowt[buf][gs][t * RT + k] = rt[k];
        if (r0 == 0) {
            if (!MIR) {
#pragma unroll
                for (int k = 0; k < kBpPrm; ++k) prm[buf][gs][al * kBpPrm + k] = pp[k];
            }
            wref[gs][al] = w;
        }
    };
    // staging loads of a chunk (after a barrier that follows its params):
    // bins outside the detector and angles past the last read as zero
    auto prefetch = [&](int ch) {
        const int a0 = ch * CH;
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            const int q = t + e * kBpThreads;
            const int al = q / kBpWin, k = q % kBpWin;
            const int a = a0 + al;
            const WinRef w = wref[gs][al];
            const int bb = w.base + k;
            const bool ok = a < G.na && (unsigned)bb < (unsigned)G.nb;
            const uint32_t vo =
                ok ? (uint32_t)(a * G.rs + kSinoPadL + bb) * (uint32_t)sizeof(T) : kBufOob;
            pre[0][e] = buf_load<T>(sino, vo, 0u) * w.m;
            if (DUAL) pre[NW - 1][e] = buf_load<T>(sino2, vo, 0u) * w.m;
            if (MIR) {
                // the mirror pixels' bins: angle na - a at the same bins, or
                // for angle 0 its own row with the bins reversed
                const int am = a == 0 ? 0 : G.na - a;
                const int bm = a == 0 ? G.nb - 1 - bb : bb;
                const uint32_t vm =
                    ok ? (uint32_t)(am * G.rs + kSinoPadL + bm) * (uint32_t)sizeof(T) : kBufOob;
                pre[1][e] = buf_load<T>(sino, vm, 0u) * w.m;
            }
        }
    };

    if (gs < nchunks) params(gs, 0);
    __syncthreads();
    if (gs < nchunks) prefetch(gs);
    for (int c0 = 0; c0 < nchunks; c0 += NS) {
        const int ch = c0 + gs;
        const int cb = (c0 / NS) & 1;
        const bool live = ch < nchunks;
        __syncthreads();
        if (live) {
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                const unsigned q = t + e * kBpThreads;   // angle q / kBpWin, bin q % kBpWin
                T *wb = &win[gs][0][0][0];
                if (NW == 1) {
                    wb[q] = pre[0][e];
                } else {
                    const unsigned o = (q / kBpWin) * (NW * kBpWin) + q % kBpWin;
                    wb[o] = pre[0][e];
                    wb[o + kBpWin] = pre[NW - 1][e];
                }
            }
        }
        // the previous chunk's window references and the other buffer's
        // parameters were read before the barrier above
        if (ch + NS < nchunks) params(ch + NS, cb ^ 1);
        __syncthreads();
        if (ch + NS < nchunks) prefetch(ch + NS);
        const int na = live ? min(CH, G.na - ch * CH) : 0;
        // the chunk's terms are summed apart and then added to the pixel's
        // sum: rounding grows with the chunk size plus the chunk count
        T s0 = T(0), s1 = T(0), e0 = T(0), e1 = T(0);
#pragma unroll 2
        for (int al = 0; al < na; ++al) {
            // the angle's footprint constants, uniform across the wavefront:
            // the mirrored form, whose LDS reads are twice as many, takes
            // them from the angle table through the scalar cache; the others
            // from the chunk's LDS copy
            T c, K, C, CK;
            if constexpr (MIR) {
                const auto &A = cst(ang)[ch * CH + al];
                if constexpr (sizeof(T) == 4) {
                    c = A.cf;
                    K = A.Kf;
                    C = A.Cf;
                    CK = A.CKf;
                } else {
                    c = A.c;
                    K = A.K;
                    C = A.C;
                    CK = A.C - A.K;
                }
            } else {
                const T *pr = &prm[cb][gs][al * kBpPrm];
                c = pr[0];
                K = pr[1];
                C = pr[2];
                CK = pr[3];
            }
            const T u0 = fma(dx, c, rowt[cb][gs][al * kBpTile + ty]);
            const T u1 = u0 + c;
            const T *row = &win[gs][al][0][0];
            const int b0 = (int)u0, b1 = (int)u1;   // u > 0: truncation is floor
            const T f0 = frc(u0), f1 = frc(u1);
            const T w00 = sat(fma(f0, -K, C)), w01 = sat(fma(f0, K, CK));
            const T w10 = sat(fma(f1, -K, C)), w11 = sat(fma(f1, K, CK));
            if (NW == 2) {
                // both windows' bins are read before they are summed
                const T x00 = row[b0], x01 = row[b0 + 1], x10 = row[b1], x11 = row[b1 + 1];
                const T y00 = row[kBpWin + b0], y01 = row[kBpWin + b0 + 1];
                const T y10 = row[kBpWin + b1], y11 = row[kBpWin + b1 + 1];
                s0 = fma(w00, x00, s0);
                s0 = fma(w01, x01, s0);
                s1 = fma(w10, x10, s1);
                s1 = fma(w11, x11, s1);
                e0 = fma(w00, y00, e0);
                e0 = fma(w01, y01, e0);
                e1 = fma(w10, y10, e1);
                e1 = fma(w11, y11, e1);
            } else {
                s0 = fma(w00, row[b0], s0);
                s0 = fma(w01, row[b0 + 1], s0);
                s1 = fma(w10, row[b1], s1);
                s1 = fma(w11, row[b1 + 1], s1);
            }
        }
        acc0 += s0;
        acc1 += s1;
        if (NW == 2) {
            bcc0 += e0;
            bcc1 += e1;
        }
    }

    if (NS > 1) {
        // groups 1..NS-1 hand their sums to group 0 through the windows
        T *red = &win[0][0][0][0];
        __syncthreads();
        if (gs > 0) {
            T *d = red + ((gs - 1) * kBpThreads + t) * 2 * NW;
            d[0] = acc0;
            d[1] = acc1;
            if (NW == 2) {
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
                if (NW == 2) {
                    bcc0 += d[2];
                    bcc1 += d[3];
                }
            }
        }
    }

    // the pixel's row and column are formed again from an opaque copy of t:
    // held across the angle loop they would take a register it lacks
    int te = t;
    asm volatile("" : "+v"(te));
    const int i = i0 + (te >> 3), j = j0 + (te & 7) * 2;
    double dsum = 0.0;
    if (MIR && gs == 0 && i < G.n) {
        // column j is written when it lies in the left ceil(n/2) columns,
        // its mirror n-1-j when j lies in the left floor(n/2)
        auto *og = gl(out);
        auto *ogt = gl(outT);
        const auto *dg = gl(dotv);
        const T va[2] = {acc0, acc1}, vm[2] = {bcc0, bcc1};
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int jq = j + q, jm = G.n - 1 - jq;
            if (jq < jm + 1) {
                const size_t p = (size_t)i * G.n + jq;
                og[p] = va[q];
                if (outT != nullptr) ogt[(size_t)jq * G.n + i] = va[q];
                if (dot == 1) dsum += (double)va[q] * (double)dg[p];
                else if (dot == 2) dsum += (double)va[q] * (double)va[q];
            }
            if (jq < jm) {
                const size_t p = (size_t)i * G.n + jm;
                og[p] = vm[q];
                if (outT != nullptr) ogt[(size_t)jm * G.n + i] = vm[q];
                if (dot == 1) dsum += (double)vm[q] * (double)dg[p];
                else if (dot == 2) dsum += (double)vm[q] * (double)vm[q];
            }
        }
    }
    if (!MIR && gs == 0 && i < G.n) {
        const size_t p = (size_t)i * G.n + j;
        auto *og = gl(out);
        auto *og2 = gl(out2);
        auto *ogt = gl(outT);
        const auto *dg = gl(dotv);
        if (j < G.n) {
            og[p] = acc0;
            if (DUAL) og2[p] = bcc0;
            if (outT != nullptr) ogt[(size_t)j * G.n + i] = acc0;
            if (dot == 1) dsum += (double)(DUAL ? bcc0 : acc0) * (double)dg[p];
            else if (dot == 2) dsum += (double)acc0 * (double)acc0;
            else if (dot == 3) dsum += (double)acc0 * (double)bcc0;
        }
        if (j + 1 < G.n) {
            og[p + 1] = acc1;
            if (DUAL) og2[p + 1] = bcc1;
            if (outT != nullptr) ogt[(size_t)(j + 1) * G.n + i] = acc1;
            if (dot == 1) dsum += (double)(DUAL ? bcc1 : acc1) * (double)dg[p + 1];
            else if (dot == 2) dsum += (double)acc1 * (double)acc1;
            else if (dot == 3) dsum += (double)acc1 * (double)bcc1;
        }
    }
    if (partials == nullptr || dot == 0) return;
    double v[1] = {dsum};
    block_store(v, partials + vb.id());
}

template <typename T, int NS, bool MIR>
__global__ __launch_bounds__(kBpThreads * NS)
__attribute__((amdgpu_waves_per_eu(kBpWaves<T, false, MIR, NS>))) void k_backproject(
    const T *__restrict__ r, Geo G, const BpAngle *__restrict__ ang, const int *__restrict__ border,
    T *__restrict__ out, int swz)
{
    const int nt = (G.n + kBpTile - 1) / kBpTile;
    // the heaviest-first tile order covers the full grid only; the mirrored
    // form always takes the XCD-contiguous order (an XCD's tiles are a band
    // of rows, whose footprint of every projection its L2 then holds)
    const int tile = (MIR || swz || border == nullptr) ? launch_index(MIR ? 1 : swz)
                                                       : border[blockIdx.x];
    backproject_body<T, false, NS, MIR>(r, nullptr, G, ang, out, nullptr, nullptr, nullptr, 0,
                                        nullptr, vblk_of(tile, MIR ? bp_mirror_cols(G.n) : nt, nt));
}

template <typename T, bool MIR>
void launch_bp_split(const T *r, const Geo &G, const BpAngle *ang, const int *border, T *out,
                     int split, int swz, hipStream_t s)
{
    dim3 grid(blocks_bp(G, MIR));
    if constexpr (MIR) {
        if (split >= 8) {
            hipLaunchKernelGGL((k_backproject<T, 8, MIR>), grid, dim3(kBpThreads * 8), 0, s, r,
                               G, ang, border, out, swz);
            return;
        }
    }
    if (split >= 4)
        hipLaunchKernelGGL((k_backproject<T, 4, MIR>), grid, dim3(kBpThreads * 4), 0, s, r, G,
                           ang, border, out, swz);
    else if (split == 2)
        hipLaunchKernelGGL((k_backproject<T, 2, MIR>), grid, dim3(kBpThreads * 2), 0, s, r, G,
                           ang, border, out, swz);
    else
        hipLaunchKernelGGL((k_backproject<T, 1, MIR>), grid, dim3(kBpThreads), 0, s, r, G, ang,
                           border, out, swz);
}

template <typename T>
void launch_backproject(const T *r, const Geo &G, const BpAngle *ang, const int *border, T *out,
                        int split, int mirror, int swz, hipStream_t s)
{
    if (mirror) launch_bp_split<T, true>(r, G, ang, border, out, split, swz, s);
    else launch_bp_split<T, false>(r, G, ang, border, out, split, swz, s);
}

template <typename T, bool DUAL, int NS, bool MIR>
__global__ __launch_bounds__(kBpThreads * NS)
__attribute__((amdgpu_waves_per_eu(kBpWaves<T, DUAL, MIR, NS>))) void kb_backproject(
    const Solve<T> *S, const BlkMap *map, int phase, int dot, int swz)
{
    // a single solve's mirrored launch takes the XCD-contiguous order always;
    // a batch's keeps the chosen one (contiguous ranges of a mixed batch give
    // XCDs unequal shares of its heavier solves)
    const BlkMap m = locate(map, MIR && map == nullptr ? 1 : swz);
    const Solve<T> d = load_solve(S, m.solve);
    if (stopped(d.st)) return;
    // descriptor fields into registers: the body's stores cannot alias them
    const Geo G = d.G;
    const BpAngle *ang = d.bang;
    const int nt = (G.n + kBpTile - 1) / kBpTile;
    // the tile of this launch position (partials are stored by tile, so the
    // sums do not depend on the order)
    const int tile = (MIR || swz || d.border == nullptr) ? m.local : gl(d.border)[m.local];
    const VBlk vb = vblk_of(tile, MIR ? bp_mirror_cols(G.n) : nt, nt);
    // one body instance: kBpH is h = A^T q (no second sinogram, no dot);
    // kBpG, kBpGZ are g' = A^T r (and z' = A^T rt) with the dot against h or g';
    // kBpGT is g' with its transpose in xs; kBpZ is z = A^T rt with the dot
    // against g
    const bool hq = phase == kBpH, zq = phase == kBpZ;
    const T *src = hq ? d.q : (zq ? d.rt : d.r);
    T *dst = hq ? d.h : (zq ? d.z : d.g);
    T *dstT = phase == kBpGT ? d.xs : nullptr;
    const T *dv = zq ? d.g : d.h;
    backproject_body<T, DUAL, NS, MIR>(src, d.rt, G, ang, dst, d.z, dstT, dv, hq ? 0 : dot,
                                       hq ? nullptr : d.partials, vb);
}

template <typename T, bool DUAL, bool MIR>
void launch_b_bp_split(const Solve<T> *S, const BlkMap *map, int nblocks, int phase, int dot,
                       int split, int swz, hipStream_t s)
{
    if constexpr (MIR) {
        if (split >= 8) {
            hipLaunchKernelGGL((kb_backproject<T, DUAL, 8, MIR>), dim3(nblocks),
                               dim3(kBpThreads * 8), 0, s, S, map, phase, dot, swz);
            return;
        }
    }
    if (split >= 4)
        hipLaunchKernelGGL((kb_backproject<T, DUAL, 4, MIR>), dim3(nblocks),
                           dim3(kBpThreads * 4), 0, s, S, map, phase, dot, swz);
    else if (split == 2)
        hipLaunchKernelGGL((kb_backproject<T, DUAL, 2, MIR>), dim3(nblocks),
                           dim3(kBpThreads * 2), 0, s, S, map, phase, dot, swz);
    else
        hipLaunchKernelGGL((kb_backproject<T, DUAL, 1, MIR>), dim3(nblocks), dim3(kBpThreads),
                           0, s, S, map, phase, dot, swz);
}

template <typename T>
void launch_b_backproject(const Solve<T> *S, const BlkMap *map, int nblocks, int phase, int dot,
                          int split, int mirror, int swz, hipStream_t s)
{
    // the two-sinogram phase (filtered variants) never runs mirrored: a
    // solve of such a variant is set up with the full tile grid
    if (phase == kBpGZ)
        launch_b_bp_split<T, true, false>(S, map, nblocks, phase, dot, split, swz, s);
    else if (mirror)
        launch_b_bp_split<T, false, true>(S, map, nblocks, phase, dot, split, swz, s);
    else
        launch_b_bp_split<T, false, false>(S, map, nblocks, phase, dot, split, swz, s);
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

// TV(x) block partials and optionally the subgradient (grid-stride over the
// image with the body's block count).
template <typename T>
__device__ void tv_body(const T *__restrict__ x_, T *__restrict__ s_out_, const Geo &G, T k2,
                        double *partials, VBlk vb)
{
    const auto *x = gl(x_);
    auto *s_out = gl(s_out_);
    const int n = G.n;
    double tv = 0.0;
    const size_t J = (size_t)n * n;
    for (size_t p = vb.id() * (size_t)blockDim.x + threadIdx.x; p < J;
         p += (size_t)vb.count() * blockDim.x) {
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
    double v[1] = {tv};
    block_store(v, partials + vb.id());
}

template <typename T>
__global__ __launch_bounds__(256) void k_tv(const T *__restrict__ x, T *__restrict__ s_out, Geo G,
                                             double kappa, double *partials)
{
    tv_body(x, s_out, G, (T)(kappa * kappa), partials, grid_vblk());
}

__global__ __launch_bounds__(256) void k_sum_to(const double *partials, int nblk, double *dst)
{
    __shared__ double tot[1];
    final_sums(partials, nblk, 1, 1, tot);
    if (threadIdx.x == 0) *dst = tot[0];
}

template <typename T>
void launch_tv(const T *x, T *s_out, const Geo &G, double kappa, double *partials,
               double *tv_dst, hipStream_t s)
{
    const int nb = vec_blocks((size_t)G.n * G.n);
    hipLaunchKernelGGL(k_tv<T>, dim3(nb), dim3(kBlock), 0, s, x, s_out, G, kappa, partials);
    hipLaunchKernelGGL(k_sum_to, dim3(1), dim3(kBlock), 0, s, partials, nb, tv_dst);
}

// TV of every solve's output image (after the loop; runs whether or not the
// solve stopped).
template <typename T>
__global__ __launch_bounds__(256) void kb_tv(const Solve<T> *S, const BlkMap *map)
{
    const BlkMap m = locate(map);
    const Solve<T> d = load_solve(S, m.solve);
    const T k2 = (T)(gl(d.st)->kappa * gl(d.st)->kappa);
    tv_body<T>(d.xout, nullptr, d.G, k2, d.partials, vblk_of(m.local, d.nb_vec, 1));
}

template <typename T>
void launch_b_tv(const Solve<T> *S, const BlkMap *map, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(kb_tv<T>, dim3(nblocks), dim3(kBlock), 0, s, S, map);
}

// ---------------------------------------------------------------------------
// Step boundary of the superiorized solvers, fused with the TV work that opens
// the next step: x_{k+1} = x_{k+1/2} + alpha p' (the last line of the previous
// step) on a 32 x 16 tile plus a one-pixel halo held in LDS, then the TV
// subgradient s at x_{k+1}; the block stores its parts of TV(x_{k+1}) and
// ||s||^2. The step is closed and the next opened by a finisher: kFinXtv in a
// batch, the first trial launch's kFinOpenTrials in a single solve.
// ---------------------------------------------------------------------------

template <typename T, typename F>
__device__ void xtv_body(const T *__restrict__ xh_, const T *__restrict__ p_, T *__restrict__ x_,
                         T *__restrict__ s_out_, const Geo &G, double *partials,
                         const DevState *st_, F alpha_of, VBlk vb)
{
    const auto *xh = gl(xh_);
    const auto *p = gl(p_);
    auto *x = gl(x_);
    auto *s_out = gl(s_out_);
    const auto *st = gl(st_);
    constexpr int TW = 32, TH = kXtvRows;
    __shared__ T tile[TH + 2][TW + 2];
    const int n = G.n;
    const int i0 = vb.y * TH, j0 = vb.x * TW;
    const T k2 = (T)(st->kappa * st->kappa);
    // S-CG-K, S-PCG-K: x_{k+1} is the pass's output, already in x
    const bool given = st->variant == SCG_S_CG_K || st->variant == SCG_S_PCG_K;
    // the tile and its halo, (TH + 2) x (TW + 2) values over the block's
    // kBlock threads: every load is issued before alpha is formed (its block
    // sums overlap the loads) and before the first is used
    constexpr int NE = (TH + 2) * (TW + 2), NI = (NE + kBlock - 1) / kBlock;
    T hv[NI], pv[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int e = threadIdx.x + kBlock * k;
        const int ii = i0 - 1 + e / (TW + 2), jj = j0 - 1 + e % (TW + 2);
        hv[k] = pv[k] = T(0);
        if (e < NE && ii >= 0 && ii < n && jj >= 0 && jj < n) {
            const size_t q = (size_t)ii * n + jj;
            if (given) {
                hv[k] = x[q];
            } else {
                hv[k] = xh[q];
                pv[k] = p[q];
            }
        }
    }
    const T al = (T)alpha_of();
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int e = threadIdx.x + kBlock * k;
        if (e < NE) tile[e / (TW + 2)][e % (TW + 2)] = given ? hv[k] : fma(al, pv[k], hv[k]);
    }
    __syncthreads();
    // each thread forms the pixels of rows ty, ty + kBlock / TW, ...
    constexpr int RS = kBlock / TW;
    const int tx = threadIdx.x % TW;
    double tv = 0.0, ss = 0.0;
#pragma unroll
    for (int ty = threadIdx.x / TW; ty < TH; ty += RS) {
        const int i = i0 + ty, j = j0 + tx;
        if (i < n && j < n) {
            T X[3][3];
#pragma unroll
            for (int di = 0; di < 3; ++di)
#pragma unroll
                for (int dj = 0; dj < 3; ++dj) X[di][dj] = tile[ty + di][tx + dj];
            T own;
            const T sg = tv_pixel(X, i, j, n, k2, own);
            const size_t q = (size_t)i * n + j;
            if (!given) x[q] = X[1][1];
            s_out[q] = sg;
            tv += (double)own;
            ss += (double)sg * (double)sg;
        }
    }
    double v[2] = {tv, ss};
    block_store(v, partials + 2 * (size_t)vb.id());
}

template <typename T>
__global__ __launch_bounds__(256) void kb_xtv(const Solve<T> *S, const BlkMap *map, int given)
{
    const BlkMap m = locate(map);
    const Solve<T> d = load_solve(S, m.solve);
    if (stopped(d.st)) return;
    const auto *st = gl(d.st);
    // alpha of the open step: from the direction update's and the
    // projection's partials (recorded by this pass's finisher) or from the
    // state (given: a finisher formed it there with the same sums)
    const bool local = !given && local_alpha(st->variant) && st->open;
    double gp = 0.0, qq = 0.0;
    auto alpha_of = [&]() -> double {
        if (!local) return st->alpha;
        block_sum2(d.partials3, d.nb_t32, d.partials, d.nb_pj, gp, qq);
        return -gp / qq;
    };
    xtv_body(d.xh, d.p, d.x, d.s, d.G, d.partials2, d.st, alpha_of,
             vblk_of(m.local, (d.G.n + 31) / 32, (d.G.n + kXtvRows - 1) / kXtvRows));
    // a single solve has no finisher between this pass and the first trial
    // launch: the solve's first block records ||A p||^2 and g^T p of the step
    // being closed for the finisher after that launch (no block reads them
    // here)
    if (local && m.local == 0 && threadIdx.x == 0) {
        auto *stw = gl(d.st);
        stw->qq = qq;
        stw->gp = gp;
    }
}

template <typename T>
void launch_b_xtv(const Solve<T> *S, const BlkMap *map, int nblocks, int given, hipStream_t s)
{
    hipLaunchKernelGGL(kb_xtv<T>, dim3(nblocks), dim3(256), 0, s, S, map, given);
}

// ---------------------------------------------------------------------------
// perturbed(): the trials of one step, TV(x + gamma_m v) for gamma_m =
// gtab[m] (gamma0 a^(l+m)) and v = -s/||s||, in up to two launches, each
// followed by a finisher. The first evaluates trials 0..kTrialsPerPass-1
// together with TV(x), summed in the same order; the second, which returns
// at once when the first accepted (and which a single solve enqueues only
// where a search needs it), evaluates the remaining ones up to max_trials in
// chunks of kTrialsPerPass. The finisher takes the first m with
// TV(x + gamma_m v) <= TV(x), exactly as trying the values one after
// another; l advances by the trials used. Partials per block: [TV(x), trial
// first_m, first_m + 1, ...].
// ---------------------------------------------------------------------------

static_assert((unsigned long long)kMaxN * kMaxN + (unsigned long long)kMaxPartials * kBlock <
                  (1ull << 32),
              "32-bit trial term indices");

// Scalars of a trial launch: go = false ends the block at once; inv =
// 1 / ||s||; gam(idx) = gamma_{l+idx}.
struct TrialScalars {
    bool go;
    double inv;
};

template <typename T, typename F, typename Gam>
__device__ void trials_body(const T *__restrict__ x_, const T *__restrict__ s_, const Geo &G,
                            double *partials, const DevState *st_, int first_m, int nchunks,
                            F scalars, Gam gam_at, VBlk vb)
{
    const auto *x = gl(x_);
    const auto *s = gl(s_);
    const auto *st = gl(st_);
    constexpr int M = kTrialsPerPass;
    const int max_trials = st->max_trials;
    const int stride = 1 + M * nchunks;
    const T k2 = (T)(st->kappa * st->kappa);
    // 32-bit indices: (n - 1)^2 plus one grid stride stays below 2^32 for
    // every accepted image side
    const unsigned n = (unsigned)G.n, m1 = n - 1u;
    const unsigned terms = m1 * m1;
    const unsigned bid = (unsigned)vb.id(), nblk = (unsigned)vb.count();
    const bool with_tvx = first_m == 0;
    // the thread's first term is loaded before the scalars are formed (their
    // block sums overlap the loads)
    const unsigned q0 = bid * blockDim.x + threadIdx.x;
    T f0[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
    if (q0 < terms) {
        const unsigned i = q0 / m1, j = q0 - i * m1;
        const unsigned cq = i * n + j;
        f0[0] = x[cq];
        f0[1] = x[cq + n];
        f0[2] = x[cq + 1];
        f0[3] = s[cq];
        f0[4] = s[cq + n];
        f0[5] = s[cq + 1];
    }
    const TrialScalars sc = scalars();
    if (!sc.go) return;
    const T inv = (T)sc.inv;
    for (int c = 0; c < nchunks; ++c) {
        const int m0 = first_m + M * c;
        T gam[M];
#pragma unroll
        for (int m = 0; m < M; ++m) gam[m] = (T)gam_at(min(m0 + m, max_trials - 1));
        T acc[M + 1];
#pragma unroll
        for (int m = 0; m <= M; ++m) acc[m] = T(0);
        for (unsigned q = q0; q < terms; q += nblk * blockDim.x) {
            T xc, xd, xr, sc_, sd, sr;
            if (c == 0 && q == q0) {
                xc = f0[0];
                xd = f0[1];
                xr = f0[2];
                sc_ = f0[3];
                sd = f0[4];
                sr = f0[5];
            } else {
                const unsigned i = q / m1, j = q - i * m1;
                const unsigned cq = i * n + j;
                xc = x[cq];
                xd = x[cq + n];
                xr = x[cq + 1];
                sc_ = s[cq];
                sd = s[cq + n];
                sr = s[cq + 1];
            }
            const T vc = -sc_ * inv, vd = -sd * inv, vr = -sr * inv;
            if (with_tvx && c == 0) acc[M] += tv_term(xd - xc, xr - xc, k2);
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const T g = gam[m];
                const T zc = fma(g, vc, xc), zd = fma(g, vd, xd), zr = fma(g, vr, xr);
                acc[m] += tv_term(zd - zc, zr - zc, k2);
            }
        }
        // [TV(x) (first chunk only), the chunk's trials] at dst + M c
        double *dst = partials + (size_t)bid * stride + M * c;
        T vals[M + 1];
        vals[0] = acc[M];
#pragma unroll
        for (int m = 0; m < M; ++m) vals[1 + m] = acc[m];
        block_store_rows(vals, dst, c == 0 ? 0 : 1);
    }
}

// open = 1 (the first trial launch of a single solve, no finisher between
// it and the TV pass): the launch forms what the step-opening finisher will
// record, with the same formulas and the same sums: whether the step runs a
// search (iteration cap, forced decisions, no perturbation, ||s|| > 0) and
// 1 / ||s|| from the TV pass's partials. Otherwise those come from the state
// the finisher left. Either way gamma_{l+m} comes from the table.
template <typename T>
__global__ __launch_bounds__(256) void kb_trials(const Solve<T> *S, const BlkMap *map,
                                                  int first_m, int open)
{
    const BlkMap m = locate(map);
    const Solve<T> d = load_solve(S, m.solve);
    const auto *st = gl(d.st);
    if (st->done) return;
    const int nchunks = first_m == 0 ? 1 : d.trB_chunks;
    if (nchunks <= 0) return;
    const int nblk = first_m == 0 ? d.nb_trA : d.nb_trB;
    const VBlk vb = vblk_of(m.local, nblk, 1);
    if (!open) {
        if (st->search_done) return;
        const auto *gtab = gl(d.gtab);
        trials_body(d.x, d.s, d.G, d.partials, d.st, first_m, nchunks,
                    [&] { return TrialScalars{true, st->inv_snorm}; },
                    [&](int i) { return gtab[i]; }, vb);
        return;
    }
    // the step the following finisher opens (see its kFinOpenTrials case)
    const int step_open = st->open ? 1 : 0;
    if (st->steps + step_open >= st->max_iter) return;
    if (st->flags & SCG_FLAG_NO_PERTURB) return;
    const int k = st->k + step_open + st->kofs;
    if (d.forced != nullptr && k >= 1 && k - 1 < st->forced_len) return;
    auto scalars = [&]() -> TrialScalars {
        double tv, s2;
        block_sum2(d.partials2, d.nb_xtv, d.partials2 + 1, d.nb_xtv, tv, s2, 2, 2);
        const bool dir = s2 > 0.0 && isfinite(s2);
        return TrialScalars{dir, dir ? 1.0 / sqrt(s2) : 0.0};
    };
    // gamma_{l+m}, m < kTrialsPerPass, for the l this step opens with: left
    // in the table by the previous step's perturbation or the initial step
    const auto *gtab = gl(d.gtab);
    trials_body(d.x, d.s, d.G, d.partials, d.st, 0, 1, scalars,
                [&](int i) { return gtab[i]; }, vb);
}

template <typename T>
void launch_b_trials(const Solve<T> *S, const BlkMap *map, int nblocks, int first_m, int open,
                     hipStream_t s)
{
    hipLaunchKernelGGL(kb_trials<T>, dim3(nblocks), dim3(kBlock), 0, s, S, map, first_m, open);
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
__device__ void perturb_body(T *__restrict__ x_, const T *__restrict__ s_,
                             T *__restrict__ xh_, T *__restrict__ xht_, const Geo &G,
                             const DevState *st_, VBlk vb)
{
    auto *x = gl(x_);
    const auto *s = gl(s_);
    auto *xh = gl(xh_);
    auto *xht = gl(xht_);
    const auto *st = gl(st_);
    __shared__ T tile[32][33];
    const bool move = st->accepted >= 0 && st->gamma != 0.0;
    // CG-K and PCG-K start from x_{k+1/2}
    const bool restart = st->variant == SCG_S_CG_K || st->variant == SCG_S_PCG_K;
    const T g = (T)st->gamma, inv = (T)st->inv_snorm;
    const int n = G.n;
    const int bx = vb.x * 32, by = vb.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    // every row's loads are issued before the first store
    constexpr int R = 4;   // rows per thread
    T xv[R], sv[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int i = by + ty + 8 * k, j = bx + tx;
        xv[k] = sv[k] = T(0);
        if (i < n && j < n) {
            const size_t q = (size_t)i * n + j;
            xv[k] = x[q];
            if (move) sv[k] = s[q];
        }
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int r = ty + 8 * k;
        const int i = by + r, j = bx + tx;
        T v = T(0);
        if (i < n && j < n) {
            const size_t q = (size_t)i * n + j;
            v = move ? fma(g, -sv[k] * inv, xv[k]) : xv[k];
            xh[q] = v;
            if (restart) x[q] = v;
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
__global__ __launch_bounds__(256) void kb_perturb(const Solve<T> *S, const BlkMap *map)
{
    const BlkMap m = locate(map);
    const Solve<T> d = load_solve(S, m.solve);
    if (stopped(d.st)) return;
    const int nt = (d.G.n + 31) / 32;
    // the next step's first trial launch reads its gammas from the table: the
    // solve's first block writes them for the l this step's search ended with
    if (m.local == 0) fill_first_gammas(d.gtab, gl(d.st));
    perturb_body(d.x, d.s, d.xh, d.xs, d.G, d.st, vblk_of(m.local, nt, nt));
}

template <typename T>
void launch_b_perturb(const Solve<T> *S, const BlkMap *map, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(kb_perturb<T>, dim3(nblocks), dim3(256), 0, s, S, map);
}

template <typename S> __device__ __forceinline__ double beta_of(S *st, int rule, int init)
{
    if (init) return 0.0;
    if (rule == 0 || rule == 2) return st->gh / st->qq_prev;
    if (rule == 1) return -st->gg / st->gp_prev;
    // CG-STEP inside a CG-K pass: a zero gradient (an exact minimiser) ends
    // the pass's progress instead of a 0/0
    if ((st->variant == SCG_S_CG_K || st->variant == SCG_S_PCG_K) && st->delta == 0.0) return 0.0;
    return st->gg / st->delta;   // rule 3 (CG-STEP), rule 4 (PCG-STEP: gg holds g^T z)
}

// Scalars of a direction update, formed by the caller's callable once the
// update's loads are in flight: go = false leaves the vectors untouched.
struct StepScalars {
    bool go;
    double beta;
};

template <typename T, typename F>
__device__ void p_update_body(const T *__restrict__ g_, const T *__restrict__ z_,
                              T *__restrict__ p_, T *__restrict__ pt_, const Geo &G,
                              double *partials, int rule, int init, F scalars, VBlk vb)
{
    const auto *g = gl(g_);
    const auto *z = gl(z_);
    auto *p = gl(p_);
    auto *pt = gl(pt_);
    __shared__ T tile[32][33];
    const auto *src = (rule == 2 || rule == 4) ? z : g;   // PCG rules step along -z
    const int n = G.n;
    const int bx = vb.x * 32, by = vb.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    // every row's loads are issued before the scalars are formed (their
    // block sums overlap the loads) and before the first store (eight or
    // twelve loads in flight per thread); then the rows are formed in order
    constexpr int R = 4;   // rows per thread
    const bool sep = src != g;
    T sv[R], pv[R], gv[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int i = by + ty + 8 * k, j = bx + tx;
        sv[k] = pv[k] = gv[k] = T(0);
        if (i < n && j < n) {
            const size_t q = (size_t)i * n + j;
            sv[k] = src[q];
            if (!init) pv[k] = p[q];
            if (sep) gv[k] = g[q];
        }
    }
    const StepScalars sc = scalars();
    if (!sc.go) return;
    const T bt = (T)sc.beta;
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int r = ty + 8 * k;
        const int i = by + r, j = bx + tx;
        T pn = T(0);
        if (i < n && j < n) {
            const size_t q = (size_t)i * n + j;
            pn = init ? -sv[k] : fma(bt, pv[k], -sv[k]);
            p[q] = pn;
            acc += (double)(sep ? gv[k] : sv[k]) * (double)pn;
        }
        tile[r][tx] = pn;
    }
    if (pt_ != nullptr) {   // uniform: the transposed copy for A p
        __syncthreads();
        for (int r = ty; r < 32; r += 8) {
            const int j = bx + r, i = by + tx;
            if (i < n && j < n) pt[(size_t)j * n + i] = tile[tx][r];
        }
    }
    double v[1] = {acc};
    block_store(v, partials + vb.id());
}

template <typename T>
__global__ __launch_bounds__(256) void kb_p_update(const Solve<T> *S, const BlkMap *map,
                                                    int rule, int init, int rec, int given)
{
    const BlkMap m = locate(map);
    const Solve<T> d = load_solve(S, m.solve);
    if (stopped(d.st)) return;
    const int nt = (d.G.n + 31) / 32;
    auto *st = gl(d.st);
    const VBlk vb = vblk_of(m.local, nt, nt);
    if (given) {
        // a finisher (kFinStepScalars) took the stop test and left beta in
        // the state: the same sums, so the same bits
        p_update_body(d.g, d.z, d.p, d.pt, d.G, d.partials3, rule, init,
                      [&] { return StepScalars{true, st->beta}; }, vb);
        return;
    }
    // formed while the update's loads are in flight
    auto scalars = [&]() -> StepScalars {
        // beta of rules 0-2 from the backprojection's dot partials, of the
        // others from the state
        const bool need_dot = !init && rule <= 2;
        double f = 0.0, dot = 0.0;
        if (rec && need_dot) {
            block_sum2(d.partials2, d.nb_pj, d.partials, d.nb_bp, f, dot);
        } else if (rec) {
            f = block_sum1(d.partials2, d.nb_pj);
        } else if (need_dot) {
            dot = block_sum1(d.partials, d.nb_bp);
        }
        if (rec) {
            // The step's loop test, f(x_{k+1/2}) <= eps, with f from the
            // residual projection's partials (kPjResXhF): every block forms
            // the same f; the solve's first block records it and, when the
            // test holds (or f is not finite), ends the solve at k + 1 with
            // output x_{k+1/2}: the rest of the step cannot change the
            // output and is skipped.
            f *= 0.5;
            const bool stop = !isfinite(f) || f <= st->eps;
            if (m.local == 0 && threadIdx.x == 0) {
                st->f_half = f;
                if (auto *tr = trace_at(st, d.trace)) tr->f_half = f;
                if (!isfinite(f)) {
                    set_done(st, SCG_ENAN);
                } else if (stop) {
                    st->steps += 1;
                    st->k += 1;
                    set_done(st, SCG_OK);
                }
            }
            if (stop) return StepScalars{false, 0.0};
        }
        double beta = beta_of(st, rule, init);
        if (need_dot) {
            beta = rule == 1 ? -dot / st->gp_prev : dot / st->qq_prev;
            // rec: no finisher follows; the solve's first block records the
            // dot and beta (fields the other blocks do not read), and g'^T p'
            // is recorded by the finisher of the TV pass that forms alpha
            // from it
            if (rec && m.local == 0 && threadIdx.x == 0) {
                if (rule == 1) st->gg = dot;
                else st->gh = dot;
                st->beta = beta;
                if (!isfinite(beta)) set_done(st, SCG_ENAN);
                if (auto *tr = trace_at(st, d.trace)) tr->beta = beta;
            }
        }
        return StepScalars{true, beta};
    };
    p_update_body(d.g, d.z, d.p, d.pt, d.G, d.partials3, rule, init, scalars, vb);
}

template <typename T>
void launch_b_p_update(const Solve<T> *S, const BlkMap *map, int nblocks, int rule, int init,
                       int rec, int given, hipStream_t s)
{
    hipLaunchKernelGGL(kb_p_update<T>, dim3(nblocks), dim3(256), 0, s, S, map, rule, init, rec,
                       given);
}

// S-CG with three operators: q' = -u + beta q over sinogram row a (u = A g'
// in rt), and the block's partial of ||q'||^2.
template <typename T>
__device__ void q_update_body(const T *__restrict__ u_, T *__restrict__ q_, const Geo &G,
                              const DevState *st_, double *partial, int a)
{
    const auto *u = gl(u_);
    auto *q = gl(q_);
    const T bt = (T)beta_of(gl(st_), 0, 0);
    const size_t row = (size_t)a * G.rs + kSinoPadL;
    double acc = 0.0;
    for (int b = threadIdx.x; b < G.nb; b += blockDim.x) {
        const T qn = fma(bt, q[row + b], -u[row + b]);
        q[row + b] = qn;
        acc += (double)qn * (double)qn;
    }
    double v[1] = {acc};
    block_store(v, partial);
}

// Blocks [0, nb_t32): p' = -g' + beta p (no transposed copy: p' is not
// projected); blocks [nb_t32, nb_t32 + nb_sv): q'. The partials land at the
// block's own index.
template <typename T>
__global__ __launch_bounds__(256) void kb_pq_update(const Solve<T> *S, const BlkMap *map)
{
    const BlkMap m = locate(map);
    const Solve<T> d = load_solve(S, m.solve);
    if (stopped(d.st)) return;
    if (m.local < d.nb_t32) {
        const int nt = (d.G.n + 31) / 32;
        p_update_body(d.g, d.z, d.p, (T *)nullptr, d.G, d.partials, 0, 0,
                      [&] { return StepScalars{true, beta_of(gl(d.st), 0, 0)}; },
                      vblk_of(m.local, nt, nt));
    } else {
        q_update_body(d.rt, d.q, d.G, d.st, d.partials + m.local, m.local - d.nb_t32);
    }
}

template <typename T>
void launch_b_pq_update(const Solve<T> *S, const BlkMap *map, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(kb_pq_update<T>, dim3(nblocks), dim3(256), 0, s, S, map);
}

// Batch admission (see Admit): block row y serves record y.
template <typename T> __global__ __launch_bounds__(256) void kb_admit(const Admit<T> *recs)
{
    const Admit<T> a = gl(recs)[blockIdx.y];
    if (blockIdx.x == 0) {
        constexpr int kSt = sizeof(DevState) / 4, kDs = sizeof(Solve<T>) / 4;
        static_assert(sizeof(DevState) % 4 == 0 && sizeof(Solve<T>) % 4 == 0, "word copies");
        const auto *ss = gl(reinterpret_cast<const unsigned *>(a.st_src));
        auto *sd = gl(reinterpret_cast<unsigned *>(a.st));
        const auto *ds = gl(reinterpret_cast<const unsigned *>(a.desc_src));
        auto *dd = gl(reinterpret_cast<unsigned *>(a.desc));
        for (int i = threadIdx.x; i < kSt; i += blockDim.x) sd[i] = ss[i];
        for (int i = threadIdx.x; i < kDs; i += blockDim.x) dd[i] = ds[i];
    }
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long t0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    auto *xs = gl(a.xs), *xst = gl(a.x_start), *xh = gl(a.xh);
    const auto *x0 = gl(a.x0);
    for (long long i = t0; i < a.J; i += stride) {
        const T v = a.x0 != nullptr ? x0[i] : T(0);
        xst[i] = v;
        if (a.xh != nullptr) xh[i] = v;
        xs[i] = T(0);
    }
    auto *r = gl(a.r), *q = gl(a.q), *rt = gl(a.rt);
    for (long long i = t0; i < a.S; i += stride) {
        r[i] = T(0);
        q[i] = T(0);
        rt[i] = T(0);
    }
}

template <typename T> void launch_admit(const Admit<T> *recs, int n, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(kb_admit<T>, dim3(64, n), dim3(256), 0, s, recs);
}

// PCG-STEP: blocks [0, nb_vec) update x' = x + alpha p and g' = g + alpha h;
// blocks [nb_vec, nb_vec + nb_sv) update sinogram row a of the recursive
// residual, r' = r + alpha q (the filtered residual gives the next z).
template <typename T>
__global__ __launch_bounds__(256) void kb_x_update_pcg(const Solve<T> *S, const BlkMap *map)
{
    const BlkMap m = locate(map);
    const Solve<T> d = load_solve(S, m.solve);
    if (stopped(d.st)) return;
    const T al = (T)gl(d.st)->alpha;
    if (m.local < d.nb_vec) {
        const size_t J = (size_t)d.G.n * d.G.n;
        auto *x = gl(d.x), *g = gl(d.g);
        const auto *p = gl(d.p), *h = gl(d.h);
        for (size_t q = m.local * (size_t)blockDim.x + threadIdx.x; q < J;
             q += (size_t)d.nb_vec * blockDim.x) {
            x[q] = fma(al, p[q], x[q]);
            g[q] = fma(al, h[q], g[q]);
        }
    } else {
        const size_t row = (size_t)(m.local - d.nb_vec) * d.G.rs + kSinoPadL;
        auto *r = gl(d.r);
        const auto *q = gl(d.q);
        for (int b = threadIdx.x; b < d.G.nb; b += blockDim.x)
            r[row + b] = fma(al, q[row + b], r[row + b]);
    }
}

template <typename T>
void launch_b_x_update_pcg(const Solve<T> *S, const BlkMap *map, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(kb_x_update_pcg<T>, dim3(nblocks), dim3(kBlock), 0, s, S, map);
}

// Plain CG (Alg. CG, CG-STEP): x' = x + alpha p and the recursive gradient
// g' = g + alpha h with the partials of ||g'||^2.
template <typename T>
__global__ __launch_bounds__(256) void kb_x_update_cg(const Solve<T> *S, const BlkMap *map)
{
    const BlkMap m = locate(map);
    const Solve<T> d = load_solve(S, m.solve);
    if (stopped(d.st)) return;
    const T al = (T)gl(d.st)->alpha;
    const size_t J = (size_t)d.G.n * d.G.n;
    auto *x = gl(d.x), *g = gl(d.g);
    const auto *p = gl(d.p), *h = gl(d.h);
    double acc = 0.0;
    for (size_t q = m.local * (size_t)blockDim.x + threadIdx.x; q < J;
         q += (size_t)d.nb_vec * blockDim.x) {
        x[q] = fma(al, p[q], x[q]);
        const T gn = fma(al, h[q], g[q]);
        g[q] = gn;
        acc += (double)gn * (double)gn;
    }
    double v[1] = {acc};
    block_store(v, d.partials + m.local);
}

template <typename T>
void launch_b_x_update_cg(const Solve<T> *S, const BlkMap *map, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(kb_x_update_cg<T>, dim3(nblocks), dim3(kBlock), 0, s, S, map);
}

// ---------------------------------------------------------------------------
// Preconditioning filter F^T C F per projection: zero padding to P =
// 2^ceil(log2(2 n_bins)) samples, DFT, multiplication by c(w_m), inverse DFT,
// the first n_bins samples kept. One block per pair of projections: the two
// real rows are the real and imaginary parts of one complex sequence (c is
// real and even, so the product's inverse keeps them apart). The transform
// runs in LDS: radix-2 decimation in frequency (natural order in, bit-
// reversed order out), the spectrum multiplied in that order (the table is
// stored bit-reversed, with 1/P folded in), then radix-2 decimation in time
// from bit-reversed order back to natural order with conjugate twiddles, so
// no reordering pass is needed. Table layout: P spectrum values, then the
// twiddles of each butterfly span h = 1, 2, 4, ..., P/2 in turn,
// e^{-2 pi i j / (2h)} for j < h as (re, im) pairs from offset h - 1: the
// lanes of a stage read consecutive entries.
// ---------------------------------------------------------------------------

template <typename T> struct Cx {
    T x, y;
};

__device__ __forceinline__ int filter_len(int nb)
{
    return 1 << (32 - __clz(2 * nb - 1));   // smallest power of two >= 2 nb
}

template <typename T>
__device__ void filter_body(const T *__restrict__ r_, T *__restrict__ out_,
                            const T *__restrict__ tab_, const Geo &G, int out_padded, int pair)
{
    const auto *r = gl(r_);
    auto *out = gl(out_);
    const auto *spec = gl(tab_);
    const int nb = G.nb, P = filter_len(nb), half = P >> 1;
    // span h's twiddles at tw[h + j], j < h
    const auto *tw = gl(reinterpret_cast<const Cx<T> *>(tab_ + P) - 1);
    extern __shared__ unsigned char smem[];
    Cx<T> *z = reinterpret_cast<Cx<T> *>(smem);
    const int a0 = 2 * pair, a1 = a0 + 1;
    const bool two = a1 < G.na;
    const size_t in_stride = G.rs;
    const auto *r0 = r + (size_t)a0 * in_stride + kSinoPadL;
    const auto *r1 = r + (size_t)(two ? a1 : a0) * in_stride + kSinoPadL;
    for (int b = threadIdx.x; b < P; b += blockDim.x) {
        Cx<T> v{T(0), T(0)};
        if (b < nb) {
            v.x = r0[b];
            v.y = two ? r1[b] : T(0);
        }
        z[b] = v;
    }
    __syncthreads();
    // forward transform: butterflies of span h, twiddle e^{-2 pi i j / (2h)}
    for (int h = half; h >= 1; h >>= 1) {
        for (int k = threadIdx.x; k < half; k += blockDim.x) {
            const int j = k & (h - 1);
            const int i = ((k - j) << 1) + j;
            const Cx<T> u = z[i], v = z[i + h];
            const Cx<T> w = tw[h + j];
            const T dx = u.x - v.x, dy = u.y - v.y;
            z[i] = Cx<T>{u.x + v.x, u.y + v.y};
            z[i + h] = Cx<T>{dx * w.x - dy * w.y, dx * w.y + dy * w.x};
        }
        __syncthreads();
    }
    for (int b = threadIdx.x; b < P; b += blockDim.x) {
        const T c = spec[b];
        z[b] = Cx<T>{z[b].x * c, z[b].y * c};
    }
    __syncthreads();
    // inverse transform: span h, twiddle e^{+2 pi i j / (2h)}
    for (int h = 1; h < P; h <<= 1) {
        for (int k = threadIdx.x; k < half; k += blockDim.x) {
            const int j = k & (h - 1);
            const int i = ((k - j) << 1) + j;
            const Cx<T> u = z[i], v = z[i + h];
            const Cx<T> w = tw[h + j];
            const Cx<T> t{v.x * w.x + v.y * w.y, v.y * w.x - v.x * w.y};
            z[i] = Cx<T>{u.x + t.x, u.y + t.y};
            z[i + h] = Cx<T>{u.x - t.x, u.y - t.y};
        }
        __syncthreads();
    }
    const size_t out_stride = out_padded ? G.rs : nb;
    const int ofs = out_padded ? kSinoPadL : 0;
    auto *o0 = out + (size_t)a0 * out_stride + ofs;
    auto *o1 = out + (size_t)a1 * out_stride + ofs;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        const Cx<T> v = z[b];
        o0[b] = v.x;
        if (two) o1[b] = v.y;
    }
}

// LDS bytes of the filter for n_bins bins in precision T: the sequence.
template <typename T> size_t filter_lds(int nb)
{
    int P = 1;
    while (P < 2 * nb) P <<= 1;
    return (size_t)P * sizeof(Cx<T>);
}

// Threads per filter block: up to P/2 = 1024 butterflies per stage each in
// a thread of its own (P = 2048 at 729 bins), more in turn.
constexpr int kFilterThreads = 1024;

template <typename T>
__global__ __launch_bounds__(kFilterThreads) void k_filter(const T *__restrict__ r, T *__restrict__ out,
                                                 const T *__restrict__ tab, Geo G,
                                                 int out_padded)
{
    filter_body(r, out, tab, G, out_padded, (int)blockIdx.x);
}

// Allows the filter kernels more than 64 KB of dynamic LDS (gfx950 has 160
// KB per workgroup); once per process and device is enough, but repeating
// it is harmless.
template <typename T> void allow_filter_lds(const void *kernel, size_t bytes)
{
    if (bytes > 65536)
        (void)hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)kFilterLds);
}

template <typename T>
void launch_filter(const T *r, T *out, const T *tab, const Geo &G, int out_padded,
                   hipStream_t s)
{
    const size_t shm = filter_lds<T>(G.nb);
    allow_filter_lds<T>(reinterpret_cast<const void *>(&k_filter<T>), shm);
    hipLaunchKernelGGL(k_filter<T>, dim3((G.na + 1) / 2), dim3(kFilterThreads), shm, s, r, out,
                       tab, G, out_padded);
}

// r~ = F^T C F r of every solve (rt, padded), one block per pair of angles.
template <typename T>
__global__ __launch_bounds__(kFilterThreads) void kb_filter(const Solve<T> *S, const BlkMap *map)
{
    const BlkMap m = locate(map);
    const Solve<T> d = load_solve(S, m.solve);
    if (stopped(d.st)) return;
    filter_body(d.r, d.rt, d.ftab, d.G, 1, m.local);
}

template <typename T>
void launch_b_filter(const Solve<T> *S, const BlkMap *map, int nblocks, int max_nb,
                     hipStream_t s)
{
    const size_t shm = filter_lds<T>(max_nb);
    allow_filter_lds<T>(reinterpret_cast<const void *>(&kb_filter<T>), shm);
    hipLaunchKernelGGL(kb_filter<T>, dim3(nblocks), dim3(kFilterThreads), shm, s, S, map);
}

// ---------------------------------------------------------------------------
// Finishers: block b serves solve b. Each sums the partials of the launch
// before it (fixed order) and applies that phase's scalar logic; a finisher
// whose launch did not run (the solve had stopped, the trials were over)
// leaves the state alone.
// ---------------------------------------------------------------------------

// Scalar logic of the finishers on the LDS copy of the state; every thread
// of the block calls it (the sums are shared), thread 0 applies the logic.
// Closes the previous step (alpha of the variants whose TV pass formed it,
// from the recorded ||A p||^2 and g^T p; k; the carried scalars), applies the
// iteration cap, and opens the new step: TV(x_k) = tv and ||s||^2 = s2 of the
// TV pass, v = -s/||s||, replayed decisions, trace, and the trials' table.
// Every thread of the block calls it.
template <typename T>
__device__ __forceinline__ void open_step(const Solve<T> &d, DevState *st, bool qa, double tv, double s2,
                          int &s_go, int &s_ell, bool fill)
{
    if (threadIdx.x == 0) {
        s_go = 0;
        if (qa) {
            const double qq = st->qq, gp = st->gp;
            if (!isfinite(qq) || !isfinite(gp)) {
                set_done(st, SCG_ENAN);
            } else if (qq == 0.0) {
                set_done(st, SCG_EBREAKDOWN);
            } else {
                st->alpha = -gp / qq;
                if (auto *tr = trace_at(st, d.trace)) tr->alpha = st->alpha;
            }
        }
    }
    if (threadIdx.x == 0 && !st->done) {
        if (st->open) {
            st->qq_prev = st->qq;
            st->gp_prev = st->gp;
            st->k += 1;
            st->steps += 1;
        }
        st->open = 1;
        if (st->steps >= st->max_iter) {
            set_done(st, SCG_ENOCONV);
        } else {
            const int k = st->k + st->kofs;   // the step opened here
            st->trials_step = 0;
            st->accepted = -1;
            st->gamma = 0.0;
            st->search_done = (st->flags & SCG_FLAG_NO_PERTURB) ? 1 : 0;
            st->tv_x = tv;
            st->s_norm2 = s2;
            const bool dir = s2 > 0.0 && isfinite(s2);
            st->inv_snorm = dir ? 1.0 / sqrt(s2) : 0.0;
            if (auto *tr = trace_at(st, d.trace)) {
                tr->k = k;
                tr->accepted = -1;
                tr->trials = 0;
                tr->ell = st->ell;
                tr->gamma = 0.0;
                tr->beta = 0.0;
                tr->alpha = 0.0;
                tr->tv_x = tv;
                tr->f_half = 0.0;
            }
            if (!st->search_done && d.forced != nullptr && k >= 1 && k - 1 < st->forced_len) {
                const auto *fc = gl(d.forced);
                const int nt = fc[2 * (k - 1)], am = fc[2 * (k - 1) + 1];
                const int l0 = st->ell;
                const double g = am >= 0 && dir ? gamma_at(st, l0, am) : 0.0;
                st->ell = l0 + nt;
                st->trials_step = nt;
                st->trials_total += nt;
                st->accepted = dir ? am : -1;
                st->gamma = g;
                st->search_done = 1;
                if (auto *tr = trace_at(st, d.trace)) {
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
    if (fill && s_go) fill_gtab(d.gtab, st, s_ell);
}

// The two reductions of the step-opening trial finisher at once, in a block
// wider than kBlock: its first kBlock / 64 waves form TV(x) and ||s||^2 of
// the TV pass exactly as block_sum2 does (so the bits are those the first
// trial launch formed), the other waves the first trial launch's 1 +
// kTrialsPerPass sums into tot exactly as final_sums does (a value's bits do
// not depend on which wave forms it). Every thread of the block calls it.
template <typename T>
__device__ __forceinline__ void open_trial_sums(const Solve<T> &d, double &tv, double &s2, double *tot)
{
    constexpr int KW = kBlock / 64;
    constexpr int U = 8;
    __shared__ double wsum[2][KW];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (wid < KW) {
        const auto *pg = gl(d.partials2);
        const int n = d.nb_xtv;
        double acc_a = 0.0, acc_b = 0.0;
        for (int b0 = threadIdx.x; b0 < n; b0 += kBlock * U) {
            double va[U], vb[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int b = b0 + kBlock * u;
                va[u] = b < n ? pg[2 * (size_t)b] : 0.0;
                vb[u] = b < n ? pg[2 * (size_t)b + 1] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (b0 + kBlock * u < n) {
                    acc_a += va[u];
                    acc_b += vb[u];
                }
            }
        }
        acc_a = wave_sum(acc_a);
        acc_b = wave_sum(acc_b);
        if (lane == 0) {
            wsum[0][wid] = acc_a;
            wsum[1][wid] = acc_b;
        }
    } else {
        const int nw = (int)(blockDim.x >> 6) - KW;
        constexpr int stride = 1 + kTrialsPerPass;
        const int nblk = d.nb_trA;
        const auto *pg = gl(d.partials);
        for (int k = wid - KW; k < stride; k += nw) {
            double acc = 0.0;
            for (int b0 = lane; b0 < nblk; b0 += 64 * U) {
                double v[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int b = b0 + 64 * u;
                    v[u] = b < nblk ? pg[(size_t)b * stride + k] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (b0 + 64 * u < nblk) acc += v[u];
            }
            acc = wave_sum(acc);
            if (lane == 0) tot[k] = acc;
        }
    }
    __syncthreads();
    tv = 0.0;
    s2 = 0.0;
#pragma unroll
    for (int w = 0; w < KW; ++w) {
        tv += wsum[0][w];
        s2 += wsum[1][w];
    }
}

// The trial decision of perturbed() after a trial launch: the first m with
// TV(x + gamma_m v) <= TV(x), exactly as trying the values one after another;
// l advances by the trials used. first_m = first trial of the launch (0 or
// kTrialsPerPass). tag > 0 (first launch only): the second trial launch does
// not follow in this iteration, and a search the first launch leaves open
// suspends the solve (done = kSuspended, susp_tag = tag; every later launch
// returns at once) until the host enqueues the rest of the step. Every
// thread of the block calls it.
template <typename T>
__device__ __forceinline__ void trial_decision(const Solve<T> &d, DevState *st, int first_m, int tag, double *tot,
                               bool summed = false)
{
    if (st->search_done) return;
    const int nchunks = first_m == 0 ? 1 : d.trB_chunks;
    if (nchunks <= 0) return;
    const int nblk = first_m == 0 ? d.nb_trA : d.nb_trB;
    const int stride = 1 + kTrialsPerPass * nchunks;
    // summed: tot already holds the launch's sums (open_trial_sums)
    if (!summed) final_sums(d.partials, nblk, stride, stride, tot);
    if (threadIdx.x != 0) return;   // the block's other threads are done
    const bool with_tvx = first_m == 0;
    const double tvx = with_tvx ? tot[0] : st->tv_x;
    if (with_tvx) st->tv_x = tvx;
    const int left = st->max_trials - first_m;
    const int cap = kTrialsPerPass * nchunks;
    const int nv = left < cap ? left : cap;
    int hit = -1;
    for (int m = 0; m < nv; ++m)
        if (tot[1 + m] <= tvx) {
            hit = m;
            break;
        }
    const int used = hit >= 0 ? hit + 1 : nv;
    st->ell += used;
    st->trials_step += used;
    st->trials_total += used;
    if (hit >= 0) {
        st->accepted = first_m + hit;
        st->gamma = gl(d.gtab)[first_m + hit];
        st->search_done = 1;
    } else if (st->trials_step >= st->max_trials) {
        st->accepted = -1;
        st->gamma = 0.0;
        st->search_done = 1;
    }
    if (st->search_done) {
        if (auto *tr = trace_at(st, d.trace)) {
            tr->accepted = st->accepted;
            tr->trials = st->trials_step;
            tr->ell = st->ell;
            tr->gamma = st->gamma;
            tr->tv_x = tvx;
        }
    } else if (first_m == 0 && tag > 0) {
        st->done = kSuspended;
        st->susp_tag = tag;
    }
}

template <typename T>
__device__ __forceinline__ void finish_logic(const Solve<T> &d, DevState *st, int fin, int arg0, int arg1,
                             double *tot, int &s_go, int &s_ell)
{
    switch (fin) {
    case kFinResidual:
    case kFinResidualStep: {
        // the superiorized variants' initial step: the first trial launch's
        // gammas (later steps get theirs from the perturbation)
        if (fin == kFinResidual && st->variant != SCG_CG && st->variant != SCG_PCG)
            fill_first_gammas(d.gtab, st);
        final_sums(d.partials, d.nb_pj, 1, 1, tot);
        if (threadIdx.x != 0) return;   // the block's other threads are done
        const double f = 0.5 * tot[0];
        st->f_half = f;
        if (fin == kFinResidualStep)
            if (auto *tr = trace_at(st, d.trace)) tr->f_half = f;
        if (!isfinite(f)) {
            set_done(st, SCG_ENAN);
        } else if (f <= st->eps) {
            // Inside a step, the next loop test f(x_{k+1/2}) <= eps ends the
            // solve at k+1 with output x_{k+1/2}; the rest of the step is not
            // needed for the output and is skipped.
            if (fin == kFinResidualStep) {
                st->steps += 1;
                st->k += 1;
            }
            set_done(st, SCG_OK);
        }
        return;
    }
    case kFinNormQ:
    case kFinNormQCG: {
        // arg0 = 1: a CG-STEP inside a CG-K pass, where a zero ||A p||^2 or
        // a zero gradient (an exact minimiser) leaves x where it is
        final_sums(d.partials, d.nb_pj, 1, 1, tot);
        if (threadIdx.x != 0) return;   // the block's other threads are done
        const double s = tot[0];
        st->qq = s;
        if (!isfinite(s)) {
            set_done(st, SCG_ENAN);
        } else if (arg0 == 1 && (s == 0.0 || st->delta == 0.0)) {
            st->alpha = 0.0;
        } else if (s == 0.0) {
            set_done(st, SCG_EBREAKDOWN);
        } else {
            st->alpha = (fin == kFinNormQCG) ? st->delta / s : -st->gp / s;
            if (auto *tr = trace_at(st, d.trace)) tr->alpha = st->alpha;
        }
        return;
    }
    case kFinDotGH:
    case kFinDotGG: {
        final_sums(d.partials, d.nb_bp, 1, 1, tot);
        if (threadIdx.x != 0) return;   // the block's other threads are done
        if (fin == kFinDotGH) st->gh = tot[0];
        else st->gg = tot[0];
        return;
    }
    case kFinPUpdate: {
        // arg0 = rule, arg1 = init. g'^T p' from the update's partials; for
        // rules 0-2 after the initial step also the backprojection's dot
        // (g'^T h or ||g'||^2), which the update formed its beta from
        const double gp = block_sum1(d.partials3, d.nb_t32);
        const bool fused = !arg1 && arg0 <= 2;
        const double dot = fused ? block_sum1(d.partials, d.nb_bp) : 0.0;
        if (threadIdx.x != 0) return;   // the block's other threads are done
        if (fused) {
            if (arg0 == 1) st->gg = dot;
            else st->gh = dot;
        }
        const double beta = beta_of(st, arg0, arg1);
        st->beta = beta;
        st->gp = gp;
        if (arg0 == 3 || arg0 == 4) st->delta = st->gg;
        if (!isfinite(beta) || !isfinite(gp)) set_done(st, SCG_ENAN);
        if (!arg1)
            if (auto *tr = trace_at(st, d.trace)) tr->beta = beta;
        return;
    }
    case kFinDotUQ: {
        final_sums(d.partials, d.nb_pj, 1, 1, tot);
        if (threadIdx.x != 0) return;   // the block's other threads are done
        st->gh = tot[0];                // (A g')^T (A p) = g'^T h
        return;
    }
    case kFinPQ: {
        // the launch stored g'^T p' at [0, nb_t32) and ||q'||^2 after it
        final_sums(d.partials, d.nb_t32, 1, 1, tot);
        final_sums(d.partials + d.nb_t32, d.nb_sv, 1, 1, tot + 1);
        if (threadIdx.x != 0) return;   // the block's other threads are done
        const double beta = beta_of(st, 0, 0);
        st->beta = beta;
        st->gp = tot[0];
        st->qq = tot[1];
        if (auto *tr = trace_at(st, d.trace)) tr->beta = beta;
        if (!isfinite(beta) || !isfinite(tot[0]) || !isfinite(tot[1])) {
            set_done(st, SCG_ENAN);
        } else if (tot[1] == 0.0) {
            set_done(st, SCG_EBREAKDOWN);
        } else {
            st->alpha = -tot[0] / tot[1];
            if (auto *tr = trace_at(st, d.trace)) tr->alpha = st->alpha;
        }
        return;
    }
    case kFinDeltaPCG: {
        // delta' = g'^T z' of a PCG-STEP; arg0 = 1: inside a PCG-K pass (the
        // pass counts as one step)
        final_sums(d.partials, d.nb_bp, 1, 1, tot);
        if (threadIdx.x != 0) return;   // the block's other threads are done
        st->gg = tot[0];
        if (!isfinite(tot[0])) set_done(st, SCG_ENAN);
        if (arg0 == 1) return;
        st->qq_prev = st->qq;
        st->k += 1;
        st->steps += 1;
        return;
    }
    case kFinXUpdateCG: {
        // arg0 = 1: a CG-STEP inside a CG-K pass (the pass counts as one step)
        final_sums(d.partials, d.nb_vec, 1, 1, tot);
        if (threadIdx.x != 0) return;   // the block's other threads are done
        st->gg = tot[0];
        if (arg0 == 1) return;
        st->qq_prev = st->qq;
        st->k += 1;
        st->steps += 1;
        return;
    }
    case kFinTrials:
        trial_decision(d, st, arg0, arg1, tot);
        return;
    case kFinAlpha: {
        // alpha of the open step for the TV pass (local-alpha variants); the
        // TV pass's finisher records it
        if (!(local_alpha(st->variant) && st->open)) return;
        double gp, qq;
        block_sum2(d.partials3, d.nb_t32, d.partials, d.nb_pj, gp, qq);
        if (threadIdx.x == 0) st->alpha = -gp / qq;
        return;
    }
    case kFinStepScalars: {
        // arg0 = rule (0-2): the loop test on f(x_{k+1/2}) from the residual
        // projection's partials and beta from the backprojection's dot, as
        // the direction update's blocks form them in a single solve
        const double f = 0.5 * block_sum1(d.partials2, d.nb_pj);
        const double dot = block_sum1(d.partials, d.nb_bp);
        if (threadIdx.x != 0) return;   // the block's other threads are done
        st->f_half = f;
        if (auto *tr = trace_at(st, d.trace)) tr->f_half = f;
        if (!isfinite(f)) {
            set_done(st, SCG_ENAN);
            return;
        }
        if (f <= st->eps) {
            st->steps += 1;
            st->k += 1;
            set_done(st, SCG_OK);
            return;
        }
        const int rule = arg0;
        const double beta = rule == 1 ? -dot / st->gp_prev : dot / st->qq_prev;
        if (rule == 1) st->gg = dot;
        else st->gh = dot;
        st->beta = beta;
        if (!isfinite(beta)) set_done(st, SCG_ENAN);
        if (auto *tr = trace_at(st, d.trace)) tr->beta = beta;
        return;
    }
    case kFinXtv: {
        // Closes the previous step, opens the new one (open_step). For the
        // variants whose TV pass formed alpha itself, first records ||A p||^2
        // and g^T p of the step being closed (the same sums).
        double tv, s2;
        block_sum2(d.partials2, d.nb_xtv, d.partials2 + 1, d.nb_xtv, tv, s2, 2, 2);
        const bool qa = local_alpha(st->variant) && st->open;
        double qq = 0.0, gp = 0.0;
        if (qa) block_sum2(d.partials3, d.nb_t32, d.partials, d.nb_pj, gp, qq);
        if (threadIdx.x == 0 && qa) {
            st->qq = qq;
            st->gp = gp;
        }
        open_step(d, st, qa, tv, s2, s_go, s_ell, true);
        return;
    }
    case kFinOpenTrials: {
        // A single solve: the step-boundary pass recorded ||A p||^2 and g^T p
        // itself, and the first trial launch formed the opening's scalars with
        // the same sums; the step is opened as kFinXtv does, then the first
        // launch's trials are decided as kFinTrials does (arg1: as there).
        // The table's first kTrialsPerPass entries already hold this step's
        // gammas; a search that goes on gets the rest for the second launch.
        double tv, s2;
        open_trial_sums(d, tv, s2, tot);
        open_step(d, st, local_alpha(st->variant) && st->open, tv, s2, s_go, s_ell, false);
        if (st->done) return;
        trial_decision(d, st, 0, arg1, tot, true);
        __syncthreads();
        if (!st->search_done) fill_gtab(d.gtab, st, s_ell);
        return;
    }
    default:
        return;
    }
}

template <typename T>
__device__ __forceinline__ void finish_body(const Solve<T> *S, int solve, int fin, int arg0, int arg1)
{
    const Solve<T> d = load_solve(S, solve);
    __shared__ double tot[1 + kTrialsPerPass * kMaxTrialChunks];
    __shared__ int s_go, s_ell;
    __shared__ DevState sst;

    if (fin == kFinTV) {
        final_sums(d.partials, d.nb_vec, 1, 1, tot);
        if (threadIdx.x == 0) *gl(d.tvd) = tot[0];
        return;
    }
    // The state comes into LDS in one round trip of all its words; thread 0
    // works on that copy and the block writes it back at the end.
    constexpr int kWords = sizeof(DevState) / 4;
    static_assert(sizeof(DevState) % 4 == 0, "state copied in 32-bit words");
    const auto *gw = reinterpret_cast<const unsigned *>(d.st);
    unsigned *sw = reinterpret_cast<unsigned *>(&sst);
    for (int i = threadIdx.x; i < kWords; i += blockDim.x) sw[i] = gl(gw)[i];
    __syncthreads();
    if (sst.done) return;
    DevState *st = &sst;
    if (fin == kFinCGCap) {
        if (threadIdx.x == 0 && st->steps >= st->max_iter) set_done(st, SCG_ENOCONV);
    } else {
        finish_logic(d, st, fin, arg0, arg1, tot, s_go, s_ell);
    }
    __syncthreads();
    auto *gwo = reinterpret_cast<unsigned *>(d.st);
    for (int i = threadIdx.x; i < kWords; i += blockDim.x) gl(gwo)[i] = sw[i];
}

template <typename T>
__global__ __launch_bounds__(256) void kb_finish(const Solve<T> *S, int fin, int arg0, int arg1)
{
    finish_body(S, (int)blockIdx.x, fin, arg0, arg1);
}

// The trials' finishers (kFinTrials, kFinOpenTrials) sum 17 values (or more)
// per block of the trial launch, one wavefront per value: 16 wavefronts take
// them in two rounds instead of five. Only those cases run here: their sums
// are width-generic or taken by the first kBlock threads (the single-value
// block sums of the other cases assume kBlock threads).
template <typename T>
__global__ __launch_bounds__(1024) void kb_finish_wide(const Solve<T> *S, int fin, int arg0,
                                                       int arg1)
{
    finish_body(S, (int)blockIdx.x, fin, arg0, arg1);
}

template <typename T>
void launch_finish(const Solve<T> *S, int ns, int fin, int arg0, int arg1, hipStream_t s)
{
    if (fin == kFinTrials || fin == kFinOpenTrials)
        hipLaunchKernelGGL(kb_finish_wide<T>, dim3(ns), dim3(1024), 0, s, S, fin, arg0, arg1);
    else
        hipLaunchKernelGGL(kb_finish<T>, dim3(ns), dim3(kBlock), 0, s, S, fin, arg0, arg1);
}

// Copies every solve's state and output TV into compact arrays for one
// read-back.
template <typename T>
__global__ void kb_gather(const Solve<T> *S, int ns, DevState *out, double *tv)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ns) return;
    const Solve<T> d = load_solve(S, i);
    gl(out)[i] = *gl(d.st);
    gl(tv)[i] = *gl(d.tvd);
}

template <typename T>
void launch_gather(const Solve<T> *S, int ns, DevState *out, double *tv, hipStream_t s)
{
    hipLaunchKernelGGL(kb_gather<T>, dim3((ns + 63) / 64), dim3(64), 0, s, S, ns, out, tv);
}

// ---- explicit instantiations ----------------------------------------------
#define SCG_INST(T)                                                                            \
    template void launch_fill<T>(T *, size_t, T, hipStream_t);                                 \
    template void launch_copy<T>(T *, const T *, size_t, const DevState *, hipStream_t);       \
    template void launch_stage<T>(const T *, T *, const Geo &, hipStream_t);                   \
    template void launch_project<T>(const T *, const T *, const Geo &, const ProjTables &, T *, \
                                    int, int, int, int, hipStream_t);                           \
    template void launch_pad_sino<T>(const T *, T *, const Geo &, hipStream_t);                \
    template void launch_backproject<T>(const T *, const Geo &, const BpAngle *, const int *,  \
                                        T *, int, int, int, hipStream_t);                       \
    template void launch_tv<T>(const T *, T *, const Geo &, double, double *, double *,        \
                               hipStream_t);                                                    \
    template void launch_filter<T>(const T *, T *, const T *, const Geo &, int, hipStream_t);  \
    template void launch_b_stage<T>(const Solve<T> *, const BlkMap *, int, int, hipStream_t);  \
    template void launch_b_project<T>(const Solve<T> *, const BlkMap *, int, int, int, int, int,    \
                                      int, hipStream_t);                                        \
    template void launch_b_backproject<T>(const Solve<T> *, const BlkMap *, int, int, int,     \
                                          int, int, int, hipStream_t);                          \
    template void launch_b_xtv<T>(const Solve<T> *, const BlkMap *, int, int, hipStream_t);    \
    template void launch_b_trials<T>(const Solve<T> *, const BlkMap *, int, int, int,         \
                                     hipStream_t);                                            \
    template void launch_b_perturb<T>(const Solve<T> *, const BlkMap *, int, hipStream_t);     \
    template void launch_b_p_update<T>(const Solve<T> *, const BlkMap *, int, int, int, int,   \
                                       int, hipStream_t);                                       \
    template void launch_b_x_update_cg<T>(const Solve<T> *, const BlkMap *, int, hipStream_t); \
    template void launch_b_pq_update<T>(const Solve<T> *, const BlkMap *, int, hipStream_t);   \
    template void launch_b_x_update_pcg<T>(const Solve<T> *, const BlkMap *, int, hipStream_t); \
    template void launch_admit<T>(const Admit<T> *, int, hipStream_t);                        \
    template void launch_b_filter<T>(const Solve<T> *, const BlkMap *, int, int, hipStream_t); \
    template void launch_b_copy_out<T>(const Solve<T> *, const BlkMap *, int, int,             \
                                       hipStream_t);                                            \
    template void launch_b_tv<T>(const Solve<T> *, const BlkMap *, int, hipStream_t);          \
    template void launch_finish<T>(const Solve<T> *, int, int, int, int, hipStream_t);        \
    template void launch_gather<T>(const Solve<T> *, int, DevState *, double *, hipStream_t);

SCG_INST(float)
SCG_INST(double)

}  // namespace scg
