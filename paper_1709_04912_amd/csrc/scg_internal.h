// Internal declarations of libscg (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/scg.h"

namespace scg {

// Forward projector tiling. A block owns up to kPjGroup consecutive angles
// that step along the same axis and kPjBins consecutive bins; it walks the
// image in bands of kPjBand rows (of the image or of its transpose), staging
// kPjWin columns of each band in LDS. The window start of every
// (group, bin chunk, band) is precomputed on the host (kWinSkip: the band
// holds no pixel any of the block's rays crosses).
constexpr int kPjBins = 128;
constexpr int kPjBand = 32;
constexpr int kPjWin = 256;
constexpr int kPjGroup = 8;
constexpr int kWinSkip = -0x40000000;
// XCDs (chiplets, each with its own L2); the hardware hands workgroup b of a
// launch to XCD b mod kXcds.
constexpr int kXcds = 8;
constexpr int kXcdCus = 32;       // compute units per XCD
// Backprojector tiling: 16 x 16 pixel tiles, groups of 128 threads (two
// adjacent pixels each; 1, 2 or 4 groups per tile split the angles), angles
// staged in LDS in chunks of kBpChunk with a window of kBpWin bins per angle
// around the tile centre's projection.
constexpr int kBpTile = 16;
constexpr int kBpThreads = 128;
constexpr int kBpChunk = 32;
constexpr int kBpWin = 32;
constexpr int kBpHalf = 15;       // window start = floor(centre projection) - kBpHalf
// Column tiles of the mirrored backprojector's launch: the tiles of the left
// ceil(n/2) columns (each thread also writes the mirror pixels).
__host__ __device__ inline int bp_mirror_cols(int n) { return ((n + 1) / 2 + kBpTile - 1) / kBpTile; }
// Padded sinogram layout (solver residuals): rows of n_bins + 4 entries, bin b
// at offset b + 1; the pads stay zero.
constexpr int kSinoPadL = 1;
constexpr int kSinoPadR = 3;

constexpr int kTrialsPerPass = 16;   // TV trials evaluated per chunk of perturbed()
// DevState::done of a single solve whose trial search needs the second trial
// launch in an iteration enqueued without it: every launch returns at once
// until the host clears the flag and enqueues the rest of that step
// (DevState::susp_tag names the iteration)
constexpr int kSuspended = 2;
constexpr int kMaxTrials = 1024;     // cap on max_trials
constexpr int kMaxTrialChunks = (kMaxTrials + kTrialsPerPass - 1) / kTrialsPerPass;
constexpr int kMaxPartials = 65536;  // block partials per reduction (max blocks x values)
constexpr int kMaxN = 2880;          // largest accepted image side
// LDS of the preconditioning filter: one complex sequence of P =
// 2^ceil(log2(2 n_bins)) points per block, within gfx950's 160 KB per
// workgroup, so n_bins <= 8192 (FP32) and n_bins <= 4096 (FP64)
constexpr size_t kFilterLds = 163840;
constexpr int kMaxT32Blocks = 8192;  // 32 x 32 image tiles (direction update blocks)
constexpr size_t kHostPinnedBytes = 4096;   // a plan's pinned host words
constexpr size_t kPinnedStagingOffset = 2048;   // where a solve's upload images sit in them

struct Geo {
    int n, na, nb;
    int rs;       // padded sinogram row stride = nb + kSinoPadL + kSinoPadR
    double h;     // (n - 1) / 2
    double hb;    // (nb - 1) / 2
    size_t staged_elems() const { return (size_t)n * n; }   // transposed image copy
    size_t sino_elems() const { return (size_t)na * rs; }
    size_t img_elems() const { return (size_t)n * n; }
};

// Ray-driven frame of one angle. A ray crosses the image one step (row or
// column of the major axis) at a time; at step i the crossing coordinate
// along the minor axis, in pixel-index units, is
//     u(i, b) = u0_base + b * u0_step + i * slope,
// the chord splits between the pixels floor(u) and floor(u) + 1, and the left
// one receives (1/m) * clamp(C - frac(u) * K, 0, 1) with m = max(|c|,|s|),
// K = m/n (n = min(|c|,|s|); K capped at 2^20 for axis-aligned rays), C = K/2+1/2.
struct ProjAngle {
    double u0_base, u0_step, slope;
    double K, C, inv_m;
    float Kf, Cf, inv_mf;
    int major;    // 0: steps over rows (|c| >= |s|), 1: steps over columns
};

struct PjGroup {
    int a0, count, major, pad;
};

// Device tables of the forward projector for one angle-group size.
struct ProjTables {
    const ProjAngle *ang;
    const PjGroup *groups;
    const int *win;      // [group][chunk][band] window start column or kWinSkip
    const int *order;    // dispatch order: block ids (group * n_chunks + chunk) by
                         // decreasing count of bands to walk (heaviest first)
    int n_groups, n_chunks, n_bands, group_max;
    int mirror;          // 1: groups cover the angles a <= n_a / 2 and each ray
                         // also forms ray (n_a - a, b) (the mirrored form)
};

// Pixel-driven frame of one angle: pixel centre projects to the bin coordinate
// u = x c + y s + (nb-1)/2; bins floor(u) and floor(u)+1 receive
// (1/m) clamp(C - d K, 0, 1) at distances d = frac(u) and 1 - frac(u), with
// K = 1/n (capped at 2^20) and C = m K / 2 + 1/2.
struct BpAngle {
    double c, s;
    double K, C, inv_m;
    float Kf, Cf, CKf, inv_mf;   // CKf = C - K
    float cf, sf;
};

// Device-resident solver state: scalars in FP64, control in int.
struct DevState {
    // parameters
    double eps, gamma0, a, kappa;
    int max_iter, max_trials, variant, flags;
    // loop control
    int k, steps, done, status;
    // perturbation
    int ell, trials_step, accepted, search_done;
    int trials_total, forced_len, trace_cap;
    int susp_tag;    // host tag of the loop iteration that suspended the solve
    double tv_x, s_norm2, inv_snorm, gamma;
    // CG scalars
    double f_half, qq_prev, qq, gh, gg, gp, gp_prev, beta, alpha, delta;
    double tv_out;
    int is_f32;
    int restart_k;   // CG-STEPs per pass (S-CG-K)
    int open;        // a step (pass) is open and is closed by the next loop launch
    int kofs;        // trace entry of the open step: k + kofs
};

// Device descriptor of one solve: its geometry tables, the workspace
// vectors and its state. Every solver kernel takes an array of these plus a
// block map, so one launch advances one phase of every solve of a batch (a
// single solve is a batch of one).
template <typename T> struct Solve {
    Geo G;
    ProjTables P;
    const BpAngle *bang;
    const int *border;          // backprojector tile of each local block index
    const T *ftab;              // filter spectrum and twiddles (S-PCG, PCG)
    const T *y;                 // data, n_angles x n_bins
    T *x, *xh, *p, *g, *h, *s, *z;
    T *r, *q, *rt;              // padded sinograms (row stride G.rs)
    T *xs, *pt;                 // transposes of x_{k+1/2} (x, or g') and of p
    T *xout;                    // caller's output image
    double *partials;           // block partial sums of the last reduction
    double *partials2;          // partial sums of the TV pass (it reads the other
                                // region's sums) and of ||r||^2 of the step's residual
    double *partials3;          // partials of g'^T p' of the direction update,
                                // read by the TV pass that forms alpha
    double *gtab;               // gamma0 a^(l+m), m < max_trials
    double *tvd;                // TV of the output
    DevState *st;
    scg_trace_entry *trace;
    const int32_t *forced;      // replayed decisions or null
    int nb_xtv, nb_trA, nb_trB, nb_t32, nb_pj, nb_bp, nb_vec, nb_sv;
    int nb_bph;   // blocks of the h = A^T q phase (mirrored where the shape is, also in the
                  // filtered variants, whose other backprojections keep every tile)
    int trB_chunks;             // trial chunks of the second trial launch
};

// Set-up of one solve admitted to a batch, done on the device with the
// other new solves in one launch: the state and the descriptor copied from
// their packed images, the sinograms r, q, rt and the staged image xs
// zeroed (their pads must be zero), and the start image x0 (or zero) written
// to x_start and, for the restarted variants, also to x_{k+1/2}.
template <typename T> struct Admit {
    const DevState *st_src;
    DevState *st;
    const Solve<T> *desc_src;
    Solve<T> *desc;
    const T *x0;       // null: start from zero
    T *x_start, *xh;   // xh null unless restarted
    T *r, *q, *rt, *xs;
    long long J, S;    // image and padded sinogram elements
};

// Block map entry of a batched launch: the solve and its local block index.
struct BlkMap {
    int solve, local;
};

// Phases of a solver iteration (which vectors a shared kernel body uses).
enum Phase : int {
    kPjResXh = 0,     // r = A x_{k+1/2} - y (S- variants)
    kPjResX = 1,      // r = A x - y (CG)
    kPjQ = 2,         // q = A p
    kBpG = 3,         // g = A^T r
    kBpGZ = 4,        // g = A^T r, z = A^T rt (S-PCG)
    kBpH = 5,         // h = A^T q
    kStageXh = 6,     // xs = x_{k+1/2}^T
    kStageX = 7,      // xs = x^T
    kPjU = 8,         // u = A g' into rt, partials of u^T q (S-CG, three operators)
    kBpGT = 9,        // g = A^T r and xs = g^T (S-CG, three operators)
    kBpZ = 10,        // z = A^T rt, partials of z^T g (PCG steps)
    kPjResXhF = 11,   // r = A x_{k+1/2} - y with the partials of ||r||^2 in partials2:
                      // the direction update after it forms f and takes the stop test
                      // (S-CG, S-CG-CD, S-PCG)
};

// Finishers: one block per solve sums the partials of the previous launch
// in a fixed order and applies its scalar logic to the solve's state.
enum Fin : int {
    kFinResidual = 0,      // f = 1/2 ||r||^2, stop test (initial point / CG)
    kFinResidualStep = 1,  // same inside an S- step; a stop closes the step
    kFinNormQ = 2,         // ||q||^2, alpha = -g^T p / ||q||^2
    kFinNormQCG = 3,       // ||q||^2, alpha = delta / ||q||^2
    kFinDotGH = 4,         // g^T h
    kFinDotGG = 5,         // ||g||^2
    kFinXtv = 6,           // closes a step, opens the next (TV, ||s||, trials table)
    kFinTrials = 7,        // picks the first accepted trial
    kFinPUpdate = 8,       // beta and g^T p of the direction update
    kFinXUpdateCG = 9,     // CG: ||g||^2 and the step count
    kFinCGCap = 10,        // CG: iteration cap at the loop top
    kFinTV = 11,           // TV of the output
    kFinDotUQ = 12,        // (A g')^T q (S-CG, three operators)
    kFinPQ = 13,           // beta, g^T p, ||q||^2 and alpha of the p and q updates
    kFinDeltaPCG = 14,     // PCG: delta' = g^T z and the step count
    // Scalars a batched launch's blocks would otherwise each form from the
    // partials (the same sums, so the same bits): alpha for the TV pass, and
    // f with the stop test and beta for the direction update
    kFinAlpha = 15,
    kFinStepScalars = 16,
    // a single solve's step opening (kFinXtv) and first trial decision
    // (kFinTrials) in one finisher after the first trial launch
    kFinOpenTrials = 17,
};

// Block counts of the solver kernels for one solve.
int blocks_xtv(const Geo &G);
int blocks_t32(const Geo &G);
int blocks_vec(size_t n);
int blocks_trials(const Geo &G, int nchunks);
int blocks_bp(const Geo &G, bool mirror = false);
int blocks_sv(const Geo &G);   // sinogram vector kernels

// ---- launchers (kernels.hip) -------------------------------------------
template <typename T> void launch_fill(T *p, size_t n, T v, hipStream_t s);
template <typename T> void launch_copy(T *dst, const T *src, size_t n, const DevState *st,
                                       hipStream_t s);

// Standalone operators (explicit buffers, no solve state).
template <typename T> void launch_stage(const T *x, T *xs, const Geo &G, hipStream_t s);
template <typename T>
void launch_project(const T *x, const T *xt, const Geo &G, const ProjTables &P, T *out,
                    int out_stride, int out_off, int nq, int swz, hipStream_t s);
template <typename T> void launch_pad_sino(const T *y, T *rpad, const Geo &G, hipStream_t s);
template <typename T>
void launch_backproject(const T *r, const Geo &G, const BpAngle *ang, const int *border, T *out,
                        int split, int mirror, int swz, hipStream_t s);
template <typename T>
void launch_tv(const T *x, T *s_out, const Geo &G, double kappa, double *partials,
               double *tv_dst, hipStream_t s);   // partials: vec_blocks(n^2) doubles
template <typename T>
void launch_filter(const T *r, T *out, const T *table, const Geo &G, int out_padded,
                   hipStream_t s);

// Solver phases over `ns` solves (S: device array; map: device block map of
// `nblocks` entries, or null when ns == 1 and the blocks are the solve's own).
template <typename T>
void launch_b_stage(const Solve<T> *S, const BlkMap *map, int nblocks, int phase, hipStream_t s);
template <typename T>
void launch_b_project(const Solve<T> *S, const BlkMap *map, int nblocks, int phase, int nq,
                      int ga, int mir, int swz, hipStream_t s);
template <typename T>
void launch_b_backproject(const Solve<T> *S, const BlkMap *map, int nblocks, int phase,
                          int dot, int split, int mirror, int swz, hipStream_t s);
template <typename T>
void launch_b_xtv(const Solve<T> *S, const BlkMap *map, int nblocks, int given,
                  hipStream_t s);
template <typename T>
void launch_b_trials(const Solve<T> *S, const BlkMap *map, int nblocks, int first_m, int open,
                     hipStream_t s);
template <typename T>
void launch_b_perturb(const Solve<T> *S, const BlkMap *map, int nblocks, hipStream_t s);
template <typename T>
void launch_b_p_update(const Solve<T> *S, const BlkMap *map, int nblocks, int rule, int init,
                       int rec, int given, hipStream_t s);
template <typename T>
void launch_b_x_update_cg(const Solve<T> *S, const BlkMap *map, int nblocks, hipStream_t s);
// p' = -g' + beta p (blocks [0, nb_t32)) and q' = -u + beta q (the next
// nb_sv blocks) in one launch, with the partials of g'^T p' and ||q'||^2
template <typename T>
void launch_b_pq_update(const Solve<T> *S, const BlkMap *map, int nblocks, hipStream_t s);
template <typename T>
void launch_admit(const Admit<T> *recs, int n, hipStream_t s);
// PCG-STEP: x' = x + alpha p, g' = g + alpha h (blocks [0, nb_vec)) and the
// recursive residual r' = r + alpha q (the next nb_sv blocks)
template <typename T>
void launch_b_x_update_pcg(const Solve<T> *S, const BlkMap *map, int nblocks, hipStream_t s);
template <typename T>
void launch_b_filter(const Solve<T> *S, const BlkMap *map, int nblocks, int max_nb,
                     hipStream_t s);
template <typename T>
void launch_b_copy_out(const Solve<T> *S, const BlkMap *map, int nblocks, int from_xh,
                       hipStream_t s);
template <typename T>
void launch_b_tv(const Solve<T> *S, const BlkMap *map, int nblocks, hipStream_t s);
template <typename T>
void launch_finish(const Solve<T> *S, int ns, int fin, int arg0, int arg1, hipStream_t s);
template <typename T>
void launch_gather(const Solve<T> *S, int ns, DevState *out, double *tv, hipStream_t s);

}  // namespace scg
