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
constexpr int kPjBand = 16;
constexpr int kPjWin = 256;
constexpr int kPjGroup = 8;
constexpr int kPjThreads = 256;
constexpr int kWinSkip = -0x40000000;
// Backprojector tiling: 16 x 16 pixel tiles, 128 threads (two adjacent
// pixels each), angles staged in LDS in chunks of kBpChunk with a window of
// kBpWin bins per angle around the tile centre's projection.
constexpr int kBpTile = 16;
constexpr int kBpThreads = 128;
constexpr int kBpChunk = 32;
constexpr int kBpWin = 32;
constexpr int kBpHalf = 15;       // window start = floor(centre projection) - kBpHalf
// Padded sinogram layout (solver residuals): rows of n_bins + 4 entries, bin b
// at offset b + 1; the pads stay zero.
constexpr int kSinoPadL = 1;
constexpr int kSinoPadR = 3;

constexpr int kTrialsPerPass = 16;   // TV trials evaluated per pass of perturbed()
constexpr int kMaxPartials = 16384;  // block partials per reduction (max blocks x values)
constexpr int kRedGroups = 32;       // first-level arrival counters of a reduction
constexpr int kRedStride = 64;       // counters are 256 bytes apart
constexpr int kCounterBytes = (kRedGroups + 1) * kRedStride * 4;

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

// Device tables of the forward projector.
struct ProjTables {
    const ProjAngle *ang;
    const PjGroup *groups;
    const int *win;      // [group][chunk][band] window start column or kWinSkip
    int n_groups, n_chunks, n_bands, pad;
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
    int trials_total, forced_len, trace_cap, pad0;
    double tv_x, s_norm2, inv_snorm, gamma;
    // CG scalars
    double f_half, qq_prev, qq, gh, gg, gp, gp_prev, beta, alpha, delta;
    double tv_out;
    double gam[16];     // gamma0 a^(l+m), m < kTrialsPerPass, for the next trial pass
    int is_f32, pad1;
};

enum RedMode : int {
    kRedNone = 0,
    kRedResidual = 1,   // f_half = 1/2 sum r^2, stop test (initial point / plain CG)
    kRedResidualStep = 7,  // as kRedResidual inside a step; a stop closes the step
    kRedNormQ = 2,      // qq = sum q^2, alpha = -gp / qq
    kRedInitNormQ = 3,  // init: qq, alpha, qq_prev
    kRedDotGH = 4,      // gh = sum g h
    kRedDotGG = 5,      // gg = sum g g
    kRedNormQCG = 6,    // plain CG: qq, alpha = delta / qq
};

// ---- launchers (kernels.hip) -------------------------------------------
template <typename T> void launch_fill(T *p, size_t n, T v, hipStream_t s);
template <typename T> void launch_copy(T *dst, const T *src, size_t n, const DevState *st,
                                       hipStream_t s);
template <typename T> void launch_stage(const T *x, T *xs, const Geo &G, const DevState *st,
                                        hipStream_t s);
template <typename T>
void launch_project(const T *x, const T *xt, const Geo &G, const ProjTables &P, const T *y,
                    int y_stride, T *out, int out_stride, int out_off, double *partials,
                    unsigned *counter, DevState *st, int mode, scg_trace_entry *trace, int nq,
                    hipStream_t s);
template <typename T> void launch_pad_sino(const T *y, T *rpad, const Geo &G, hipStream_t s);
template <typename T>
void launch_backproject(const T *r, const T *r2, const Geo &G, const BpAngle *ang, T *out,
                        T *out2, const T *dotv, double *partials, unsigned *counter,
                        DevState *st, int mode, int split, hipStream_t s);
template <typename T>
void launch_tv(const T *x, T *s_out, const Geo &G, double kappa, double *partials,
               unsigned *counter, double *tv_dst, hipStream_t s);
template <typename T>
void launch_xtv(const T *xh, const T *p, T *x, T *s_out, const Geo &G, double *partials,
                unsigned *counter, DevState *st, const int32_t *forced, scg_trace_entry *trace,
                hipStream_t s);
template <typename T>
void launch_trials(const T *x, const T *s, const Geo &G, double *partials, unsigned *counter,
                   DevState *st, scg_trace_entry *trace, hipStream_t stream);
template <typename T>
void launch_perturb(const T *x, const T *s, T *xh, T *xht, const Geo &G, DevState *st,
                    hipStream_t stream);
template <typename T>
void launch_p_update(const T *g, const T *z, T *p, T *pt, const Geo &G, double *partials,
                     unsigned *counter, DevState *st, int rule, int init,
                     scg_trace_entry *trace, hipStream_t s);
template <typename T>
void launch_x_update_cg(T *x, const T *p, const T *h, T *g, const Geo &G, DevState *st,
                        double *partials, unsigned *counter, hipStream_t s);
template <typename T>
void launch_filter(const T *r, T *out, const T *kernel, const Geo &G, int out_padded,
                   const DevState *st, hipStream_t s);
void launch_iter_begin(DevState *st, hipStream_t s);

}  // namespace scg
