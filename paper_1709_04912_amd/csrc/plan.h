// Host-side plan object and helpers shared by the C-ABI files of libscg.
#pragma once

#include <climits>
#include <cstdint>
#include <vector>

#include "scg_internal.h"

using scg::BpAngle;
using scg::DevState;
using scg::Geo;
using scg::PjGroup;
using scg::ProjAngle;
using scg::ProjTables;

struct scg_plan {
    int device = 0;
    Geo G{};
    std::vector<double> cosv, sinv;
    ProjAngle *pang = nullptr;
    BpAngle *bang = nullptr;
    // projector tables: 8 and 4 angles per group, then the same two mirrored
    PjGroup *pgroups[4] = {nullptr, nullptr, nullptr, nullptr};
    int *pwin[4] = {nullptr, nullptr, nullptr, nullptr};
    int *porder[4] = {nullptr, nullptr, nullptr, nullptr};
    int *border = nullptr;                // backprojector tile of each launch position
    ProjTables ptab[4] = {};
    void *xs[2] = {nullptr, nullptr};     // transposed-image scratch per precision
    void *rpad[2] = {nullptr, nullptr};   // padded sinogram scratch per precision
    double *partials = nullptr;           // standalone TV partials
    double *tvbuf = nullptr;
    // pinned host words the solver reads its stop flag and final state into
    // (a read into pinned memory is one DMA, not a staged pageable copy)
    void *host_pinned = nullptr;
    // preconditioning filter per precision: P spectrum values at bit-reversed
    // positions, then the twiddles of each butterfly span (null where the
    // transform exceeds the LDS bound)
    void *ftab[2] = {nullptr, nullptr};
    scg_tuning tune[2] = {{4, 4, 8, 0, 0, 0}, {4, 2, 8, 0, 0, 0}};  // launch shapes (F32, F64)
    double filt_mu[2] = {-1.0, -1.0};      // mu of each precision's spectrum
    // kernel timing (scg_profile): HIP events around launches of chosen classes
    struct ProfRec {
        int cls;
        int iter;   // loop iteration that enqueued the launch (0: initial step)
        hipEvent_t a, b;
    };
    uint32_t prof_mask = 0;
    int prof_iter = 0;
    int prof_every = 1;                   // time one launch in this many per class
    int64_t prof_seq[SCG_KC_COUNT] = {};  // launches of each class seen
    std::vector<hipEvent_t> ev_free;
    std::vector<ProfRec> prof_pending;
    hipEvent_t prof_open[SCG_KC_COUNT] = {};
    int64_t prof_count[SCG_KC_COUNT] = {};
    double prof_ms[SCG_KC_COUNT] = {};
    int64_t prof_tail_count[SCG_KC_COUNT] = {};
    double prof_tail_ms[SCG_KC_COUNT] = {};
};


namespace scg {

// Makes `dev` the current device for the scope.
struct Device {
    int prev = -1;
    explicit Device(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~Device()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

template <typename T> inline int prec_index();
template <> inline int prec_index<float>() { return 0; }
template <> inline int prec_index<double>() { return 1; }

// Spectrum of the S-PCG preconditioner for mu (<= 0: 2 pi / P) in the plan's
// table of precision prec; SCG_EINVAL when n_bins exceeds that precision's
// LDS bound (filter_fits).
int ensure_filter(scg_plan *p, double mu, int prec);
bool filter_fits(int nb, int prec);
double filter_mu(const scg_plan *p, double mu);   // mu, or 2 pi / P for mu <= 0

// Kernel timing of scg_profile: event pairs around launches of timed classes.
void prof_mark(scg_plan *p, int cls, hipStream_t s, bool begin);
void prof_drain(scg_plan *p, int last_iter = INT_MAX);
void prof_to_tail(scg_plan *p, size_t from);

int check_params(const scg_params *pr);

// Projector tables of a launch shape.
inline const ProjTables &proj_tables(const scg_plan *p, const scg_tuning &t)
{
    return p->ptab[(t.project_angles == 4 ? 1 : 0) + (t.project_mirror ? 2 : 0)];
}

}  // namespace scg

#define HIP_TRY(expr)                                 \
    do {                                              \
        hipError_t _e = (expr);                       \
        if (_e != hipSuccess) return SCG_EDEVICE;     \
    } while (0)
