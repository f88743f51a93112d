// C-ABI of libscg: plans, operators and the superiorized CG solver driver.
//
// The solver keeps all state on the device. Each loop iteration is a fixed
// sequence of kernels that read the device-resident scalars (alpha, beta,
// f, the TV-trial decision) and return at once when the device `done` flag is
// set; the host enqueues iterations in chunks and reads the flag between
// chunks, so the iteration count is decided on the device.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <climits>
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
    PjGroup *pgroups = nullptr;
    int *pwin = nullptr;
    ProjTables ptab{};
    void *xs[2] = {nullptr, nullptr};     // transposed-image scratch per precision
    void *rpad[2] = {nullptr, nullptr};   // padded sinogram scratch per precision
    double *partials = nullptr;
    unsigned *counter = nullptr;
    double *tvbuf = nullptr;
    void *kern[2] = {nullptr, nullptr};   // filter taps k[d], d < n_bins
    scg_tuning tune[2] = {{4, 2}, {4, 2}};  // launch shapes per precision
    double kern_mu = -1.0;
    // kernel timing (scg_profile): HIP events around launches of chosen classes
    struct ProfRec {
        int cls;
        int iter;   // loop iteration that enqueued the launch (0: initial step)
        hipEvent_t a, b;
    };
    uint32_t prof_mask = 0;
    int prof_iter = 0;
    std::vector<hipEvent_t> ev_free;
    std::vector<ProfRec> prof_pending;
    hipEvent_t prof_open[SCG_KC_COUNT] = {};
    int64_t prof_count[SCG_KC_COUNT] = {};
    double prof_ms[SCG_KC_COUNT] = {};
    int64_t prof_tail_count[SCG_KC_COUNT] = {};
    double prof_tail_ms[SCG_KC_COUNT] = {};
};

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kKCap = 1048576.0;   // 2^20: K for axis-aligned rays

int hip_status(hipError_t e) { return e == hipSuccess ? SCG_OK : SCG_EDEVICE; }

#define HIP_TRY(expr)                                 \
    do {                                              \
        hipError_t _e = (expr);                       \
        if (_e != hipSuccess) return SCG_EDEVICE;     \
    } while (0)

double snap(double v)
{
    if (std::fabs(v) < 1e-12) return 0.0;
    if (std::fabs(1.0 - std::fabs(v)) < 1e-12) return v > 0 ? 1.0 : -1.0;
    return v;
}

// Per-angle frames for the ray-driven projector and the pixel-driven
// backprojector, from the FP64 trig table.
void build_angles(const Geo &G, const std::vector<double> &cv, const std::vector<double> &sv,
                  std::vector<ProjAngle> &pa, std::vector<BpAngle> &ba)
{
    const double h = G.h, hb = G.hb;
    pa.resize(G.na);
    ba.resize(G.na);
    for (int a = 0; a < G.na; ++a) {
        const double c = cv[a], s = sv[a];
        const double ac = std::fabs(c), as = std::fabs(s);
        const double m = std::max(ac, as), n = std::min(ac, as);
        ProjAngle P{};
        if (ac >= as) {     // step over rows: x = (t - y s) / c
            P.major = 0;
            P.u0_base = (-hb - h * s) / c + h;
            P.u0_step = 1.0 / c;
            P.slope = s / c;
        } else {            // step over columns: y = (t - x c) / s
            P.major = 1;
            P.u0_base = h - (h * c - hb) / s;
            P.u0_step = -1.0 / s;
            P.slope = c / s;
        }
        P.K = n > 0.0 ? std::min(m / n, kKCap) : kKCap;
        P.C = 0.5 * P.K + 0.5;
        P.inv_m = 1.0 / m;
        P.Kf = (float)P.K;
        P.Cf = (float)P.C;
        P.inv_mf = (float)P.inv_m;
        pa[a] = P;

        BpAngle B{};
        B.c = c;
        B.s = s;
        B.K = n > 0.0 ? std::min(1.0 / n, kKCap) : kKCap;
        B.C = 0.5 * m * B.K + 0.5;
        B.inv_m = 1.0 / m;
        B.Kf = (float)B.K;
        B.Cf = (float)B.C;
        B.CKf = (float)(B.C - B.K);
        B.inv_mf = (float)B.inv_m;
        B.cf = (float)c;
        B.sf = (float)s;
        ba[a] = B;
    }
}

// Groups of consecutive angles stepping along the same axis and, for every
// (group, bin chunk, band), the first LDS-staged column: the band's columns
// crossed by any of the block's rays, with two columns of margin each side.
// The group size shrinks until every window fits kPjWin columns.
int build_proj_tables(scg_plan *p, const std::vector<ProjAngle> &pa)
{
    const Geo &G = p->G;
    const int n_chunks = (G.nb + scg::kPjBins - 1) / scg::kPjBins;
    const int n_bands = (G.n + scg::kPjBand - 1) / scg::kPjBand;
    for (int gmax = scg::kPjGroup; gmax >= 1; --gmax) {
        std::vector<PjGroup> groups;
        for (int a = 0; a < G.na;) {
            PjGroup g{a, 1, pa[a].major, 0};
            while (g.count < gmax && a + g.count < G.na && pa[a + g.count].major == g.major)
                ++g.count;
            groups.push_back(g);
            a += g.count;
        }
        if ((size_t)groups.size() * n_chunks > (size_t)scg::kMaxPartials) return SCG_EINVAL;
        std::vector<int> win((size_t)groups.size() * n_chunks * n_bands);
        bool ok = true;
        for (size_t gi = 0; gi < groups.size() && ok; ++gi) {
            for (int ch = 0; ch < n_chunks && ok; ++ch) {
                const int b_lo = ch * scg::kPjBins;
                const int b_hi = std::min(G.nb, b_lo + scg::kPjBins) - 1;
                for (int band = 0; band < n_bands; ++band) {
                    const int i_lo = band * scg::kPjBand, i_hi = i_lo + scg::kPjBand - 1;
                    double umin = INFINITY, umax = -INFINITY;
                    for (int g = 0; g < groups[gi].count; ++g) {
                        const ProjAngle &A = pa[groups[gi].a0 + g];
                        for (int b : {b_lo, b_hi})
                            for (int i : {i_lo, i_hi}) {
                                const double u0 = std::fma((double)b, A.u0_step, A.u0_base);
                                const double u = std::fma((double)i, A.slope, u0);
                                umin = std::min(umin, u);
                                umax = std::max(umax, u);
                            }
                    }
                    int &w = win[((size_t)gi * n_chunks + ch) * n_bands + band];
                    if (umax < -2.0 || umin > (double)G.n + 1.0) {
                        w = scg::kWinSkip;
                        continue;
                    }
                    const double fmin = std::floor(umin), fmax = std::floor(umax);
                    if (fmax - fmin > (double)(scg::kPjWin - 5)) {
                        ok = false;
                        break;
                    }
                    w = (int)fmin - 2;
                }
            }
        }
        if (!ok) continue;
        if (hipMalloc(&p->pgroups, groups.size() * sizeof(PjGroup)) != hipSuccess ||
            hipMalloc(&p->pwin, win.size() * sizeof(int)) != hipSuccess)
            return SCG_ENOMEM;
        if (hipMemcpy(p->pgroups, groups.data(), groups.size() * sizeof(PjGroup),
                      hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(p->pwin, win.data(), win.size() * sizeof(int), hipMemcpyHostToDevice) !=
                hipSuccess)
            return SCG_EDEVICE;
        p->ptab.ang = p->pang;
        p->ptab.groups = p->pgroups;
        p->ptab.win = p->pwin;
        p->ptab.n_groups = (int)groups.size();
        p->ptab.n_chunks = n_chunks;
        p->ptab.n_bands = n_bands;
        return SCG_OK;
    }
    return SCG_EINVAL;
}

int filter_pad(int nb)
{
    int P = 1;
    while (P < 2 * nb) P <<= 1;
    return P;
}

// k[d] = (1/P) sum_{m=-P/2}^{P/2-1} c(w_m) cos(w_m d), c(w) = (|w| + mu)(0.54 + 0.46 cos w).
int ensure_filter(scg_plan *p, double mu)
{
    const int nb = p->G.nb, P = filter_pad(nb);
    if (mu <= 0.0) mu = 2.0 * kPi / P;
    if (p->kern[0] != nullptr && p->kern_mu == mu) return SCG_OK;
    std::vector<double> k(nb);
    std::vector<double> cw(P);
    for (int m = -P / 2; m < P / 2; ++m) {
        const double w = 2.0 * kPi * m / P;
        cw[m + P / 2] = (std::fabs(w) + mu) * (0.54 + 0.46 * std::cos(w));
    }
    for (int d = 0; d < nb; ++d) {
        double acc = 0.0;
        for (int m = -P / 2; m < P / 2; ++m) acc += cw[m + P / 2] * std::cos(2.0 * kPi * m * d / P);
        k[d] = acc / P;
    }
    std::vector<float> kf(k.begin(), k.end());
    if (p->kern[0] == nullptr) {
        HIP_TRY(hipMalloc(&p->kern[0], nb * sizeof(float)));
        HIP_TRY(hipMalloc(&p->kern[1], nb * sizeof(double)));
    }
    HIP_TRY(hipMemcpy(p->kern[0], kf.data(), nb * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(p->kern[1], k.data(), nb * sizeof(double), hipMemcpyHostToDevice));
    p->kern_mu = mu;
    return SCG_OK;
}

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

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

hipEvent_t take_event(scg_plan *p)
{
    if (!p->ev_free.empty()) {
        hipEvent_t e = p->ev_free.back();
        p->ev_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Marks the start (begin = true) or end of a launch of class `cls` when the
// class is being timed.
void prof_mark(scg_plan *p, int cls, hipStream_t s, bool begin)
{
    if (!(p->prof_mask & (1u << cls))) return;
    hipEvent_t e = take_event(p);
    if (e == nullptr) return;
    (void)hipEventRecord(e, s);
    if (begin) {
        p->prof_open[cls] = e;
    } else if (p->prof_open[cls] != nullptr) {
        p->prof_pending.push_back({cls, p->prof_iter, p->prof_open[cls], e});
        p->prof_open[cls] = nullptr;
    } else {
        p->ev_free.push_back(e);
    }
}

// Accumulates the elapsed times of recorded launches. Launches enqueued by
// loop iterations past `last_iter` (the solve had already stopped; their
// kernels returned at once) are kept apart, except the TV kernel of the
// iteration after it, which still closes the last step.
void prof_drain(scg_plan *p, int last_iter = INT_MAX)
{
    for (const auto &r : p->prof_pending) {
        float ms = 0.0f;
        if (hipEventSynchronize(r.b) == hipSuccess &&
            hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            const int lim = last_iter == INT_MAX ? INT_MAX : last_iter + (r.cls == SCG_KC_TV);
            if (r.iter <= lim) {
                p->prof_ms[r.cls] += ms;
                p->prof_count[r.cls] += 1;
            } else {
                p->prof_tail_ms[r.cls] += ms;
                p->prof_tail_count[r.cls] += 1;
            }
        }
        p->ev_free.push_back(r.a);
        p->ev_free.push_back(r.b);
    }
    p->prof_pending.clear();
}

#define PROF(cls, call)                          \
    do {                                         \
        prof_mark(plan, (cls), st0, true);       \
        call;                                    \
        prof_mark(plan, (cls), st0, false);      \
    } while (0)

// Workspace layout of scg_solve.
struct Layout {
    size_t x, xh, p, g, h, s, z, r, q, rt, xs, pt, partials, counter, state, forced, trace, tv,
        total;
};

Layout layout(const Geo &G, size_t esz, int max_iter)
{
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    const size_t J = G.img_elems(), S = G.sino_elems();
    L.x = take(J * esz);
    L.xh = take(J * esz);
    L.p = take(J * esz);
    L.g = take(J * esz);
    L.h = take(J * esz);
    L.s = take(J * esz);
    L.z = take(J * esz);
    L.r = take(S * esz);
    L.q = take(S * esz);
    L.rt = take(S * esz);
    L.xs = take(G.staged_elems() * esz);
    L.pt = take(G.staged_elems() * esz);
    L.partials = take(scg::kMaxPartials * sizeof(double));
    L.counter = take(scg::kCounterBytes);
    L.state = take(sizeof(DevState));
    L.forced = take((size_t)2 * (max_iter + 1) * sizeof(int32_t));
    L.trace = take((size_t)(max_iter + 1) * sizeof(scg_trace_entry));
    L.tv = take(sizeof(double));
    L.total = off;
    return L;
}

int check_params(const scg_params *pr)
{
    if (pr == nullptr) return SCG_EINVAL;
    if (pr->variant < SCG_CG || pr->variant > SCG_S_PCG) return SCG_EINVAL;
    if (pr->prec != SCG_F32 && pr->prec != SCG_F64) return SCG_EINVAL;
    if (!(pr->eps > 0.0) || !std::isfinite(pr->eps)) return SCG_EINVAL;
    if (!(pr->gamma0 >= 0.0) || !std::isfinite(pr->gamma0)) return SCG_EINVAL;
    if (!(pr->a > 0.0 && pr->a < 1.0)) return SCG_EINVAL;
    if (pr->max_iter < 0 || pr->max_iter > 1000000) return SCG_EINVAL;
    if (pr->max_trials < 1 || pr->max_trials > 1024) return SCG_EINVAL;
    if (!(pr->tv_kappa >= 0.0) || !std::isfinite(pr->tv_kappa)) return SCG_EINVAL;
    return SCG_OK;
}

template <typename T> int prec_index();
template <> int prec_index<float>() { return 0; }
template <> int prec_index<double>() { return 1; }

template <typename T>
int solve_impl(scg_plan *plan, const scg_params *pr, const void *y_, const void *x0_, void *xout_,
               char *ws, scg_report *rep, scg_trace_entry *trace_host, int32_t trace_cap,
               const int32_t *forced_host, int32_t forced_len, hipStream_t st0)
{
    const Geo &G = plan->G;
    const size_t J = G.img_elems(), S = G.sino_elems();
    const Layout Lw = layout(G, sizeof(T), pr->max_iter);
    T *x = reinterpret_cast<T *>(ws + Lw.x);
    T *xh = reinterpret_cast<T *>(ws + Lw.xh);
    T *p = reinterpret_cast<T *>(ws + Lw.p);
    T *g = reinterpret_cast<T *>(ws + Lw.g);
    T *h = reinterpret_cast<T *>(ws + Lw.h);
    T *s = reinterpret_cast<T *>(ws + Lw.s);
    T *z = reinterpret_cast<T *>(ws + Lw.z);
    T *r = reinterpret_cast<T *>(ws + Lw.r);
    T *q = reinterpret_cast<T *>(ws + Lw.q);
    T *rt = reinterpret_cast<T *>(ws + Lw.rt);
    T *xs = reinterpret_cast<T *>(ws + Lw.xs);   // transpose of x_{k+1/2} (or of x in CG)
    T *pt = reinterpret_cast<T *>(ws + Lw.pt);   // transpose of p
    double *partials = reinterpret_cast<double *>(ws + Lw.partials);
    unsigned *counter = reinterpret_cast<unsigned *>(ws + Lw.counter);
    DevState *st = reinterpret_cast<DevState *>(ws + Lw.state);
    int32_t *forced = reinterpret_cast<int32_t *>(ws + Lw.forced);
    scg_trace_entry *trace = reinterpret_cast<scg_trace_entry *>(ws + Lw.trace);
    double *tvd = reinterpret_cast<double *>(ws + Lw.tv);
    const T *y = static_cast<const T *>(y_);
    const T *x0 = static_cast<const T *>(x0_);
    T *xout = static_cast<T *>(xout_);
    const int variant = pr->variant;
    const bool is_cg = variant == SCG_CG;

    if (variant == SCG_S_PCG) {
        int rc = ensure_filter(plan, pr->precond_mu);
        if (rc) return rc;
    }
    const T *kern = static_cast<const T *>(plan->kern[prec_index<T>()]);

    // Pads of the staged image and of the sinograms must be zero.
    scg::launch_fill<T>(r, S, T(0), st0);
    scg::launch_fill<T>(q, S, T(0), st0);
    scg::launch_fill<T>(rt, S, T(0), st0);
    scg::launch_fill<T>(xs, G.staged_elems(), T(0), st0);
    HIP_TRY(hipMemsetAsync(counter, 0, scg::kCounterBytes, st0));

    DevState hs{};
    hs.eps = pr->eps;
    hs.gamma0 = pr->gamma0;
    hs.a = pr->a;
    hs.kappa = pr->tv_kappa;
    hs.max_iter = pr->max_iter;
    hs.max_trials = pr->max_trials;
    hs.variant = variant;
    hs.flags = (int)pr->flags;
    hs.k = 0;
    hs.steps = is_cg ? 0 : -1;   // the initial step of the S- variants is not counted
    hs.accepted = -1;
    hs.is_f32 = sizeof(T) == 4 ? 1 : 0;
    hs.trace_cap = std::min<int32_t>(trace_cap > 0 ? trace_cap : 0, pr->max_iter + 1);
    if (trace_host == nullptr) hs.trace_cap = pr->max_iter + 1;
    const int nf = forced_host ? std::min<int32_t>(std::max<int32_t>(forced_len, 0), pr->max_iter + 1) : 0;
    hs.forced_len = nf;
    HIP_TRY(hipMemcpyAsync(st, &hs, sizeof(DevState), hipMemcpyHostToDevice, st0));
    if (nf > 0)
        HIP_TRY(hipMemcpyAsync(forced, forced_host, (size_t)2 * nf * sizeof(int32_t),
                               hipMemcpyHostToDevice, st0));
    const int32_t *forced_d = nf > 0 ? forced : nullptr;

    // x_{1/2} = x0 (S- variants) or x_0 (CG).
    T *x_start = is_cg ? x : xh;
    if (x0 != nullptr) scg::launch_copy<T>(x_start, x0, J, nullptr, st0);
    else scg::launch_fill<T>(x_start, J, T(0), st0);

    const int rs = G.rs, off = scg::kSinoPadL;
    const scg_tuning tn = plan->tune[prec_index<T>()];
    // Forward projections read an image and its transpose: x_{k+1/2} with
    // xs (written by the perturbation), p with pt (written by the direction
    // update); x0 and the CG iterate are transposed explicitly.
    auto project_res = [&](const T *img, int mode) {
        PROF(SCG_KC_PROJECT, scg::launch_project<T>(img, xs, G, plan->ptab, y, G.nb, r, rs, off,
                                                    partials, counter, st, mode, trace, tn.project_groups,
                                                    st0));
    };
    auto project_q = [&](int mode) {
        PROF(SCG_KC_PROJECT, scg::launch_project<T>(p, pt, G, plan->ptab, nullptr, 0, q, rs, off,
                                                    partials, counter, st, mode, trace,
                                                    tn.project_groups, st0));
    };
    auto backproject = [&](const T *src, const T *src2, T *dst, T *dst2, const T *dotv,
                            int mode) {
        PROF(SCG_KC_BACKPROJECT, scg::launch_backproject<T>(src, src2, G, plan->bang, dst, dst2,
                                                            dotv, partials, counter, st, mode,
                                                            tn.backproject_split, st0));
    };
    auto p_update = [&](const T *src_z, int rule, int init) {
        PROF(SCG_KC_VECTOR, scg::launch_p_update<T>(g, src_z, p, pt, G, partials, counter, st,
                                                    rule, init, trace, st0));
    };
    auto filter = [&]() {
        PROF(SCG_KC_FILTER, scg::launch_filter<T>(r, rt, kern, G, 1, st, st0));
    };

    // ---- initial step -------------------------------------------------
    if (is_cg) {
        // Alg. CG: g0 = A^T(A x0 - y), p0 = -g0, delta0 = ||g0||^2.
        PROF(SCG_KC_STAGE, scg::launch_stage<T>(x, xs, G, st, st0));
        project_res(x, scg::kRedResidual);
        backproject(r, nullptr, g, nullptr, nullptr, scg::kRedDotGG);
        p_update(nullptr, 3, 1);
    } else {
        // S-CG / S-CG-CD / S-PCG steps 1-6: x_{1/2} = x0, g0, (z0), p0, h0,
        // alpha = -g0^T p0 / p0^T h0. x1 = x0 + alpha p0 and k = 1 are formed
        // by the first loop kernel, which closes every step.
        PROF(SCG_KC_STAGE, scg::launch_stage<T>(xh, xs, G, st, st0));
        project_res(xh, scg::kRedResidual);
        if (variant == SCG_S_PCG) {
            filter();
            backproject(r, rt, g, z, nullptr, scg::kRedNone);
            p_update(z, 2, 1);
        } else {
            backproject(r, nullptr, g, nullptr, nullptr, scg::kRedNone);
            p_update(nullptr, 0, 1);
        }
        project_q(scg::kRedNormQ);
        if (variant != SCG_S_CG_CD) backproject(q, nullptr, h, nullptr, nullptr, scg::kRedNone);
    }

    const int passes = (pr->max_trials + scg::kTrialsPerPass - 1) / scg::kTrialsPerPass;
    auto enqueue_iteration = [&]() {
        if (is_cg) {
            PROF(SCG_KC_CONTROL, scg::launch_iter_begin(st, st0));
            project_q(scg::kRedNormQCG);
            backproject(q, nullptr, h, nullptr, nullptr, scg::kRedNone);
            PROF(SCG_KC_VECTOR, scg::launch_x_update_cg<T>(x, p, h, g, G, st, partials, counter,
                                                           st0));
            p_update(nullptr, 3, 0);
            PROF(SCG_KC_STAGE, scg::launch_stage<T>(x, xs, G, st, st0));
            project_res(x, scg::kRedResidual);
            return;
        }
        // close the previous step (x_{k+1} = x_{k+1/2} + alpha p) and start
        // perturbed(x_k): TV subgradient, then the trials
        PROF(SCG_KC_TV, scg::launch_xtv<T>(xh, p, x, s, G, partials, counter, st, forced_d, trace,
                                           st0));
        for (int ps = 0; ps < passes; ++ps)
            PROF(SCG_KC_TRIALS, scg::launch_trials<T>(x, s, G, partials, counter, st, trace, st0));
        PROF(SCG_KC_VECTOR, scg::launch_perturb<T>(x, s, xh, xs, G, st, st0));
        // the step (CG-PR-STEP / CG-CD-STEP / PCG-PR-STEP) from x_{k+1/2}
        project_res(xh, scg::kRedResidualStep);
        if (variant == SCG_S_PCG) {
            filter();
            backproject(r, rt, g, z, h, scg::kRedDotGH);
            p_update(z, 2, 0);
        } else if (variant == SCG_S_CG_CD) {
            backproject(r, nullptr, g, nullptr, nullptr, scg::kRedDotGG);
            p_update(nullptr, 1, 0);
        } else {
            backproject(r, nullptr, g, nullptr, h, scg::kRedDotGH);
            p_update(nullptr, 0, 0);
        }
        project_q(scg::kRedNormQ);
        if (variant != SCG_S_CG_CD) backproject(q, nullptr, h, nullptr, nullptr, scg::kRedNone);
    };

    // ---- loop: chunks of iterations, device decides when to stop ---------
    int done = 0;
    long issued = 0;
    int chunk = 2;
    HIP_TRY(hipMemcpyAsync(&done, &st->done, sizeof(int), hipMemcpyDeviceToHost, st0));
    HIP_TRY(hipStreamSynchronize(st0));
    while (!done && issued <= (long)pr->max_iter) {
        for (int c = 0; c < chunk; ++c) {
            plan->prof_iter = (int)std::min<long>(issued + c + 1, INT_MAX - 1);
            enqueue_iteration();
        }
        issued += chunk;
        chunk = std::min(chunk * 2, 16);
        HIP_TRY(hipMemcpyAsync(&done, &st->done, sizeof(int), hipMemcpyDeviceToHost, st0));
        HIP_TRY(hipStreamSynchronize(st0));
    }
    plan->prof_iter = INT_MAX;

    // ---- output ---------------------------------------------------------
    const T *out = is_cg ? x : xh;
    scg::launch_copy<T>(xout, out, J, nullptr, st0);
    scg::launch_tv<T>(out, nullptr, G, pr->tv_kappa, partials, counter, tvd, st0);
    DevState fs{};
    double tv_out = 0.0;
    HIP_TRY(hipMemcpyAsync(&fs, st, sizeof(DevState), hipMemcpyDeviceToHost, st0));
    HIP_TRY(hipMemcpyAsync(&tv_out, tvd, sizeof(double), hipMemcpyDeviceToHost, st0));
    if (trace_host != nullptr && trace_cap > 0) {
        const int n = std::min<int>(trace_cap, pr->max_iter + 1);
        HIP_TRY(hipMemcpyAsync(trace_host, trace, (size_t)n * sizeof(scg_trace_entry),
                               hipMemcpyDeviceToHost, st0));
    }
    HIP_TRY(hipStreamSynchronize(st0));
    prof_drain(plan, std::max(fs.steps, 0));
    plan->prof_iter = 0;
    if (rep != nullptr) {
        std::memset(rep, 0, sizeof(*rep));
        rep->status = fs.done ? fs.status : SCG_ENOCONV;
        rep->k = is_cg ? fs.k : std::max(fs.k, 1);
        rep->steps = std::max(fs.steps, 0);
        rep->trials_total = fs.trials_total;
        rep->ell = fs.ell;
        rep->f_out = fs.f_half;
        rep->tv_out = tv_out;
    }
    return fs.done ? fs.status : SCG_ENOCONV;
}

}  // namespace

namespace {

bool tuning_valid(const scg_tuning &t)
{
    return (t.project_groups == 2 || t.project_groups == 4) &&
           (t.backproject_split == 1 || t.backproject_split == 2 ||
            t.backproject_split == 4);
}

// Mean time of `reps` launches of `fn` on stream s, after one untimed launch.
template <typename F> float time_launches(F fn, hipStream_t s, int reps)
{
    hipEvent_t a = nullptr, b = nullptr;
    float ms = -1.0f;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) goto out;
    fn();
    if (hipEventRecord(a, s) != hipSuccess) goto out;
    for (int i = 0; i < reps; ++i) fn();
    if (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
        hipEventElapsedTime(&ms, a, b) != hipSuccess)
        ms = -1.0f;
    else
        ms /= (float)reps;
out:
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    return ms;
}

template <typename T>
int autotune_impl(scg_plan *plan, hipStream_t s, scg_tuning *chosen)
{
    const Geo &G = plan->G;
    const int pi = prec_index<T>();
    T *x = nullptr, *y = nullptr;
    if (hipMalloc(&x, G.img_elems() * sizeof(T)) != hipSuccess) return SCG_ENOMEM;
    if (hipMalloc(&y, G.sino_elems() * sizeof(T)) != hipSuccess) {
        (void)hipFree(x);
        return SCG_ENOMEM;
    }
    scg::launch_fill<T>(x, G.img_elems(), T(1), s);
    scg::launch_fill<T>(y, G.sino_elems(), T(1), s);
    T *xs = static_cast<T *>(plan->xs[pi]);
    scg::launch_stage<T>(x, xs, G, nullptr, s);
    constexpr int kReps = 5;
    scg_tuning best = plan->tune[pi];
    float best_pj = -1.0f, best_bp = -1.0f;
    for (int nq : {2, 4}) {
        const float ms = time_launches(
            [&] {
                scg::launch_project<T>(x, xs, G, plan->ptab, nullptr, 0, y, G.rs, scg::kSinoPadL,
                                       nullptr, nullptr, nullptr, scg::kRedNone, nullptr, nq, s);
            },
            s, kReps);
        if (ms > 0.0f && (best_pj < 0.0f || ms < best_pj)) {
            best_pj = ms;
            best.project_groups = nq;
        }
    }
    for (int sp : {1, 2, 4}) {
        const float ms = time_launches(
            [&] {
                scg::launch_backproject<T>(y, nullptr, G, plan->bang, x, nullptr, nullptr, nullptr,
                                           nullptr, nullptr, scg::kRedNone, sp, s);
            },
            s, kReps);
        if (ms > 0.0f && (best_bp < 0.0f || ms < best_bp)) {
            best_bp = ms;
            best.backproject_split = sp;
        }
    }
    const hipError_t e = hipStreamSynchronize(s);
    (void)hipFree(x);
    (void)hipFree(y);
    if (e != hipSuccess || best_pj < 0.0f || best_bp < 0.0f) return SCG_EDEVICE;
    plan->tune[pi] = best;
    if (chosen != nullptr) *chosen = best;
    return SCG_OK;
}

}  // namespace

extern "C" {

void scg_default_params(scg_params *p)
{
    if (p == nullptr) return;
    std::memset(p, 0, sizeof(*p));
    p->variant = SCG_S_CG;
    p->prec = SCG_F32;
    p->eps = 0.0;
    p->gamma0 = 0.0;
    p->a = 0.975;
    p->max_iter = 1000;
    p->max_trials = 100;
    p->tv_kappa = 0.0;
    p->precond_mu = 0.0;
    p->flags = 0;
}

const char *scg_strerror(int status)
{
    switch (status) {
    case SCG_OK: return "ok";
    case SCG_EINVAL: return "invalid argument";
    case SCG_ENOMEM: return "out of device memory or workspace too small";
    case SCG_EDEVICE: return "HIP runtime error";
    case SCG_ENOCONV: return "iteration cap reached with f > eps";
    case SCG_ENAN: return "non-finite value in a CG scalar";
    case SCG_EBREAKDOWN: return "breakdown: ||A p||^2 = 0";
    case SCG_EAGAIN: return "no free slot or memory";
    case SCG_EINPROGRESS: return "in progress";
    case SCG_ENOTFOUND: return "unknown ticket";
    default: return "unknown status";
    }
}

int scg_plan_create(const scg_geom *g, int device, scg_plan **out)
{
    if (out == nullptr) return SCG_EINVAL;
    *out = nullptr;
    if (g == nullptr || g->n < 2 || g->n_angles < 1 || g->n_bins < 1) return SCG_EINVAL;
    if (g->n > 16384 || g->n_angles > 65536 || g->n_bins > 65536) return SCG_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return SCG_EDEVICE;
    Device dg(device);
    scg_plan *p = new (std::nothrow) scg_plan();
    if (p == nullptr) return SCG_ENOMEM;
    p->device = device;
    Geo &G = p->G;
    G.n = g->n;
    G.na = g->n_angles;
    G.nb = g->n_bins;
    G.rs = G.nb + scg::kSinoPadL + scg::kSinoPadR;
    G.h = 0.5 * (G.n - 1);
    G.hb = 0.5 * (G.nb - 1);
    // The backprojector grid must fit the reduction partials, and a padded
    // projection plus the filter taps must fit in LDS.
    const size_t bp_tiles = (size_t)((G.n + scg::kBpTile - 1) / scg::kBpTile);
    if (bp_tiles * bp_tiles > (size_t)scg::kMaxPartials ||
        (size_t)3 * G.nb * sizeof(double) > 65536) {
        delete p;
        return SCG_EINVAL;
    }
    p->cosv.resize(G.na);
    p->sinv.resize(G.na);
    for (int a = 0; a < G.na; ++a) {
        const double th = (double)a * kPi / (double)G.na;
        p->cosv[a] = snap(std::cos(th));
        p->sinv[a] = snap(std::sin(th));
    }
    std::vector<ProjAngle> pa;
    std::vector<BpAngle> ba;
    build_angles(G, p->cosv, p->sinv, pa, ba);
    bool ok = hipMalloc(&p->pang, pa.size() * sizeof(ProjAngle)) == hipSuccess &&
              hipMalloc(&p->bang, ba.size() * sizeof(BpAngle)) == hipSuccess &&
              hipMalloc(&p->xs[0], G.staged_elems() * sizeof(float)) == hipSuccess &&
              hipMalloc(&p->xs[1], G.staged_elems() * sizeof(double)) == hipSuccess &&
              hipMalloc(&p->rpad[0], G.sino_elems() * sizeof(float)) == hipSuccess &&
              hipMalloc(&p->rpad[1], G.sino_elems() * sizeof(double)) == hipSuccess &&
              hipMalloc(&p->partials, scg::kMaxPartials * sizeof(double)) == hipSuccess &&
              hipMalloc(&p->counter, scg::kCounterBytes) == hipSuccess &&
              hipMalloc(&p->tvbuf, sizeof(double)) == hipSuccess;
    if (!ok) {
        scg_plan_destroy(p);
        return SCG_ENOMEM;
    }
    ok = hipMemcpy(p->pang, pa.data(), pa.size() * sizeof(ProjAngle), hipMemcpyHostToDevice) ==
             hipSuccess &&
         hipMemcpy(p->bang, ba.data(), ba.size() * sizeof(BpAngle), hipMemcpyHostToDevice) ==
             hipSuccess &&
         hipMemset(p->xs[0], 0, G.staged_elems() * sizeof(float)) == hipSuccess &&
         hipMemset(p->xs[1], 0, G.staged_elems() * sizeof(double)) == hipSuccess &&
         hipMemset(p->rpad[0], 0, G.sino_elems() * sizeof(float)) == hipSuccess &&
         hipMemset(p->rpad[1], 0, G.sino_elems() * sizeof(double)) == hipSuccess &&
         hipMemset(p->counter, 0, scg::kCounterBytes) == hipSuccess && hipDeviceSynchronize() == hipSuccess;
    if (!ok) {
        scg_plan_destroy(p);
        return SCG_EDEVICE;
    }
    int rc = build_proj_tables(p, pa);
    if (rc != SCG_OK) {
        scg_plan_destroy(p);
        return rc;
    }
    *out = p;
    return SCG_OK;
}

void scg_plan_destroy(scg_plan *p)
{
    if (p == nullptr) return;
    Device dg(p->device);
    (void)hipFree(p->pang);
    (void)hipFree(p->bang);
    (void)hipFree(p->pgroups);
    (void)hipFree(p->pwin);
    for (int i = 0; i < 2; ++i) {
        (void)hipFree(p->xs[i]);
        (void)hipFree(p->rpad[i]);
        (void)hipFree(p->kern[i]);
    }
    (void)hipFree(p->partials);
    (void)hipFree(p->counter);
    (void)hipFree(p->tvbuf);
    prof_drain(p);
    for (hipEvent_t e : p->ev_free) (void)hipEventDestroy(e);
    for (hipEvent_t e : p->prof_open)
        if (e != nullptr) (void)hipEventDestroy(e);
    delete p;
}

int scg_profile(scg_plan *plan, uint32_t class_mask)
{
    if (plan == nullptr) return SCG_EINVAL;
    Device dg(plan->device);
    prof_drain(plan);
    for (int c = 0; c < SCG_KC_COUNT; ++c) {
        plan->prof_count[c] = 0;
        plan->prof_ms[c] = 0.0;
        plan->prof_tail_count[c] = 0;
        plan->prof_tail_ms[c] = 0.0;
        if (plan->prof_open[c] != nullptr) plan->ev_free.push_back(plan->prof_open[c]);
        plan->prof_open[c] = nullptr;
    }
    plan->prof_mask = class_mask & ((1u << SCG_KC_COUNT) - 1);
    return SCG_OK;
}

int scg_profile_read(scg_plan *plan, scg_kernel_time *out)
{
    if (plan == nullptr || out == nullptr) return SCG_EINVAL;
    Device dg(plan->device);
    prof_drain(plan);
    for (int c = 0; c < SCG_KC_COUNT; ++c) {
        out[c].launches = plan->prof_count[c];
        out[c].total_ms = plan->prof_ms[c];
        out[c].tail_launches = plan->prof_tail_count[c];
        out[c].tail_ms = plan->prof_tail_ms[c];
    }
    return SCG_OK;
}

int scg_workspace_bytes(const scg_plan *plan, const scg_params *params, size_t *bytes)
{
    if (plan == nullptr || bytes == nullptr) return SCG_EINVAL;
    int rc = check_params(params);
    if (rc) return rc;
    const size_t esz = params->prec == SCG_F64 ? sizeof(double) : sizeof(float);
    *bytes = layout(plan->G, esz, params->max_iter).total;
    return SCG_OK;
}

int scg_project(scg_plan *plan, int prec, const void *x, void *y, void *stream)
{
    if (plan == nullptr || x == nullptr || y == nullptr) return SCG_EINVAL;
    if (prec != SCG_F32 && prec != SCG_F64) return SCG_EINVAL;
    Device dg(plan->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Geo &G = plan->G;
    if (prec == SCG_F32) {
        float *xs = static_cast<float *>(plan->xs[0]);
        const float *xf = static_cast<const float *>(x);
        scg::launch_stage<float>(xf, xs, G, nullptr, s);
        scg::launch_project<float>(xf, xs, G, plan->ptab, nullptr, 0, static_cast<float *>(y),
                                   G.nb, 0, nullptr, nullptr, nullptr, scg::kRedNone, nullptr,
                                   plan->tune[0].project_groups, s);
    } else {
        double *xs = static_cast<double *>(plan->xs[1]);
        const double *xd = static_cast<const double *>(x);
        scg::launch_stage<double>(xd, xs, G, nullptr, s);
        scg::launch_project<double>(xd, xs, G, plan->ptab, nullptr, 0, static_cast<double *>(y),
                                    G.nb, 0, nullptr, nullptr, nullptr, scg::kRedNone, nullptr,
                                    plan->tune[1].project_groups, s);
    }
    return hip_status(hipGetLastError());
}

int scg_backproject(scg_plan *plan, int prec, const void *y, void *x, void *stream)
{
    if (plan == nullptr || x == nullptr || y == nullptr) return SCG_EINVAL;
    if (prec != SCG_F32 && prec != SCG_F64) return SCG_EINVAL;
    Device dg(plan->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Geo &G = plan->G;
    if (prec == SCG_F32) {
        float *rp = static_cast<float *>(plan->rpad[0]);
        scg::launch_pad_sino<float>(static_cast<const float *>(y), rp, G, s);
        scg::launch_backproject<float>(rp, nullptr, G, plan->bang, static_cast<float *>(x), nullptr,
                                       nullptr, nullptr, nullptr, nullptr, scg::kRedNone,
                                       plan->tune[0].backproject_split, s);
    } else {
        double *rp = static_cast<double *>(plan->rpad[1]);
        scg::launch_pad_sino<double>(static_cast<const double *>(y), rp, G, s);
        scg::launch_backproject<double>(rp, nullptr, G, plan->bang, static_cast<double *>(x),
                                        nullptr, nullptr, nullptr, nullptr, nullptr, scg::kRedNone,
                                        plan->tune[1].backproject_split, s);
    }
    return hip_status(hipGetLastError());
}

int scg_plan_get_tuning(const scg_plan *plan, int prec, scg_tuning *out)
{
    if (plan == nullptr || out == nullptr || (prec != SCG_F32 && prec != SCG_F64))
        return SCG_EINVAL;
    *out = plan->tune[prec == SCG_F32 ? 0 : 1];
    return SCG_OK;
}

int scg_plan_set_tuning(scg_plan *plan, int prec, const scg_tuning *in)
{
    if (plan == nullptr || in == nullptr || (prec != SCG_F32 && prec != SCG_F64) ||
        !tuning_valid(*in))
        return SCG_EINVAL;
    plan->tune[prec == SCG_F32 ? 0 : 1] = *in;
    return SCG_OK;
}

int scg_plan_autotune(scg_plan *plan, int prec, void *stream, scg_tuning *chosen)
{
    if (plan == nullptr || (prec != SCG_F32 && prec != SCG_F64)) return SCG_EINVAL;
    Device dg(plan->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    return prec == SCG_F32 ? autotune_impl<float>(plan, s, chosen)
                           : autotune_impl<double>(plan, s, chosen);
}

int scg_tv(scg_plan *plan, int prec, const void *x, double kappa, void *s_out, double *tv_host,
           void *stream)
{
    if (plan == nullptr || x == nullptr || tv_host == nullptr) return SCG_EINVAL;
    if (prec != SCG_F32 && prec != SCG_F64) return SCG_EINVAL;
    if (!(kappa >= 0.0)) return SCG_EINVAL;
    Device dg(plan->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Geo &G = plan->G;
    if (prec == SCG_F32)
        scg::launch_tv<float>(static_cast<const float *>(x), static_cast<float *>(s_out), G, kappa,
                              plan->partials, plan->counter, plan->tvbuf, s);
    else
        scg::launch_tv<double>(static_cast<const double *>(x), static_cast<double *>(s_out), G,
                               kappa, plan->partials, plan->counter, plan->tvbuf, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(tv_host, plan->tvbuf, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return SCG_OK;
}

int scg_filter(scg_plan *plan, int prec, double mu, const void *r, void *out, void *stream)
{
    if (plan == nullptr || r == nullptr || out == nullptr) return SCG_EINVAL;
    if (prec != SCG_F32 && prec != SCG_F64) return SCG_EINVAL;
    Device dg(plan->device);
    int rc = ensure_filter(plan, mu);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Geo &G = plan->G;
    if (prec == SCG_F32) {
        float *rp = static_cast<float *>(plan->rpad[0]);
        scg::launch_pad_sino<float>(static_cast<const float *>(r), rp, G, s);
        scg::launch_filter<float>(rp, static_cast<float *>(out),
                                  static_cast<const float *>(plan->kern[0]), G, 0, nullptr, s);
    } else {
        double *rp = static_cast<double *>(plan->rpad[1]);
        scg::launch_pad_sino<double>(static_cast<const double *>(r), rp, G, s);
        scg::launch_filter<double>(rp, static_cast<double *>(out),
                                   static_cast<const double *>(plan->kern[1]), G, 0, nullptr, s);
    }
    return hip_status(hipGetLastError());
}

int scg_solve(scg_plan *plan, const scg_params *params, const void *y, const void *x0,
              void *x_out, void *ws, size_t ws_bytes, scg_report *rep, scg_trace_entry *trace,
              int32_t trace_cap, const int32_t *forced, int32_t forced_len, void *stream)
{
    if (plan == nullptr || y == nullptr || x_out == nullptr || ws == nullptr) return SCG_EINVAL;
    int rc = check_params(params);
    if (rc) return rc;
    size_t need = 0;
    scg_workspace_bytes(plan, params, &need);
    if (ws_bytes < need) return SCG_ENOMEM;
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return SCG_EINVAL;
    Device dg(plan->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (params->prec == SCG_F32)
        rc = solve_impl<float>(plan, params, y, x0, x_out, static_cast<char *>(ws), rep, trace,
                               trace_cap, forced, forced_len, s);
    else
        rc = solve_impl<double>(plan, params, y, x0, x_out, static_cast<char *>(ws), rep, trace,
                                trace_cap, forced, forced_len, s);
    if (hipGetLastError() != hipSuccess) return SCG_EDEVICE;
    return rc;
}

}  // extern "C"
