// Solver driver of libscg. A solve lives in one workspace on the device: its
// vectors, its FP64 scalars and control state, and a descriptor the kernels
// read. Every iteration is a fixed sequence of phase launches, each followed
// where needed by a finisher that turns block partial sums into the
// algorithm's scalars; kernels return at once when their solve's `done` flag
// is set, so the host enqueues iterations without reading anything back and
// the iteration count is decided on the device.
//
// scg_solve runs one solve, enqueuing iterations in growing chunks and
// reading the flag between chunks. The batch engine (scg_batch_*) keeps many
// solves resident in one device arena and advances all of them with one
// launch per phase (solves grouped by precision, variant and launch shape),
// the whole iteration captured once as a HIP graph per set of solves;
// finished solves retire between steps and new ones are admitted as slots
// and arena memory free up.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "plan.h"

// Workspace of scg_solve_static: a file-scope device array, one per device
// the library runs on, held until the process ends. Host code never passes
// its name to a kernel or a copy (on the host it only stands for the
// symbol): the device address comes from hipGetSymbolAddress, taken once per
// device with that device current (static_workspace below).
constexpr size_t kStaticWsBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticWsBytes];

using scg::BlkMap;
using scg::Solve;

namespace scg {

namespace {

// Workspace layout of one solve.
struct Layout {
    size_t x, xh, p, g, h, s, z, r, q, rt, xs, pt, partials, partials2, partials3, state, forced,
        trace, tv,
        gtab, desc, total;
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
    L.partials = take(kMaxPartials * sizeof(double));
    L.partials2 = take(kMaxPartials * sizeof(double));
    L.partials3 = take(kMaxT32Blocks * sizeof(double));
    L.state = take(sizeof(DevState));
    L.forced = take((size_t)2 * (max_iter + 1) * sizeof(int32_t));
    L.trace = take((size_t)(max_iter + 1) * sizeof(scg_trace_entry));
    L.tv = take(sizeof(double));
    L.gtab = take(kMaxTrials * sizeof(double));
    L.desc = take(sizeof(Solve<double>));
    L.total = off;
    return L;
}

// Block kinds of the phase launches.
enum Kind { kKT32 = 0, kKXtv, kKTrA, kKTrB, kKPj, kKBp, kKBpH, kKVec, kKFilt, kKPQ, kKXR, kKinds };

template <typename T> int count_of(const Solve<T> &d, int kind)
{
    switch (kind) {
    case kKT32: return d.nb_t32;
    case kKXtv: return d.nb_xtv;
    case kKTrA: return d.nb_trA;
    case kKTrB: return d.nb_trB;
    case kKPj: return d.nb_pj;
    case kKBp: return d.nb_bp;
    case kKBpH: return d.nb_bph;
    case kKVec: return d.nb_vec;
    case kKFilt: return (d.G.na + 1) / 2;
    case kKPQ: return d.nb_t32 + d.nb_sv;
    case kKXR: return d.nb_vec + d.nb_sv;
    default: return 0;
    }
}

inline bool restarted(int variant) { return variant == SCG_S_CG_K || variant == SCG_S_PCG_K; }
inline bool unsuperiorized(int variant) { return variant == SCG_CG || variant == SCG_PCG; }
inline bool filtered(int variant)
{
    return variant == SCG_S_PCG || variant == SCG_PCG || variant == SCG_S_PCG_K;
}

// A set of solves advanced together: same precision, variant and launch shapes.
template <typename T> struct Group {
    int ns = 0;
    int variant = SCG_S_CG;
    scg_tuning tune{4, 2, 8, 0, 0};
    int max_nb = 1;
    int restart_k = 2;                      // S-CG-K
    const Solve<T> *S = nullptr;            // device descriptors
    const BlkMap *map[kKinds] = {};         // device block maps (null for a single solve)
    int nblk[kKinds] = {};
    bool any_trB = false;
    scg_plan *prof = nullptr;               // event timing (single solves only)
};

struct Prof {
    scg_plan *p;
    int cls;
    hipStream_t s;
    Prof(scg_plan *p_, int cls_, hipStream_t s_) : p(p_), cls(cls_), s(s_)
    {
        if (p) prof_mark(p, cls, s, true);
    }
    ~Prof()
    {
        if (p) prof_mark(p, cls, s, false);
    }
};

template <typename T> struct Enq {
    const Group<T> &g;
    hipStream_t s;
    const BlkMap *m(int k) const { return g.map[k]; }
    int n(int k) const { return g.nblk[k]; }
    void stage(int phase) const
    {
        Prof t(g.prof, SCG_KC_STAGE, s);
        launch_b_stage<T>(g.S, m(kKT32), n(kKT32), phase, s);
    }
    void project(int phase) const
    {
        Prof t(g.prof, SCG_KC_PROJECT, s);
        launch_b_project<T>(g.S, m(kKPj), n(kKPj), phase, g.tune.project_groups,
                            g.tune.project_angles, g.tune.project_mirror, g.tune.swizzle, s);
    }
    // The filtered variants' two-sinogram phase and their z' = A^T r~ with
    // its dot run on every tile (no mirrored form; their partials are laid
    // out by tile); their h = A^T q, which stores no partials, and every
    // phase of the other variants follow the shape.
    void backproject(int phase, int dot) const
    {
        Prof t(g.prof, SCG_KC_BACKPROJECT, s);
        const bool fil = filtered(g.variant);
        const int kind = fil && phase == kBpH ? kKBpH : kKBp;
        const int mir = (!fil || phase == kBpH) ? g.tune.backproject_mirror : 0;
        launch_b_backproject<T>(g.S, m(kind), n(kind), phase, dot, g.tune.backproject_split, mir,
                                g.tune.swizzle, s);
    }
    void finish(int fin, int a0 = 0, int a1 = 0) const
    {
        Prof t(g.prof, SCG_KC_CONTROL, s);
        launch_finish<T>(g.S, g.ns, fin, a0, a1, s);
    }
    // A single solve's launches form the scalars they need from the previous
    // launch's partials in every block; a batch of many solves has a
    // finisher form them once per solve (the same sums, the same bits), so
    // that its blocks do not each reread the partials.
    bool given() const { return g.ns > 1; }
    void p_update(int rule, int init) const
    {
        // S-CG, S-CG-CD, S-PCG after the initial step: the update records beta
        // itself and g'^T p' is recorded with the next step's opening (by the
        // TV pass's first block in a single solve, by kFinXtv in a batch), so
        // no finisher of its own follows
        const bool rec = !init && rule <= 2 &&
                         (g.variant == SCG_S_CG || g.variant == SCG_S_CG_CD ||
                          g.variant == SCG_S_PCG);
        if (rec && given()) finish(kFinStepScalars, rule);
        {
            Prof t(g.prof, SCG_KC_VECTOR, s);
            launch_b_p_update<T>(g.S, m(kKT32), n(kKT32), rule, init, rec ? 1 : 0,
                                 rec && given() ? 1 : 0, s);
        }
        if (!rec) finish(kFinPUpdate, rule, init);
    }
    void xtv() const
    {
        const bool local = g.variant == SCG_S_CG || g.variant == SCG_S_CG_CD ||
                           g.variant == SCG_S_PCG;
        if (local && given()) finish(kFinAlpha);
        Prof t(g.prof, SCG_KC_TV, s);
        launch_b_xtv<T>(g.S, m(kKXtv), n(kKXtv), local && given() ? 1 : 0, s);
    }
    void pq_update() const
    {
        {
            Prof t(g.prof, SCG_KC_VECTOR, s);
            launch_b_pq_update<T>(g.S, m(kKPQ), n(kKPQ), s);
        }
        finish(kFinPQ);
    }
    void filter() const
    {
        Prof t(g.prof, SCG_KC_FILTER, s);
        launch_b_filter<T>(g.S, m(kKFilt), n(kKFilt), g.max_nb, s);
    }
    // PCG-STEP after alpha: h = A^T q, x, g and r updated; then (unless the
    // step ends a PCG-K pass) z' = A^T F r', delta' = g'^T z', p' = -z' + beta p
    void pcg_step(int in_pass, bool last) const
    {
        backproject(kBpH, 0);
        {
            Prof t(g.prof, SCG_KC_VECTOR, s);
            launch_b_x_update_pcg<T>(g.S, m(kKXR), n(kKXR), s);
        }
        if (last) return;
        filter();
        backproject(kBpZ, 1);
        finish(kFinDeltaPCG, in_pass);
        p_update(4, 0);
    }
    // z0 = M g0 with g0 (from r0 in r): delta0 = g0^T z0, p0 = -z0
    void pcg_start() const
    {
        filter();
        backproject(kBpGZ, 3);
        finish(kFinDotGG);
        p_update(4, 1);
    }
};

// The launch shapes a solve runs with: the plan's. (The filtered variants'
// two-sinogram phase and their single-sinogram phase with a dot have no
// mirrored form and keep every tile; their h = A^T q phase follows the
// shape; see Enq::backproject.)
inline scg_tuning solve_tuning(scg_tuning t, int /*variant*/) { return t; }

// Initial step. S- variants (steps 1-6 of the algorithms): x_{1/2} = x0, g0
// (and z0), p0, h0 and alpha; x1 = x0 + alpha p0 and k = 1 are formed by the
// first loop launch, which closes every step. CG: g0 = A^T(A x0 - y), p0 =
// -g0, delta0 = ||g0||^2.
template <typename T> void enqueue_init(const Group<T> &g, hipStream_t s)
{
    const Enq<T> e{g, s};
    if (restarted(g.variant)) {
        // S-CG-K, S-PCG-K: x_{-1/2} = x_0 = x0 and the loop test f(x0) > eps
        e.stage(kStageX);
        e.project(kPjResX);
        e.finish(kFinResidual);
        return;
    }
    if (g.variant == SCG_CG) {
        e.stage(kStageX);
        e.project(kPjResX);
        e.finish(kFinResidual);
        e.backproject(kBpG, 2);
        e.finish(kFinDotGG);
        e.p_update(3, 1);
        return;
    }
    if (g.variant == SCG_PCG) {
        // r0 = A x0 - y, g0 = A^T r0, z0 = A^T F r0, p0 = -z0
        e.stage(kStageX);
        e.project(kPjResX);
        e.finish(kFinResidual);
        e.pcg_start();
        return;
    }
    e.stage(kStageXh);
    e.project(kPjResXh);
    e.finish(kFinResidual);
    if (g.variant == SCG_S_PCG) {
        e.filter();
        e.backproject(kBpGZ, 0);
        e.p_update(2, 1);
    } else {
        e.backproject(kBpG, 0);
        e.p_update(0, 1);
    }
    e.project(kPjQ);
    // alpha: the first TV pass forms it (S-CG, S-CG-CD, S-PCG)
    if (g.variant == SCG_S_CG_3OP) e.finish(kFinNormQ);
    if (g.variant != SCG_S_CG_CD && g.variant != SCG_S_CG_3OP) e.backproject(kBpH, 0);
}

// The rest of an S- iteration after the trial search: x_{k+1/2}, then the
// step from it.
template <typename T> void enqueue_after_search(const Group<T> &g, hipStream_t s)
{
    const Enq<T> e{g, s};
    {
        Prof t(g.prof, SCG_KC_VECTOR, s);
        launch_b_perturb<T>(g.S, e.m(kKT32), e.n(kKT32), s);
    }
    // S-CG, S-CG-CD, S-PCG: the direction update takes the step's loop test
    // (no finisher); the others test in a finisher
    const bool fused_stop = g.variant == SCG_S_CG || g.variant == SCG_S_CG_CD ||
                            g.variant == SCG_S_PCG;
    e.project(fused_stop ? kPjResXhF : kPjResXh);
    if (!fused_stop) e.finish(kFinResidualStep);
    if (g.variant == SCG_S_CG_K) {
        // CG-K from x_{k+1/2} (copied into x by the perturbation): g0 =
        // A^T r (r formed above), p0 = -g0, delta0 = ||g0||^2, then K
        // CG-STEPs; the direction update after the last one is not needed
        e.backproject(kBpG, 2);
        e.finish(kFinDotGG);
        e.p_update(3, 1);
        for (int j = 0; j < g.restart_k; ++j) {
            e.project(kPjQ);
            e.finish(kFinNormQCG, 1);
            e.backproject(kBpH, 0);
            {
                Prof t(g.prof, SCG_KC_VECTOR, s);
                launch_b_x_update_cg<T>(g.S, e.m(kKVec), e.n(kKVec), s);
            }
            e.finish(kFinXUpdateCG, 1);
            if (j + 1 < g.restart_k) e.p_update(3, 0);
        }
        return;
    }
    if (g.variant == SCG_S_PCG_K) {
        // PCG-K from x_{k+1/2}: r0 (formed above), g0, z0, delta0, p0, then K
        // PCG-STEPs; the direction update after the last one is not needed
        e.pcg_start();
        for (int j = 0; j < g.restart_k; ++j) {
            e.project(kPjQ);
            e.finish(kFinNormQCG, 1);
            e.pcg_step(1, j + 1 == g.restart_k);
        }
        return;
    }
    if (g.variant == SCG_S_CG_3OP) {
        // CG-PR-STEP with q = A p carried by linearity: g' = A^T r (and its
        // transpose), u = A g' with u^T q = g'^T h, then p' and q' = -u + beta q
        e.backproject(kBpGT, 0);
        e.project(kPjU);
        e.finish(kFinDotUQ);
        e.pq_update();
        return;
    }
    // beta comes from the backprojection's dot inside the direction update,
    // alpha from ||A p'||^2 inside the next TV pass; their finishers record
    // them (no finisher launch of their own)
    if (g.variant == SCG_S_PCG) {
        e.filter();
        e.backproject(kBpGZ, 1);
        e.p_update(2, 0);
    } else if (g.variant == SCG_S_CG_CD) {
        e.backproject(kBpG, 2);
        e.p_update(1, 0);
    } else {
        e.backproject(kBpG, 1);
        e.p_update(0, 0);
    }
    e.project(kPjQ);
    if (g.variant != SCG_S_CG_CD) e.backproject(kBpH, 0);
}

// Head of a loop iteration of an S- variant: the TV pass that closes the
// previous step (x_{k+1} = x_{k+1/2} + alpha p) and opens this one, and the
// first trial launch of perturbed(x_k). suspend_tag > 0: the second trial
// launch is left out of this iteration, and a search the first leaves open
// suspends the solve under that tag.
template <typename T> void enqueue_head(const Group<T> &g, hipStream_t s, int suspend_tag)
{
    const Enq<T> e{g, s};
    const int tag = g.any_trB ? suspend_tag : 0;
    e.xtv();
    if (!e.given()) {
        // a single solve: the trial launch forms the opening's scalars
        // itself and one finisher opens the step and decides its trials
        {
            Prof t(g.prof, SCG_KC_TRIALS, s);
            launch_b_trials<T>(g.S, e.m(kKTrA), e.n(kKTrA), 0, 1, s);
        }
        e.finish(kFinOpenTrials, 0, tag);
        return;
    }
    e.finish(kFinXtv);
    {
        Prof t(g.prof, SCG_KC_TRIALS, s);
        launch_b_trials<T>(g.S, e.m(kKTrA), e.n(kKTrA), 0, 0, s);
    }
    e.finish(kFinTrials, 0, tag);
}

// The rest of the iteration after the head: the second trial launch (with_b),
// x_{k+1/2}, then the step (CG-PR-STEP / CG-CD-STEP / PCG-PR-STEP, or the
// CG-K / PCG-K pass) from x_{k+1/2}.
template <typename T> void enqueue_tail(const Group<T> &g, hipStream_t s, bool with_b)
{
    const Enq<T> e{g, s};
    if (g.any_trB && with_b) {
        // the second trial launch and its finisher return at once where the
        // first launch accepted a step
        {
            Prof t(g.prof, SCG_KC_TRIALS, s);
            launch_b_trials<T>(g.S, e.m(kKTrB), e.n(kKTrB), kTrialsPerPass, 0, s);
        }
        e.finish(kFinTrials, kTrialsPerPass);
    }
    enqueue_after_search(g, s);
}

// One loop iteration. S- variants: close the previous step (x_{k+1} =
// x_{k+1/2} + alpha p), perturbed(x_k) (TV subgradient, trials, x_{k+1/2}),
// then the step (CG-PR-STEP / CG-CD-STEP / PCG-PR-STEP) from x_{k+1/2}.
// CG: the cap test, then CG-STEP.
template <typename T> void enqueue_iteration(const Group<T> &g, hipStream_t s)
{
    const Enq<T> e{g, s};
    if (g.variant == SCG_CG) {
        e.finish(kFinCGCap);
        e.project(kPjQ);
        e.finish(kFinNormQCG);
        e.backproject(kBpH, 0);
        {
            Prof t(g.prof, SCG_KC_VECTOR, s);
            launch_b_x_update_cg<T>(g.S, e.m(kKVec), e.n(kKVec), s);
        }
        e.finish(kFinXUpdateCG);
        e.p_update(3, 0);
        e.stage(kStageX);
        e.project(kPjResX);
        e.finish(kFinResidual);
        return;
    }
    if (g.variant == SCG_PCG) {
        // cap test, PCG-STEP (recursive g and r), then f(x) explicitly
        e.finish(kFinCGCap);
        e.project(kPjQ);
        e.finish(kFinNormQCG);
        e.pcg_step(0, false);
        e.stage(kStageX);
        e.project(kPjResX);
        e.finish(kFinResidual);
        return;
    }
    enqueue_head(g, s, 0);
    enqueue_tail(g, s, true);
}

// Output image (x_{k+1/2} of the S- variants, x of CG) and its TV.
template <typename T> void enqueue_final(const Group<T> &g, hipStream_t s)
{
    launch_b_copy_out<T>(g.S, g.map[kKVec], g.nblk[kKVec], !unsuperiorized(g.variant), s);
    launch_b_tv<T>(g.S, g.map[kKVec], g.nblk[kKVec], s);
    launch_finish<T>(g.S, g.ns, kFinTV, 0, 0, s);
}

// Sets up one solve in workspace `ws`: zero pads, the start image, the
// device state and the descriptor (host copy in *d, device copy in the
// workspace). Enqueued on s; host arrays are staged before this returns.
// Host staging of the uploads of prepare_solve; it must stay valid until the
// stream has passed them.
template <typename T> struct Staging {
    DevState st;
    Solve<T> desc;
};

template <typename T>
int prepare_solve(scg_plan *plan, const scg_params *pr, const scg_tuning &tune, char *ws,
                  const void *y_, const void *x0_, void *xout_, int trace_cap,
                  const int32_t *forced_host, int forced_len, Staging<T> *stage, hipStream_t s,
                  bool defer = false)
{
    const Geo &G = plan->G;
    const size_t J = G.img_elems(), S = G.sino_elems();
    const Layout L = layout(G, sizeof(T), pr->max_iter);
    auto at = [&](size_t off) { return reinterpret_cast<T *>(ws + off); };
    Solve<T> &h = stage->desc;
    h = Solve<T>{};
    h.G = G;
    h.P = proj_tables(plan, tune);
    h.bang = plan->bang;
    h.border = plan->border;
    h.ftab = static_cast<const T *>(plan->ftab[prec_index<T>()]);
    h.y = static_cast<const T *>(y_);
    h.x = at(L.x);
    h.xh = at(L.xh);
    h.p = at(L.p);
    h.g = at(L.g);
    h.h = at(L.h);
    h.s = at(L.s);
    h.z = at(L.z);
    h.r = at(L.r);
    h.q = at(L.q);
    h.rt = at(L.rt);
    h.xs = at(L.xs);
    h.pt = at(L.pt);
    h.xout = static_cast<T *>(xout_);
    h.partials = reinterpret_cast<double *>(ws + L.partials);
    h.partials2 = reinterpret_cast<double *>(ws + L.partials2);
    h.partials3 = reinterpret_cast<double *>(ws + L.partials3);
    h.gtab = reinterpret_cast<double *>(ws + L.gtab);
    h.tvd = reinterpret_cast<double *>(ws + L.tv);
    h.st = reinterpret_cast<DevState *>(ws + L.state);
    h.trace = reinterpret_cast<scg_trace_entry *>(ws + L.trace);
    int32_t *forced = reinterpret_cast<int32_t *>(ws + L.forced);
    h.nb_xtv = blocks_xtv(G);
    h.nb_t32 = blocks_t32(G);
    h.nb_vec = blocks_vec(J);
    h.nb_pj = h.P.n_chunks * h.P.n_groups;
    h.nb_bp = blocks_bp(G, tune.backproject_mirror != 0 && !filtered(pr->variant));
    h.nb_bph = blocks_bp(G, tune.backproject_mirror != 0);
    h.nb_sv = blocks_sv(G);
    h.trB_chunks = (std::max(pr->max_trials - kTrialsPerPass, 0) + kTrialsPerPass - 1) /
                   kTrialsPerPass;
    h.nb_trA = blocks_trials(G, 1);
    h.nb_trB = h.trB_chunks > 0 ? blocks_trials(G, h.trB_chunks) : 0;

    // Pads of the staged image and of the sinograms must be zero (a batch
    // admission does this with the device set-up below: see Admit).
    if (!defer) {
        launch_fill<T>(h.r, S, T(0), s);
        launch_fill<T>(h.q, S, T(0), s);
        launch_fill<T>(h.rt, S, T(0), s);
        launch_fill<T>(h.xs, G.staged_elems(), T(0), s);
    }

    const bool is_cg = unsuperiorized(pr->variant);
    DevState &hs = stage->st;
    hs = DevState{};
    hs.eps = pr->eps;
    hs.gamma0 = pr->gamma0;
    hs.a = pr->a;
    hs.kappa = pr->tv_kappa;
    hs.max_iter = pr->max_iter;
    hs.max_trials = pr->max_trials;
    hs.variant = pr->variant;
    hs.flags = (int)pr->flags;
    const bool is_k = restarted(pr->variant);
    hs.k = 0;
    // the initial step of S-CG, S-CG-CD and S-PCG is open until the first
    // loop launch closes it (and is not counted); S-CG-K has none
    hs.steps = (is_cg || is_k) ? 0 : -1;
    hs.open = (is_cg || is_k) ? 0 : 1;
    hs.kofs = is_k ? 1 : 0;
    hs.restart_k = pr->restart_k;
    hs.accepted = -1;
    hs.is_f32 = sizeof(T) == 4 ? 1 : 0;
    hs.trace_cap = std::min<int32_t>(std::max(trace_cap, 0), pr->max_iter + 1);
    const int nf = forced_host ? std::min<int32_t>(std::max<int32_t>(forced_len, 0),
                                                   pr->max_iter + 1)
                               : 0;
    hs.forced_len = nf;
    h.forced = nf > 0 ? forced : nullptr;
    if (defer) return SCG_OK;
    HIP_TRY(hipMemcpyAsync(h.st, &hs, sizeof(DevState), hipMemcpyHostToDevice, s));
    if (nf > 0)
        HIP_TRY(hipMemcpyAsync(forced, forced_host, (size_t)2 * nf * sizeof(int32_t),
                               hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(ws + L.desc, &h, sizeof(h), hipMemcpyHostToDevice, s));

    // x_{1/2} = x0 (S-CG, S-CG-CD, S-PCG) or x_0 (CG, PCG, S-CG-K, S-PCG-K).
    // S-CG-K and S-PCG-K also start x_{-1/2} = x0 in x_{k+1/2}'s buffer: the
    // output when f(x0) <= eps ends the loop before the first pass.
    T *x_start = (is_cg || is_k) ? h.x : h.xh;
    if (x0_ != nullptr) launch_copy<T>(x_start, static_cast<const T *>(x0_), J, nullptr, s);
    else launch_fill<T>(x_start, J, T(0), s);
    if (is_k) launch_copy<T>(h.xh, h.x, J, nullptr, s);
    return SCG_OK;
}

template <typename T>
Group<T> single_group(const scg_params *pr, const scg_tuning &tune, const Solve<T> &h, char *ws)
{
    Group<T> g;
    g.ns = 1;
    g.variant = pr->variant;
    g.tune = tune;
    g.max_nb = h.G.nb;
    g.restart_k = pr->restart_k;
    g.S = reinterpret_cast<const Solve<T> *>(ws + layout(h.G, sizeof(T), pr->max_iter).desc);
    for (int k = 0; k < kKinds; ++k) g.nblk[k] = count_of(h, k);
    g.any_trB = h.trB_chunks > 0;
    return g;
}

template <typename T>
int solve_impl(scg_plan *plan, const scg_params *pr, const void *y, const void *x0, void *xout,
               char *ws, scg_report *rep, scg_trace_entry *trace_host, int32_t trace_cap,
               const int32_t *forced_host, int32_t forced_len, hipStream_t st0,
               bool timed = true)
{
    if (filtered(pr->variant)) {
        int rc = ensure_filter(plan, pr->precond_mu, pr->prec);
        if (rc) return rc;
    }
    // the state and descriptor images are uploaded from the plan's pinned
    // host words (a DMA of pinned memory, no staged pageable copy)
    static_assert(kPinnedStagingOffset + sizeof(Staging<double>) <= kHostPinnedBytes,
                  "pinned staging");
    Staging<T> &stage = *new (static_cast<char *>(plan->host_pinned) + kPinnedStagingOffset)
        Staging<T>{};
    const int cap = trace_host != nullptr ? trace_cap : pr->max_iter + 1;
    const scg_tuning tune = solve_tuning(plan->tune[prec_index<T>()], pr->variant);
    int rc = prepare_solve<T>(plan, pr, tune, ws, y, x0, xout, cap, forced_host, forced_len,
                              &stage, st0);
    if (rc) return rc;
    const Solve<T> &h = stage.desc;
    Group<T> g = single_group<T>(pr, tune, h, ws);
    // kernel timing takes HIP events from the plan (created on first use)
    g.prof = timed ? plan : nullptr;

    plan->prof_iter = 0;
    enqueue_init(g, st0);
    // loop: chunks of iterations (4, 8, 16, 16, ...) queued behind the
    // initial step without waiting for it; the device decides when to stop,
    // and launches queued after the stop return at once. The state comes
    // back through the plan's pinned host words after each chunk.
    //
    // Trial launches: once the global counter ell has grown, a step's search
    // rarely outlives the first trial launch. The first chunk takes both
    // launches of every step; later chunks take the first only, and a step
    // whose search goes on past it suspends the solve (kFinTrials). The host
    // then clears the flag, enqueues that step's remainder with the second
    // launch and gives the next chunk both launches; after a second
    // suspension every chunk has both.
    static_assert(sizeof(DevState) + 2 * sizeof(double) <= kHostPinnedBytes, "pinned words");
    auto *fs_h = reinterpret_cast<DevState *>(static_cast<char *>(plan->host_pinned) + 64);
    auto *tv_h = reinterpret_cast<double *>(static_cast<char *>(plan->host_pinned) + 64 +
                                            ((sizeof(DevState) + 7) / 8) * 8);
    const bool may_suspend = g.any_trB && !unsuperiorized(pr->variant);
    int suspensions = 0;
    bool both = true;                // the next chunk takes both trial launches
    std::vector<size_t> tail_mark;   // timing records before each iteration's tail
    long issued = 0;
    int chunk = 4;
    for (;;) {
        const bool split = may_suspend && !both;
        tail_mark.assign(chunk, 0);
        for (int c = 0; c < chunk; ++c) {
            plan->prof_iter = (int)std::min<long>(issued + c + 1, INT_MAX - 1);
            if (split) {
                enqueue_head(g, st0, c + 1);
                tail_mark[c] = plan->prof_pending.size();
                enqueue_tail(g, st0, false);
            } else {
                enqueue_iteration(g, st0);
            }
        }
        const long first = issued + 1;
        issued += chunk;
        chunk = std::min(chunk * 2, 16);
        both = suspensions >= 2;
        HIP_TRY(hipMemcpyAsync(fs_h, h.st, sizeof(DevState), hipMemcpyDeviceToHost, st0));
        HIP_TRY(hipStreamSynchronize(st0));
        DevState cs;
        std::memcpy(&cs, fs_h, sizeof cs);
        if (split && cs.done == kSuspended) {
            const int c = cs.susp_tag - 1;
            if (c < 0 || c >= (int)tail_mark.size()) return SCG_EDEVICE;
            // the launches after the suspending step's head returned at once
            if (g.prof) prof_to_tail(plan, tail_mark[c]);
            HIP_TRY(hipMemsetAsync(&h.st->done, 0, sizeof(int), st0));
            issued = first + c;
            plan->prof_iter = (int)std::min<long>(issued, INT_MAX - 1);
            enqueue_tail(g, st0, true);
            ++suspensions;
            both = true;
            continue;
        }
        if (cs.done || issued > (long)pr->max_iter) break;
    }
    plan->prof_iter = INT_MAX;
    g.prof = nullptr;
    enqueue_final(g, st0);

    HIP_TRY(hipMemcpyAsync(fs_h, h.st, sizeof(DevState), hipMemcpyDeviceToHost, st0));
    HIP_TRY(hipMemcpyAsync(tv_h, h.tvd, sizeof(double), hipMemcpyDeviceToHost, st0));
    if (trace_host != nullptr && trace_cap > 0) {
        const int n = std::min<int>(trace_cap, pr->max_iter + 1);
        HIP_TRY(hipMemcpyAsync(trace_host, h.trace, (size_t)n * sizeof(scg_trace_entry),
                               hipMemcpyDeviceToHost, st0));
    }
    HIP_TRY(hipStreamSynchronize(st0));
    const DevState fs = *fs_h;
    const double tv_out = *tv_h;
    prof_drain(plan, std::max(fs.steps, 0));
    plan->prof_iter = 0;
    const bool plain_k = unsuperiorized(pr->variant) || restarted(pr->variant);
    if (rep != nullptr) {
        std::memset(rep, 0, sizeof(*rep));
        rep->status = fs.done ? fs.status : SCG_ENOCONV;
        rep->k = plain_k ? fs.k : std::max(fs.k, 1);
        rep->steps = std::max(fs.steps, 0);
        rep->trials_total = fs.trials_total;
        rep->ell = fs.ell;
        rep->f_out = fs.f_half;
        rep->tv_out = tv_out;
    }
    return fs.done ? fs.status : SCG_ENOCONV;
}

}  // namespace

size_t workspace_bytes(const Geo &G, int prec, int max_iter)
{
    return layout(G, prec == SCG_F64 ? sizeof(double) : sizeof(float), max_iter).total;
}

}  // namespace scg

// ---------------------------------------------------------------------------
// Batch engine
// ---------------------------------------------------------------------------

namespace {

// First-fit allocator over one device allocation (256-byte granules).
struct Arena {
    char *base = nullptr;
    size_t size = 0, used = 0;
    std::map<size_t, size_t> free_;   // offset -> bytes
    void reset(char *b, size_t n)
    {
        base = b;
        size = n;
        used = 0;
        free_.clear();
        if (n) free_[0] = n;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = scg::align256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used += bytes;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = scg::align256(bytes);
        used -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Slot {
    uint64_t ticket = 0;
    scg_plan *plan = nullptr;
    scg_params params{};
    scg_tuning tune{};           // launch shapes fixed at admission
    size_t off = 0, bytes = 0;
    int staging = -1;            // index of the slot's pinned staging entry
    bool fresh = false;          // admitted; its set-up and initial step run at the next
                                 // rebuild, with the other new solves
    const void *x0 = nullptr;    // start image (null: zero)
    Solve<float> df{};
    Solve<double> dd{};
};

// Pinned staging entry of a slot: the uploads of its set-up.
struct StagingEntry {
    scg::Staging<float> f;
    scg::Staging<double> d;
};

}  // namespace

struct scg_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipEvent_t order_ev = nullptr;   // a caller stream's point the batch waits for
    uint32_t flags = 0;
    int max_slots = 0;
    char *arena_mem = nullptr;
    Arena arena;
    std::vector<Slot> active;
    std::map<uint64_t, scg_report> finished;
    uint64_t next_ticket = 1;
    // the current set of solves on the device
    bool dirty = true;
    char *comp = nullptr;
    size_t comp_bytes = 0;
    std::vector<scg::Group<float>> gf;
    std::vector<scg::Group<double>> gd;
    std::vector<std::vector<int>> members_f, members_d;   // slot indices per group
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // state read-back
    DevState *dstates = nullptr;
    double *dtv = nullptr;
    DevState *hstates = nullptr;   // pinned
    double *htv = nullptr;         // pinned
    char *fin_dev = nullptr;       // descriptors and maps of retiring solves
    size_t fin_bytes = 0;
    StagingEntry *staging = nullptr;   // pinned, one entry per slot
    std::vector<int> staging_free;
    scg_batch_stats stats{};
};

namespace {

template <typename T> scg::Staging<T> &staging_of(StagingEntry &e);
template <> scg::Staging<float> &staging_of<float>(StagingEntry &e) { return e.f; }
template <> scg::Staging<double> &staging_of<double>(StagingEntry &e) { return e.d; }

template <typename T> Solve<T> &desc_of(Slot &s);
template <> Solve<float> &desc_of<float>(Slot &s) { return s.df; }
template <> Solve<double> &desc_of<double>(Slot &s) { return s.dd; }

// Host image of a set of groups: descriptors and block maps, packed for one
// upload; device pointers are assigned by `place`.
struct Packer {
    std::vector<char> bytes;
    template <typename V> size_t put(const std::vector<V> &v)
    {
        const size_t off = scg::align256(bytes.size());
        bytes.resize(off + v.size() * sizeof(V));
        if (!v.empty()) std::memcpy(bytes.data() + off, v.data(), v.size() * sizeof(V));
        return off;
    }
};

template <typename T> struct GroupImage {
    scg::Group<T> g;
    size_t desc_off = 0;
    size_t map_off[scg::kKinds] = {};
};

template <typename T>
GroupImage<T> pack_group(Packer &pk, std::vector<Slot> &slots, const std::vector<int> &members,
                         int variant, scg_tuning tune, bool with_maps)
{
    GroupImage<T> gi;
    gi.g.restart_k = slots[members.front()].params.restart_k;
    std::vector<Solve<T>> descs;
    for (int i : members) descs.push_back(desc_of<T>(slots[i]));
    gi.g.ns = (int)descs.size();
    gi.g.variant = variant;
    gi.g.tune = tune;
    gi.desc_off = pk.put(descs);
    for (int k = 0; k < scg::kKinds; ++k) {
        std::vector<BlkMap> map;
        for (int si = 0; si < (int)descs.size(); ++si) {
            const int c = scg::count_of(descs[si], k);
            for (int l = 0; l < c; ++l) map.push_back(BlkMap{si, l});
        }
        gi.g.nblk[k] = (int)map.size();
        gi.map_off[k] = with_maps ? pk.put(map) : 0;
    }
    for (const auto &d : descs) {
        gi.g.max_nb = std::max(gi.g.max_nb, d.G.nb);
        gi.g.any_trB = gi.g.any_trB || d.trB_chunks > 0;
    }
    return gi;
}

template <typename T> void place(GroupImage<T> &gi, char *dev)
{
    gi.g.S = reinterpret_cast<const Solve<T> *>(dev + gi.desc_off);
    for (int k = 0; k < scg::kKinds; ++k)
        gi.g.map[k] = gi.g.nblk[k] ? reinterpret_cast<const BlkMap *>(dev + gi.map_off[k])
                                   : nullptr;
}

int ensure_buf(char **buf, size_t *cap, size_t need)
{
    if (need <= *cap && *buf != nullptr) return SCG_OK;
    if (*buf) (void)hipFree(*buf);
    *buf = nullptr;
    *cap = 0;
    if (hipMalloc(buf, need) != hipSuccess) {
        *buf = nullptr;
        return SCG_ENOMEM;
    }
    *cap = need;
    return SCG_OK;
}

void drop_graph(scg_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// Groups the active solves, uploads their descriptors and block maps and
// (unless disabled) captures one iteration of all groups as a graph.
// Device set-up of the fresh solves of one precision: their state and
// descriptor images and the Admit records go into the composition upload; the
// records' device pointers are filled in once the buffer's address is known.
template <typename T> struct AdmitPack {
    std::vector<int> who;
    size_t st_off = 0, desc_off = 0, rec_off = 0;
};

template <typename T> AdmitPack<T> pack_admits(Packer &pk, scg_batch *b)
{
    AdmitPack<T> ap;
    std::vector<DevState> sts;
    std::vector<Solve<T>> ds;
    for (int i = 0; i < (int)b->active.size(); ++i) {
        Slot &sl = b->active[i];
        if (!sl.fresh || (sl.params.prec == SCG_F64) != (sizeof(T) == 8)) continue;
        ap.who.push_back(i);
        sts.push_back(staging_of<T>(b->staging[sl.staging]).st);
        ds.push_back(desc_of<T>(sl));
    }
    if (ap.who.empty()) return ap;
    ap.st_off = pk.put(sts);
    ap.desc_off = pk.put(ds);
    ap.rec_off = pk.put(std::vector<scg::Admit<T>>(ap.who.size()));
    return ap;
}

template <typename T> void fill_admits(Packer &pk, scg_batch *b, const AdmitPack<T> &ap)
{
    auto *recs = reinterpret_cast<scg::Admit<T> *>(pk.bytes.data() + ap.rec_off);
    for (size_t k = 0; k < ap.who.size(); ++k) {
        Slot &sl = b->active[ap.who[k]];
        const Solve<T> &h = desc_of<T>(sl);
        const scg::Layout L = scg::layout(h.G, sizeof(T), sl.params.max_iter);
        const bool from_x = scg::unsuperiorized(sl.params.variant) ||
                            scg::restarted(sl.params.variant);
        scg::Admit<T> a{};
        a.st_src = reinterpret_cast<const DevState *>(b->comp + ap.st_off) + k;
        a.st = h.st;
        a.desc_src = reinterpret_cast<const Solve<T> *>(b->comp + ap.desc_off) + k;
        a.desc = reinterpret_cast<Solve<T> *>(b->arena.base + sl.off + L.desc);
        a.x0 = static_cast<const T *>(sl.x0);
        a.x_start = from_x ? h.x : h.xh;
        a.xh = scg::restarted(sl.params.variant) ? h.xh : nullptr;
        a.r = h.r;
        a.q = h.q;
        a.rt = h.rt;
        a.xs = h.xs;
        a.J = (long long)h.G.img_elems();
        a.S = (long long)h.G.sino_elems();
        recs[k] = a;
    }
}

int rebuild(scg_batch *b)
{
    HIP_TRY(hipStreamSynchronize(b->stream));
    // the executable graph is kept for an in-place update below; it is not
    // launched before this rebuild has succeeded
    b->gf.clear();
    b->gd.clear();
    b->members_f.clear();
    b->members_d.clear();
    // group key: precision, variant, launch shape
    std::map<std::tuple<int, int, int, int>, std::vector<int>> keys;
    for (int i = 0; i < (int)b->active.size(); ++i) {
        const Slot &s = b->active[i];
        const int pi = s.params.prec == SCG_F64 ? 1 : 0;
        const scg_tuning t = s.tune;
        keys[std::make_tuple(pi, (int)s.params.variant * 100 + s.params.restart_k,
                             t.project_mirror * 10000 + t.project_groups * 1000 +
                                 t.backproject_split * 100 + t.backproject_mirror * 10 +
                                 t.swizzle,
                             t.project_angles)]
            .push_back(i);
    }
    Packer pk;
    const AdmitPack<float> apf = pack_admits<float>(pk, b);
    const AdmitPack<double> apd = pack_admits<double>(pk, b);
    std::vector<GroupImage<float>> imf, inf;
    std::vector<GroupImage<double>> imd, ind;
    for (auto &kv : keys) {
        const int pi = std::get<0>(kv.first);
        const Slot &first = b->active[kv.second.front()];
        const int variant = first.params.variant;
        const scg_tuning t = first.tune;
        // the newly admitted solves of the group take their initial step
        // together, one launch per phase
        std::vector<int> fresh;
        for (int i : kv.second)
            if (b->active[i].fresh) fresh.push_back(i);
        if (pi == 0) {
            imf.push_back(pack_group<float>(pk, b->active, kv.second, variant, t, true));
            b->members_f.push_back(kv.second);
            if (!fresh.empty()) inf.push_back(pack_group<float>(pk, b->active, fresh, variant, t, true));
        } else {
            imd.push_back(pack_group<double>(pk, b->active, kv.second, variant, t, true));
            b->members_d.push_back(kv.second);
            if (!fresh.empty()) ind.push_back(pack_group<double>(pk, b->active, fresh, variant, t, true));
        }
    }
    int rc = ensure_buf(&b->comp, &b->comp_bytes, std::max<size_t>(pk.bytes.size(), 256));
    if (rc) return rc;
    fill_admits<float>(pk, b, apf);
    fill_admits<double>(pk, b, apd);
    if (!pk.bytes.empty())
        HIP_TRY(hipMemcpy(b->comp, pk.bytes.data(), pk.bytes.size(), hipMemcpyHostToDevice));
    scg::launch_admit<float>(reinterpret_cast<const scg::Admit<float> *>(b->comp + apf.rec_off),
                             (int)apf.who.size(), b->stream);
    scg::launch_admit<double>(reinterpret_cast<const scg::Admit<double> *>(b->comp + apd.rec_off),
                              (int)apd.who.size(), b->stream);
    for (auto &gi : imf) {
        place(gi, b->comp);
        b->gf.push_back(gi.g);
    }
    for (auto &gi : imd) {
        place(gi, b->comp);
        b->gd.push_back(gi.g);
    }
    for (auto &gi : inf) {
        place(gi, b->comp);
        scg::enqueue_init(gi.g, b->stream);
    }
    for (auto &gi : ind) {
        place(gi, b->comp);
        scg::enqueue_init(gi.g, b->stream);
    }
    for (auto &sl : b->active) sl.fresh = false;
    if (!(b->flags & SCG_BATCH_NO_GRAPH) && !b->active.empty()) {
        HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        for (auto &g : b->gf) scg::enqueue_iteration(g, b->stream);
        for (auto &g : b->gd) scg::enqueue_iteration(g, b->stream);
        hipGraph_t graph = nullptr;
        if (hipStreamEndCapture(b->stream, &graph) != hipSuccess || graph == nullptr) {
            drop_graph(b);
            return SCG_EDEVICE;
        }
        // A composition with the same launches (the same groups and phases;
        // only block counts, maps and descriptors differ, as when solves
        // retire) updates the executable graph's kernel parameters in place,
        // which costs far less than instantiating a new one.
        bool updated = false;
        if (b->exec != nullptr) {
            hipGraphNode_t err_node = nullptr;
            hipGraphExecUpdateResult res = hipGraphExecUpdateError;
            updated = hipGraphExecUpdate(b->exec, graph, &err_node, &res) == hipSuccess &&
                      res == hipGraphExecUpdateSuccess;
            if (updated) {
                b->stats.graph_updates += 1;
            } else {
                (void)hipGetLastError();   // the refused update leaves no error behind
                drop_graph(b);
            }
        }
        if (b->graph) (void)hipGraphDestroy(b->graph);
        b->graph = graph;
        if (!updated) {
            if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
                drop_graph(b);
                return SCG_EDEVICE;
            }
            b->stats.graph_builds += 1;
        }
    } else {
        drop_graph(b);
    }
    b->stats.groups = (int32_t)(b->gf.size() + b->gd.size());
    b->dirty = false;
    return SCG_OK;
}

template <typename T>
void gather(const scg::Group<T> &g, DevState *dst, double *tv, hipStream_t s)
{
    scg::launch_gather<T>(g.S, g.ns, dst, tv, s);
}

void fill_report(const Slot &s, const DevState &fs, double tv, scg_report *rep)
{
    std::memset(rep, 0, sizeof(*rep));
    const bool plain_k = scg::unsuperiorized(s.params.variant) || scg::restarted(s.params.variant);
    rep->status = fs.done ? fs.status : SCG_ENOCONV;
    rep->k = plain_k ? fs.k : std::max(fs.k, 1);
    rep->steps = std::max(fs.steps, 0);
    rep->trials_total = fs.trials_total;
    rep->ell = fs.ell;
    rep->f_out = fs.f_half;
    rep->tv_out = tv;
}

// Output copy, TV and report of the solves `idx` (indices into active),
// then frees their slots.
int retire(scg_batch *b, const std::vector<int> &idx)
{
    if (idx.empty()) return SCG_OK;
    // per (precision, CG or not): one finalize group without graph
    Packer pk;
    std::vector<GroupImage<float>> imf;
    std::vector<GroupImage<double>> imd;
    std::vector<std::vector<int>> mf, md;
    for (int pi = 0; pi < 2; ++pi)
        for (int cg = 0; cg < 2; ++cg) {
            std::vector<int> sel;
            for (int i : idx) {
                const Slot &s = b->active[i];
                if ((s.params.prec == SCG_F64 ? 1 : 0) == pi &&
                    (scg::unsuperiorized(s.params.variant) ? 1 : 0) == cg)
                    sel.push_back(i);
            }
            if (sel.empty()) continue;
            const int variant = cg ? SCG_CG : SCG_S_CG;
            if (pi == 0) {
                imf.push_back(pack_group<float>(pk, b->active, sel, variant, {4, 2, 8, 0}, true));
                mf.push_back(sel);
            } else {
                imd.push_back(pack_group<double>(pk, b->active, sel, variant, {4, 2, 8, 0}, true));
                md.push_back(sel);
            }
        }
    int rc = ensure_buf(&b->fin_dev, &b->fin_bytes, std::max<size_t>(pk.bytes.size(), 256));
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(b->fin_dev, pk.bytes.data(), pk.bytes.size(), hipMemcpyHostToDevice,
                           b->stream));
    int at = 0;
    std::vector<int> order;
    for (size_t k = 0; k < imf.size(); ++k) {
        place(imf[k], b->fin_dev);
        scg::enqueue_final(imf[k].g, b->stream);
        gather(imf[k].g, b->dstates + at, b->dtv + at, b->stream);
        at += imf[k].g.ns;
        order.insert(order.end(), mf[k].begin(), mf[k].end());
    }
    for (size_t k = 0; k < imd.size(); ++k) {
        place(imd[k], b->fin_dev);
        scg::enqueue_final(imd[k].g, b->stream);
        gather(imd[k].g, b->dstates + at, b->dtv + at, b->stream);
        at += imd[k].g.ns;
        order.insert(order.end(), md[k].begin(), md[k].end());
    }
    HIP_TRY(hipMemcpyAsync(b->hstates, b->dstates, at * sizeof(DevState), hipMemcpyDeviceToHost,
                           b->stream));
    HIP_TRY(hipMemcpyAsync(b->htv, b->dtv, at * sizeof(double), hipMemcpyDeviceToHost,
                           b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    for (int k = 0; k < at; ++k) {
        const Slot &s = b->active[order[k]];
        scg_report rep;
        fill_report(s, b->hstates[k], b->htv[k], &rep);
        b->finished[s.ticket] = rep;
        b->arena.release(s.off, s.bytes);
        b->staging_free.push_back(s.staging);
        b->stats.retired += 1;
    }
    std::vector<int> sorted = idx;
    std::sort(sorted.rbegin(), sorted.rend());
    for (int i : sorted) b->active.erase(b->active.begin() + i);
    b->dirty = true;
    return SCG_OK;
}

template <typename T>
int submit_impl(scg_batch *b, scg_plan *plan, const scg_params *pr, const void *y,
                const void *x0, void *x_out, Slot &slot)
{
    if (scg::filtered(pr->variant)) {
        // a plan holds one filter spectrum per precision: the resident
        // filtered solves of this plan must share mu
        const double mu = scg::filter_mu(plan, pr->precond_mu);
        for (const Slot &o : b->active)
            if (o.plan == plan && scg::filtered(o.params.variant) && o.params.prec == pr->prec &&
                scg::filter_mu(plan, o.params.precond_mu) != mu)
                return SCG_EINVAL;
        int rc = scg::ensure_filter(plan, pr->precond_mu, pr->prec);
        if (rc) return rc;
    }
    char *ws = b->arena.base + slot.off;
    scg::Staging<T> &stage = staging_of<T>(b->staging[slot.staging]);
    slot.tune = scg::solve_tuning(plan->tune[scg::prec_index<T>()], pr->variant);
    int rc = scg::prepare_solve<T>(plan, pr, slot.tune, ws, y, x0, x_out, 0, nullptr, 0, &stage,
                                   b->stream, true);
    if (rc) return rc;
    desc_of<T>(slot) = stage.desc;
    slot.x0 = x0;
    slot.fresh = true;   // set-up and initial step run with the other new solves
    return SCG_OK;
}

std::mutex static_ws_mu;
std::vector<char *> static_ws;   // device address of `scratch`, by device

// The device address of the calling device's scratch (the device must be
// current).
int static_workspace(int device, char **out)
{
    std::lock_guard<std::mutex> lock(static_ws_mu);
    if ((int)static_ws.size() <= device) static_ws.resize(device + 1, nullptr);
    if (static_ws[device] == nullptr) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr)
            return SCG_EDEVICE;
        static_ws[device] = static_cast<char *>(ptr);
    }
    *out = static_ws[device];
    return SCG_OK;
}

}  // namespace

extern "C" {

int scg_workspace_bytes(const scg_plan *plan, const scg_params *params, size_t *bytes)
{
    if (plan == nullptr || bytes == nullptr) return SCG_EINVAL;
    int rc = scg::check_params(params);
    if (rc) return rc;
    *bytes = scg::workspace_bytes(plan->G, params->prec, params->max_iter);
    return SCG_OK;
}

int scg_solve(scg_plan *plan, const scg_params *params, const void *y, const void *x0,
              void *x_out, void *ws, size_t ws_bytes, scg_report *rep, scg_trace_entry *trace,
              int32_t trace_cap, const int32_t *forced, int32_t forced_len, void *stream)
{
    if (plan == nullptr || y == nullptr || x_out == nullptr || ws == nullptr) return SCG_EINVAL;
    int rc = scg::check_params(params);
    if (rc) return rc;
    if (ws_bytes < scg::workspace_bytes(plan->G, params->prec, params->max_iter))
        return SCG_ENOMEM;
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return SCG_EINVAL;
    scg::Device dg(plan->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (params->prec == SCG_F32)
        rc = scg::solve_impl<float>(plan, params, y, x0, x_out, static_cast<char *>(ws), rep,
                                    trace, trace_cap, forced, forced_len, s);
    else
        rc = scg::solve_impl<double>(plan, params, y, x0, x_out, static_cast<char *>(ws), rep,
                                     trace, trace_cap, forced, forced_len, s);
    if (hipGetLastError() != hipSuccess) return SCG_EDEVICE;
    return rc;
}

int scg_solve_static(scg_plan *plan, const scg_params *params, const void *y, const void *x0,
                     void *x_out, scg_report *rep, scg_trace_entry *trace, int32_t trace_cap,
                     const int32_t *forced, int32_t forced_len, void *stream)
{
    if (plan == nullptr || y == nullptr || x_out == nullptr) return SCG_EINVAL;
    int rc = scg::check_params(params);
    if (rc) return rc;
    if (scg::workspace_bytes(plan->G, params->prec, params->max_iter) > kStaticWsBytes)
        return SCG_ENOMEM;
    scg::Device dg(plan->device);
    char *ws = nullptr;
    rc = static_workspace(plan->device, &ws);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (params->prec == SCG_F32)
        rc = scg::solve_impl<float>(plan, params, y, x0, x_out, ws, rep, trace, trace_cap, forced,
                                    forced_len, s, false);
    else
        rc = scg::solve_impl<double>(plan, params, y, x0, x_out, ws, rep, trace, trace_cap,
                                     forced, forced_len, s, false);
    if (hipGetLastError() != hipSuccess) return SCG_EDEVICE;
    return rc;
}

size_t scg_static_workspace_bytes(void) { return kStaticWsBytes; }

int scg_batch_create(int device, size_t arena_bytes, int max_slots, uint32_t flags,
                     scg_batch **out)
{
    if (out == nullptr) return SCG_EINVAL;
    *out = nullptr;
    if (max_slots < 1 || max_slots > 4096 || arena_bytes < 4096) return SCG_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return SCG_EDEVICE;
    scg::Device dg(device);
    scg_batch *b = new (std::nothrow) scg_batch();
    if (b == nullptr) return SCG_ENOMEM;
    b->device = device;
    b->flags = flags;
    b->max_slots = max_slots;
    arena_bytes = scg::align256(arena_bytes);
    bool ok = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) == hipSuccess;
    b->own_stream = ok;
    ok = ok && hipEventCreateWithFlags(&b->order_ev, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipMalloc(&b->arena_mem, arena_bytes) == hipSuccess &&
         hipMalloc(&b->dstates, (size_t)max_slots * sizeof(DevState)) == hipSuccess &&
         hipMalloc(&b->dtv, (size_t)max_slots * sizeof(double)) == hipSuccess &&
         hipHostMalloc(&b->hstates, (size_t)max_slots * sizeof(DevState), hipHostMallocDefault) ==
             hipSuccess &&
         hipHostMalloc(&b->htv, (size_t)max_slots * sizeof(double), hipHostMallocDefault) ==
             hipSuccess &&
         hipHostMalloc(&b->staging, (size_t)max_slots * sizeof(StagingEntry),
                       hipHostMallocDefault) == hipSuccess;
    if (!ok) {
        scg_batch_destroy(b);
        return SCG_ENOMEM;
    }
    b->arena.reset(b->arena_mem, arena_bytes);
    for (int i = max_slots - 1; i >= 0; --i) b->staging_free.push_back(i);
    b->stats.slots = max_slots;
    b->stats.arena_bytes = arena_bytes;
    *out = b;
    return SCG_OK;
}

void scg_batch_destroy(scg_batch *b)
{
    if (b == nullptr) return;
    scg::Device dg(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    (void)hipFree(b->arena_mem);
    (void)hipFree(b->comp);
    (void)hipFree(b->fin_dev);
    (void)hipFree(b->dstates);
    (void)hipFree(b->dtv);
    if (b->hstates) (void)hipHostFree(b->hstates);
    if (b->htv) (void)hipHostFree(b->htv);
    if (b->staging) (void)hipHostFree(b->staging);
    if (b->order_ev) (void)hipEventDestroy(b->order_ev);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

int scg_batch_submit(scg_batch *b, scg_plan *plan, const scg_params *params, const void *y,
                     const void *x0, void *x_out, uint64_t *ticket)
{
    if (b == nullptr || plan == nullptr || y == nullptr || x_out == nullptr || ticket == nullptr)
        return SCG_EINVAL;
    int rc = scg::check_params(params);
    if (rc) return rc;
    if (plan->device != b->device) return SCG_EINVAL;
    if ((int)b->active.size() >= b->max_slots) return SCG_EAGAIN;
    scg::Device dg(b->device);
    Slot slot;
    slot.plan = plan;
    slot.params = *params;
    slot.bytes = scg::workspace_bytes(plan->G, params->prec, params->max_iter);
    if (b->staging_free.empty()) return SCG_EAGAIN;
    if (!b->arena.alloc(slot.bytes, &slot.off)) return SCG_EAGAIN;
    slot.staging = b->staging_free.back();
    b->staging_free.pop_back();
    rc = params->prec == SCG_F32 ? submit_impl<float>(b, plan, params, y, x0, x_out, slot)
                                 : submit_impl<double>(b, plan, params, y, x0, x_out, slot);
    if (rc == SCG_OK && hipGetLastError() != hipSuccess) rc = SCG_EDEVICE;
    if (rc) {
        (void)hipStreamSynchronize(b->stream);
        b->arena.release(slot.off, slot.bytes);
        b->staging_free.push_back(slot.staging);
        return rc;
    }
    slot.ticket = b->next_ticket++;
    *ticket = slot.ticket;
    b->active.push_back(slot);
    b->dirty = true;
    b->stats.submitted += 1;
    return SCG_OK;
}

int scg_batch_step(scg_batch *b, int iters)
{
    if (b == nullptr || iters < 0) return SCG_EINVAL;
    scg::Device dg(b->device);
    if (b->active.empty()) return 0;
    if (b->dirty) {
        const auto t0 = std::chrono::steady_clock::now();
        int rc = rebuild(b);
        b->stats.rebuild_ns += (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
                                   std::chrono::steady_clock::now() - t0)
                                   .count();
        if (rc) return rc;
    }
    for (int it = 0; it < iters; ++it) {
        if (b->exec) {
            HIP_TRY(hipGraphLaunch(b->exec, b->stream));
        } else {
            for (auto &g : b->gf) scg::enqueue_iteration(g, b->stream);
            for (auto &g : b->gd) scg::enqueue_iteration(g, b->stream);
        }
        b->stats.macro_steps += 1;
    }
    // read every solve's state; retire the finished ones
    int at = 0;
    std::vector<int> order;
    for (size_t k = 0; k < b->gf.size(); ++k) {
        gather(b->gf[k], b->dstates + at, b->dtv + at, b->stream);
        at += b->gf[k].ns;
        order.insert(order.end(), b->members_f[k].begin(), b->members_f[k].end());
    }
    for (size_t k = 0; k < b->gd.size(); ++k) {
        gather(b->gd[k], b->dstates + at, b->dtv + at, b->stream);
        at += b->gd[k].ns;
        order.insert(order.end(), b->members_d[k].begin(), b->members_d[k].end());
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(b->hstates, b->dstates, at * sizeof(DevState), hipMemcpyDeviceToHost,
                           b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    std::vector<int> fin;
    for (int k = 0; k < at; ++k) {
        const DevState &fs = b->hstates[k];
        const Slot &s = b->active[order[k]];
        (void)s;
        if (fs.done) fin.push_back(order[k]);
    }
    int rc = retire(b, fin);
    if (rc) return rc;
    return (int)b->active.size();
}

int scg_batch_poll(scg_batch *b, uint64_t ticket, scg_report *rep)
{
    if (b == nullptr) return SCG_EINVAL;
    auto it = b->finished.find(ticket);
    if (it != b->finished.end()) {
        if (rep != nullptr) *rep = it->second;
        b->finished.erase(it);
        return SCG_OK;
    }
    for (const Slot &s : b->active)
        if (s.ticket == ticket) return SCG_EINPROGRESS;
    return SCG_ENOTFOUND;
}

int scg_batch_cancel(scg_batch *b, uint64_t ticket)
{
    if (b == nullptr) return SCG_EINVAL;
    scg::Device dg(b->device);
    for (size_t i = 0; i < b->active.size(); ++i) {
        if (b->active[i].ticket != ticket) continue;
        HIP_TRY(hipStreamSynchronize(b->stream));
        b->arena.release(b->active[i].off, b->active[i].bytes);
        b->staging_free.push_back(b->active[i].staging);
        b->active.erase(b->active.begin() + i);
        b->dirty = true;
        return SCG_OK;
    }
    b->finished.erase(ticket);
    return SCG_ENOTFOUND;
}

int scg_batch_get_stats(const scg_batch *b, scg_batch_stats *out)
{
    if (b == nullptr || out == nullptr) return SCG_EINVAL;
    *out = b->stats;
    out->active = (int32_t)b->active.size();
    out->arena_used = b->arena.used;
    return SCG_OK;
}

void *scg_batch_stream(const scg_batch *b) { return b ? static_cast<void *>(b->stream) : nullptr; }

int scg_batch_wait_stream(scg_batch *b, void *stream)
{
    if (b == nullptr) return SCG_EINVAL;
    scg::Device dg(b->device);
    HIP_TRY(hipEventRecord(b->order_ev, static_cast<hipStream_t>(stream)));
    HIP_TRY(hipStreamWaitEvent(b->stream, b->order_ev, 0));
    return SCG_OK;
}

}  // extern "C"
