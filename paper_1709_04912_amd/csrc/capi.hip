// C-ABI of libscg: plans (geometry tables), the standalone operators, launch
// shapes and their autotuner, kernel timing, parameters and status strings.
// The solver driver and the batch engine are in engine.hip.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <climits>
#include <vector>

#include "plan.h"


namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kKCap = 1048576.0;   // 2^20: K for axis-aligned rays

int hip_status(hipError_t e) { return e == hipSuccess ? SCG_OK : SCG_EDEVICE; }


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
// Starting from `start` angles, the group size shrinks until every window
// fits kPjWin columns. Tables for group sizes of 8 and 4 (index 0 and 1),
// and their mirrored forms (index 2 and 3), whose groups cover only the
// angles a <= n_a / 2: the rays of angle n_a - a are those of angle a in the
// image mirrored about the vertical axis, so they cross the same window
// columns of the mirrored band.
int build_proj_tables(scg_plan *p, const std::vector<ProjAngle> &pa, int start, int ti,
                      bool mirror)
{
    const Geo &G = p->G;
    const int n_chunks = (G.nb + scg::kPjBins - 1) / scg::kPjBins;
    const int n_bands = (G.n + scg::kPjBand - 1) / scg::kPjBand;
    const int a_end = mirror ? G.na / 2 + 1 : G.na;
    for (int gmax = start; gmax >= 1; --gmax) {
        std::vector<PjGroup> groups;
        for (int a = 0; a < a_end;) {
            PjGroup g{a, 1, pa[a].major, 0};
            while (g.count < gmax && a + g.count < a_end && pa[a + g.count].major == g.major)
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
        // Blocks differ in work by the bands they skip; dispatching the
        // heaviest first lets the light ones fill the tail of the launch.
        // The hardware hands workgroup b to XCD b mod 8: launch positions on
        // XCDs 0-3 take the groups that step over rows (they read x), those
        // on XCDs 4-7 the groups that step over columns (they read x^T), so
        // each XCD's L2 fetches one orientation of the image instead of both.
        const int nblk = (int)groups.size() * n_chunks;
        std::vector<int> bands(nblk, 0), order;
        std::vector<int> by_major[2];
        for (int id = 0; id < nblk; ++id) {
            for (int band = 0; band < n_bands; ++band)
                bands[id] += win[(size_t)id * n_bands + band] != scg::kWinSkip;
            by_major[groups[id / n_chunks].major].push_back(id);
        }
        for (auto &v : by_major)
            std::stable_sort(v.begin(), v.end(), [&](int a, int b) { return bands[a] > bands[b]; });
        size_t next[2] = {0, 0};
        for (int pos = 0; pos < nblk; ++pos) {
            int mj = (pos % scg::kXcds) < scg::kXcds / 2 ? 0 : 1;
            if (next[mj] == by_major[mj].size()) mj ^= 1;
            order.push_back(by_major[mj][next[mj]++]);
        }
        // An XCD deals its blocks to its CUs in turn, so with a plain
        // heaviest-first sequence the first CU would receive the heaviest
        // block of every round. Reversing every other round of kXcdCus
        // blocks (a snake) pairs heavy with light on each CU.
        for (int x = 0; x < scg::kXcds; ++x) {
            std::vector<int> pos;
            for (int p0 = x; p0 < nblk; p0 += scg::kXcds) pos.push_back(p0);
            for (size_t r0 = scg::kXcdCus; r0 < pos.size(); r0 += 2 * scg::kXcdCus) {
                const size_t r1 = std::min(pos.size(), r0 + scg::kXcdCus);
                for (size_t a = r0, b = r1 - 1; a < b; ++a, --b) std::swap(order[pos[a]], order[pos[b]]);
            }
        }
        if (hipMalloc(&p->pgroups[ti], groups.size() * sizeof(PjGroup)) != hipSuccess ||
            hipMalloc(&p->pwin[ti], win.size() * sizeof(int)) != hipSuccess ||
            hipMalloc(&p->porder[ti], order.size() * sizeof(int)) != hipSuccess)
            return SCG_ENOMEM;
        if (hipMemcpy(p->porder[ti], order.data(), order.size() * sizeof(int),
                      hipMemcpyHostToDevice) != hipSuccess)
            return SCG_EDEVICE;
        if (hipMemcpy(p->pgroups[ti], groups.data(), groups.size() * sizeof(PjGroup),
                      hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(p->pwin[ti], win.data(), win.size() * sizeof(int), hipMemcpyHostToDevice) !=
                hipSuccess)
            return SCG_EDEVICE;
        ProjTables &t = p->ptab[ti];
        t.ang = p->pang;
        t.groups = p->pgroups[ti];
        t.win = p->pwin[ti];
        t.order = p->porder[ti];
        t.n_groups = (int)groups.size();
        t.n_chunks = n_chunks;
        t.n_bands = n_bands;
        t.group_max = start;
        t.mirror = mirror ? 1 : 0;
        return SCG_OK;
    }
    return SCG_EINVAL;
}

// Backprojector tile of each launch position: the tile grid is cut into
// kXcds regions (4 x 2, as square as the grid allows) and position b takes
// the next tile of region b mod kXcds, the XCD the hardware hands workgroup b
// to. Each XCD's L2 then holds the sinogram footprint of one region (about a
// third of every projection at 512^2) instead of the whole sinogram. Tiles
// are equal work, so the regions balance; a region that runs out lends the
// position to the next one.
std::vector<int> bp_tile_order(const Geo &G)
{
    const int nt = (G.n + scg::kBpTile - 1) / scg::kBpTile;
    constexpr int kRx = 4, kRy = scg::kXcds / 4;
    std::vector<std::vector<int>> region(scg::kXcds);
    for (int ty = 0; ty < nt; ++ty)
        for (int tx = 0; tx < nt; ++tx)
            region[(ty * kRy / nt) * kRx + tx * kRx / nt].push_back(ty * nt + tx);
    std::vector<int> order;
    std::vector<size_t> next(scg::kXcds, 0);
    for (int pos = 0; pos < nt * nt; ++pos) {
        int r = pos % scg::kXcds;
        while (next[r] == region[r].size()) r = (r + 1) % scg::kXcds;
        order.push_back(region[r][next[r]++]);
    }
    return order;
}

int filter_pad(int nb)
{
    int P = 1;
    while (P < 2 * nb) P <<= 1;
    return P;
}

// Elements of a filter table: P spectrum values and the P - 1 complex
// twiddles of the spans 1, 2, ..., P/2.
size_t filter_table_len(int P) { return (size_t)P + 2 * (size_t)(P - 1); }

// Spectrum of the preconditioning filter at the transform's bit-reversed
// positions: c(w_k) / P with w_k = 2 pi k / P taken in [-pi, pi), k the
// frequency stored at position i (k = bit reverse of i over log2 P bits),
// c(w) = (|w| + mu)(0.54 + 0.46 cos w).
void filter_spectrum(int P, double mu, std::vector<double> &out)
{
    int bits = 0;
    while ((1 << bits) < P) ++bits;
    out.resize(P);
    for (int i = 0; i < P; ++i) {
        int k = 0;
        for (int b = 0; b < bits; ++b) k |= ((i >> b) & 1) << (bits - 1 - b);
        const int m = k < P / 2 ? k : k - P;   // m in [-P/2, P/2)
        const double w = 2.0 * kPi * m / P;
        out[i] = (std::fabs(w) + mu) * (0.54 + 0.46 * std::cos(w)) / P;
    }
}

template <typename T>
int upload_filter(scg_plan *p, int pi, double mu, bool twiddles)
{
    const int P = filter_pad(p->G.nb);
    std::vector<double> sp;
    filter_spectrum(P, mu, sp);
    std::vector<T> tab(twiddles ? filter_table_len(P) : (size_t)P);
    for (int i = 0; i < P; ++i) tab[i] = (T)sp[i];
    if (twiddles)
        for (int h = 1; h < P; h <<= 1)
            for (int j = 0; j < h; ++j) {
                const double w = -kPi * j / h;   // e^{-2 pi i j / (2h)}
                tab[P + 2 * (h - 1 + j)] = (T)std::cos(w);
                tab[P + 2 * (h - 1 + j) + 1] = (T)std::sin(w);
            }
    HIP_TRY(hipMemcpy(p->ftab[pi], tab.data(), tab.size() * sizeof(T), hipMemcpyHostToDevice));
    p->filt_mu[pi] = mu;
    return SCG_OK;
}

}  // namespace

namespace scg {

bool filter_fits(int nb, int prec)
{
    const size_t esz = prec == SCG_F64 ? sizeof(double) : sizeof(float);
    return (size_t)filter_pad(nb) * 2 * esz <= kFilterLds;
}

double filter_mu(const scg_plan *p, double mu)
{
    return mu > 0.0 ? mu : 2.0 * kPi / filter_pad(p->G.nb);
}

// The filter tables of precision prec hold the spectrum for mu (<= 0: 2 pi
// / P); they were allocated with the plan, so this only uploads.
int ensure_filter(scg_plan *p, double mu, int prec)
{
    const int pi = prec == SCG_F64 ? 1 : 0;
    if (p->ftab[pi] == nullptr) return SCG_EINVAL;   // n_bins beyond the LDS bound
    mu = filter_mu(p, mu);
    if (p->filt_mu[pi] == mu) return SCG_OK;
    return pi ? upload_filter<double>(p, 1, mu, false) : upload_filter<float>(p, 0, mu, false);
}

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
// Events around one launch in every p->prof_every of a timed class: an event
// record between two launches holds the next one back by a few
// microseconds, so sampling keeps the timed solve close to an untimed one.
void prof_mark(scg_plan *p, int cls, hipStream_t s, bool begin)
{
    if (!(p->prof_mask & (1u << cls))) return;
    if (begin) {
        if (p->prof_seq[cls]++ % p->prof_every != 0) return;
    } else if (p->prof_open[cls] == nullptr) {
        return;   // the launch was not sampled
    }
    hipEvent_t e = take_event(p);
    if (e == nullptr) return;
    (void)hipEventRecord(e, s);
    if (begin) {
        p->prof_open[cls] = e;
    } else {
        p->prof_pending.push_back({cls, p->prof_iter, p->prof_open[cls], e});
        p->prof_open[cls] = nullptr;
    }
}

// Accumulates the elapsed times of recorded launches. Launches enqueued by
// loop iterations past `last_iter` (the solve had already stopped; their
// kernels returned at once) are kept apart, except the TV kernel and the
// finishers of the iteration after it, which still close the last step.
void prof_drain(scg_plan *p, int last_iter)
{
    for (const auto &r : p->prof_pending) {
        float ms = 0.0f;
        if (hipEventSynchronize(r.b) == hipSuccess &&
            hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            const bool closes = r.cls == SCG_KC_TV || r.cls == SCG_KC_CONTROL;
            const int lim = last_iter == INT_MAX ? INT_MAX : last_iter + (closes ? 1 : 0);
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

// Moves the timing records from index `from` on to the tail sums: launches
// that returned at once because the solve was suspended.
void prof_to_tail(scg_plan *p, size_t from)
{
    for (size_t i = from; i < p->prof_pending.size(); ++i) {
        const auto &r = p->prof_pending[i];
        float ms = 0.0f;
        if (hipEventSynchronize(r.b) == hipSuccess &&
            hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            p->prof_tail_ms[r.cls] += ms;
            p->prof_tail_count[r.cls] += 1;
        }
        p->ev_free.push_back(r.a);
        p->ev_free.push_back(r.b);
    }
    if (from < p->prof_pending.size()) p->prof_pending.resize(from);
}

int check_params(const scg_params *pr)
{
    if (pr == nullptr) return SCG_EINVAL;
    if (pr->variant < SCG_CG || pr->variant > SCG_S_PCG_K) return SCG_EINVAL;
    if ((pr->variant == SCG_S_CG_K || pr->variant == SCG_S_PCG_K) &&
        (pr->restart_k < 1 || pr->restart_k > 64))
        return SCG_EINVAL;
    if (pr->prec != SCG_F32 && pr->prec != SCG_F64) return SCG_EINVAL;
    if (!(pr->eps > 0.0) || !std::isfinite(pr->eps)) return SCG_EINVAL;
    if (!(pr->gamma0 >= 0.0) || !std::isfinite(pr->gamma0)) return SCG_EINVAL;
    if (!(pr->a > 0.0 && pr->a < 1.0)) return SCG_EINVAL;
    if (pr->max_iter < 0 || pr->max_iter > 1000000) return SCG_EINVAL;
    if (pr->max_trials < 1 || pr->max_trials > scg::kMaxTrials) return SCG_EINVAL;
    if (!(pr->tv_kappa >= 0.0) || !std::isfinite(pr->tv_kappa)) return SCG_EINVAL;
    return SCG_OK;
}

}  // namespace scg

namespace {

bool tuning_valid(const scg_tuning &t)
{
    return (t.project_groups == 2 || t.project_groups == 4) &&
           (t.backproject_split == 1 || t.backproject_split == 2 ||
            t.backproject_split == 4 || (t.backproject_split == 8 && t.backproject_mirror == 1)) &&
           (t.project_angles == 8 || t.project_angles == 4) && (t.swizzle == 0 || t.swizzle == 1) &&
           (t.backproject_mirror == 0 || t.backproject_mirror == 1) &&
           (t.project_mirror == 0 || t.project_mirror == 1);
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
    const int pi = scg::prec_index<T>();
    T *x = nullptr, *y = nullptr;
    if (hipMalloc(&x, G.img_elems() * sizeof(T)) != hipSuccess) return SCG_ENOMEM;
    if (hipMalloc(&y, G.sino_elems() * sizeof(T)) != hipSuccess) {
        (void)hipFree(x);
        return SCG_ENOMEM;
    }
    scg::launch_fill<T>(x, G.img_elems(), T(1), s);
    scg::launch_fill<T>(y, G.sino_elems(), T(1), s);
    T *xs = static_cast<T *>(plan->xs[pi]);
    scg::launch_stage<T>(x, xs, G, s);
    // Each candidate is timed twice, in two rounds over all candidates, and
    // keeps its faster time; a warm-up before the first round brings the
    // clocks up, so the candidates timed first are not penalised.
    constexpr int kReps = 10;
    constexpr int kRounds = 2;
    scg_tuning best = plan->tune[pi];
    struct PjCand { int ga, nq, mir, swz; float ms; };
    struct BpCand { int sp, mir, swz; float ms; };
    std::vector<PjCand> pj;
    std::vector<BpCand> bp;
    for (int ga : {8, 4})
        for (int nq : {2, 4})
            for (int mir : {0, 1})
                for (int swz : {0, 1}) pj.push_back({ga, nq, mir, swz, -1.0f});
    for (int sp : {1, 2, 4, 8})
        for (int mir : {0, 1})
            for (int swz : {0, 1})
                if (sp < 8 || mir) bp.push_back({sp, mir, swz, -1.0f});
    auto run_pj = [&](const PjCand &c) {
        scg::launch_project<T>(x, xs, G, plan->ptab[(c.ga == 8 ? 0 : 1) + (c.mir ? 2 : 0)], y,
                               G.rs, scg::kSinoPadL, c.nq, c.swz, s);
    };
    auto run_bp = [&](const BpCand &c) {
        scg::launch_backproject<T>(y, G, plan->bang, plan->border, x, c.sp, c.mir, c.swz, s);
    };
    (void)time_launches([&] { run_pj(pj.front()); run_bp(bp.front()); }, s, 2 * kReps);
    auto keep = [](float &acc, float ms) {
        if (ms > 0.0f && (acc < 0.0f || ms < acc)) acc = ms;
    };
    for (int round = 0; round < kRounds; ++round) {
        for (auto &c : pj) keep(c.ms, time_launches([&] { run_pj(c); }, s, kReps));
        for (auto &c : bp) keep(c.ms, time_launches([&] { run_bp(c); }, s, kReps));
    }
    // one swizzle flag serves both operators, and a step applies each as
    // often as the other: the flag with the smaller sum of the two best times
    float best_sum = -1.0f;
    for (int swz : {0, 1}) {
        const PjCand *bpj = nullptr;
        const BpCand *bbp = nullptr;
        for (const auto &c : pj)
            if (c.swz == swz && c.ms > 0.0f && (bpj == nullptr || c.ms < bpj->ms)) bpj = &c;
        for (const auto &c : bp)
            if (c.swz == swz && c.ms > 0.0f && (bbp == nullptr || c.ms < bbp->ms)) bbp = &c;
        if (bpj == nullptr || bbp == nullptr) continue;
        const float sum = bpj->ms + bbp->ms;
        if (best_sum < 0.0f || sum < best_sum) {
            best_sum = sum;
            best.project_angles = bpj->ga;
            best.project_groups = bpj->nq;
            best.project_mirror = bpj->mir;
            best.backproject_split = bbp->sp;
            best.backproject_mirror = bbp->mir;
            best.swizzle = swz;
        }
    }
    const hipError_t e = hipStreamSynchronize(s);
    (void)hipFree(x);
    (void)hipFree(y);
    if (e != hipSuccess || best_sum < 0.0f) return SCG_EDEVICE;
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
    p->restart_k = 2;
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
    // the largest image the parity tests cover (the block partials of every
    // reduction fit the partials buffer well beyond it)
    if (g->n > scg::kMaxN || g->n_angles > 65536 || g->n_bins > 65536) return SCG_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return SCG_EDEVICE;
    scg::Device dg(device);
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
    // Every reduction's block partials must fit the partials buffer (the
    // preconditioning filter's LDS bound is checked where the filter is set
    // up).
    if ((size_t)scg::blocks_bp(G) > (size_t)scg::kMaxPartials ||
        2 * (size_t)scg::blocks_xtv(G) > (size_t)scg::kMaxPartials ||
        (size_t)scg::blocks_t32(G) + scg::blocks_sv(G) > (size_t)scg::kMaxPartials ||
        scg::blocks_t32(G) > scg::kMaxT32Blocks) {
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
    const std::vector<int> bord = bp_tile_order(G);
    bool ok = hipMalloc(&p->pang, pa.size() * sizeof(ProjAngle)) == hipSuccess &&
              hipMalloc(&p->bang, ba.size() * sizeof(BpAngle)) == hipSuccess &&
              hipMalloc(&p->border, bord.size() * sizeof(int)) == hipSuccess &&
              hipMalloc(&p->xs[0], G.staged_elems() * sizeof(float)) == hipSuccess &&
              hipMalloc(&p->xs[1], G.staged_elems() * sizeof(double)) == hipSuccess &&
              hipMalloc(&p->rpad[0], G.sino_elems() * sizeof(float)) == hipSuccess &&
              hipMalloc(&p->rpad[1], G.sino_elems() * sizeof(double)) == hipSuccess &&
              hipMalloc(&p->partials, scg::kMaxPartials * sizeof(double)) == hipSuccess &&
              hipMalloc(&p->tvbuf, sizeof(double)) == hipSuccess &&
              hipHostMalloc(&p->host_pinned, scg::kHostPinnedBytes, hipHostMallocDefault) ==
                  hipSuccess;
    if (!ok) {
        scg_plan_destroy(p);
        return SCG_ENOMEM;
    }
    ok = hipMemcpy(p->pang, pa.data(), pa.size() * sizeof(ProjAngle), hipMemcpyHostToDevice) ==
             hipSuccess &&
         hipMemcpy(p->bang, ba.data(), ba.size() * sizeof(BpAngle), hipMemcpyHostToDevice) ==
             hipSuccess &&
         hipMemcpy(p->border, bord.data(), bord.size() * sizeof(int), hipMemcpyHostToDevice) ==
             hipSuccess &&
         hipMemset(p->xs[0], 0, G.staged_elems() * sizeof(float)) == hipSuccess &&
         hipMemset(p->xs[1], 0, G.staged_elems() * sizeof(double)) == hipSuccess &&
         hipMemset(p->rpad[0], 0, G.sino_elems() * sizeof(float)) == hipSuccess &&
         hipMemset(p->rpad[1], 0, G.sino_elems() * sizeof(double)) == hipSuccess &&
         hipDeviceSynchronize() == hipSuccess;
    if (!ok) {
        scg_plan_destroy(p);
        return SCG_EDEVICE;
    }
    int rc = build_proj_tables(p, pa, 8, 0, false);
    if (rc == SCG_OK) rc = build_proj_tables(p, pa, 4, 1, false);
    if (rc == SCG_OK) rc = build_proj_tables(p, pa, 8, 2, true);
    if (rc == SCG_OK) rc = build_proj_tables(p, pa, 4, 3, true);
    // filter tables (spectrum for the default mu and twiddles) for each
    // precision whose transform fits the LDS bound; a solve later changes
    // only the spectrum, without allocating
    const double mu0 = 2.0 * kPi / filter_pad(G.nb);
    if (rc == SCG_OK && scg::filter_fits(G.nb, SCG_F32)) {
        if (hipMalloc(&p->ftab[0], filter_table_len(filter_pad(G.nb)) * sizeof(float)) !=
            hipSuccess)
            rc = SCG_ENOMEM;
        else
            rc = upload_filter<float>(p, 0, mu0, true);
    }
    if (rc == SCG_OK && scg::filter_fits(G.nb, SCG_F64)) {
        if (hipMalloc(&p->ftab[1], filter_table_len(filter_pad(G.nb)) * sizeof(double)) !=
            hipSuccess)
            rc = SCG_ENOMEM;
        else
            rc = upload_filter<double>(p, 1, mu0, true);
    }
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
    scg::Device dg(p->device);
    (void)hipFree(p->pang);
    (void)hipFree(p->bang);
    (void)hipFree(p->border);
    for (int i = 0; i < 4; ++i) {
        (void)hipFree(p->pgroups[i]);
        (void)hipFree(p->pwin[i]);
        (void)hipFree(p->porder[i]);
    }
    for (int i = 0; i < 2; ++i) {
        (void)hipFree(p->xs[i]);
        (void)hipFree(p->rpad[i]);
        (void)hipFree(p->ftab[i]);
    }
    (void)hipFree(p->partials);
    (void)hipFree(p->tvbuf);
    if (p->host_pinned) (void)hipHostFree(p->host_pinned);
    scg::prof_drain(p);
    for (hipEvent_t e : p->ev_free) (void)hipEventDestroy(e);
    for (hipEvent_t e : p->prof_open)
        if (e != nullptr) (void)hipEventDestroy(e);
    delete p;
}

int scg_profile(scg_plan *plan, uint32_t class_mask)
{
    if (plan == nullptr) return SCG_EINVAL;
    scg::Device dg(plan->device);
    scg::prof_drain(plan);
    for (int c = 0; c < SCG_KC_COUNT; ++c) {
        plan->prof_seq[c] = 0;
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

int scg_profile_every(scg_plan *plan, int32_t every)
{
    if (plan == nullptr || every < 1) return SCG_EINVAL;
    plan->prof_every = every;
    for (int c = 0; c < SCG_KC_COUNT; ++c) plan->prof_seq[c] = 0;
    return SCG_OK;
}

int scg_profile_read(scg_plan *plan, scg_kernel_time *out)
{
    if (plan == nullptr || out == nullptr) return SCG_EINVAL;
    scg::Device dg(plan->device);
    scg::prof_drain(plan);
    for (int c = 0; c < SCG_KC_COUNT; ++c) {
        out[c].launches = plan->prof_count[c];
        out[c].total_ms = plan->prof_ms[c];
        out[c].tail_launches = plan->prof_tail_count[c];
        out[c].tail_ms = plan->prof_tail_ms[c];
    }
    return SCG_OK;
}

int scg_project(scg_plan *plan, int prec, const void *x, void *y, void *stream)
{
    if (plan == nullptr || x == nullptr || y == nullptr) return SCG_EINVAL;
    if (prec != SCG_F32 && prec != SCG_F64) return SCG_EINVAL;
    scg::Device dg(plan->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Geo &G = plan->G;
    if (prec == SCG_F32) {
        float *xs = static_cast<float *>(plan->xs[0]);
        const float *xf = static_cast<const float *>(x);
        const scg_tuning &t = plan->tune[0];
        scg::launch_stage<float>(xf, xs, G, s);
        scg::launch_project<float>(xf, xs, G, scg::proj_tables(plan, t), static_cast<float *>(y),
                                   G.nb, 0, t.project_groups, t.swizzle, s);
    } else {
        double *xs = static_cast<double *>(plan->xs[1]);
        const double *xd = static_cast<const double *>(x);
        const scg_tuning &t = plan->tune[1];
        scg::launch_stage<double>(xd, xs, G, s);
        scg::launch_project<double>(xd, xs, G, scg::proj_tables(plan, t),
                                    static_cast<double *>(y), G.nb, 0, t.project_groups,
                                    t.swizzle, s);
    }
    return hip_status(hipGetLastError());
}

int scg_backproject(scg_plan *plan, int prec, const void *y, void *x, void *stream)
{
    if (plan == nullptr || x == nullptr || y == nullptr) return SCG_EINVAL;
    if (prec != SCG_F32 && prec != SCG_F64) return SCG_EINVAL;
    scg::Device dg(plan->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Geo &G = plan->G;
    if (prec == SCG_F32) {
        float *rp = static_cast<float *>(plan->rpad[0]);
        scg::launch_pad_sino<float>(static_cast<const float *>(y), rp, G, s);
        const scg_tuning &t = plan->tune[0];
        scg::launch_backproject<float>(rp, G, plan->bang, plan->border, static_cast<float *>(x),
                                       t.backproject_split, t.backproject_mirror, t.swizzle, s);
    } else {
        double *rp = static_cast<double *>(plan->rpad[1]);
        scg::launch_pad_sino<double>(static_cast<const double *>(y), rp, G, s);
        const scg_tuning &t = plan->tune[1];
        scg::launch_backproject<double>(rp, G, plan->bang, plan->border, static_cast<double *>(x),
                                        t.backproject_split, t.backproject_mirror, t.swizzle, s);
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
    scg::Device dg(plan->device);
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
    scg::Device dg(plan->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Geo &G = plan->G;
    if (prec == SCG_F32)
        scg::launch_tv<float>(static_cast<const float *>(x), static_cast<float *>(s_out), G, kappa,
                              plan->partials, plan->tvbuf, s);
    else
        scg::launch_tv<double>(static_cast<const double *>(x), static_cast<double *>(s_out), G,
                               kappa, plan->partials, plan->tvbuf, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(tv_host, plan->tvbuf, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return SCG_OK;
}

int scg_filter(scg_plan *plan, int prec, double mu, const void *r, void *out, void *stream)
{
    if (plan == nullptr || r == nullptr || out == nullptr) return SCG_EINVAL;
    if (prec != SCG_F32 && prec != SCG_F64) return SCG_EINVAL;
    scg::Device dg(plan->device);
    int rc = scg::ensure_filter(plan, mu, prec);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Geo &G = plan->G;
    if (prec == SCG_F32) {
        float *rp = static_cast<float *>(plan->rpad[0]);
        scg::launch_pad_sino<float>(static_cast<const float *>(r), rp, G, s);
        scg::launch_filter<float>(rp, static_cast<float *>(out),
                                  static_cast<const float *>(plan->ftab[0]), G, 0, s);
    } else {
        double *rp = static_cast<double *>(plan->rpad[1]);
        scg::launch_pad_sino<double>(static_cast<const double *>(r), rp, G, s);
        scg::launch_filter<double>(rp, static_cast<double *>(out),
                                   static_cast<const double *>(plan->ftab[1]), G, 0, s);
    }
    return hip_status(hipGetLastError());
}

}  // extern "C"
