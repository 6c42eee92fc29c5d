// C ABI of the energy-point Green's-function engine: argument checks, HBM
// layout, job/span scheduling, energy chunking and the launch sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "negf_internal.hpp"
#include "negf_reduce.hpp"

using negf::cx;

namespace negf_host {

thread_local std::string g_err;

negf_status fail(negf_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

const negf::Launchers* launchers_for(int b) {
    switch (b) {
#define CASE(B) case B: return negf::launchers_b##B();
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10)
        CASE(11) CASE(12) CASE(13) CASE(14) CASE(15) CASE(16) CASE(17) CASE(18) CASE(19)
        CASE(20) CASE(21) CASE(22) CASE(23) CASE(24)
#undef CASE
        default: return nullptr;
    }
}

bool finite_c(const negf_c64* p, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i].re) || !std::isfinite(p[i].im)) return false;
    return true;
}

const char* const kKernelNames[KT_COUNT] = {"decimate", "recur", "cdiag", "column", "reduce", "fp64_recompute"};


negf_status dalloc_raw(size_t* counter, void** p, size_t bytes) {
    if (bytes == 0) bytes = 16;
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) return fail(NEGF_ENOMEM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    *p = q;
    *counter += bytes;
    return NEGF_OK;
}

template <typename P>
negf_status dalloc(negf_device* d, P** p, size_t bytes) {
    void* q = nullptr;
    TRY(dalloc_raw(&d->bytes, &q, bytes));
    *p = static_cast<P*>(q);
    return NEGF_OK;
}

// waits until the last enqueued solve of w has finished on the device
negf_status wait_prev(negf_workspace* w) {
    HIPCHK(hipEventSynchronize(w->done));
    return NEGF_OK;
}

// Arena mode: the next 256-byte-aligned piece of the caller's fixed area.
negf_status carve(negf_workspace* w, DBuf& buf, size_t bytes) {
    const size_t at = (w->arena_off + 255) & ~size_t(255);
    const size_t want = std::max<size_t>(bytes, 256);
    if (at > w->arena_cap || want > w->arena_cap - at)
        return fail(NEGF_EINVAL,
                    "problem needs more than the %zu bytes of the static scratch area (%zu bytes placed, %zu more "
                    "requested)",
                    w->arena_cap, at, want);
    buf.p = w->arena + at;
    buf.cap = want;
    w->arena_off = at + want;
    return NEGF_OK;
}

negf_status grow(negf_workspace* w, DBuf& buf, size_t bytes) {
    if (w->arena) return carve(w, buf, bytes);
    if (bytes <= buf.cap && buf.p) return NEGF_OK;
    if (w->capturing) return fail(NEGF_EINVAL, "graph capture needs a workspace sized by an eager solve");
    if (buf.p) {
        TRY(wait_prev(w));   // the previous solve may still use it
        (void)hipFree(buf.p);
        w->bytes -= std::min(w->bytes, buf.cap);
        buf.p = nullptr;
        buf.cap = 0;
    }
    const size_t want = std::max<size_t>(bytes, 256);
    TRY(dalloc_raw(&w->bytes, &buf.p, want));
    buf.cap = want;
    return NEGF_OK;
}

constexpr size_t kDefaultStoreCap = (size_t)8 << 30;

negf_status upload_lead_D(negf_device* d, int l) {
    LeadDev& ld = d->lead[l];
    const int b = d->b;
    std::vector<negf_c64> D = ld.h_diag;
    for (int p = 0; p < ld.period; ++p)
        for (int i = 0; i < b; ++i) D[(size_t)p * b * b + (size_t)i * b + i].re += d->U_lead[l];
    HIPCHK(hipMemcpy(ld.D, D.data(), D.size() * 16, hipMemcpyHostToDevice));
    if (ld.circ) {   // the on-site mode values (rows 0 and 1) shift with the lead potential
        std::vector<negf_c64> m = ld.modes0;
        for (int q = 0; q < 2 * b; ++q) m[q].re += d->U_lead[l];
        HIPCHK(hipMemcpy(ld.modes, m.data(), m.size() * 16, hipMemcpyHostToDevice));
    }
    return NEGF_OK;
}

bool is_circulant(const negf_c64* M, int b) {
    for (int i = 0; i < b; ++i)
        for (int j = 0; j < b; ++j) {
            const negf_c64 a = M[(size_t)i * b + j], c = M[(size_t)((j - i + b) % b)];
            if (a.re != c.re || a.im != c.im) return false;
        }
    return true;
}

// eigenvalue of a circulant block on the ring Fourier vector q: sum_k C[0][k] e^{2 pi i q k / b}
negf_c64 ring_mode(const negf_c64* C, int b, int q) {
    double re = 0.0, im = 0.0;
    const double pi = 3.14159265358979323846;
    for (int k = 0; k < b; ++k) {
        const double ph = 2.0 * pi * (double)(((long long)q * k) % b) / b;
        const double cs = std::cos(ph), sn = std::sin(ph);
        re += C[k].re * cs - C[k].im * sn;
        im += C[k].re * sn + C[k].im * cs;
    }
    return negf_c64{re, im};
}

negf_status check_lead(const negf_lead* ld, int b, const char* which) {
    if (!ld) return fail(NEGF_EINVAL, "%s lead is NULL", which);
    if (ld->period < 1 || ld->period > NEGF_MAX_PERIOD)
        return fail(NEGF_EINVAL, "%s lead period %d not in [1,%d]", which, ld->period, NEGF_MAX_PERIOD);
    if (!ld->h_diag || !ld->h_up || !ld->tau) return fail(NEGF_EINVAL, "%s lead has a NULL block", which);
    const size_t b2 = (size_t)b * b;
    if (!finite_c(ld->h_diag, ld->period * b2) || !finite_c(ld->h_up, ld->period * b2) || !finite_c(ld->tau, b2))
        return fail(NEGF_EINVAL, "%s lead has non-finite entries", which);
    return NEGF_OK;
}

negf_status check_job(const negf_job& j, int idx, bool host) {
    if (!j.dev) return fail(NEGF_EINVAL, "job %d: device handle is NULL", idx);
    const negf_bias& b = j.bias;
    if (!(b.kT_L > 0) || !(b.kT_R > 0) || !std::isfinite(b.mu_L) || !std::isfinite(b.mu_R) ||
        !std::isfinite(b.kT_L) || !std::isfinite(b.kT_R))
        return fail(NEGF_EINVAL, "job %d: bias needs finite mu and kT > 0", idx);
    if (j.n_c < 0 || j.n_r < 0)
        return fail(NEGF_EINVAL, "job %d: negative node count (n_c=%d, n_r=%d)", idx, j.n_c, j.n_r);
    if (j.n_poles < 0 || j.n_poles > (1 << 20)) return fail(NEGF_EINVAL, "job %d: n_poles = %d", idx, j.n_poles);
    if (j.n_c + j.n_poles + j.n_r < 1) return fail(NEGF_EINVAL, "job %d: no energy nodes", idx);
    if ((long long)j.n_c + j.n_poles + j.n_r > (1LL << 26))
        return fail(NEGF_EINVAL, "job %d: too many energy nodes", idx);
    if (j.n_c > 0 && (!j.z_c || !j.w_c)) return fail(NEGF_EINVAL, "job %d: contour nodes/weights are NULL", idx);
    if (j.n_r > 0 && (!j.E_r || !j.w_r)) return fail(NEGF_EINVAL, "job %d: real-axis nodes/weights are NULL", idx);
    if (!j.charge) return fail(NEGF_EINVAL, "job %d: charge output is NULL", idx);
    if (j.sigma_mode < 0 || j.sigma_mode > 2) return fail(NEGF_EINVAL, "job %d: sigma_mode %d", idx, j.sigma_mode);
    if (j.sigma_mode && !j.sigma_cache) return fail(NEGF_EINVAL, "job %d: sigma_cache is NULL", idx);
    if (host) {
        for (int i = 0; i < j.n_c; ++i)
            if (!std::isfinite(j.z_c[i].re) || !std::isfinite(j.z_c[i].im) || !std::isfinite(j.w_c[i].re) ||
                !std::isfinite(j.w_c[i].im))
                return fail(NEGF_EINVAL, "job %d: contour node %d is not finite", idx, i);
        for (int i = 0; i < j.n_r; ++i)
            if (!std::isfinite(j.E_r[i]) || !std::isfinite(j.w_r[i]))
                return fail(NEGF_EINVAL, "job %d: real node %d is not finite", idx, i);
    }
    return NEGF_OK;
}

void ev_begin(negf_workspace* w, hipStream_t s, hipEvent_t* a) {
    *a = nullptr;
    if (!w->prof || w->capturing) return;
    (void)hipEventCreate(a);
    (void)hipEventRecord(*a, s);
}
void ev_end(negf_workspace* w, int kind, hipStream_t s, hipEvent_t a) {
    if (!w->prof || !a) return;
    hipEvent_t b;
    (void)hipEventCreate(&b);
    (void)hipEventRecord(b, s);
    w->pending.push_back({kind, a, b});
}
void ev_collect(negf_workspace* w) {
    for (auto& e : w->pending) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, e.a, e.b) == hipSuccess) {
            w->ms[e.kind] += t;
            w->calls[e.kind] += 1;
        }
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    w->pending.clear();
}

// persistent grid: resident workgroups x CUs x grid_scale, capped by the units
int persistent_grid(negf_workspace* w, const void* func, size_t dyn, long long units) {
    int per_cu = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, func, 64, dyn) != hipSuccess || per_cu < 1) per_cu = 1;
    const long long g = (long long)per_cu * std::max(1, w->cus) * std::max(1, w->grid_scale);
    return (int)std::max<long long>(1, std::min<long long>(g, units));
}

struct JobPlan {
    negf_device* d;
    int ne;
    size_t o_node, o_sigma, o_gr, o_ad, o_part;   // element offsets in the workspace arrays
};

// Enqueues one solve of all jobs on stream s.  All job pointers are device pointers.
negf_status enqueue(negf_workspace* w, int n_jobs, const negf_job* jobs, hipStream_t s, bool decimation_only) {
    HIPCHK(hipSetDevice(w->dev_id));
    // a solve on another stream starts after the previous one (shared arrays)
    if (!w->capturing) HIPCHK(hipStreamWaitEvent(s, w->done, 0));
    if (w->arena) {   // every buffer is placed afresh in the fixed area
        DBuf* bufs[] = {&w->tables, &w->counters, &w->z,       &w->sigma,   &w->iters, &w->status,
                        &w->coef_c, &w->coef_r,   &w->T,       &w->gr,      &w->ad,    &w->part, &w->Trl, &w->amax,
                        &w->store_f, &w->store_b, &w->scratch, &w->flags, &w->fp64_spans, &w->fp64_first,
                        &w->fp64_all, &w->fp64_ctl, &w->cscale};
        for (DBuf* b : bufs) *b = DBuf{};
        w->arena_off = 0;
        w->last_tables.clear();
    }
    // ---- per-job array layout
    std::vector<JobPlan> plan(n_jobs);
    size_t nodes = 0, sig = 0, gr64 = 0, gr32 = 0, ad = 0, part = 0;
    int max_ne = 0, max_nb = 0;
    w->last_max_iter.assign(n_jobs, 0);
    for (int i = 0; i < n_jobs; ++i) {
        negf_device* d = jobs[i].dev;
        const int ncz = jobs[i].n_c + jobs[i].n_poles;   // contour-type nodes: given + poles
        const int ne = ncz + jobs[i].n_r;
        const size_t Nb = (size_t)d->N * d->b, b2 = (size_t)d->b * d->b;
        JobPlan& p = plan[i];
        p.d = d;
        p.ne = ne;
        p.o_node = nodes;
        p.o_sigma = sig;
        p.o_part = part;
        size_t& gr = d->opt.precision == NEGF_FP32_BULK ? gr32 : gr64;
        p.o_gr = gr;
        p.o_ad = ad;
        gr += (size_t)ncz * Nb;
        ad += (size_t)jobs[i].n_r * 2 * Nb;
        nodes += ne;
        if (!jobs[i].sigma_mode) sig += (size_t)ne * 2 * b2;   // otherwise the job's own cache holds them
        part += (size_t)negf::RED_SEGS * Nb;
        max_ne = std::max(max_ne, ne);
        max_nb = std::max(max_nb, (int)Nb);
        w->last_max_iter[i] = d->opt.decim_max_iter;
    }
    TRY(grow(w, w->z, nodes * 16));
    TRY(grow(w, w->sigma, sig * 16));
    TRY(grow(w, w->iters, nodes * 2 * 4));
    TRY(grow(w, w->status, nodes * 4));
    TRY(grow(w, w->coef_c, nodes * 16));
    TRY(grow(w, w->coef_r, nodes * 4 * 8));
    TRY(grow(w, w->T, nodes * 8));
    TRY(grow(w, w->Trl, nodes * 8));
    TRY(grow(w, w->amax, nodes * 2 * 8));
    TRY(grow(w, w->gr, gr64 * 16 + gr32 * 8));   // FP64 jobs first, FP32 jobs behind them
    TRY(grow(w, w->ad, ad * 8));                   // A_L, A_R diagonals are FP64 in both forms
    TRY(grow(w, w->part, part * 8));
    TRY(grow(w, w->flags, (size_t)n_jobs * kFlagInts * 4));
    if (n_jobs > w->cap_flags) {
        if (w->capturing) return fail(NEGF_EINVAL, "graph capture needs a workspace sized by an eager solve");
        if (w->arena) return fail(NEGF_EINVAL, "allocation-free solve: more jobs than status slots");
        TRY(wait_prev(w));
        if (w->h_flags) (void)hipHostFree(w->h_flags);
        w->h_flags = nullptr;
        w->cap_flags = 0;
        HIPCHK(hipHostMalloc((void**)&w->h_flags, (size_t)n_jobs * kFlagInts * sizeof(int), hipHostMallocDefault));
        w->cap_flags = n_jobs;
    }
    char* gr_base = static_cast<char*>(w->gr.p);
    char* ad_base = static_cast<char*>(w->ad.p);

    std::vector<negf::JobDesc> jd(n_jobs);
    std::vector<negf::RedJob> rj(n_jobs);
    for (int i = 0; i < n_jobs; ++i) {
        const JobPlan& p = plan[i];
        const negf_job& J = jobs[i];
        negf_device* d = p.d;
        const bool f32 = d->opt.precision == NEGF_FP32_BULK;
        negf::JobDesc& D = jd[i];
        D.N = d->N;
        D.n_c = J.n_c + J.n_poles;
        D.n_r = J.n_r;
        D.K = d->K;
        D.n_uniq = d->n_uniq;
        D.hdiag_zero = d->hdiag_zero ? 1 : 0;
        D.U = d->d_U;
        D.hdiag = d->d_hdiag;
        D.ell_map = d->d_ell_map;
        D.cidx = d->d_cidx;
        D.cval = d->d_cval;
        D.ridx = d->d_ridx;
        D.rval = d->d_rval;
        D.z = static_cast<cx<double>*>(w->z.p) + p.o_node;
        D.sigma = J.sigma_mode ? reinterpret_cast<cx<double>*>(J.sigma_cache)
                               : static_cast<cx<double>*>(w->sigma.p) + p.o_sigma;
        D.gr_diag = f32 ? (void*)(gr_base + gr64 * 16 + p.o_gr * 8) : (void*)(gr_base + p.o_gr * 16);
        D.a_diag = (void*)(ad_base + p.o_ad * 8);
        D.Tout = J.T ? J.T : static_cast<double*>(w->T.p) + p.o_node;
        D.Trl = static_cast<double*>(w->Trl.p) + p.o_node;
        D.amax = static_cast<double*>(w->amax.p) + 2 * p.o_node;
        D.iters = static_cast<int*>(w->iters.p) + 2 * p.o_node;
        D.status = static_cast<int*>(w->status.p) + p.o_node;
        D.n_fp64 = static_cast<int*>(w->flags.p) + kFlagInts * i + 2;
        D.hnorm = d->hnorm;
        D.fp64_policy = w->fp64_policy;
        for (int l = 0; l < 2; ++l) {
            D.period[l] = d->lead[l].period;
            D.D[l] = d->lead[l].D;
            D.V[l] = d->lead[l].V;
            D.VH[l] = d->lead[l].VH;
            D.W[l] = d->lead[l].W;
            D.tau[l] = d->lead[l].tau;
            D.lmodes[l] = d->lead[l].circ ? d->lead[l].modes : nullptr;
        }
        D.sigma_circ = (D.lmodes[0] && D.lmodes[1] && w->circ_decimation) ? 1 : 0;
        negf::RedJob& R = rj[i];
        R.Nb = d->N * d->b;
        R.n_c = J.n_c + J.n_poles;
        R.n_ci = J.n_c;
        R.n_p = J.n_poles;
        R.no_fermi = J.contour_no_fermi ? 1 : 0;
        R.conductance = J.conductance;
        R.n_r = J.n_r;
        R.g_s = d->opt.g_s;
        R.eta = d->opt.eta;
        R.mu_L = J.bias.mu_L;
        R.mu_R = J.bias.mu_R;
        R.kT_L = J.bias.kT_L;
        R.kT_R = J.bias.kT_R;
        R.z_c = reinterpret_cast<const cx<double>*>(J.z_c);
        R.w_c = reinterpret_cast<const cx<double>*>(J.w_c);
        R.E_r = J.E_r;
        R.w_r = J.w_r;
        R.z = static_cast<cx<double>*>(w->z.p) + p.o_node;
        R.coef_c = static_cast<cx<double>*>(w->coef_c.p) + p.o_node;
        R.coef_r = static_cast<double*>(w->coef_r.p) + 4 * p.o_node;
        R.gr_diag = D.gr_diag;
        R.a_diag = D.a_diag;
        R.T = D.Tout;
        R.part = static_cast<double*>(w->part.p) + p.o_part;
        R.charge = J.charge;
        R.current = J.current;
        R.status = D.status;
        R.flags = static_cast<int*>(w->flags.p) + kFlagInts * i;
    }

    // ---- groups: jobs sharing kernels (ring size, precision, decimation limits),
    // longest chains first inside a group so that the long units start early
    struct Group {
        const negf::Launchers* L;
        bool f32;
        double tol;
        int maxit;
        std::vector<int> ids;
    };
    std::vector<Group> groups;
    std::vector<int> order(n_jobs);
    std::iota(order.begin(), order.end(), 0);
    if (w->order == 0)
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return plan[a].d->N > plan[b].d->N; });
    for (int i : order) {
        negf_device* d = plan[i].d;
        const bool f32 = d->opt.precision == NEGF_FP32_BULK;
        Group* g = nullptr;
        for (auto& x : groups)
            if (x.L == d->L && x.f32 == f32 && x.tol == d->opt.decim_tol && x.maxit == d->opt.decim_max_iter) g = &x;
        if (!g) {
            groups.push_back({d->L, f32, d->opt.decim_tol, d->opt.decim_max_iter, {}});
            g = &groups.back();
        }
        g->ids.push_back(i);
    }

    // ---- schedules: spans and unit prefixes of every launch
    struct Launch {
        int kind, kt, group;
        size_t span_at, first_at;
        int n_spans, sides, side0;
        long long units;
        size_t dyn;
        int fp64;        // 1: k_fp64_list over a group's column spans; 3: one recomputation round;
                         // 2: a launch over the round's node list
        long long cap;   // fp64 == 1: offset of the group's node list; 3: FP64 store elements (< 0: last round)
        int gpw;         // nodes (or items) per unit
    };
    std::vector<int> nfirsts;       // node prefixes of the column spans of k_fp64_list launches
    std::vector<std::vector<negf::Span>> gcol(groups.size());   // FP32 groups: every column span
    std::vector<size_t> gdyn64(groups.size(), 0);
    size_t fp64_all = 0, fp64_max = 0, node64_max = 0;
    std::vector<negf::Span> spans;
    std::vector<int> firsts;
    std::vector<Launch> launches;
    auto add_launch = [&](int kind, int kt, int gidx, const std::vector<negf::Span>& sp, int sides, int side0,
                          int G, bool items, size_t dyn) -> negf_status {
        if (sp.empty()) return NEGF_OK;
        Launch L{kind, kt, gidx, spans.size(), firsts.size(), (int)sp.size(), sides, side0, 0, dyn, 0, 0, G};
        long long acc = 0;
        for (const auto& x : sp) {
            firsts.push_back((int)acc);
            const long long work = items ? (long long)x.cnt * jd[x.job].N : x.cnt;
            acc += sides * ((work + G - 1) / G);
            if (acc > (1LL << 30)) return fail(NEGF_EINVAL, "too many work units in one launch");
            spans.push_back(x);
        }
        firsts.push_back((int)acc);
        L.units = acc;
        launches.push_back(L);
        return NEGF_OK;
    };

    size_t scratch_need = 16, store_need = 0;
    std::vector<int> dec_grid_cap(groups.size(), 0);   // dense one-ring decimation: workgroups its state is sized for
    size_t store_cap = w->store_cap ? w->store_cap : w->default_store_cap;
    // Arena mode: what is left after the per-node arrays, less a reserve for the
    // decimation state, the tables and the counters, is split between the two
    // recursion stores; a dense one-ring decimation runs on fewer workgroups so
    // that its state fits the reserve.
    size_t dec_budget = 0;
    if (w->arena) {
        size_t ne_all = 0;
        for (int i = 0; i < n_jobs; ++i) ne_all += (size_t)plan[i].ne;
        dec_budget = (size_t)16 << 20;
        const size_t tab_bound = (size_t)n_jobs * (sizeof(negf::JobDesc) + sizeof(negf::RedJob)) +
                                 (8 * ne_all + 16 * (size_t)n_jobs + 64) * (sizeof(negf::Span) + 2 * sizeof(int)) +
                                 16 * 256;
        const size_t used = (w->arena_off + 255) & ~size_t(255);
        const size_t reserve = dec_budget + tab_bound;
        const size_t left = w->arena_cap > used + reserve ? w->arena_cap - used - reserve : 0;
        store_cap = (left / 2) & ~size_t(255);
    }
    for (int gi = 0; gi < (int)groups.size(); ++gi) {
        Group& g = groups[gi];
        const int B = g.L->B, G = g.L->groups;
        const int gpw = w->gpw_b[B] > 0 ? std::min(w->gpw_b[B], G) : G;   // chains per wavefront
        const size_t cb = g.f32 ? 8 : 16;   // bytes per store element
        // bytes of store reserved per element: with every real node recomputed in
        // FP64 the FP32 chunk's store must hold all of them in FP64
        const size_t cbs = cb;
        // a1: decimation at every node.  One-ring and two-ring principal layers
        // have their own kernels; a job whose leads share the layer size runs
        // both leads in one span (sides 2), otherwise each lead in its own launch.
        {
            std::vector<negf::Span> sp[2][3];   // [period - 1][both, left only, right only]
            std::vector<negf::Span> sp_circ;      // both leads ring-circulant: mode-basis doubling
            for (int j : g.ids) {
                if (jobs[j].sigma_mode == 2) continue;   // cached self-energies
                if (jd[j].lmodes[0] && jd[j].lmodes[1] && w->circ_decimation) {
                    sp_circ.push_back({j, 0, plan[j].ne, 0, 0});
                    continue;
                }
                const int p0 = jd[j].period[0], p1 = jd[j].period[1];
                if (p0 == p1) {
                    sp[p0 - 1][0].push_back({j, 0, plan[j].ne, 0, 0});
                } else {
                    sp[p0 - 1][1].push_back({j, 0, plan[j].ne, 0, 0});
                    sp[p1 - 1][2].push_back({j, 0, plan[j].ne, 0, 0});
                }
            }
            TRY(add_launch(negf::KIND_DECIMATE_CIRC, KT_DECIMATE, gi, sp_circ, 2, 0, G, false, 0));
            for (int P = 1; P <= 2; ++P) {
                const int kind = P == 1 ? negf::KIND_DECIMATE : negf::KIND_DECIMATE2;
                const int Gd = P == 1 ? G : 64 / (2 * B);
                if (P == 1 && (!sp[0][0].empty() || !sp[0][1].empty() || !sp[0][2].empty())) {
                    int gdec = persistent_grid(w, g.L->func[kind], 0, 1LL << 40);
                    const size_t per_wg = (size_t)G * 4 * B * B * 16;
                    if (w->arena) gdec = (int)std::max<size_t>(1, std::min<size_t>(gdec, dec_budget / per_wg));
                    dec_grid_cap[gi] = gdec;
                    scratch_need = std::max(scratch_need, (size_t)gdec * per_wg);
                }
                for (int m = 0; m < 3; ++m)
                    TRY(add_launch(kind, KT_DECIMATE, gi, sp[P - 1][m], m == 0 ? 2 : 1, m == 2 ? 1 : 0, Gd, false,
                                   0));
            }
        }
        if (decimation_only) continue;
        // a3-a5: chunks of nodes whose recursion store fits the cap
        size_t dyn = 0;
        for (int j : g.ids) {
            dyn = std::max(dyn, (size_t)jd[j].n_uniq * B * jd[j].K * (cb + 1));
            gdyn64[gi] = std::max(gdyn64[gi], (size_t)jd[j].n_uniq * B * jd[j].K * 17);
        }
        size_t ji = 0;
        int e_at = 0;
        while (ji < g.ids.size()) {
            std::vector<negf::Span> rec, cdg, col;
            size_t used = 0;   // store elements (cx<T>) of this chunk
            while (ji < g.ids.size()) {
                const int j = g.ids[ji];
                const size_t per = (size_t)jd[j].N * B * B;
                const long long fit = (long long)((store_cap / cbs - used) / per);
                if (fit <= 0) {
                    if (used == 0) {
                        if (w->arena)
                            return fail(NEGF_EINVAL,
                                        "the static scratch area (%zu bytes) cannot hold one node's recursion "
                                        "stores (2 x %zu bytes) next to the per-node arrays",
                                        w->arena_cap, per * cb);
                        return fail(NEGF_ENOMEM, "one node's recursion store (%zu bytes) exceeds the store cap",
                                    per * cb);
                    }
                    break;
                }
                const int take = (int)std::min<long long>(fit, plan[j].ne - e_at);
                rec.push_back({j, e_at, take, 0, (long long)used});
                const int c_hi = std::min(e_at + take, jd[j].n_c);
                if (c_hi > e_at) cdg.push_back({j, e_at, c_hi - e_at, 0, (long long)used});
                const int r_lo = std::max(e_at, jd[j].n_c), r_hi = e_at + take;
                if (r_hi > r_lo)
                    col.push_back({j, r_lo, r_hi - r_lo, 0, (long long)(used + (size_t)(r_lo - e_at) * per)});
                used += (size_t)take * per;
                e_at += take;
                if (e_at >= plan[j].ne) {
                    ++ji;
                    e_at = 0;
                }
            }
            store_need = std::max(store_need, used * cbs);
            // ring size 1: the column kernel runs a real node's recursions itself and the
            // recursion kernel a contour node's (both without stores between checkpoints),
            // so the recursion launch covers the contour nodes only
            TRY(add_launch(g.f32 ? negf::KIND_RECUR32 : negf::KIND_RECUR64, KT_RECUR, gi, B == 1 ? cdg : rec, 2, 0,
                           gpw, false, dyn));
            if (B != 1)   // ring size 1: the recursion kernel writes the contour diagonals itself
                TRY(add_launch(g.f32 ? negf::KIND_CDIAG32 : negf::KIND_CDIAG64, KT_CDIAG, gi, cdg, 1, 0, gpw, true,
                               0));
            TRY(add_launch(g.f32 ? negf::KIND_COLUMN32 : negf::KIND_COLUMN64, KT_COLUMN, gi, col, 2, 0, gpw, false,
                           0));
            if (g.f32) gcol[gi].insert(gcol[gi].end(), col.begin(), col.end());
        }
    }
    // FP32-bulk: after every group's chunks, the real-axis nodes whose FP32 results
    // are doubtful are recomputed in FP64 in the (now free) recursion stores, in
    // rounds of what the stores hold.  The rounds cover a quarter of the real-axis
    // nodes' FP64 stores (all of them when every node is recomputed); nodes beyond
    // that are an error.
    std::vector<size_t> gall(groups.size(), 0);   // offset of each group's node list
    for (int gi = 0; gi < (int)groups.size(); ++gi) {
        if (gcol[gi].empty()) continue;
        const int B = groups[gi].L->B;
        long long nreal = 0;
        for (const auto& x : gcol[gi]) {
            nreal += x.cnt;
            node64_max = std::max(node64_max, (size_t)jd[x.job].N * B * B * 16);
        }
        gall[gi] = fp64_all;
        fp64_all += (size_t)nreal;
        fp64_max = std::max(fp64_max, (size_t)nreal);
    }
    store_need = std::max(store_need, node64_max);
    const long long cap64 = (long long)(store_need / 16);
    for (int gi = 0; gi < (int)groups.size(); ++gi) {
        if (gcol[gi].empty()) continue;
        const int B = groups[gi].L->B;
        double elems = 0.0;
        long long nreal = 0;
        Launch LL{negf::KIND_COUNT, KT_FP64, gi, spans.size(), nfirsts.size(), (int)gcol[gi].size(), 1, 0, 0, 0, 1,
                  (long long)gall[gi], 1};
        for (const auto& x : gcol[gi]) {
            nfirsts.push_back((int)nreal);
            nreal += x.cnt;
            elems += (double)x.cnt * jd[x.job].N * B * B;
            spans.push_back(x);
        }
        nfirsts.push_back((int)nreal);
        LL.units = nreal;
        launches.push_back(LL);
        const double frac = w->fp64_policy == 1 ? 1.0 : 0.25;
        const long long per = (long long)(store_need / 16) - (long long)(node64_max / 16);   // fill guaranteed per round
        const int rounds = 1 + (int)std::ceil(frac * elems / (double)std::max<long long>(per, 1));
        for (int r = 0; r < rounds; ++r) {
            launches.push_back(Launch{negf::KIND_COUNT, KT_FP64, gi, 0, 0, (int)nreal, 1, 0, nreal, 0, 3,
                                      r == rounds - 1 ? -cap64 : cap64, 1});
            if (B != 1)   // ring size 1: the column kernel recomputes the recursions itself
                launches.push_back(
                    Launch{negf::KIND_RECUR64, KT_FP64, gi, 0, 0, (int)nreal, 2, 0, 2 * nreal, gdyn64[gi], 2, 0, 1});
            launches.push_back(Launch{negf::KIND_COLUMN64, KT_FP64, gi, 0, 0, (int)nreal, 2, 0, 2 * nreal, 0, 2, 0, 1});
        }
    }
    TRY(grow(w, w->scratch, scratch_need));
    if (store_need) {
        TRY(grow(w, w->store_f, store_need));
        TRY(grow(w, w->store_b, store_need));
    }
    const size_t n_counters = std::max<size_t>(1, launches.size());
    TRY(grow(w, w->counters, n_counters * 4));
    if (fp64_max) {
        TRY(grow(w, w->fp64_all, fp64_all * sizeof(negf::Span)));
        TRY(grow(w, w->fp64_spans, fp64_max * sizeof(negf::Span)));
        TRY(grow(w, w->fp64_first, (fp64_max + 1) * sizeof(int)));
        TRY(grow(w, w->fp64_ctl, groups.size() * 2 * sizeof(int)));
        TRY(grow(w, w->cscale, (size_t)n_jobs * sizeof(double)));
    }

    // ---- tables: one image [JobDesc][RedJob][Span][first], uploaded only when it
    // differs from the last one (repeated solves of the same jobs upload nothing)
    std::vector<char> img;
    auto put = [&](const void* src, size_t bytes) {
        const size_t at = (img.size() + 15) & ~size_t(15);
        img.resize(at + bytes);
        if (bytes) memcpy(img.data() + at, src, bytes);
        return at;
    };
    const size_t o_jd = put(jd.data(), jd.size() * sizeof(negf::JobDesc));
    const size_t o_rj = put(rj.data(), rj.size() * sizeof(negf::RedJob));
    const size_t o_sp = put(spans.data(), spans.size() * sizeof(negf::Span));
    const size_t o_fi = put(firsts.data(), firsts.size() * sizeof(int));
    const size_t o_nf = put(nfirsts.data(), nfirsts.size() * sizeof(int));
    if (img != w->last_tables || !w->tables.p) {
        if (w->capturing) return fail(NEGF_EINVAL, "graph capture: job tables differ from the eager solve");
        TRY(grow(w, w->tables, img.size()));
        TRY(wait_prev(w));
        HIPCHK(hipMemcpy(w->tables.p, img.data(), img.size(), hipMemcpyHostToDevice));
        w->last_tables.swap(img);
    }
    char* tab = static_cast<char*>(w->tables.p);
    const negf::JobDesc* d_jobs = reinterpret_cast<const negf::JobDesc*>(tab + o_jd);
    const negf::RedJob* d_red = reinterpret_cast<const negf::RedJob*>(tab + o_rj);
    const negf::Span* d_spans = reinterpret_cast<const negf::Span*>(tab + o_sp);
    const int* d_first = reinterpret_cast<const int*>(tab + o_fi);
    const int* d_nfirst = reinterpret_cast<const int*>(tab + o_nf);
    negf::Span* d_fp64_spans = static_cast<negf::Span*>(w->fp64_spans.p);
    int* d_fp64_first = static_cast<int*>(w->fp64_first.p);
    negf::Span* d_fp64_all = static_cast<negf::Span*>(w->fp64_all.p);
    int* d_fp64_ctl = static_cast<int*>(w->fp64_ctl.p);   // per group: listed nodes, cursor

    hipEvent_t ev;
    ev_begin(w, s, &ev);
    hipLaunchKernelGGL(negf::k_fill_int, dim3((unsigned)((n_counters + 255) / 256)), dim3(256), 0, s,
                       static_cast<int*>(w->counters.p), (int)n_counters, 0);
    hipLaunchKernelGGL(negf::k_nodes, dim3((max_ne + 255) / 256, n_jobs), dim3(256), 0, s, d_red,
                       static_cast<int*>(w->status.p), (int)nodes);
    ev_end(w, KT_REDUCE, s, ev);

    const negf::Span* cur_all = nullptr;   // node list of the group being recomputed
    bool side_open = false;                 // a contour-diagonal launch on the side stream is not joined yet
    bool cscale_done = false;
    for (size_t li = 0; li < launches.size(); ++li) {
        const Launch& L = launches[li];
        const Group& g = groups[L.group];
        const bool to_side = w->side && !L.fp64 && (L.kind == negf::KIND_CDIAG64 || L.kind == negf::KIND_CDIAG32);
        const bool beside = !L.fp64 && (L.kind == negf::KIND_COLUMN64 || L.kind == negf::KIND_COLUMN32);
        if (side_open && !beside) {   // nothing but the chunk's lead columns runs beside the diagonals
            HIPCHK(hipStreamWaitEvent(s, w->ev_join, 0));
            side_open = false;
        }
        if (L.fp64 == 1) {   // list of the group's nodes to recompute; the cursor is reset
            int* ctl = d_fp64_ctl + 2 * L.group;
            hipLaunchKernelGGL(negf::k_fill_int, dim3(1), dim3(64), 0, s, ctl + 1, 1, 0);
            if (!cscale_done) {   // every job's lead columns are done: its current scale
                hipLaunchKernelGGL(negf::k_cur_scale, dim3(n_jobs), dim3(64), 0, s, d_jobs, d_red,
                                   static_cast<double*>(w->cscale.p));
                cscale_done = true;
            }
            hipLaunchKernelGGL(negf::k_fp64_list, dim3(1), dim3(1024), 0, s, d_jobs, d_red, d_spans + L.span_at,
                               d_nfirst + L.first_at, L.n_spans, g.L->B, d_fp64_all + L.cap, ctl,
                               static_cast<const double*>(w->cscale.p));
            cur_all = d_fp64_all + L.cap;
            continue;
        }
        if (L.fp64 == 3) {   // the next round of the list that fits the stores
            int* ctl = d_fp64_ctl + 2 * L.group;
            hipLaunchKernelGGL(negf::k_fp64_round, dim3(1), dim3(1024), 0, s, d_jobs, cur_all, ctl, ctl + 1, g.L->B,
                               L.cap < 0 ? -L.cap : L.cap, d_fp64_spans, d_fp64_first, L.n_spans, L.cap < 0 ? 1 : 0);
            continue;
        }
        negf::Sched S{};
        S.jobs = d_jobs;
        S.spans = L.fp64 ? d_fp64_spans : d_spans + L.span_at;
        S.first = L.fp64 ? d_fp64_first : d_first + L.first_at;
        S.n_spans = L.n_spans;
        S.sides = L.sides;
        S.side0 = L.side0;
        S.counter = static_cast<int*>(w->counters.p) + li;
        S.store_f = w->store_f.p;
        S.store_b = w->store_b.p;
        S.scratch = static_cast<cx<double>*>(w->scratch.p);
        S.tol = g.tol;
        S.maxit = g.maxit;
        S.gpw = L.gpw;
        S.lane_spans = (L.fp64 == 2 && g.L->B == 1 && L.kind == negf::KIND_COLUMN64) ? 1 : 0;
        int grid = persistent_grid(w, g.L->func[L.kind], L.dyn, L.units);
        if (L.kind == negf::KIND_DECIMATE && dec_grid_cap[L.group] > 0) grid = std::min(grid, dec_grid_cap[L.group]);
        hipStream_t ls = s;
        if (to_side) {   // fork: the side stream waits for the recursion of this chunk
            HIPCHK(hipEventRecord(w->ev_fork, s));
            HIPCHK(hipStreamWaitEvent(w->side, w->ev_fork, 0));
            ls = w->side;
        }
        ev_begin(w, ls, &ev);
        g.L->launch[L.kind](S, grid, L.dyn, ls);
        ev_end(w, L.kt, ls, ev);
        if (to_side) {
            HIPCHK(hipEventRecord(w->ev_join, w->side));
            side_open = true;
        } else if (side_open) {   // the lead columns are queued: join behind them
            HIPCHK(hipStreamWaitEvent(s, w->ev_join, 0));
            side_open = false;
        }
    }
    if (side_open) HIPCHK(hipStreamWaitEvent(s, w->ev_join, 0));

    // ---- a6: weighted energy sums (status folded into the flags by k_coef)
    ev_begin(w, s, &ev);
    hipLaunchKernelGGL(negf::k_coef, dim3((max_ne + 255) / 256, n_jobs), dim3(256), 0, s, d_red);
    if (!decimation_only) {
        // one launch per run of consecutive jobs in the same precision (blockIdx.z: job in the run)
        for (int i = 0; i < n_jobs;) {
            const bool f32 = plan[i].d->opt.precision == NEGF_FP32_BULK;
            int k = i, bx = 1;
            while (k < n_jobs && k - i < 65535 && (plan[k].d->opt.precision == NEGF_FP32_BULK) == f32) {
                bx = std::max(bx, (plan[k].d->N * plan[k].d->b + 255) / 256);
                ++k;
            }
            const dim3 rgrid((unsigned)bx, negf::RED_SEGS, (unsigned)(k - i));
            if (f32)
                hipLaunchKernelGGL((negf::k_reduce_part<float, double>), rgrid, dim3(256), 0, s, d_red + i);
            else
                hipLaunchKernelGGL((negf::k_reduce_part<double, double>), rgrid, dim3(256), 0, s, d_red + i);
            i = k;
        }
        hipLaunchKernelGGL(negf::k_reduce_final, dim3((max_nb + 255) / 256, n_jobs), dim3(256), 0, s, d_red);
        hipLaunchKernelGGL(negf::k_current, dim3(n_jobs), dim3(64), 0, s, d_red);
    }
    ev_end(w, KT_REDUCE, s, ev);
    HIPCHK(hipMemcpyAsync(w->h_flags, w->flags.p, (size_t)n_jobs * kFlagInts * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipGetLastError());
    if (!w->capturing) HIPCHK(hipEventRecord(w->done, s));
    w->last_n_jobs = n_jobs;
    return NEGF_OK;
}

negf_status finish(negf_workspace* w, int* failed_job) {
    if (failed_job) *failed_job = -1;
    TRY(wait_prev(w));
    ev_collect(w);
    const int n = w->last_n_jobs;
    w->last_n_jobs = 0;
    w->last_fp64.assign(n, 0);
    for (int j = 0; j < n; ++j) w->last_fp64[j] = w->h_flags[kFlagInts * j + 2];
    for (int j = 0; j < n; ++j) {
        const int fl = w->h_flags[kFlagInts * j];
        if (!fl) continue;
        if (failed_job) *failed_job = j;
        const int node = w->h_flags[kFlagInts * j + 1];
        if (fl & negf::ST_NOCONV)
            return fail(NEGF_ENOCONV, "job %d: lead decimation did not converge in %d steps (first node %d)", j,
                        w->last_max_iter[j], node);
        if (fl & negf::ST_NOROOM)
            return fail(NEGF_ESINGULAR,
                        "job %d: FP32-bulk: more real-axis nodes need FP64 recomputation than the recursion store "
                        "holds (first node %d); solve this job in FP64",
                        j, node);
        return fail(NEGF_ESINGULAR,
                    "job %d: non-finite or impossible output at node %d (negative spectral density, T outside [0, "
                    "b], or a non-finite charge or current)",
                    j, node);
    }
    return NEGF_OK;
}

negf_status ws_create(negf_workspace** out, size_t store_bytes) {
    negf_workspace* w = new negf_workspace();
    w->store_cap = store_bytes;
    hipDeviceProp_t prop;
    if (hipGetDevice(&w->dev_id) != hipSuccess || hipGetDeviceProperties(&prop, w->dev_id) != hipSuccess) {
        delete w;
        return fail(NEGF_EHIP, "no HIP device");
    }
    w->cus = prop.multiProcessorCount;
    // default recursion-store cap per direction: 30 % of the free HBM at creation,
    // between 8 and 64 GiB, so that long batches run in few large chunks
    {
        size_t fr = 0, tot = 0;
        w->default_store_cap = kDefaultStoreCap;
        if (hipMemGetInfo(&fr, &tot) == hipSuccess)
            w->default_store_cap = std::min<size_t>((size_t)64 << 30, std::max<size_t>(kDefaultStoreCap, fr / 10 * 3));
    }
    if (hipStreamCreateWithFlags(&w->own_stream, hipStreamNonBlocking) != hipSuccess) {
        delete w;
        return fail(NEGF_EHIP, "stream creation failed");
    }
    if (hipEventCreateWithFlags(&w->done, hipEventDisableTiming) != hipSuccess) {
        (void)hipStreamDestroy(w->own_stream);
        delete w;
        return fail(NEGF_EHIP, "event creation failed");
    }
    if (hipStreamCreateWithFlags(&w->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&w->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&w->ev_join, hipEventDisableTiming) != hipSuccess) {
        if (w->ev_fork) (void)hipEventDestroy(w->ev_fork);
        if (w->side) (void)hipStreamDestroy(w->side);
        (void)hipEventDestroy(w->done);
        (void)hipStreamDestroy(w->own_stream);
        delete w;
        return fail(NEGF_EHIP, "side stream creation failed");
    }
    if (hipHostMalloc((void**)&w->h_flags, kFlagInts * sizeof(int), hipHostMallocDefault) != hipSuccess) {
        (void)hipEventDestroy(w->ev_join);
        (void)hipEventDestroy(w->ev_fork);
        (void)hipStreamDestroy(w->side);
        (void)hipEventDestroy(w->done);
        (void)hipStreamDestroy(w->own_stream);
        delete w;
        return fail(NEGF_ENOMEM, "pinned flag buffer");
    }
    w->cap_flags = 1;
    for (int k = 0; k < kFlagInts; ++k) w->h_flags[k] = 0;
    *out = w;
    return NEGF_OK;
}

void ws_destroy(negf_workspace* w) {
    if (!w) return;
    (void)hipSetDevice(w->dev_id);
    (void)hipEventSynchronize(w->done);
    for (auto& e : w->pending) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    DBuf* bufs[] = {&w->tables, &w->counters, &w->z,       &w->sigma,  &w->iters,      &w->status,
                    &w->coef_c, &w->coef_r,   &w->T,       &w->gr,     &w->ad,         &w->part, &w->Trl, &w->amax,
                    &w->store_f, &w->store_b, &w->scratch, &w->flags,  &w->in_zc,      &w->in_wc, &w->fp64_spans, &w->fp64_first, &w->fp64_all, &w->fp64_ctl, &w->cscale,
                    &w->in_Er,  &w->in_wr,    &w->out_charge, &w->out_T, &w->out_cur};
    for (DBuf* b : bufs)
        if (b->p) (void)hipFree(b->p);
    if (w->h_flags) (void)hipHostFree(w->h_flags);
    if (w->done) (void)hipEventDestroy(w->done);
    if (w->ev_join) (void)hipEventDestroy(w->ev_join);
    if (w->ev_fork) (void)hipEventDestroy(w->ev_fork);
    if (w->side) (void)hipStreamDestroy(w->side);
    if (w->own_stream) (void)hipStreamDestroy(w->own_stream);
    delete w;
}

// Host-pointer batch: stage the inputs, solve on the workspace stream, copy the
// outputs back.  `outs` (optional, single-job calls only) receives the
// energy-resolved arrays of job 0.
negf_status solve_host(negf_workspace* w, int n_jobs, const negf_job* jobs, const negf_outputs* outs) {
    HIPCHK(hipSetDevice(w->dev_id));
    size_t nc = 0, nr = 0, nb = 0;
    for (int i = 0; i < n_jobs; ++i) {
        nc += jobs[i].n_c;
        nr += jobs[i].n_r;
        nb += (size_t)jobs[i].dev->N * jobs[i].dev->b;
    }
    TRY(grow(w, w->in_zc, nc * 16));
    TRY(grow(w, w->in_wc, nc * 16));
    TRY(grow(w, w->in_Er, nr * 8));
    TRY(grow(w, w->in_wr, nr * 8));
    TRY(grow(w, w->out_charge, nb * 8));
    TRY(grow(w, w->out_T, nr * 8));
    TRY(grow(w, w->out_cur, (size_t)n_jobs * 2 * 8));   // current, conductance
    hipStream_t s = w->own_stream;
    std::vector<negf_job> dj(jobs, jobs + n_jobs);
    size_t oc = 0, orr = 0, ob = 0;
    for (int i = 0; i < n_jobs; ++i) {
        negf_job& j = dj[i];
        negf_c64* zc = static_cast<negf_c64*>(w->in_zc.p) + oc;
        negf_c64* wc = static_cast<negf_c64*>(w->in_wc.p) + oc;
        double* Er = static_cast<double*>(w->in_Er.p) + orr;
        double* wr = static_cast<double*>(w->in_wr.p) + orr;
        if (j.n_c) {
            HIPCHK(hipMemcpy(zc, jobs[i].z_c, (size_t)j.n_c * 16, hipMemcpyHostToDevice));
            HIPCHK(hipMemcpy(wc, jobs[i].w_c, (size_t)j.n_c * 16, hipMemcpyHostToDevice));
        }
        if (j.n_r) {
            HIPCHK(hipMemcpy(Er, jobs[i].E_r, (size_t)j.n_r * 8, hipMemcpyHostToDevice));
            HIPCHK(hipMemcpy(wr, jobs[i].w_r, (size_t)j.n_r * 8, hipMemcpyHostToDevice));
        }
        j.z_c = zc;
        j.w_c = wc;
        j.E_r = Er;
        j.w_r = wr;
        j.charge = static_cast<double*>(w->out_charge.p) + ob;
        j.T = static_cast<double*>(w->out_T.p) + orr;
        j.current = static_cast<double*>(w->out_cur.p) + 2 * i;
        j.conductance = jobs[i].conductance ? static_cast<double*>(w->out_cur.p) + 2 * i + 1 : nullptr;
        oc += j.n_c;
        orr += j.n_r;
        ob += (size_t)j.dev->N * j.dev->b;
    }
    TRY(enqueue(w, n_jobs, dj.data(), s));
    const negf_status st = finish(w, nullptr);
    const std::string msg = g_err;
    // outputs are copied on a device-side error status too, for inspection
    for (int i = 0; i < n_jobs; ++i) {
        const negf_job& j = dj[i];
        const size_t Nb = (size_t)j.dev->N * j.dev->b;
        HIPCHK(hipMemcpy(jobs[i].charge, j.charge, Nb * 8, hipMemcpyDeviceToHost));
        if (jobs[i].T && j.n_r) HIPCHK(hipMemcpy(jobs[i].T, j.T, (size_t)j.n_r * 8, hipMemcpyDeviceToHost));
        if (jobs[i].current) HIPCHK(hipMemcpy(jobs[i].current, j.current, 8, hipMemcpyDeviceToHost));
        if (jobs[i].conductance) HIPCHK(hipMemcpy(jobs[i].conductance, j.conductance, 8, hipMemcpyDeviceToHost));
    }
    if (outs) {   // with one job, its arrays start at offset 0 of their buffers
        negf_device* d = dj[0].dev;
        const negf_job& j = dj[0];
        const size_t Nb = (size_t)d->N * d->b;
        const bool f32 = d->opt.precision == NEGF_FP32_BULK;
        if (outs->gr_diag && j.n_c) {
            if (f32) {
                std::vector<float> tmp((size_t)j.n_c * Nb * 2);
                HIPCHK(hipMemcpy(tmp.data(), w->gr.p, tmp.size() * 4, hipMemcpyDeviceToHost));
                for (size_t i = 0; i < (size_t)j.n_c * Nb; ++i)
                    outs->gr_diag[i] = negf_c64{tmp[2 * i], tmp[2 * i + 1]};
            } else {
                HIPCHK(hipMemcpy(outs->gr_diag, w->gr.p, (size_t)j.n_c * Nb * 16, hipMemcpyDeviceToHost));
            }
        }
        if ((outs->al_diag || outs->ar_diag) && j.n_r) {
            std::vector<double> ad((size_t)j.n_r * 2 * Nb);
            HIPCHK(hipMemcpy(ad.data(), w->ad.p, ad.size() * 8, hipMemcpyDeviceToHost));
            for (int q = 0; q < j.n_r; ++q) {
                if (outs->al_diag) memcpy(outs->al_diag + (size_t)q * Nb, ad.data() + ((size_t)q * 2 + 0) * Nb, Nb * 8);
                if (outs->ar_diag) memcpy(outs->ar_diag + (size_t)q * Nb, ad.data() + ((size_t)q * 2 + 1) * Nb, Nb * 8);
            }
        }
        if (outs->T_rl && j.n_r)
            HIPCHK(hipMemcpy(outs->T_rl, w->Trl.p, (size_t)j.n_r * 8, hipMemcpyDeviceToHost));
        if (outs->decim_iters)
            HIPCHK(hipMemcpy(outs->decim_iters, w->iters.p, (size_t)(j.n_c + j.n_r) * 2 * 4, hipMemcpyDeviceToHost));
    }
    g_err = msg;
    return st;
}

negf_job make_job(negf_device* d, const negf_bias* bias, int n_c, const negf_c64* z_c, const negf_c64* w_c, int n_r,
                  const double* E_r, const double* w_r, double* charge, double* T, double* current) {
    negf_job j{};
    j.dev = d;
    if (bias) j.bias = *bias;
    j.n_c = n_c;
    j.z_c = z_c;
    j.w_c = w_c;
    j.n_r = n_r;
    j.E_r = E_r;
    j.w_r = w_r;
    j.charge = charge;
    j.T = T;
    j.current = current;
    return j;
}

negf_status check_batch(negf_workspace* w, int n_jobs, const negf_job* jobs, bool host) {
    if (!w) return fail(NEGF_EINVAL, "workspace is NULL");
    if (n_jobs < 1 || !jobs) return fail(NEGF_EINVAL, "no jobs");
    for (int i = 0; i < n_jobs; ++i) {
        TRY(check_job(jobs[i], i, host));
        if (jobs[i].dev->dev_id != w->dev_id) return fail(NEGF_EINVAL, "job %d lives on another HIP device", i);
    }
    return NEGF_OK;
}

}  // namespace negf_host

using namespace negf_host;

extern "C" {

void negf_default_options(negf_options* opt) {
    if (!opt) return;
    opt->precision = NEGF_FP64;
    opt->eta = 1e-6;
    opt->decim_tol = 1e-12;
    opt->decim_max_iter = 64;
    opt->g_s = 2.0;
    opt->workspace_bytes = 0;
}

const char* negf_last_error(void) { return g_err.c_str(); }

}  // extern "C"

negf_status negf_host::create_device(negf_device** out, int n_rings, int b, const negf_c64* h_diag,
                                     const negf_c64* h_up, const negf_lead* left, const negf_lead* right,
                                     const negf_options* opt, bool own_ws) {
    if (!out) return fail(NEGF_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_rings < 1) return fail(NEGF_EINVAL, "n_rings = %d < 1", n_rings);
    if (b < 1 || b > NEGF_MAX_RING) return fail(NEGF_EINVAL, "ring size b = %d not in [1,%d]", b, NEGF_MAX_RING);
    if ((long long)n_rings * b * b > (1LL << 31)) return fail(NEGF_EINVAL, "device too large");
    if (!h_diag) return fail(NEGF_EINVAL, "h_diag is NULL");
    if (n_rings > 1 && !h_up) return fail(NEGF_EINVAL, "h_up is NULL");
    const size_t b2 = (size_t)b * b;
    if (!finite_c(h_diag, (size_t)n_rings * b2) || (n_rings > 1 && !finite_c(h_up, (size_t)(n_rings - 1) * b2)))
        return fail(NEGF_EINVAL, "Hamiltonian has non-finite entries");
    TRY(check_lead(left, b, "left"));
    TRY(check_lead(right, b, "right"));
    negf_options o;
    negf_default_options(&o);
    if (opt) o = *opt;
    if (o.precision != NEGF_FP64 && o.precision != NEGF_FP32_BULK)
        return fail(NEGF_EINVAL, "unknown precision %d", o.precision);
    if (!(o.eta >= 0) || !std::isfinite(o.eta)) return fail(NEGF_EINVAL, "eta must be finite and >= 0");
    if (!(o.decim_tol > 0)) return fail(NEGF_EINVAL, "decim_tol must be > 0");
    if (o.decim_max_iter < 1 || o.decim_max_iter > 4096) return fail(NEGF_EINVAL, "decim_max_iter out of range");
    if (!(o.g_s > 0)) return fail(NEGF_EINVAL, "g_s must be > 0");
    const negf::Launchers* L = launchers_for(b);
    if (!L) return fail(NEGF_EINVAL, "no kernels for ring size %d", b);

    // couplings: the distinct blocks as column- and row-ELL of a common width K,
    // plus the map ring coupling -> distinct block (periodic tubes have few)
    const int nc = std::max(0, n_rings - 1);
    std::vector<int> ell_map((size_t)std::max(1, nc), 0);
    std::vector<int> uniq;   // ring index n of the first coupling of each distinct block
    for (int n = 0; n < nc; ++n) {
        const negf_c64* H = h_up + (size_t)n * b2;
        int found = -1;
        for (size_t u = 0; u < uniq.size() && found < 0; ++u)
            if (memcmp(H, h_up + (size_t)uniq[u] * b2, b2 * sizeof(negf_c64)) == 0) found = (int)u;
        if (found < 0) {
            found = (int)uniq.size();
            uniq.push_back(n);
        }
        ell_map[n] = found;
    }
    const int nu = std::max<int>(1, (int)uniq.size());
    int K = 1;
    for (int u = 0; u < (int)uniq.size(); ++u) {
        const negf_c64* H = h_up + (size_t)uniq[u] * b2;
        for (int j = 0; j < b; ++j) {
            int cc = 0, rc = 0;
            for (int l = 0; l < b; ++l) {
                if (H[(size_t)l * b + j].re != 0.0 || H[(size_t)l * b + j].im != 0.0) ++cc;
                if (H[(size_t)j * b + l].re != 0.0 || H[(size_t)j * b + l].im != 0.0) ++rc;
            }
            K = std::max(K, std::max(cc, rc));
        }
    }
    const size_t ell = (size_t)nu * b * K;
    if (ell * (sizeof(negf_c64) + 1) > 32768)
        return fail(NEGF_EINVAL, "coupling table of %d distinct blocks (width %d) exceeds the 32 KiB LDS table", nu,
                    K);

    negf_device* d = new negf_device();
    d->N = n_rings;
    d->b = b;
    d->opt = o;
    d->L = L;
    d->K = K;
    d->n_uniq = nu;
    auto bail = [&](negf_status s) {
        const std::string m = g_err;
        negf_destroy(d);
        g_err = m;
        return s;
    };
    if (hipGetDevice(&d->dev_id) != hipSuccess) return bail(fail(NEGF_EHIP, "no HIP device"));
    negf_status s;
    if (own_ws && (s = ws_create(&d->ws, o.workspace_bytes ? o.workspace_bytes / 2 : 0)) != NEGF_OK) return bail(s);

    // max row sum of |H| over the device rows (on-site block, coupling to the next
    // ring and from the previous one): the scale of M in the FP32-bulk checks
    for (int j = 0; j < n_rings; ++j)
        for (int i = 0; i < b; ++i) {
            double rs = 0.0;
            for (int k = 0; k < b; ++k) {
                rs += std::hypot(h_diag[(size_t)j * b2 + (size_t)i * b + k].re, h_diag[(size_t)j * b2 + (size_t)i * b + k].im);
                if (j + 1 < n_rings)
                    rs += std::hypot(h_up[(size_t)j * b2 + (size_t)i * b + k].re, h_up[(size_t)j * b2 + (size_t)i * b + k].im);
                if (j > 0)   // (H_{j-1,j})^H row i = conj of column i of h_up[j-1]
                    rs += std::hypot(h_up[(size_t)(j - 1) * b2 + (size_t)k * b + i].re,
                                     h_up[(size_t)(j - 1) * b2 + (size_t)k * b + i].im);
            }
            d->hnorm = std::max(d->hnorm, rs);
        }
    d->hdiag_zero = true;
    for (size_t i = 0; i < (size_t)n_rings * b2; ++i)
        if (h_diag[i].re != 0.0 || h_diag[i].im != 0.0) {
            d->hdiag_zero = false;
            break;
        }
    if ((s = dalloc(d, &d->d_hdiag, (size_t)n_rings * b2 * 16)) != NEGF_OK) return bail(s);
    if (hipMemcpy(d->d_hdiag, h_diag, (size_t)n_rings * b2 * 16, hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(NEGF_EHIP, "copy of h_diag failed"));
    if ((s = dalloc(d, &d->d_U, (size_t)n_rings * b * 8)) != NEGF_OK) return bail(s);
    if (hipMemset(d->d_U, 0, (size_t)n_rings * b * 8) != hipSuccess) return bail(fail(NEGF_EHIP, "memset U"));

    std::vector<int> cidx(ell, 0), ridx(ell, 0);
    std::vector<negf_c64> cval(ell, negf_c64{0, 0}), rval(ell, negf_c64{0, 0});
    for (int u = 0; u < (int)uniq.size(); ++u) {
        const negf_c64* H = h_up + (size_t)uniq[u] * b2;
        for (int j = 0; j < b; ++j) {
            int cc = 0, rc = 0;
            for (int l = 0; l < b; ++l) {
                const negf_c64 hc = H[(size_t)l * b + j], hr = H[(size_t)j * b + l];
                if (hc.re != 0.0 || hc.im != 0.0) {
                    cidx[((size_t)u * b + j) * K + cc] = l;
                    cval[((size_t)u * b + j) * K + cc] = hc;
                    ++cc;
                }
                if (hr.re != 0.0 || hr.im != 0.0) {
                    ridx[((size_t)u * b + j) * K + rc] = l;
                    rval[((size_t)u * b + j) * K + rc] = hr;
                    ++rc;
                }
            }
        }
    }
    if ((s = dalloc(d, &d->d_ell_map, ell_map.size() * 4)) != NEGF_OK) return bail(s);
    if ((s = dalloc(d, &d->d_cidx, ell * 4)) != NEGF_OK) return bail(s);
    if ((s = dalloc(d, &d->d_ridx, ell * 4)) != NEGF_OK) return bail(s);
    if ((s = dalloc(d, &d->d_cval, ell * 16)) != NEGF_OK) return bail(s);
    if ((s = dalloc(d, &d->d_rval, ell * 16)) != NEGF_OK) return bail(s);
    if (hipMemcpy(d->d_ell_map, ell_map.data(), ell_map.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d->d_cidx, cidx.data(), ell * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d->d_ridx, ridx.data(), ell * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d->d_cval, cval.data(), ell * 16, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d->d_rval, rval.data(), ell * 16, hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(NEGF_EHIP, "copy of couplings failed"));

    const negf_lead* leads[2] = {left, right};
    for (int l = 0; l < 2; ++l) {
        LeadDev& ld = d->lead[l];
        const negf_lead* src = leads[l];
        ld.period = src->period;
        ld.h_diag.assign(src->h_diag, src->h_diag + (size_t)src->period * b2);
        std::vector<negf_c64> V(src->h_up, src->h_up + b2), VH(b2),
            W(src->h_up + (size_t)(src->period - 1) * b2, src->h_up + (size_t)src->period * b2);
        for (int i = 0; i < b; ++i)
            for (int j = 0; j < b; ++j) {
                const negf_c64 v = V[(size_t)j * b + i];
                VH[(size_t)i * b + j] = negf_c64{v.re, -v.im};
            }
        if ((s = dalloc(d, &ld.D, (size_t)src->period * b2 * 16)) != NEGF_OK) return bail(s);
        if ((s = dalloc(d, &ld.V, b2 * 16)) != NEGF_OK) return bail(s);
        if ((s = dalloc(d, &ld.VH, b2 * 16)) != NEGF_OK) return bail(s);
        if ((s = dalloc(d, &ld.W, b2 * 16)) != NEGF_OK) return bail(s);
        if ((s = dalloc(d, &ld.tau, b2 * 16)) != NEGF_OK) return bail(s);
        if (hipMemcpy(ld.V, V.data(), b2 * 16, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(ld.VH, VH.data(), b2 * 16, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(ld.W, W.data(), b2 * 16, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(ld.tau, src->tau, b2 * 16, hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(NEGF_EHIP, "copy of lead blocks failed"));
        // ring-circulant lead: mode values for the decimation in the ring Fourier basis
        const int P = src->period;
        bool circ = is_circulant(src->tau, b);
        for (int r = 0; r < P && circ; ++r)
            circ = is_circulant(src->h_diag + r * b2, b) && is_circulant(src->h_up + r * b2, b);
        if (circ) {
            ld.circ = true;
            ld.modes0.resize((size_t)5 * b);
            const negf_c64* blk[5] = {src->h_diag, src->h_diag + (size_t)(P - 1) * b2, src->h_up,
                                      src->h_up + (size_t)(P - 1) * b2, src->tau};
            for (int t = 0; t < 5; ++t)
                for (int q = 0; q < b; ++q) ld.modes0[(size_t)t * b + q] = ring_mode(blk[t], b, q);
            if ((s = dalloc(d, &ld.modes, (size_t)5 * b * 16)) != NEGF_OK) return bail(s);
        }
        if ((s = upload_lead_D(d, l)) != NEGF_OK) return bail(s);
    }
    *out = d;
    return NEGF_OK;
}

extern "C" {

negf_status negf_create_device(negf_device** out, int n_rings, int b, const negf_c64* h_diag, const negf_c64* h_up,
                               const negf_lead* left, const negf_lead* right, const negf_options* opt) {
    return create_device(out, n_rings, b, h_diag, h_up, left, right, opt, true);
}

negf_status negf_set_potential(negf_device* d, const double* U, double U_left, double U_right) {
    if (!d) return fail(NEGF_EINVAL, "device handle is NULL");
    if (!U) return fail(NEGF_EINVAL, "U is NULL");
    const size_t nb = (size_t)d->N * d->b;
    for (size_t i = 0; i < nb; ++i)
        if (!std::isfinite(U[i])) return fail(NEGF_EINVAL, "U[%zu] is not finite", i);
    if (!std::isfinite(U_left) || !std::isfinite(U_right)) return fail(NEGF_EINVAL, "lead potential not finite");
    HIPCHK(hipSetDevice(d->dev_id));
    HIPCHK(hipMemcpy(d->d_U, U, nb * 8, hipMemcpyHostToDevice));
    d->U_lead[0] = U_left;
    d->U_lead[1] = U_right;
    TRY(upload_lead_D(d, 0));
    TRY(upload_lead_D(d, 1));
    return NEGF_OK;
}

negf_status negf_set_potential_dev(negf_device* d, const double* U_dev, double U_left, double U_right,
                                   void* hip_stream) {
    if (!d) return fail(NEGF_EINVAL, "device handle is NULL");
    if (!U_dev) return fail(NEGF_EINVAL, "U is NULL");
    if (!std::isfinite(U_left) || !std::isfinite(U_right)) return fail(NEGF_EINVAL, "lead potential not finite");
    HIPCHK(hipSetDevice(d->dev_id));
    hipStream_t s = (hipStream_t)hip_stream;
    HIPCHK(hipMemcpyAsync(d->d_U, U_dev, (size_t)d->N * d->b * 8, hipMemcpyDeviceToDevice, s));
    if (U_left != d->U_lead[0] || U_right != d->U_lead[1]) {
        HIPCHK(hipStreamSynchronize(s));
        d->U_lead[0] = U_left;
        d->U_lead[1] = U_right;
        TRY(upload_lead_D(d, 0));
        TRY(upload_lead_D(d, 1));
    }
    return NEGF_OK;
}

negf_status negf_solve_dev(negf_device* d, const negf_bias* bias, int n_c, const negf_c64* z_c, const negf_c64* w_c,
                           int n_r, const double* E_r, const double* w_r, double* charge, double* T, double* current,
                           void* hip_stream) {
    if (!d) return fail(NEGF_EINVAL, "device handle is NULL");
    if (!bias) return fail(NEGF_EINVAL, "bias is NULL");
    const negf_job j = make_job(d, bias, n_c, z_c, w_c, n_r, E_r, w_r, charge, T, current);
    TRY(check_job(j, 0, false));
    return enqueue(d->ws, 1, &j, (hipStream_t)hip_stream);
}

negf_status negf_sync(negf_device* d) {
    if (!d) return fail(NEGF_EINVAL, "device handle is NULL");
    HIPCHK(hipSetDevice(d->dev_id));
    return finish(d->ws, nullptr);
}

negf_status negf_solve_ex(negf_device* d, const negf_bias* bias, int n_c, const negf_c64* z_c, const negf_c64* w_c,
                          int n_r, const double* E_r, const double* w_r, const negf_outputs* out) {
    if (!out) return fail(NEGF_EINVAL, "outputs are NULL");
    if (!d) return fail(NEGF_EINVAL, "device handle is NULL");
    if (!bias) return fail(NEGF_EINVAL, "bias is NULL");
    const negf_job j = make_job(d, bias, n_c, z_c, w_c, n_r, E_r, w_r, out->charge, out->T, out->current);
    TRY(check_job(j, 0, true));
    return solve_host(d->ws, 1, &j, out);
}

negf_status negf_solve(negf_device* d, const negf_bias* bias, int n_c, const negf_c64* z_c, const negf_c64* w_c,
                       int n_r, const double* E_r, const double* w_r, double* charge, double* T, double* current) {
    negf_outputs o{};
    o.charge = charge;
    o.T = T;
    o.current = current;
    return negf_solve_ex(d, bias, n_c, z_c, w_c, n_r, E_r, w_r, &o);
}

negf_status negf_lead_self_energy(negf_device* d, int lead, int n, const negf_c64* z, negf_c64* sigma, int* iters) {
    if (!d) return fail(NEGF_EINVAL, "device handle is NULL");
    if (lead != NEGF_LEAD_LEFT && lead != NEGF_LEAD_RIGHT) return fail(NEGF_EINVAL, "lead must be 0 or 1");
    if (n < 1) return fail(NEGF_EINVAL, "n = %d < 1", n);
    if (n > (1 << 26)) return fail(NEGF_EINVAL, "n = %d too large", n);
    if (!z || !sigma) return fail(NEGF_EINVAL, "z or sigma is NULL");
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(z[i].re) || !std::isfinite(z[i].im)) return fail(NEGF_EINVAL, "z[%d] not finite", i);
    negf_workspace* w = d->ws;
    HIPCHK(hipSetDevice(d->dev_id));
    TRY(grow(w, w->in_zc, (size_t)n * 16));
    TRY(grow(w, w->out_charge, (size_t)d->N * d->b * 8));
    hipStream_t s = w->own_stream;
    HIPCHK(hipMemcpy(w->in_zc.p, z, (size_t)n * 16, hipMemcpyHostToDevice));
    // the nodes enter as contour nodes (used as given); only the decimation runs
    const negf_bias b{0.0, 0.0, 1.0, 1.0};
    const negf_job j = make_job(d, &b, n, static_cast<negf_c64*>(w->in_zc.p), static_cast<negf_c64*>(w->in_zc.p), 0,
                                nullptr, nullptr, static_cast<double*>(w->out_charge.p), nullptr, nullptr);
    TRY(enqueue(w, 1, &j, s, true));
    const negf_status st = finish(w, nullptr);
    const std::string msg = g_err;
    const size_t b2 = (size_t)d->b * d->b;
    std::vector<negf_c64> all((size_t)n * 2 * b2);
    HIPCHK(hipMemcpy(all.data(), w->sigma.p, all.size() * 16, hipMemcpyDeviceToHost));
    for (int i = 0; i < n; ++i) memcpy(sigma + (size_t)i * b2, all.data() + ((size_t)i * 2 + lead) * b2, b2 * 16);
    if (iters) {
        std::vector<int> it((size_t)n * 2);
        HIPCHK(hipMemcpy(it.data(), w->iters.p, it.size() * 4, hipMemcpyDeviceToHost));
        for (int i = 0; i < n; ++i) iters[i] = it[(size_t)i * 2 + lead];
    }
    g_err = msg;
    return st;
}

negf_status negf_workspace_set_profiling(negf_workspace* w, int enable) {
    if (!w) return fail(NEGF_EINVAL, "workspace is NULL");
    w->prof = enable != 0;
    for (int k = 0; k < KT_COUNT; ++k) {
        w->ms[k] = 0;
        w->calls[k] = 0;
    }
    return NEGF_OK;
}

negf_status negf_workspace_kernel_times(negf_workspace* w, const char** names, double* ms, int* calls, int* count) {
    if (!w || !count) return fail(NEGF_EINVAL, "NULL argument");
    const int n = std::min(*count, (int)KT_COUNT);
    for (int k = 0; k < n; ++k) {
        if (names) names[k] = kKernelNames[k];
        if (ms) ms[k] = w->ms[k];
        if (calls) calls[k] = w->calls[k];
    }
    *count = KT_COUNT;
    return NEGF_OK;
}

negf_status negf_set_profiling(negf_device* d, int enable) {
    if (!d) return fail(NEGF_EINVAL, "device handle is NULL");
    return negf_workspace_set_profiling(d->ws, enable);
}

negf_status negf_kernel_times(negf_device* d, const char** names, double* ms, int* calls, int* count) {
    if (!d) return fail(NEGF_EINVAL, "NULL argument");
    return negf_workspace_kernel_times(d->ws, names, ms, calls, count);
}

negf_status negf_fp64_nodes(negf_device* d, int* count) {
    if (!d || !count) return fail(NEGF_EINVAL, "NULL argument");
    *count = d->ws->last_fp64.empty() ? 0 : d->ws->last_fp64[0];
    return NEGF_OK;
}

negf_status negf_workspace_fp64_nodes(negf_workspace* w, int n_jobs, int* counts) {
    if (!w || !counts || n_jobs < 0) return fail(NEGF_EINVAL, "bad argument");
    for (int j = 0; j < n_jobs; ++j) counts[j] = j < (int)w->last_fp64.size() ? w->last_fp64[j] : 0;
    return NEGF_OK;
}

size_t negf_device_bytes(const negf_device* d) { return d ? d->bytes + (d->ws ? d->ws->bytes : 0) : 0; }

void negf_destroy(negf_device* d) {
    if (!d) return;
    (void)hipSetDevice(d->dev_id);
    ws_destroy(d->ws);
    void* ptrs[] = {d->d_U, d->d_hdiag, d->d_ell_map, d->d_cidx, d->d_cval, d->d_ridx, d->d_rval};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    for (auto& ld : d->lead) {
        void* lp[] = {ld.D, ld.V, ld.VH, ld.W, ld.tau, ld.modes};
        for (void* p : lp)
            if (p) (void)hipFree(p);
    }
    delete d;
}

negf_status negf_workspace_create(negf_workspace** out, size_t store_bytes) {
    if (!out) return fail(NEGF_EINVAL, "out is NULL");
    *out = nullptr;
    return ws_create(out, store_bytes);
}

void negf_workspace_destroy(negf_workspace* w) { ws_destroy(w); }

negf_status negf_workspace_set_grid_scale(negf_workspace* w, int scale) {
    if (!w) return fail(NEGF_EINVAL, "workspace is NULL");
    if (scale < 1 || scale > 64) return fail(NEGF_EINVAL, "grid scale %d not in [1,64]", scale);
    w->grid_scale = scale;
    return NEGF_OK;
}

size_t negf_workspace_bytes(const negf_workspace* w) { return w ? w->bytes : 0; }

negf_status negf_batch_solve_dev(negf_workspace* w, int n_jobs, const negf_job* jobs, void* hip_stream) {
    TRY(check_batch(w, n_jobs, jobs, false));
    return enqueue(w, n_jobs, jobs, (hipStream_t)hip_stream);
}

negf_status negf_batch_sync(negf_workspace* w, int* failed_job) {
    if (!w) return fail(NEGF_EINVAL, "workspace is NULL");
    HIPCHK(hipSetDevice(w->dev_id));
    return finish(w, failed_job);
}

negf_status negf_batch_solve(negf_workspace* w, int n_jobs, const negf_job* jobs) {
    TRY(check_batch(w, n_jobs, jobs, true));
    return solve_host(w, n_jobs, jobs, nullptr);
}

negf_status negf_workspace_set_fp64_recompute(negf_workspace* w, int policy) {
    if (!w) return fail(NEGF_EINVAL, "workspace is NULL");
    if (policy < 0 || policy > 2) return fail(NEGF_EINVAL, "policy must be 0, 1 or 2");
    w->fp64_policy = policy;
    return NEGF_OK;
}

negf_status negf_set_fp64_recompute(negf_device* d, int policy) {
    if (!d) return fail(NEGF_EINVAL, "device handle is NULL");
    return negf_workspace_set_fp64_recompute(d->ws, policy);
}

negf_status negf_workspace_set_chains_per_wave(negf_workspace* w, int b, int chains) {
    if (!w) return fail(NEGF_EINVAL, "workspace is NULL");
    if (b < 1 || b > NEGF_MAX_RING) return fail(NEGF_EINVAL, "ring size %d not in [1,%d]", b, NEGF_MAX_RING);
    if (chains < 0 || chains > 64 / b) return fail(NEGF_EINVAL, "chains per wavefront %d not in [0,%d]", chains, 64 / b);
    w->gpw_b[b] = chains;
    return NEGF_OK;
}

negf_status negf_workspace_set_order(negf_workspace* w, int order) {
    if (!w) return fail(NEGF_EINVAL, "workspace is NULL");
    if (order != 0 && order != 1) return fail(NEGF_EINVAL, "order must be 0 or 1");
    w->order = order;
    return NEGF_OK;
}

negf_status negf_workspace_set_lead_basis(negf_workspace* w, int ring_modes) {
    if (!w) return fail(NEGF_EINVAL, "workspace is NULL");
    if (ring_modes != 0 && ring_modes != 1) return fail(NEGF_EINVAL, "ring_modes must be 0 or 1");
    w->circ_decimation = ring_modes == 1;
    return NEGF_OK;
}

negf_status negf_workspace_autotune(negf_workspace* w, int n_jobs, const negf_job* jobs, void* hip_stream,
                                    int reps, negf_schedule* best) {
    TRY(check_batch(w, n_jobs, jobs, false));
    if (reps < 1 || reps > 100) return fail(NEGF_EINVAL, "reps %d not in [1,100]", reps);
    hipStream_t s = (hipStream_t)hip_stream;
    HIPCHK(hipSetDevice(w->dev_id));
    // warm once: buffers and tables are sized before anything is timed
    TRY(enqueue(w, n_jobs, jobs, s));
    TRY(finish(w, nullptr));
    hipEvent_t t0, t1;
    HIPCHK(hipEventCreate(&t0));
    HIPCHK(hipEventCreate(&t1));
    negf_status st = NEGF_OK;
    // mean time of `reps` solves with the workspace's current settings
    auto timed = [&](double* ms_out) -> negf_status {
        negf_status e;
        if ((e = enqueue(w, n_jobs, jobs, s)) != NEGF_OK || (e = finish(w, nullptr)) != NEGF_OK) return e;
        (void)hipEventRecord(t0, s);
        for (int r = 0; r < reps && e == NEGF_OK; ++r) e = enqueue(w, n_jobs, jobs, s);
        (void)hipEventRecord(t1, s);
        if (e == NEGF_OK) e = finish(w, nullptr);
        if (e != NEGF_OK) return e;
        float ms = 0.f;
        if (hipEventSynchronize(t1) != hipSuccess || hipEventElapsedTime(&ms, t0, t1) != hipSuccess)
            return fail(NEGF_EHIP, "autotune timing events failed");
        *ms_out = ms / reps;
        return NEGF_OK;
    };
    negf_schedule bs{};
    bs.grid_scale = 1;
    // family 1: persistent grid size x job order, every ring size at full chains per wavefront
    for (int b = 0; b <= NEGF_MAX_RING; ++b) w->gpw_b[b] = 0;
    const int scales[] = {1, 2, 4};
    for (int order = 0; order < 2 && st == NEGF_OK; ++order)
        for (int sc : scales) {
            w->grid_scale = sc;
            w->order = order;
            double per = 0.0;
            if ((st = timed(&per)) != NEGF_OK) break;
            if (bs.ms_per_solve == 0.0 || per < bs.ms_per_solve) {
                bs.grid_scale = sc;
                bs.order = order;
                bs.ms_per_solve = per;
            }
        }
    w->grid_scale = bs.grid_scale;
    w->order = bs.order;
    // family 2: chains per wavefront, per ring size (coordinate descent over the ring
    // sizes present): all that fit (the tile schedule), half of them, or one (a
    // wavefront per energy node)
    bool present[NEGF_MAX_RING + 1] = {false};
    for (int i = 0; i < n_jobs; ++i) present[jobs[i].dev->b] = true;
    for (int b = 1; b <= NEGF_MAX_RING && st == NEGF_OK; ++b) {
        bs.chains_per_wave[b] = present[b] ? 64 / b : 0;
        if (!present[b] || 64 / b < 2) continue;
        const int cand[2] = {(64 / b + 1) / 2, 1};
        for (int c : cand) {
            if (c == 64 / b) continue;
            w->gpw_b[b] = c;
            double per = 0.0;
            if ((st = timed(&per)) != NEGF_OK) break;
            if (per < bs.ms_per_solve) {
                bs.ms_per_solve = per;
                bs.chains_per_wave[b] = c;
            }
        }
        w->gpw_b[b] = bs.chains_per_wave[b] == 64 / b ? 0 : bs.chains_per_wave[b];
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (best) *best = bs;
    return st;
}

}  // extern "C"

struct negf_graph {
    negf_workspace* ws = nullptr;   // private workspace: its buffers and tables never change
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int n_jobs = 0;
    std::vector<int> max_iter;
};

extern "C" {

void negf_graph_destroy(negf_graph* g) {
    if (!g) return;
    if (g->ws) (void)hipSetDevice(g->ws->dev_id);
    if (g->ws) (void)hipEventSynchronize(g->ws->done);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    ws_destroy(g->ws);
    delete g;
}

negf_status negf_graph_create(negf_graph** out, int n_jobs, const negf_job* jobs, size_t store_bytes,
                              void* hip_stream) {
    if (!out) return fail(NEGF_EINVAL, "out is NULL");
    *out = nullptr;
    if (!hip_stream) return fail(NEGF_EINVAL, "graph capture needs a created stream (not the null stream)");
    negf_graph* g = new negf_graph();
    auto bail = [&](negf_status st) {
        const std::string m = g_err;
        negf_graph_destroy(g);
        g_err = m;
        return st;
    };
    negf_status st;
    if ((st = ws_create(&g->ws, store_bytes)) != NEGF_OK) return bail(st);
    if ((st = check_batch(g->ws, n_jobs, jobs, false)) != NEGF_OK) return bail(st);
    hipStream_t s = (hipStream_t)hip_stream;
    // eager solve: sizes the buffers, uploads the tables, checks the jobs
    if ((st = enqueue(g->ws, n_jobs, jobs, s)) != NEGF_OK) return bail(st);
    if ((st = finish(g->ws, nullptr)) != NEGF_OK) return bail(st);
    g->max_iter = g->ws->last_max_iter;
    g->n_jobs = n_jobs;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return bail(fail(NEGF_EHIP, "hipStreamBeginCapture failed"));
    g->ws->capturing = true;
    st = enqueue(g->ws, n_jobs, jobs, s);
    g->ws->capturing = false;
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &graph);
    g->graph = graph;
    if (st != NEGF_OK) return bail(st);
    if (e != hipSuccess) return bail(fail(NEGF_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e)));
    if (hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess)
        return bail(fail(NEGF_EHIP, "hipGraphInstantiate failed"));
    g->ws->last_n_jobs = 0;
    *out = g;
    return NEGF_OK;
}

negf_status negf_graph_launch(negf_graph* g, void* hip_stream) {
    if (!g || !g->exec) return fail(NEGF_EINVAL, "graph is NULL");
    hipStream_t s = (hipStream_t)hip_stream;
    HIPCHK(hipSetDevice(g->ws->dev_id));
    HIPCHK(hipStreamWaitEvent(s, g->ws->done, 0));
    HIPCHK(hipGraphLaunch(g->exec, s));
    HIPCHK(hipEventRecord(g->ws->done, s));
    g->ws->last_n_jobs = g->n_jobs;
    g->ws->last_max_iter = g->max_iter;
    return NEGF_OK;
}

negf_status negf_graph_sync(negf_graph* g, int* failed_job) {
    if (!g) return fail(NEGF_EINVAL, "graph is NULL");
    HIPCHK(hipSetDevice(g->ws->dev_id));
    return finish(g->ws, failed_job);
}

}  // extern "C"
