// Serving runtime: self-consistent bias-point requests solved with continuous
// batching on one GPU.
//
// A native thread owns the GPU work.  Each pass of its loop
//   1. admits queued requests, first come first served, while their estimated
//      HBM footprint fits the budget (device, grid, self-energy cache,
//      per-node energy arrays, mixing state);
//   2. solves the NEGF step of every running request in one batched solve (the
//      persistent kernels of the batch API; lead self-energies are decimated
//      once per request and reused, since they depend only on the nodes and the
//      lead potentials, which a bias point fixes);
//   3. runs one self-consistency workgroup per request (ring charges, Broyden
//      update, Poisson, new potential);
//   4. retires requests that converged or hit their pass limit.
// New requests join at the next pass while the others keep iterating, so their
// work overlaps on the device.  A request's arithmetic never depends on the
// others in the batch: its results are the same alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "negf_internal.hpp"
#include "negf_sc.hpp"

using namespace negf_host;

namespace {

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct ScJob {
    long long id = 0;
    int slot = -1;
    // host copy of the request
    int N = 0, b = 0;
    std::vector<negf_c64> h_diag, h_up, lead_hd[2], lead_hu[2], lead_tau[2];
    int lead_period[2] = {1, 1};
    negf_options opt{};
    negf_bias bias{};
    double V_DS = 0, V_GS = 0;
    std::vector<negf_c64> z_c, w_c;
    std::vector<double> E_r, w_r, n_ref;
    double a = 0, c = 0, zeta = 0, tol = 0;
    int H = 0, max_iter = 0, norm = 0;
    bool want_modes = false;      // every block ring-circulant and mode space not declined
    // semi-adaptive real-axis grid, rebuilt before NEGF pass 1, 1 + refresh, ...
    bool adaptive = false;
    double density[3] = {0, 0, 0}, g_l1 = 0, g_l2 = 0, g_a = 0, g_b = 0;
    int refresh = 50;
    int n_r = 0, n_r_cap = 0;     // real-axis nodes now, and the capacity of their arrays
    size_t footprint = 0;
    // device state
    negf_device* dev = nullptr;   // real space
    negf_modes* modes = nullptr;  // mode space: one scalar chain per ring mode
    void* mem = nullptr;          // one allocation for grid, outputs, self-energies and mixing state
    negf_c64 *d_zc = nullptr, *d_wc = nullptr, *d_sigma = nullptr;
    double *d_Er = nullptr, *d_wr = nullptr, *d_charge = nullptr, *d_cur = nullptr;
    double *d_nref = nullptr, *d_state = nullptr;
    double** d_Uptr = nullptr;    // potentials that the self-consistency step writes
    bool sigma_ready = false;
    negf::ScReq rq{};
    // results
    double t_submit = 0, t_admit = 0, t_done = 0;
    int status = NEGF_OK;
    int passes = 0;
    double eps_max = 0, current = 0;
    bool done = false;
    std::vector<double> charge_out, U_out;
    std::vector<double> trace;    // stopping norm of every pass
    // warm start, deadline, eviction
    std::vector<double> rho_init;  // [N] starting rho_in (empty: n_ref)
    double deadline_ms = 0;
    bool evict_req = false;        // evict at the end of the next pass (set under the lock)
    bool resume = false;           // re-admission: restore the host state below
    int evictions = 0, admitted_pass = 0;
    std::vector<double> sv_state;  // saved at eviction: mixing state, Poisson factors and scratch
    int sv_stat[4] = {0, 0, 0, 0};   // saved pass counters and state
    double sv_diag[2] = {0, 0};
    size_t n_state = 0;

    int n_jobs() const { return modes ? (int)modes->devs.size() : 1; }
    int ring_width() const { return modes ? 1 : b; }   // entries per ring of each NEGF job
    size_t ne_cap() const { return z_c.size() + (size_t)n_r_cap; }
};

}  // namespace

struct negf_server {
    int dev_id = 0;
    size_t budget = 0, used = 0, fixed = 0;
    int max_inflight = 0;
    negf_workspace* ws = nullptr;
    hipStream_t stream = nullptr;
    int* d_stat = nullptr;        // [max_inflight][4]
    double* d_diag = nullptr;     // [max_inflight][2]
    int* h_stat = nullptr;        // pinned copies
    double* h_diag = nullptr;
    negf::ScReq* d_reqs = nullptr;   // [max_inflight]
    DBuf probe;                   // grid-probe nodes and throwaway outputs
    std::vector<int> free_slots;
    std::thread th;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    std::deque<ScJob*> pending;
    std::vector<ScJob*> running;  // written by the server thread under mu, read by it freely
    std::map<long long, ScJob*> jobs;
    long long next_id = 1;
    negf_status fatal = NEGF_OK;
    int slice = 0;                // passes after which a running request yields to queued ones
    std::string fatal_msg;
    long long passes = 0;
};

namespace {

double clip(double v, double lo, double hi) { return std::min(std::max(v, lo), hi); }

size_t estimate_footprint(const ScJob& j) {
    const size_t N = j.N, Nb = N * j.b, b2 = (size_t)j.b * j.b, nc = j.z_c.size(), nr = j.n_r_cap;
    const size_t ne = nc + nr;
    const bool f32 = j.opt.precision == NEGF_FP32_BULK;
    size_t s = 0;
    if (j.want_modes)
        s += (size_t)j.b * (N * 64 + 8192);                            // b scalar chains
    else
        s += N * b2 * 16 + Nb * 8 + 8192;                              // device Hamiltonian, potential, couplings
    s += nc * 32 + nr * 16;                                            // grid
    s += Nb * 8 + (size_t)j.b * 16;                                    // outputs, potential pointers
    s += ne * 2 * (j.want_modes ? (size_t)j.b : b2) * 16;              // self-energy cache
    s += (size_t)(12 + 2 * (j.H + 1)) * N * 8;                         // mixing state, Poisson factors and scratch
    s += nc * Nb * (f32 ? 8 : 16) + nr * 2 * Nb * 8;                   // per-node diagonals
    s += (size_t)32 * Nb * 8 + ne * (j.want_modes ? (size_t)j.b : 1) * 96;   // reduction partials, per-node scalars
    if (j.adaptive) s += nr * 16 * (j.want_modes ? (size_t)j.b : 1);  // grid probe at the capacity
    return s;
}

// frees the request's device memory; the caller returns its slot under the lock
void release(ScJob* j) {
    if (j->dev) negf_destroy(j->dev);
    j->dev = nullptr;
    if (j->modes) negf_modes_destroy(j->modes);
    j->modes = nullptr;
    if (j->mem) (void)hipFree(j->mem);
    j->mem = nullptr;
}

negf_status setup(negf_server* S, ScJob* j) {
    negf_lead leads[2];
    for (int l = 0; l < 2; ++l)
        leads[l] = negf_lead{j->lead_period[l], j->lead_hd[l].data(), j->lead_hu[l].data(), j->lead_tau[l].data()};
    const size_t N = j->N;
    if (j->want_modes) {
        TRY(negf_modes_create(&j->modes, j->N, j->b, j->h_diag.data(), j->N > 1 ? j->h_up.data() : nullptr,
                              &leads[0], &leads[1], &j->opt, 0, nullptr));
        std::vector<double> U0(N, 0.0);
        TRY(negf_modes_set_potential(j->modes, U0.data(), 0.0, -j->V_DS));
    } else {
        TRY(negf_create_device(&j->dev, j->N, j->b, j->h_diag.data(), j->N > 1 ? j->h_up.data() : nullptr,
                               &leads[0], &leads[1], &j->opt));
        std::vector<double> U0(N * j->b, 0.0);
        TRY(negf_set_potential(j->dev, U0.data(), 0.0, -j->V_DS));
    }
    const int nj = j->n_jobs();
    const size_t nc = j->z_c.size(), nr = j->n_r_cap, ne = j->ne_cap(), Nb = N * j->b;
    const size_t sig_per_node = j->modes ? (size_t)j->b : (size_t)j->b * j->b;   // 2 x this per node
    const size_t n_state = 5 * N + 2 * (size_t)(j->H + 1) * N + 4 * N + 3 * N;
    // eleven sub-arrays, each rounded up to 256 bytes
    const size_t bytes = nc * 32 + ne * 2 * sig_per_node * 16 + (2 * nr + Nb + nj + 2 * N + n_state) * 8 + nj * 8 +
                         12 * 256;
    j->n_state = n_state;
    HIPCHK(hipMalloc(&j->mem, bytes));
    char* p = static_cast<char*>(j->mem);
    auto take = [&](size_t n) { char* q = p; p += (n + 255) & ~size_t(255); return q; };
    j->d_zc = reinterpret_cast<negf_c64*>(take(nc * 16));
    j->d_wc = reinterpret_cast<negf_c64*>(take(nc * 16));
    j->d_sigma = reinterpret_cast<negf_c64*>(take(ne * 2 * sig_per_node * 16));
    j->d_Er = reinterpret_cast<double*>(take(nr * 8));
    j->d_wr = reinterpret_cast<double*>(take(nr * 8));
    j->d_charge = reinterpret_cast<double*>(take(Nb * 8));
    j->d_cur = reinterpret_cast<double*>(take(nj * 8));
    j->d_nref = reinterpret_cast<double*>(take(N * 8));
    double* d_rho0 = reinterpret_cast<double*>(take(N * 8));
    j->d_state = reinterpret_cast<double*>(take(n_state * 8));
    j->d_Uptr = reinterpret_cast<double**>(take(nj * 8));
    if (nc) {
        HIPCHK(hipMemcpy(j->d_zc, j->z_c.data(), nc * 16, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(j->d_wc, j->w_c.data(), nc * 16, hipMemcpyHostToDevice));
    }
    if (j->n_r) {
        HIPCHK(hipMemcpy(j->d_Er, j->E_r.data(), (size_t)j->n_r * 8, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(j->d_wr, j->w_r.data(), (size_t)j->n_r * 8, hipMemcpyHostToDevice));
    }
    HIPCHK(hipMemcpy(j->d_nref, j->n_ref.data(), N * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(d_rho0, (j->rho_init.empty() ? j->n_ref : j->rho_init).data(), N * 8, hipMemcpyHostToDevice));
    if (j->resume) {   // re-admission: the mixing state as it was when the request was evicted
        HIPCHK(hipMemcpy(j->d_state, j->sv_state.data(), n_state * 8, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(S->d_stat + 4 * j->slot, j->sv_stat, 4 * sizeof(int), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(S->d_diag + 2 * j->slot, j->sv_diag, 2 * sizeof(double), hipMemcpyHostToDevice));
    }
    std::vector<double*> uptr(nj);
    for (int k = 0; k < nj; ++k) uptr[k] = j->modes ? j->modes->devs[k]->d_U : j->dev->d_U;
    HIPCHK(hipMemcpy(j->d_Uptr, uptr.data(), nj * 8, hipMemcpyHostToDevice));
    negf::ScReq& R = j->rq;
    R.N = j->N;
    R.H = j->H;
    R.max_iter = j->max_iter;
    R.norm = j->norm;
    R.n_part = j->b;
    R.q_ring = j->modes ? 1 : j->b;                // real space: the ring's atoms are adjacent
    R.q_part = j->modes ? j->N : 1;                // mode space: mode k's chain starts at k N
    R.n_U = nj;
    R.U_w = j->ring_width();
    R.zeta = j->zeta;
    R.tol = j->tol;
    R.a = j->a;
    R.c = j->c;
    R.V_GS = j->V_GS;
    R.V_DS = j->V_DS;
    R.charge = j->d_charge;
    R.U = j->d_Uptr;
    R.n_ref = j->d_nref;
    R.rho0 = d_rho0;
    double* st = j->d_state;
    R.rho_in = st;
    R.rho_in_old = st + N;
    R.f_old = st + 2 * N;
    R.s = st + 3 * N;
    R.Vt = st + 5 * N;
    R.Wc = st + 5 * N + (size_t)(j->H + 1) * N;
    R.work = st + 5 * N + 2 * (size_t)(j->H + 1) * N;
    R.alf = R.work + 4 * N;
    R.invden = R.work + 5 * N;
    R.mcp = R.work + 6 * N;
    R.stat = S->d_stat + 4 * j->slot;
    R.diag = S->d_diag + 2 * j->slot;
    return NEGF_OK;
}

// gathers the A_L, A_R diagonals of ring jc from the probe's per-job arrays
// [n_jobs][np][2][N w] into out[n_jobs][np][2][w]
__global__ void k_gather_ring(const double* ad, double* out, int n_jobs, int np, int Nw, int jc, int w) {
    const long long n = (long long)n_jobs * np * 2 * w;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(q % w);
        const long long row = q / w;   // (job, node, lead)
        out[q] = ad[row * Nw + (long long)jc * w + i];
    }
}

negf_device* job_dev(ScJob* j, int k) { return j->modes ? j->modes->devs[k] : j->dev; }

// the NEGF jobs of one request: one real-space job, or one scalar chain per mode
void jobs_of(ScJob* j, std::vector<negf_job>& out) {
    const int nj = j->n_jobs();
    const size_t sig = j->ne_cap() * 2 * (j->modes ? 1 : (size_t)j->b * j->b);
    for (int k = 0; k < nj; ++k) {
        negf_job q{};
        q.dev = job_dev(j, k);
        q.bias = j->bias;
        q.n_c = (int)j->z_c.size();
        q.z_c = j->d_zc;
        q.w_c = j->d_wc;
        q.n_r = j->n_r;
        q.E_r = j->d_Er;
        q.w_r = j->d_wr;
        q.charge = j->d_charge + (size_t)k * j->N * j->ring_width();
        q.T = nullptr;
        q.current = j->d_cur + k;
        q.sigma_cache = j->d_sigma + (size_t)k * sig;
        q.sigma_mode = j->sigma_ready ? 2 : 1;
        out.push_back(q);
    }
}

// Semi-adaptive grid (Section 3.3) at the request's current potential: the
// integrand f_L A_L + f_R A_R of ring N/2 (atoms, or modes, summed) on the grid
// of the guessed limits, then the refined grid written into the request's arrays.
negf_status refresh_grid(negf_server* S, ScJob* j) {
    double E_min, E_max, kT;
    grid_window(j->bias, &E_min, &E_max, &kT);
    const double l1 = clip(j->g_l1, E_min, E_max), l2 = clip(j->g_l2, E_min, E_max);
    std::vector<double> Ep, Wp;
    grid_parts(E_min, E_max, l1, l2, j->density, kT, Ep, Wp);
    const int np = (int)Ep.size(), nj = j->n_jobs(), w = j->ring_width(), N = j->N;
    const size_t Nbj = (size_t)N * w;
    const size_t n_ring = (size_t)nj * np * 2 * w;   // gathered diagonals of ring N/2
    TRY(grow(S->ws, S->probe, ((size_t)2 * np + (size_t)nj * Nbj + nj + n_ring) * 8));
    double* pE = static_cast<double*>(S->probe.p);
    double* pW = pE + np;
    double* pq = pW + np;
    double* pg = pq + (size_t)nj * Nbj + nj;
    HIPCHK(hipMemcpy(pE, Ep.data(), (size_t)np * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(pW, Wp.data(), (size_t)np * 8, hipMemcpyHostToDevice));
    std::vector<negf_job> jobs(nj);
    for (int k = 0; k < nj; ++k) {
        negf_job& q = jobs[k];
        q = negf_job{};
        q.dev = job_dev(j, k);
        q.bias = j->bias;
        q.n_r = np;
        q.E_r = pE;
        q.w_r = pW;
        q.charge = pq + (size_t)k * Nbj;
        q.current = pq + (size_t)nj * Nbj + k;
    }
    TRY(enqueue(S->ws, nj, jobs.data(), S->stream));
    TRY(finish(S->ws, nullptr));
    // A_L, A_R of ring N/2: job k's diagonals are [np][2][Nbj] at k np 2 Nbj
    const int jc = N / 2;
    std::vector<double> ad(n_ring);
    hipLaunchKernelGGL(k_gather_ring, dim3((unsigned)std::min<size_t>((n_ring + 255) / 256, 4096)), dim3(256), 0,
                       S->stream, static_cast<const double*>(S->ws->ad.p), pg, nj, np, (int)Nbj, jc, w);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(ad.data(), pg, n_ring * 8, hipMemcpyDeviceToHost, S->stream));
    HIPCHK(hipStreamSynchronize(S->stream));
    std::vector<double> g(np);
    for (int e = 0; e < np; ++e) {
        const double fl = host_fermi(Ep[e], j->bias.mu_L, j->bias.kT_L);
        const double fr = host_fermi(Ep[e], j->bias.mu_R, j->bias.kT_R);
        double acc = 0.0;
        for (int k = 0; k < nj; ++k)
            for (int i = 0; i < w; ++i) {
                const double* row = ad.data() + ((size_t)k * np + e) * 2 * w;
                acc += fl * row[i] + fr * row[w + i];
            }
        g[e] = acc;
    }
    double n1, n2, Es;
    grid_refine(j->bias, Ep, g, l1, j->g_a, j->g_b, &n1, &n2, &Es);
    std::vector<double> Ef, Wf;
    grid_parts(E_min, E_max, n1, n2, j->density, kT, Ef, Wf);
    if ((int)Ef.size() > j->n_r_cap)
        return fail(NEGF_EINVAL, "refined grid of %d nodes exceeds its capacity %d", (int)Ef.size(), j->n_r_cap);
    HIPCHK(hipMemcpy(j->d_Er, Ef.data(), Ef.size() * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(j->d_wr, Wf.data(), Wf.size() * 8, hipMemcpyHostToDevice));
    j->n_r = (int)Ef.size();
    j->E_r = Ef;   // host copy: a re-admitted request resumes on this grid
    j->w_r = Wf;
    j->sigma_ready = false;      // the real-axis nodes moved: decimate again
    return NEGF_OK;
}

void finish_job(negf_server* S, ScJob* j, int status) {
    j->status = status;
    j->t_done = now_ms();
    const int N = j->N, b = j->b, nj = j->n_jobs();
    const size_t Nb = (size_t)N * b;
    if (j->mem && (j->dev || j->modes)) {
        j->charge_out.resize(Nb);
        j->U_out.resize(Nb);
        std::vector<double> q(Nb), u(j->modes ? (size_t)N : Nb), cur(nj);
        if (hipMemcpy(q.data(), j->d_charge, Nb * 8, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(u.data(), job_dev(j, 0)->d_U, u.size() * 8, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(cur.data(), j->d_cur, (size_t)nj * 8, hipMemcpyDeviceToHost) != hipSuccess) {
            j->status = NEGF_EHIP;
        } else if (j->modes) {
            // per-atom charge: the ring's mode charges shared equally by its b atoms
            for (int r = 0; r < N; ++r) {
                double acc = 0.0;
                for (int k = 0; k < nj; ++k) acc += q[(size_t)k * N + r];
                for (int i = 0; i < b; ++i) {
                    j->charge_out[(size_t)r * b + i] = acc / b;
                    j->U_out[(size_t)r * b + i] = u[r];
                }
            }
            double I = 0.0;
            for (int k = 0; k < nj; ++k) I += cur[k];
            j->current = I;
        } else {
            j->charge_out = q;
            j->U_out = u;
            j->current = cur[0];
        }
    }
    release(j);
    std::lock_guard<std::mutex> lk(S->mu);
    if (j->slot >= 0) S->free_slots.push_back(j->slot);
    j->slot = -1;
    S->used -= std::min(S->used, j->footprint);
    j->done = true;
    S->cv_done.notify_all();
}

// Moves a running request's state to host memory, frees its device memory and slot,
// and queues it again at the back (the caller has taken it out of the running set).
negf_status evict_job(negf_server* S, ScJob* j) {
    j->sv_state.resize(j->n_state);
    HIPCHK(hipMemcpy(j->sv_state.data(), j->d_state, j->n_state * 8, hipMemcpyDeviceToHost));
    for (int k = 0; k < 4; ++k) j->sv_stat[k] = S->h_stat[4 * j->slot + k];
    for (int k = 0; k < 2; ++k) j->sv_diag[k] = S->h_diag[2 * j->slot + k];
    release(j);
    j->resume = true;
    j->sigma_ready = false;
    j->evictions++;
    std::lock_guard<std::mutex> lk(S->mu);
    j->evict_req = false;
    S->free_slots.push_back(j->slot);
    j->slot = -1;
    S->used -= std::min(S->used, j->footprint);
    S->pending.push_back(j);
    return NEGF_OK;
}

// one pass over the running set; returns a non-OK status only for errors that stop the server
negf_status server_pass(negf_server* S, std::vector<ScJob*>& admitted) {
    // set up the newly admitted requests and start their mixing state
    std::vector<ScJob*> fresh;
    for (ScJob* j : admitted) {
        if (j->t_admit == 0) j->t_admit = now_ms();
        const negf_status st = setup(S, j);
        if (st != NEGF_OK) {
            finish_job(S, j, st);
            continue;
        }
        fresh.push_back(j);
    }
    admitted.clear();
    if (!fresh.empty()) {
        // new requests start their mixing state (mode 0); re-admitted ones rebuild their
        // potential from the restored state (mode 2)
        for (int mode : {0, 2}) {
            std::vector<negf::ScReq> rq;
            for (ScJob* j : fresh)
                if (j->resume == (mode == 2)) rq.push_back(j->rq);
            if (rq.empty()) continue;
            HIPCHK(hipMemcpy(S->d_reqs, rq.data(), rq.size() * sizeof(negf::ScReq), hipMemcpyHostToDevice));
            hipLaunchKernelGGL(negf::k_sc_step, dim3((unsigned)rq.size()), dim3(negf::SC_THREADS), 0, S->stream,
                               S->d_reqs, mode);
            HIPCHK(hipGetLastError());
            HIPCHK(hipStreamSynchronize(S->stream));
        }
        std::lock_guard<std::mutex> lk(S->mu);   // negf_server_stats reads the running set
        for (ScJob* j : fresh) {
            j->resume = false;
            j->sv_state.clear();
            j->sv_state.shrink_to_fit();
            j->admitted_pass = j->passes;
            S->running.push_back(j);
        }
    }
    if (S->running.empty()) return NEGF_OK;

    // semi-adaptive grids due at this pass (before NEGF pass 1, 1 + refresh, ...)
    {
        std::vector<ScJob*> keep;
        for (ScJob* j : S->running) {
            if (j->adaptive && j->passes % j->refresh == 0) {
                const negf_status st = refresh_grid(S, j);
                if (st != NEGF_OK) {
                    finish_job(S, j, st);
                    continue;
                }
            }
            keep.push_back(j);
        }
        std::lock_guard<std::mutex> lk(S->mu);
        S->running.swap(keep);
    }
    if (S->running.empty()) return NEGF_OK;

    // NEGF step of every running request, one batched solve
    std::vector<negf_job> jobs;
    std::vector<int> first;
    for (ScJob* j : S->running) {
        first.push_back((int)jobs.size());
        jobs_of(j, jobs);
    }
    TRY(enqueue(S->ws, (int)jobs.size(), jobs.data(), S->stream));
    // self-consistency pass, one workgroup per request
    std::vector<negf::ScReq> rq;
    for (ScJob* j : S->running) rq.push_back(j->rq);
    HIPCHK(hipMemcpyAsync(S->d_reqs, rq.data(), rq.size() * sizeof(negf::ScReq), hipMemcpyHostToDevice, S->stream));
    hipLaunchKernelGGL(negf::k_sc_step, dim3((unsigned)rq.size()), dim3(negf::SC_THREADS), 0, S->stream, S->d_reqs,
                       1);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(S->h_stat, S->d_stat, (size_t)S->max_inflight * 4 * sizeof(int), hipMemcpyDeviceToHost,
                          S->stream));
    HIPCHK(hipMemcpyAsync(S->h_diag, S->d_diag, (size_t)S->max_inflight * 2 * sizeof(double),
                          hipMemcpyDeviceToHost, S->stream));
    HIPCHK(hipEventRecord(S->ws->done, S->stream));
    HIPCHK(hipStreamSynchronize(S->stream));   // rq stays alive until the upload has run
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->passes++;
    }
    // per-request NEGF flags (ST_NOCONV: decimation; ST_BAD / ST_NOROOM: bad result)
    std::vector<ScJob*> keep, evict;
    bool waiting;
    int slice;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        waiting = !S->pending.empty();
        slice = S->slice;
    }
    const double t_now = now_ms();
    for (size_t r = 0; r < S->running.size(); ++r) {
        ScJob* j = S->running[r];
        j->sigma_ready = true;
        int fl = 0;
        for (int k = 0; k < j->n_jobs(); ++k) fl |= S->ws->h_flags[kFlagInts * (first[r] + k)];
        const int* st = S->h_stat + 4 * j->slot;
        j->passes = st[1];
        j->eps_max = S->h_diag[2 * j->slot];
        j->trace.push_back(j->eps_max);
        bool ask;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            ask = j->evict_req;
        }
        if (fl) {
            finish_job(S, j, (fl & negf::ST_NOCONV) ? NEGF_ENOCONV : NEGF_ESINGULAR);
        } else if (st[2] == 1) {
            finish_job(S, j, NEGF_OK);
        } else if (st[2] == 2) {
            finish_job(S, j, NEGF_ENOCONV);
        } else if (j->deadline_ms > 0 && t_now - j->t_submit > j->deadline_ms) {
            finish_job(S, j, NEGF_ETIMEDOUT);
        } else if (ask || (slice > 0 && waiting && j->passes - j->admitted_pass >= slice)) {
            evict.push_back(j);
        } else {
            keep.push_back(j);
        }
    }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->running.swap(keep);
    }
    for (ScJob* j : evict) {
        const negf_status st = evict_job(S, j);
        if (st != NEGF_OK) finish_job(S, j, st);
    }
    S->ws->last_n_jobs = 0;
    return NEGF_OK;
}

void server_loop(negf_server* S) {
    (void)hipSetDevice(S->dev_id);
    std::vector<ScJob*> admitted;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_work.wait(lk, [&] { return S->stop || !S->pending.empty() || !S->running.empty(); });
            if (S->stop && S->running.empty()) {
                for (ScJob* j : S->pending) {
                    j->status = NEGF_EINVAL;
                    j->done = true;
                }
                S->pending.clear();
                S->cv_done.notify_all();
                return;
            }
            // queued requests whose deadline passed end here (no device state to return)
            const double tn = now_ms();
            bool expired = false;
            for (auto it = S->pending.begin(); it != S->pending.end();) {
                ScJob* j = *it;
                if (j->deadline_ms > 0 && tn - j->t_submit > j->deadline_ms) {
                    j->status = NEGF_ETIMEDOUT;
                    j->t_done = tn;
                    j->done = true;
                    it = S->pending.erase(it);
                    expired = true;
                } else {
                    ++it;
                }
            }
            if (expired) S->cv_done.notify_all();
            while (!S->stop && !S->pending.empty() && (int)(S->running.size() + admitted.size()) < S->max_inflight) {
                ScJob* j = S->pending.front();
                if (S->used + j->footprint > S->budget && !(S->running.empty() && admitted.empty())) break;
                S->pending.pop_front();
                S->used += j->footprint;
                j->slot = S->free_slots.back();
                S->free_slots.pop_back();
                admitted.push_back(j);
            }
        }
        const negf_status st = server_pass(S, admitted);
        if (st != NEGF_OK) {
            // a HIP or allocation failure: fail the running requests and keep serving
            const std::string msg = g_err;
            std::vector<ScJob*> failed;
            {
                std::lock_guard<std::mutex> lk(S->mu);
                failed.swap(S->running);
            }
            for (ScJob* j : failed) finish_job(S, j, st);
            std::lock_guard<std::mutex> lk(S->mu);
            S->fatal = st;
            S->fatal_msg = msg;
        }
    }
}

}  // namespace

extern "C" {

negf_status negf_server_create(negf_server** out, size_t hbm_budget, int max_inflight, size_t store_bytes) {
    if (!out) return fail(NEGF_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_inflight < 1 || max_inflight > 4096) return fail(NEGF_EINVAL, "max_inflight %d not in [1,4096]",
                                                             max_inflight);
    negf_server* S = new negf_server();
    auto bail = [&](negf_status st) {
        const std::string m = g_err;
        negf_server_destroy(S);
        g_err = m;
        return st;
    };
    if (hipGetDevice(&S->dev_id) != hipSuccess) return bail(fail(NEGF_EHIP, "no HIP device"));
    S->max_inflight = max_inflight;
    negf_status st;
    if ((st = ws_create(&S->ws, store_bytes)) != NEGF_OK) return bail(st);
    const size_t cap = store_bytes ? store_bytes : S->ws->default_store_cap;
    S->fixed = 2 * cap;
    if (hbm_budget <= S->fixed) return bail(fail(NEGF_EINVAL, "budget %zu bytes leaves nothing beyond the two "
                                                             "recursion stores (%zu bytes)", hbm_budget, S->fixed));
    S->budget = hbm_budget - S->fixed;
    if (hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(NEGF_EHIP, "stream creation failed"));
    if (hipMalloc(&S->d_stat, (size_t)max_inflight * 4 * sizeof(int)) != hipSuccess ||
        hipMalloc(&S->d_diag, (size_t)max_inflight * 2 * sizeof(double)) != hipSuccess ||
        hipMalloc(&S->d_reqs, (size_t)max_inflight * sizeof(negf::ScReq)) != hipSuccess)
        return bail(fail(NEGF_ENOMEM, "server tables"));
    if (hipHostMalloc((void**)&S->h_stat, (size_t)max_inflight * 4 * sizeof(int), hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc((void**)&S->h_diag, (size_t)max_inflight * 2 * sizeof(double), hipHostMallocDefault) !=
            hipSuccess)
        return bail(fail(NEGF_ENOMEM, "pinned server tables"));
    for (int k = max_inflight - 1; k >= 0; --k) S->free_slots.push_back(k);
    S->th = std::thread(server_loop, S);
    *out = S;
    return NEGF_OK;
}

negf_status negf_server_submit(negf_server* S, const negf_sc_request* r, long long* id) {
    if (!S || !r || !id) return fail(NEGF_EINVAL, "NULL argument");
    if (r->n_rings < 2) return fail(NEGF_EINVAL, "n_rings = %d < 2", r->n_rings);
    if (r->b < 1 || r->b > NEGF_MAX_RING) return fail(NEGF_EINVAL, "ring size %d", r->b);
    if (!r->h_diag || !r->h_up || !r->left || !r->right || !r->n_ref)
        return fail(NEGF_EINVAL, "request has a NULL array");
    if (r->basis < 0 || r->basis > 1) return fail(NEGF_EINVAL, "basis %d not 0 or 1", r->basis);
    if (!(r->deadline_ms >= 0) || !std::isfinite(r->deadline_ms)) return fail(NEGF_EINVAL, "deadline not >= 0");
    if (r->rho_init)
        for (int k = 0; k < r->n_rings; ++k)
            if (!std::isfinite(r->rho_init[k])) return fail(NEGF_EINVAL, "rho_init[%d] not finite", k);
    if (r->norm < 0 || r->norm > 1) return fail(NEGF_EINVAL, "norm %d not 0 or 1", r->norm);
    const bool adaptive = r->grid_density[0] != 0 || r->grid_density[1] != 0 || r->grid_density[2] != 0;
    if (adaptive) {
        for (int p = 0; p < 3; ++p)
            if (!(r->grid_density[p] > 0) || r->grid_density[p] > 1e6)
                return fail(NEGF_EINVAL, "grid_density[%d] out of range", p);
        if (!std::isfinite(r->grid_l1) || !std::isfinite(r->grid_l2) || !std::isfinite(r->grid_a) ||
            !std::isfinite(r->grid_b) || r->grid_refresh < 0)
            return fail(NEGF_EINVAL, "grid limits not finite or refresh interval negative");
    }
    if (r->n_c < 0 || r->n_r < 0 || (!adaptive && r->n_c + r->n_r < 1)) return fail(NEGF_EINVAL, "no energy nodes");
    if ((r->n_c && (!r->z_c || !r->w_c)) || (!adaptive && r->n_r && (!r->E_r || !r->w_r)))
        return fail(NEGF_EINVAL, "grid arrays are NULL");
    if (!(r->dz > 0) || !(r->eps_1d > 0) || !(r->c_gate > 0)) return fail(NEGF_EINVAL, "electrostatics must be > 0");
    if (!(r->zeta > 0) || !(r->tol > 0) || r->max_iter < 1 || r->history < 0 ||
        r->history > negf::SC_MAX_HISTORY)
        return fail(NEGF_EINVAL, "mixing settings out of range (history <= %d)", negf::SC_MAX_HISTORY);
    if (!(r->kT > 0) || !std::isfinite(r->mu_S) || !std::isfinite(r->V_DS) || !std::isfinite(r->V_GS))
        return fail(NEGF_EINVAL, "bias point not finite");
    ScJob* j = new ScJob();
    const int N = r->n_rings, b = r->b;
    const size_t b2 = (size_t)b * b;
    j->N = N;
    j->b = b;
    j->h_diag.assign(r->h_diag, r->h_diag + (size_t)N * b2);
    j->h_up.assign(r->h_up, r->h_up + (size_t)(N - 1) * b2);
    const negf_lead* ls[2] = {r->left, r->right};
    for (int l = 0; l < 2; ++l) {
        const int P = ls[l]->period;
        if (P < 1 || P > NEGF_MAX_PERIOD || !ls[l]->h_diag || !ls[l]->h_up || !ls[l]->tau) {
            delete j;
            return fail(NEGF_EINVAL, "bad lead %d", l);
        }
        j->lead_period[l] = P;
        j->lead_hd[l].assign(ls[l]->h_diag, ls[l]->h_diag + P * b2);
        j->lead_hu[l].assign(ls[l]->h_up, ls[l]->h_up + P * b2);
        j->lead_tau[l].assign(ls[l]->tau, ls[l]->tau + b2);
    }
    j->opt = r->opt;
    j->V_DS = r->V_DS;
    j->V_GS = r->V_GS;
    j->bias = negf_bias{r->mu_S, r->mu_S - r->V_DS, r->kT, r->kT};
    j->z_c.assign(r->z_c, r->z_c + r->n_c);
    j->w_c.assign(r->w_c, r->w_c + r->n_c);
    if (adaptive) {
        j->adaptive = true;
        double E_min, E_max, kT;
        grid_window(j->bias, &E_min, &E_max, &kT);
        double dmax = 0.0;
        for (int p = 0; p < 3; ++p) {
            j->density[p] = r->grid_density[p];
            dmax = std::max(dmax, r->grid_density[p]);
        }
        // each part holds at most density x width / kT + 1 nodes
        const double cap = std::floor(dmax * (E_max - E_min) / kT) + 4.0;
        if (!(cap <= (double)(1 << 22))) {
            delete j;
            return fail(NEGF_EINVAL, "semi-adaptive grid of up to %.0f nodes", cap);
        }
        j->n_r_cap = (int)cap;
        j->g_l1 = r->grid_l1;
        j->g_l2 = r->grid_l2;
        j->g_a = r->grid_a;
        j->g_b = r->grid_b;
        j->refresh = r->grid_refresh ? r->grid_refresh : 50;
    } else {
        j->E_r.assign(r->E_r, r->E_r + r->n_r);
        j->w_r.assign(r->w_r, r->w_r + r->n_r);
        j->n_r = j->n_r_cap = r->n_r;
    }
    j->norm = r->norm;
    if (r->rho_init) j->rho_init.assign(r->rho_init, r->rho_init + N);
    j->deadline_ms = r->deadline_ms;
    if (r->basis == 0) {   // mode space when every block is ring-circulant (the potential always is ring-uniform)
        bool circ = true;
        for (int k = 0; k < N && circ; ++k) circ = ring_circulant(r->h_diag + (size_t)k * b2, b);
        for (int k = 0; k + 1 < N && circ; ++k) circ = ring_circulant(r->h_up + (size_t)k * b2, b);
        for (int l = 0; l < 2 && circ; ++l) {
            for (int q = 0; q < j->lead_period[l]; ++q)
                circ = circ && ring_circulant(j->lead_hd[l].data() + q * b2, b) &&
                       ring_circulant(j->lead_hu[l].data() + q * b2, b);
            circ = circ && ring_circulant(j->lead_tau[l].data(), b);
        }
        j->want_modes = circ;
    }
    j->n_ref.assign(r->n_ref, r->n_ref + N);
    const double e = 1.602176634e-19;
    j->a = r->eps_1d / (r->c_gate * r->dz * r->dz);
    j->c = e / (r->c_gate * r->dz);
    j->zeta = r->zeta;
    j->tol = r->tol;
    j->H = r->history;
    j->max_iter = r->max_iter;
    j->footprint = estimate_footprint(*j);
    j->t_submit = now_ms();
    std::lock_guard<std::mutex> lk(S->mu);
    if (j->footprint > S->budget) {
        delete j;
        return fail(NEGF_ENOMEM, "request footprint exceeds the server's HBM budget");
    }
    if (S->stop) {
        delete j;
        return fail(NEGF_EINVAL, "server is stopping");
    }
    j->id = S->next_id++;
    S->jobs[j->id] = j;
    S->pending.push_back(j);
    *id = j->id;
    S->cv_work.notify_all();
    return NEGF_OK;
}

negf_status negf_server_poll(negf_server* S, long long id, int wait, negf_sc_result* res, double* charge,
                             double* U, double* eps_trace) {
    if (!S) return fail(NEGF_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->jobs.find(id);
    if (it == S->jobs.end()) return fail(NEGF_EINVAL, "unknown request %lld", id);
    ScJob* j = it->second;
    if (!j->done) {
        if (!wait) return NEGF_PENDING;
        S->cv_done.wait(lk, [&] { return j->done; });
    }
    if (res) {
        res->status = j->status;
        res->iterations = j->passes;
        res->eps_max = j->eps_max;
        res->current = j->current;
        res->t_queue_ms = j->t_admit > 0 ? j->t_admit - j->t_submit : 0.0;
        res->t_run_ms = j->t_admit > 0 ? j->t_done - j->t_admit : 0.0;
        res->t_total_ms = j->t_done - j->t_submit;
        res->n_r = j->n_r;
        res->mode_space = j->want_modes ? 1 : 0;
        res->evictions = j->evictions;
    }
    if (charge && !j->charge_out.empty()) memcpy(charge, j->charge_out.data(), j->charge_out.size() * 8);
    if (U && !j->U_out.empty()) memcpy(U, j->U_out.data(), j->U_out.size() * 8);
    if (eps_trace && !j->trace.empty()) memcpy(eps_trace, j->trace.data(), j->trace.size() * 8);
    S->jobs.erase(it);
    delete j;
    return NEGF_OK;
}

negf_status negf_server_evict(negf_server* S, long long id) {
    if (!S) return fail(NEGF_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(id);
    if (it == S->jobs.end()) return fail(NEGF_EINVAL, "unknown request %lld", id);
    if (it->second->done) return fail(NEGF_EINVAL, "request %lld has finished", id);
    it->second->evict_req = true;
    return NEGF_OK;
}

negf_status negf_server_set_time_slice(negf_server* S, int passes) {
    if (!S) return fail(NEGF_EINVAL, "server is NULL");
    if (passes < 0) return fail(NEGF_EINVAL, "time slice %d < 0", passes);
    std::lock_guard<std::mutex> lk(S->mu);
    S->slice = passes;
    return NEGF_OK;
}

negf_status negf_server_stats(negf_server* S, negf_server_info* info) {
    if (!S || !info) return fail(NEGF_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    info->pending = (int)S->pending.size();
    info->running = (int)S->running.size();
    info->passes = S->passes;
    info->hbm_used = S->used + S->fixed;
    info->hbm_budget = S->budget + S->fixed;
    info->workspace_bytes = S->ws ? S->ws->bytes : 0;
    return S->fatal;
}

void negf_server_destroy(negf_server* S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv_work.notify_all();
    }
    if (S->th.joinable()) S->th.join();
    (void)hipSetDevice(S->dev_id);
    for (auto& kv : S->jobs) {
        release(kv.second);
        delete kv.second;
    }
    if (S->stream) (void)hipStreamSynchronize(S->stream);
    if (S->d_stat) (void)hipFree(S->d_stat);
    if (S->d_diag) (void)hipFree(S->d_diag);
    if (S->d_reqs) (void)hipFree(S->d_reqs);
    if (S->probe.p) (void)hipFree(S->probe.p);
    if (S->h_stat) (void)hipHostFree(S->h_stat);
    if (S->h_diag) (void)hipHostFree(S->h_diag);
    if (S->stream) (void)hipStreamDestroy(S->stream);
    ws_destroy(S->ws);
    delete S;
}

}  // extern "C"
