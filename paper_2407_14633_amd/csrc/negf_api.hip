// C ABI of the energy-point Green's-function engine: argument checks, HBM
// layout, energy chunking and the launch sequence of one solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "negf.h"
#include "negf_launch.hpp"
#include "negf_reduce.hpp"

using negf::cx;

namespace {

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

#define HIPCHK(expr)                                                                    \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) return fail(NEGF_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

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

enum { KT_DECIMATE = 0, KT_RECUR, KT_CDIAG, KT_COLUMN, KT_REDUCE, KT_COUNT };
const char* const kKernelNames[KT_COUNT] = {"decimate", "recur", "cdiag", "column", "reduce"};

struct LeadDev {
    int period = 1;
    std::vector<negf_c64> h_diag;   // host copy, potential added at set_potential
    cx<double>* D = nullptr;        // [P][b][b] incl. lead potential
    cx<double>* V = nullptr;        // h_up[0]
    cx<double>* VH = nullptr;       // h_up[0]^H
    cx<double>* W = nullptr;        // h_up[P-1]
    cx<double>* tau = nullptr;
};

}  // namespace

struct negf_device {
    int dev_id = 0;
    int N = 0, b = 0;
    negf_options opt{};
    const negf::Launchers* L = nullptr;
    int K = 1;
    bool hdiag_zero = true;
    double* d_U = nullptr;
    cx<double>* d_hdiag = nullptr;
    int n_uniq = 1;
    int* d_ell_map = nullptr;
    int* d_cidx = nullptr;
    cx<double>* d_cval = nullptr;
    int* d_ridx = nullptr;
    cx<double>* d_rval = nullptr;
    LeadDev lead[2];
    double U_lead[2] = {0.0, 0.0};

    // per-energy workspace (capacity in energies)
    int cap_e = 0;
    cx<double>* d_z = nullptr;
    cx<double>* d_sigma = nullptr;
    int* d_iters = nullptr;
    int* d_status = nullptr;
    cx<double>* d_dscratch = nullptr;
    cx<double>* d_coef_c = nullptr;
    double* d_coef_r = nullptr;
    void* d_gr = nullptr;
    void* d_ad = nullptr;
    double* d_T = nullptr;
    double* d_part = nullptr;     // [RED_SEGS][N*b] reduction partials
    // recursion store (capacity in energies)
    int cap_store = 0;
    void* d_store_f = nullptr;
    void* d_store_b = nullptr;
    // host-pointer staging
    int cap_io = 0;
    cx<double>* d_in_zc = nullptr;
    cx<double>* d_in_wc = nullptr;
    double* d_in_Er = nullptr;
    double* d_in_wr = nullptr;
    double* d_out_charge = nullptr;
    double* d_out_cur = nullptr;
    int* d_flags = nullptr;     // [0] flags, [1] first bad energy
    int* h_flags = nullptr;     // pinned
    hipStream_t own_stream = nullptr;
    hipStream_t last_stream = nullptr;
    int last_ne = 0;

    bool prof = false;
    struct Ev { int kind; hipEvent_t a, b; };
    std::vector<Ev> pending;
    double ms[KT_COUNT] = {0};
    int calls[KT_COUNT] = {0};

    size_t bytes = 0;
    std::vector<void*> allocs_fixed;
};

namespace {

template <typename P>
negf_status dalloc(negf_device* d, P** p, size_t bytes) {
    if (bytes == 0) bytes = 16;
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) return fail(NEGF_ENOMEM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    *p = static_cast<P*>(q);
    d->bytes += bytes;
    return NEGF_OK;
}

void dfree(negf_device* d, void* p, size_t bytes) {
    if (p) {
        (void)hipFree(p);
        d->bytes -= std::min(d->bytes, bytes);
    }
}

#define TRY(expr)                       \
    do {                                \
        negf_status s_ = (expr);        \
        if (s_ != NEGF_OK) return s_;   \
    } while (0)

// element sizes per precision: recursion store / contour diagonals (complex), A diagonals (real)
size_t cplx_bytes(const negf_device* d) { return d->opt.precision == NEGF_FP32_BULK ? 8 : 16; }
size_t adiag_bytes(const negf_device* d) { return d->opt.precision == NEGF_FP32_BULK ? 4 : 8; }

size_t store_bytes_per_energy(const negf_device* d) {
    return (size_t)d->N * d->b * d->b * cplx_bytes(d);
}

negf_status ensure_energy_ws(negf_device* d, int ne) {
    if (ne <= d->cap_e) return NEGF_OK;
    const size_t b2 = (size_t)d->b * d->b, Nb = (size_t)d->N * d->b;
    const size_t cb = cplx_bytes(d), rb = adiag_bytes(d);
    size_t old = d->cap_e;
    dfree(d, d->d_z, old * 16);
    dfree(d, d->d_sigma, old * 2 * b2 * 16);
    dfree(d, d->d_iters, old * 2 * 4);
    dfree(d, d->d_status, old * 4);
    dfree(d, d->d_dscratch, old * 2 * 6 * b2 * 16);
    dfree(d, d->d_coef_c, old * 16);
    dfree(d, d->d_coef_r, old * 3 * 8);
    dfree(d, d->d_gr, old * Nb * cb);
    dfree(d, d->d_ad, old * 2 * Nb * rb);
    dfree(d, d->d_T, old * 8);
    d->cap_e = 0;
    const size_t n = (size_t)ne;
    TRY(dalloc(d, &d->d_z, n * 16));
    TRY(dalloc(d, &d->d_sigma, n * 2 * b2 * 16));
    TRY(dalloc(d, &d->d_iters, n * 2 * 4));
    TRY(dalloc(d, &d->d_status, n * 4));
    TRY(dalloc(d, &d->d_dscratch, n * 2 * 6 * b2 * 16));
    TRY(dalloc(d, &d->d_coef_c, n * 16));
    TRY(dalloc(d, &d->d_coef_r, n * 3 * 8));
    TRY(dalloc(d, &d->d_gr, n * Nb * cb));
    TRY(dalloc(d, &d->d_ad, n * 2 * Nb * rb));
    TRY(dalloc(d, &d->d_T, n * 8));
    d->cap_e = ne;
    return NEGF_OK;
}

negf_status ensure_store(negf_device* d, int ne_chunk) {
    if (ne_chunk <= d->cap_store) return NEGF_OK;
    const size_t per = store_bytes_per_energy(d);
    dfree(d, d->d_store_f, (size_t)d->cap_store * per);
    dfree(d, d->d_store_b, (size_t)d->cap_store * per);
    d->cap_store = 0;
    TRY(dalloc(d, &d->d_store_f, (size_t)ne_chunk * per));
    TRY(dalloc(d, &d->d_store_b, (size_t)ne_chunk * per));
    d->cap_store = ne_chunk;
    return NEGF_OK;
}

negf_status ensure_io(negf_device* d, int n_c, int n_r) {
    const int need = std::max(n_c, n_r);
    if (need > d->cap_io) {
        const size_t old = d->cap_io;
        dfree(d, d->d_in_zc, old * 16);
        dfree(d, d->d_in_wc, old * 16);
        dfree(d, d->d_in_Er, old * 8);
        dfree(d, d->d_in_wr, old * 8);
        d->cap_io = 0;
        TRY(dalloc(d, &d->d_in_zc, (size_t)need * 16));
        TRY(dalloc(d, &d->d_in_wc, (size_t)need * 16));
        TRY(dalloc(d, &d->d_in_Er, (size_t)need * 8));
        TRY(dalloc(d, &d->d_in_wr, (size_t)need * 8));
        d->cap_io = need;
    }
    return NEGF_OK;
}

int chunk_energies(const negf_device* d, int ne) {
    size_t cap = d->opt.workspace_bytes ? d->opt.workspace_bytes : ((size_t)16 << 30);
    const size_t per = 2 * store_bytes_per_energy(d);
    size_t c = std::max<size_t>(1, cap / per);
    return (int)std::min<size_t>(c, (size_t)ne);
}

negf_status upload_lead_D(negf_device* d, int l) {
    LeadDev& ld = d->lead[l];
    const int b = d->b;
    std::vector<negf_c64> D = ld.h_diag;
    for (int p = 0; p < ld.period; ++p)
        for (int i = 0; i < b; ++i) D[(size_t)p * b * b + (size_t)i * b + i].re += d->U_lead[l];
    HIPCHK(hipMemcpy(ld.D, D.data(), D.size() * 16, hipMemcpyHostToDevice));
    return NEGF_OK;
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

negf_status check_solve_args(negf_device* d, const negf_bias* bias, int n_c, const void* z_c, const void* w_c,
                             int n_r, const void* E_r, const void* w_r, const void* charge) {
    if (!d) return fail(NEGF_EINVAL, "device handle is NULL");
    if (!bias) return fail(NEGF_EINVAL, "bias is NULL");
    if (!(bias->kT_L > 0) || !(bias->kT_R > 0) || !std::isfinite(bias->mu_L) || !std::isfinite(bias->mu_R) ||
        !std::isfinite(bias->kT_L) || !std::isfinite(bias->kT_R))
        return fail(NEGF_EINVAL, "bias needs finite mu and kT > 0");
    if (n_c < 0 || n_r < 0) return fail(NEGF_EINVAL, "negative node count (n_c=%d, n_r=%d)", n_c, n_r);
    if (n_c + n_r < 1) return fail(NEGF_EINVAL, "no energy nodes");
    if ((long long)n_c + n_r > (1LL << 26)) return fail(NEGF_EINVAL, "too many energy nodes");
    if (n_c > 0 && (!z_c || !w_c)) return fail(NEGF_EINVAL, "contour nodes/weights are NULL");
    if (n_r > 0 && (!E_r || !w_r)) return fail(NEGF_EINVAL, "real-axis nodes/weights are NULL");
    if (!charge) return fail(NEGF_EINVAL, "charge output is NULL");
    return NEGF_OK;
}

void ev_begin(negf_device* d, int kind, hipStream_t s, hipEvent_t* a) {
    *a = nullptr;
    if (!d->prof) return;
    (void)hipEventCreate(a);
    (void)hipEventRecord(*a, s);
    (void)kind;
}
void ev_end(negf_device* d, int kind, hipStream_t s, hipEvent_t a) {
    if (!d->prof || !a) return;
    hipEvent_t b;
    (void)hipEventCreate(&b);
    (void)hipEventRecord(b, s);
    d->pending.push_back({kind, a, b});
}
void ev_collect(negf_device* d) {
    for (auto& e : d->pending) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, e.a, e.b) == hipSuccess) {
            d->ms[e.kind] += t;
            d->calls[e.kind] += 1;
        }
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    d->pending.clear();
}

__global__ void k_fill_int(int* p, int n, int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_zero_double(double* p) { *p = 0.0; }

negf::DecArgs dec_args(negf_device* d, int n, int lead_only) {
    negf::DecArgs a{};
    a.b = d->b;
    a.n = n;
    a.maxit = d->opt.decim_max_iter;
    a.tol = d->opt.decim_tol;
    a.lead_only = lead_only;
    a.z = d->d_z;
    for (int l = 0; l < 2; ++l) {
        a.period[l] = d->lead[l].period;
        a.D[l] = d->lead[l].D;
        a.V[l] = d->lead[l].V;
        a.VH[l] = d->lead[l].VH;
        a.W[l] = d->lead[l].W;
        a.tau[l] = d->lead[l].tau;
    }
    a.scratch = d->d_dscratch;
    a.sigma = d->d_sigma;
    a.iters = d->d_iters;
    a.status = d->d_status;
    return a;
}

// The device-side launch sequence of one solve.  All arrays are device pointers.
negf_status run_solve(negf_device* d, const negf_bias* bias, int n_c, const cx<double>* z_c, const cx<double>* w_c,
                      int n_r, const double* E_r, const double* w_r, double* charge, double* T, double* current,
                      hipStream_t s) {
    HIPCHK(hipSetDevice(d->dev_id));
    const int ne = n_c + n_r;
    TRY(ensure_energy_ws(d, ne));
    const int chunk = chunk_energies(d, ne);
    TRY(ensure_store(d, chunk));
    const int N = d->N, b = d->b, G = d->L->groups;
    const bool f32 = d->opt.precision == NEGF_FP32_BULK;       // everything but a1/a6 in FP32
    hipEvent_t ev;

    ev_begin(d, KT_REDUCE, s, &ev);
    hipLaunchKernelGGL(negf::k_nodes, dim3((ne + 255) / 256), dim3(256), 0, s, z_c, n_c, E_r, n_r, d->opt.eta, d->d_z);
    hipLaunchKernelGGL(k_fill_int, dim3((ne + 255) / 256), dim3(256), 0, s, d->d_status, ne, 0);
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, s, d->d_flags, 1, 0);
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, s, d->d_flags + 1, 1, 0x7fffffff);
    ev_end(d, KT_REDUCE, s, ev);

    // a1: lead self-energies for every node, both leads in one launch
    ev_begin(d, KT_DECIMATE, s, &ev);
    {
        negf::DecArgs a = dec_args(d, ne, -1);
        d->L->decimate(a, 2 * ((ne + G - 1) / G), s);
    }
    ev_end(d, KT_DECIMATE, s, ev);
    hipLaunchKernelGGL(negf::k_status, dim3((ne + 255) / 256), dim3(256), 0, s, d->d_status, ne, d->d_flags,
                       d->d_flags + 1);

    negf::RgfArgs A{};
    A.N = N;
    A.b = b;
    A.n_c = n_c;
    A.K = d->K;
    A.n_uniq = d->n_uniq;
    A.ell_map = d->d_ell_map;
    A.hdiag_zero = d->hdiag_zero ? 1 : 0;
    A.U = d->d_U;
    A.hdiag = d->d_hdiag;
    A.cidx = d->d_cidx;
    A.cval = d->d_cval;
    A.ridx = d->d_ridx;
    A.rval = d->d_rval;
    A.z = d->d_z;
    A.sigma = d->d_sigma;
    A.store_f = d->d_store_f;
    A.store_b = d->d_store_b;
    A.gr_diag = d->d_gr;
    A.a_diag = d->d_ad;
    A.Tout = d->d_T;

    for (int e0 = 0; e0 < ne; e0 += chunk) {
        const int cn = std::min(chunk, ne - e0);
        A.e0 = e0;
        A.ne = cn;
        // a3-a4 recursions: both directions of every node of the chunk
        ev_begin(d, KT_RECUR, s, &ev);
        const int wv = (cn + G - 1) / G;
        (f32 ? d->L->recur32 : d->L->recur64)(A, 2 * wv, s);
        ev_end(d, KT_RECUR, s, ev);
        // contour nodes of the chunk: diagonal blocks
        const int c_end = std::min(e0 + cn, n_c);
        if (c_end > e0) {
            const int nc = c_end - e0;
            const long long items = (long long)nc * N;
            ev_begin(d, KT_CDIAG, s, &ev);
            (f32 ? d->L->cdiag32 : d->L->cdiag64)(A, nc, (int)((items + G - 1) / G), s);
            ev_end(d, KT_CDIAG, s, ev);
        }
        // real-axis nodes of the chunk: lead columns, A_l diagonals, T
        const int r0 = std::max(e0, n_c);
        if (e0 + cn > r0) {
            const int nr = e0 + cn - r0;
            ev_begin(d, KT_COLUMN, s, &ev);
            (f32 ? d->L->column32 : d->L->column64)(A, r0, nr, 2 * ((nr + G - 1) / G), s);
            ev_end(d, KT_COLUMN, s, ev);
        }
    }

    // a6: weighted energy sums
    negf::RedArgs R{};
    R.Nb = N * b;
    R.n_c = n_c;
    R.n_r = n_r;
    R.g_s = d->opt.g_s;
    R.mu_L = bias->mu_L;
    R.mu_R = bias->mu_R;
    R.kT_L = bias->kT_L;
    R.kT_R = bias->kT_R;
    R.z_c = z_c;
    R.w_c = w_c;
    R.E_r = E_r;
    R.w_r = w_r;
    R.coef_c = d->d_coef_c;
    R.coef_r = d->d_coef_r;
    R.gr_diag = d->d_gr;
    R.a_diag = d->d_ad;
    R.T = d->d_T;
    R.charge = charge;
    R.current = current;
    R.flags = d->d_flags;
    ev_begin(d, KT_REDUCE, s, &ev);
    hipLaunchKernelGGL(negf::k_coef, dim3((ne + 255) / 256), dim3(256), 0, s, R);
    if (!d->d_part) TRY(dalloc(d, &d->d_part, (size_t)negf::RED_SEGS * R.Nb * 8));
    const dim3 rgrid((R.Nb + 255) / 256, negf::RED_SEGS);
    if (f32)
        hipLaunchKernelGGL((negf::k_reduce_part<float, float>), rgrid, dim3(256), 0, s, R, d->d_part);
    else
        hipLaunchKernelGGL((negf::k_reduce_part<double, double>), rgrid, dim3(256), 0, s, R, d->d_part);
    hipLaunchKernelGGL(negf::k_reduce_final, dim3((R.Nb + 255) / 256), dim3(256), 0, s, R, d->d_part);
    if (n_r > 0)
        hipLaunchKernelGGL(negf::k_current, dim3(1), dim3(64), 0, s, R);
    else if (current)
        hipLaunchKernelGGL(k_zero_double, dim3(1), dim3(1), 0, s, current);
    if (T && n_r > 0) HIPCHK(hipMemcpyAsync(T, d->d_T, (size_t)n_r * 8, hipMemcpyDeviceToDevice, s));
    ev_end(d, KT_REDUCE, s, ev);
    HIPCHK(hipMemcpyAsync(d->h_flags, d->d_flags, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipGetLastError());
    d->last_stream = s;
    d->last_ne = ne;
    return NEGF_OK;
}

negf_status finish(negf_device* d) {
    HIPCHK(hipStreamSynchronize(d->last_stream));
    ev_collect(d);
    const int fl = d->h_flags[0];
    if (fl & 1)
        return fail(NEGF_ENOCONV, "lead decimation did not converge in %d steps (first energy index %d)",
                    d->opt.decim_max_iter, d->h_flags[1]);
    if (fl & 2) return fail(NEGF_ESINGULAR, "non-finite charge or current (singular block or overflow)");
    return NEGF_OK;
}

}  // namespace

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

negf_status negf_create_device(negf_device** out, int n_rings, int b, const negf_c64* h_diag, const negf_c64* h_up,
                               const negf_lead* left, const negf_lead* right, const negf_options* opt) {
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

    negf_device* d = new negf_device();
    d->N = n_rings;
    d->b = b;
    d->opt = o;
    d->L = L;
    auto bail = [&](negf_status s) { std::string m = g_err; negf_destroy(d); g_err = m; return s; };
    if (hipGetDevice(&d->dev_id) != hipSuccess) return bail(fail(NEGF_EHIP, "no HIP device"));

    // hdiag
    d->hdiag_zero = true;
    for (size_t i = 0; i < (size_t)n_rings * b2; ++i)
        if (h_diag[i].re != 0.0 || h_diag[i].im != 0.0) { d->hdiag_zero = false; break; }
    negf_status s;
    if ((s = dalloc(d, &d->d_hdiag, (size_t)n_rings * b2 * 16)) != NEGF_OK) return bail(s);
    if (hipMemcpy(d->d_hdiag, h_diag, (size_t)n_rings * b2 * 16, hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(NEGF_EHIP, "copy of h_diag failed"));
    if ((s = dalloc(d, &d->d_U, (size_t)n_rings * b * 8)) != NEGF_OK) return bail(s);
    if (hipMemset(d->d_U, 0, (size_t)n_rings * b * 8) != hipSuccess) return bail(fail(NEGF_EHIP, "memset U"));

    // couplings: distinct blocks as column- and row-ELL with a common width K, plus
    // the map ring coupling -> distinct block (periodic structures have few blocks)
    const int nc = std::max(0, n_rings - 1);
    std::vector<int> ell_map((size_t)std::max(1, nc), 0);
    std::vector<int> uniq;   // index n of the first coupling of each distinct block
    for (int n = 0; n < nc; ++n) {
        const negf_c64* H = h_up + (size_t)n * b2;
        int found = -1;
        for (size_t u = 0; u < uniq.size() && found < 0; ++u)
            if (memcmp(H, h_up + (size_t)uniq[u] * b2, b2 * sizeof(negf_c64)) == 0) found = (int)u;
        if (found < 0) { found = (int)uniq.size(); uniq.push_back(n); }
        ell_map[n] = found;
    }
    const int nu = std::max<int>(1, (int)uniq.size());
    d->n_uniq = nu;
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
    d->K = K;
    const size_t ell = (size_t)nu * b * K;
    if (ell * (sizeof(negf_c64) + 1) > 32768)
        return bail(fail(NEGF_EINVAL, "coupling table of %d distinct blocks (width %d) exceeds the 32 KiB LDS table",
                         nu, K));
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

    // leads
    const negf_lead* leads[2] = {left, right};
    for (int l = 0; l < 2; ++l) {
        LeadDev& ld = d->lead[l];
        const negf_lead* src = leads[l];
        ld.period = src->period;
        ld.h_diag.assign(src->h_diag, src->h_diag + (size_t)src->period * b2);
        std::vector<negf_c64> V(src->h_up, src->h_up + b2), VH(b2), W(src->h_up + (size_t)(src->period - 1) * b2,
                                                                     src->h_up + (size_t)src->period * b2);
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
        if ((s = upload_lead_D(d, l)) != NEGF_OK) return bail(s);
    }
    if (hipStreamCreateWithFlags(&d->own_stream, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(NEGF_EHIP, "stream creation failed"));
    if ((s = dalloc(d, &d->d_flags, 2 * sizeof(int))) != NEGF_OK) return bail(s);
    if (hipHostMalloc((void**)&d->h_flags, 2 * sizeof(int), hipHostMallocDefault) != hipSuccess)
        return bail(fail(NEGF_ENOMEM, "pinned flag buffer"));
    d->h_flags[0] = 0;
    d->h_flags[1] = 0;
    d->last_stream = d->own_stream;
    *out = d;
    return NEGF_OK;
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
    TRY(check_solve_args(d, bias, n_c, z_c, w_c, n_r, E_r, w_r, charge));
    return run_solve(d, bias, n_c, reinterpret_cast<const cx<double>*>(z_c), reinterpret_cast<const cx<double>*>(w_c),
                     n_r, E_r, w_r, charge, T, current, (hipStream_t)hip_stream);
}

negf_status negf_sync(negf_device* d) {
    if (!d) return fail(NEGF_EINVAL, "device handle is NULL");
    HIPCHK(hipSetDevice(d->dev_id));
    return finish(d);
}

negf_status negf_solve_ex(negf_device* d, const negf_bias* bias, int n_c, const negf_c64* z_c, const negf_c64* w_c,
                          int n_r, const double* E_r, const double* w_r, const negf_outputs* out) {
    if (!out) return fail(NEGF_EINVAL, "outputs are NULL");
    TRY(check_solve_args(d, bias, n_c, z_c, w_c, n_r, E_r, w_r, out->charge));
    for (int i = 0; i < n_c; ++i)
        if (!std::isfinite(z_c[i].re) || !std::isfinite(z_c[i].im) || !std::isfinite(w_c[i].re) ||
            !std::isfinite(w_c[i].im))
            return fail(NEGF_EINVAL, "contour node %d is not finite", i);
    for (int i = 0; i < n_r; ++i)
        if (!std::isfinite(E_r[i]) || !std::isfinite(w_r[i])) return fail(NEGF_EINVAL, "real node %d is not finite", i);
    HIPCHK(hipSetDevice(d->dev_id));
    TRY(ensure_io(d, n_c, n_r));
    const size_t Nb = (size_t)d->N * d->b;
    if (!d->d_out_charge) {
        TRY(dalloc(d, &d->d_out_cur, 8));
        TRY(dalloc(d, &d->d_out_charge, Nb * 8));
    }
    hipStream_t s = d->own_stream;
    if (n_c) {
        HIPCHK(hipMemcpyAsync(d->d_in_zc, z_c, (size_t)n_c * 16, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(d->d_in_wc, w_c, (size_t)n_c * 16, hipMemcpyHostToDevice, s));
    }
    if (n_r) {
        HIPCHK(hipMemcpyAsync(d->d_in_Er, E_r, (size_t)n_r * 8, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(d->d_in_wr, w_r, (size_t)n_r * 8, hipMemcpyHostToDevice, s));
    }
    TRY(run_solve(d, bias, n_c, d->d_in_zc, d->d_in_wc, n_r, d->d_in_Er, d->d_in_wr, d->d_out_charge, nullptr,
                  d->d_out_cur, s));
    negf_status st = finish(d);
    // outputs are copied even on a device-side error status so that callers can inspect them
    HIPCHK(hipMemcpy(out->charge, d->d_out_charge, Nb * 8, hipMemcpyDeviceToHost));
    if (out->current) HIPCHK(hipMemcpy(out->current, d->d_out_cur, 8, hipMemcpyDeviceToHost));
    if (out->T && n_r) HIPCHK(hipMemcpy(out->T, d->d_T, (size_t)n_r * 8, hipMemcpyDeviceToHost));
    const bool f32 = d->opt.precision == NEGF_FP32_BULK;
    const bool ad32 = f32;
    if (out->gr_diag && n_c) {
        if (f32) {
            std::vector<float> tmp((size_t)n_c * Nb * 2);
            HIPCHK(hipMemcpy(tmp.data(), d->d_gr, tmp.size() * 4, hipMemcpyDeviceToHost));
            for (size_t i = 0; i < (size_t)n_c * Nb; ++i) out->gr_diag[i] = negf_c64{tmp[2 * i], tmp[2 * i + 1]};
        } else {
            HIPCHK(hipMemcpy(out->gr_diag, d->d_gr, (size_t)n_c * Nb * 16, hipMemcpyDeviceToHost));
        }
    }
    if ((out->al_diag || out->ar_diag) && n_r) {
        std::vector<double> ad((size_t)n_r * 2 * Nb);
        if (ad32) {
            std::vector<float> tmp(ad.size());
            HIPCHK(hipMemcpy(tmp.data(), d->d_ad, tmp.size() * 4, hipMemcpyDeviceToHost));
            for (size_t i = 0; i < ad.size(); ++i) ad[i] = tmp[i];
        } else {
            HIPCHK(hipMemcpy(ad.data(), d->d_ad, ad.size() * 8, hipMemcpyDeviceToHost));
        }
        for (int q = 0; q < n_r; ++q) {
            if (out->al_diag) memcpy(out->al_diag + (size_t)q * Nb, ad.data() + ((size_t)q * 2 + 0) * Nb, Nb * 8);
            if (out->ar_diag) memcpy(out->ar_diag + (size_t)q * Nb, ad.data() + ((size_t)q * 2 + 1) * Nb, Nb * 8);
        }
    }
    if (out->decim_iters)
        HIPCHK(hipMemcpy(out->decim_iters, d->d_iters, (size_t)(n_c + n_r) * 2 * 4, hipMemcpyDeviceToHost));
    return st;
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
    if (!z || !sigma) return fail(NEGF_EINVAL, "z or sigma is NULL");
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(z[i].re) || !std::isfinite(z[i].im)) return fail(NEGF_EINVAL, "z[%d] not finite", i);
    HIPCHK(hipSetDevice(d->dev_id));
    TRY(ensure_energy_ws(d, n));
    hipStream_t s = d->own_stream;
    const int b = d->b, G = d->L->groups;
    HIPCHK(hipMemcpyAsync(d->d_z, z, (size_t)n * 16, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, s, d->d_status, n, 0);
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, s, d->d_flags, 1, 0);
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, s, d->d_flags + 1, 1, 0x7fffffff);
    negf::DecArgs a = dec_args(d, n, lead);
    d->L->decimate(a, (n + G - 1) / G, s);
    hipLaunchKernelGGL(negf::k_status, dim3((n + 255) / 256), dim3(256), 0, s, d->d_status, n, d->d_flags,
                       d->d_flags + 1);
    HIPCHK(hipMemcpyAsync(d->h_flags, d->d_flags, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    const size_t b2 = (size_t)b * b;
    std::vector<negf_c64> all((size_t)n * 2 * b2);
    HIPCHK(hipMemcpy(all.data(), d->d_sigma, all.size() * 16, hipMemcpyDeviceToHost));
    for (int i = 0; i < n; ++i) memcpy(sigma + (size_t)i * b2, all.data() + ((size_t)i * 2 + lead) * b2, b2 * 16);
    if (iters) {
        std::vector<int> it((size_t)n * 2);
        HIPCHK(hipMemcpy(it.data(), d->d_iters, it.size() * 4, hipMemcpyDeviceToHost));
        for (int i = 0; i < n; ++i) iters[i] = it[(size_t)i * 2 + lead];
    }
    if (d->h_flags[0] & 1)
        return fail(NEGF_ENOCONV, "lead decimation did not converge in %d steps (first node %d)",
                    d->opt.decim_max_iter, d->h_flags[1]);
    return NEGF_OK;
}

negf_status negf_set_profiling(negf_device* d, int enable) {
    if (!d) return fail(NEGF_EINVAL, "device handle is NULL");
    d->prof = enable != 0;
    for (int k = 0; k < KT_COUNT; ++k) { d->ms[k] = 0; d->calls[k] = 0; }
    return NEGF_OK;
}

negf_status negf_kernel_times(negf_device* d, const char** names, double* ms, int* calls, int* count) {
    if (!d || !count) return fail(NEGF_EINVAL, "NULL argument");
    const int n = std::min(*count, (int)KT_COUNT);
    for (int k = 0; k < n; ++k) {
        if (names) names[k] = kKernelNames[k];
        if (ms) ms[k] = d->ms[k];
        if (calls) calls[k] = d->calls[k];
    }
    *count = KT_COUNT;
    return NEGF_OK;
}

size_t negf_device_bytes(const negf_device* d) { return d ? d->bytes : 0; }

void negf_destroy(negf_device* d) {
    if (!d) return;
    (void)hipSetDevice(d->dev_id);
    if (d->own_stream) (void)hipStreamSynchronize(d->own_stream);
    for (auto& e : d->pending) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
    void* ptrs[] = {d->d_U, d->d_hdiag, d->d_ell_map, d->d_part, d->d_cidx, d->d_cval, d->d_ridx, d->d_rval, d->d_z, d->d_sigma,
                    d->d_iters, d->d_status, d->d_dscratch, d->d_coef_c, d->d_coef_r, d->d_gr, d->d_ad, d->d_T,
                    d->d_store_f, d->d_store_b, d->d_in_zc, d->d_in_wc, d->d_in_Er, d->d_in_wr, d->d_out_charge,
                    d->d_out_cur, d->d_flags};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    for (auto& ld : d->lead) {
        void* lp[] = {ld.D, ld.V, ld.VH, ld.W, ld.tau};
        for (void* p : lp)
            if (p) (void)hipFree(p);
    }
    if (d->h_flags) (void)hipHostFree(d->h_flags);
    if (d->own_stream) (void)hipStreamDestroy(d->own_stream);
    delete d;
}

}  // extern "C"
