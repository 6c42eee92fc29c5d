// Host-side internals shared by the C-ABI units (solves, batches, graphs, server).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "negf.h"
#include "negf_launch.hpp"

using negf::cx;

namespace negf_host {

extern thread_local std::string g_err;

negf_status fail(negf_status s, const char* fmt, ...);

#define HIPCHK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail(NEGF_EHIP, "%s: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

#define TRY(expr)                       \
    do {                                \
        negf_status s_ = (expr);        \
        if (s_ != NEGF_OK) return s_;   \
    } while (0)

const negf::Launchers* launchers_for(int b);

bool finite_c(const negf_c64* p, size_t n);

enum { KT_DECIMATE = 0, KT_RECUR, KT_CDIAG, KT_COLUMN, KT_REDUCE, KT_FP64, KT_COUNT };

// Device flag slots per job: status bits of any node, first bad node, nodes
// recomputed in FP64 (FP32-bulk form), unused.
constexpr int kFlagInts = 4;
extern const char* const kKernelNames[KT_COUNT];

struct LeadDev {
    int period = 1;
    std::vector<negf_c64> h_diag;   // host copy, lead potential added on upload
    cx<double>* D = nullptr;        // [P][b][b] incl. lead potential
    cx<double>* V = nullptr;        // h_up[0]
    cx<double>* VH = nullptr;       // h_up[0]^H
    cx<double>* W = nullptr;        // h_up[P-1]
    cx<double>* tau = nullptr;
    bool circ = false;              // every lead block and tau ring-circulant
    std::vector<negf_c64> modes0;   // [5][b] ring-mode eigenvalues, lead potential excluded
    cx<double>* modes = nullptr;    // device copy with the lead potential added
};

// A growable device buffer (contents are not preserved when it grows).
struct DBuf {
    void* p = nullptr;
    size_t cap = 0;
};

}  // namespace negf_host

using negf_host::DBuf;
using negf_host::LeadDev;
using negf_host::KT_COUNT;
using negf_host::kFlagInts;

struct negf_workspace {
    int dev_id = 0;
    size_t store_cap = 0;     // bytes per recursion store direction; 0 = default
    size_t default_store_cap = (size_t)8 << 30;   // set at creation from the free HBM
    int cus = 0;
    DBuf cscale;              // FP32-bulk: per-job current scale for the recomputation test
    DBuf tables, counters, z, sigma, iters, status, coef_c, coef_r, T, gr, ad, part, store_f, store_b, scratch,
        flags, in_zc, in_wc, in_Er, in_wr, out_charge, out_T, out_cur, fp64_spans, fp64_first, Trl, amax, fp64_all, fp64_ctl;
    std::vector<char> last_tables;   // host image of `tables` (re-uploaded only when it changes)
    hipEvent_t done = nullptr;       // recorded after each enqueued solve
    int* h_flags = nullptr;   // pinned [2 * cap_flags]
    int cap_flags = 0;
    int last_n_jobs = 0;
    std::vector<int> last_max_iter;
    std::vector<int> last_fp64;      // per job of the last finished solve: nodes recomputed in FP64
    hipStream_t own_stream = nullptr;
    // contour diagonals run on `side` beside the lead columns of the same chunk:
    // forked after the recursion, joined before anything else touches the stores
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // profiling
    bool prof = false;
    struct Ev { int kind; hipEvent_t a, b; };
    std::vector<Ev> pending;
    double ms[KT_COUNT] = {0};
    int calls[KT_COUNT] = {0};
    size_t bytes = 0;
    // schedule knobs (results do not depend on them)
    int grid_scale = 1;       // persistent workgroups per (resident workgroups x CU)
    int order = 0;            // 0: longest chains first, 1: jobs in the caller's order
    bool circ_decimation = true;   // ring-circulant leads decimated in the ring Fourier basis
    int fp64_policy = 0;      // FP32-bulk real nodes recomputed in FP64: 0 marked ones, 1 all, 2 none
    int gpw_b[NEGF_MAX_RING + 1] = {0};   // chains per wavefront by ring size (0: as many as fit)
    bool capturing = false;   // enqueue is being recorded into a graph
    // Arena mode (allocation-free solves): every buffer is carved from [arena,
    // arena + arena_cap) at each enqueue instead of being grown with hipMalloc.
    char* arena = nullptr;
    size_t arena_cap = 0, arena_off = 0;
};

struct negf_device {
    int dev_id = 0;
    int N = 0, b = 0;
    negf_options opt{};
    const negf::Launchers* L = nullptr;
    int K = 1, n_uniq = 1;
    bool hdiag_zero = true;
    double hnorm = 0.0;             // max row sum of |H| (on-site blocks and both couplings)
    double* d_U = nullptr;
    cx<double>* d_hdiag = nullptr;
    int* d_ell_map = nullptr;
    int* d_cidx = nullptr;
    cx<double>* d_cval = nullptr;
    int* d_ridx = nullptr;
    cx<double>* d_rval = nullptr;
    LeadDev lead[2];
    double U_lead[2] = {0.0, 0.0};
    negf_workspace* ws = nullptr;   // private workspace of the single-device calls
    size_t bytes = 0;
};


namespace negf_host {

negf_status grow(negf_workspace* w, DBuf& buf, size_t bytes);
negf_status wait_prev(negf_workspace* w);
negf_status check_job(const negf_job& j, int idx, bool host);
negf_status check_batch(negf_workspace* w, int n_jobs, const negf_job* jobs, bool host);
negf_status enqueue(negf_workspace* w, int n_jobs, const negf_job* jobs, hipStream_t s,
                    bool decimation_only = false);
negf_status finish(negf_workspace* w, int* failed_job);
negf_status ws_create(negf_workspace** out, size_t store_bytes);
void ws_destroy(negf_workspace* w);

// negf_create_device; own_ws = false leaves out the handle's private workspace
// (stream, event, pinned flags), for devices that only ever run in batches on a
// caller's workspace (the scalar chains of a mode-space tube).
negf_status create_device(negf_device** out, int n_rings, int b, const negf_c64* h_diag, const negf_c64* h_up,
                          const negf_lead* left, const negf_lead* right, const negf_options* opt, bool own_ws);

// Ring-circulant test of a b x b block: M[i][j] == M[0][(j - i) mod b], exactly.
bool ring_circulant(const negf_c64* M, int b);

// Semi-adaptive real-axis grid (Section 3.3).  grid_window: [E_min, E_max] of
// Eq. 4 and kT_min.  grid_parts: Gauss-Legendre nodes/weights on the three parts
// split at l1 <= l2, density[p] nodes per kT (at least one per non-empty part).
// grid_refine: peak E_s of the probe integrand on the grid of the guessed limits
// (first maximum), refined limits {l1 - a kT, E_s + b kT} clipped to the window.
void grid_window(const negf_bias& bias, double* E_min, double* E_max, double* kT);
void grid_parts(double E_min, double E_max, double l1, double l2, const double* density, double kT,
                std::vector<double>& E, std::vector<double>& W);
void grid_refine(const negf_bias& bias, const std::vector<double>& Ep, const std::vector<double>& integrand,
                 double l1, double a, double b, double* n1, double* n2, double* Es);
double host_fermi(double E, double mu, double kT);

}  // namespace negf_host

// A tube in mode space: one scalar chain (ring size 1) per kept ring mode.
struct negf_modes {
    int N = 0, b = 0;
    std::vector<int> modes;
    std::vector<negf_device*> devs;
};
