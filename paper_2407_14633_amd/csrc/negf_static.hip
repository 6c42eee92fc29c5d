// Allocation-free single-device solve: the solve of negf_solve_dev with every
// work buffer (per-node arrays, recursion stores, decimation state, schedule
// tables, counters) placed in one fixed device array instead of memory from
// hipMalloc.  For callers that cannot allocate device memory while they run.
#include <hip/hip_runtime.h>

#include <mutex>

#include "negf_internal.hpp"

// Size of the fixed work area (MiB): with a 512 MiB area a 400-ring (17,0) tube
// with 2048 nodes runs in chunks of about 70 nodes.
#ifndef NEGF_STATIC_SCRATCH_MIB
#define NEGF_STATIC_SCRATCH_MIB 512
#endif

static constexpr size_t kScratchBytes = (size_t)NEGF_STATIC_SCRATCH_MIB << 20;

// The fixed work area: every GPU the library runs on holds its own copy until
// the process ends.  In host code this name is only a handle for the symbol
// lookup below; kernels receive the device address it resolves to.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char* g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch`, per HIP device

// Address of this device's copy of `scratch`, looked up once per device with
// that device current.
negf_status scratch_ptr(int dev, char** out) {
    if (dev < 0 || dev >= kMaxDevices) return negf_host::fail(NEGF_EINVAL, "HIP device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return negf_host::fail(NEGF_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<char*>(p);
    }
    *out = g_scratch_ptr[dev];
    return NEGF_OK;
}

}  // namespace

using namespace negf_host;

extern "C" {

size_t negf_static_scratch_bytes(void) { return kScratchBytes; }

negf_status negf_solve_dev_static(negf_device* d, const negf_bias* bias, int n_c, const negf_c64* z_c,
                                  const negf_c64* w_c, int n_r, const double* E_r, const double* w_r,
                                  double* charge, double* T, double* current, void* hip_stream) {
    if (!d) return fail(NEGF_EINVAL, "device handle is NULL");
    if (!bias) return fail(NEGF_EINVAL, "bias is NULL");
    negf_job j{};
    j.dev = d;
    j.bias = *bias;
    j.n_c = n_c;
    j.z_c = z_c;
    j.w_c = w_c;
    j.n_r = n_r;
    j.E_r = E_r;
    j.w_r = w_r;
    j.charge = charge;
    j.T = T;
    j.current = current;
    TRY(check_job(j, 0, false));
    HIPCHK(hipSetDevice(d->dev_id));
    char* area = nullptr;
    TRY(scratch_ptr(d->dev_id, &area));
    // A workspace that owns nothing: buffers come from the fixed area; the status
    // slots, the completion event and the schedule settings are the handle's own
    // (created with the handle), so negf_sync(d) reports this solve's status.
    negf_workspace* own = d->ws;
    negf_workspace w;
    w.dev_id = own->dev_id;
    w.cus = own->cus;
    w.done = own->done;
    w.side = own->side;
    w.ev_fork = own->ev_fork;
    w.ev_join = own->ev_join;
    w.h_flags = own->h_flags;
    w.cap_flags = own->cap_flags;
    w.grid_scale = own->grid_scale;
    w.order = own->order;
    w.circ_decimation = own->circ_decimation;
    w.fp64_policy = own->fp64_policy;
    for (int b = 0; b <= NEGF_MAX_RING; ++b) w.gpw_b[b] = own->gpw_b[b];
    w.arena = area;
    w.arena_cap = kScratchBytes;
    const negf_status st = enqueue(&w, 1, &j, (hipStream_t)hip_stream);
    own->last_n_jobs = w.last_n_jobs;
    own->last_max_iter = w.last_max_iter;
    return st;
}

}  // extern "C"
