// Energy-sum kernels (Eq. 4-5) and per-job helpers; used by the C-ABI unit only.
// Every kernel covers all jobs of a solve (job index = blockIdx.y or .z).
#pragma once
#include <hip/hip_runtime.h>

#include "negf_kernels.hpp"

namespace negf {

struct RedJob {
    int Nb, n_c, n_r;          // n_c counts every contour-type node: given nodes, then poles
    int n_ci, n_p;             // given contour nodes, Fermi poles (residue nodes)
    int no_fermi;              // 1: contour weights are used without F (zero-temperature arc)
    double g_s, eta;
    double mu_L, mu_R, kT_L, kT_R;
    const cx<double>* z_c;     // [n_c] inputs (device)
    const cx<double>* w_c;     // [n_c]
    const double* E_r;         // [n_r]
    const double* w_r;         // [n_r]
    cx<double>* z;             // [n_c + n_r] node array of the job (written by k_nodes)
    cx<double>* coef_c;        // [n_c]   w_c F(z_c - mu_min; kT_min)
    double* coef_r;            // [n_r][4] w fL, w fR, w (fL - fR), w (-dF/dE)(E - mu_L; kT_L)
    const void* gr_diag;       // [n_c][Nb] cx<TG>
    const void* a_diag;        // [n_r][2][Nb] TA
    const double* T;           // [n_r]
    double* part;              // [RED_SEGS][Nb]
    double* charge;            // [Nb]
    double* current;           // [1] or null
    double* conductance;       // [1] or null: g_s (e^2/h) sum w T (-dF/dE), Eq. 6
    const int* status;         // [n_c + n_r] ST_* bits per node
    int* flags;                // [4]: ST_NOCONV | ST_BAD | ST_NOROOM of any node; first bad node;
                               //      nodes recomputed in FP64; unused
};

__device__ __forceinline__ double fermi_real(double E, double mu, double kT) {
    const double x = (E - mu) / kT;
    if (x > 0) { const double e = exp(-x); return e / (1.0 + e); }
    return 1.0 / (1.0 + exp(x));
}

// f_L(E) - f_R(E) (Eq. 5) as -expm1(x_L - x_R) f(x_L) f(-x_R), an identity whose
// factors all keep full relative precision; the plain difference of two Fermi
// factors close to 1 (E far below both levels, where in-band transmissions are
// of order one) keeps only a few digits.  Beyond |x_L - x_R| > 700 the plain
// difference is exact enough and the exponential would overflow.
__device__ __forceinline__ double fermi_diff(double E, double mu_L, double kT_L, double mu_R, double kT_R) {
    const double xL = (E - mu_L) / kT_L, xR = (E - mu_R) / kT_R;
    const double d = xL - xR;
    const double fl = fermi_real(E, mu_L, kT_L);
    if (fabs(d) > 700.0) return fl - fermi_real(E, mu_R, kT_R);
    return -expm1(d) * fl * fermi_real(-E, -mu_R, kT_R);
}

__device__ __forceinline__ cx<double> fermi_cplx(cx<double> z, double mu, double kT) {
    // 1/(1 + exp(u)), u = (z - mu)/kT, evaluated through exp(-u) when Re u > 0
    const double ur = (z.re - mu) / kT, ui = z.im / kT;
    const bool pos = ur > 0;
    const double m = exp(pos ? -ur : ur);
    const double c = m * cos(pos ? -ui : ui), s = m * sin(pos ? -ui : ui);   // e = exp(+-u)
    const double dr = 1.0 + c, di = s;                                      // 1 + e
    const double den = dr * dr + di * di;
    // pos: F = e / (1 + e);  else: F = 1 / (1 + e)
    const double nr = pos ? c : 1.0, ni = pos ? s : 0.0;
    return cx<double>{(nr * dr + ni * di) / den, (ni * dr - nr * di) / den};
}

// node array (contour nodes as given, then the Fermi poles mu_min + i(2k+1) pi kT_min,
// then real nodes E + i eta), status and flags reset
__global__ void k_nodes(const RedJob* jobs, int* status_all, int status_n) {
    const RedJob& J = jobs[blockIdx.y];
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < J.n_ci) {
        J.z[e] = J.z_c[e];
    } else if (e < J.n_c) {
        const double pi = 3.14159265358979323846;
        J.z[e] = cx<double>{fmin(J.mu_L, J.mu_R), (2 * (e - J.n_ci) + 1) * pi * fmin(J.kT_L, J.kT_R)};
    } else if (e < J.n_c + J.n_r) {
        J.z[e] = cx<double>{J.E_r[e - J.n_c], J.eta};
    }
    if (blockIdx.y == 0) {
        for (int i = e; i < status_n; i += gridDim.x * blockDim.x) status_all[i] = 0;
    }
    if (e == 0) { J.flags[0] = 0; J.flags[1] = 0x7fffffff; J.flags[2] = 0; J.flags[3] = 0; }
}

__global__ void k_coef(const RedJob* jobs) {
    const RedJob& R = jobs[blockIdx.y];
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const double mu_min = fmin(R.mu_L, R.mu_R), kT_min = fmin(R.kT_L, R.kT_R);
    if (e < R.n_ci) {
        const cx<double> w = R.w_c[e];
        if (R.no_fermi) {
            R.coef_c[e] = w;
        } else {
            const cx<double> F = fermi_cplx(R.z_c[e], mu_min, kT_min);
            R.coef_c[e] = cx<double>{w.re * F.re - w.im * F.im, w.re * F.im + w.im * F.re};
        }
    } else if (e < R.n_c) {
        // residue of G F at a pole of F: -kT G(z_k); the closed path adds -2 pi i kT G(z_k)
        const double pi = 3.14159265358979323846;
        R.coef_c[e] = cx<double>{0.0, -2.0 * pi * kT_min};
    } else if (e < R.n_c + R.n_r) {
        const int q = e - R.n_c;
        const double fl = fermi_real(R.E_r[q], R.mu_L, R.kT_L);
        const double fr = fermi_real(R.E_r[q], R.mu_R, R.kT_R);
        const double w = R.w_r[q];
        const double x = 0.5 * (R.E_r[q] - R.mu_L) / R.kT_L;
        const double ch = cosh(fmin(fabs(x), 350.0));
        R.coef_r[4 * q + 0] = w * fl;
        R.coef_r[4 * q + 1] = w * fr;
        R.coef_r[4 * q + 2] = w * fermi_diff(R.E_r[q], R.mu_L, R.kT_L, R.mu_R, R.kT_R);
        R.coef_r[4 * q + 3] = w / (4.0 * R.kT_L * ch * ch);
    }
    const int st = e < R.n_c + R.n_r ? (R.status[e] & (ST_NOCONV | ST_BAD | ST_NOROOM)) : 0;
    if (st) {
        atomicOr(R.flags, st);
        atomicMin(R.flags + 1, e);
    }
}

// charge_i in two fixed-order passes: energy segment `seg` (a fixed split of the
// job's node index range) is summed in index order into part[seg][i], then the
// segments are added in order.  The result depends only on the job's node list.
constexpr int RED_SEGS = 32;

template <typename TG, typename TA>
__global__ void k_reduce_part(const RedJob* jobs) {
    const RedJob& R = jobs[blockIdx.z];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int seg = blockIdx.y;
    if (i >= R.Nb) return;
    const int ne = R.n_c + R.n_r;
    const int e_lo = (int)(((long long)ne * seg) / RED_SEGS), e_hi = (int)(((long long)ne * (seg + 1)) / RED_SEGS);
    double acc_c = 0.0, acc_r = 0.0;
    const cx<TG>* gr = reinterpret_cast<const cx<TG>*>(R.gr_diag);
    const TA* ad = reinterpret_cast<const TA*>(R.a_diag);
    for (int e = e_lo; e < e_hi; ++e) {
        if (e < R.n_c) {
            const cx<TG> gv = gr[(size_t)e * R.Nb + i];
            const cx<double> w = R.coef_c[e];
            acc_c += w.re * (double)gv.im + w.im * (double)gv.re;    // Im(w G)
        } else {
            const int q = e - R.n_c;
            const double al = (double)ad[((size_t)q * 2 + 0) * R.Nb + i];
            const double ar = (double)ad[((size_t)q * 2 + 1) * R.Nb + i];
            acc_r += R.coef_r[4 * q + 0] * al + R.coef_r[4 * q + 1] * ar;
        }
    }
    const double inv_pi = 0.31830988618379067154;
    R.part[(size_t)seg * R.Nb + i] = -inv_pi * acc_c + 0.5 * inv_pi * acc_r;
}

__global__ void k_reduce_final(const RedJob* jobs) {
    const RedJob& R = jobs[blockIdx.y];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= R.Nb) return;
    double acc = 0.0;
    for (int seg = 0; seg < RED_SEGS; ++seg) acc += R.part[(size_t)seg * R.Nb + i];
    const double ch = R.g_s * acc;
    R.charge[i] = ch;
    if (!isfinite(ch)) atomicOr(R.flags, (int)ST_BAD);
}

// current: one wavefront per job, lane l sums nodes l, l+64, ... then a fixed tree
__global__ __launch_bounds__(64) void k_current(const RedJob* jobs) {
    const RedJob& R = jobs[blockIdx.x];
    __shared__ double red[2][64];
    const int l = threadIdx.x;
    double acc = 0.0, accg = 0.0;
    for (int q = l; q < R.n_r; q += 64) {
        acc += R.coef_r[4 * q + 2] * R.T[q];
        accg += R.coef_r[4 * q + 3] * R.T[q];
    }
    red[0][l] = acc;
    red[1][l] = accg;
    __syncthreads();
    for (int s = 32; s > 0; s >>= 1) {
        if (l < s) {
            red[0][l] += red[0][l + s];
            red[1][l] += red[1][l + s];
        }
        __syncthreads();
    }
    if (l == 0) {
        const double G0 = 1.602176634e-19 * 1.602176634e-19 / 6.62607015e-34;   // e^2/h
        const double cur = R.g_s * G0 * red[0][0];
        if (R.current) *R.current = cur;
        if (R.conductance) *R.conductance = R.g_s * G0 * red[1][0];
        if (!isfinite(cur)) atomicOr(R.flags, (int)ST_BAD);
    }
}

// Charge (electrons per atom) a node may move before its FP32 result is replaced.
#ifndef NEGF_FP32_QTOL
#define NEGF_FP32_QTOL 1e-7
#endif

// Current a node's transmission may move, relative to its job's current scale,
// before its FP32 result is replaced.
#ifndef NEGF_FP32_ITOL
#define NEGF_FP32_ITOL 1e-6
#endif

// FP32-bulk: per job, the scale of its current, sum_q |w_q (f_L - f_R)(E_q) T_q| over
// its real-axis nodes, in a fixed order (one wavefront per job).
__global__ __launch_bounds__(64) void k_cur_scale(const JobDesc* jobs, const RedJob* red, double* scale) {
    const RedJob& R = red[blockIdx.x];
    const JobDesc& J = jobs[blockIdx.x];
    __shared__ double s[64];
    const int l = threadIdx.x;
    double acc = 0.0;
    for (int q = l; q < R.n_r; q += 64)
        acc += fabs(R.w_r[q] * fermi_diff(R.E_r[q], R.mu_L, R.kT_L, R.mu_R, R.kT_R) * J.Tout[q]);
    s[l] = acc;
    __syncthreads();
    for (int d = 32; d > 0; d >>= 1) {
        if (l < d) s[l] += s[l + d];
        __syncthreads();
    }
    if (l == 0) scale[blockIdx.x] = s[0];
}

// FP32-bulk, after the lead columns of every chunk of one kernel group: the
// real-axis nodes to recompute in FP64.  A node is taken when the lead columns
// marked it (ST_FP64), or when its two transmissions disagree by more than its
// weight allows: T_LR comes from the right lead column (forward recursion), T_RL
// from the left one (backward recursion), and they agree up to O(eta) unless an
// FP32 recursion lost digits; with r = |T_LR - T_RL| / max(T_LR, T_RL) and the
// node's largest charge term c = g_s (|w|/pi) (f_L max_i A_L,ii + f_R max_i A_R,ii)
// the node is taken when c sqrt(r) > NEGF_FP32_QTOL, or when |w (f_L - f_R)| |T_LR - T_RL|
// exceeds NEGF_FP32_ITOL of the job's sum_q |w_q (f_L - f_R) T_q| (sqrt(r): the spectral
// densities were measured to be off by up to ~100 r on the nanotube workloads).
// The taken nodes are listed in node order as one-node spans whose `off` is the
// running sum of their FP64 store sizes (N b^2 elements each); *count receives
// their number.  col[0..n_col) are the group's column spans, col_first their node
// prefix.  One workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_fp64_list(const JobDesc* jobs, const RedJob* red, const Span* col,
                                                   const int* col_first, int n_col, int B, Span* all, int* count,
                                                   const double* cscale) {
    __shared__ long long s_wsz[16];   // per-wavefront totals of a chunk
    __shared__ int s_wct[16];
    __shared__ long long s_base;
    __shared__ int s_seen;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid == 0) {
        s_base = 0;
        s_seen = 0;
    }
    __syncthreads();
    const int total = col_first[n_col];
    int top = 1;   // largest power of two <= n_col
    while (2 * top <= n_col) top *= 2;
    constexpr int PER = 4;   // consecutive nodes per thread, their loads in flight together
    for (int base = 0; base < total; base += 1024 * PER) {
        const int t0 = base + PER * tid;
        // span of each node: the largest lo with col_first[lo] <= t (a non-empty span),
        // by a fixed number of halving steps so the searches of the PER nodes interleave
        int lo[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) lo[k] = 0;
        for (int step = top; step >= 1; step >>= 1) {
#pragma unroll
            for (int k = 0; k < PER; ++k)
                if (lo[k] + step < n_col && col_first[lo[k] + step] <= t0 + k) lo[k] += step;
        }
        int job[PER], e[PER], ct[PER];
        long long sz[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int t = t0 + k;
            job[k] = 0;
            e[k] = 0;
            ct[k] = 0;
            sz[k] = 0;
            if (t >= total) continue;
            const Span sp = col[lo[k]];
            job[k] = sp.job;
            e[k] = sp.e0 + (t - col_first[lo[k]]);
            const JobDesc& J = jobs[job[k]];
            const RedJob& R = red[job[k]];
            const int ir = e[k] - J.n_c;
            const double t1 = J.Tout[ir], t2 = J.Trl[ir];
            const double tmax = fmax(fabs(t1), fabs(t2));
            const double r = tmax > 0.0 ? fabs(t1 - t2) / tmax : 0.0;
            const double E = R.E_r[ir];
            const double c = R.g_s * fabs(R.w_r[ir]) * 0.31830988618379067154 *
                             (fermi_real(E, R.mu_L, R.kT_L) * J.amax[2 * ir] +
                              fermi_real(E, R.mu_R, R.kT_R) * J.amax[2 * ir + 1]);
            const bool recip = !(c * sqrt(r) <= NEGF_FP32_QTOL);
            // and when the mismatch could move the job's current by more than NEGF_FP32_ITOL of its scale
            const double wf = fabs(R.w_r[ir] * fermi_diff(E, R.mu_L, R.kT_L, R.mu_R, R.kT_R));
            const bool cur = wf * fabs(t1 - t2) > NEGF_FP32_ITOL * cscale[job[k]];
            const bool take =
                J.fp64_policy == 1 || (J.fp64_policy == 0 && ((J.status[e[k]] & ST_FP64) || recip || cur));
            if (take) {
                ct[k] = 1;
                sz[k] = (long long)J.N * B * B;
            }
        }
        long long ts = 0;   // this thread's totals
        int tc = 0;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            ts += sz[k];
            tc += ct[k];
        }
        const long long b0 = s_base;   // list so far (updated below, after every thread has read it)
        const int c0 = s_seen;
        // inclusive scans of the thread totals in node order: within the wavefront by
        // shuffles, then over the totals of the wavefronts before this one
        long long xs = ts;
        int xc = tc;
        for (int d = 1; d < 64; d <<= 1) {
            const long long ys = __shfl_up(xs, d, 64);
            const int yc = __shfl_up(xc, d, 64);
            if (lane >= d) {
                xs += ys;
                xc += yc;
            }
        }
        if (lane == 63) {
            s_wsz[wv] = xs;
            s_wct[wv] = xc;
        }
        __syncthreads();
        for (int q = 0; q < wv; ++q) {
            xs += s_wsz[q];
            xc += s_wct[q];
        }
        long long off = b0 + xs - ts;   // store offset and list slot of this thread's first taken node
        int slot = c0 + xc - tc;
#pragma unroll
        for (int k = 0; k < PER; ++k)
            if (ct[k]) {
                all[slot++] = Span{job[k], e[k], 1, 0, off};
                off += sz[k];
            }
        if (tid == 1023) {
            s_base = b0 + xs;
            s_seen = c0 + xc;
        }
        __syncthreads();
    }
    if (tid == 0) *count = s_seen;
}

// One round of FP64 recomputation: the listed nodes from *cursor on whose FP64
// stores fit `cap` elements (a prefix, the store offsets growing along the list)
// become the spans of this round, with offsets relative to the round's first
// node; the unit prefix out_first[k] = 2 min(k, taken) serves the recursion
// (two directions) and the lead-column launches (two leads).  The cursor moves
// past them; on the last round the nodes left are marked ST_NOROOM.  One
// workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_fp64_round(const JobDesc* jobs, const Span* all, const int* count,
                                                    int* cursor, int B, long long cap, Span* out, int* out_first,
                                                    int max_out, int last) {
    __shared__ int s_take;
    const int tid = threadIdx.x;
    const int n = *count, c0 = *cursor;
    const long long base = c0 < n ? all[c0].off : 0;
    if (tid == 0) {
        // largest m with end(c0 + m - 1) - base <= cap, by bisection on the monotone ends
        int lo = 0, hi = min(n - c0, max_out);   // m in [lo, hi]
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            const Span sp = all[c0 + mid - 1];
            const long long end = sp.off + (long long)jobs[sp.job].N * B * B;
            if (end - base <= cap) lo = mid; else hi = mid - 1;
        }
        s_take = lo;
    }
    __syncthreads();
    const int m = s_take;
    for (int k = tid; k < m; k += 1024) {
        Span sp = all[c0 + k];
        sp.off -= base;
        out[k] = sp;
        atomicAdd(jobs[sp.job].n_fp64, 1);
    }
    for (int k = tid; k <= max_out; k += 1024) out_first[k] = 2 * min(k, m);
    if (last) {
        for (int k = c0 + m + tid; k < n; k += 1024) atomicOr(&jobs[all[k].job].status[all[k].e0], (int)ST_NOROOM);
    }
    __syncthreads();
    if (tid == 0) *cursor = c0 + m;
}

__global__ void k_fill_int(int* p, int n, int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace negf
