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
    const int* status;         // [n_c + n_r] decimation status
    int* flags;                // [2]: bit 1 no convergence, bit 2 non-finite; first bad node
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
    if (e == 0) { J.flags[0] = 0; J.flags[1] = 0x7fffffff; }
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
    if (e < R.n_c + R.n_r && R.status[e]) {
        atomicOr(R.flags, R.status[e]);
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
    if (!isfinite(ch)) atomicOr(R.flags, 2);
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
        if (!isfinite(cur)) atomicOr(R.flags, 2);
    }
}

__global__ void k_fill_int(int* p, int n, int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace negf
