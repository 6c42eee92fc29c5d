// Self-consistency kernel of the serving loop: per request, one workgroup
// turns the NEGF charge into the next potential (Section 2.3, Algorithm 3):
//   rho_out_j = sum_i charge_{j,i}                     electrons per ring
//   Broyden's modified second method on rho (f = rho_in - rho_out)
//   1-D finite-difference Poisson along the axis with a coaxial gate:
//     a (2 phi_j - phi_{j-1} - phi_{j+1}) + phi_j = V_GS - c (rho_in_j - n_ref_j)
//     a = eps_1d / (c_gate dz^2),  c = e / (c_gate dz),  phi_{-1} = 0,  phi_N = V_DS
//   U_{j,i} = -phi_j (eV) written into the device's potential; the tridiagonal
//   system is solved with its Thomas factors (computed once per request) by two
//   workgroup-wide scans of the substitution recurrences.
// Stopping norm: the relative charge change max_j |f_j| / (rho_in_j + rho_out_j)
// of Algorithm 3, or the potential residual max_j |phi(rho_out)_j - phi(rho_in)_j|
// (eV for one electron), which the linear Poisson operator gives as the solution
// delta of  a (2 delta_j - delta_{j-1} - delta_{j+1}) + delta_j = c f_j  with
// delta_{-1} = delta_N = 0.
// The per-ring charge is a strided sum over the NEGF output (the atoms of a ring
// in real space, the ring's mode chains in mode space), and the new potential is
// written to every array that the request's NEGF step reads (one real-space
// device, or one scalar chain per mode).
// Reductions run in a fixed order inside the workgroup, so a request's
// iterates do not depend on which other requests share the launch.
#pragma once
#include <hip/hip_runtime.h>

namespace negf {

constexpr int SC_THREADS = 256;
constexpr int SC_MAX_HISTORY = 32;

struct ScReq {
    int N, H, max_iter;
    int norm;                 // 0: relative charge change; 1: potential residual (eV)
    int n_part, q_ring, q_part;   // rho_out_j = sum_{i < n_part} charge[j q_ring + i q_part]
    int n_U, U_w;             // potential arrays written, entries per ring in each
    double zeta, tol;
    double a, c;              // Poisson coefficients (see above)
    double V_GS, V_DS;
    const double* charge;     // NEGF output of this pass
    double* const* U;         // [n_U] device potentials, each [N * U_w] (written)
    const double* n_ref;      // [N]
    const double* rho0;       // [N] starting rho_in (n_ref, or a warm start)
    double* rho_in;           // [N]
    double* rho_in_old;       // [N]
    double* f_old;            // [N]
    double* s;                // [N]
    double* Vt;               // [H+1][N] rows 1..H of V^T
    double* Wc;               // [H+1][N] columns 1..H of W
    double* work;             // [4N]
    double* alf;              // [N] Thomas factors of the Poisson operator (set by mode 0):
    double* invden;           // [N]   invden_j = 1 / (2a + 1 + a cp_{j-1}), alf_j = a invden_j,
    double* mcp;              // [N]   mcp_j = -cp_j = a invden_j
    int* stat;                // [4]: m, passes, state (0 running, 1 converged, 2 pass limit)
    double* diag;             // [2]: eps_max of the last pass, |Delta f|^2
};

__device__ __forceinline__ double sc_block_sum(double v, double* red) {
    const int t = threadIdx.x;
    __syncthreads();
    red[t] = v;
    __syncthreads();
    for (int w = SC_THREADS / 2; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    return red[0];
}

// maximum that keeps a NaN (fmax would drop it)
__device__ __forceinline__ double nan_max(double x, double y) { return (x != x || y != y) ? x + y : fmax(x, y); }

__device__ __forceinline__ double sc_block_max(double v, double* red) {
    const int t = threadIdx.x;
    __syncthreads();
    red[t] = v;
    __syncthreads();
    for (int w = SC_THREADS / 2; w > 0; w >>= 1) {
        if (t < w) red[t] = nan_max(red[t], red[t + w]);
        __syncthreads();
    }
    return red[0];
}

// x_j = alpha_j x_{j-1} + beta_j for j = 0..N-1 with x_{-1} = 0 (rev: j = N-1..0 with
// x_N = 0), by the whole workgroup: every thread composes its chunk of steps into one
// affine map, the maps are combined in thread order by a fixed Hillis-Steele scan,
// and each chunk is re-run from the value it receives.  The order of operations
// depends only on N, not on the other requests of the launch.
__device__ __forceinline__ void sc_affine_scan(const double* alpha, const double* beta, double* x, int N, bool rev,
                                               double* sA, double* sB) {
    const int t = threadIdx.x;
    const int C = (N + SC_THREADS - 1) / SC_THREADS;
    const int lo = min(t * C, N), hi = min(lo + C, N);
    __syncthreads();   // beta was written by other threads (strided, not in these chunks)
    double A = 1.0, B = 0.0;
    for (int q = lo; q < hi; ++q) {
        const int j = rev ? N - 1 - q : q;
        A = alpha[j] * A;
        B = fma(alpha[j], B, beta[j]);
    }
    __syncthreads();
    sA[t] = A;
    sB[t] = B;
    __syncthreads();
    for (int o = 1; o < SC_THREADS; o <<= 1) {
        double a2 = 1.0, b2 = 0.0;
        if (t >= o) {
            a2 = sA[t - o];
            b2 = sB[t - o];
        }
        __syncthreads();
        if (t >= o) {
            const double a1 = sA[t], b1 = sB[t];
            sA[t] = a1 * a2;
            sB[t] = fma(a1, b2, b1);
        }
        __syncthreads();
    }
    double v = t > 0 ? sB[t - 1] : 0.0;
    for (int q = lo; q < hi; ++q) {
        const int j = rev ? N - 1 - q : q;
        v = fma(alpha[j], v, beta[j]);
        x[j] = v;
    }
    __syncthreads();
}

// Solves a (2 p_j - p_{j-1} - p_{j+1}) + p_j = rhs_j (p_{-1} = p_N = 0) with the
// request's Thomas factors: forward dp_j = invden_j rhs_j + alf_j dp_{j-1}, then
// p_j = dp_j + mcp_j p_{j+1}.  rhs is overwritten with invden_j rhs_j.
__device__ __forceinline__ void sc_poisson(const ScReq& R, double* rhs, double* dp, double* out, double* sA,
                                           double* sB) {
    const int N = R.N;
    for (int j = threadIdx.x; j < N; j += SC_THREADS) rhs[j] *= R.invden[j];
    sc_affine_scan(R.alf, rhs, dp, N, false, sA, sB);
    sc_affine_scan(R.mcp, dp, out, N, true, sA, sB);
}

// mode 0: start (rho_in = rho0, empty history), then Poisson.
// mode 2: resume from a restored state (re-admission), Poisson only.
// mode 1: one pass after a NEGF solve; Poisson unless the request has stopped.
__global__ __launch_bounds__(SC_THREADS) void k_sc_step(const ScReq* reqs, int mode) {
    const ScReq& R = reqs[blockIdx.x];
    __shared__ double red[SC_THREADS];
    __shared__ double s_k[SC_MAX_HISTORY + 1];
    __shared__ double s_eps;
    __shared__ double s_scanA[SC_THREADS], s_scanB[SC_THREADS];
    const int t = threadIdx.x, N = R.N;
    double* f = R.work;           // [N] f of this pass
    double* df = R.work + N;      // [N] Delta f
    if (mode == 0) {
        for (int j = t; j < N; j += SC_THREADS) {
            R.rho_in[j] = R.rho0[j];
            R.rho_in_old[j] = 0.0;
            R.f_old[j] = 0.0;
            R.s[j] = 0.0;
        }
        if (t == 0) {
            R.stat[0] = 0;
            R.stat[1] = 0;
            R.stat[2] = 0;
            R.diag[0] = 0.0;
            R.diag[1] = 0.0;
            // Thomas factors of the constant Poisson matrix (once per request)
            const double a = R.a, dg = 2.0 * a + 1.0;
            double cprev = 0.0;
            for (int j = 0; j < N; ++j) {
                const double iv = 1.0 / (dg + a * cprev);   // sub-diagonal is -a
                R.invden[j] = iv;
                R.alf[j] = a * iv;
                R.mcp[j] = a * iv;
                cprev = -a * iv;
            }
        }
    } else if (mode == 1) {
        if (R.stat[2] != 0) return;
        double emax = 0.0, dsum = 0.0;
        for (int j = t; j < N; j += SC_THREADS) {
            double ro = 0.0;
            for (int i = 0; i < R.n_part; ++i) ro += R.charge[(size_t)j * R.q_ring + (size_t)i * R.q_part];
            const double ri = R.rho_in[j];
            const double fj = ri - ro;
            const double dj = fj - R.f_old[j];
            f[j] = fj;
            df[j] = dj;
            emax = nan_max(emax, fabs(fj / (ri + ro)));
            dsum += dj * dj;
        }
        emax = sc_block_max(emax, red);
        const double d = sc_block_sum(dsum, red);
        if (R.norm == 1) {                 // potential residual: the Poisson operator on c f
            double* rhs = R.work + 2 * N;
            double* dp = R.work + 3 * N;
            __syncthreads();
            for (int j = t; j < N; j += SC_THREADS) rhs[j] = R.c * f[j];
            sc_poisson(R, rhs, dp, rhs, s_scanA, s_scanB);
            double m = 0.0;
            for (int j = t; j < N; j += SC_THREADS) m = nan_max(m, fabs(rhs[j]));
            emax = sc_block_max(m, red);
        }
        const int passes = R.stat[1] + 1;
        int m = R.stat[0];
        __syncthreads();
        if (t == 0) {
            R.stat[1] = passes;
            R.diag[0] = emax;
            R.diag[1] = d;
        }
        if (!(emax >= R.tol)) {            // converged (a NaN norm stops at the pass limit instead)
            if (t == 0 && emax == emax) R.stat[2] = 1;
            if (emax == emax) return;
        }
        if (passes >= R.max_iter || emax != emax) {
            if (t == 0) R.stat[2] = 2;
            return;
        }
        if (m > R.H) {                      // history exhausted: restart
            m = 0;
            for (int j = t; j < N; j += SC_THREADS) R.s[j] = 0.0;
        }
        if (m > 0) {
            if (m > 1) {
                for (int q = 1; q < m; ++q) {
                    double p = 0.0;
                    for (int j = t; j < N; j += SC_THREADS) p += R.Vt[(size_t)q * N + j] * df[j];
                    const double kq = sc_block_sum(p, red);
                    if (t == 0) s_k[q] = kq;
                }
                __syncthreads();
                for (int j = t; j < N; j += SC_THREADS) {
                    double acc = 0.0;
                    for (int q = 1; q < m; ++q) acc += R.Wc[(size_t)q * N + j] * s_k[q];
                    R.s[j] = acc;
                }
            }
            for (int j = t; j < N; j += SC_THREADS) {
                R.Vt[(size_t)m * N + j] = df[j] / d;
                R.Wc[(size_t)m * N + j] = -R.zeta * df[j] + R.rho_in[j] - R.rho_in_old[j] - R.s[j];
            }
            __syncthreads();
            for (int q = 1; q <= m; ++q) {
                double p = 0.0;
                for (int j = t; j < N; j += SC_THREADS) p += R.Vt[(size_t)q * N + j] * f[j];
                const double kq = sc_block_sum(p, red);
                if (t == 0) s_k[q] = kq;
            }
            __syncthreads();
            for (int j = t; j < N; j += SC_THREADS) {
                double acc = 0.0;
                for (int q = 1; q <= m; ++q) acc += R.Wc[(size_t)q * N + j] * s_k[q];
                R.s[j] = acc;
            }
        }
        for (int j = t; j < N; j += SC_THREADS) {
            const double ri = R.rho_in[j];
            R.rho_in_old[j] = ri;
            R.rho_in[j] = ri - R.zeta * f[j] - R.s[j];
            R.f_old[j] = f[j];
        }
        if (t == 0) R.stat[0] = m + 1;
    }
    // Poisson: Thomas factors and two workgroup scans (the matrix is diagonally dominant)
    __syncthreads();
    double* rhs = R.work;            // [N] right-hand side
    double* dp = R.work + N;         // [N] forward substitution
    double* phi = R.work + 2 * N;    // [N]
    for (int j = t; j < N; j += SC_THREADS) {
        double r = R.V_GS - R.c * (R.rho_in[j] - R.n_ref[j]);
        if (j == N - 1) r += R.a * R.V_DS;
        rhs[j] = r;
    }
    sc_poisson(R, rhs, dp, phi, s_scanA, s_scanB);
    for (int u = 0; u < R.n_U; ++u) {
        double* Uu = R.U[u];
        const int w = R.U_w;
        for (int q = t; q < N * w; q += SC_THREADS) Uu[q] = -phi[q / w];
    }
}

}  // namespace negf
