// Self-consistency kernel of the serving loop: per request, one workgroup
// turns the NEGF charge into the next potential (Section 2.3, Algorithm 3):
//   rho_out_j = sum_i charge_{j,i}                     electrons per ring
//   Broyden's modified second method on rho (f = rho_in - rho_out)
//   1-D finite-difference Poisson along the axis with a coaxial gate:
//     a (2 phi_j - phi_{j-1} - phi_{j+1}) + phi_j = V_GS - c (rho_in_j - n_ref_j)
//     a = eps_1d / (c_gate dz^2),  c = e / (c_gate dz),  phi_{-1} = 0,  phi_N = V_DS
//   U_{j,i} = -phi_j (eV) written into the device's potential.
// Reductions run in a fixed order inside the workgroup, so a request's
// iterates do not depend on which other requests share the launch.
#pragma once
#include <hip/hip_runtime.h>

namespace negf {

constexpr int SC_THREADS = 256;
constexpr int SC_MAX_HISTORY = 32;

struct ScReq {
    int N, b, H, max_iter;
    double zeta, tol;
    double a, c;              // Poisson coefficients (see above)
    double V_GS, V_DS;
    const double* charge;     // [N*b] NEGF output of this pass
    double* U;                // [N*b] device potential (written)
    const double* n_ref;      // [N]
    double* rho_in;           // [N]
    double* rho_in_old;       // [N]
    double* f_old;            // [N]
    double* s;                // [N]
    double* Vt;               // [H+1][N] rows 1..H of V^T
    double* Wc;               // [H+1][N] columns 1..H of W
    double* work;             // [3N]
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

__device__ __forceinline__ double sc_block_max(double v, double* red) {
    const int t = threadIdx.x;
    __syncthreads();
    red[t] = v;
    __syncthreads();
    for (int w = SC_THREADS / 2; w > 0; w >>= 1) {
        if (t < w) red[t] = fmax(red[t], red[t + w]);
        __syncthreads();
    }
    return red[0];
}

// mode 0: start (rho_in = n_ref, empty history), then Poisson.
// mode 1: one pass after a NEGF solve; Poisson unless the request has stopped.
__global__ __launch_bounds__(SC_THREADS) void k_sc_step(const ScReq* reqs, int mode) {
    const ScReq& R = reqs[blockIdx.x];
    __shared__ double red[SC_THREADS];
    __shared__ double s_k[SC_MAX_HISTORY + 1];
    const int t = threadIdx.x, N = R.N, b = R.b;
    double* f = R.work;           // [N] f of this pass
    double* df = R.work + N;      // [N] Delta f
    if (mode == 0) {
        for (int j = t; j < N; j += SC_THREADS) {
            R.rho_in[j] = R.n_ref[j];
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
        }
    } else {
        if (R.stat[2] != 0) return;
        double emax = 0.0, dsum = 0.0;
        for (int j = t; j < N; j += SC_THREADS) {
            double ro = 0.0;
            for (int i = 0; i < b; ++i) ro += R.charge[(size_t)j * b + i];
            const double ri = R.rho_in[j];
            const double fj = ri - ro;
            const double dj = fj - R.f_old[j];
            f[j] = fj;
            df[j] = dj;
            emax = fmax(emax, fabs(fj / (ri + ro)));
            dsum += dj * dj;
        }
        emax = sc_block_max(emax, red);
        const double d = sc_block_sum(dsum, red);
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
    // Poisson: Thomas sweep on one lane (the matrix is diagonally dominant)
    __syncthreads();
    double* cp = R.work;             // [N] modified super-diagonal
    double* dp = R.work + N;         // [N] modified right-hand side
    double* phi = R.work + 2 * N;    // [N]
    if (t == 0) {
        const double a = R.a, diag = 2.0 * a + 1.0;
        double cprev = 0.0, dprev = 0.0;
        for (int j = 0; j < N; ++j) {
            double rhs = R.V_GS - R.c * (R.rho_in[j] - R.n_ref[j]);
            if (j == N - 1) rhs += a * R.V_DS;
            const double den = diag + a * cprev;          // sub-diagonal is -a
            const double cj = -a / den;
            const double dj = (rhs + a * dprev) / den;
            cp[j] = cj;
            dp[j] = dj;
            cprev = cj;
            dprev = dj;
        }
        double next = 0.0;
        for (int j = N - 1; j >= 0; --j) {
            const double v = dp[j] - (j + 1 < N ? cp[j] * next : 0.0);
            phi[j] = v;
            next = v;
        }
    }
    __syncthreads();
    for (int q = t; q < N * b; q += SC_THREADS) R.U[q] = -phi[q / b];
}

}  // namespace negf
