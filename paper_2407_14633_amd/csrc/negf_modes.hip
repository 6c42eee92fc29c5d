// Mode-space solves (Section 2.2.2: the CNT in the mode-space approximation, with blocks
// that are single numbers, one per mode).
//
// When every ring block is circulant (H[i][j] depends only on (j - i) mod b, as
// for a nanotube ring whose atoms are related by the rotation symmetry) and the
// potential is uniform on each ring, the Fourier vectors v_q[j] = e^{2 pi i q j/b}
// / sqrt(b) diagonalise every block at once: block C becomes the scalar
// lambda_q(C) = sum_k C[0][k] e^{2 pi i q k / b} in mode q, and the device splits
// into b independent chains with 1 x 1 blocks.  The solve then costs O(b N) per
// node instead of O(b^3 N).  With every mode kept the result is exact; keeping a
// subset is the paper's mode-space approximation (charge and current of the kept
// modes only).  Per-atom charge of ring j: (1/b) sum_q charge_q[j], since
// |v_q[j]|^2 = 1/b; transmission and current add over modes.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <vector>

#include "negf_internal.hpp"

using namespace negf_host;

namespace {

negf_c64 mode_value(const negf_c64* M, int b, int q) {
    std::complex<double> acc(0.0, 0.0);
    const double pi = 3.14159265358979323846;
    for (int k = 0; k < b; ++k) {
        const double ph = 2.0 * pi * (double)((long long)q * k % b) / b;
        acc += std::complex<double>(M[k].re, M[k].im) * std::complex<double>(std::cos(ph), std::sin(ph));
    }
    return negf_c64{acc.real(), acc.imag()};
}

}  // namespace

bool negf_host::ring_circulant(const negf_c64* M, int b) {
    for (int i = 0; i < b; ++i)
        for (int j = 0; j < b; ++j) {
            const negf_c64 a = M[(size_t)i * b + j], c = M[(size_t)((j - i + b) % b)];
            if (a.re != c.re || a.im != c.im) return false;
        }
    return true;
}

extern "C" {

void negf_modes_destroy(negf_modes* m) {
    if (!m) return;
    for (negf_device* d : m->devs) negf_destroy(d);
    delete m;
}

negf_status negf_modes_create(negf_modes** out, int n_rings, int b, const negf_c64* h_diag, const negf_c64* h_up,
                              const negf_lead* left, const negf_lead* right, const negf_options* opt, int n_modes,
                              const int* modes) {
    if (!out) return fail(NEGF_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_rings < 1 || b < 1) return fail(NEGF_EINVAL, "n_rings and b must be >= 1");
    if (!h_diag || (n_rings > 1 && !h_up) || !left || !right) return fail(NEGF_EINVAL, "NULL argument");
    if (n_modes < 0 || n_modes > b || (n_modes > 0 && !modes)) return fail(NEGF_EINVAL, "bad mode list");
    const size_t b2 = (size_t)b * b;
    for (int j = 0; j < n_rings; ++j)
        if (!ring_circulant(h_diag + j * b2, b)) return fail(NEGF_EINVAL, "h_diag[%d] is not circulant", j);
    for (int j = 0; j + 1 < n_rings; ++j)
        if (!ring_circulant(h_up + j * b2, b)) return fail(NEGF_EINVAL, "h_up[%d] is not circulant", j);
    const negf_lead* ls[2] = {left, right};
    for (int l = 0; l < 2; ++l) {
        const negf_lead* L = ls[l];
        if (L->period < 1 || L->period > NEGF_MAX_PERIOD || !L->h_diag || !L->h_up || !L->tau)
            return fail(NEGF_EINVAL, "bad lead %d", l);
        for (int r = 0; r < L->period; ++r)
            if (!ring_circulant(L->h_diag + r * b2, b) || !ring_circulant(L->h_up + r * b2, b))
                return fail(NEGF_EINVAL, "lead %d blocks are not circulant", l);
        if (!ring_circulant(L->tau, b)) return fail(NEGF_EINVAL, "lead %d coupling is not circulant", l);
    }
    negf_modes* m = new negf_modes();
    m->N = n_rings;
    m->b = b;
    if (n_modes == 0) {
        for (int q = 0; q < b; ++q) m->modes.push_back(q);
    } else {
        for (int k = 0; k < n_modes; ++k) {
            if (modes[k] < 0 || modes[k] >= b) {
                delete m;
                return fail(NEGF_EINVAL, "mode %d out of range", modes[k]);
            }
            m->modes.push_back(modes[k]);
        }
    }
    for (int q : m->modes) {
        std::vector<negf_c64> hd(n_rings), hu(std::max(1, n_rings - 1));
        for (int j = 0; j < n_rings; ++j) hd[j] = mode_value(h_diag + j * b2, b, q);
        for (int j = 0; j + 1 < n_rings; ++j) hu[j] = mode_value(h_up + j * b2, b, q);
        std::vector<negf_c64> lhd[2], lhu[2], lt[2];
        negf_lead sl[2];
        for (int l = 0; l < 2; ++l) {
            const negf_lead* L = ls[l];
            for (int r = 0; r < L->period; ++r) {
                lhd[l].push_back(mode_value(L->h_diag + r * b2, b, q));
                lhu[l].push_back(mode_value(L->h_up + r * b2, b, q));
            }
            lt[l].push_back(mode_value(L->tau, b, q));
            sl[l] = negf_lead{L->period, lhd[l].data(), lhu[l].data(), lt[l].data()};
        }
        negf_device* d = nullptr;
        const negf_status st =
            create_device(&d, n_rings, 1, hd.data(), n_rings > 1 ? hu.data() : nullptr, &sl[0], &sl[1], opt, false);
        if (st != NEGF_OK) {
            const std::string msg = g_err;
            negf_modes_destroy(m);
            g_err = msg;
            return st;
        }
        m->devs.push_back(d);
    }
    *out = m;
    return NEGF_OK;
}

negf_status negf_modes_set_potential(negf_modes* m, const double* U_ring, double U_left, double U_right) {
    if (!m || !U_ring) return fail(NEGF_EINVAL, "NULL argument");
    for (negf_device* d : m->devs) TRY(negf_set_potential(d, U_ring, U_left, U_right));
    return NEGF_OK;
}

negf_status negf_modes_solve(negf_modes* m, negf_workspace* w, const negf_bias* bias, int n_c, const negf_c64* z_c,
                             const negf_c64* w_c, int n_r, const double* E_r, const double* w_r, double* charge,
                             double* T, double* current) {
    if (!m || !w || !bias || !charge) return fail(NEGF_EINVAL, "NULL argument");
    const int M = (int)m->devs.size(), N = m->N, b = m->b;
    std::vector<double> q_modes((size_t)M * N), T_modes((size_t)M * std::max(n_r, 1)), I_modes(M);
    std::vector<negf_job> jobs(M);
    for (int k = 0; k < M; ++k) {
        negf_job& j = jobs[k];
        j = negf_job{};
        j.dev = m->devs[k];
        j.bias = *bias;
        j.n_c = n_c;
        j.z_c = z_c;
        j.w_c = w_c;
        j.n_r = n_r;
        j.E_r = E_r;
        j.w_r = w_r;
        j.charge = q_modes.data() + (size_t)k * N;
        j.T = n_r ? T_modes.data() + (size_t)k * n_r : nullptr;
        j.current = &I_modes[k];
    }
    TRY(negf_batch_solve(w, M, jobs.data()));
    // per-atom charge: the ring's mode charges shared equally by its b atoms
    for (int r = 0; r < N; ++r) {
        double acc = 0.0;
        for (int k = 0; k < M; ++k) acc += q_modes[(size_t)k * N + r];
        for (int i = 0; i < b; ++i) charge[(size_t)r * b + i] = acc / b;
    }
    if (T)
        for (int e = 0; e < n_r; ++e) {
            double acc = 0.0;
            for (int k = 0; k < M; ++k) acc += T_modes[(size_t)k * n_r + e];
            T[e] = acc;
        }
    if (current) {
        double acc = 0.0;
        for (int k = 0; k < M; ++k) acc += I_modes[k];
        *current = acc;
    }
    return NEGF_OK;
}

}  // extern "C"
