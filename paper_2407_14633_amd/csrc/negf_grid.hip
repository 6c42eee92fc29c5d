// Semi-adaptive real-axis grid (Section 3.3, on the number of integration points):
// the window [E_min, E_max] of Eq. 4 is split at E_l1 < E_l2 into three parts,
// each integrated by Gauss-Legendre with its own density of nodes per kT; the
// integrand f_L A_L + f_R A_R at the centre of the channel (ring N/2, atoms
// summed) is evaluated on the grid of the guessed limits, its peak E_s located,
// and the limits refined as E_l1 <- E_l1 - a kT, E_l2 <- E_s + b kT before the
// grid is rebuilt.  The probe runs as an ordinary real-axis solve on the GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "negf_internal.hpp"

using namespace negf_host;

namespace {

// Gauss-Legendre nodes (ascending) and weights on [-1, 1] by Newton's method on P_n
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(pi * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;   // P_0, P_1
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            const double pn = n == 0 ? 1.0 : (n == 1 ? z : p1);
            const double pm = n == 1 ? 1.0 : p0;   // P_{n-1}
            dp = n * (z * pn - pm) / (z * z - 1.0);
            const double dz = pn / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        // recompute the derivative at the converged root
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * (n == 1 ? z : p1) - (n == 1 ? 1.0 : p0)) / (z * z - 1.0);
        const double wi = 2.0 / ((1.0 - z * z) * dp * dp);
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = wi;
        w[n - 1 - i] = wi;
    }
    if (n % 2 == 1) x[n / 2] = 0.0;
}

double clip(double v, double lo, double hi) { return std::min(std::max(v, lo), hi); }

}  // namespace

namespace negf_host {

void grid_parts(double E_min, double E_max, double l1, double l2, const double* dens, double kT,
                std::vector<double>& E, std::vector<double>& W) {
    E.clear();
    W.clear();
    const double lo[3] = {E_min, l1, l2}, hi[3] = {l1, l2, E_max};
    std::vector<double> x, w;
    for (int p = 0; p < 3; ++p) {
        if (!(hi[p] > lo[p])) continue;
        const int n = std::max(1, (int)std::ceil(dens[p] * (hi[p] - lo[p]) / kT - 1e-9));
        gauss_legendre(n, x, w);
        for (int k = 0; k < n; ++k) {
            E.push_back(0.5 * (hi[p] + lo[p]) + 0.5 * (hi[p] - lo[p]) * x[k]);
            W.push_back(0.5 * (hi[p] - lo[p]) * w[k]);
        }
    }
}

double host_fermi(double E, double mu, double kT) {
    const double x = (E - mu) / kT;
    if (x > 0) {
        const double e = std::exp(-x);
        return e / (1.0 + e);
    }
    return 1.0 / (1.0 + std::exp(x));
}

void grid_window(const negf_bias& bias, double* E_min, double* E_max, double* kT) {
    const double tail = 14.0;
    *kT = std::min(bias.kT_L, bias.kT_R);
    *E_min = std::min(bias.mu_L, bias.mu_R) - tail * std::min(bias.kT_L, bias.kT_R);
    *E_max = std::max(bias.mu_L, bias.mu_R) + tail * std::max(bias.kT_L, bias.kT_R);
}

void grid_refine(const negf_bias& bias, const std::vector<double>& Ep, const std::vector<double>& integrand,
                 double l1, double a, double b, double* n1, double* n2, double* Es) {
    double E_min, E_max, kT;
    grid_window(bias, &E_min, &E_max, &kT);
    int best = 0;
    double fbest = -1.0;
    for (size_t k = 0; k < Ep.size(); ++k)
        if (integrand[k] > fbest) {
            fbest = integrand[k];
            best = (int)k;
        }
    *Es = Ep.empty() ? E_min : Ep[best];
    *n1 = clip(clip(l1, E_min, E_max) - a * kT, E_min, E_max);
    *n2 = clip(*Es + b * kT, *n1, E_max);
}

}  // namespace negf_host

extern "C" negf_status negf_semi_adaptive_grid(negf_device* d, const negf_bias* bias, double E_l1, double E_l2,
                                               double a, double b, const double* density, double* E_r, double* w_r,
                                               int cap, int* n_r, double* limits) {
    if (!d || !bias || !density || !n_r) return fail(NEGF_EINVAL, "NULL argument");
    if (!(bias->kT_L > 0) || !(bias->kT_R > 0)) return fail(NEGF_EINVAL, "kT must be > 0");
    for (int p = 0; p < 3; ++p)
        if (!(density[p] > 0) || density[p] > 1e6) return fail(NEGF_EINVAL, "density[%d] out of range", p);
    if (!std::isfinite(E_l1) || !std::isfinite(E_l2) || !std::isfinite(a) || !std::isfinite(b))
        return fail(NEGF_EINVAL, "limits not finite");
    double E_min, E_max, kT;
    grid_window(*bias, &E_min, &E_max, &kT);
    const double l1 = clip(E_l1, E_min, E_max), l2 = clip(E_l2, E_min, E_max);
    std::vector<double> Ep, Wp;
    grid_parts(E_min, E_max, l1, l2, density, kT, Ep, Wp);
    const int np = (int)Ep.size();
    if (np > (1 << 22)) return fail(NEGF_EINVAL, "probe grid of %d nodes", np);
    // probe: A_L, A_R on the grid of the guessed limits
    const int N = d->N, B = d->b;
    std::vector<double> AL((size_t)np * N * B), AR((size_t)np * N * B), charge((size_t)N * B);
    negf_outputs o{};
    o.charge = charge.data();
    o.al_diag = AL.data();
    o.ar_diag = AR.data();
    TRY(negf_solve_ex(d, bias, 0, nullptr, nullptr, np, Ep.data(), Wp.data(), &o));
    const int jc = N / 2;
    std::vector<double> g(np);
    for (int k = 0; k < np; ++k) {
        const double fl = host_fermi(Ep[k], bias->mu_L, bias->kT_L), fr = host_fermi(Ep[k], bias->mu_R, bias->kT_R);
        double acc = 0.0;
        for (int i = 0; i < B; ++i) {
            const size_t q = (size_t)k * N * B + (size_t)jc * B + i;
            acc += fl * AL[q] + fr * AR[q];
        }
        g[k] = acc;
    }
    double n1, n2, Es;
    grid_refine(*bias, Ep, g, l1, a, b, &n1, &n2, &Es);
    std::vector<double> Ef, Wf;
    grid_parts(E_min, E_max, n1, n2, density, kT, Ef, Wf);
    *n_r = (int)Ef.size();
    if (limits) {
        limits[0] = n1;
        limits[1] = n2;
        limits[2] = Es;
    }
    if (!E_r || !w_r || (int)Ef.size() > cap)
        return fail(NEGF_EINVAL, "grid needs %d nodes, capacity %d", (int)Ef.size(), cap);
    std::copy(Ef.begin(), Ef.end(), E_r);
    std::copy(Wf.begin(), Wf.end(), w_r);
    return NEGF_OK;
}
