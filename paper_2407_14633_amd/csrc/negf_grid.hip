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
#include <map>
#include <mutex>
#include <vector>

#include "negf_internal.hpp"

using namespace negf_host;

namespace {

// Gauss-Legendre nodes (ascending) and weights on [-1, 1] by Newton's method on P_n,
// all roots at once (the three-term recurrence runs over k outside and over the
// roots inside, with its coefficients (2k-1)/k and (k-1)/k tabulated).  Newton
// converges quadratically from the asymptotic first guess: once a root's step is
// below 1e-10, one more step reaches rounding level and that root stops.
void gauss_legendre_newton(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    if (n < 1) return;
    const double pi = 3.14159265358979323846;
    const int m = (n + 1) / 2;
    std::vector<double> z(m), p0(m), p1(m), ak(n + 1, 0.0), ck(n + 1, 0.0);
    std::vector<char> live(m, 1), polish(m, 0);
    for (int k = 2; k <= n; ++k) {
        ak[k] = (2.0 * k - 1.0) / k;
        ck[k] = (k - 1.0) / k;
    }
    for (int i = 0; i < m; ++i) z[i] = std::cos(pi * (i + 0.75) / (n + 0.5));
    auto legendre = [&]() {   // p1 = P_n(z), p0 = P_{n-1}(z) at every root
        for (int i = 0; i < m; ++i) {
            p0[i] = 1.0;
            p1[i] = z[i];
        }
        for (int k = 2; k <= n; ++k) {
            const double a = ak[k], c = ck[k];
            for (int i = 0; i < m; ++i) {
                const double p2 = a * z[i] * p1[i] - c * p0[i];
                p0[i] = p1[i];
                p1[i] = p2;
            }
        }
    };
    for (int it = 0; it < 100; ++it) {
        legendre();
        int n_live = 0;
        for (int i = 0; i < m; ++i) {
            if (!live[i]) continue;
            const double dp = n * (z[i] * p1[i] - p0[i]) / (z[i] * z[i] - 1.0);
            const double dz = p1[i] / dp;
            z[i] -= dz;
            if (std::fabs(dz) < 1e-16 || polish[i])
                live[i] = 0;
            else
                polish[i] = std::fabs(dz) < 1e-10;
            n_live += live[i];
        }
        if (!n_live) break;
    }
    legendre();   // the derivative at the converged roots
    for (int i = 0; i < m; ++i) {
        const double dp = n * (z[i] * p1[i] - p0[i]) / (z[i] * z[i] - 1.0);
        const double wi = 2.0 / ((1.0 - z[i] * z[i]) * dp * dp);
        x[i] = -z[i];
        x[n - 1 - i] = z[i];
        w[i] = wi;
        w[n - 1 - i] = wi;
    }
    if (n % 2 == 1) x[n / 2] = 0.0;
}

// Rules already built, by order (each costs O(n^2)); at most 64 MiB are kept.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    static std::mutex mu;
    static std::map<int, std::pair<std::vector<double>, std::vector<double>>> cache;
    static size_t cached = 0;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(n);
        if (it != cache.end()) {
            x = it->second.first;
            w = it->second.second;
            return;
        }
    }
    gauss_legendre_newton(n, x, w);
    std::lock_guard<std::mutex> lk(mu);
    if (cached + (size_t)n * 16 > ((size_t)64 << 20)) {
        cache.clear();
        cached = 0;
    }
    cache[n] = {x, w};
    cached += (size_t)n * 16;
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
