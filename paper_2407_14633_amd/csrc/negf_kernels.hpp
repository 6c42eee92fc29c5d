// Device kernels of the energy-point Green's-function engine (gfx950).
//
// Work decomposition.  Every energy node is independent.  Inside one node the
// block recursions over the N rings are strictly sequential, so the unit of
// GPU work is a *chain*: one recursion over all rings for one energy.  A chain
// is handled by a group of B lanes (B = ring block size), lane r owning row r of
// every b x b block in its registers; a 64-lane wavefront carries 64/B chains.
// Cross-row data (pivot rows, right operands of block products) goes through
// the group's slice of LDS.  Workgroups are a single wavefront.
//
// Kernels (see the host side for launch shapes):
//   k_decimate   lead self-energies by Sancho-Rubio layer doubling, FP64
//   k_recur      left- and right-connected recursions (Algorithm 2), one chain
//                per (energy, direction); stores y~/x~ (real axis) or y/x
//                (contour) block by block
//   k_cdiag      diag G^R_nn = (a_n - x_n - y_n)^{-1} at contour nodes,
//                one item per (energy, ring)
//   k_column     lead block columns of G^R propagated with y~/x~ (Algorithm 1),
//                diag(G Gamma G^H) per ring and T_LR, one chain per (energy, lead)
//   k_coef / k_reduce / k_current   fixed-order FP64 energy sums (Eq. 4-5)
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace negf {

template <typename T> struct cx { T re, im; };

// ------------------------------------------------------------ scalar helpers
template <typename T>
__device__ __forceinline__ void crecip(T ar, T ai, T& rr, T& ri) {
    // 1/(ar + i ai) by Smith's scaling (no intermediate overflow/underflow)
    if (fabs(ar) >= fabs(ai)) {
        const T q = ai / ar, d = ar + ai * q;
        rr = T(1) / d;
        ri = -q / d;
    } else {
        const T q = ar / ai, d = ai + ar * q;
        rr = q / d;
        ri = T(-1) / d;
    }
}

template <typename T>
__device__ __forceinline__ cx<T> ld_cx(const cx<double>* p) {
    const cx<double> v = *p;
    return cx<T>{T(v.re), T(v.im)};
}

// Per-group slice of LDS used by the block toolkit.
template <typename T, int B>
struct Grp {
    int r;            // row owned by this lane
    bool act;         // lane belongs to a live chain
    cx<T>* stage;     // B*B staging matrix (row-major)
    cx<T>* prow;      // B   pivot row
    unsigned* keys;   // B   pivot keys, one per elimination step
};

// Workgroups are a single wavefront, so lanes run in lockstep and the LDS unit
// serves one wave's instructions in order: cross-lane exchange through LDS only
// needs the compiler not to move memory operations across this point.
__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_wave_barrier(); }

template <typename T>
__device__ __forceinline__ unsigned pivot_key(T re, T im, int r) {
    const float mag = (float)(fabs(re) + fabs(im));
    return (__float_as_uint(mag) & 0xFFFFFFC0u) | (unsigned)(r + 32);
}

__device__ __forceinline__ int key_row(unsigned key, int B) {
    const int p = (int)(key & 63u) - 32;
    return p < 0 ? 0 : (p >= B ? B - 1 : p);
}

// --------------------------------------------------------------- inversion
// In-place Gauss-Jordan inversion with partial pivoting of the B x B matrix
// whose row r sits in (ar, ai) of lane r.
//  * Pivot of column k: the unused row of largest |re|+|im|, by an LDS max over
//    keys packing the magnitude (float, top 26 bits) with the row (low 6 bits).
//    The key of column k+1 is published while column k's update is still
//    running (look-ahead), so the search costs no extra round trip.
//  * Rows are never exchanged: the pivot row is relabelled, and the final
//    scatter writes the un-permuted inverse to g.stage.
//  * Row scaling is deferred: a pivot row keeps its unscaled values R_p, with
//    R_pk = 1 and its scale s_p = 1/M_pk remembered.  Every later elimination
//    step is linear in the row, so all rows use the same update
//        R_ij -= (R_ik / P_k) P_j   (j != k),   R_ik = -R_ik / P_k,
//    where P is the unscaled pivot row; the scale is applied once at the end.
template <typename T, int B>
__device__ __forceinline__ void gj_inverse(T (&ar)[B], T (&ai)[B], const Grp<T, B>& g) {
    if (g.act) g.keys[g.r] = 0u;
    wave_sync();
    bool used = !g.act;
    int my_k = 0;
    T sr = T(1), si = T(0);   // deferred row scale
    if (!used) atomicMax(&g.keys[0], pivot_key(ar[0], ai[0], g.r));
    wave_sync();
#pragma unroll
    for (int k = 0; k < B; ++k) {
        const int p = key_row(g.keys[k], B);
        const bool piv = g.act && (g.r == p);
        if (piv) {
#pragma unroll
            for (int j = 0; j < B; ++j) g.prow[j] = cx<T>{ar[j], ai[j]};
        }
        wave_sync();
        const cx<T> pk = g.prow[k];
        const T inv_d = T(1) / (pk.re * pk.re + pk.im * pk.im);
        const T qr = pk.re * inv_d, qi = -pk.im * inv_d;          // 1/P_k
        // f = R_ik / P_k for the other rows, 0 for the pivot row
        T fr = ar[k] * qr - ai[k] * qi;
        T fi = ar[k] * qi + ai[k] * qr;
        fr = piv ? T(0) : fr;
        fi = piv ? T(0) : fi;
        if (k + 1 < B) {
            const cx<T> q = g.prow[k + 1];
            ar[k + 1] = fma(-fr, q.re, fma(fi, q.im, ar[k + 1]));
            ai[k + 1] = fma(-fr, q.im, fma(-fi, q.re, ai[k + 1]));
            if (!used && !piv) atomicMax(&g.keys[k + 1], pivot_key(ar[k + 1], ai[k + 1], g.r));
        }
#pragma unroll
        for (int j = 0; j < B; ++j) {
            if (j == k || j == k + 1) continue;
            const cx<T> q = g.prow[j];
            ar[j] = fma(-fr, q.re, fma(fi, q.im, ar[j]));
            ai[j] = fma(-fr, q.im, fma(-fi, q.re, ai[j]));
        }
        ar[k] = piv ? T(1) : -fr;
        ai[k] = piv ? T(0) : -fi;
        if (piv) { sr = qr; si = qi; used = true; my_k = k; }
        wave_sync();
    }
    // apply the deferred scale, then scatter: lane with logical row my_k holds
    // column perm[j] in register j
    if (g.act) {
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const T xr = ar[j], xi = ai[j];
            ar[j] = xr * sr - xi * si;
            ai[j] = xr * si + xi * sr;
        }
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const int pj = key_row(g.keys[j], B);
            g.stage[my_k * B + pj] = cx<T>{ar[j], ai[j]};
        }
    }
    wave_sync();
}

// out = x * Y, x = this lane's row (registers), Y = B x B in LDS (broadcast reads).
template <typename T, int B>
__device__ __forceinline__ void row_mul(const T (&xr)[B], const T (&xi)[B], const cx<T>* Y,
                                        T (&orr)[B], T (&oi)[B]) {
#pragma unroll
    for (int j = 0; j < B; ++j) { orr[j] = T(0); oi[j] = T(0); }
#pragma unroll
    for (int k = 0; k < B; ++k) {
        const T a = xr[k], b = xi[k];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const cx<T> q = Y[k * B + j];
            orr[j] = fma(a, q.re, fma(-b, q.im, orr[j]));
            oi[j] = fma(a, q.im, fma(b, q.re, oi[j]));
        }
    }
}

// out = X[r,:] * Y with both operands in LDS; the k loop is not unrolled so the
// code stays small (used by the decimation's op sequence).
template <typename T, int B>
__device__ __forceinline__ void lds_row_mul(const cx<T>* X, int r, const cx<T>* Y,
                                            T (&orr)[B], T (&oi)[B]) {
#pragma unroll
    for (int j = 0; j < B; ++j) { orr[j] = T(0); oi[j] = T(0); }
#pragma unroll 1
    for (int k = 0; k < B; ++k) {
        const cx<T> x = X[r * B + k];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const cx<T> q = Y[k * B + j];
            orr[j] = fma(x.re, q.re, fma(-x.im, q.im, orr[j]));
            oi[j] = fma(x.re, q.im, fma(x.im, q.re, oi[j]));
        }
    }
}

template <typename T, int B>
struct ZeroRow { T v[B]; };
template <typename T, int B>
__device__ __forceinline__ const T (&zero_row())[B] {
    static constexpr ZeroRow<T, B> z{};
    return z.v;
}

template <typename T, int B>
__device__ __forceinline__ void stage_row(const T (&xr)[B], const T (&xi)[B], cx<T>* S, int r, bool act) {
    if (act) {
#pragma unroll
        for (int j = 0; j < B; ++j) S[r * B + j] = cx<T>{xr[j], xi[j]};
    }
}

// ------------------------------------------------------------- arguments
struct RgfArgs {
    int N, b, n_c;            // rings, ring size, number of contour energies (first n_c)
    int e0, ne;               // energies of this chunk: [e0, e0+ne)
    int K;                    // ELL width of the ring couplings
    int n_uniq;               // number of distinct coupling blocks
    int hdiag_zero;           // 1 when every H_jj is zero (potential only)
    const double* U;          // [N*b]
    const cx<double>* hdiag;  // [N][b][b]
    const int* ell_map;       // [N-1] distinct-block id of H_{n,n+1}
    const int* cidx;          // [n_uniq][b][K]  column-ELL: row index per (col j, t)
    const cx<double>* cval;   // [n_uniq][b][K]  H[cidx][j]
    const int* ridx;          // [n_uniq][b][K]  row-ELL: column index per (row j, t)
    const cx<double>* rval;   // [n_uniq][b][K]  H[j][ridx]
    const cx<double>* z;      // [n_e] energy nodes (real nodes already carry i*eta)
    const cx<double>* sigma;  // [n_e][2][b][b] lead self-energies (left, right)
    void* store_f;            // [ne][N][b][b] cx<T>: slot n = y~_n (real) / y_n (contour); slot 0 = G_{N-1,N-1}
    void* store_b;            // [ne][N][b][b] cx<T>: slot n = x~_n (real) / x_n (contour); slot N-1 = G_00
    void* gr_diag;            // [n_c][N*b] cx<T>
    void* a_diag;             // [n_r][2][N*b] T
    double* Tout;             // [n_r]
};

// a_n row r:  z delta - H_nn[r,:] - U[n b + r] delta - [n==0] Sigma_L[r,:] - [n==N-1] Sigma_R[r,:]
template <typename T, int B>
__device__ __forceinline__ void load_a_row(const RgfArgs& A, int e, int n, int r, bool act,
                                           T (&xr)[B], T (&xi)[B]) {
#pragma unroll
    for (int j = 0; j < B; ++j) { xr[j] = T(0); xi[j] = T(0); }
    if (!act) return;
    const cx<double> z = A.z[e];
    if (!A.hdiag_zero) {
        const cx<double>* h = A.hdiag + ((size_t)n * B + r) * B;
#pragma unroll
        for (int j = 0; j < B; ++j) { xr[j] = T(-h[j].re); xi[j] = T(-h[j].im); }
    }
    // the diagonal term is formed in FP64 before rounding to T
    double dre = z.re - A.U[(size_t)n * B + r];
    double dim = z.im;
#pragma unroll
    for (int j = 0; j < B; ++j) {
        if (j == r) { xr[j] += T(dre); xi[j] += T(dim); }
    }
    if (n == 0) {
        const cx<double>* s = A.sigma + ((size_t)e * 2 + 0) * B * B + (size_t)r * B;
#pragma unroll
        for (int j = 0; j < B; ++j) { xr[j] -= T(s[j].re); xi[j] -= T(s[j].im); }
    }
    if (n == A.N - 1) {
        const cx<double>* s = A.sigma + ((size_t)e * 2 + 1) * B * B + (size_t)r * B;
#pragma unroll
        for (int j = 0; j < B; ++j) { xr[j] -= T(s[j].re); xi[j] -= T(s[j].im); }
    }
}

// Writes the group's stage matrix to a store slot, coalesced: lane r writes
// elements t*B + r for t = 0..B-1.
template <typename T, int B>
__device__ __forceinline__ void stage_to_global(const cx<T>* S, cx<T>* dst, int r, bool act) {
    if (act) {
#pragma unroll
        for (int t = 0; t < B; ++t) dst[t * B + r] = S[t * B + r];
    }
}

// ================================================================ k_recur ==
// Chain = (energy, direction).  Direction 0 (forward) runs the left-connected
// recursion y_{n+1} = c_n (a_n - y_n)^{-1} b_n; direction 1 (backward) runs the
// right-connected x_{n-1} = b_{n-1} (a_n - x_n)^{-1} c_{n-1}, with
// b_n = -H_{n,n+1}, c_n = -H_{n+1,n} (Algorithm 2 in blocks of M).
// Grid: [2 * ceil(ne / G)], first half forward; a workgroup never mixes directions.

template <typename T, int B>
__global__ __launch_bounds__(64, 2) void k_recur(RgfArgs A) {
    constexpr int G = 64 / B;
    __shared__ cx<T> s_stage[G][B * B];
    __shared__ cx<T> s_prow[G][B];
    __shared__ unsigned s_keys[G][B];

    const int lane = threadIdx.x;
    const int gi = lane / B;
    const int half = gridDim.x / 2;
    const int dir = blockIdx.x >= half ? 1 : 0;
    const int wave = dir ? blockIdx.x - half : blockIdx.x;
    const int el = wave * G + gi;
    const bool act = (gi < G) && (el < A.ne);
    const int gsafe = gi < G ? gi : 0;
    Grp<T, B> g{lane - gi * B, act, s_stage[gsafe], s_prow[gsafe], s_keys[gsafe]};
    const int r = g.r;
    const int e = A.e0 + (act ? el : 0);
    const bool contour = e < A.n_c;
    const int N = A.N, K = A.K;
    cx<T>* store = reinterpret_cast<cx<T>*>(dir ? A.store_b : A.store_f) + (size_t)(act ? el : 0) * N * B * B;

    // coupling table (dynamic LDS): forward chains use the column-ELL, backward
    // chains the row-ELL of the distinct coupling blocks
    extern __shared__ unsigned char s_dyn[];
    const int n_ell = A.n_uniq * B * K;
    cx<T>* s_eval = reinterpret_cast<cx<T>*>(s_dyn);
    unsigned char* s_eidx = s_dyn + (size_t)n_ell * sizeof(cx<T>);
    {
        const int* gidx = dir ? A.ridx : A.cidx;
        const cx<double>* gval = dir ? A.rval : A.cval;
        for (int q = lane; q < n_ell; q += 64) {
            s_eidx[q] = (unsigned char)gidx[q];
            const cx<double> v = gval[q];
            s_eval[q] = cx<T>{T(v.re), T(v.im)};
        }
    }
    wave_sync();
    const cx<double> z = A.z[e];
    double u_next = act ? A.U[(size_t)(dir ? N - 1 : 0) * B + r] : 0.0;

    // the recursion state (y_n or x_n) is kept in the group's stage between steps
    stage_row<T, B>(zero_row<T, B>(), zero_row<T, B>(), g.stage, r, act);
    wave_sync();

    for (int s = 0; s < N; ++s) {
        const int n = dir ? N - 1 - s : s;
        const bool last = (s == N - 1);
        if (last && __all(!act || contour)) break;
        const double u = u_next;
        if (!last && act) u_next = A.U[(size_t)(dir ? N - 2 - s : s + 1) * B + r];
        // K = a_n - y_n, a_n = z - H_nn - U_n - [n==0] Sigma_L - [n==N-1] Sigma_R
        T kr[B], ki[B];
#pragma unroll
        for (int j = 0; j < B; ++j) { const cx<T> y = g.stage[r * B + j]; kr[j] = -y.re; ki[j] = -y.im; }
        if (act) {
            if (!A.hdiag_zero) {
                const cx<double>* h = A.hdiag + ((size_t)n * B + r) * B;
#pragma unroll
                for (int j = 0; j < B; ++j) { kr[j] -= T(h[j].re); ki[j] -= T(h[j].im); }
            }
            const T dre = T(z.re - u), dim = T(z.im);   // diagonal formed in FP64, then rounded
#pragma unroll
            for (int j = 0; j < B; ++j) {
                if (j == r) { kr[j] += dre; ki[j] += dim; }
            }
            if (n == 0 || n == N - 1) {
#pragma unroll
                for (int lr = 0; lr < 2; ++lr) {
                    if ((lr == 0 && n == 0) || (lr == 1 && n == N - 1)) {
                        const cx<double>* sg = A.sigma + ((size_t)e * 2 + lr) * B * B + (size_t)r * B;
#pragma unroll
                        for (int j = 0; j < B; ++j) { kr[j] -= T(sg[j].re); ki[j] -= T(sg[j].im); }
                    }
                }
            }
        }
        gj_inverse<T, B>(kr, ki, g);   // (a_n - y_n)^{-1} -> stage
        if (last) {
            // G_{N-1,N-1} (forward) / G_00 (backward): exact, the other side is empty
            if (!contour) stage_to_global<T, B>(g.stage, store + (size_t)(dir ? N - 1 : 0) * B * B, r, act);
            break;
        }
        const int c = dir ? N - 2 - s : s;   // coupling block index
        const int slot = dir ? N - 2 - s : s + 1;
        const int base = A.ell_map[c] * B * K;
        // P product: t[r][j] = sum_l X[r][l] P[l][j]
        //   fwd: P[l][j] = -H[l][j] (column-ELL);  bwd: P[l][j] = -conj(H[j][l]) (row-ELL)
        T tr[B], ti[B];
#pragma unroll
        for (int j = 0; j < B; ++j) { tr[j] = T(0); ti[j] = T(0); }
        if (act) {
            for (int t = 0; t < K; ++t) {
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    const int q = base + j * K + t;
                    const int l = s_eidx[q];
                    const cx<T> h = s_eval[q];
                    const T pr = -h.re, pi = dir ? h.im : -h.im;
                    const cx<T> x = g.stage[r * B + l];
                    tr[j] = fma(x.re, pr, fma(-x.im, pi, tr[j]));
                    ti[j] = fma(x.re, pi, fma(x.im, pr, ti[j]));
                }
            }
        }
        wave_sync();
        stage_row<T, B>(tr, ti, g.stage, r, act);
        wave_sync();
        if (!contour) stage_to_global<T, B>(g.stage, store + (size_t)slot * B * B, r, act);
        // Q product: y[r][:] = sum_l Q[r][l] t[l][:]
        //   fwd: Q[r][l] = -conj(H[l][r]) (column-ELL of column r);  bwd: Q[r][l] = -H[r][l] (row-ELL)
        T yr[B], yi[B];
#pragma unroll
        for (int j = 0; j < B; ++j) { yr[j] = T(0); yi[j] = T(0); }
        if (act) {
            for (int t = 0; t < K; ++t) {
                const int q = base + r * K + t;
                const int l = s_eidx[q];
                const cx<T> h = s_eval[q];
                const T qr = -h.re, qi = dir ? -h.im : h.im;
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    const cx<T> x = g.stage[l * B + j];
                    yr[j] = fma(qr, x.re, fma(-qi, x.im, yr[j]));
                    yi[j] = fma(qr, x.im, fma(qi, x.re, yi[j]));
                }
            }
        }
        wave_sync();
        stage_row<T, B>(yr, yi, g.stage, r, act);
        wave_sync();
        if (contour) stage_to_global<T, B>(g.stage, store + (size_t)slot * B * B, r, act);
    }
}

// ================================================================ k_cdiag ==
// Item = (contour energy, ring n): G_nn = (a_n - x_n - y_n)^{-1}, diagonal kept.
template <typename T, int B>
__global__ __launch_bounds__(64, 2) void k_cdiag(RgfArgs A, int nc_chunk) {
    constexpr int G = 64 / B;
    __shared__ cx<T> s_stage[G][B * B];
    __shared__ cx<T> s_prow[G][B];
    __shared__ unsigned s_keys[G][B];

    const int lane = threadIdx.x;
    const int gi = lane / B;
    const int item = blockIdx.x * G + gi;
    const int N = A.N;
    const bool act = (gi < G) && (item < nc_chunk * N);
    const int gsafe = gi < G ? gi : 0;
    Grp<T, B> g{lane - gi * B, act, s_stage[gsafe], s_prow[gsafe], s_keys[gsafe]};
    const int r = g.r;
    const int el = act ? item / N : 0;
    const int n = act ? item - el * N : 0;
    const int e = A.e0 + el;

    T kr[B], ki[B];
    load_a_row<T, B>(A, e, n, r, act, kr, ki);
    if (act) {
        const cx<T>* sf = reinterpret_cast<const cx<T>*>(A.store_f) + ((size_t)el * N + n) * B * B + (size_t)r * B;
        const cx<T>* sb = reinterpret_cast<const cx<T>*>(A.store_b) + ((size_t)el * N + n) * B * B + (size_t)r * B;
        if (n > 0) {
#pragma unroll
            for (int j = 0; j < B; ++j) { const cx<T> v = sf[j]; kr[j] -= v.re; ki[j] -= v.im; }
        }
        if (n < N - 1) {
#pragma unroll
            for (int j = 0; j < B; ++j) { const cx<T> v = sb[j]; kr[j] -= v.re; ki[j] -= v.im; }
        }
    }
    gj_inverse<T, B>(kr, ki, g);
    if (act) {
        const cx<T> d = g.stage[r * B + r];
        reinterpret_cast<cx<T>*>(A.gr_diag)[(size_t)e * N * B + (size_t)n * B + r] = d;
    }
}

// =============================================================== k_column ==
// Chain = (real energy, lead).  Right lead: W_n = G_{n,N-1}, W_{N-1} from the
// forward store, W_{n-1} = -y~_n W_n.  Left lead: W_n = G_{n,0}, W_0 from the
// backward store, W_{n+1} = -x~_n W_n (Algorithm 1, lines 3-4 and 6-8).
// Each ring's diag(W Gamma W^H) is written; the right chain ends with
// T_LR = Tr[Gamma_L W_0 Gamma_R W_0^H] (Eq. 5).
// Grid: [2 * ceil(nr_chunk / G)], first half left lead.
template <typename T, typename TS, int B>
__global__ __launch_bounds__(64, 2) void k_column(RgfArgs A, int er0, int nr_chunk) {
    constexpr int G = 64 / B;
    __shared__ cx<T> s_stage[G][B * B];
    __shared__ cx<T> s_gam[G][B * B];

    const int lane = threadIdx.x;
    const int gi = lane / B;
    const int half = gridDim.x / 2;
    const int lead = blockIdx.x >= half ? 1 : 0;
    const int wave = lead ? blockIdx.x - half : blockIdx.x;
    const int k = wave * G + gi;                 // real energy within the chunk's real part
    const bool act = (gi < G) && (k < nr_chunk);
    const int gsafe = gi < G ? gi : 0;
    const int r = lane - gi * B;
    cx<T>* S = s_stage[gsafe];
    cx<T>* Gm = s_gam[gsafe];
    const int N = A.N;
    const int e = er0 + (act ? k : 0);          // global energy index (>= n_c)
    const int el = e - A.e0;                    // index inside the chunk's store
    const int ir = e - A.n_c;                   // real-axis index

    // Gamma of this chain's lead, FP64 -> T
    if (act) {
        const cx<double>* s = A.sigma + ((size_t)e * 2 + lead) * B * B;
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const cx<double> a = s[r * B + j], b = s[j * B + r];
            // Gamma[r][j] = i (Sigma[r][j] - conj(Sigma[j][r]))
            Gm[r * B + j] = cx<T>{T(-(a.im + b.im)), T(a.re - b.re)};
        }
    }
    const cx<TS>* store = reinterpret_cast<const cx<TS>*>(lead ? A.store_f : A.store_b) + (size_t)(act ? el : 0) * N * B * B;
    T wr[B], wi[B];
#pragma unroll
    for (int j = 0; j < B; ++j) { wr[j] = T(0); wi[j] = T(0); }
    if (act) {
        const cx<TS>* w0 = store + ((size_t)(lead ? 0 : N - 1) * B + r) * B;
#pragma unroll
        for (int j = 0; j < B; ++j) { const cx<TS> v = w0[j]; wr[j] = T(v.re); wi[j] = T(v.im); }
    }
    stage_row<T, B>(wr, wi, S, r, act);
    wave_sync();
    T* aout = reinterpret_cast<T*>(A.a_diag) + ((size_t)(act ? ir : 0) * 2 + lead) * N * B;

    T vr[B], vi[B];
    for (int s = 0; s < N; ++s) {
        const int n = lead ? N - 1 - s : s;
        // propagator row for this step, loaded ahead of the Gamma product
        T pr[B], pi[B];
#pragma unroll
        for (int j = 0; j < B; ++j) { pr[j] = T(0); pi[j] = T(0); }
        if (act && s < N - 1) {
            const cx<TS>* p = store + ((size_t)n * B + r) * B;
#pragma unroll
            for (int j = 0; j < B; ++j) { const cx<TS> v = p[j]; pr[j] = -T(v.re); pi[j] = -T(v.im); }
        }
        // diag(W Gamma W^H)_rr = Re sum_j (W Gamma)[r][j] conj(W[r][j])
        row_mul<T, B>(wr, wi, Gm, vr, vi);
        if (act) {
            T acc = T(0);
#pragma unroll
            for (int j = 0; j < B; ++j) acc = fma(vr[j], wr[j], fma(vi[j], wi[j], acc));
            aout[(size_t)n * B + r] = acc;
        }
        if (s == N - 1) break;
        // W_next[r][:] = -sum_k P[r][k] W[k][:],  P = y~_n (right) or x~_n (left)
        row_mul<T, B>(pr, pi, S, wr, wi);
        wave_sync();
        stage_row<T, B>(wr, wi, S, r, act);
        wave_sync();
    }
    if (lead == 1) {
        // W = G_{0,N-1} (in S and registers), v = W Gamma_R (registers).
        // T_LR = sum_{r,j'} Gamma_L[j'][r] (W Gamma_R W^H)[r][j']
        double t = 0.0;
        if (act) {
            const cx<double>* sl = A.sigma + ((size_t)e * 2 + 0) * B * B;
            for (int jp = 0; jp < B; ++jp) {
                double mr = 0.0, mi = 0.0;   // (W Gamma_R W^H)[r][jp] = sum_j v[j] conj(W[jp][j])
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    const cx<T> w = S[jp * B + j];
                    mr += (double)vr[j] * (double)w.re + (double)vi[j] * (double)w.im;
                    mi += (double)vi[j] * (double)w.re - (double)vr[j] * (double)w.im;
                }
                const cx<double> a = sl[jp * B + r], b = sl[r * B + jp];
                const double gre = -(a.im + b.im), gim = a.re - b.re;   // Gamma_L[jp][r]
                t += gre * mr - gim * mi;
            }
        }
        // group sum in fixed order through LDS (reuse Gm: everyone is done with it)
        wave_sync();
        double* red = reinterpret_cast<double*>(Gm);
        if (act) red[r] = t;
        wave_sync();
        if (act && r == 0) {
            double sum = 0.0;
            for (int q = 0; q < B; ++q) sum += red[q];
            A.Tout[ir] = sum;
        }
    }
}

// ============================================================= k_decimate ==
// Chain = (energy, lead).  Sancho-Rubio layer doubling written on the ring
// blocks of a principal layer of `period` rings.  For a nearest-ring lead the
// doubling keeps alpha (beta) non-zero only in its (P-1,0) ((0,P-1)) block and
// changes only the corner diagonal blocks of eps, so every product is b x b:
//   P = 1:  g = (z-e)^{-1}; es += A g Bm; e += A g Bm + Bm g A; A <- A g A; Bm <- Bm g Bm
//   P = 2:  eps = [[e00, V],[V^H, e11]], eps_s(1,1) == e11, eps_s(0,0) = D0;
//           g00 = (z-e00 - V (z-e11)^{-1} V^H)^{-1},  g11 = (z-e11 - V^H (z-e00)^{-1} V)^{-1}
//           g01 = g00 V (z-e11)^{-1},  g10 = g11 V^H (z-e00)^{-1}
//           e11 += A g00 Bm;  e00 += Bm g11 A;  A <- A g01 A;  Bm <- Bm g10 Bm
// until every |A_ij|, |Bm_ij| < tol.  Then Sigma = tau g_s[0,0] tau^H.
// Chain state lives in a global scratch (each lane touches only its own rows);
// right operands are staged in three LDS matrices per group.
struct DecArgs {
    int b, n, maxit;             // n energies
    double tol;
    int lead_only;               // -1: both leads (grid = 2 halves); 0/1: that lead only
    int period[2];               // per lead: 1 or 2
    const cx<double>* z;         // [n] nodes, used as given
    const cx<double>* D[2];      // [period][b][b] lead on-site blocks incl. lead potential
    const cx<double>* V[2];      // [b][b]  h_up[0] (period 2: intra-cell coupling)
    const cx<double>* VH[2];     // [b][b]  V^H
    const cx<double>* W[2];      // [b][b]  h_up[period-1] (inter-cell coupling)
    const cx<double>* tau[2];    // [b][b]
    cx<double>* scratch;         // [2][n][6][b][b]
    cx<double>* sigma;           // [n][2][b][b]  written at [k][lead]
    int* iters;                  // [n][2]
    int* status;                 // [n]  |= 1 on non-convergence
};

template <int B>
__device__ __forceinline__ void gl_row(const cx<double>* M, int r, double (&xr)[B], double (&xi)[B]) {
#pragma unroll
    for (int j = 0; j < B; ++j) { const cx<double> v = M[r * B + j]; xr[j] = v.re; xi[j] = v.im; }
}
template <int B>
__device__ __forceinline__ void gs_row(cx<double>* M, int r, const double (&xr)[B], const double (&xi)[B]) {
#pragma unroll
    for (int j = 0; j < B; ++j) M[r * B + j] = cx<double>{xr[j], xi[j]};
}

template <int B>
__global__ __launch_bounds__(64) void k_decimate(DecArgs Dg) {
    constexpr int G = 64 / B;
    using T = double;
    __shared__ cx<T> s_buf[3][G][B * B];
    __shared__ cx<T> s_prow[G][B];
    __shared__ unsigned s_keys[G][B];
    __shared__ int s_flag[G];

    const int lane = threadIdx.x;
    const int gi = lane / B;
    const int half = gridDim.x / 2;
    const int lead = Dg.lead_only >= 0 ? Dg.lead_only : (blockIdx.x >= half ? 1 : 0);
    const int wave = (Dg.lead_only < 0 && lead == 1) ? blockIdx.x - half : blockIdx.x;
    const int k = wave * G + gi;
    const bool act = (gi < G) && (k < Dg.n);
    struct {
        int period, maxit, lead;
        double tol;
        const cx<double> *D, *V, *VH, *W, *tau;
    } D{Dg.period[lead], Dg.maxit, lead, Dg.tol, Dg.D[lead], Dg.V[lead], Dg.VH[lead], Dg.W[lead], Dg.tau[lead]};
    const int gsafe = gi < G ? gi : 0;
    const int r = lane - gi * B;
    cx<T>* L0 = s_buf[0][gsafe];
    cx<T>* L1 = s_buf[1][gsafe];
    cx<T>* L2 = s_buf[2][gsafe];
    const int kk = act ? k : 0;
    const cx<double> z = Dg.z[kk];
    cx<double>* sc = Dg.scratch + ((size_t)lead * Dg.n + kk) * 6 * B * B;
    cx<double>* E0 = sc;               // e00 (P=2) or e (P=1)
    cx<double>* E1 = sc + 1 * B * B;   // e11 == eps_s(1,1) (P=2) or eps_s (P=1)
    cx<double>* MA = sc + 2 * B * B;   // alpha corner block
    cx<double>* MB = sc + 3 * B * B;   // beta corner block
    cx<double>* X1 = sc + 4 * B * B;   // g01
    cx<double>* X2 = sc + 5 * B * B;   // g10

    bool live = act;   // chain still iterating
    T xr[B], xi[B], ur[B], ui[B], dr[B], di[B], nr[B], ni[B];
    if (act) {
        gl_row<B>(D.D, r, xr, xi);
        gs_row<B>(E0, r, xr, xi);
        if (D.period == 2) gl_row<B>(D.D + B * B, r, xr, xi);
        gs_row<B>(E1, r, xr, xi);
        gl_row<B>(D.W, r, xr, xi);
        gs_row<B>(MA, r, xr, xi);
#pragma unroll
        for (int j = 0; j < B; ++j) { const cx<double> v = D.W[j * B + r]; xr[j] = v.re; xi[j] = -v.im; }
        gs_row<B>(MB, r, xr, xi);
    }

    // dst <- (z I - M[r,:] - [sub_u] u)^{-1} for the live chains
    auto inv_from = [&](const cx<double>* M, bool sub_u, cx<T>* dst) {
        T kr[B], ki[B];
#pragma unroll
        for (int j = 0; j < B; ++j) { kr[j] = T(0); ki[j] = T(0); }
        if (live) {
            gl_row<B>(M, r, kr, ki);
#pragma unroll
            for (int j = 0; j < B; ++j) {
                kr[j] = -kr[j] - (sub_u ? ur[j] : T(0));
                ki[j] = -ki[j] - (sub_u ? ui[j] : T(0));
                if (j == r) { kr[j] += z.re; ki[j] += z.im; }
            }
        }
        Grp<T, B> gg{r, live, dst, s_prow[gsafe], s_keys[gsafe]};
        gj_inverse<T, B>(kr, ki, gg);
    };
    auto stage_global = [&](const cx<double>* M, cx<T>* dst) {
        if (live) { T a[B], b[B]; gl_row<B>(M, r, a, b); stage_row<T, B>(a, b, dst, r, true); }
    };
    // u <- u * M where M (global, uniform across lanes of the wave) is B x B
    auto mul_uniform = [&](const cx<double>* M) {
        if (live) {
#pragma unroll
            for (int j = 0; j < B; ++j) { dr[j] = T(0); di[j] = T(0); }
#pragma unroll
            for (int q = 0; q < B; ++q) {
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    const cx<double> h = M[q * B + j];
                    dr[j] += ur[q] * h.re - ui[q] * h.im;
                    di[j] += ur[q] * h.im + ui[q] * h.re;
                }
            }
#pragma unroll
            for (int j = 0; j < B; ++j) { ur[j] = dr[j]; ui[j] = di[j]; }
        }
    };
    auto add_global = [&](cx<double>* M, const T (&ar)[B], const T (&ai)[B]) {
        if (live) {
            T er[B], ei[B];
            gl_row<B>(M, r, er, ei);
#pragma unroll
            for (int j = 0; j < B; ++j) { er[j] += ar[j]; ei[j] += ai[j]; }
            gs_row<B>(M, r, er, ei);
        }
    };

    int it_done = D.maxit;
    for (int it = 1; it <= D.maxit; ++it) {
        if (D.period == 1) {
            inv_from(E0, false, L0);                      // L0 = g
            stage_global(MB, L1);
            stage_global(MA, L2);
            wave_sync();
            if (live) gl_row<B>(MA, r, xr, xi);
            row_mul<T, B>(xr, xi, L0, ur, ui);            // A g
            row_mul<T, B>(ur, ui, L1, dr, di);            // A g Bm
            row_mul<T, B>(ur, ui, L2, nr, ni);            // A g A
            add_global(E1, dr, di);                       // eps_s += A g Bm
            if (live) { gs_row<B>(MA, r, nr, ni); gl_row<B>(MB, r, xr, xi); }
            row_mul<T, B>(xr, xi, L0, ur, ui);            // Bm g
            row_mul<T, B>(ur, ui, L2, nr, ni);            // Bm g A
#pragma unroll
            for (int j = 0; j < B; ++j) { nr[j] += dr[j]; ni[j] += di[j]; }
            add_global(E0, nr, ni);                       // eps += A g Bm + Bm g A
            row_mul<T, B>(ur, ui, L1, nr, ni);            // Bm g Bm
            if (live) gs_row<B>(MB, r, nr, ni);
            wave_sync();
        } else {
            inv_from(E1, false, L0);                      // L0 = (z - e11)^{-1}
            if (live) gl_row<B>(D.V, r, xr, xi);
            row_mul<T, B>(xr, xi, L0, ur, ui);            // R1 = V (z - e11)^{-1}
            stage_row<T, B>(ur, ui, L1, r, live);         // L1 = R1
            mul_uniform(D.VH);                            // u = R1 V^H
            wave_sync();
            inv_from(E0, true, L2);                       // L2 = g00
            lds_row_mul<T, B>(L2, r, L1, dr, di);         // g01 = g00 R1
            if (live) gs_row<B>(X1, r, dr, di);
            wave_sync();
            inv_from(E0, false, L0);                      // L0 = (z - e00)^{-1}
            if (live) gl_row<B>(D.VH, r, xr, xi);
            row_mul<T, B>(xr, xi, L0, ur, ui);            // Q = V^H (z - e00)^{-1}
            wave_sync();
            stage_row<T, B>(ur, ui, L1, r, live);         // L1 = Q
            mul_uniform(D.V);                             // u = Q V
            wave_sync();
            inv_from(E1, true, L0);                       // L0 = g11
            lds_row_mul<T, B>(L0, r, L1, dr, di);         // g10 = g11 Q
            if (live) gs_row<B>(X2, r, dr, di);
            wave_sync();
            stage_global(MB, L1);                         // L1 = Bm
            wave_sync();
            if (live) gl_row<B>(MA, r, xr, xi);
            row_mul<T, B>(xr, xi, L2, ur, ui);            // A g00
            row_mul<T, B>(ur, ui, L1, dr, di);            // A g00 Bm
            add_global(E1, dr, di);
            wave_sync();
            stage_global(MA, L2);                         // L2 = A
            wave_sync();
            if (live) gl_row<B>(MB, r, xr, xi);
            row_mul<T, B>(xr, xi, L0, ur, ui);            // Bm g11
            row_mul<T, B>(ur, ui, L2, dr, di);            // Bm g11 A
            add_global(E0, dr, di);
            wave_sync();
            stage_global(X1, L0);                         // L0 = g01
            wave_sync();
            if (live) gl_row<B>(MA, r, xr, xi);
            row_mul<T, B>(xr, xi, L0, ur, ui);            // A g01
            row_mul<T, B>(ur, ui, L2, dr, di);            // A g01 A
            if (live) gs_row<B>(MA, r, dr, di);
            wave_sync();
            stage_global(X2, L0);                         // L0 = g10
            wave_sync();
            if (live) gl_row<B>(MB, r, xr, xi);
            row_mul<T, B>(xr, xi, L0, ur, ui);            // Bm g10
            row_mul<T, B>(ur, ui, L1, dr, di);            // Bm g10 Bm
            if (live) gs_row<B>(MB, r, dr, di);
            wave_sync();
        }
        // convergence of the live chains: every |A_ij|, |Bm_ij| < tol
        if (live && r == 0) s_flag[gi] = 0;
        wave_sync();
        if (live) {
            bool big = false;
            gl_row<B>(MA, r, xr, xi);
#pragma unroll
            for (int j = 0; j < B; ++j) big |= !(hypot(xr[j], xi[j]) < D.tol);
            gl_row<B>(MB, r, xr, xi);
#pragma unroll
            for (int j = 0; j < B; ++j) big |= !(hypot(xr[j], xi[j]) < D.tol);
            if (big) s_flag[gi] = 1;
        }
        wave_sync();
        if (live && s_flag[gi] == 0) { live = false; it_done = it; }
        wave_sync();
        if (__all(!live)) break;
    }
    const bool converged = act && !live;

    // surface block: P=1: g_s = (z - eps_s)^{-1};  P=2: g_s00 = (z - D0 - V (z - e11)^{-1} V^H)^{-1}
    live = act;
    if (D.period == 1) {
        inv_from(E1, false, L0);
    } else {
        inv_from(E1, false, L0);
        if (live) gl_row<B>(D.V, r, xr, xi);
        row_mul<T, B>(xr, xi, L0, ur, ui);
        mul_uniform(D.VH);
        wave_sync();
        inv_from(D.D, true, L0);
    }
    // Sigma = tau g tau^H
    if (live) gl_row<B>(D.tau, r, xr, xi);
    row_mul<T, B>(xr, xi, L0, ur, ui);
    if (live) {
#pragma unroll
        for (int j = 0; j < B; ++j) { dr[j] = T(0); di[j] = T(0); }
#pragma unroll
        for (int q = 0; q < B; ++q) {
#pragma unroll
            for (int j = 0; j < B; ++j) {
                const cx<double> h = D.tau[j * B + q];       // tau^H[q][j] = conj(tau[j][q])
                dr[j] += ur[q] * h.re + ui[q] * h.im;
                di[j] += ui[q] * h.re - ur[q] * h.im;
            }
        }
        gs_row<B>(Dg.sigma + ((size_t)k * 2 + lead) * B * B, r, dr, di);
        if (r == 0) {
            Dg.iters[(size_t)k * 2 + lead] = it_done;
            if (!converged) atomicOr(&Dg.status[k], 1);
        }
    }
}

}  // namespace negf
