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
// Batching.  A *job* is one device with its energy nodes (JobDesc).  A *unit*
// is up to G consecutive nodes of one job handled by one wavefront, plus a
// side (recursion direction or lead).  Kernels are persistent: each workgroup
// pulls units from an atomic counter until the list is exhausted, so one
// launch covers every job of a ring size, longest chains first.  A chain's
// arithmetic never depends on which other chains share its wavefront, so a
// job's results are bit-identical alone and in a batch.
//
// Kernels (see the host side for launch shapes):
//   k_decimate_circ  lead self-energies of ring-circulant leads: Sancho-Rubio
//                layer doubling per ring Fourier mode (scalar chains), FP64
//   k_decimate   lead self-energies by dense Sancho-Rubio layer doubling, FP64,
//   k_decimate2  one-ring (k_decimate) and two-ring (k_decimate2) principal layers
//   k_recur      left- and right-connected recursions (Algorithm 2), one chain
//                per (node, direction); stores y~/x~ (real axis) or y/x
//                (contour) block by block
//   k_cdiag      diag G^R_nn = (a_n - x_n - y_n)^{-1} at contour nodes,
//                one item per (node, ring)
//   k_column     lead block columns of G^R propagated with y~/x~ (Algorithm 1),
//                diag(G Gamma G^H) per ring and T_LR, one chain per (node, lead)
//   k_coef / k_reduce_* / k_current   fixed-order FP64 energy sums (Eq. 4-5)
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Resident waves per SIMD the recursion kernels are compiled for (register budget).
#ifndef NEGF_RGF_WAVES
#define NEGF_RGF_WAVES 2
#endif

namespace negf {

// aligned to its full size so that one element moves with one 128-bit (FP64)
// or 64-bit (FP32) LDS or global access
template <typename T> struct alignas(2 * sizeof(T)) cx { T re, im; };

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

// Loads and stores through the global address space: global (not flat)
// instructions, which count only against the vector-memory counter, so waits on
// LDS results never also wait for HBM traffic.
template <typename T>
__device__ __forceinline__ cx<T> gload(const cx<T>* p) {
    const __attribute__((address_space(1))) cx<T>* g = (const __attribute__((address_space(1))) cx<T>*)(p);
    return cx<T>{g->re, g->im};
}
template <typename T>
__device__ __forceinline__ T gload_s(const T* p) {
    return *(const __attribute__((address_space(1))) T*)(p);
}
template <typename T>
__device__ __forceinline__ void gstore(cx<T>* p, cx<T> v) {
    __attribute__((address_space(1))) cx<T>* g = (__attribute__((address_space(1))) cx<T>*)(p);
    g->re = v.re;
    g->im = v.im;
}
template <typename T>
__device__ __forceinline__ void gstore_s(T* p, T v) {
    *(__attribute__((address_space(1))) T*)(p) = v;
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
    return (__float_as_uint(mag) & 0xFFFFFF80u) | (unsigned)(r + 64);
}

__device__ __forceinline__ int key_row(unsigned key, int B) {
    const int p = (int)(key & 127u) - 64;
    return p < 0 ? 0 : (p >= B ? B - 1 : p);
}

// --------------------------------------------------------------- inversion
// Pins a value in registers at this point of the instruction stream: the
// compiler cannot compute it later or keep an earlier copy alive past it, and
// memory accesses are not moved across.
template <typename T>
__device__ __forceinline__ void pin(T& v) { asm volatile("" : "+v"(v) : : "memory"); }

// Column of update slot t at pivot step k: all columns but k, and but k+1 while
// k+1 < B (updated ahead for the look-ahead); B when the slot is unused.
template <int B>
__device__ __forceinline__ constexpr int gj_col(int t, int k) {
    return k + 1 < B ? (t < k ? t : t + 2) : t;
}

// Pivot-row entries in flight per chunk of the elimination update.
#ifndef GJ_CHUNK
#define GJ_CHUNK 8
#endif

// 1 / (re + i im) = conj / |.|^2, the form every pivot reciprocal uses.
template <typename T>
__device__ __forceinline__ void pivot_recip(T re, T im, T& qr, T& qi) {
    const T inv_d = T(1) / fma(re, re, im * im);   // explicit fma: every kernel rounds alike
    qr = re * inv_d;
    qi = -im * inv_d;
}

// In-place Gauss-Jordan inversion with partial pivoting of the B x B matrix
// whose row r sits in (ar, ai) of lane r.
//  * Pivot of column k: the unused row of largest |re|+|im|, by an LDS max over
//    keys packing the magnitude (float, top 25 bits) with the row (low 7 bits).
//    Column k+1 is updated first and its key published while column k's update
//    is still running (look-ahead); the key is read back right away, so the
//    next pivot is known before the bulk of the update is done.
//  * Every row also computes the reciprocal of its column k+1 entry during step
//    k; the row that becomes pivot publishes it in place of its pivot entry, so
//    the division is off the chain of dependent steps.
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
    T cr, ci;                 // 1 / (this row's entry in the next pivot column)
    pivot_recip(ar[0], ai[0], cr, ci);
    asm volatile("" : "+v"(cr), "+v"(ci));   // computed here, not inside the pivot branch
    if (!used) atomicMax(&g.keys[0], pivot_key(ar[0], ai[0], g.r));
    wave_sync();
    int p = key_row(g.keys[0], B);
    // fully unrolled for every block size used (up to 48 rows): the register rows may
    // only be indexed by compile-time constants
#pragma clang loop unroll(full)
    for (int k = 0; k < B; ++k) {
        const bool piv = g.act && (g.r == p);
        if (piv) {
#pragma unroll
            for (int j = 0; j < B; ++j) g.prow[j] = j == k ? cx<T>{cr, ci} : cx<T>{ar[j], ai[j]};
        }
        wave_sync();
        const cx<T> q = g.prow[k];                                 // 1 / P_k
        const cx<T> q1 = g.prow[k + 1 < B ? k + 1 : k];
        // f = R_ik / P_k for the other rows, 0 for the pivot row
        T fr = fma(ar[k], q.re, -(ai[k] * q.im));
        T fi = fma(ar[k], q.im, ai[k] * q.re);
        fr = piv ? T(0) : fr;
        fi = piv ? T(0) : fi;
        // pivot bookkeeping without a branch (a branch would wait for q alone)
        sr = piv ? q.re : sr;
        si = piv ? q.im : si;
        used = used || piv;
        my_k = piv ? k : my_k;
        unsigned key_next = 0u;
        if (k + 1 < B) {
            ar[k + 1] = fma(-fr, q1.re, fma(fi, q1.im, ar[k + 1]));
            ai[k + 1] = fma(-fr, q1.im, fma(-fi, q1.re, ai[k + 1]));
            if (!used) atomicMax(&g.keys[k + 1], pivot_key(ar[k + 1], ai[k + 1], g.r));
            wave_sync();
            key_next = g.keys[k + 1];
            pivot_recip(ar[k + 1], ai[k + 1], cr, ci);
            asm volatile("" : "+v"(cr), "+v"(ci));
        }
        // The remaining columns, their pivot-row entries read GJ_CHUNK at a time one
        // chunk ahead of the arithmetic; the next key is read before them and
        // decoded only after the first chunk is out, so LDS latency overlaps FMAs.
        // slot t < B - 1 stands for column gj_col(t, k): every column but k (and but
        // k+1 while k+1 < B, whose update was done above); gj_col = B marks no column
        constexpr int NJ = B - 1 > 0 ? B - 1 : 0;
        constexpr int CW = B >= 20 ? GJ_CHUNK / 2 : GJ_CHUNK;   // fewer in flight for wide rows
        constexpr int C = CW < NJ ? CW : (NJ > 0 ? NJ : 1);
        constexpr int NC = NJ > 0 ? (NJ + C - 1) / C : 0;
        cx<T> qv[2][C];
#pragma unroll
        for (int q = 0; q < C; ++q)
            if (q < NJ && gj_col<B>(q, k) < B) qv[0][q] = g.prow[gj_col<B>(q, k)];
        asm volatile("" : "+v"(key_next) : : "memory");   // decoded only after the reads are out
        const int p_next = k + 1 < B ? key_row(key_next, B) : p;
#pragma clang loop unroll(full)
        for (int c = 0; c < NC; ++c) {
            if (c + 1 < NC) {
#pragma unroll
                for (int q = 0; q < C; ++q) {
                    const int t = (c + 1) * C + q;
                    if (t < NJ && gj_col<B>(t, k) < B) qv[(c + 1) & 1][q] = g.prow[gj_col<B>(t, k)];
                }
            }
#pragma unroll
            for (int q = 0; q < C; ++q)
                if (c * C + q < NJ && gj_col<B>(c * C + q, k) < B) { pin(qv[c & 1][q].re); pin(qv[c & 1][q].im); }
#pragma unroll
            for (int q = 0; q < C; ++q) {
                const int t = c * C + q;
                if (t < NJ && gj_col<B>(t, k) < B) {
                    const int j = gj_col<B>(t, k);
                    const cx<T> qj = qv[c & 1][q];
                    ar[j] = fma(-fr, qj.re, fma(fi, qj.im, ar[j]));
                    ai[j] = fma(-fr, qj.im, fma(-fi, qj.re, ai[j]));
                    pin(ar[j]);
                    pin(ai[j]);
                }
            }
        }
        ar[k] = piv ? T(1) : -fr;
        ai[k] = piv ? T(0) : -fi;
        wave_sync();
        p = p_next;
    }
    // apply the deferred scale, then scatter: lane with logical row my_k holds
    // column perm[j] in register j
    if (g.act) {
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const T xr = ar[j], xi = ai[j];
            ar[j] = fma(xr, sr, -(xi * si));
            ai[j] = fma(xr, si, xi * sr);
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

// out = x * Y like row_mul, with the LDS reads of Y issued C elements at a time
// one chunk ahead of the arithmetic on the previous chunk, so their latency
// hides behind the FMAs.  Same order of operations as row_mul.
template <typename T, int B, int C = (B >= 20 ? 4 : 8)>
__device__ __forceinline__ void row_mul_pipe(const T (&xr)[B], const T (&xi)[B], const cx<T>* Y,
                                             T (&orr)[B], T (&oi)[B]) {
    constexpr int NE = B * B, NC = (NE + C - 1) / C;
#pragma unroll
    for (int j = 0; j < B; ++j) { orr[j] = T(0); oi[j] = T(0); }
    cx<T> buf[2][C];
#pragma unroll
    for (int q = 0; q < C; ++q)
        if (q < NE) buf[0][q] = Y[q];
#pragma clang loop unroll(full)
    for (int c = 0; c < NC; ++c) {
        if (c + 1 < NC) {
#pragma unroll
            for (int q = 0; q < C; ++q)
                if ((c + 1) * C + q < NE) buf[(c + 1) & 1][q] = Y[(c + 1) * C + q];
        }
#pragma unroll
        for (int q = 0; q < C; ++q)
            if (c * C + q < NE) { pin(buf[c & 1][q].re); pin(buf[c & 1][q].im); }
#pragma unroll
        for (int q = 0; q < C; ++q) {
            const int e = c * C + q;
            if (e < NE) {
                const int k = e / B, j = e % B;
                const cx<T> y = buf[c & 1][q];
                orr[j] = fma(xr[k], y.re, fma(-xi[k], y.im, orr[j]));
                oi[j] = fma(xr[k], y.im, fma(xi[k], y.re, oi[j]));
                pin(orr[j]);
                pin(oi[j]);
            }
        }
    }
}

// Re sum_j (x Y)[j] conj(x[j]) without keeping the row x Y: element (k, j) of Y is
// taken column by column (j outer, k inner), read C elements ahead as in
// row_mul_pipe.  Same order of operations as row_mul followed by the dot product.
template <typename T, int B, int C = (B >= 20 ? 4 : 8)>
__device__ __forceinline__ T row_quad_pipe(const T (&xr)[B], const T (&xi)[B], const cx<T>* Y) {
    constexpr int NE = B * B, NC = (NE + C - 1) / C;
    T acc = T(0), vr = T(0), vi = T(0);
    cx<T> buf[2][C];
#pragma unroll
    for (int q = 0; q < C; ++q)
        if (q < NE) buf[0][q] = Y[(q % B) * B + q / B];
#pragma clang loop unroll(full)
    for (int c = 0; c < NC; ++c) {
        if (c + 1 < NC) {
#pragma unroll
            for (int q = 0; q < C; ++q) {
                const int e = (c + 1) * C + q;
                if (e < NE) buf[(c + 1) & 1][q] = Y[(e % B) * B + e / B];
            }
        }
#pragma unroll
        for (int q = 0; q < C; ++q)
            if (c * C + q < NE) { pin(buf[c & 1][q].re); pin(buf[c & 1][q].im); }
#pragma unroll
        for (int q = 0; q < C; ++q) {
            const int e = c * C + q;
            if (e < NE) {
                const int j = e / B, k = e % B;
                const cx<T> y = buf[c & 1][q];
                vr = fma(xr[k], y.re, fma(-xi[k], y.im, vr));
                vi = fma(xr[k], y.im, fma(xi[k], y.re, vi));
                if (k == B - 1) {
                    acc = fma(vr, xr[j], fma(vi, xi[j], acc));
                    vr = T(0);
                    vi = T(0);
                }
            }
        }
        pin(vr);
        pin(vi);
        pin(acc);
    }
    return acc;
}

// row_quad_pipe for a circulant Y (Y[k][j] = Y[0][(j - k) mod B]): its first row is
// read once into registers and the B*B products take no further LDS reads.
template <typename T, int B>
__device__ __forceinline__ T row_quad_circ(const T (&xr)[B], const T (&xi)[B], const cx<T>* Y) {
    T gr[B], gi[B];
#pragma unroll
    for (int d = 0; d < B; ++d) { const cx<T> y = Y[d]; gr[d] = y.re; gi[d] = y.im; }
    T acc = T(0);
#pragma unroll
    for (int j = 0; j < B; ++j) {
        T vr = T(0), vi = T(0);
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int d = (j - k + B) % B;
            vr = fma(xr[k], gr[d], fma(-xi[k], gi[d], vr));
            vi = fma(xr[k], gi[d], fma(xi[k], gr[d], vi));
        }
        acc = fma(vr, xr[j], fma(vi, xi[j], acc));
    }
    return acc;
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
// Per-node status bits: decimation did not converge; non-finite or impossible
// output (negative spectral density, T outside [0, B]); FP64 recomputation needed
// but no room left in the chunk's store; FP32 result marked for FP64 recomputation.
enum { ST_NOCONV = 1, ST_BAD = 2, ST_NOROOM = 4, ST_FP64 = 256 };

struct JobDesc {
    int N, n_c, n_r;          // rings, contour nodes (first n_c), real-axis nodes
    int K, n_uniq;            // ELL width and number of distinct coupling blocks
    int hdiag_zero;           // 1 when every H_jj is zero (potential only)
    const double* U;          // [N*b]
    const cx<double>* hdiag;  // [N][b][b]
    const int* ell_map;       // [N-1] distinct-block id of H_{n,n+1}
    const int* cidx;          // [n_uniq][b][K]  column-ELL: row index per (col j, t)
    const cx<double>* cval;   // [n_uniq][b][K]  H[cidx][j]
    const int* ridx;          // [n_uniq][b][K]  row-ELL: column index per (row j, t)
    const cx<double>* rval;   // [n_uniq][b][K]  H[j][ridx]
    const cx<double>* z;      // [n_e] nodes (real nodes carry i*eta)
    cx<double>* sigma;        // [n_e][2][b][b] lead self-energies (left, right)
    void* gr_diag;            // [n_c][N*b] cx<T>
    void* a_diag;             // [n_r][2][N*b] double
    double* Tout;             // [n_r] T_LR
    double* Trl;              // [n_r] T_RL (from the left lead column)
    double* amax;             // [n_r][2] max_i A_l,ii per real node and lead
    int* iters;               // [n_e][2] decimation steps
    int* status;              // [n_e]    ST_* bits: decimation, bad output, FP64 recompute
    int* n_fp64;              // number of nodes recomputed in FP64 (FP32-bulk form)
    double hnorm;             // max row sum of |H| over the device (couplings included)
    int fp64_policy;          // FP32-bulk: 0 recompute the marked real nodes, 1 all, 2 none
    int period[2];            // lead principal-layer sizes
    const cx<double>* D[2];   // [period][b][b] lead on-site blocks incl. lead potential
    const cx<double>* V[2];   // h_up[0]
    const cx<double>* VH[2];  // h_up[0]^H
    const cx<double>* W[2];   // h_up[period-1]
    const cx<double>* tau[2]; // H_{device edge, lead ring 0}
    // ring-circulant leads: per lead [5][b] eigenvalues of D_0, D_{P-1}, h_up[0],
    // h_up[P-1], tau on the ring Fourier vectors (lead potential included); null otherwise
    const cx<double>* lmodes[2];
    int sigma_circ;               // Sigma from the ring-mode decimation: exactly circulant
};

// A span: the nodes [e0, e0+cnt) of one job that one kernel launch covers
// (all nodes, only the contour nodes or only the real-axis nodes of a chunk).
// Its work is cut into units of G nodes (G (node, ring) items for k_cdiag),
// each unit once per side (direction or lead).  Units are numbered span by
// span: first[s] = units before span s, so unit w belongs to the span with
// first[s] <= w < first[s+1], and within it side = local % sides.
struct Span {
    int job, e0, cnt, pad;
    long long off;            // store element offset of node e0 (recursion stores)
};

struct Sched {
    const JobDesc* jobs;
    const Span* spans;
    const int* first;         // [n_spans + 1] unit prefix
    int n_spans;
    int sides;                // sides per span: 2 (both directions / leads) or 1
    int side0;                // first side (1 = backward direction / right lead alone)
    int* counter;             // zero before launch
    int gpw;                  // nodes per unit (recursions, lead columns) or (node, ring) items
                              // per unit (contour diagonals): at most the chains one
                              // wavefront holds; fewer leave groups of lanes idle
    void* store_f;            // recursion stores: slot n = y~_n (real) / y_n (contour); slot 0 = G_{N-1,N-1}
    void* store_b;            //                   slot n = x~_n (real) / x_n (contour); slot N-1 = G_00
    cx<double>* scratch;      // decimation state, per workgroup: G chains x 6 b x b blocks
    double tol;               // decimation tolerance
    int maxit;                // decimation step limit
    int lane_spans;           // 1: every span is one node and a unit takes 64 of them, one per
                              // lane (ring size 1, FP64 recomputation rounds)
};

struct Unit {
    int span, job, side, e0, cnt, i0;
    long long off;
};

// next unit for this workgroup (one atomic per wavefront, uniform result); false when done
template <int G>
__device__ __forceinline__ bool next_unit(const Sched& S, Unit& u, bool items = false) {
    int w = 0;
    if (threadIdx.x == 0) w = atomicAdd(S.counter, 1);
    w = __builtin_amdgcn_readfirstlane(w);
    if (w >= S.first[S.n_spans]) return false;
    int lo = 0, hi = S.n_spans;          // first[lo] <= w < first[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (S.first[mid] <= w) lo = mid; else hi = mid;
    }
    const Span sp = S.spans[lo];
    const int local = w - S.first[lo];
    u.span = lo;
    u.job = sp.job;
    u.side = S.side0 + local % S.sides;
    const int blk = local / S.sides;
    if (items) {                          // k_cdiag: G (node, ring) items
        u.i0 = blk * S.gpw;
        u.e0 = sp.e0;
        u.off = sp.off;
        u.cnt = 0;                        // set by the caller from N
    } else {
        u.e0 = sp.e0 + blk * S.gpw;
        u.cnt = min(S.gpw, sp.e0 + sp.cnt - u.e0);
        u.off = sp.off;
        u.i0 = blk * S.gpw;               // node offset of the unit inside the span
    }
    return true;
}

// Writes the group's stage matrix to a store slot, coalesced: lane r writes
// elements t*B + r for t = 0..B-1.
template <typename T, int B>
__device__ __forceinline__ void stage_to_global(const cx<T>* S, cx<T>* dst, int r, bool act) {
    if (act) {
        // the addresses are formed here, not hoisted ahead where they would hold
        // registers through the inversion
        cx<T>* d = dst + r;
        asm volatile("" : "+v"(d));
#pragma unroll
        for (int t = 0; t < B; ++t) gstore(d + t * B, S[t * B + r]);
    }
}

// a_n row r into (xr, xi), optionally minus m:  z - H_nn - U_n - [n==0] Sigma_L - [n==N-1] Sigma_R
// kDiag: how z - u reaches the diagonal entry.  0: a branch per entry; 1: a select on
// every entry (with a branch per entry the compiler may merge the cases into a
// pointer choice that keeps the row in scratch memory, as it does in k_cdiag for
// the larger ring sizes); 2: not at all (the caller has put it on the diagonal).
template <typename T, int B, int kDiag = 0>
__device__ __forceinline__ void add_a_row(const JobDesc& J, int e, int n, int r, double u, cx<double> z,
                                          T (&xr)[B], T (&xi)[B]) {
    if (!J.hdiag_zero) {
        const cx<double>* h = J.hdiag + ((size_t)n * B + r) * B;
#pragma unroll
        for (int j = 0; j < B; ++j) { const cx<double> hv = gload(h + j); xr[j] -= T(hv.re); xi[j] -= T(hv.im); }
    }
    const T dre = T(z.re - u), dim = T(z.im);   // diagonal formed in FP64, then rounded
    if constexpr (kDiag == 0) {
#pragma unroll
        for (int j = 0; j < B; ++j) {
            if (j == r) { xr[j] += dre; xi[j] += dim; }
        }
    } else if constexpr (kDiag == 1) {
#pragma unroll
        for (int j = 0; j < B; ++j) {
            xr[j] += j == r ? dre : T(0);
            xi[j] += j == r ? dim : T(0);
        }
    }
    if (n == 0 || n == J.N - 1) {
#pragma unroll
        for (int lr = 0; lr < 2; ++lr) {
            if ((lr == 0 && n == 0) || (lr == 1 && n == J.N - 1)) {
                const cx<double>* sg = J.sigma + ((size_t)e * 2 + lr) * B * B + (size_t)r * B;
#pragma unroll
                for (int j = 0; j < B; ++j) { const cx<double> sv = gload(sg + j); xr[j] -= T(sv.re); xi[j] -= T(sv.im); }
            }
        }
    }
}

// ======================================================= scalar (B = 1) paths ==
// a_n - state for a ring of size 1, formed in FP64: z - H_nn - U_n - Sigma (boundary
// rings) - state.
__device__ __forceinline__ cx<double> scalar_a(const JobDesc& J, int e, int n, double u, cx<double> z) {
    double re = z.re - u, im = z.im;
    if (!J.hdiag_zero) {
        const cx<double> h = gload(J.hdiag + n);
        re -= h.re;
        im -= h.im;
    }
    if (n == 0) {
        const cx<double> sv = gload(J.sigma + (size_t)e * 2 + 0);
        re -= sv.re;
        im -= sv.im;
    }
    if (n == J.N - 1) {
        const cx<double> sv = gload(J.sigma + (size_t)e * 2 + 1);
        re -= sv.re;
        im -= sv.im;
    }
    return cx<double>{re, im};
}

// a contour node of a scalar chain, whole (defined with the real-node form below)
template <typename TS>
__device__ __forceinline__ void chain_contour(const JobDesc& J, cx<TS>* ckf, int e);

// ================================================================ k_recur ==
// Chain = (node, direction).  Direction 0 (forward) runs the left-connected
// recursion y_{n+1} = c_n (a_n - y_n)^{-1} b_n; direction 1 (backward) runs the
// right-connected x_{n-1} = b_{n-1} (a_n - x_n)^{-1} c_{n-1}, with
// b_n = -H_{n,n+1}, c_n = -H_{n+1,n} (Algorithm 2 in blocks of M).
// Boundary inversion of the FP32-bulk form: the row of (a_n - state) is built and
// inverted in FP64, then rounded into the FP32 stage.  Used for the rings that
// carry a lead self-energy: near a pole of Sigma (an edge state of the lead
// surface) a_n - Sigma has entries far larger than its inverse's, and an FP32
// inversion loses the small directions entirely.
template <int B>
__device__ __forceinline__ void invert_fp64_into(const JobDesc& J, int e, int n, int r, bool act, double uu,
                                                 cx<double> z, cx<float>* stage, cx<double>* stage64,
                                                 cx<double>* prow64, unsigned* keys) {
    double kr[B], ki[B];
#pragma unroll
    for (int j = 0; j < B; ++j) {
        const cx<float> y = stage[r * B + j];
        kr[j] = -(double)y.re;
        ki[j] = -(double)y.im;
    }
    if (act) add_a_row<double, B>(J, e, n, r, uu, z, kr, ki);
    Grp<double, B> g64{r, act, stage64, prow64, keys};
    gj_inverse<double, B>(kr, ki, g64);
    if (act) {
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const cx<double> v = stage64[r * B + j];
            stage[r * B + j] = cx<float>{(float)v.re, (float)v.im};
        }
    }
    wave_sync();
}

template <typename T, int B>
__global__ __launch_bounds__(64, NEGF_RGF_WAVES) __attribute__((amdgpu_waves_per_eu(NEGF_RGF_WAVES, NEGF_RGF_WAVES))) void k_recur(Sched S) {
    constexpr int G = 64 / B;
    constexpr bool kF32 = sizeof(T) == 4;
    constexpr int G64 = kF32 ? G : 1;   // FP64 boundary buffers (FP32-bulk form only)
    __shared__ cx<T> s_stage[G][B * B];
    __shared__ cx<T> s_prow[G][B];
    __shared__ unsigned s_keys[G][B];
    __shared__ cx<double> s_stage64[G64][kF32 ? B * B : 1];
    __shared__ cx<double> s_prow64[G64][kF32 ? B : 1];
    extern __shared__ __attribute__((aligned(16))) unsigned char s_dyn[];

    const int lane = threadIdx.x;
    const int gi = lane / B;
    const int gsafe = gi < G ? gi : 0;
    const int r = lane - gi * B;

    Unit u;
    while (next_unit<G>(S, u)) {
        const JobDesc& J = S.jobs[u.job];
        const int dir = u.side;
        const bool act = (gi < G) && (gi < u.cnt);
        Grp<T, B> g{r, act, s_stage[gsafe], s_prow[gsafe], s_keys[gsafe]};
        const int e = u.e0 + (act ? gi : 0);
        const bool contour = e < J.n_c;
        const int N = J.N, K = J.K;
        cx<T>* store = reinterpret_cast<cx<T>*>(dir ? S.store_b : S.store_f) + u.off +
                       (size_t)(u.i0 + (act ? gi : 0)) * N * B * B;

        // coupling table in LDS: forward chains use the column-ELL, backward the row-ELL
        const int n_ell = J.n_uniq * B * K;
        cx<T>* s_eval = reinterpret_cast<cx<T>*>(s_dyn);
        unsigned char* s_eidx = s_dyn + (size_t)n_ell * sizeof(cx<T>);
        wave_sync();
        {
            const int* gidx = dir ? J.ridx : J.cidx;
            const cx<double>* gval = dir ? J.rval : J.cval;
            for (int q = lane; q < n_ell; q += 64) {
                s_eidx[q] = (unsigned char)gload_s(gidx + q);
                const cx<double> v = gload(gval + q);
                s_eval[q] = cx<T>{T(v.re), T(v.im)};
            }
        }
        const cx<double> z = gload(J.z + e);
        if constexpr (B == 1) {
            // scalar chains (ring size 1, e.g. one mode of a mode-space tube): this launch
            // covers the contour nodes, each whole in one lane (side 0; real nodes run in
            // the column kernel)
            if (act && dir == 0) chain_contour<T>(J, store, e);
            continue;
        }
        double u_next = act ? gload_s(J.U + (size_t)(dir ? N - 1 : 0) * B + r) : 0.0;
        // the recursion state (y_n or x_n) is kept in the group's stage between steps
        stage_row<T, B>(zero_row<T, B>(), zero_row<T, B>(), g.stage, r, act);
        wave_sync();

        for (int s = 0; s < N; ++s) {
            const int n = dir ? N - 1 - s : s;
            const bool last = (s == N - 1);
            if (last && __all(!act || contour)) break;
            const double uu = u_next;
            if (!last && act) u_next = gload_s(J.U + (size_t)(dir ? N - 2 - s : s + 1) * B + r);
            bool done64 = false;
            if constexpr (kF32) {
                if (s == 0 || last) {       // rings 0 and N-1 carry Sigma: invert in FP64
                    invert_fp64_into<B>(J, e, n, r, act, uu, z, g.stage, s_stage64[gsafe], s_prow64[gsafe],
                                        s_keys[gsafe]);
                    done64 = true;
                }
            }
            if (!done64) {
                // z - u goes onto the diagonal through the stage (this lane's own entry),
                // so the row below is loaded without a per-entry diagonal test
                if (act) {
                    const cx<T> d = g.stage[r * B + r];
                    g.stage[r * B + r] = cx<T>{d.re - T(z.re - uu), d.im - T(z.im)};
                }
                T kr[B], ki[B];
#pragma unroll
                for (int j = 0; j < B; ++j) { const cx<T> y = g.stage[r * B + j]; kr[j] = -y.re; ki[j] = -y.im; }
                if (act) add_a_row<T, B, 2>(J, e, n, r, uu, z, kr, ki);
                gj_inverse<T, B>(kr, ki, g);   // (a_n - y_n)^{-1} -> stage
            }
            if (last) {
                // G_{N-1,N-1} (forward) / G_00 (backward): exact, the other side is empty
                if (!contour) stage_to_global<T, B>(g.stage, store + (size_t)(dir ? N - 1 : 0) * B * B, r, act);
                break;
            }
            const int c = dir ? N - 2 - s : s;   // coupling block index
            const int slot = dir ? N - 2 - s : s + 1;
            const int base = gload_s(J.ell_map + c) * B * K;
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
        wave_sync();
    }
}

// ================================================================ k_cdiag ==
// Item = (contour node, ring n): G_nn = (a_n - x_n - y_n)^{-1}, diagonal kept.
template <typename T, int B>
__global__ __launch_bounds__(64, NEGF_RGF_WAVES) __attribute__((amdgpu_waves_per_eu(NEGF_RGF_WAVES, NEGF_RGF_WAVES))) void k_cdiag(Sched S) {
    constexpr int G = 64 / B;
    constexpr bool kF32 = sizeof(T) == 4;
    constexpr int G64 = kF32 ? G : 1;
    __shared__ cx<T> s_stage[G][B * B];
    __shared__ cx<T> s_prow[G][B];
    __shared__ unsigned s_keys[G][B];
    __shared__ cx<double> s_stage64[G64][kF32 ? B * B : 1];
    __shared__ cx<double> s_prow64[G64][kF32 ? B : 1];

    const int lane = threadIdx.x;
    const int gi = lane / B;
    const int gsafe = gi < G ? gi : 0;
    const int r = lane - gi * B;

    Unit u;
    while (next_unit<G>(S, u, true)) {
        const JobDesc& J = S.jobs[u.job];
        const int N = J.N;
        const int n_items = S.spans[u.span].cnt * N;
        const bool live = (gi < S.gpw) && (u.i0 + gi < n_items);
        const int item = u.i0 + (live ? gi : 0);
        const int el = item / N;                 // node inside the span
        const int e = u.e0 + el;                 // node inside the job
        const int n = item - el * N;
        const size_t o_row = u.off + ((size_t)el * N + n) * B * B + (size_t)r * B;
        // FP32-bulk: the rings that carry a lead self-energy are inverted in FP64
        const bool bnd = kF32 && (n == 0 || n == N - 1);
        if constexpr (kF32) {
            const bool act64 = live && bnd;
            if (__any(act64)) {
                double kr[B], ki[B];
#pragma unroll
                for (int j = 0; j < B; ++j) { kr[j] = 0.0; ki[j] = 0.0; }
                if (act64) {
                    const cx<T>* sf = reinterpret_cast<const cx<T>*>(S.store_f) + o_row;
                    const cx<T>* sb = reinterpret_cast<const cx<T>*>(S.store_b) + o_row;
                    if (n > 0) {
#pragma unroll
                        for (int j = 0; j < B; ++j) { const cx<T> v = gload(sf + j); kr[j] -= v.re; ki[j] -= v.im; }
                    }
                    if (n < N - 1) {
#pragma unroll
                        for (int j = 0; j < B; ++j) { const cx<T> v = gload(sb + j); kr[j] -= v.re; ki[j] -= v.im; }
                    }
                    add_a_row<double, B, 1>(J, e, n, r, gload_s(J.U + (size_t)n * B + r), gload(J.z + e), kr, ki);
                }
                Grp<double, B> g64{r, act64, s_stage64[gsafe], s_prow64[gsafe], s_keys[gsafe]};
                gj_inverse<double, B>(kr, ki, g64);
                if (act64) {
                    const cx<double> d = s_stage64[gsafe][r * B + r];
                    gstore(reinterpret_cast<cx<T>*>(J.gr_diag) + (size_t)e * N * B + (size_t)n * B + r,
                           cx<T>{(T)d.re, (T)d.im});
                }
                wave_sync();
            }
        }
        const bool act = live && !bnd;
        Grp<T, B> g{r, act, s_stage[gsafe], s_prow[gsafe], s_keys[gsafe]};

        T kr[B], ki[B];
#pragma unroll
        for (int j = 0; j < B; ++j) { kr[j] = T(0); ki[j] = T(0); }
        if (act) {
            const cx<T>* sf = reinterpret_cast<const cx<T>*>(S.store_f) + o_row;
            const cx<T>* sb = reinterpret_cast<const cx<T>*>(S.store_b) + o_row;
            if (n > 0) {
#pragma unroll
                for (int j = 0; j < B; ++j) { const cx<T> v = gload(sf + j); kr[j] -= v.re; ki[j] -= v.im; }
            }
            if (n < N - 1) {
#pragma unroll
                for (int j = 0; j < B; ++j) { const cx<T> v = gload(sb + j); kr[j] -= v.re; ki[j] -= v.im; }
            }
            add_a_row<T, B, 1>(J, e, n, r, gload_s(J.U + (size_t)n * B + r), gload(J.z + e), kr, ki);
        }
        gj_inverse<T, B>(kr, ki, g);
        if (act) {
            const cx<T> d = g.stage[r * B + r];
            gstore(reinterpret_cast<cx<T>*>(J.gr_diag) + (size_t)e * N * B + (size_t)n * B + r, d);
        }
        wave_sync();
    }
}

// =============================================================== k_column ==
// Chain = (real node, lead).  Right lead: W_n = G_{n,N-1}, W_{N-1} from the
// forward store, W_{n-1} = -y~_n W_n.  Left lead: W_n = G_{n,0}, W_0 from the
// backward store, W_{n+1} = -x~_n W_n (the off-diagonal column recursions of Algorithm 1).
// Each ring's diag(W Gamma W^H) is written; the right chain ends with
// T_LR = Tr[Gamma_L W_0 Gamma_R W_0^H] (Eq. 5).
//
// The propagation runs in FP64 whatever the store precision TS: the product
// chain W_{n+1} = -x~_n W_n is unstable in FP32 where W's columns span many
// orders of magnitude (real nodes next to a pole of a lead's surface Green's
// function), even when the recursion stores are exact.
//
// Output checks at the end of every chain: the spectral densities diag(W Gamma W^H)
// must not be negative (Gamma is positive semidefinite) and T_LR must lie in
// [0, B] (at most B channels through a B-atom ring).  With FP64 stores a
// violation sets status bit 2 of the node (an error); with FP32 stores it, or a
// large lead column (max |W_ij| (|z| + ||H||) > NEGF_FP32_WMAX: the whole-device
// Green's function is then large, i.e. M is near-singular and the FP32
// recursion has lost digits), marks the node for recomputation in FP64 (bit 8).
#ifndef NEGF_FP32_WMAX
#define NEGF_FP32_WMAX 16.0
#endif
// ------------------------------------------------- real nodes at ring size 1
// One real-axis node of a scalar chain, whole (Algorithms 1-2 for 1 x 1 blocks),
// in one lane and without recursion stores: the stores of the block form would
// cost 2 x 16 bytes per ring written and read again, which bounds those kernels
// by HBM.  Instead the recursion states are kept every K rings (checkpoints, in
// the node's own store slots) and the K values a column step needs are
// recomputed from the nearest checkpoint into registers:
//   pass 1  forward recursion y_n, checkpoint y_{jK-1} (j >= 1); G_{N-1,N-1};
//   pass 2  down the rings in segments of K: recompute the segment's y~ from its
//           checkpoint, step the right-lead column W <- -y~_n W (A_R of every
//           ring), and run the backward recursion x_n alongside, checkpointing
//           x_{jK}; G_00 at the end, and T_LR from W = G_{0,N-1};
//   pass 3  up the rings: recompute each segment's x~ from its checkpoint and
//           step the left-lead column W <- -x~_n W (A_L); T_RL from G_{N-1,0}.
// The step arithmetic is that of k_recur / k_column at ring size 1, so the
// outputs are those of the store-based form; the recursion runs 4 steps per ring
// instead of 2 and touches no store between checkpoints.
constexpr int CHAIN1_K = 16;

template <typename TS>
struct Chain1 {
    static constexpr bool kF32 = sizeof(TS) == 4;
    const JobDesc& J;
    int e, N, K;
    cx<double> z;

    // coupling h of ring block c (n -> n+1)
    __device__ __forceinline__ cx<TS> coupling(int c) const {
        const int base = gload_s(J.ell_map + c) * K;
        TS hr = TS(0), hi = TS(0);
        for (int t = 0; t < K; ++t) {
            const cx<double> h = gload(J.cval + base + t);
            hr += TS(h.re);
            hi += TS(h.im);
        }
        return cx<TS>{hr, hi};
    }
    // (a_n - state)^{-1}; FP32-bulk inverts the two rings with a lead self-energy in FP64
    __device__ __forceinline__ cx<TS> inv(int n, double u, TS sr, TS si) const {
        if (!kF32 || n == 0 || n == N - 1) {
            const cx<double> a = scalar_a(J, e, n, u, z);
            double qr, qi;
            pivot_recip(a.re - (double)sr, a.im - (double)si, qr, qi);
            return cx<TS>{TS(qr), TS(qi)};
        }
        TS mr = TS(z.re - u) - sr, mi = TS(z.im) - si;
        if (!J.hdiag_zero) {
            const cx<double> h = gload(J.hdiag + n);
            mr -= TS(h.re);
            mi -= TS(h.im);
        }
        TS ir, ii;
        pivot_recip(mr, mi, ir, ii);
        return cx<TS>{ir, ii};
    }
    // one recursion step from the inverse: t = inv p, next state = q t
    // (dir 0: p = -h, q = -conj(h); dir 1: p = -conj(h), q = -h)
    __device__ __forceinline__ static cx<TS> tilde(cx<TS> in, cx<TS> h, int dir) {
        const TS pr = -h.re, pi = dir ? h.im : -h.im;
        return cx<TS>{fma(in.re, pr, -(in.im * pi)), fma(in.re, pi, in.im * pr)};
    }
    __device__ __forceinline__ static cx<TS> next(cx<TS> t, cx<TS> h, int dir) {
        const TS qr = -h.re, qi = dir ? -h.im : h.im;
        return cx<TS>{fma(qr, t.re, -(qi * t.im)), fma(qr, t.im, qi * t.re)};
    }
};

// W <- -p W in FP64
__device__ __forceinline__ void col_step(double& wr, double& wi, double pre, double pim) {
    const double pr = -pre, pi = -pim;
    const double nr = fma(pr, wr, -(pi * wi)), ni = fma(pr, wi, pi * wr);
    wr = nr;
    wi = ni;
}

template <typename TS>
__device__ __forceinline__ void chain_scalar(const JobDesc& J, cx<TS>* ckf, cx<TS>* ckb, int e, int ir) {
    constexpr int KS = CHAIN1_K;
    const int N = J.N;
    const Chain1<TS> C{J, e, N, J.K, gload(J.z + e)};
    const double gR = -2.0 * gload(J.sigma + (size_t)e * 2 + 1).im;
    const double gL = -2.0 * gload(J.sigma + (size_t)e * 2 + 0).im;
    double* aL = reinterpret_cast<double*>(J.a_diag) + ((size_t)ir * 2 + 0) * N;
    double* aR = reinterpret_cast<double*>(J.a_diag) + ((size_t)ir * 2 + 1) * N;
    cx<TS> y{TS(0), TS(0)};
    // ---- pass 1: forward recursion (a segment's potentials and couplings loaded first)
    cx<TS> gNN{TS(0), TS(0)};
    const int nseg = (N + KS - 1) / KS;
    for (int j = 0; j < nseg; ++j) {
        const int lo = j * KS;
        double uu[KS];
        cx<TS> hh[KS];
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int n = lo + k;
            uu[k] = n < N ? gload_s(J.U + n) : 0.0;
            hh[k] = n < N - 1 ? C.coupling(n) : cx<TS>{TS(0), TS(0)};
        }
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int n = lo + k;
            if (n < N) {
                if (k == KS - 1) gstore(ckf + j + 1, y);         // y_{jK-1}: checkpoint j + 1 (n = (j+1)K - 1)
                const cx<TS> iv = C.inv(n, uu[k], y.re, y.im);
                if (n == N - 1)
                    gNN = iv;
                else
                    y = Chain1<TS>::next(Chain1<TS>::tilde(iv, hh[k], 0), hh[k], 0);
            }
        }
    }
    // ---- pass 2: right-lead column down the rings, backward recursion alongside
    double wr = (double)gNN.re, wi = (double)gNN.im, wmR = 0.0, amnR = 0.0, amxR = 0.0;
    cx<TS> x{TS(0), TS(0)}, g00{TS(0), TS(0)};
    for (int j = nseg - 1; j >= 0; --j) {
        const int lo = j * KS;
        // potentials of rings lo-1 .. lo+K-1 and couplings of blocks lo-1 .. lo+K-2
        double uu[KS + 1];
        cx<TS> hh[KS];
#pragma unroll
        for (int k = 0; k <= KS; ++k) {
            const int n = lo - 1 + k;
            uu[k] = n >= 0 && n < N ? gload_s(J.U + n) : 0.0;
            if (k < KS) hh[k] = n >= 0 && n < N - 1 ? C.coupling(n) : cx<TS>{TS(0), TS(0)};
        }
        // y~_n for the rings of this segment (n >= 1): forward steps lo-1 .. lo+K-2
        cx<TS> buf[KS];
        cx<TS> ys = j == 0 ? cx<TS>{TS(0), TS(0)} : gload(ckf + j);
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int n = lo - 1 + k;               // forward step n gives y~_{n+1} = buf[k]
            if (n >= 0 && n < N - 1) {
                const cx<TS> t = Chain1<TS>::tilde(C.inv(n, uu[k], ys.re, ys.im), hh[k], 0);
                buf[k] = t;
                ys = Chain1<TS>::next(t, hh[k], 0);
            } else {
                buf[k] = cx<TS>{TS(0), TS(0)};
            }
        }
#pragma unroll
        for (int k = KS - 1; k >= 0; --k) {
            const int n = lo + k;
            if (n < N) {
                const double acc = gR * fma(wr, wr, wi * wi);
                gstore_s(aR + n, acc);
                wmR = fmax(wmR, fabs(wr) + fabs(wi));
                amnR = n == N - 1 ? acc : fmin(amnR, acc);
                amxR = n == N - 1 ? acc : fmax(amxR, acc);
                // backward recursion at ring n (state x_n), checkpoint x_{jK}
                if (k == 0 && n > 0) gstore(ckb + j, x);
                const cx<TS> iv = C.inv(n, uu[k + 1], x.re, x.im);
                if (n == 0) {
                    g00 = iv;
                } else {
                    x = Chain1<TS>::next(Chain1<TS>::tilde(iv, hh[k], 1), hh[k], 1);   // block n-1
                    col_step(wr, wi, (double)buf[k].re, (double)buf[k].im);
                }
            }
        }
    }
    const double tLR = gL * gR * fma(wr, wr, wi * wi);
    // ---- pass 3: left-lead column up the rings
    wr = (double)g00.re;
    wi = (double)g00.im;
    double wmL = 0.0, amnL = 0.0, amxL = 0.0;
    for (int j = 0; j < nseg; ++j) {
        const int lo = j * KS;
        const int top = min(lo + KS, N - 1);
        // potentials of rings lo+1 .. lo+K and couplings of blocks lo .. lo+K-1
        double uu[KS];
        cx<TS> hh[KS];
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int n = lo + k + 1;
            uu[k] = n <= top ? gload_s(J.U + n) : 0.0;
            hh[k] = n <= top ? C.coupling(n - 1) : cx<TS>{TS(0), TS(0)};
        }
        // x~_n for the rings of this segment (n < N-1): backward steps top .. lo+1
        cx<TS> buf[KS];
        cx<TS> xs = top == N - 1 ? cx<TS>{TS(0), TS(0)} : gload(ckb + j + 1);
#pragma unroll
        for (int k = KS - 1; k >= 0; --k) {
            const int n = lo + k + 1;               // backward step n gives x~_{n-1} = buf[k]
            if (n <= top) {
                const cx<TS> t = Chain1<TS>::tilde(C.inv(n, uu[k], xs.re, xs.im), hh[k], 1);
                buf[k] = t;
                xs = Chain1<TS>::next(t, hh[k], 1);
            } else {
                buf[k] = cx<TS>{TS(0), TS(0)};
            }
        }
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int n = lo + k;
            if (n < N) {
                const double acc = gL * fma(wr, wr, wi * wi);
                gstore_s(aL + n, acc);
                wmL = fmax(wmL, fabs(wr) + fabs(wi));
                amnL = n == 0 ? acc : fmin(amnL, acc);
                amxL = n == 0 ? acc : fmax(amxL, acc);
                if (n < N - 1) col_step(wr, wi, (double)buf[k].re, (double)buf[k].im);
            }
        }
    }
    const double tRL = gR * gL * fma(wr, wr, wi * wi);
    gstore_s(J.Tout + ir, tLR);
    gstore_s(J.Trl + ir, tRL);
    gstore_s(J.amax + 2 * ir + 0, amxL);
    gstore_s(J.amax + 2 * ir + 1, amxR);
    bool bad = false, big = false;
    const double ts[2] = {tRL, tLR}, amn[2] = {amnL, amnR}, amx[2] = {amxL, amxR}, wm[2] = {wmL, wmR};
#pragma unroll
    for (int l = 0; l < 2; ++l) {
        bad = bad || !(ts[l] >= -1e-6 && ts[l] <= 1.0 + 1e-6) || !(amn[l] >= -1e-6 * fabs(amx[l])) ||
              !(amx[l] < 1e300);
        big = big || wm[l] * (fabs(C.z.re) + fabs(C.z.im) + J.hnorm) > NEGF_FP32_WMAX;
    }
    if constexpr (sizeof(TS) == 4) {
        if (bad || big) atomicOr(&J.status[e], (int)ST_FP64);
    } else {
        if (bad) atomicOr(&J.status[e], (int)ST_BAD);
    }
}

// One contour node of a scalar chain, whole: diag G^R_nn = (a_n - x_n - y_n)^{-1}
// (Algorithm 1) without recursion stores.  Pass 1 runs the forward recursion
// and keeps y_{jK}; pass 2 walks down the rings in segments of K, recomputes the
// segment's y_n from its checkpoint into registers and runs the backward
// recursion x_n alongside, writing G_nn per ring.  Same arithmetic as k_recur
// and k_cdiag at ring size 1.
template <typename TS>
__device__ __forceinline__ void chain_contour(const JobDesc& J, cx<TS>* ckf, int e) {
    constexpr int KS = CHAIN1_K;
    constexpr bool kF32 = sizeof(TS) == 4;
    const int N = J.N;
    const Chain1<TS> C{J, e, N, J.K, gload(J.z + e)};
    cx<TS>* out = reinterpret_cast<cx<TS>*>(J.gr_diag) + (size_t)e * N;
    const int nseg = (N + KS - 1) / KS;
    // ---- pass 1: forward recursion, checkpoint y_{jK}
    cx<TS> y{TS(0), TS(0)};
    for (int j = 0; j < nseg; ++j) {
        const int lo = j * KS;
        double uu[KS];
        cx<TS> hh[KS];
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int n = lo + k;
            uu[k] = n < N - 1 ? gload_s(J.U + n) : 0.0;
            hh[k] = n < N - 1 ? C.coupling(n) : cx<TS>{TS(0), TS(0)};
        }
        if (j > 0) gstore(ckf + j, y);
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int n = lo + k;
            if (n < N - 1) y = Chain1<TS>::next(Chain1<TS>::tilde(C.inv(n, uu[k], y.re, y.im), hh[k], 0), hh[k], 0);
        }
    }
    // ---- pass 2: down the rings; y_n recomputed per segment, x_n alongside
    cx<TS> x{TS(0), TS(0)};
    for (int j = nseg - 1; j >= 0; --j) {
        const int lo = j * KS;
        // potentials of rings lo .. lo+K-1, couplings of blocks lo-1 .. lo+K-2
        double uu[KS];
        cx<TS> hh[KS + 1];
#pragma unroll
        for (int k = 0; k <= KS; ++k) {
            const int c = lo - 1 + k;
            hh[k] = c >= 0 && c < N - 1 ? C.coupling(c) : cx<TS>{TS(0), TS(0)};
            if (k < KS) uu[k] = lo + k < N ? gload_s(J.U + lo + k) : 0.0;
        }
        cx<TS> ys[KS];
        ys[0] = j == 0 ? cx<TS>{TS(0), TS(0)} : gload(ckf + j);
#pragma unroll
        for (int k = 0; k + 1 < KS; ++k) {
            const int n = lo + k;
            ys[k + 1] = n < N - 1 ? Chain1<TS>::next(Chain1<TS>::tilde(C.inv(n, uu[k], ys[k].re, ys[k].im), hh[k + 1], 0),
                                                     hh[k + 1], 0)
                                  : ys[k];
        }
#pragma unroll
        for (int k = KS - 1; k >= 0; --k) {
            const int n = lo + k;
            if (n < N) {
                // G_nn = (a_n - x_n - y_n)^{-1}
                cx<TS> g;
                if (!kF32 || n == 0 || n == N - 1) {
                    const cx<double> a = scalar_a(J, e, n, uu[k], C.z);
                    double qr, qi;
                    pivot_recip(a.re - (double)ys[k].re - (double)x.re, a.im - (double)ys[k].im - (double)x.im, qr, qi);
                    g = cx<TS>{TS(qr), TS(qi)};
                } else {
                    TS mr = TS(C.z.re - uu[k]) - ys[k].re - x.re, mi = TS(C.z.im) - ys[k].im - x.im;
                    if (!J.hdiag_zero) {
                        const cx<double> h = gload(J.hdiag + n);
                        mr -= TS(h.re);
                        mi -= TS(h.im);
                    }
                    TS qr, qi;
                    pivot_recip(mr, mi, qr, qi);
                    g = cx<TS>{qr, qi};
                }
                gstore(out + n, g);
                // backward recursion step at ring n (block n-1)
                if (n > 0) x = Chain1<TS>::next(Chain1<TS>::tilde(C.inv(n, uu[k], x.re, x.im), hh[k], 1), hh[k], 1);
            }
        }
    }
}

template <typename TS, int B>
__global__ __launch_bounds__(64, NEGF_RGF_WAVES) __attribute__((amdgpu_waves_per_eu(NEGF_RGF_WAVES, NEGF_RGF_WAVES))) void k_column(Sched S) {
    using T = double;
    constexpr int G = 64 / B;
    __shared__ cx<T> s_stage[G][B * B];
    __shared__ cx<T> s_gam[G][B * B];
    __shared__ double s_chk[G][4][B];
    __shared__ double s_lam[G][B];   // eigenvalues of a circulant Gamma (FP64 stores)

    const int lane = threadIdx.x;
    const int gi = lane / B;
    const int gsafe = gi < G ? gi : 0;
    const int r = lane - gi * B;
    cx<T>* St = s_stage[gsafe];
    cx<T>* Gm = s_gam[gsafe];

    if constexpr (B == 1) {
        if (S.lane_spans) {
            // the round's node list: node k = span k, taken 64 at a time; m nodes this round
            // (the unit prefix holds two units per node)
            const int m = S.first[S.n_spans] / 2;
            for (;;) {
                int w = 0;
                if (threadIdx.x == 0) w = atomicAdd(S.counter, 1);
                w = __builtin_amdgcn_readfirstlane(w);
                if (w * 64 >= m) break;
                const int k = w * 64 + lane;
                if (k < m) {
                    const Span sp = S.spans[k];
                    const JobDesc& J = S.jobs[sp.job];
                    chain_scalar<TS>(J, reinterpret_cast<cx<TS>*>(S.store_f) + sp.off,
                                     reinterpret_cast<cx<TS>*>(S.store_b) + sp.off, sp.e0, sp.e0 - J.n_c);
                }
            }
            return;
        }
    }
    Unit u;
    while (next_unit<G>(S, u)) {
        const JobDesc& J = S.jobs[u.job];
        const int lead = u.side;
        // Sigma of this lead came from the ring-mode decimation and is exactly circulant
        const bool gcirc = J.lmodes[lead] != nullptr && J.sigma_circ;
        const bool act = (gi < G) && (gi < u.cnt);
        const int N = J.N;
        const int e = u.e0 + (act ? gi : 0);     // node index within the job (>= n_c)
        const int ir = e - J.n_c;                 // real-axis index
        if constexpr (B == 1) {   // scalar chains: a real node whole per lane (both leads, side 0)
            if (act && lead == 0) {
                const size_t o = u.off + (size_t)(u.i0 + gi) * N;
                chain_scalar<TS>(J, reinterpret_cast<cx<TS>*>(S.store_f) + o, reinterpret_cast<cx<TS>*>(S.store_b) + o,
                                 e, ir);
            }
            continue;
        }
        wave_sync();
        if (act) {
            const cx<double>* s = J.sigma + ((size_t)e * 2 + lead) * B * B;
#pragma unroll
            for (int j = 0; j < B; ++j) {
                const cx<double> a = gload(s + r * B + j), b = gload(s + j * B + r);
                // Gamma[r][j] = i (Sigma[r][j] - conj(Sigma[j][r]))
                Gm[r * B + j] = cx<T>{T(-(a.im + b.im)), T(a.re - b.re)};
            }
        }
        const cx<TS>* store = reinterpret_cast<const cx<TS>*>(lead ? S.store_f : S.store_b) + u.off +
                              (size_t)(u.i0 + (act ? gi : 0)) * N * B * B;
        T wr[B], wi[B];
#pragma unroll
        for (int j = 0; j < B; ++j) { wr[j] = T(0); wi[j] = T(0); }
        if (act) {
            const cx<TS>* w0 = store + ((size_t)(lead ? 0 : N - 1) * B + r) * B;
#pragma unroll
            for (int j = 0; j < B; ++j) { const cx<TS> v = gload(w0 + j); wr[j] = v.re; wi[j] = v.im; }
        }
        // A circulant Gamma = sum_q lambda_q v_q v_q^H (v_q[j] = e^{2 pi i q j / B} / sqrt(B),
        // lambda_q = sum_d Gamma[0][d] e^{2 pi i q d / B}): with W' = W F^H (columns in the
        // ring Fourier basis, F^H[k][q] = v_q[k]) the propagation W' <- -P W' is unchanged
        // and diag(W Gamma W^H)_rr = sum_q lambda_q |W'[r][q]|^2, B terms instead of B^2.
        // The FP32 size check then uses sqrt(2) |W_r|_2, the same in both bases and never
        // below max_j (|Re W_rj| + |Im W_rj|).
        const bool four = gcirc;
        stage_row<T, B>(wr, wi, St, r, act);
        if (four) {
            wave_sync();   // Gamma and the rows of W are in LDS
            {
                double lr = 0.0;   // lambda_r (real: Gamma is Hermitian)
                for (int d = 0; d < B; ++d) {
                    double sn, cs;
                    sincospi(2.0 * (double)((r * d) % B) / B, &sn, &cs);
                    const cx<T> c = Gm[d];
                    lr = fma((double)c.re, cs, fma(-(double)c.im, sn, lr));
                }
                if (act) s_lam[gsafe][r] = lr;
            }
            T twr[B], twi[B];   // e^{2 pi i m / B}
#pragma unroll
            for (int m = 0; m < B; ++m) {
                double sn, cs;
                sincospi(2.0 * m / B, &sn, &cs);
                twr[m] = cs;
                twi[m] = sn;
            }
            const T sc = T(1) / sqrt(T(B));
            const cx<T>* row = St + r * B;   // this lane's row of W
#pragma unroll
            for (int q = 0; q < B; ++q) {
                T ar = T(0), ai = T(0);
#pragma unroll
                for (int k = 0; k < B; ++k) {
                    const int m = (q * k) % B;
                    const cx<T> x = row[k];
                    ar = fma(x.re, twr[m], fma(-x.im, twi[m], ar));
                    ai = fma(x.re, twi[m], fma(x.im, twr[m], ai));
                }
                wr[q] = ar * sc;
                wi[q] = ai * sc;
            }
            wave_sync();
            stage_row<T, B>(wr, wi, St, r, act);   // the rows of W'
        }
        wave_sync();
        double* aout = reinterpret_cast<double*>(J.a_diag) + ((size_t)(act ? ir : 0) * 2 + lead) * N * B;
        // this row's max |W_rj| and range of A_rr along the chain, kept in LDS (the
        // propagation holds every register)
        double* trk = &s_chk[gsafe][0][0] + 4 * r;   // [wmag, amin, amax, -] of row r

        for (int s = 0; s < N; ++s) {
            const int n = lead ? N - 1 - s : s;
            // propagator row for this step, loaded ahead of the Gamma product
            T pr[B], pi[B];
#pragma unroll
            for (int j = 0; j < B; ++j) { pr[j] = T(0); pi[j] = T(0); }
            if (act && s < N - 1) {
                const cx<TS>* p = store + ((size_t)n * B + r) * B;
#pragma unroll
                for (int j = 0; j < B; ++j) { const cx<TS> v = gload(p + j); pr[j] = -T(v.re); pi[j] = -T(v.im); }
            }
            double wm = 0.0;   // read by the FP32 checks only
            if (sizeof(TS) == 4 && four) {
                double s2 = 0.0;
#pragma unroll
                for (int j = 0; j < B; ++j) s2 = fma(wr[j], wr[j], fma(wi[j], wi[j], s2));
                wm = sqrt(2.0 * s2);
            } else {
#pragma unroll
                for (int j = 0; j < B; ++j) wm = fmax(wm, fabs(wr[j]) + fabs(wi[j]));
            }
            // diag(W Gamma W^H)_rr = Re sum_j (W Gamma)[r][j] conj(W[r][j]).  Gamma does not
            // change along the chain; its offset is made opaque each step so that its
            // B*B reads are not hoisted out of the loop into (spilled) registers.
            // For a ring-circulant lead (Sigma, hence Gamma, circulant by construction of the
            // ring-mode decimation) only Gamma's first row is read.
            int goff = gsafe * B * B;
            asm volatile("" : "+v"(goff));
            T acc;
            if (four) {   // sum_q lambda_q |W'[r][q]|^2
                int loff = gsafe * B;
                asm volatile("" : "+v"(loff));
                const double* lam = &s_lam[0][0] + loff;
                acc = T(0);
#pragma unroll
                for (int q = 0; q < B; ++q) acc = fma(T(lam[q]), fma(wr[q], wr[q], wi[q] * wi[q]), acc);
            } else {
                acc = gcirc ? row_quad_circ<T, B>(wr, wi, &s_gam[0][0] + goff)
                            : row_quad_pipe<T, B>(wr, wi, &s_gam[0][0] + goff);
            }
            if (act) {
                gstore_s(aout + (size_t)n * B + r, acc);
                if (s == 0) {
                    trk[0] = wm;
                    trk[1] = acc;
                    trk[2] = acc;
                } else {
                    trk[0] = fmax(trk[0], wm);
                    trk[1] = fmin(trk[1], acc);
                    trk[2] = fmax(trk[2], acc);
                }
            }
            if (s == N - 1) break;
            // W_next[r][:] = -sum_k P[r][k] W[k][:],  P = y~_n (right) or x~_n (left)
            row_mul_pipe<T, B>(pr, pi, St, wr, wi);
            wave_sync();
            stage_row<T, B>(wr, wi, St, r, act);
            wave_sync();
        }
        // Transmission from the far end of the chain (Eq. 5): the right chain ends with
        // W = G_{0,N-1} and gives T_LR = Tr[Gamma_L W Gamma_R W^H]; the left chain ends
        // with W = G_{N-1,0} and gives T_RL = Tr[Gamma_R W Gamma_L W^H].  Both are formed
        // as sum_{r,j'} Gamma_o[j'][r] (W Gamma_l W^H)[r][j'] with this lead's Gamma_l in
        // LDS and the other lead's Gamma_o read from its self-energy.
        double t = 0.0;
        {
            T vr[B], vi[B];
            if (four) {   // (W' diag(lambda))[r][q]; St holds the rows of W'
#pragma unroll
                for (int q = 0; q < B; ++q) {
                    const T l = T(s_lam[gsafe][q]);
                    vr[q] = l * wr[q];
                    vi[q] = l * wi[q];
                }
            } else {
                row_mul<T, B>(wr, wi, Gm, vr, vi);
            }
            if (act) {
                const cx<double>* sl = J.sigma + ((size_t)e * 2 + (1 - lead)) * B * B;
                for (int jp = 0; jp < B; ++jp) {
                    double mr = 0.0, mi = 0.0;   // (W Gamma_R W^H)[r][jp] = sum_j v[j] conj(W[jp][j])
#pragma unroll
                    for (int j = 0; j < B; ++j) {
                        const cx<T> wv = St[jp * B + j];
                        mr += vr[j] * wv.re + vi[j] * wv.im;
                        mi += vi[j] * wv.re - vr[j] * wv.im;
                    }
                    const cx<double> a = gload(sl + jp * B + r), b = gload(sl + r * B + jp);
                    const double gre = -(a.im + b.im), gim = a.re - b.re;   // Gamma_o[jp][r]
                    t += gre * mr - gim * mi;
                }
            }
        }
        // chain-wide sums and extremes in fixed order through LDS
        wave_sync();
        if (act) trk[3] = t;
        wave_sync();
        if (act && r == 0) {
            const double* tk = &s_chk[gsafe][0][0];
            double tsum = 0.0, wm = 0.0, amn = tk[1], amx = tk[2];
            for (int q = 0; q < B; ++q) {
                tsum += tk[4 * q + 3];
                wm = fmax(wm, tk[4 * q + 0]);
                amn = fmin(amn, tk[4 * q + 1]);
                amx = fmax(amx, tk[4 * q + 2]);
            }
            gstore_s((lead == 1 ? J.Tout : J.Trl) + ir, tsum);
            gstore_s(J.amax + 2 * ir + lead, amx);
            const bool bad_T = !(tsum >= -1e-6 && tsum <= B * (1.0 + 1e-6));
            const bool bad_A = !(amn >= -1e-6 * fabs(amx)) || !(amx < 1e300);
            if constexpr (sizeof(TS) == 4) {
                const cx<double> z = gload(J.z + e);
                const bool big_w = wm * (fabs(z.re) + fabs(z.im) + J.hnorm) > NEGF_FP32_WMAX;
                if (bad_T || bad_A || big_w) atomicOr(&J.status[e], (int)ST_FP64);
            } else {
                if (bad_T || bad_A) atomicOr(&J.status[e], (int)ST_BAD);
            }
        }
        wave_sync();
    }
}

// ============================================================= k_decimate ==
// Chain = (energy, lead).  Sancho-Rubio layer doubling on the principal layer
// of `period` rings (Section 2.2.2).  The coupling of a layer to the next, alpha,
// is non-zero only in its (P-1,0) block A, and beta = alpha^H only in its
// (0,P-1) block Bm; the doubling keeps that shape and changes only the corner
// diagonal blocks of eps, so every product is b x b.  Convergence: every
// |A_ij|, |Bm_ij| < tol.  Then Sigma = tau g_s[0,0] tau^H.  Nodes are used as
// given (real nodes carry i*eta).
//
//   P = 1 (k_decimate):  g = (z-e)^{-1}; es += A g Bm; e += A g Bm + Bm g A;
//                        A <- A g A; Bm <- Bm g Bm;  g_s = (z-es)^{-1}
//   P = 2 (k_decimate2): eps = [[e00, V],[V^H, e11]], eps_s(0,0) = D0,
//                        eps_s(0,1) = V and eps_s(1,1) == e11 at every step;
//                        g = (z-eps)^{-1} by one pivoted 2b x 2b inversion;
//                        e11 += A g00 Bm; e00 += Bm g11 A; A <- A g01 A;
//                        Bm <- Bm g10 Bm;  g_s00 = [(z-eps_s)^{-1}]_00.
// The 2b x 2b inversion matters: forming g00 from the Schur complement
// z-e00 - V (z-e11)^{-1} V^H loses about |V|^2 |(z-e11)^{-1}| / |g00^{-1}| of
// the working precision, which is total where z meets an eigenvalue of a single
// ring block (E = 0 for zigzag rings with zero on-site energy).

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

// out = x * Y for a B x B block Y inside an LDS matrix of row stride LD (unrolled:
// x lives in registers and may only be indexed by compile-time constants)
template <int B, int LD>
__device__ __forceinline__ void row_mul_ld(const double (&xr)[B], const double (&xi)[B], const cx<double>* Y,
                                           double (&orr)[B], double (&oi)[B]) {
#pragma unroll
    for (int j = 0; j < B; ++j) { orr[j] = 0.0; oi[j] = 0.0; }
#pragma unroll
    for (int k = 0; k < B; ++k) {
        const double a = xr[k], b = xi[k];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const cx<double> q = Y[k * LD + j];
            orr[j] = fma(a, q.re, fma(-b, q.im, orr[j]));
            oi[j] = fma(a, q.im, fma(b, q.re, oi[j]));
        }
    }
}

// Sigma row r = (tau[r,:] g) tau^H, g = B x B block of row stride LD in LDS
template <int B, int LD>
__device__ __forceinline__ void sigma_row(const cx<double>* tau, const cx<double>* g, int r, cx<double>* out) {
    double xr[B], xi[B], ur[B], ui[B], dr[B], di[B];
    gl_row<B>(tau, r, xr, xi);
    row_mul_ld<B, LD>(xr, xi, g, ur, ui);
#pragma unroll
    for (int j = 0; j < B; ++j) { dr[j] = 0.0; di[j] = 0.0; }
#pragma unroll
    for (int q = 0; q < B; ++q) {
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const cx<double> h = tau[j * B + q];   // tau^H[q][j] = conj(tau[j][q])
            dr[j] += ur[q] * h.re + ui[q] * h.im;
            di[j] += ui[q] * h.re - ur[q] * h.im;
        }
    }
    gs_row<B>(out, r, dr, di);
}

// ---- P = 1: group of B lanes per chain, state in a per-workgroup global scratch
template <int B>
__device__ __forceinline__ void decimate_chain1(const JobDesc& J, int lead, double tol, int maxit, int k, bool act,
                                                cx<double>* sc, cx<double> (&s_buf)[3][64 / B][B * B],
                                                cx<double> (&s_prow)[64 / B][B], unsigned (&s_keys)[64 / B][B],
                                                int (&s_flag)[64 / B]) {
    constexpr int G = 64 / B;
    using T = double;
    const int lane = threadIdx.x;
    const int gi = lane / B;
    const int gsafe = gi < G ? gi : 0;
    const int r = lane - gi * B;
    cx<T>* L0 = s_buf[0][gsafe];
    cx<T>* L1 = s_buf[1][gsafe];
    cx<T>* L2 = s_buf[2][gsafe];
    const cx<double> z = J.z[k];
    cx<double>* E0 = sc;               // e
    cx<double>* E1 = sc + 1 * B * B;   // eps_s
    cx<double>* MA = sc + 2 * B * B;   // alpha
    cx<double>* MB = sc + 3 * B * B;   // beta

    bool live = act;   // chain still iterating
    T xr[B], xi[B], ur[B], ui[B], dr[B], di[B], nr[B], ni[B];
    if (act) {
        gl_row<B>(J.D[lead], r, xr, xi);
        gs_row<B>(E0, r, xr, xi);
        gs_row<B>(E1, r, xr, xi);
        gl_row<B>(J.W[lead], r, xr, xi);
        gs_row<B>(MA, r, xr, xi);
#pragma unroll
        for (int j = 0; j < B; ++j) { const cx<double> v = J.W[lead][j * B + r]; xr[j] = v.re; xi[j] = -v.im; }
        gs_row<B>(MB, r, xr, xi);
    }

    // dst <- (z I - M)^{-1} for the live chains
    auto inv_from = [&](const cx<double>* M, cx<T>* dst) {
        T kr[B], ki[B];
#pragma unroll
        for (int j = 0; j < B; ++j) { kr[j] = T(0); ki[j] = T(0); }
        if (live) {
            gl_row<B>(M, r, kr, ki);
#pragma unroll
            for (int j = 0; j < B; ++j) {
                kr[j] = -kr[j];
                ki[j] = -ki[j];
                if (j == r) { kr[j] += z.re; ki[j] += z.im; }
            }
        }
        Grp<T, B> gg{r, live, dst, s_prow[gsafe], s_keys[gsafe]};
        gj_inverse<T, B>(kr, ki, gg);
    };
    auto stage_global = [&](const cx<double>* M, cx<T>* dst) {
        if (live) { T a[B], b[B]; gl_row<B>(M, r, a, b); stage_row<T, B>(a, b, dst, r, true); }
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

    int it_done = maxit;
    for (int it = 1; it <= maxit; ++it) {
        inv_from(E0, L0);                             // L0 = g
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
        // convergence of the live chains: every |A_ij|, |Bm_ij| < tol
        if (live && r == 0) s_flag[gi] = 0;
        wave_sync();
        if (live) {
            bool big = false;
            gl_row<B>(MA, r, xr, xi);
#pragma unroll
            for (int j = 0; j < B; ++j) big |= !(hypot(xr[j], xi[j]) < tol);
            gl_row<B>(MB, r, xr, xi);
#pragma unroll
            for (int j = 0; j < B; ++j) big |= !(hypot(xr[j], xi[j]) < tol);
            if (big) s_flag[gi] = 1;
        }
        wave_sync();
        if (live && s_flag[gi] == 0) { live = false; it_done = it; }
        wave_sync();
        if (__all(!live)) break;
    }
    const bool converged = act && !live;

    live = act;
    inv_from(E1, L0);                                 // g_s = (z - eps_s)^{-1}
    if (act) sigma_row<B, B>(J.tau[lead], L0, r, J.sigma + ((size_t)k * 2 + lead) * B * B);
    if (act && r == 0) {
        J.iters[(size_t)k * 2 + lead] = it_done;
        if (!converged) atomicOr(&J.status[k], (int)ST_NOCONV);
    }
}

template <int B>
__global__ __launch_bounds__(64) void k_decimate(Sched S) {
    constexpr int G = 64 / B;
    __shared__ cx<double> s_buf[3][G][B * B];
    __shared__ cx<double> s_prow[G][B];
    __shared__ unsigned s_keys[G][B];
    __shared__ int s_flag[G];
    const int lane = threadIdx.x;
    const int gi = lane / B;
    Unit u;
    // chain state is per workgroup: chains of earlier units are finished
    cx<double>* sc_wg = S.scratch + (size_t)blockIdx.x * G * 4 * B * B;
    while (next_unit<G>(S, u)) {
        const JobDesc& J = S.jobs[u.job];
        const bool act = (gi < G) && (gi < u.cnt);
        const int k = u.e0 + (act ? gi : 0);
        cx<double>* sc = sc_wg + (size_t)(gi < G ? gi : 0) * 4 * B * B;
        decimate_chain1<B>(J, u.side, S.tol, S.maxit, k, act, sc, s_buf, s_prow, s_keys, s_flag);
        wave_sync();
    }
}

// ---- P = 2: group of 2B lanes per chain.  Lane q < B owns row q of the top
// half of z - eps ([z-e00 | -V]) and row q of e00 and Bm; lane B+i owns row i
// of the bottom half ([-V^H | z-e11]) and row i of e11 and A.  A and Bm are
// also kept in LDS as right operands; the layer Green's function g lands in
// the group's 2B x 2B stage.
template <int B>
__global__ __launch_bounds__(64) void k_decimate2(Sched S) {
    constexpr int BB = 2 * B;
    constexpr int G = 64 / BB;
    __shared__ cx<double> s_g[G][BB * BB];
    __shared__ cx<double> s_E[G][BB * B];     // row q: e00 row q (top) / e11 row q - B (bottom)
    __shared__ cx<double> s_A[G][B * B];
    __shared__ cx<double> s_Bm[G][B * B];
    __shared__ cx<double> s_prow[G][BB];
    __shared__ unsigned s_keys[G][BB];
    __shared__ int s_flag[G];
    const int lane = threadIdx.x;
    const int gi = lane / BB;
    const int gsafe = gi < G ? gi : 0;
    const int q = lane - gi * BB;          // row of the layer matrix
    const bool top = q < B;
    const int i = top ? q : q - B;         // row inside the ring block
    cx<double>* Sg = s_g[gsafe];
    cx<double>* SE = s_E[gsafe] + q * B;   // this lane's e row
    cx<double>* SA = s_A[gsafe];
    cx<double>* SB = s_Bm[gsafe];

    Unit u;
    while (next_unit<G>(S, u)) {
        const JobDesc& J = S.jobs[u.job];
        const int lead = u.side;
        const bool act = (gi < G) && (gi < u.cnt);
        const int k = u.e0 + (act ? gi : 0);
        const cx<double> z = J.z[k];
        const cx<double>* D = J.D[lead];
        const cx<double>* V = J.V[lead];
        const cx<double>* VH = J.VH[lead];
        const cx<double>* W = J.W[lead];

        // e row (e00 on top lanes, e11 on bottom lanes), A = W, Bm = W^H, all in LDS
        wave_sync();
        if (act) {
            const cx<double>* d = D + (top ? 0 : B * B) + i * B;
#pragma unroll
            for (int j = 0; j < B; ++j) {
                SE[j] = d[j];
                if (top) { const cx<double> w = W[j * B + i]; SB[i * B + j] = cx<double>{w.re, -w.im}; }
                else SA[i * B + j] = W[i * B + j];
            }
        }
        wave_sync();

        // row q of z - eps, eps = [[e, V],[V^H, e']] (register indices stay compile-time
        // constants: the halves are selected by value)
        auto layer_row = [&](double (&mr)[BB], double (&mi)[BB]) {
#pragma unroll
            for (int j = 0; j < BB; ++j) { mr[j] = 0.0; mi[j] = 0.0; }
            if (act) {
                const cx<double>* cpl = (top ? V : VH) + i * B;
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    const cx<double> c = cpl[j];
                    const cx<double> e = SE[j];
                    const double dre = (j == i ? z.re : 0.0) - e.re;   // diagonal block entry
                    const double dim = (j == i ? z.im : 0.0) - e.im;
                    mr[j] = top ? dre : -c.re;
                    mi[j] = top ? dim : -c.im;
                    mr[B + j] = top ? -c.re : dre;
                    mi[B + j] = top ? -c.im : dim;
                }
            }
        };
        // out = X[row, :] * Y[:B, :B] with X (row stride B) and Y (row stride LY) in LDS
        auto lds_mul = [&](const cx<double>* Xrow, const cx<double>* Y, int LY, double (&orr)[B], double (&oi)[B]) {
#pragma unroll
            for (int j = 0; j < B; ++j) { orr[j] = 0.0; oi[j] = 0.0; }
#pragma unroll 1
            for (int kk = 0; kk < B; ++kk) {
                const cx<double> x = Xrow[kk];
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    const cx<double> y = Y[kk * LY + j];
                    orr[j] = fma(x.re, y.re, fma(-x.im, y.im, orr[j]));
                    oi[j] = fma(x.re, y.im, fma(x.im, y.re, oi[j]));
                }
            }
        };

        bool live = act;
        int it_done = S.maxit;
        for (int it = 1; it <= S.maxit; ++it) {
            {
                double mr[BB], mi[BB];
                layer_row(mr, mi);
                Grp<double, BB> g{q, live, Sg, s_prow[gsafe], s_keys[gsafe]};
                gj_inverse<double, BB>(mr, mi, g);        // Sg = g = (z - eps)^{-1}
            }
            // top row i:    e00 += (Bm g11) A,  Bm' = (Bm g10) Bm
            // bottom row i: e11 += (A g00) Bm,  A'  = (A g01) A
            const cx<double>* Xrow = (top ? SB : SA) + i * B;
            const cx<double>* g_diag = Sg + (top ? B * BB + B : 0);   // g11 (top) / g00 (bottom)
            const cx<double>* g_off = Sg + (top ? B * BB : B);        // g10 (top) / g01 (bottom)
            double tr[B], ti[B], nr[B], ni[B];
            lds_mul(Xrow, g_diag, BB, tr, ti);
            row_mul_ld<B, B>(tr, ti, top ? SA : SB, nr, ni);
            if (live) {
#pragma unroll
                for (int j = 0; j < B; ++j) {
                    const cx<double> e = SE[j];
                    SE[j] = cx<double>{e.re + nr[j], e.im + ni[j]};
                }
            }
            lds_mul(Xrow, g_off, BB, tr, ti);
            row_mul_ld<B, B>(tr, ti, top ? SB : SA, nr, ni);
            wave_sync();
            if (live) {
                cx<double>* dst = (top ? SB : SA) + i * B;
#pragma unroll
                for (int j = 0; j < B; ++j) dst[j] = cx<double>{nr[j], ni[j]};
            }
            // convergence of the live chains: every |A_ij|, |Bm_ij| < tol
            if (live && q == 0) s_flag[gi] = 0;
            wave_sync();
            if (live) {
                bool big = false;
#pragma unroll
                for (int j = 0; j < B; ++j) big |= !(hypot(nr[j], ni[j]) < S.tol);
                if (big) s_flag[gi] = 1;
            }
            wave_sync();
            if (live && s_flag[gi] == 0) { live = false; it_done = it; }
            wave_sync();
            if (__all(!live)) break;
        }
        const bool converged = act && !live;

        // surface layer: eps_s = [[D0, V],[V^H, e11]]
        live = act;
        if (act && top) {
#pragma unroll
            for (int j = 0; j < B; ++j) SE[j] = D[i * B + j];
        }
        wave_sync();
        {
            double mr[BB], mi[BB];
            layer_row(mr, mi);
            Grp<double, BB> g{q, live, Sg, s_prow[gsafe], s_keys[gsafe]};
            gj_inverse<double, BB>(mr, mi, g);
        }
        if (act && top) sigma_row<B, BB>(J.tau[lead], Sg, i, J.sigma + ((size_t)k * 2 + lead) * B * B);
        if (act && q == 0) {
            J.iters[(size_t)k * 2 + lead] = it_done;
            if (!converged) atomicOr(&J.status[k], (int)ST_NOCONV);
        }
        wave_sync();
    }
}

// ---- Ring-circulant leads: every lead block C satisfies C[i][j] = C[0][(j - i) mod b],
// so the ring Fourier vectors diagonalise all of them at once and the doubling runs
// on b independent scalar chains (lane = mode q): the same Sancho-Rubio steps with
// 1 x 1 blocks (period 1) or with the 2 x 2 layer [[z - e00, -v],[-v*, z - e11]]
// inverted in closed form (period 2, no single-ring Schur complement).  A chain is
// done when |A_q|, |Bm_q| < tol for every mode (a circulant block's entries are
// averages of its eigenvalues, so this is at least as strict as the entrywise rule).
// Sigma_q = tau_q g_q conj(tau_q); back in the ring basis Sigma[i][j] =
// c_{(i-j) mod b}, c_d = (1/b) sum_q Sigma_q e^{2 pi i q d / b}.
__device__ __forceinline__ cx<double> cmul(cx<double> a, cx<double> b) {
    return cx<double>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cx<double> cdiv(cx<double> a, cx<double> b) {
    double rr, ri;
    crecip<double>(b.re, b.im, rr, ri);
    return cmul(a, cx<double>{rr, ri});
}

template <int B>
__global__ __launch_bounds__(64) void k_decimate_circ(Sched S) {
    constexpr int G = 64 / B;
    __shared__ cx<double> s_sig[G][B];
    __shared__ cx<double> s_tw[B];           // e^{2 pi i k / B}
    __shared__ int s_live[G];
    const int lane = threadIdx.x;
    const int gi = lane / B;
    const int gsafe = gi < G ? gi : 0;
    const int q = lane - gi * B;             // mode
    if (lane < B) {
        double sn, cs;
        sincospi(2.0 * lane / B, &sn, &cs);
        s_tw[lane] = cx<double>{cs, sn};
    }
    wave_sync();
    Unit u;
    while (next_unit<G>(S, u)) {
        const JobDesc& J = S.jobs[u.job];
        const int lead = u.side;
        const bool act = (gi < G) && (gi < u.cnt);
        const int k = u.e0 + (act ? gi : 0);
        const cx<double> z = J.z[k];
        const cx<double>* m = J.lmodes[lead];
        const bool two = J.period[lead] == 2;
        const cx<double> e0 = m[0 * B + q], e1 = m[1 * B + q], v = m[2 * B + q], w = m[3 * B + q];
        const cx<double> tq = m[4 * B + q];
        const cx<double> vc{v.re, -v.im}, wc{w.re, -w.im};
        // state: period 1: e (e00), es (e11 slot); period 2: e00, e11 (== eps_s(1,1))
        cx<double> E0 = e0, E1 = two ? e1 : e0, A = w, Bm = wc;
        bool live = act;
        int it_done = S.maxit;
        for (int it = 1; it <= S.maxit; ++it) {
            if (live) {
                if (two) {
                    const cx<double> a{z.re - E0.re, z.im - E0.im}, c{z.re - E1.re, z.im - E1.im};
                    const cx<double> ac = cmul(a, c), vv{v.re * v.re + v.im * v.im, 0.0};
                    const cx<double> det{ac.re - vv.re, ac.im};
                    const cx<double> g00 = cdiv(c, det), g11 = cdiv(a, det);
                    const cx<double> g01 = cdiv(v, det), g10 = cdiv(vc, det);
                    const cx<double> dE1 = cmul(cmul(A, g00), Bm), dE0 = cmul(cmul(Bm, g11), A);
                    const cx<double> nA = cmul(cmul(A, g01), A), nB = cmul(cmul(Bm, g10), Bm);
                    E1 = cx<double>{E1.re + dE1.re, E1.im + dE1.im};
                    E0 = cx<double>{E0.re + dE0.re, E0.im + dE0.im};
                    A = nA;
                    Bm = nB;
                } else {
                    const cx<double> g = cdiv(cx<double>{1.0, 0.0}, cx<double>{z.re - E0.re, z.im - E0.im});
                    const cx<double> agb = cmul(cmul(A, g), Bm), bga = cmul(cmul(Bm, g), A);
                    E1 = cx<double>{E1.re + agb.re, E1.im + agb.im};                       // eps_s
                    E0 = cx<double>{E0.re + agb.re + bga.re, E0.im + agb.im + bga.im};    // eps
                    const cx<double> nA = cmul(cmul(A, g), A), nB = cmul(cmul(Bm, g), Bm);
                    A = nA;
                    Bm = nB;
                }
            }
            // a chain stops when all its modes are below tol
            if (q == 0 && gi < G) s_live[gi] = 0;
            wave_sync();
            if (live && !(hypot(A.re, A.im) < S.tol && hypot(Bm.re, Bm.im) < S.tol)) s_live[gsafe] = 1;
            wave_sync();
            if (live && s_live[gsafe] == 0) { live = false; it_done = it; }
            wave_sync();
            if (__all(!live)) break;
        }
        const bool converged = act && !live;
        // surface Green's function of the mode and its self-energy
        cx<double> gs;
        if (two) {
            const cx<double> a{z.re - e0.re, z.im - e0.im}, c{z.re - E1.re, z.im - E1.im};
            const cx<double> ac = cmul(a, c);
            gs = cdiv(c, cx<double>{ac.re - (v.re * v.re + v.im * v.im), ac.im});
        } else {
            gs = cdiv(cx<double>{1.0, 0.0}, cx<double>{z.re - E1.re, z.im - E1.im});
        }
        const double t2 = tq.re * tq.re + tq.im * tq.im;
        if (act) s_sig[gsafe][q] = cx<double>{t2 * gs.re, t2 * gs.im};
        wave_sync();
        if (act) {
            // c_d for d = q, then row q of Sigma: Sigma[q][j] = c_{(q - j) mod B}
            cx<double> cd{0.0, 0.0};
            for (int p = 0; p < B; ++p) {
                const cx<double> sp = s_sig[gsafe][p], tw = s_tw[(p * q) % B];
                cd.re += sp.re * tw.re - sp.im * tw.im;
                cd.im += sp.re * tw.im + sp.im * tw.re;
            }
            cd.re *= 1.0 / B;
            cd.im *= 1.0 / B;
            wave_sync();
            s_sig[gsafe][q] = cd;       // every lane has read s_sig before this write
            wave_sync();
            cx<double>* out = J.sigma + ((size_t)k * 2 + lead) * B * B + (size_t)q * B;
            for (int j = 0; j < B; ++j) out[j] = s_sig[gsafe][(q - j + B) % B];
            if (q == 0) {
                J.iters[(size_t)k * 2 + lead] = it_done;
                if (!converged) atomicOr(&J.status[k], (int)ST_NOCONV);
            }
        } else {
            wave_sync();
            wave_sync();
        }
        wave_sync();
    }
}

}  // namespace negf
