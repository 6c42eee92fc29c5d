/*
 * negf.h -- C ABI of the MI355X energy-point Green's-function engine.
 *
 * The library solves, for a batch of energy nodes, the non-equilibrium Green's
 * function problem of a block-tridiagonal tight-binding device coupled to two
 * semi-infinite leads (paper Section 2.2.1, Eq. 2-5):
 *
 *   G^R(z) = [ z I - H - diag(U) - Sigma_L(z) - Sigma_R(z) ]^{-1}          (Eq. 2)
 *   Sigma_l = tau_l g_l tau_l^H,  g_l by Sancho-Rubio decimation           (Eq. 2)
 *   Gamma_l = i (Sigma_l - Sigma_l^H),  A_l = G Gamma_l G^H                 (Eq. 3)
 *   charge_i = g_s [ -(1/pi) sum_c Im(w_c F_min(z_c) G^R_ii(z_c))
 *                   + (1/2pi) sum_r w_r (f_L A_L,ii + f_R A_R,ii)(E_r) ]  (Eq. 4)
 *   T_LR(E)  = Tr[Gamma_L G Gamma_R G^H]                                   (Eq. 5)
 *   current  = g_s (e^2/h) sum_r w_r T_LR(E_r) (f_L - f_R)(E_r)            (Eq. 5, Landauer form)
 *
 * Units: energies in eV, current in A.  `charge` is an electron count per atom
 * including spin; the paper's density is rho = -e * charge.
 *
 * Layouts: complex values are interleaved {re, im} doubles (the layout of
 * std::complex<double> and torch.complex128).  Matrices are row-major.  Atom i
 * of ring j has flat index j*b + i.
 *
 * Ownership: create/set_potential copy their inputs; callers keep their arrays.
 * Output arrays are caller-allocated.  A handle runs one solve at a time and is
 * not thread-safe; separate handles are independent.
 *
 * Errors: every call returns a negf_status; negf_last_error() gives a
 * thread-local message for the last non-OK status.  On error no output is
 * guaranteed to have been written.
 */
#ifndef NEGF_H
#define NEGF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct negf_device negf_device;
typedef struct { double re, im; } negf_c64;

typedef enum {
    NEGF_OK = 0,
    NEGF_EINVAL = -1,     /* bad size, NULL pointer, unsupported ring size  */
    NEGF_ENOMEM = -2,     /* device memory allocation failed               */
    NEGF_ENOCONV = -3,    /* decimation did not converge in decim_max_iter */
    NEGF_ESINGULAR = -4,  /* non-finite or impossible output (negative
                             spectral density, T_LR outside [0, b])      */
    NEGF_EHIP = -5,       /* HIP runtime error                             */
    NEGF_ETIMEDOUT = -6,  /* serving: the request's deadline passed         */
    NEGF_PENDING = 1      /* negf_server_poll: the request has not finished */
} negf_status;

enum { NEGF_FP64 = 0, NEGF_FP32_BULK = 1 };
enum { NEGF_LEAD_LEFT = 0, NEGF_LEAD_RIGHT = 1 };
enum { NEGF_MAX_RING = 24, NEGF_MAX_PERIOD = 2 };

/*
 * A semi-infinite lead as a periodic continuation of the ring chain, listed
 * outward from the device (lead ring 0 touches the device).  `period` rings
 * (1 or 2) form the principal layer of the decimation (Section 2.2.2).
 *   h_diag[period][b][b]  on-site blocks of the lead rings (lead potential excluded)
 *   h_up  [period][b][b]  h_up[r] = H_{ring r, ring r+1}; h_up[period-1] couples to
 *                         ring 0 of the next cell
 *   tau   [b][b]          H_{device edge ring, lead ring 0}; Sigma = tau g_00 tau^H
 * This is the paper's contact (Section 2.2.1: each contact continues the tube
 * semi-infinitely): a principal layer of one or two rings of the device's ring
 * size, coupled to the next layer only through its last ring.  A generic dense
 * layer {m, h00, h01, tau} with couplings beyond adjacent rings, or more than two
 * rings per layer, is not expressible: EINVAL for period outside [1, 2].
 */
typedef struct {
    int period;
    const negf_c64 *h_diag;
    const negf_c64 *h_up;
    const negf_c64 *tau;
} negf_lead;

typedef struct {
    int precision;            /* NEGF_FP64, or NEGF_FP32_BULK: the ring recursions of
                                 Algorithm 2 (block inversions, coupling products,
                                 recursion stores) and the contour diagonals in complex
                                 FP32 with FP32 accumulation; decimation, the lead-column
                                 propagation of Algorithm 1 and the energy sums FP64.
                                 A real-axis node whose FP32 result fails the output
                                 checks (negative spectral density, T_LR outside
                                 [0, b]) or whose lead column is large (max |G_{n,0}|,
                                 |G_{n,N-1}| times (|z| + max row sum of |H|) above 16:
                                 M is near-singular, as at a bound state) is recomputed
                                 in FP64 within the same solve; negf_fp64_nodes counts
                                 them.  ESINGULAR if they do not fit the recursion
                                 store next to the other nodes.                      */
    double eta;               /* i*eta added to real-axis nodes (device and leads)   */
    double decim_tol;         /* stop when max |alpha_ij|, |beta_ij| < decim_tol (eV) */
    int decim_max_iter;       /* NEGF_ENOCONV beyond this many doubling steps        */
    double g_s;               /* spin degeneracy (2)                                 */
    size_t workspace_bytes;   /* cap on the two recursion stores together; 0 = default
                                 (each: 30% of the free HBM when the handle is made,
                                 between 8 and 64 GiB)                               */
} negf_options;

typedef struct { double mu_L, mu_R, kT_L, kT_R; } negf_bias;

/* Optional energy-resolved outputs of negf_solve_ex (host pointers; NULL = skip). */
typedef struct {
    double   *charge;       /* [N*b]                                              */
    double   *T;            /* [n_r]    T_LR at the real-axis nodes               */
    double   *current;      /* [1]                                                */
    negf_c64 *gr_diag;      /* [n_c][N*b]  diag G^R at the contour nodes          */
    double   *al_diag;      /* [n_r][N*b]  diag A_L at the real-axis nodes        */
    double   *ar_diag;      /* [n_r][N*b]  diag A_R at the real-axis nodes        */
    int      *decim_iters;  /* [n_c+n_r][2] doubling steps taken, left and right  */
    double   *T_rl;         /* [n_r]    T_RL = Tr[Gamma_R G_{N-1,0} Gamma_L G_{N-1,0}^H]
                               (Eq. 5 with p = R, q = L; equals T_LR up to O(eta))  */
} negf_outputs;

/* Fills *opt with eta=1e-6, decim_tol=1e-12, decim_max_iter=64, g_s=2, FP64. */
void negf_default_options(negf_options *opt);

/*
 * Creates a device handle on the current HIP device and copies the Hamiltonian
 * to HBM (Eq. 2: block-tridiagonal H).
 *   n_rings >= 1, 1 <= b <= NEGF_MAX_RING
 *   h_diag [n_rings][b][b]  H_{j,j}, potential excluded
 *   h_up   [n_rings-1][b][b] H_{j,j+1}; H_{j+1,j} = h_up^H (may be NULL if n_rings == 1)
 * The potential starts at zero.  EINVAL on bad sizes/NULLs, ENOMEM, EHIP.
 */
negf_status negf_create_device(negf_device **out, int n_rings, int b,
                               const negf_c64 *h_diag, const negf_c64 *h_up,
                               const negf_lead *left, const negf_lead *right,
                               const negf_options *opt);

/* Sets the on-site potential energy: U[N*b] per atom (eV, added to H_jj's diagonal)
 * and the flat lead potentials U_left, U_right (added to the lead rings). */
negf_status negf_set_potential(negf_device *d, const double *U, double U_left, double U_right);

/* Device-pointer form of negf_set_potential; U is read on `hip_stream`. */
negf_status negf_set_potential_dev(negf_device *d, const double *U_dev, double U_left,
                                   double U_right, void *hip_stream);

/*
 * One solve over n_c contour nodes and n_r real-axis nodes (host pointers),
 * synchronous.  z_c/w_c: contour nodes and complex quadrature weights (dz Jacobian
 * included, Fermi factor NOT included: the library applies F(z - mu_min; kT_min)).
 * E_r/w_r: real nodes (i*eta added inside) and weights.  Outputs: charge[N*b],
 * T[n_r] (may be NULL), current[1] (may be NULL).
 */
negf_status negf_solve(negf_device *d, const negf_bias *bias,
                       int n_c, const negf_c64 *z_c, const negf_c64 *w_c,
                       int n_r, const double *E_r, const double *w_r,
                       double *charge, double *T, double *current);

/* negf_solve with the optional energy-resolved outputs of negf_outputs. */
negf_status negf_solve_ex(negf_device *d, const negf_bias *bias,
                          int n_c, const negf_c64 *z_c, const negf_c64 *w_c,
                          int n_r, const double *E_r, const double *w_r,
                          const negf_outputs *out);

/*
 * Asynchronous solve with every array in device memory, enqueued on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  Returns after enqueueing; the status
 * of the device-side checks (decimation convergence, finite outputs) is returned
 * by negf_sync().  T and current may be NULL.
 */
negf_status negf_solve_dev(negf_device *d, const negf_bias *bias,
                           int n_c, const negf_c64 *z_c, const negf_c64 *w_c,
                           int n_r, const double *E_r, const double *w_r,
                           double *charge, double *T, double *current, void *hip_stream);

/* Waits for the last negf_solve_dev and returns its device-side status. */
negf_status negf_sync(negf_device *d);

/*
 * Allocation-free form of negf_solve_dev, for callers that cannot allocate device
 * memory while they run (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, layouts, asynchrony and
 * results as negf_solve_dev (status through negf_sync); no hipMalloc, hipFree or
 * other allocating call is made.  Every work buffer (self-energies, per-node
 * diagonals, recursion stores, schedule tables, counters) is placed in one fixed
 * device area of negf_static_scratch_bytes() bytes (512 MiB) that the library
 * holds on each GPU it runs on until the process ends; node ranges whose
 * recursion stores do not fit next to the per-node arrays run in several chunks.
 * EINVAL, with the sizes in the message, when the per-node arrays plus one
 * node's stores exceed the area.  All calls on one GPU share the area, which
 * keeps the last call's contents: calls that overlap on one GPU (other handles,
 * other streams) race and must be serialised by the caller.
 */
negf_status negf_solve_dev_static(negf_device *d, const negf_bias *bias,
                                  int n_c, const negf_c64 *z_c, const negf_c64 *w_c,
                                  int n_r, const double *E_r, const double *w_r,
                                  double *charge, double *T, double *current, void *hip_stream);

/* Size in bytes of the fixed device area of negf_solve_dev_static. */
size_t negf_static_scratch_bytes(void);

/*
 * Lead self-energies alone (decimation, Eq. 2), host pointers, synchronous:
 * sigma[n][b][b] = Sigma_lead(z[k]), iters[n] = doubling steps (may be NULL).
 * Contour-style nodes: z is used as given (no eta is added).
 */
negf_status negf_lead_self_energy(negf_device *d, int lead, int n, const negf_c64 *z,
                                  negf_c64 *sigma, int *iters);

/* Per-kernel GPU time (ms) accumulated since the last reset when profiling is on:
 * names[k] / ms[k] for k < *count (count in: capacity, out: entries). */
negf_status negf_set_profiling(negf_device *d, int enable);
negf_status negf_kernel_times(negf_device *d, const char **names, double *ms, int *calls, int *count);

/* FP32-bulk form: real-axis nodes of the last finished solve of d (negf_solve*,
 * after negf_sync for negf_solve_dev*) that were recomputed in FP64. */
negf_status negf_fp64_nodes(negf_device *d, int *count);

/* FP32-bulk real-axis nodes recomputed in FP64: 0 (default) the nodes the output
 * checks mark, 1 every real-axis node (the result then equals the FP64 solve's on
 * those nodes, bit for bit), 2 none (the plain FP32 result, for measurements). */
negf_status negf_set_fp64_recompute(negf_device *d, int policy);

/* Device memory held by the handle and its private workspace (bytes). */
size_t negf_device_bytes(const negf_device *d);

void negf_destroy(negf_device *d);
const char *negf_last_error(void);

/* ------------------------------------------------------------ batches ----
 * Many devices' energy nodes in the same launches (one set of persistent
 * kernels per ring size and precision, longest chains first).  A job's
 * results are bit-identical to its solo solve: no arithmetic depends on which
 * other chains share a launch.  Jobs may use different ring sizes, lengths,
 * node counts, biases and precisions; all devices must live on the workspace's
 * HIP device.  The same negf_device may not appear twice in one batch only if
 * the jobs need different potentials (the potential belongs to the device).
 */
typedef struct negf_workspace negf_workspace;

typedef struct {
    negf_device *dev;          /* device (Hamiltonian, leads, potential, options)    */
    negf_bias bias;
    int n_c; const negf_c64 *z_c, *w_c;   /* contour nodes and weights                */
    int n_r; const double *E_r, *w_r;     /* real-axis nodes and weights              */
    double *charge;            /* [N*b] output                                        */
    double *T;                 /* [n_r] output or NULL                                */
    double *current;           /* [1]   output or NULL                                */
    negf_c64 *sigma_cache;     /* optional device array [n_c+n_r][2][b][b] of lead
                                  self-energies (left, right) at the job's nodes      */
    int sigma_mode;            /* 0: self-energies live in the workspace (default);
                                  1: decimate and keep them in sigma_cache;
                                  2: reuse sigma_cache, no decimation (valid while the
                                     nodes, eta and the lead potentials are unchanged,
                                     Eq. 2: Sigma depends on nothing else)            */
    /* Equilibrium density and conductance (text after Eq. 4; Eq. 6): */
    int n_poles;               /* residue nodes mu_min + i(2k+1) pi kT_min, k < n_poles,
                                  added after the contour nodes with weight
                                  -2 pi i kT_min and no Fermi factor: the poles of F
                                  enclosed between the contour and the real axis     */
    int contour_no_fermi;      /* 1: contour weights used as given (no F): the
                                  zero-temperature arc of the reference density     */
    double *conductance;       /* [1] output or NULL: g_s (e^2/h) sum_r w_r T(E_r)
                                  (-dF/dE)(E_r - mu_L; kT_L), A/V (Eq. 6)            */
    /* sigma_cache, when used, and every per-node quantity cover n_c + n_poles + n_r
       nodes in that order. */
} negf_job;

/* Workspace for batches: recursion stores, per-node arrays and the job/span
 * tables, grown on demand and kept between solves.  store_bytes caps each of the
 * two recursion stores (0 = 30% of the free HBM at creation, between 8 and 64 GiB);
 * node ranges that do not fit run in several
 * chunks.  Solves on one workspace are serialised on the device (a solve on
 * another stream waits for the previous one); the tables are uploaded only when
 * the job list changes.  Not thread-safe. */
negf_status negf_workspace_create(negf_workspace **out, size_t store_bytes);
void negf_workspace_destroy(negf_workspace *w);
size_t negf_workspace_bytes(const negf_workspace *w);
negf_status negf_workspace_set_profiling(negf_workspace *w, int enable);
negf_status negf_workspace_kernel_times(negf_workspace *w, const char **names, double *ms, int *calls, int *count);
/* Persistent workgroups launched per (resident workgroups x compute units), 1..64. */
negf_status negf_workspace_set_grid_scale(negf_workspace *w, int scale);

/* Host pointers, synchronous.  Returns the first failing job's status. */
negf_status negf_batch_solve(negf_workspace *w, int n_jobs, const negf_job *jobs);
/* Device pointers, asynchronous on hip_stream; statuses via negf_batch_sync
 * (failed_job, if not NULL, receives the index of a failed job or -1). */
negf_status negf_batch_solve_dev(negf_workspace *w, int n_jobs, const negf_job *jobs, void *hip_stream);
negf_status negf_batch_sync(negf_workspace *w, int *failed_job);
/* counts[j] = real-axis nodes of job j recomputed in FP64 in the last finished
 * batch solve (FP32-bulk jobs; 0 for FP64 jobs). */
negf_status negf_workspace_fp64_nodes(negf_workspace *w, int n_jobs, int *counts);

/* ---------------------------------------------------------- schedules ----
 * Knobs of the persistent launches; results are bit-identical for every
 * setting.  order 0 runs the longest chains first, 1 keeps the caller's order. */
typedef struct {
    int grid_scale;        /* persistent workgroups per (resident workgroups x CUs) */
    int order;
    double ms_per_solve;   /* autotuner: measured time of the chosen setting        */
    int chains_per_wave[NEGF_MAX_RING + 1];   /* autotuner: chosen chains per wavefront
                              for each ring size b of the jobs (64/b: tiles of b-lane
                              chains; 1: one wavefront per energy node); 0 for ring
                              sizes not in the jobs                                  */
} negf_schedule;

negf_status negf_workspace_set_order(negf_workspace *w, int order);
/* Chains per wavefront for the recursions, contour diagonals and lead columns of
 * ring size b: 1..64/b (a chain is one node's recursion on b lanes), 0 = 64/b. */
negf_status negf_workspace_set_chains_per_wave(negf_workspace *w, int b, int chains);
/* negf_set_fp64_recompute for the FP32-bulk jobs of a workspace's batches. */
negf_status negf_workspace_set_fp64_recompute(negf_workspace *w, int policy);
/* Basis of the lead decimation (Section 2.2.2).  1 (default): a lead whose
 * blocks and coupling are all ring-circulant (H[i][j] depends on (j - i) mod b,
 * as for a nanotube ring) is decimated in the ring Fourier basis, b scalar
 * chains per node, and Sigma is transformed back; its stopping test applies
 * decim_tol to the mode values of alpha and beta, which bound every entry, so
 * it stops at the same step as the dense test or later.  0: every lead uses
 * the dense b x b (or 2b x 2b) layer.  With ring modes Sigma is exactly
 * circulant and the lead-column kernel reads only the first row of Gamma; a job
 * that reuses a self-energy cache (sigma_mode 2) should run with the basis the
 * cache was filled with (otherwise its results move at the rounding level). */
negf_status negf_workspace_set_lead_basis(negf_workspace *w, int ring_modes);
/* Times the schedule settings on this job list (reps solves each, device
 * pointers, on hip_stream): persistent grid scale {1, 2, 4} x job order, then,
 * per ring size present, chains per wavefront {64/b, half of that, 1}; keeps the
 * fastest in w and returns it in *best. */
negf_status negf_workspace_autotune(negf_workspace *w, int n_jobs, const negf_job *jobs, void *hip_stream,
                                    int reps, negf_schedule *best);

/* ------------------------------------------------------------- graphs ----
 * A batch solve recorded once into a HIP graph and replayed with one launch.
 * The graph owns a private workspace (store_bytes as in negf_workspace_create)
 * and fixes the job list: device handles, biases, node counts and every
 * pointer.  The contents behind the pointers may change between launches: a
 * replay sees new potentials (negf_set_potential*), energy nodes and weights.
 * The devices must outlive the graph.  hip_stream must be a created stream
 * (capture is not possible on the null stream); creation runs one eager solve.
 * Replays on one graph are serialised on the device; statuses via
 * negf_graph_sync as in negf_batch_sync. */
typedef struct negf_graph negf_graph;
negf_status negf_graph_create(negf_graph **out, int n_jobs, const negf_job *jobs, size_t store_bytes,
                              void *hip_stream);
negf_status negf_graph_launch(negf_graph *g, void *hip_stream);
negf_status negf_graph_sync(negf_graph *g, int *failed_job);
void negf_graph_destroy(negf_graph *g);

/* ------------------------------------------------ semi-adaptive grid ----
 * Section 3.3 (number of integration points): the real-axis window [E_min, E_max]
 * (Eq. 4, f1 = f2 = 14) is split at E_l1 < E_l2 into three parts, each integrated
 * by Gauss-Legendre with density[p] nodes per kT_min (at least one node).  The
 * integrand f_L A_L + f_R A_R summed over the atoms of ring N/2 is evaluated on
 * the grid of the guessed limits by a real-axis solve of d (at its current
 * potential), its peak E_s located, and the limits refined as
 *     E_l1 <- E_l1 - a kT_min,  E_l2 <- E_s + b kT_min
 * (clipped to the window and kept ordered; the paper uses a = 3, b = 1).  The
 * refined grid is written to E_r/w_r (host arrays of capacity cap); *n_r always
 * receives its size and limits[3] (if not NULL) = {E_l1, E_l2, E_s}.  EINVAL if
 * cap is too small (call again with *n_r). */
negf_status negf_semi_adaptive_grid(negf_device *d, const negf_bias *bias, double E_l1, double E_l2,
                                    double a, double b, const double *density,
                                    double *E_r, double *w_r, int cap, int *n_r, double *limits);

/* --------------------------------------------------------- mode space ----
 * Section 2.2.2 (blocks as scalars or arrays of modes): a tube in the mode-space representation, one
 * scalar chain per ring mode.  Every ring block (h_diag, h_up, lead blocks, tau)
 * must be circulant, H[i][j] = H[0][(j - i) mod b], and the potential uniform on
 * each ring; then mode q sees the scalar lambda_q(C) = sum_k C[0][k] e^{2 pi i qk/b}
 * of every block C and the b modes decouple exactly.  n_modes = 0 keeps all b
 * modes (exact); otherwise modes[n_modes] lists the kept ones (the mode-space
 * approximation: charge and current of those modes only).  A solve runs the kept
 * modes as one batch on workspace w; per-atom charge is (1/b) sum_q charge_q of
 * the atom's ring, T and current add over modes.  EINVAL if a block is not
 * circulant.  Host pointers, synchronous. */
typedef struct negf_modes negf_modes;
negf_status negf_modes_create(negf_modes **out, int n_rings, int b, const negf_c64 *h_diag, const negf_c64 *h_up,
                              const negf_lead *left, const negf_lead *right, const negf_options *opt,
                              int n_modes, const int *modes);
/* U_ring[n_rings]: on-site potential energy of every atom of ring j (eV). */
negf_status negf_modes_set_potential(negf_modes *m, const double *U_ring, double U_left, double U_right);
negf_status negf_modes_solve(negf_modes *m, negf_workspace *w, const negf_bias *bias,
                             int n_c, const negf_c64 *z_c, const negf_c64 *w_c,
                             int n_r, const double *E_r, const double *w_r,
                             double *charge, double *T, double *current);
void negf_modes_destroy(negf_modes *m);

/* ------------------------------------------------------------ serving ----
 * Self-consistent bias points (Section 2.3, Algorithm 3) served with continuous
 * batching.  A request is a device with flat leads, a bias point and an energy
 * grid (fixed, or semi-adaptive and rebuilt as the potential moves).  The server
 * iterates
 *     rho_in -> Poisson -> U -> NEGF (batched with every running request) -> rho_out
 *     -> Broyden's modified second method on rho (per-ring electron counts)
 * until the stopping norm (request field norm) falls below tol, starting from
 * rho_in = n_ref.  Electrostatics: per ring j, potential phi_j (V),
 *     -(eps_1d/dz^2)(phi_{j+1} - 2 phi_j + phi_{j-1}) + c_gate (phi_j - V_GS)
 *         = -e (rho_j - n_ref_j)/dz,   phi_{-1} = 0 (source), phi_N = V_DS (drain),
 * and the electron potential energy U_j = -phi_j eV on every atom of ring j.  The
 * source lead sits at U = 0 and level mu_S, the drain lead at U = -V_DS and level
 * mu_S - V_DS, both at temperature kT.  Lead self-energies are decimated once per
 * grid and reused on every pass until the grid is rebuilt.  Since U is uniform on
 * each ring, a ring-circulant tube (every zigzag tube) runs in mode space by
 * default: b scalar chains per energy, exact, at O(b N) instead of O(b^3 N) per
 * node.  A request's results do not depend on the other requests that share its
 * passes.
 *
 * Admission: first come first served while the estimated HBM footprint of the
 * running requests fits hbm_budget minus the two recursion stores
 * (2 x store_bytes, 0 = the workspace default each); at most max_inflight run at once.  A request
 * whose footprint alone exceeds the budget is refused at submission (ENOMEM).
 * Submission copies every array.  The server's thread owns the GPU work on the
 * device that was current at creation; all calls are thread-safe.
 */
typedef struct negf_server negf_server;

typedef struct {
    int n_rings, b;                       /* as negf_create_device (n_rings >= 2)       */
    const negf_c64 *h_diag, *h_up;
    const negf_lead *left, *right;
    negf_options opt;                     /* precision, eta, decimation, g_s            */
    double mu_S, kT, V_DS, V_GS;          /* eV, eV, V, V                               */
    int n_c; const negf_c64 *z_c, *w_c;   /* energy grid as in negf_solve               */
    int n_r; const double *E_r, *w_r;
    double dz;                            /* ring spacing (m)                           */
    double eps_1d;                        /* axial permittivity x area (F m)            */
    double c_gate;                        /* gate capacitance per length (F/m)          */
    const double *n_ref;                  /* [n_rings] electrons per ring when neutral  */
    double zeta, tol;                     /* Broyden fraction; stopping norm            */
    int history, max_iter;                /* stored Broyden columns (<= 32); pass limit */
    int basis;              /* 0: mode space (Section 2.2.2, exact: every mode kept) when every
                               device and lead block is ring-circulant, else real space;
                               1: real space always                                          */
    int norm;               /* stopping norm compared with tol:
                               0: max_j |rho_in_j - rho_out_j| / (rho_in_j + rho_out_j)
                                  (Algorithm 3);
                               1: max_j |phi(rho_out)_j - phi(rho_in)_j| in eV (per electron),
                                  the change of the potential that the output charge implies
                                  (the linear Poisson operator with zero boundary values on
                                  rho_in - rho_out)                                         */
    double grid_density[3]; /* all 0: the fixed real-axis grid E_r/w_r.  All > 0: the
                               semi-adaptive grid (Section 3.3; see negf_semi_adaptive_grid)
                               with these densities (nodes per kT) in its three parts,
                               rebuilt at the request's current potential before NEGF pass
                               1, 1 + grid_refresh, 1 + 2 grid_refresh, ...; E_r/w_r and n_r
                               are then ignored                                              */
    double grid_l1, grid_l2;  /* guessed part limits of every rebuild (eV)                  */
    double grid_a, grid_b;    /* refinement E_l1 - a kT, E_s + b kT (the paper: 3, 1)       */
    int grid_refresh;         /* passes between rebuilds; 0 = 50                            */
    const double *rho_init;   /* [n_rings] starting per-ring electron counts, e.g. the
                                 converged rho of a neighbouring bias point (Section 3.3:
                                 each bias point starts from the previous one); NULL: n_ref */
    double deadline_ms;       /* > 0: the request ends with NEGF_ETIMEDOUT when it has not
                                 finished this long after submission (queued or running;
                                 a running one returns its last pass's charge and U)      */
} negf_sc_request;

typedef struct {
    int status;          /* NEGF_OK: converged; NEGF_ENOCONV: pass limit or decimation;
                            NEGF_ETIMEDOUT: deadline; other: solve or HIP error            */
    int iterations;      /* NEGF passes taken                                              */
    double eps_max;      /* stopping norm of the last pass                                 */
    double current;      /* A, at the last potential                                       */
    double t_queue_ms, t_run_ms, t_total_ms;   /* submit->admit, admit->done, submit->done */
    int n_r;             /* real-axis nodes of the last pass                               */
    int mode_space;      /* 1: the request ran as b scalar mode chains                     */
    int evictions;       /* times the request was evicted to host state and re-admitted   */
} negf_sc_result;

typedef struct {
    int pending, running;
    long long passes;
    size_t hbm_used, hbm_budget, workspace_bytes;
} negf_server_info;

negf_status negf_server_create(negf_server **out, size_t hbm_budget, int max_inflight, size_t store_bytes);
negf_status negf_server_submit(negf_server *s, const negf_sc_request *req, long long *id);
/* Result of request id; wait = 0 returns NEGF_PENDING while it runs.  On NEGF_OK the
 * request is released: charge[N*b] (per atom), U[N*b] (final potential energy) and
 * eps_trace[iterations] (stopping norm of every pass, capacity max_iter) are filled
 * when not NULL. */
negf_status negf_server_poll(negf_server *s, long long id, int wait, negf_sc_result *res,
                             double *charge, double *U, double *eps_trace);
/* Queue and memory counters; returns the last fatal status of the server thread. */
negf_status negf_server_stats(negf_server *s, negf_server_info *info);
/* Eviction to host state and re-admission.  A running request can be evicted between
 * passes: its mixing state (rho_in, the previous rho_in and f, s, the stored Broyden
 * columns, pass counters), its current real-axis grid and its trace are copied to
 * host memory, its device memory and slot are freed, and it is queued again at the
 * back; when re-admitted it resumes from that state (the potential is rebuilt from
 * rho_in, self-energies are decimated again), so its results are bit-identical to an
 * uninterrupted run.  negf_server_evict(s, id) asks for one eviction at the end of the
 * request's next pass (the current one if it is running; its first one after admission
 * if it is queued); EINVAL if the request is unknown or has finished.  negf_server_set_time_slice(s, passes) makes the server
 * evict, whenever requests are waiting for admission, every running request that has
 * run `passes` passes since it was (re)admitted (0 = never, the default): round-robin
 * service under overload. */
negf_status negf_server_evict(negf_server *s, long long id);
negf_status negf_server_set_time_slice(negf_server *s, int passes);
/* Stops admitting, finishes the running requests, cancels the queued ones, frees all. */
void negf_server_destroy(negf_server *s);

#ifdef __cplusplus
}
#endif
#endif /* NEGF_H */
