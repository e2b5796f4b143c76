/*
 * spmps.h -- C ABI of the spin-projected MPS (SP-MPS) hot path on one
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Li & Chan, "Spin-projected matrix product states" (SP-MPS).  The
 * underlying MPS has definite particle number N and spin projection M
 * (Sec. 2.2, Eq. [SPMPS2]).  The energy functional is
 *     E = <Psi| H P |Psi> / <Psi| P |Psi>                  (Eq. [efunctional])
 * with the projector written as a Gauss-Legendre sum over rotation angles
 *     P = sum_g coef_g exp(-i beta_g S_y),
 *     coef_g = (2S+1)/2 w_g d^S_MM(beta_g),  x_g = cos(beta_g)
 * (Eqs. [PSMM], [pmpo]); exp(-i beta S_y) is a product of 4x4 local
 * rotations (Eq. [expSy]).  A one-site sweep solves at each site the local
 * generalised eigenproblem H_eff x = E N_eff x (Eqs. [spmpsopt],
 * [geproblem]) and restores the canonical form (Sec. 2.3).
 *
 * Conventions
 *   - Sites k = 1..L are spatial orbitals, local basis sigma = 2 n_a + n_b,
 *     i.e. (|0>, |b>, |a>, |ab>) with |ab> = a+_alpha a+_beta |0>.
 *   - Bond k (0..L) lies right of site k; its sectors q = (N, 2M) count the
 *     particles and twice the spin projection of sites 1..k, sorted by
 *     (N, 2M).  Bond 0 is (0,0) of dimension 1, bond L is (N, 2M) of
 *     dimension 1.
 *   - A site tensor is packed as blocks, one per (left sector a, sigma)
 *     whose right sector a + q_sigma exists, ordered by a then sigma, each
 *     a dense dim(a) x dim(b) row-major matrix.  The packed vector of a site
 *     is what H_eff acts on.
 *   - All device pointers are HIP device memory on the device that was
 *     current at sp_init_mps; all work is ordered on the stream given there.
 *
 * Errors: every call returns an int status; 0 = SP_OK, > 0 = warning, < 0 =
 * error.  sp_last_error() gives a message for the calling thread.
 */
#ifndef SPMPS_H
#define SPMPS_H

#ifdef __cplusplus
extern "C" {
#endif

#define SP_OK 0
#define SP_ENOCONV 1      /* warning: a local solve stopped at max_iter        */
#define SP_WINEXACT 2     /* warning: G below the exact point count             */
#define SP_EINVAL (-1)    /* invalid argument (shape, parity, range, layout)    */
#define SP_ENORM (-2)     /* projected norm <Psi|P|Psi> vanishes (< 1e-12)      */
#define SP_EHIP (-3)      /* HIP runtime error                                  */
#define SP_ENOMEM (-4)    /* device allocation failed                           */
#define SP_ESTATE (-5)    /* environments needed by the call are not built      */
#define SP_ENAN (-6)      /* NaN or Inf met in a local solve                    */

#define SP_FP64 0         /* every contraction in FP64 */
#define SP_FP32 1         /* the H_eff x / N_eff x products inside the local
                             solves use FP32 copies of the environments,
                             FP32 tiles and FP32 accumulation (tiled path
                             only); environment updates, the Davidson
                             orthogonalisation and subspace solve, and a
                             final FP64 Rayleigh quotient per site step
                             (the reported energy) stay FP64           */
#define SP_BF16X3 2       /* as SP_FP32, and the LDS-tiled block products of
                             sites too wide for the fused kernel run in
                             split BF16 on the matrix cores: each operand
                             value v ~ hi + lo (two bf16, round to nearest
                             even), three products hi hi + hi lo + lo hi
                             with FP32 accumulation (relative error of
                             order 1e-5); values must lie in FP32 range  */

#define SP_SOLVER_AUTO 0    /* sp_sweep_opts.solver */
#define SP_SOLVER_HOST 1
#define SP_SOLVER_DEVICE 2

#define SP_PATH_TILED 0   /* environment updates as LDS-tiled block products
                             over particle-number blocks (FP64 matrix
                             cores); H_eff x per site either in one fused
                             launch with per-g partial outputs, or as block
                             products from the left environment with the
                             rotated MPO mixed in (formed once per L[site-1])
                             - the latter where a particle-number block is
                             too wide for the fused kernel's LDS, where the
                             fused plan has one row per task, or where
                             sp_autotune / sp_set_heff_plan choose it.  The
                             block products are FP64 in SP_FP64 and SP_FP32
                             and split BF16 in SP_BF16X3                  */
#define SP_PATH_PLAIN 1   /* one work-group per (N, M) block product, the
                             plain FP64 reference path                      */

typedef struct sp_handle sp_handle;
typedef struct sp_mlp sp_mlp;

/* Problem: L sites, d must be 4, N electrons, spin S = twoS/2 with projection
 * M = twoM/2, G quadrature points.  Requires N + twoS even, N + twoM even,
 * |twoM| <= twoS <= Omega_max (largest seniority, Eq. [exactQuadrature]),
 * G >= 1.  G below ceil((Omega_max/2 + S + 1)/2) is allowed and makes the
 * projector approximate (warning SP_WINEXACT). */
typedef struct sp_problem {
    int L;
    int d;
    int N;
    int twoS;
    int twoM;
    int G;
    int precision; /* SP_FP64, SP_FP32 or SP_BF16X3 */
    int path;      /* SP_PATH_TILED or SP_PATH_PLAIN: same results to rounding */
} sp_problem;

/* MPO in the operator-valued-matrix form of Sec. 2.1, Eq. [FSMPO]:
 * w[k] (k = 0..L) are the bond dimensions with w[0] = w[L] = 1; site k
 * (1..L) holds w[k-1]*w[k]*16 doubles, element ((a*w[k] + b)*4 + s)*4 + t
 * = <s| O_ab |t>.  Channel 0 of every inner bond must be the left identity
 * string (W[k]_{a,0} = delta_{a,0} I for k < L) and the last channel the
 * right identity string (W[k]_{w[k-1]-1, b} = delta_{b, w[k]-1} I for
 * k > 1), the triangular form of Eq. [Sfac]; every operator entry must
 * change the particle number consistently.  Host memory, copied. */
typedef struct sp_mpo {
    const int* w;
    const double* data;
} sp_mpo;

/* Bond sectors: nsec[k] sectors for bond k = 0..L; sec_n, sec_2m, sec_dim
 * concatenated over bonds, each bond sorted by (N, 2M).  Host memory,
 * copied.  Every sector must be reachable through one site from both
 * neighbouring bonds with at least as many states as it holds. */
typedef struct sp_block_table {
    const int* nsec;
    const int* sec_n;
    const int* sec_2m;
    const int* sec_dim;
} sp_block_table;

/* Local solver settings (the paper leaves the solver open; Davidson with a
 * Euclidean-orthonormal search space, canonical orthogonalisation of the
 * projected metric, a diagonal preconditioner and restarts). */
typedef struct sp_sweep_opts {
    int n_sweeps;     /* full sweeps: right-moving 1..L-1, then left L..2   */
    double tol;       /* residual 2-norm for a unit-norm site tensor        */
    int max_iter;     /* Ritz evaluations per local solve                   */
    int max_sub;      /* search-space size that triggers a restart          */
    int keep;         /* Ritz vectors kept at a restart                     */
    int solver;       /* where the Davidson iteration is driven:
                         SP_SOLVER_HOST: the FP64 subspace solve on a host
                         core between the device passes (one round trip
                         per iteration); SP_SOLVER_DEVICE: device resident
                         - the FP64 subspace solve in one work-group per
                         state, every iteration of all states replayed from
                         one HIP graph, no host decision inside a local
                         solve (tiled path, max_sub <= 47, keep <= 16, no
                         constraint or learned model; otherwise the host
                         driver runs); SP_SOLVER_AUTO (0): device resident
                         for two or more states, host for one state (a
                         single work-group solve is slower than a host core,
                         in a batch the states' solves run side by side).
                         The same algorithm either way; results agree to
                         rounding                                          */
    int verbose;      /* nonzero: one line per finished site step on stderr
                         (state, sweep, site, direction, energy, matvecs,
                         wall time)                                        */
} sp_sweep_opts;

typedef struct sp_step_report {
    int sweep, site, dir, iters, converged, matvecs;
    double theta;     /* local eigenvalue = projected energy after the step */
    double pnorm;     /* x^T N_eff x for the unit-norm site tensor          */
    double rnorm;     /* final residual norm                                */
    double usec;      /* wall time of the step                              */
} sp_step_report;

/* Caller-owned host array of `capacity` steps; n_steps is set. */
typedef struct sp_sweep_report {
    int capacity;
    int n_steps;
    sp_step_report* steps;
} sp_sweep_report;

/* Build the state: quadrature table (Eq. [pmpo]), rotated MPO W[k] r(beta_g)
 * for every g (Eq. [expSy]), device copies of the MPS blocks
 * (`init_blocks`: host, packed, all sites concatenated), right-canonical
 * form of sites L..2 by positive-diagonal LQ per left sector, and the right
 * environments of every quadrature point.  `hip_stream` is a hipStream_t
 * (NULL = default stream).  On success *out owns all device memory. */
int sp_init_mps(const sp_problem* p, const sp_mpo* W, const sp_block_table* bonds,
                const double* init_blocks, void* hip_stream, sp_handle** out);

/* Environments (Fig. [spmpsOpt]): dir = +1 builds the left environments
 * L_g[site] (sites 1..site) from L_g[site-1] and the current site tensor,
 * for every g; dir = -1 builds R_g[site] (sites site..L) from R_g[site+1].
 * site in 1..L.  SP_ESTATE if the input environment was never built.
 * An interior bond (1..L-1) stores its left and right environments in one
 * device buffer, as a sweep never needs both at once: building L[k] marks
 * R[k] as not built and building R[k] marks L[k] as not built, so a later
 * call that needs the retired one returns SP_ESTATE until it is rebuilt. */
int sp_env_update(sp_handle* h, int site, int dir);

/* y = H_eff x and ny = N_eff x at `site` (Eq. [geproblem]) with the current
 * environments L_g[site-1], R_g[site+1]:
 *   y  = P_NM sum_g coef_g L_g (W[site] r_g) x R_g
 *   ny = P_NM sum_g coef_g L_g^I r_g x R_g^I
 * where the identity-channel environments give N_eff and P_NM keeps the
 * (N, M) blocks of the packed layout.  x, y, ny: caller-owned device arrays
 * of sp_site_size(site) doubles; y and ny must not alias x or each other.
 * Asynchronous on the handle's stream. */
int sp_heff_apply(sp_handle* h, int site, const double* x, double* y, double* ny);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * y = H_eff x and ny = N_eff x as sp_heff_apply (same kernels, the same
 * bits), with the per-quadrature-point partial outputs held in a fixed
 * device array of the library (2 x 2^21 doubles, 32 MiB per device, kept
 * until the process ends) instead of the handle's buffers.  The call
 * allocates nothing.  Tiled path only (SP_EINVAL otherwise); SP_EINVAL when
 * the site needs more than 2^21 partial slots per output (G x site size on
 * a fused site, G x the channel split x site size on the block products).
 * Every handle on one GPU shares that GPU's array: calls that overlap on one
 * GPU (on different streams, or from several threads) race and must be
 * ordered by the caller.  Its contents after a call are undefined. */
int sp_heff_apply_noalloc(sp_handle* h, int site, const double* x, double* y, double* ny);

/* Diagonals of H_eff and N_eff at `site` (device arrays, site size). */
int sp_heff_diag(sp_handle* h, int site, double* dh, double* dn);

/* One-site sweeps (Sec. 2.3) from the current state, which must have its
 * canonical centre at site 1 (as after sp_init_mps or a completed sweep).
 * Each step solves the local problem, moves the centre with a
 * positive-diagonal QR (right-moving) or LQ (left-moving) per sector and
 * updates the environments of all g.  Returns SP_ENOCONV if any local
 * solve stopped at max_iter.  `r` may be NULL. */
int sp_sweep(sp_handle* h, const sp_sweep_opts* o, sp_sweep_report* r);

/* Sweeps of n states together (each as sp_sweep would run them, same
 * results to rounding): every round advances each unfinished state by one
 * site step; the Davidson iterations of the states run in lockstep, with one
 * fused H_eff launch (per row count) covering every state and quadrature
 * point, batched Davidson passes, and the subspace solves on host threads.
 * All handles: tiled path, one precision, one device and one stream,
 * centre at site 1, each listed once.  Sites without a fused plan run their
 * tiled products per state in the same round.  r: n reports (or NULL).  The ability to
 * run many states at once follows the paper's use of several
 * broken-symmetry starting guesses (Sec. 3). */
int sp_sweep_batch(sp_handle** hs, int n, const sp_sweep_opts* o, sp_sweep_report* r);

/* Autotuner of the H_eff plans (tiled path): for every site, time `reps`
 * applications of the fused kernel for each LDS budget of the work-group
 * (36, 72, 108 and 144 KB, which set the rows per task) and of the LDS-tiled
 * block products, and keep the fastest.  The products are the same to
 * rounding whatever the choice.  Optional outputs (L entries each): the
 * budget in doubles (0: block products), the rows per task (0: block
 * products) and the time per application in microseconds.  Synchronises. */
int sp_autotune(sp_handle* h, int reps, int* budget_out, int* rows_out, double* usec_out);

/* Current H_eff plan of a site: rows per task of the fused kernel and its
 * LDS in doubles, or 0 and 0 (plain path, or a tiled-path site that runs the
 * tiled block products).  Host only. */
int sp_heff_plan(const sp_handle* h, int site, int* rows, int* lds_doubles);

/* Choose the H_eff plan of one site (tiled path): the fused kernel with an
 * LDS budget of `lds_budget` doubles per work-group (1..18432; it sets the
 * rows per task), or 0 for the LDS-tiled block products.  A budget that no
 * particle-number block of the site fits also selects the tiled products.
 * *rows (optional) receives the rows per task, 0 for the tiled products.
 * The products are the same to rounding either way.  Synchronises. */
int sp_set_heff_plan(sp_handle* h, int site, int lds_budget, int* rows);

/* Excited states (Sec. 2.3, Eq. [orthoB]): later sp_sweep calls on h keep
 * h's state orthogonal to `lower` in the projected metric,
 * <lower|P|h> = 0.  At every site step the vectors B[k] = d<lower|P|h>/dA[k]
 * of all constraints are built from environments of <h|R(beta_g)|lower>
 * (this state on the bra side), orthonormalised in the order the
 * constraints were added (a vector dependent on the earlier ones to 1e-10
 * is skipped), and the local solve runs on (Q H_eff Q, Q N_eff Q) with
 * Q = 1 - C C^T: start vector, products and corrections are projected.
 * `lower`'s tensors are copied at this call (later changes to `lower` are
 * not seen); it must have the same L, N, S, M, G, block table and device.
 * h's centre must be at site 1 (as after sp_init_mps or a full sweep); at
 * most 8 constraints.  sp_set_site on h invalidates the constraint
 * environments until the next sp_add_orthogonality.  States with
 * constraints cannot go through sp_sweep_batch. */
int sp_add_orthogonality(sp_handle* h, sp_handle* lower);
/* Remove every orthogonality constraint of h. */
int sp_clear_orthogonality(sp_handle* h);
/* out[j] = <lower_j|P|h> / (|lower_j| |h|) for the current site tensors
 * (host, one double per constraint, in the order added), from the
 * environments at the canonical centre.  Synchronises. */
int sp_orthogonality_overlaps(sp_handle* h, double* out);

/* Learned Davidson preconditioner.  The paper leaves the local solver of
 * Sec. 2.3 open; the library's Davidson corrects with the diagonal rule
 * t = -r / (diag H_eff - theta diag N_eff) (floored at 1e-8).  A model
 * replaces it by a two-layer perceptron (hidden width H <= 256, ReLU)
 * applied to each element of the site tensor separately, on the features
 * f0 = |r_i| / rms(r), f1 = asinh(d_i), f2 = asinh(dN_i),
 * f3 = asinh(-f0/d_i'), f4 = sign(r_i) t_i / rms(t) (d = dH - theta dN,
 * d' = d floored, t = -r / d' the diagonal correction), with
 * t_i = sign(r_i) g(f) (odd in r; Davidson normalises t).  While a model
 * is in use, a local solve falls back to the diagonal rule for good once
 * its residual norm has missed a new minimum three iterations in a row or
 * has fallen by less than a factor of two over the last four iterations.
 * Training pairs come from the solver: for iteration
 * j of a converged solve with Ritz vector x_j and final vector x_f, the
 * target of g at element i is sign(r_i) e_i / rms(e),
 * e = x_f / (xh_j . x_f) - xh_j (xh_j =
 * x_j / |x_j|): the step that puts x_f in the search space.  Weights and
 * pairs are FP32 in device memory, arithmetic FP64; Adam (beta 0.9, 0.999,
 * eps 1e-8) on the mean squared error.  A model belongs to the device that
 * was current at sp_mlp_create; it must outlive every state that uses it. */

#define SP_MLP_VECTOR 0  /* root mean squares over the whole site vector   */
#define SP_MLP_NBLOCK 1  /* per N-block: see sp_mlp_set_scope            */

/* w_init: mlp_size(H) = 7H + 1 floats, packed W1 (H x 5 row-major) | b1 (H)
 * | w2 (H) | b2 (host, copied); capacity: rows (elements) of training
 * pairs the model can record (0: none). */
int sp_mlp_create(int hidden, const float* w_init, long long capacity, sp_mlp** out);
/* Scope of the model (default SP_MLP_VECTOR).  SP_MLP_NBLOCK: the model
 * sees the residual restricted to one N-block of the site tensor (the
 * elements that share the particle numbers of both bonds, whatever their
 * M; Sec. 2.3 solves in these blocks after the subduction to N-only
 * symmetry): rms(r) and rms(t) in f0 and f4 are taken over the element's
 * block, the correction is sign(r_i) g(f) rms_block(t), so the model shapes
 * the correction inside each block while the diagonal rule keeps the
 * weight of the block, and the targets divide e by its rms over the
 * element's block.  Set it before the model records or is used: a model
 * holding training pairs of the other scope is refused (SP_EINVAL), as are
 * a model in use and a recording one of different scopes (sp_set_precond). */
int sp_mlp_set_scope(sp_mlp* m, int scope);
int sp_mlp_destroy(sp_mlp* m);
/* Current weights (host, 7H + 1 floats; may be NULL) and recorded rows. */
int sp_mlp_get(sp_mlp* m, float* w_out, long long* rows);
/* Recorded pairs [first, first + count): features (count x 5) and targets
 * (host). */
int sp_mlp_dataset(sp_mlp* m, long long first, long long count, float* F_out, float* Y_out);
/* y = model(F) for n feature rows (device pointers, FP32) on `stream`
 * (a hipStream_t, NULL = default). */
int sp_mlp_forward(sp_mlp* m, const float* F, long long n, float* y, void* stream);
/* One Adam step on the n pairs (F, Y) (device pointers); *loss (optional)
 * = 0.5 mean (y - Y)^2 before the step.  Synchronises. */
int sp_mlp_train_step(sp_mlp* m, const float* F, const float* Y, long long n, double lr, double* loss, void* stream);
/* `epochs` passes over the recorded pairs in ceil(rows / batch) batches
 * (at most 4096; batch b holds rows b, b + nb, b + 2 nb, ...), one Adam
 * step per batch; loss_out[e] (optional) = the mean batch loss of epoch e.
 * Synchronises. */
int sp_mlp_train(sp_mlp* m, int epochs, long long batch, double lr, double* loss_out, void* stream);
/* Local solves of later sp_sweep calls on h correct with `use` (NULL: the
 * diagonal rule) and record their training pairs into `record` (NULL:
 * none) until its capacity is reached.  States with a model cannot go
 * through sp_sweep_batch. */
int sp_set_precond(sp_handle* h, sp_mlp* use, sp_mlp* record);

/* Projected energy and norm at the canonical centre:
 * E = <x|H_eff x>/<x|N_eff x>, normP = <x|N_eff x> (the spin-S weight of
 * the underlying MPS when it is normalised).  Host scalars; synchronises. */
int sp_energy(sp_handle* h, double* E, double* normP);

/* Release all device memory of the handle. */
int sp_destroy(sp_handle* h);

/* Packed size (doubles) of a site. */
int sp_site_size(const sp_handle* h, int site, long long* n);

/* Copy a site tensor to / from host memory (packed layout).  sp_set_site
 * leaves the environments untouched. */
int sp_get_site(sp_handle* h, int site, double* host);
int sp_set_site(sp_handle* h, int site, const double* host);

/* Current canonical centre (1..L). */
int sp_center(const sp_handle* h, int* site);

/* Algorithmic flops of one sp_heff_apply at `site`: 2 m n k per block
 * product of the minimal-work contraction order over non-zero blocks only
 * (L_g x, the W r mixing, then R_g, for both H_eff and N_eff). */
int sp_heff_flops(const sp_handle* h, int site, double* flops);

/* Timing of the phases of sp_heff_apply at `site`, each averaged over
 * `reps` launches.  Plain path: left product, W r mixing, right product.
 * Tiled path: the fused launch (left product, mixing and right product in
 * one kernel) or, at a site without a fused plan, the tiled block-product
 * lists; then the pre-mixing of the left environment that the block
 * products build once per local problem (timed once, before the products,
 * and not part of their time; 0 at a fused site); then the g sum.  Phases
 * are timed with HIP events on the handle's stream.  out[0..2]: mean
 * milliseconds per launch; out[3..5]: algorithmic flops per launch (tiled
 * path: the product, the pre-mixing's scaled adds, the g sum);
 * out[6..8]: algorithmic bytes per launch (every array read or written once:
 * environments, site vector, intermediates, outputs).  x, y, ny as in
 * sp_heff_apply.  Synchronises. */
int sp_heff_profile(sp_handle* h, int site, int reps, const double* x, double* y, double* ny, double* out);

/* Timing of one batched fused H_eff launch (as sp_sweep_batch issues it):
 * every state i at site sites[i] (tiled path, fused plan, environments
 * built), all quadrature points, x = the site tensors themselves; per-g
 * partial outputs land in each state's scratch.  out[0]: mean microseconds
 * over `reps` launches (HIP events on the states' stream), out[1]: summed
 * algorithmic flops, out[2]: summed algorithmic bytes (environments and x
 * read once, partials written), out[3]: work-groups per launch, out[4]:
 * mean microseconds per replay of the same launches captured once in a HIP
 * graph (replayed on a private stream), out[5]: largest difference between
 * the partials of three checked replays (each after eager work that clears
 * them) and those of an eager launch (0 when the replays are exact).  All
 * states on one device, stream and precision, each listed once; out holds
 * 6 doubles.  Synchronises. */
int sp_heff_batch_profile(sp_handle** hs, int n, const int* sites, int reps, double* out);

/* Message of the last error on this thread. */
const char* sp_last_error(void);

/* ---- host-only helpers (no GPU needed) ----------------------------------- */

/* Quadrature of Eq. [pmpo] with the (2S+1)/2 factor of Eq. [PSMM]: nodes x
 * ascending (Newton on the Legendre polynomial), weights w, and
 * coef_g = (2S+1)/2 w_g d^S_MM(arccos x_g).  Arrays of G doubles. */
int sp_quadrature(int G, int twoS, int twoM, double* x, double* w, double* coef);

/* Exact point count ceil((Omega_max/2 + S + 1)/2), Eq. [exactQuadrature]. */
int sp_exact_points(int N, int K, int twoS, int twoM);

/* MPO builders in the layout of sp_mpo.  Call with data == NULL to get the
 * bond dimensions in w (L+1 ints) and the element count in *n; then again
 * with data of that size.  Hubbard: open chain, hopping t, on-site U,
 * bond dimension 6.  S2: total spin squared, bond dimension 5 (Eq. [Sfac]).
 * Identity: bond dimension 1. */
int sp_mpo_hubbard(int L, double t, double U, int* w, double* data, long long* n);
int sp_mpo_s2(int L, int* w, double* data, long long* n);
int sp_mpo_identity(int L, int* w, double* data, long long* n);

/* Spin-free property operators (Sec. 2.4), same layout: a single-site
 * operator op (16 doubles, <s|op|t> at s*4+t) at site p; E_pq =
 * sum_sigma a+_{p sigma} a_{q sigma} (the spin-free one-body density
 * operator; E_pp = n_p), bond dimension 4; S_X . S_Y, bond dimension 5
 * (X == Y: the local S^2).  Sites are 1-based. */
int sp_mpo_site_op(int L, int p, const double* op, int* w, double* data, long long* n);
int sp_mpo_epq(int L, int p, int q, int* w, double* data, long long* n);
int sp_mpo_spin_corr(int L, int X, int Y, int* w, double* data, long long* n);

/* The ab-initio Hamiltonian of Eq. [sqH] for K real orbitals (Sec. 2.1):
 * H = sum_pq h_pq sum_s a+_ps a_qs + 1/2 sum_pqrs (pq|rs) sum_st a+_ps a+_rt
 * a_st a_qs, chemists' notation, no core energy.  h: K*K row-major; eri:
 * K^4 with (pq|rs) at ((p*K + q)*K + r)*K + s (host memory, read only; no
 * symmetry is assumed or enforced).  Output as for the builders above
 * (w: K+1 ints; data == NULL returns the sizes only; the terms are
 * enumerated on every call).  The bond dimension is O(K^2): every channel
 * holds a partial product with at most two fermion operators named on one
 * side of the bond.  SP_EINVAL if K is outside 2..64 or a bond would need
 * more than 4096 channels. */
int sp_mpo_abinitio(int K, const double* h, const double* eri, int* w, double* data, long long* n);

/* Energy component H_p of orbital p (1-based) for the fragment energies of
 * Sec. 2.4 (e_p = <H_p P>/<P>, sum_p e_p = E): the terms of the Hamiltonian
 * above whose first creator acts on orbital p,
 *   H_p = sum_q h_pq sum_s a+_ps a_qs + 1/2 sum_qrs (pq|rs) sum_st a+_ps a+_rt a_st a_qs,
 * so sum_p H_p = H and both spin orbitals of p lie in H_p (spin-free in the
 * expectation of Eq. [PropSpinFree] for real states).  Arguments and output
 * as for sp_mpo_abinitio; SP_EINVAL if p is outside 1..K.  The Hubbard form
 * takes the open chain's integrals (h = -t on nearest neighbours,
 * (pp|pp) = U), i.e. H_p = -t sum_s (a+_ps a_{p+1,s} + a+_ps a_{p-1,s})
 * + U n_pa n_pb; L in 2..64. */
int sp_mpo_abinitio_component(int K, int p, const double* h, const double* eri, int* w, double* data, long long* n);
int sp_mpo_hubbard_component(int L, int p, double t, double U, int* w, double* data, long long* n);

/* Projected expectation value of a spin-free operator given as an MPO,
 * Eq. [PropSpinFree]: <O> = <Psi|O P|Psi> / <Psi|P|Psi> for the current
 * state of h (any canonical centre), through the same environment and
 * H_eff contractions with O in place of H, in FP64.  *normP (optional) =
 * <P>.  The operator must commute with the total spin for this to be the
 * expectation in the projected state.  Synchronises. */
int sp_expect(sp_handle* h, const sp_mpo* O, double* value, double* normP);

/* Symmetric eigensolver used for the Davidson subspace problem
 * (Householder tridiagonalisation + implicit QL): a is n x n row-major
 * (destroyed), eigenvalues ascending in ev, eigenvectors as columns of vec
 * (n x n row-major). */
int sp_small_eigh(int n, double* a, double* ev, double* vec);

/* The same subspace solve on the GPU (the device-resident iteration's
 * kernel, one work-group), for tests: H, N (m x m row-major, host, copied)
 * with m <= 47.  need_all = 0: theta and a as sp_small_gen_lowest, *rank
 * the dimension kept.  need_all = 1 (a restart): also the Ritz vectors of
 * the `keep` lowest values (keep <= 16), orthonormalised (modified
 * Gram-Schmidt), in Qk (m x nk row-major, nk = min(keep, rank) in *rank),
 * and H, N overwritten by Qk^T H Qk, Qk^T N Qk in their leading nk x nk
 * (row stride m).  Synchronises the current device.  SP_ENORM if N
 * vanishes. */
int sp_small_gen_lowest_gpu(int m, double* H, double* N, double drop, int need_all, int keep, double* theta,
                            double* a, double* Qk, int* rank);

/* The Davidson subspace solve: lowest eigenpair of the symmetric pencil
 * H c = theta N c (m x m, row-major, not modified) restricted to the span of
 * the eigenvectors of N whose eigenvalues exceed drop * lambda_max(N)
 * (canonical orthogonalisation; the local problem of Eq. [geproblem] in the
 * search space).  On return theta, a (m coefficients, a^T N a = 1) and rank
 * (the dimension kept).  SP_ENORM if N vanishes. */
int sp_small_gen_lowest(int m, const double* H, const double* N, double drop, double* theta, double* a,
                        int* rank);

#ifdef __cplusplus
}
#endif
#endif /* SPMPS_H */
