/*
 * pe.h -- C ABI of the MI355X polarization-electrostatics library.
 *
 * Immersed-boundary electrostatics of ideally polarizable rigid bodies in
 * explicit-ion electrolytes (Krucker-Velasquez, Swan, Sherman, arXiv
 * 2401.04865): bodies are rigid sets of surface beads carrying regularized
 * charges, ions are single-bead bodies with fixed charge, the whole periodic
 * system sits in a uniform applied field E0.
 *
 * The library evaluates the regularized potential tensor M with a spectral
 * Ewald method (real-space pair sum over a cell list + Gaussian spreading,
 * 3-D FFT, Green's-function scaling, inverse FFT, Gaussian contraction),
 * solves the conductor saddle-point system for the induced bead charges and
 * the body potentials with GMRES, and returns dipoles, energies, forces and
 * torques.  Everything runs on one GPU in hand-written HIP kernels for
 * gfx950.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns a pe_status; no C++ exception crosses the ABI.
 *   On an error, pe_last_error() returns a message for the context.
 * - "dev" pointers are device pointers (e.g. torch CUDA tensors) owned by
 *   the caller and valid for the duration of the call; "host" pointers are
 *   ordinary host memory.  All floating point arrays are IEEE double,
 *   row-major, C-contiguous.
 * - Beads are stored body-major: beads body_offsets[i] .. body_offsets[i+1]-1
 *   belong to body i (the global bead index of the paper).  Ions follow
 *   their own caller order.  Positions are unwrapped lab-frame coordinates;
 *   the library wraps them into the periodic box internally.
 * - Work is enqueued on the HIP stream given to pe_create.  Entry points that
 *   return host data (solve, forces, apply) synchronize that stream before
 *   returning; pe_set_system synchronizes once (to size the neighbour data).
 * - The library never allocates device memory.  All of a context's device
 *   buffers lie in one region the caller owns and registers with
 *   pe_set_workspace (pe_workspace_size says how large); a call that needs
 *   more returns PE_ERR_NOMEM and can be repeated with the same arguments
 *   after a larger region is registered.
 * - A context is not thread safe; use one context per host thread.
 */
#ifndef PE_H
#define PE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pe_context pe_context;

typedef enum {
  PE_OK = 0,
  PE_ERR_ARG = 1,           /* invalid argument (checked before any launch) */
  PE_ERR_STATE = 2,         /* call out of order (e.g. solve before set_system) */
  PE_ERR_DEVICE = 3,        /* a HIP runtime call failed */
  PE_ERR_NOMEM = 4,         /* device allocation failed */
  PE_ERR_NOT_CONVERGED = 5, /* Krylov solve hit max_iters; outputs hold the last iterate */
  PE_ERR_NUMERIC = 6        /* NaN/Inf appeared in the solve */
} pe_status;

typedef enum {
  PE_FP64 = 0,  /* every kernel in double */
  PE_MIXED = 1  /* spread/FFT/gather/real-space in float; Krylov basis,
                   reductions, constraints, energies and the outer residual
                   of an iterative refinement in double */
} pe_precision;

typedef enum {
  PE_REG_GAUSSIAN = 0, /* Gaussian charges of per-particle standard deviation sigma */
  PE_REG_SHELL = 1,    /* uniformly charged shells of one radius (the paper's own), with the
                          whole regularization in the real-space kernel and the wave space
                          of point charges */
  PE_REG_SHELL_PAPER = 2 /* the same shells with the paper's own split (section
                          "Spectrally-accurate Ewald summation"): j0^2(ka) multiplies the
                          Green's function of the wave space, the real-space kernel is the
                          closed form of section "Real-space sum" (its Heaviside term read
                          as -(1/(4 pi r) - (4a - r)/(16 pi a^2)) H(2a - r)) with the printed
                          self term; the same potential tensor M */
} pe_reg;

/*
 * Parameters.  pe_default_params fills the defaults listed here.
 *
 * Spectral Ewald (section "Spectrally-accurate Ewald summation"):
 *   split h(k) = exp(-k^2/4 xi^2); grid spacing h_d = box[d]/mesh[d]; window
 *   support P points per axis; eta = (h xi)^2 P / (pi eta_c^2) with h the
 *   largest spacing (eta_c = 1 is the paper's choice of eta).
 * Derived when xi <= 0 / r_cut <= 0 (tolerance tau = split_tol):
 *   k_c = pi min_d (mesh[d]-1)/box[d]  (the paper's N_g = 1 + L k_c / pi),
 *   xi = k_c / (2 sqrt(ln 1/tau)),
 *   r_cut = sqrt(ln 1/tau) * max(1/xi, 2 sigma_max) for Gaussians,
 *           max(sqrt(ln 1/tau)/xi, 2 a) for shells, and
 *           2 a + sqrt(ln 1/tau)/xi for shells with the paper's split (its
 *           real-space kernel decays like erfc(xi (r - 2a))).
 */
typedef struct pe_params {
  double box[3];          /* periodic box lengths */
  int32_t mesh[3];        /* FFT grid points per axis; mesh[2] even; factors 2,3,5 only */
  int32_t P;              /* window support per axis (default 8) */
  double eta_c;           /* default 1 */
  double xi;              /* <= 0: derived (default) */
  double r_cut;           /* <= 0: derived (default); must be <= min(box)/2 */
  double split_tol;       /* tau, default 1e-8 */
  double eps;             /* permittivity, default 1 */
  int32_t precision;      /* pe_precision, default PE_FP64 */
  int32_t reg;            /* pe_reg, default PE_REG_GAUSSIAN */
  double shell_radius;    /* PE_REG_SHELL only */
  int32_t gmres_restart;  /* Krylov basis size before a restart, default 100, at most 255 */
  int32_t max_iters;      /* total Krylov iterations, default 1000 */
  double rel_tol;         /* target ||b - A x|| / ||b|| with the double operator, default 1e-6 */
  double inner_tol;       /* PE_MIXED: floor of each inner solve's relative tolerance, default 1e-7
                             (each inner solve aims at half of rel_tol, see pe_solve_polarization) */
  int32_t max_refine;     /* PE_MIXED: max outer refinement steps, default 8 */
  int32_t use_learned_guess; /* 1: start from the network's prediction (needs a loaded model) */
  int32_t precond;        /* 1 (default): block-Jacobi preconditioner (inverse of each body's
                             free-space saddle block) inside flexible GMRES; 0: none */
  int32_t rhs_fp64;       /* PE_MIXED: 1 (default) forms the ion potential of the right-hand
                             side in double, so the double residual is that of the system the
                             PE_FP64 path solves; 0 forms it with the float kernels */
  double hs_radius;       /* pe_bd_step: hard-sphere radius a of every particle (ions and beads;
                             beads of one body never interact), section "Brownian dynamics":
                             the potential-free pair potential gamma/(4 dt) (r - 2a)^2 for
                             r < 2a.  0 (default): none.  2a must not exceed a third of the box */
} pe_params;

typedef struct pe_solve_info {
  int32_t iters;              /* Krylov iterations (inner ones in PE_MIXED) */
  int32_t outer_refinements;  /* PE_MIXED outer steps (0 for PE_FP64) */
  int32_t matvecs_fp64;       /* double-precision operator applications */
  int32_t matvecs_fp32;       /* float operator applications */
  double rel_residual;        /* final ||b - A x||/||b||, double operator */
  double rel_residual_guess;  /* same, at the initial guess */
  double rhs_norm;            /* ||b||, so ||b - A x|| = rel_residual * rhs_norm */
  double t_rhs, t_guess, t_solve, t_total; /* seconds */
  int32_t n_hist;             /* residual estimates recorded in hist */
  double hist[1024];
} pe_solve_info;

/* Fill p with the defaults above (box/mesh zeroed: the caller sets them). */
pe_status pe_default_params(pe_params* p);

/* Create a context.  hip_stream: a hipStream_t (NULL = the null stream).
 * Checks mesh factors, P <= min(mesh), positive box/eps. */
pe_status pe_create(const pe_params* params, void* hip_stream, pe_context** out);
pe_status pe_destroy(pe_context* ctx);
const char* pe_last_error(const pe_context* ctx);

/*
 * Device workspace (the library's only device memory, owned by the caller).
 *
 * pe_workspace_size  bytes (host size_t) a system of n_bead beads, n_body
 *                    bodies and n_ion ions needs: every buffer at its size
 *                    for these counts, the data-dependent ones (stored bead
 *                    pairs, spreading lists, body-shape blocks, one recorded
 *                    training solve) estimated from the mean densities; after
 *                    a call failed with PE_ERR_NOMEM it returns at least what
 *                    that call needed.  PE_ERR_ARG for a null pointer or a
 *                    negative count.
 * pe_set_workspace   registers [dev_ptr, dev_ptr + bytes) (device memory,
 *                    256-byte aligned, e.g. a torch uint8 tensor) as the
 *                    region.  Buffers already live (tables, the last
 *                    system, shapes, the network) are copied into it, so the
 *                    previous region may be released once this returns; it
 *                    must not overlap the new one unless it is the same base
 *                    address.  Waits for the context's streams first.
 *                    PE_ERR_NOMEM if the live buffers do not fit.  The caller
 *                    keeps the region alive and unused by others until
 *                    pe_destroy or the next pe_set_workspace.
 * pe_workspace_info  out[0] registered bytes, out[1] bytes in live buffers,
 *                    out[2] the most ever live, out[3] the size the last
 *                    failed request needed (0 if none failed).
 */
pe_status pe_workspace_size(const pe_context* ctx, int64_t n_bead, int64_t n_body, int64_t n_ion, size_t* bytes);
pe_status pe_set_workspace(pe_context* ctx, void* dev_ptr, size_t bytes);
pe_status pe_workspace_info(const pe_context* ctx, size_t out[4]);

/* The split parameters in use (valid after pe_set_system):
 * out[0]=xi, out[1]=r_cut, out[2]=eta, out[3]=h (largest spacing),
 * out[4]=number of real-space bead pairs stored (incl. self), out[5]=cells per axis (x). */
pe_status pe_get_derived(const pe_context* ctx, double out[6]);

/*
 * Load a configuration (section "Induced Surface Charge Distribution of
 * Polarizable Bodies").  Given: bead positions x_ij, body centres X_i (the
 * centre of mass; r_ij = x_ij - X_i is formed from the unwrapped inputs),
 * body charges Q_i, ions (single-bead bodies with fixed charge), field E0.
 *   body_offsets  host, n_body+1 int64, nondecreasing, [0] = 0, [n_body] = n_bead
 *   bead_pos      dev n_bead x 3;  bead_sigma dev n_bead (> 0; ignored for shells)
 *   body_center   dev n_body x 3;  body_quat dev n_body x 4 (w,x,y,z) or NULL
 *                 (body frame = lab frame); body_charge dev n_body
 *   ion_pos/ion_charge/ion_sigma  dev n_ion x 3 / n_ion / n_ion (may be NULL if n_ion = 0)
 *   E0            host 3
 * Copies everything it needs, wraps positions, sorts beads and ions into
 * cells, and builds the bead-bead real-space operator once (positions are
 * fixed during a solve).  Errors: PE_ERR_ARG for sizes, non-finite values,
 * non-positive widths or r_cut > min(box)/2.
 */
pe_status pe_set_system(pe_context* ctx, int64_t n_body, const int64_t* body_offsets,
                        const double* bead_pos, const double* bead_sigma,
                        const double* body_center, const double* body_quat,
                        const double* body_charge, int64_t n_ion, const double* ion_pos,
                        const double* ion_charge, const double* ion_sigma,
                        const double E0[3]);

/*
 * The bare operator (section "Spectral Ewald implementation", steps 1-6):
 * potentials psi = M c of all particles for charges c, and optionally the
 * field E = -grad (M c) at each particle (its own self term contributes
 * nothing).  Particles are the beads followed by the ions.
 *   charges   dev n_bead + n_ion;  psi_out dev n_bead + n_ion
 *   field_out dev (n_bead + n_ion) x 3 or NULL
 *   precision PE_FP64 or PE_MIXED (float kernels)
 * The k = 0 constant of the split is removed exactly, so psi is the
 * potential of the k != 0 definition of M.
 */
pe_status pe_apply_potential(pe_context* ctx, const double* charges, double* psi_out,
                             double* field_out, int32_t precision);

/*
 * Solve the saddle-point system (eq. "saddle")
 *   [ -M     Sigma^T ] [ q    ]   [ -r.E0 + M_bead,ion q_ion ]
 *   [ Sigma  0       ] [ dPsi ] = [  Q                       ]
 * for the bead charges q and dPsi = Psi - Psi_0 (ions are eliminated into the
 * right-hand side).  Restarted flexible GMRES with classical Gram-Schmidt
 * applied twice, Givens rotations and back substitution in double on the
 * device, preconditioned (precond = 1, the default) by the block-Jacobi
 * inverse of each body's free-space saddle block, or unpreconditioned
 * (precond = 0).  With PE_MIXED the inner solves use the float operator
 * inside a double iterative refinement whose residuals b - A x are formed
 * with the double operator (and, with rhs_fp64, a double b); convergence is
 * only ever declared on such a double residual, also for a warm start.  Each
 * inner solve starts from the current residual r (relative size rel) and
 * stops when the float residual estimate has fallen by
 * max(inner_tol, 0.5 rel_tol / rel), at most 0.5: it aims at half the target,
 * so one double residual usually confirms convergence, and the floor keeps it
 * from chasing the float operator's rounding.
 *   q_init   dev n_bead or NULL (zero guess, or the network's when enabled)
 *   q_out    dev n_bead;  dpsi_out dev n_body;  dipole_out dev n_body x 3 or NULL
 *            (S_i = sum_j r_ij q_ij, eq. "rigid_dipole")
 *   info     host or NULL
 * Returns PE_ERR_NOT_CONVERGED (outputs = last iterate) or PE_ERR_NUMERIC.
 */
pe_status pe_solve_polarization(pe_context* ctx, const double* q_init, double* q_out,
                                double* dpsi_out, double* dipole_out, pe_solve_info* info);

/*
 * Forces, torques and energies from the last solve (section "Forces and
 * Torques" and its appendix derivation): bead and ion forces
 * f = q (E0 + E), E = -grad of M over all charges; F_i = sum_j f_ij,
 * L_i = sum_j r_ij x f_ij; energy U = 1/2 q.Mq - sum q x.E0 over all charges,
 * split per body (body_energy) with the ion share included in total_energy.
 * Every output may be NULL except total_energy (host).
 *   body_force/body_torque dev n_body x 3; body_energy dev n_body;
 *   ion_force dev n_ion x 3; bead_force dev n_bead x 3.
 */
pe_status pe_forces_torques(pe_context* ctx, double* body_force, double* body_torque,
                            double* body_energy, double* ion_force, double* bead_force,
                            double* total_energy);

/*
 * Grand capacitance tensor and effective permittivity of the loaded
 * configuration (section "Induced Surface Charge Distribution of Polarizable
 * Bodies", the rigid-body moment equation [Q; S] = C [Psi - Psi_0; E0] with
 * C = Sigma' M^-1 Sigma'^T; section "Cubic array of spheres in an electric
 * field" for the permittivity).  Ions do not enter (M is the bead-bead
 * potential tensor).  Rows and columns: body i's charge is index i, its
 * dipole components d = x, y, z are n_body + 3 i + d.
 *   C_out    dev (4 n_body) x (4 n_body), row-major, or NULL
 *   eps_eff  host 3 x 3, row-major, or NULL: for neutral bodies in the mean
 *            field, eps I + (1/V) sum_ij [C_SE - C_SPsi C_qPsi^-1 C_qE]_ij
 *   info     host or NULL: iters = most conjugate-gradient iterations of any
 *            column, matvecs_fp64 = operator applications, rel_residual =
 *            largest final ||b - M x|| / ||b|| over the columns
 * The 4 n_body systems M x = (column of Sigma'^T) are solved with the double
 * operator whatever the context precision, by conjugate gradients (block
 * Jacobi over the bodies' free-space self blocks when precond = 1) to
 * rel_tol, blocks of up to 32 columns sharing each step's launches.
 * PE_ERR_STATE before pe_set_system; PE_ERR_ARG without bodies;
 * PE_ERR_NOT_CONVERGED if a column misses rel_tol within max_iters.
 */
pe_status pe_grand_capacitance(pe_context* ctx, double* C_out, double* eps_eff, pe_solve_info* info);

/*
 * The saddle-point operator itself (the matrix of eq. "saddle", ions
 * eliminated): y = [-M q + Sigma^T dPsi ; Sigma q] for x = [q ; dPsi].  This is
 * the product every Krylov iteration evaluates: one bead-only spectral-Ewald
 * pass (spread, FFT, scale, inverse FFT, gather) plus the stored bead-bead
 * real-space operator, plus the per-body sums.
 *   x, y  dev n_bead + n_body;  precision PE_FP64 or PE_MIXED (float kernels)
 */
pe_status pe_apply_saddle(pe_context* ctx, const double* x, double* y, int32_t precision);

/*
 * Kernel timing with HIP events recorded around every launch on the
 * context's stream, accumulated per kernel class and precision, with the
 * work each class did.  pe_profile_enable(ctx, 1) resets and starts;
 * pe_profile_read fills out[6*PE_PROF_NCLASS] with (launch count, total
 * milliseconds, work units) per class in enum order, first for the float
 * kernels, then for the double kernels (the Krylov vector kernels are always
 * double).  Work units: particles spread or contracted (SPREAD, GATHER),
 * pairs inside the real-space cutoff evaluated (PAIR), stored sparse
 * real-space entries applied (SPMV), multiply-adds of the dense per-shape
 * products (NEAR, PRECOND), launches (FFT passes), 0 otherwise.
 */
typedef enum {
  PE_PROF_SPREAD = 0,
  PE_PROF_FFT_Z_R2C,
  PE_PROF_FFT_Y_FWD,
  PE_PROF_FFT_X_SCALE,
  PE_PROF_FFT_Y_INV,
  PE_PROF_FFT_Z_C2R,
  PE_PROF_GATHER,
  PE_PROF_SPMV,
  PE_PROF_PAIR,
  PE_PROF_KRYLOV,
  PE_PROF_PRECOND,
  PE_PROF_NEAR,
  PE_PROF_MATVEC,   /* one whole Krylov operator application (pe_apply_saddle and every
                       product inside a solve), around all of its kernels; work = beads.
                       It encloses launches of the other classes, so it is not a kernel class */
  PE_PROF_NCLASS
} pe_prof_class;
pe_status pe_profile_enable(pe_context* ctx, int32_t on);
pe_status pe_profile_read(pe_context* ctx, double* out);
/*
 * Restrict the event recording to the classes whose bit is set in
 * class_mask (bit c = class c, float and double launches alike); the others
 * run without events while profiling is on, so one class can be timed inside
 * a run without slowing the rest.  The mask persists until changed;
 * 0xffffffff (the default) records every class.  PE_ERR_ARG if ctx is null.
 */
pe_status pe_profile_select(pe_context* ctx, uint32_t class_mask);

/*
 * Learned initial guess (a per-bead network, not in the paper).  Features of
 * bead ij: body-frame position R_i^T r_ij (3), body-frame local applied
 * field R_i^T (E0 + E_ion(x_ij)) (3), one-hot body type (2).  Two hidden
 * layers of 64 (tanh), output 3 numbers w dotted with the body-frame local
 * field, plus Q_i / N_i; the guess is then projected onto sum_j q_ij = Q_i.
 * The Krylov solve always runs to the same residual afterwards.
 *
 * pe_guess_init       random weights from a seed.
 * pe_guess_record     after a solve: append (features, solved q) of every bead
 *                     of the current system to the device training set.
 * pe_guess_train      Adam on the recorded set for `epochs` passes with batch
 *                     size `batch` and learning rate `lr`; returns the last
 *                     mean squared error in *loss (host).
 * pe_guess_predict    q_out (dev n_bead) = projected prediction for the current
 *                     system (needs pe_set_system).
 * pe_guess_save/load  weights as a little-endian binary with a header.
 * pe_guess_set_types  body type ids (host n_body int32, 0 or 1) for the features.
 */
pe_status pe_guess_init(pe_context* ctx, uint64_t seed);
pe_status pe_guess_set_types(pe_context* ctx, const int32_t* body_type);
pe_status pe_guess_record(pe_context* ctx, const double* q_solved);
pe_status pe_guess_clear(pe_context* ctx);
pe_status pe_guess_train(pe_context* ctx, int32_t epochs, int32_t batch, double lr,
                         uint64_t seed, double* loss);
pe_status pe_guess_predict(pe_context* ctx, double* q_out);
pe_status pe_guess_save(const pe_context* ctx, const char* path);
pe_status pe_guess_load(pe_context* ctx, const char* path);

/*
 * Test hooks of the learned guess.  pe_guess_debug: copy the kNPar = 4996
 * float parameters out (set_params = 0) or in (1), and if n_rows > 0 return
 * the gradient of the mean squared loss over the first n_rows recorded rows
 * (grad host kNPar floats, loss host).  Parameter order: W1[64][8], b1[64],
 * W2[64][64], b2[64], W3[4][64], b3[4].  pe_guess_rows: copy the first n_rows
 * recorded rows (11 floats each: 8 features, Q_i/N_i, solved q, 0) to host;
 * pe_guess_add_rows appends host rows of the same layout to the training set.
 */
pe_status pe_guess_debug(pe_context* ctx, float* params_inout, int32_t set_params, int64_t n_rows,
                         float* grad, double* loss);
pe_status pe_guess_rows(pe_context* ctx, float* rows, int64_t n_rows);
pe_status pe_guess_add_rows(pe_context* ctx, const float* rows, int64_t n_rows);

/*
 * One overdamped Brownian-dynamics step (section "Brownian dynamics
 * simulations...": Euler-Maruyama, free draining, no hydrodynamic
 * interactions) using the forces of the last pe_forces_torques call:
 * ions x += f dt / gamma + sqrt(2 kT dt / gamma) N(0,1);
 * bodies move rigidly: U_i = F_i / (N_i gamma) + Brownian term,
 * Omega_i = K_i^{-1} L_i + Brownian term, K_i = gamma sum_j (|r|^2 I - r r^T),
 * beads follow x_ij = X_i + R_i r'_ij.  With hs_radius > 0 the forces of the
 * potential-free hard-sphere pair potential at the current positions are
 * added first (bead parts into each body's force and torque).  Gaussian noise comes from a
 * counter-based Philox-4x32-10 generator keyed by (seed, step, particle).
 * Updates the caller's arrays in place (same layouts as pe_set_system):
 *   bead_pos dev n_bead x 3 (rebuilt from the body frame), body_center,
 *   body_quat (n_body x 4), ion_pos.  Call pe_set_system again afterwards.
 */
pe_status pe_bd_step(pe_context* ctx, double dt, double kT, double gamma, uint64_t seed,
                     uint64_t step, double* bead_pos, double* body_center, double* body_quat,
                     double* ion_pos);

/*
 * pe_bd_step without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid it): the same step and the same kernels as
 * pe_bd_step, bit for bit, with the per-body rotations kept in a static
 * device array of the library (one per GPU, 9 doubles for each of at most
 * 65536 bodies, held until the process ends) instead of the workspace.
 * Arguments and state requirements as pe_bd_step; PE_ERR_ARG for more than
 * 65536 bodies.  Every call on one GPU uses that GPU's array: calls that
 * overlap on one GPU (several contexts or threads) race.
 */
pe_status pe_bd_step_noalloc(pe_context* ctx, double dt, double kT, double gamma, uint64_t seed,
                             uint64_t step, double* bead_pos, double* body_center, double* body_quat,
                             double* ion_pos);

#ifdef __cplusplus
}
#endif
#endif /* PE_H */
