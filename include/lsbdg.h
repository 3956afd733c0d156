/*
 * lsbdg -- matrix-free discontinuous-Galerkin operators for the
 * scale-resolved lithium-sulfur cathode model of arXiv 2511.05233
 * ("Structure Matters"), for AMD Instinct MI355X (gfx950).
 *
 * The problem (Sec. 2.2-2.6, Tab. 4): on a voxelised porous cathode of
 * nx x ny x nz cubic voxels of edge h (x = transport axis), the unknowns per
 * DG node are the six dissolved-species concentrations
 *     c = (Li+, S8(L), S8^2-, S6^2-, S4^2-, S^2-)  [mol/m^3],
 * the liquid potential Phi_L [V], and the solid volume fractions
 * (eps_S8, eps_Li2S) of Tab. 4's solid-phase mass equations.  The solid is
 * equipotential at V = dPhi0 of Tab. InitialState (the gauge of Sec. 2.10).
 * Species obey Nernst-Planck transport with Bruggeman-effective,
 * viscosity-scaled diffusivities (Eq. 02-03, 16a); Phi_L obeys the
 * anion-eliminated charge balance (Tab. 4; Sec. 2.7 item (i)); reactions
 * are the Tradeoff Chemistry of Tab. 3 with Butler-Volmer kinetics
 * (Eq. 05-06, 18-24).  Space: interior-penalty DG with harmonic-mean
 * coefficients (Eq. 43-47) on tensor-product Gauss-Legendre nodes of degree
 * k per axis: k = 1 (Q1, 8 nodes per voxel) for every entry point, k = 0
 * (Eq. 48) for the operators, k = 3 (64 nodes) for the operators and the
 * element block-Jacobi preconditioner; time: backward Euler
 * (Eq. 50).  The separator face
 * x = L_x receives the Li+ flux j_el/F and the ionic current j_el; all other
 * faces are no-flux (Eq. 47 with the paper's galvanostatic condition).
 *
 * Memory layout of every state-like array: field-major  a[f][e][n]
 *     f  field index (9 for a state, 7 for Krylov vectors, 8 for old mass)
 *     e  = ix + nx*(iy + ny*iz)            (x fastest)
 *     n  = a0 + K*(a1 + K*a2), K = k + 1   (x fastest within the voxel)
 * in the precision selected per call (double for DG_F64, float for DG_F32;
 * dg_blockjacobi_apply_bf16 streams bfloat16 copies of FP32 block inverses).
 * Batches of several structures (dg_batch_*) concatenate them voxel by
 * voxel in the same layout.
 *
 * Ownership: the caller owns every array passed in (state, residual and
 * vector buffers, on the device unless stated).  The library allocates its
 * own device tables in dg_setup and frees them in dg_destroy.  Work is
 * enqueued on the caller's HIP stream (0 = the null stream); entry points
 * that return host scalars synchronise that stream.
 *
 * Errors: every entry point returns a dg_status; no C++ exception crosses
 * the boundary.  On failure dg_last_error() describes the cause (valid
 * until the next call on the same thread).
 */
#ifndef LSBDG_H
#define LSBDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dg_ctx dg_ctx;           /* opaque, library-owned */
typedef void* dg_stream;                 /* a hipStream_t */

typedef enum {
  DG_OK = 0,
  DG_EINVAL = -1,        /* bad argument: null pointer, size, order, ... */
  DG_ENOMEM = -2,        /* device allocation failed */
  DG_EHIP = -3,          /* a HIP runtime call or kernel launch failed */
  DG_ENOCONV = -4,       /* Newton did not converge (report filled) */
  DG_ENAN = -5,          /* non-finite residual norm */
  DG_ESTATE = -6,        /* call out of order (e.g. apply before setup) */
  DG_EUNSUPPORTED = -7   /* valid but not implemented (order, precision) */
} dg_status;

typedef enum { DG_F64 = 0, DG_F32 = 1 } dg_prec;

/* Jacobian-vector product modes.
 *   DG_JVP_FULL9:      v and J v over all 9 fields.
 *   DG_JVP_CONDENSED7: v and J v over the 7 transported fields; the solid
 *     fractions are eliminated node by node (their rows hold no spatial
 *     coupling): J_red v = J_uu v + J_ue w with w = -J_ee^-1 J_eu v.  The
 *     node-local coefficients of w (w = C v, C: 2 x 7 per node) are formed
 *     first (as dg_linearize does), then applied.
 *   DG_JVP_LINEARIZED7: as DG_JVP_CONDENSED7 with the coefficients of the
 *     last dg_linearize call of the same precision, which must have been at
 *     this u, t_new and dt (the Krylov operator of one Newton iteration). */
typedef enum { DG_JVP_FULL9 = 0, DG_JVP_CONDENSED7 = 1, DG_JVP_LINEARIZED7 = 2 } dg_jvp_mode;

/* Mesh: voxel counts, voxel edge h [m], polynomial degree per axis. */
typedef struct {
  int32_t nx, ny, nz;
  int32_t order;
  double h;
} dg_mesh;

/* Physical and numerical parameters, SI units.  dg_params_default() fills
 * the paper's values (Tab. 5, Tab. 2, Eq. 02); workloads override D0 and kE.
 * Fields set to a negative value are derived in dg_setup as noted. */
typedef struct {
  double T;             /* temperature [K] (298.15: reproduces Tab. 5 "Equi.") */
  double D0[7];         /* infinite-dilution diffusivities [m^2/s]:
                           Li+, S8(L), S8^2-, S6^2-, S4^2-, S^2-, anion */
  double kE[6];         /* electrochemical rate constants E1..E6 [mol/(s m^2)] */
  double f_C;           /* discharge rate [1/h] (Eq. 18 passivation, App. C) */
  double j_el;          /* applied current density [A/m^2]; < 0: App. C,
                           f_C * c_theo * m_A with m_A from the structure */
  double eps_struct;    /* structure fraction of Eq. 57; < 0: 1 - pore fraction */
  double sigma;         /* interior-penalty factor; <= 0: 1 for k = 0, (k+1)^2 else */
  double c_min;         /* activity clamp [mol/m^3] */
  double epsL_min;      /* floor of the liquid fraction */
  int32_t use_TH;       /* 1: multiply C2 and E4 by T_H(t) (Eq. 56, Sec. 2.10) */
  int32_t reserved;
} dg_params;

/* Fill *p with the paper's parameters (Tab. 5) and defaults. */
void dg_params_default(dg_params* p);

/* Create a context for one voxel structure; the library allocates its
 * device memory as it is first needed (dg_setup_ws: in a caller-owned
 * workspace instead).
 *   mesh   mesh and degree: order 1 (Q1: every entry point); order 0
 *          (the finite-volume scheme of Eq. 48) and order 3 (tricubic,
 *          4 x 4 x 4 Gauss nodes per voxel, Eq. 43-47 with sigma = 16): the
 *          operators dg_mass, dg_residual, dg_linearize and dg_jvp, and at
 *          order 3 also dg_blockjacobi_setup/apply/export/info; the other
 *          entry points return DG_EUNSUPPORTED for them
 *   phase  HOST array of nx*ny*nz bytes, x fastest: 0 = pore voxel
 *          (electrolyte only, no reactions), 1 = cathode structure voxel
 *          (Eq. 57 localisation); copied, may be freed after the call
 *   params parameters (copied)
 *   out    receives the context
 * Errors: DG_EINVAL (null pointer, non-positive size, phase not 0/1,
 * order not one of 0, 1, 3), DG_ENOMEM, DG_EHIP. */
int dg_setup(const dg_mesh* mesh, const uint8_t* phase, const dg_params* params,
             dg_ctx** out);

/* Free the context and its device tables (never the caller's arrays). */
int dg_destroy(dg_ctx* ctx);

/* Derived scalars of the context (host): dPhi0 = V of Tab. InitialState,
 * the equilibrium concentrations c0[6], U0[6] (U0_5, U0_6 recomputed from
 * Tab. InitialState), the applied current j_el [A/m^2] and eps_struct. */
int dg_info(const dg_ctx* ctx, double* V, double* c0, double* U0, double* j_el,
            double* eps_struct);

/* Old mass of a state (Eq. 50 with Eq. 16a/17a time derivatives):
 *   m[i] = eps_L c_i (i = 0..5),  m[6 + s] = eps_s (s = 0, 1)
 * u: device, 9 fields; m: device, 8 fields; same precision. */
int dg_mass(dg_ctx* ctx, dg_prec prec, const void* u, void* m, dg_stream stream);

/* DG residual of the backward-Euler step ending at t_new [s] with step dt:
 *   species i: W (eps_L c_i - m_i)/dt + transport_i - W S_i - separator inflow
 *   charge:    transport_Phi - W S_Phi - separator current
 *   solids s:  W ((rho/M)_s (eps_s - m_{6+s})/dt - S_s)
 * (Eq. 43-47 and 50; W = nodal quadrature weight times (h/2)^3).
 * u: device, 9 fields; m_old: device, 8 fields from dg_mass of the old
 * state; r: device, 9 fields.  T_H is evaluated at t_new. */
int dg_residual(dg_ctx* ctx, dg_prec prec, const void* u, const void* m_old,
                double t_new, double dt, void* r, dg_stream stream);

/* Jacobian-vector product of dg_residual at (u, t_new, dt) in direction v:
 * the exact derivative of the same arithmetic (forward-mode dual numbers;
 * the Q1 product at a stored linearisation, DG_JVP_LINEARIZED7, has its
 * tangents written out by hand), with zero derivative where a clamp is
 * active.  The old mass does not
 * enter.  u: device, 9 fields; v and jv: device, 9 fields (DG_JVP_FULL9) or
 * 7 fields (condensed modes); all in the precision prec.  DG_ESTATE:
 * DG_JVP_LINEARIZED7 without a linearisation of that precision. */
int dg_jvp(dg_ctx* ctx, dg_prec prec, dg_jvp_mode mode, const void* u, const void* v,
           double t_new, double dt, void* jv, dg_stream stream);

/* Linearisation point of the condensed tangent: stores in library-owned
 * device memory (14 values per node, precision prec) the coefficients C of
 * the node-local elimination w = -J_ee^-1 J_eu v = C v at (u, t_new, dt),
 * for later DG_JVP_LINEARIZED7 products.  u: device, 9 fields. */
int dg_linearize(dg_ctx* ctx, dg_prec prec, const void* u, double t_new, double dt, dg_stream stream);

/* Element block-Jacobi preconditioner (replaces the paper's BoomerAMG
 * preconditioner of Sec. 2.9 inside GMRES).  Builds the exact
 * element-diagonal blocks of the condensed 7-field Jacobian at (u, t_new,
 * dt) -- volume, own-face, time and source terms of each voxel's rows with
 * respect to its own nb = 7 * nodes unknowns (56 at k = 1, 448 at k = 3) --
 * and inverts them in place (Gauss-Jordan with partial pivoting) into
 * library-owned device storage of Ne * nb * nb values of precision prec
 * (FP32: 22 GB for the 96x96x192 slab at k = 1, 88.8 GB for 48^3 voxels
 * at k = 3).  At k = 3 the blocks are probed from the Krylov operator
 * (2 x 448 applications, one checkerboard colour at a time; the
 * linearisation at u is left stored) and inverted by a blocked
 * Gauss-Jordan on the matrix cores, keeping a pivot list of Ne * 448 int16.
 * Synchronises the stream.  DG_ENAN if a block is singular or not finite;
 * DG_EUNSUPPORTED at order 0. */
int dg_blockjacobi_setup(dg_ctx* ctx, dg_prec prec, const void* u, double t_new, double dt,
                         dg_stream stream);

/* y_e = B_e^{-1} x_e for every voxel e, with the blocks of the last setup.
 * x, y: device, 7 fields, precision of the setup (DG_EINVAL otherwise;
 * DG_ESTATE before any setup). x and y must not overlap.  Orders 1 and 3. */
int dg_blockjacobi_apply(dg_ctx* ctx, dg_prec prec, const void* x, void* y, dg_stream stream);

/* As dg_blockjacobi_apply after an FP32 setup, but streaming a bfloat16
 * copy of the stored inverses (each entry rounded to nearest even; made on
 * the first call after a setup and kept, Ne * 56 * 56 * 2 bytes): y_e =
 * bf16(B_e^{-1}) x_e with FP32 accumulation.  This is the preconditioner
 * apply of FP32 inner solves with block_bf16; such solves (dg_step,
 * dg_initial_state, dg_advance) invert their blocks straight into the
 * bfloat16 copy, which this call then applies, and leave no FP32 inverses
 * (dg_blockjacobi_apply then needs a new setup).  x, y: device, FP32,
 * 7 fields, not overlapping.  DG_ESTATE without an FP32 setup or such a
 * solve before; DG_EUNSUPPORTED at orders other than 1. */
int dg_blockjacobi_apply_bf16(dg_ctx* ctx, const void* x, void* y, dg_stream stream);

/* Copy the stored inverse blocks (Ne blocks of nb x nb, column-major:
 * out[e][col][row], row/col = field * nodes + node; at k = 3 with the
 * pivoting undone) to the device buffer out, in the precision of the setup
 * (dg_blockjacobi_info); out must hold Ne * nb * nb values of that
 * precision.  DG_ESTATE when no inverses are
 * stored (none set up, or only the bfloat16 copy of a solve). */
int dg_blockjacobi_export(dg_ctx* ctx, void* out, dg_stream stream);

/* Precision (DG_F64 or DG_F32) and edge (56, or 448 at k = 3) of the stored inverse blocks,
 * so that a caller sizes the buffer of dg_blockjacobi_export from the
 * library's own state.  Host call, no device work.  DG_ESTATE when no
 * inverses are stored. */
int dg_blockjacobi_info(const dg_ctx* ctx, int32_t* prec, int32_t* block_size);

/* Options of the Newton-Krylov step solver. */
typedef struct {
  int32_t inner_prec;    /* DG_F32: FP32 JVP, blocks and GMRES (mixed precision);
                            DG_F64: everything in FP64 */
  int32_t gmres_restart; /* GMRES restart length m, 1..30 (default 30) */
  int32_t gmres_maxit;   /* GMRES iterations per Newton iteration (default 1500) */
  int32_t newton_maxit;  /* Newton iterations (default 60) */
  double gmres_rtol;     /* relative reduction of the preconditioned, scaled
                            residual per Newton iteration (default 1e-4) */
  double gmres_rtol_final; /* tolerance once the Newton update is below 1e-7
                            (default 1e-11; FP32 inner solves stop at 1e-5) */
  double newton_tol;     /* converged when a full step changes no unknown by
                            more than this relative amount (default 1e-11) */
  int32_t coarse;        /* coarse space of the preconditioner: 0 = default
                            (3, or 4 where the multilevel cycle of
                            mg_levels is used), 1 = global per-field
                            constants,
                            additive, 2 = global per-field constants with
                            deflation (exact coarse solve), 3 = per-field
                            constants on voxel aggregates, additive (a
                            two-level method; LU of the coarse operator in
                            FP64), 4 = the same space applied
                            multiplicatively (coarse solve, then the element
                            blocks on the remaining residual), -1 = none */
  int32_t coarse_agg;    /* aggregate edge in voxels for coarse = 3, 4 (0: the
                            smallest edge >= 4 with at most 8192 coarse
                            unknowns) */
  int32_t block_bf16;    /* DG_F32 inner solves: 1 (default) streams the
                            element block inverses as bfloat16 in the
                            preconditioner apply (half the bytes; only the
                            preconditioner changes, not the Newton root);
                            0 streams them in FP32 */
  int32_t verbose;       /* 1: one line per Newton iteration on stderr */
  int32_t coarse_every;  /* coarse = 3, 4: the coarse operator E = Z^T J Z
                            and its inverse are rebuilt at the first Newton
                            iterate, after an update whose largest
                            relative change of an unknown exceeded 2, and
                            every coarse_every iterates (0:
                            default 3; 1: every iterate); the element blocks
                            are rebuilt at every iterate */
  int32_t limiter;       /* 1: every converged step's root (and, with H211b,
                            the extrapolated state) is limited by dg_limit;
                            the multiplicative Newton update is then capped
                            from above only, so that a concentration can fall
                            to zero and continue additively (roots with
                            negative nodal values are reached before
                            limiting).  0 (default): no limiter */
  int32_t mg_levels;     /* coarse = 3, 4: 0 solves the coarse system
                            exactly (dense LU); 2..8 replaces that
                            solve by one V-cycle over mg_levels levels of
                            nested voxel aggregates (the multigrid stand-in
                            for Sec. 2.9's algebraic multigrid): level 1 has
                            aggregates of coarse_agg voxels per edge (0: 4),
                            each further level groups 2 x 2 x 2 aggregates
                            of the one above, operators are Galerkin
                            products, the last level (at most 8192
                            unknowns) is solved exactly; see dg_mg_setup.
                            -1 (default): automatic -- 0 while
                            aggregates of coarse_agg voxels per edge (0:
                            8) give at most 8192 coarse unknowns, else
                            level-1 aggregates of coarse_agg (0: 4) voxels
                            and the fewest levels whose last has at most
                            4096 unknowns (3 on the 96 x 96 x 192 slab) */
  int32_t mg_sweeps;     /* damped block-Jacobi sweeps before and after each
                            coarse correction of the cycle, 0..8 (default 3) */
  double mg_omega;       /* their damping, in (0, 1] (default 0.7) */
  double block_reuse;    /* > 0 (default 1): the element blocks are built
                            at the first Newton iterate and rebuilt after an
                            update whose largest relative change of an
                            unknown exceeded block_reuse (the blocks of an
                            earlier iterate precondition the later ones;
                            only the preconditioner changes, not the root);
                            0: rebuilt at every iterate */
} dg_solver_opts;

void dg_solver_opts_default(dg_solver_opts* o);

/* ---- Multilevel coarse correction (multigrid for the elliptic coupling) ----
 *
 * The paper preconditions its Krylov solves with algebraic multigrid,
 * tuned for the potential coupling (Sec. 2.9).  Here the coarse correction
 * of the element block-Jacobi preconditioner can be a V-cycle over nested
 * voxel aggregates (dg_solver_opts.mg_levels); these two calls expose that
 * cycle on its own, with unit basis weights:
 *   Z (fine -> level 1): 1 on every node of a field's aggregate;
 *   P_l (level l+1 -> l): 1 from a parent aggregate to each of its
 *     (up to) 2 x 2 x 2 children; coarse vectors are (field, aggregate),
 *     aggregates x fastest;
 *   E_1 = Z^T J Z with J the condensed 7-field tangent at u (the Krylov
 *     operator, DG_JVP_LINEARIZED7), E_{l+1} = P_l^T E_l P_l;
 *   V-cycle: on every level but the last, opts->mg_sweeps damped
 *     block-Jacobi sweeps x <- x + mg_omega D^-1 (b - E x) from x = 0 (D:
 *     the 7 x 7 blocks of one aggregate's fields), the next level's cycle on
 *     P^T (b - E x), its prolongation added, mg_sweeps more sweeps; the
 *     last level solved exactly (FP64 LU of the equilibrated operator).
 * Level operators and vectors are FP64 whatever prec is.
 *
 * dg_mg_setup: linearises at u (as dg_linearize, precision prec; u: 9
 * fields) and builds the hierarchy for opts->mg_levels (2..8) levels with
 * level-1 aggregates of opts->coarse_agg voxels per edge (0: 4).  Replaces
 * the stored linearisation.  Q1 only.  Synchronises the stream.  Errors:
 * DG_EINVAL (null array, dt <= 0, bad precision or options, a last level
 * of more than 1024 aggregates: it is solved densely with 8 unknowns per
 * aggregate, the seven fields and a zero pad), DG_EUNSUPPORTED (order !=
 * 1), DG_ENOMEM, DG_ENAN (singular last level), DG_EHIP.  A later solve
 * (dg_step, dg_initial_state, dg_advance) that runs the multilevel cycle
 * reuses these buffers and ends this hierarchy's validity.
 *
 * dg_mg_apply: out = Z V_1(Z^T r) for 7-field vectors r, out of precision
 * prec (that of the setup); out is overwritten.  Errors: DG_EINVAL (null
 * array, other precision), DG_ESTATE (no current dg_mg_setup). */
int dg_mg_setup(dg_ctx* ctx, dg_prec prec, const void* u, double t_new, double dt, const dg_solver_opts* opts,
                dg_stream stream);
int dg_mg_apply(dg_ctx* ctx, dg_prec prec, const void* r, void* out, dg_stream stream);

/* The operator E_level (level 1..mg_levels) of the current dg_mg_setup
 * hierarchy, copied to the device array out of n >= 343 na doubles (na:
 * the level's aggregates), as seven 7 x 7 blocks per aggregate:
 * out[((s 7 + g) 7 + f) na + a] = E[(g, a), (f, neighbour s of a)], slots
 * s = itself, -x, +x, -y, +y, -z, +z (zero where the neighbour lies
 * outside).  Errors: DG_EINVAL (null array, level, n too small), DG_ESTATE
 * (no current setup). */
int dg_mg_export(dg_ctx* ctx, int32_t level, double* out, int64_t n, dg_stream stream);

/* ---- Caller-owned device workspace ----
 *
 * A context set up with dg_setup_ws takes every device buffer it will use
 * -- phase map, linearisation, element blocks, Krylov basis, Newton
 * vectors, coarse space, controller states, output partial sums and the
 * rocSOLVER scratch of the coarse LU -- from one caller-owned device
 * workspace, carved at set-up; no later call allocates device memory, and
 * dg_destroy frees only the host object.  What the workspace must hold
 * depends on the uses it is sized for (features, a DG_WS_* mask) and on
 * the solver options (inner precision, restart length, coarse space,
 * bfloat16 inverses).  A call outside those uses (an FP64 block setup on a
 * workspace sized for FP32 inner solves, a longer restart, the H211b
 * controller without DG_WS_H211B) returns DG_ENOMEM, and dg_last_error()
 * says how many bytes the workspace lacks.  The batch entry points
 * (dg_batch_*) allocate their own storage. */
typedef enum {
  DG_WS_OPERATORS = 1,  /* dg_mass, dg_residual, dg_jvp, dg_linearize, dg_outputs */
  DG_WS_BLOCKS = 2,     /* dg_blockjacobi_setup/apply/export in opts->inner_prec (k = 1, 3) */
  DG_WS_STEP = 4,       /* dg_step, dg_initial_state with opts */
  DG_WS_NAIVE = 8,      /* dg_advance, naive controller (one saved state) */
  DG_WS_H211B = 16,     /* dg_advance, H211b (three saved states) */
  DG_WS_LIMITER = 32,   /* dg_limit (implied for steps when opts->limiter = 1) */
  DG_WS_MG = 64,        /* dg_mg_setup/apply with opts->mg_levels, coarse_agg */
  DG_WS_ALL = 127
} dg_workspace_use;

/* Bytes of device workspace a dg_setup_ws context of this mesh needs for
 * the uses in `features` with solver options opts (NULL: defaults).  Host
 * call (it queries rocSOLVER for the scratch of the coarse LU).  The
 * slab of 96 x 96 x 192 voxels with FP32 inner solves, bfloat16 inverses
 * and the naive controller needs about 60 GB.  Errors: DG_EINVAL (null
 * pointer, mesh, unknown feature bits, bad options); DG_EUNSUPPORTED for
 * uses beyond DG_WS_OPERATORS at order 0 and beyond DG_WS_OPERATORS |
 * DG_WS_BLOCKS at order 3. */
int dg_workspace_bytes(const dg_mesh* mesh, const dg_params* params, const dg_solver_opts* opts,
                       int32_t features, size_t* bytes);

/* As dg_setup (Sec. 2.2-2.6 problem, Tab. 5 parameters, Eq. 57 phases),
 * with every device buffer of the context carved from `workspace`: device
 * memory of ws_bytes bytes, 256-byte aligned, owned by the caller, which
 * must outlive the context and is never freed by the library.  The phase
 * map is copied on `stream` (synchronised before return).  opts and
 * features as for dg_workspace_bytes; the same values must be passed here.
 * Errors: as dg_setup; DG_EINVAL for a null or misaligned workspace;
 * DG_ENOMEM when ws_bytes is too small (the message gives the shortfall). */
int dg_setup_ws(const dg_mesh* mesh, const uint8_t* phase, const dg_params* params, const dg_solver_opts* opts,
                int32_t features, void* workspace, size_t ws_bytes, dg_stream stream, dg_ctx** out);

typedef struct {
  int32_t newton_its, gmres_its, line_search_cuts, status;
  int32_t stalled;        /* 1: stopped because full steps no longer shrank the
                             update (below 1e-7): the attainable accuracy */
  int32_t mg_levels;      /* levels of the multilevel coarse correction the
                             solve used (0: none; see dg_solver_opts) */
  double merit0;          /* preconditioned scaled residual norm at the start */
  double merit_final;     /* ... after the last accepted update */
  double last_update;     /* largest relative change of the last update */
  double gmres_last_rel;  /* relative GMRES residual of the last solve */
  int32_t block_builds;   /* element-block assemblies and inversions */
  int32_t pad2;
} dg_step_report;

/* One backward-Euler step (Eq. 50) from t_n to t_n + dt: on entry u holds
 * u^n (device, FP64, 9 fields), on exit the Newton root u^{n+1} of
 * dg_residual (T_H at t_n + dt).  Newton's method in FP64 with a backtracking
 * line search (the paper uses PETSc newtonls, Sec. 2.9); positive unknowns
 * are updated multiplicatively (Newton in their logarithms).  Each linear
 * solve is GMRES(m) on the condensed 7-field Jacobian, scaled by the unknown
 * magnitudes and preconditioned by the element blocks plus a coarse
 * correction (opts.coarse: an exact two-level solve, or the multigrid
 * V-cycle of opts.mg_levels), in the inner precision of opts (NULL:
 * defaults).  The operator is rebuilt at every Newton iterate, the element
 * blocks at the first and after large updates (opts.block_reuse), the
 * coarse operator every opts.coarse_every iterates and after large
 * updates.  Device workspace is allocated on first use and kept (a
 * context of dg_setup_ws takes it from the caller's workspace).
 * Converged when a full step changes no unknown by more than newton_tol,
 * or, once an update below 1e-7 has been reached (the attainable accuracy
 * of the iterative solve; report.stalled = 1), when three full steps in a
 * row (six with DG_F32 inner solves, whose refinement contracts more
 * slowly) fail to halve the update, when the linear solve stagnates above
 * its tolerance, or when the line search finds no decrease.
 * Synchronises the stream.  DG_ENOCONV: u holds the last iterate and the
 * report is filled; the controller halves dt (Sec. 2.8).  DG_ENAN: non-finite
 * residual. */
int dg_step(dg_ctx* ctx, double t_n, double dt, void* u, const dg_solver_opts* opts,
            dg_step_report* report, dg_stream stream);

/* Initial state (Tab. InitialState, Sec. 2.10): u (device, FP64, 9 fields)
 * is set to the chemical-equilibrium concentrations, the phase's solid
 * fractions and the electrolyte potential of the steady charge balance at
 * time t0: the charge rows of dg_residual are solved for Phi_L with the
 * concentrations and solid fractions frozen and the full current applied.
 * (The paper reaches the same fixed point by relaxing a pseudo-transient
 * potential problem under a ramped current.)  The solve is the Newton-GMRES
 * of dg_step restricted to Phi_L (opts and report as there).  Synchronises
 * the stream.  Errors as dg_step. */
int dg_initial_state(dg_ctx* ctx, double t0, void* u, const dg_solver_opts* opts,
                     dg_step_report* report, dg_stream stream);

/* Battery outputs of a state u (device, FP64, 9 fields) at time t (the
 * time enters the reaction current through T_H).  Any output pointer may
 * be NULL.  Host results:
 *   U_cell      cell voltage [V]: the anode Butler-Volmer law (Eq. 27,
 *               k_E,Ano = 5e-3 mol/(s m^2), U0_Ano = 0) inverted in closed
 *               form at each separator-face point, V - Phi_L - (2RT/F) ln y,
 *               averaged over the separator face (App. A);
 *   means[10]   volume averages of the nine unknowns and of the dissolved
 *               sulfur c_S (Eq. A3);
 *   sums[4]     sulfur atoms, lithium atoms, stored electrons [mol] and the
 *               reaction current [A], with the nodal quadrature of the time
 *               terms (at a step root the current equals j_el times the
 *               separator area, and the atom counts change only by the
 *               separator flux).
 * Synchronises the stream. */
int dg_outputs(dg_ctx* ctx, const void* u, double t, double* U_cell, double* means, double* sums,
               dg_stream stream);

/* dg_outputs for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same results, bit for bit, with no device allocation.
 * Its partial sums live in a library-owned static device array of
 * 15 x 1024 + 15 doubles (123 KB), which every GPU the library runs on
 * holds until the process ends; the array's need does not grow with the
 * mesh (a fixed grid of 1024 blocks strides over any number of nodes), so
 * no size limit applies beyond those of dg_outputs.  Every call on one GPU
 * shares that GPU's array and overwrites all of it before reading it:
 * calls that overlap on one GPU (concurrent streams or host threads) race
 * and must be serialised by the caller.  Arguments, results and errors as
 * dg_outputs; synchronises the stream. */
int dg_outputs_noalloc(dg_ctx* ctx, const void* u, double t, double* U_cell, double* means, double* sums,
                       dg_stream stream);

/* Adaptive time control (Sec. 2.8). */
typedef enum { DG_CTRL_NAIVE = 0, DG_CTRL_H211B = 1 } dg_controller_kind;

typedef struct {
  int32_t kind;          /* dg_controller_kind */
  int32_t max_halvings;  /* consecutive halvings before DG_ENOCONV (30) */
  int32_t successes;     /* naive: converged steps before the step grows (3) */
  int32_t sct;           /* naive: success counter (state) */
  double dt;             /* size of the next trial step [s] (state) */
  double dt_max;         /* cap on the step size [s] (100) */
  double grow;           /* naive growth factor (1.2) */
  double tol;            /* H211b tolerance on the relative step error */
  double err_prev;       /* H211b history (state): error of the last accepted step */
  double dt_prev;        /* H211b history (state): its step size */
} dg_controller;

/* Controller with the paper's settings, first trial step dt0 and (H211b)
 * tolerance tol; before the first accepted step err_prev = tol and
 * dt_prev = dt0. */
void dg_controller_init(dg_controller* c, int32_t kind, double dt0, double tol);

typedef struct {
  double dt;             /* size of the accepted step [s] */
  double err;            /* H211b: relative error of the accepted step (0 for naive) */
  int32_t trials;        /* trial steps (H211b: coarse + two fine solves each) */
  int32_t halvings;      /* solver failures answered by halving dt */
  int32_t newton_its;    /* over all solves of this call */
  int32_t gmres_its;
} dg_advance_report;

/* One accepted step of the controller c from time *t: on return u holds the
 * state at *t (advanced by report.dt) and c its updated state.
 * Naive: backward-Euler step of size c->dt; a failed solve halves dt and
 * retries (the success counter restarts); after `successes` converged steps
 * in a row dt grows by `grow`, capped at dt_max.
 * H211b (Eq. 51-54): one coarse step (dt) and two fine steps (dt/2);
 * err = ||z_F - z_C||_2 / ||z_F||_2 over all unknowns; rho = (tol/err)^(1/4)
 * (tol/err_prev)^(1/4) (dt/dt_prev)^(-1/4), lim = 1 + atan(rho - 1); the
 * trial is repeated with dt <- min(lim, 0.9) dt while err > 1.02 tol or
 * lim < 0.9; on acceptance u = 2 z_F - z_C and the next dt is
 * min(lim dt, dt_max).  A failed solve inside a trial halves dt.
 * Non-convergence and non-finite residuals count as failed solves; after
 * more than max_halvings in one call, or (H211b) more than 100 trials
 * rejected by their error (an error estimate whose floor lies above tol):
 * DG_ENOCONV with u and *t unchanged (c->dt keeps the last trial size).
 * Device workspace: up to three extra FP64 states, kept.  Synchronises the
 * stream. */
int dg_advance(dg_ctx* ctx, dg_controller* c, double* t, void* u, const dg_solver_opts* opts,
               dg_advance_report* report, dg_stream stream);

/* ---- Batches: many structures of uneven size, one launch per operator ----
 *
 * A batch holds n independent voxel structures (each set up as by dg_setup
 * with its own mesh, phase map and parameters, so its own applied current,
 * Eq. 57 localisation and App. C loading).  Batch arrays concatenate the
 * structures voxel by voxel in the field-major layout a[f][E][n]: E is the
 * total voxel count, structure s owns voxels [off[s], off[s+1]) in its own
 * x-fastest order, n = 0..7 the Q1 node.  Every operator runs as one launch
 * over work items of 32 voxels of one structure (the residual and tangents
 * in a tunable shape: dg_batch_shape) and gives, structure by
 * structure, the values of the single-structure call (dg_mass, dg_residual,
 * dg_jvp, dg_linearize, dg_blockjacobi_*) on that structure's slice.
 * t_new and dt are HOST arrays of n values (each structure steps on its own
 * clock).  Parameter blocks are staged through library-owned pinned memory;
 * calls on one batch must not overlap (they share that staging, the
 * linearisation and the block storage).  The batch workload these serve is
 * the configuration of many microstructures solved side by side; the
 * operators are those of Eq. 43-47 and 50 as for one structure. */
typedef struct dg_batch dg_batch;

/* n >= 1 structures: meshes[n], phases[n] (HOST arrays of nx*ny*nz bytes,
 * copied), params[n] (copied).  Errors as dg_setup, for the first structure
 * that fails (named in dg_last_error). */
int dg_batch_setup(int32_t n, const dg_mesh* meshes, const uint8_t* const* phases,
                   const dg_params* params, dg_batch** out);

/* Free the batch and its device storage. */
int dg_batch_destroy(dg_batch* b);

/* Voxel offsets off[0..n] (HOST array of n + 1 values; off[n] = E) and the
 * number of work items (may be null). */
int dg_batch_layout(const dg_batch* b, int64_t* offsets, int64_t* n_tiles);

/* dg_mass of every structure.  u: device, 9 x E x 8; m: device, 8 x E x 8. */
int dg_batch_mass(dg_batch* b, dg_prec prec, const void* u, void* m, dg_stream stream);

/* dg_residual of every structure (t_new[s], dt[s] > 0).  u, r: 9 x E x 8;
 * m_old: 8 x E x 8 (dg_batch_mass of the old states). */
int dg_batch_residual(dg_batch* b, dg_prec prec, const void* u, const void* m_old, const double* t_new,
                      const double* dt, void* r, dg_stream stream);

/* dg_linearize of every structure into the batch's own storage. */
int dg_batch_linearize(dg_batch* b, dg_prec prec, const void* u, const double* t_new, const double* dt,
                       dg_stream stream);

/* dg_jvp of every structure; modes and shapes as dg_jvp with E voxels.
 * DG_ESTATE: DG_JVP_LINEARIZED7 without a batch linearisation of that
 * precision. */
int dg_batch_jvp(dg_batch* b, dg_prec prec, dg_jvp_mode mode, const void* u, const void* v,
                 const double* t_new, const double* dt, void* jv, dg_stream stream);

/* dg_blockjacobi_setup of every structure: E condensed 56 x 56 inverses in
 * batch-owned device memory (also stores the linearisation at u).
 * Synchronises the stream; DG_ENAN if any block is singular or not finite. */
int dg_batch_blockjacobi_setup(dg_batch* b, dg_prec prec, const void* u, const double* t_new,
                               const double* dt, dg_stream stream);

/* y = B^-1 x for every voxel of the batch (7 x E x 8, precision of the
 * setup).  DG_ESTATE before a setup. */
int dg_batch_blockjacobi_apply(dg_batch* b, dg_prec prec, const void* x, void* y, dg_stream stream);

/* Launch shapes of the batched residual and tangents.  A work item is a
 * tile of tile_voxels voxels of one structure (8 lanes per voxel, so 64,
 * 128 or 256 lanes per workgroup).  persistent = 0 launches one workgroup
 * per work item; persistent = k > 0 launches k workgroups per compute unit
 * (rounded down to a multiple of 8, at least 8, at most one per work item),
 * each looping over work items in a fixed stride, so every workgroup ends.
 * Among the tile shapes only the workgroup that computes a node changes:
 * their results are the same.  The condensed tangent also has the brick
 * shape {64, 0}: one 512-lane workgroup per brick of 4 x 4 x 4 voxels of a
 * structure, each inner face evaluated once, as dg_jvp's Krylov operator;
 * it gives every structure dg_jvp's values on it, and differs from the
 * tile shapes by rounding only.  Defaults: {64, 0} for the condensed
 * tangent, {32, 0} for the others, unless dg_batch_autotune has run in this
 * process on a batch of the same precision and size class (the bit length
 * of E), whose choice a new batch starts from. */
typedef struct dg_batch_shape {
  int32_t tile_voxels; /* 8, 16 or 32; 64 (bricks, condensed tangent only) */
  int32_t persistent;  /* 0, or workgroups per compute unit in [1, 64] (tiles) */
} dg_batch_shape;

/* Batched operators whose launch shape is tunable. */
typedef enum dg_batch_op {
  DG_BOP_RESIDUAL = 0,      /* dg_batch_residual */
  DG_BOP_JVP_FULL9 = 1,     /* dg_batch_jvp, DG_JVP_FULL9 */
  DG_BOP_JVP_CONDENSED7 = 2 /* dg_batch_jvp, DG_JVP_CONDENSED7 and DG_JVP_LINEARIZED7 */
} dg_batch_op;

typedef struct dg_batch_tuning {
  dg_batch_shape shape[3]; /* chosen shape, by dg_batch_op */
  double ms[3];            /* mean time per launch in that shape */
  double ms_default[3];    /* mean time per launch in the operator's default shape */
  int32_t candidates;      /* tile shapes timed per operator (6, or 3 without occupancy
                              data); the condensed tangent also times the brick shape */
  int32_t pad;
} dg_batch_tuning;

/* Set or read the launch shape of operator op (a dg_batch_op) in precision
 * prec.  DG_EINVAL for an unknown op or precision, tile_voxels outside
 * {8, 16, 32} (or 64 for the condensed tangent, with persistent = 0) or
 * persistent outside [0, 64]. */
int dg_batch_set_shape(dg_batch* b, dg_prec prec, int32_t op, const dg_batch_shape* shape);
int dg_batch_get_shape(const dg_batch* b, dg_prec prec, int32_t op, dg_batch_shape* shape);

/* Autotuner: times the three tunable operators on these arrays in every
 * launch shape (tile sizes 8, 16 and 32, each with one workgroup per work
 * item and as a persistent grid at the occupancy the compiled kernel
 * allows; bricks for the condensed tangent), reps launches each after one warm-up (reps <= 0: 5; at most
 * 1000), keeps the fastest shape per operator for this batch and for later
 * batches of its precision and size class, and fills report.  u, v: device,
 * 9 x E x 8 (the condensed tangent reads v's first 7 fields); m_old: device,
 * 8 x E x 8; work: device, 9 x E x 8, overwritten.  Leaves the batch
 * linearisation at u.  Synchronises the stream. */
int dg_batch_autotune(dg_batch* b, dg_prec prec, const void* u, const void* v, const void* m_old,
                      const double* t_new, const double* dt, void* work, int32_t reps,
                      dg_batch_tuning* report, dg_stream stream);

/* Initial state (as dg_initial_state, at t0[s]) of every structure into the
 * batch state u (device, FP64, 9 x E x 8).  The structures' solves run side
 * by side on `workers` host threads (<= 0: 4), each with a HIP stream of its
 * own and a library-owned contiguous state of the largest structure; each
 * structure's result is that of dg_initial_state on it.  reports: HOST array
 * of n (may be null).  Synchronises `stream` first (u may be written on it)
 * and returns when every structure is done.  The first failing structure
 * (in structure order) gives the status, named in dg_last_error; the other
 * structures are still solved. */
int dg_batch_initial_state(dg_batch* b, const double* t0, void* u, const dg_solver_opts* opts,
                           dg_step_report* reports, int32_t workers, dg_stream stream);

/* One backward-Euler step of every structure, from t_n[s] by dt[s] (HOST
 * arrays of n): dg_step on each structure's slice of u (device, FP64,
 * 9 x E x 8), the solves side by side as in dg_batch_initial_state.  Each
 * structure's slice ends as dg_step leaves its state (the root, or the last
 * iterate on DG_ENOCONV); reports[s] is its dg_step report.  Errors: as
 * dg_step, for the first failing structure; DG_EINVAL for dt[s] <= 0. */
int dg_batch_step(dg_batch* b, const double* t_n, const double* dt, void* u, const dg_solver_opts* opts,
                  dg_step_report* reports, int32_t workers, dg_stream stream);

/* Vertex-based slope limiter of the Q1 state u (device, FP64, 9 fields),
 * in place: Kuzmin's limiter, which the paper's DG1 runs use (App. B.1,
 * B.2), applied to the conserved densities m_i = eps_L c_i of the six
 * dissolved species so that every voxel keeps the amount of each species.
 * Each voxel's deviation from its mean of m_i is scaled by the largest
 * alpha in [0, 1] that keeps the corner values of its trilinear polynomial
 * between the smallest and largest voxel mean at each corner vertex; then
 * c_i = m_i / eps_L.  Every limited nodal value lies within the means of
 * the voxels around it, so non-negative means give a non-negative state
 * (the positivity-preserving p = 1 scheme of the paper's outlook, Sec. 4).
 * Phi_L and the solid fractions are not changed.  alpha: optional device
 * array (FP64, 6 x n_elem, species-major) that receives the factors, or
 * NULL.  Order 0: no-op; order 3: DG_EUNSUPPORTED (Kuzmin's hierarchical
 * form for degree above 1 is not implemented).  Enqueued on `stream`;
 * device workspace of
 * 48 bytes per voxel, allocated on first use and kept (DG_WS_LIMITER on a
 * workspace context). */
int dg_limit(dg_ctx* ctx, void* u, void* alpha, dg_stream stream);

/* Measurement: the STREAM triad out[i] = a[i] + s b[i] (McCalpin's
 * bandwidth benchmark) for i < n, on device arrays of doubles, enqueued on
 * `stream`.  It moves 24 bytes per element through HBM, so its rate bounds
 * what a streaming kernel of this library can reach.  The arrays must be
 * 16-byte aligned and n even (DG_EINVAL otherwise); out must not overlap
 * a or b.  n = 0 is a no-op. */
int dg_triad(double* out, const double* a, const double* b, double s, int64_t n, dg_stream stream);

/* Human-readable description of the last error on this thread. */
const char* dg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LSBDG_H */
