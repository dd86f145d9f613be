/*
 * pd_fcbm.h -- C ABI of the MI355X-native fast convolution-based method with
 * embedded constraints (FCBM-EC) for peridynamics.
 *
 * The library evaluates nonlocal peridynamic integrals as FFT convolutions
 * (Jafarzadeh, Mousavi, Larios, Bobaru, "A general and fast convolution-based
 * method for peridynamics", Sec. 3 and 4): the bond sums of the one-point
 * quadrature (Eq. 55) are computed as circular convolutions on a periodic box
 * that encloses the body with at least one horizon of padding (Sec. 4.2.2),
 * the masks chi_B / chi_Omega cut the bonds to the padding and carry the
 * volume constraints (Eq. 73-75, 83-84, 89).
 *
 * Conventions shared by every entry point
 *  - Fields live on the body box only (body_n[0] x body_n[1] x body_n[2]
 *    nodes, x fastest), component-major ("SoA"): f[c][z][y][x].  The body box
 *    occupies the low corner of the FFT grid; the remaining grid points are
 *    the padding and are never stored by the caller.
 *  - Vector fields have `dim` components, scalar fields one.
 *  - Floating-point fields have the plan's dtype (float for PD_F32, double
 *    for PD_F64), except where an entry point states FP64 explicitly.
 *  - Field pointers passed to per-call entry points are DEVICE pointers owned
 *    by the caller (e.g. PyTorch tensors); plan-time inputs (masks) are HOST
 *    pointers and are copied.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Calls enqueue work
 *    on that stream and return without waiting, except where a status needs
 *    device data (PD_ENUMERIC, PD_ENOTCONV and the solver info), which the
 *    call obtains by synchronising the stream.
 *  - A plan owns its spectra, static fields and FFT workspaces: calls that
 *    use the same plan must not run concurrently (they share workspaces).
 *  - No entry point aborts; every error is returned as a pd_status and the
 *    outputs are then unspecified.
 */
#ifndef PD_FCBM_H
#define PD_FCBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pd_plan_s* pd_plan;

typedef enum {
    PD_OK = 0,
    PD_EINVAL = 1,        /* invalid argument (sizes, padding, null pointer, dt) */
    PD_ENOMEM = 2,        /* device allocation failed */
    PD_EDEVICE = 3,       /* a HIP runtime call failed */
    PD_ENOTCONV = 4,      /* iterative solver reached maxit */
    PD_ENUMERIC = 5,      /* NaN or Inf detected */
    PD_EUNSUPPORTED = 6   /* valid request the library does not implement */
} pd_status;

typedef enum { PD_F32 = 0, PD_F64 = 1 } pd_dtype;

typedef enum {
    PD_BB_LINEAR = 0,     /* linearized bond-based solid, Eq. 17-18 */
    PD_LPS_LINEAR = 1,    /* linearized state-based (LPS) solid, Eq. 33-39, 3D only */
    PD_BB_NONLINEAR = 2   /* nonlinear, rotation-invariant bond-based solid,
                             Eq. 19-20 in the convolution form of Eq. 21-26;
                             same micromodulus constant alpha as PD_BB_LINEAR
                             (it is the small-displacement limit); pd_force only,
                             PD_WEIGHT_NONE */
} pd_model;

typedef enum {
    PD_WEIGHT_NONE = 0,       /* bond weight chi_B chi_B' (Eq. 75) */
    PD_WEIGHT_INTEGRITY = 1,  /* chi_B lambda chi_B' lambda' with a uint8 integrity
                                 lambda per node (Eq. 44, 46, 100); enables the
                                 energy failure rule W <= G0/delta (Eq. 40, 51, 63) */
    PD_WEIGHT_SCALE = 2       /* chi_B s chi_B' s' with a floating s per node:
                                 heterogeneous micromodulus c0 s(x) s(x'),
                                 s = sqrt(c(x)/c0) */
} pd_weight_kind;

typedef struct {
    int dim;              /* 2 or 3 */
    int64_t fft_n[3];     /* FFT grid (x, y, z): y and z powers of two in [16, 1024];
                             x in [16, 2048], a power of two or 2 R 2^p with
                             R = 3, 5 or 9 and 2^p >= 8 (minimum padding, Sec.
                             4.2.2); fft_n[2] = 1 when dim == 2 */
    int64_t body_n[3];    /* body box (x, y, z), >= 1; body_n[2] = 1 when dim == 2.
                             Requires fft_n[d] - body_n[d] >= ceil(delta/dx[d]) so
                             that no bond wraps around the periodic box (Sec. 4.2.2:
                             the body must sit at least one horizon from the box edge) */
    double dx[3];         /* node spacing (m); dx[2] ignored when dim == 2 */
} pd_grid;

typedef struct {
    double delta;         /* horizon radius (m); bonds o*dx with |o*dx| <= delta
                             (relative slack 1e-10 so grid points on the horizon
                             sphere count as inside) */
    int influence;        /* 0: omega = 1/|xi| (the paper's choice), 1: omega = 1 */
} pd_horizon;

typedef struct {
    pd_model model;
    double E;             /* Young modulus (Pa) */
    double nu;            /* Poisson ratio (LPS; bond-based is fixed at 1/3 plane
                             stress in 2D and 1/4 in 3D and ignores this) */
    double rho;           /* mass density (kg/m^3), used by pd_verlet_step */
    double G0;            /* critical energy release rate (J/m^2); with
                             PD_WEIGHT_INTEGRITY the failure threshold is
                             W_c = G0/delta (Eq. 51); 0 disables failure */
    pd_weight_kind weight;
} pd_kernel;

typedef struct {
    const uint8_t* chi_B;      /* HOST, body box, 1 = node belongs to the body B
                                  (Eq. 73); NULL = every body-box node */
    const uint8_t* chi_Omega;  /* HOST, [dim][body box], 1 = component is an unknown
                                  (Eq. 74), 0 = prescribed (Gamma_i); NULL = chi_B
                                  for every component */
} pd_mask;

/* plan flags */
#define PD_PLAN_MIXED 1   /* on a PD_F64 plan, also build the FP32 operator used by
                             the mixed-precision static solve */

typedef struct {
    int dim;
    int64_t body_nodes;       /* body-box nodes */
    int64_t fft_points;       /* FFT grid points */
    int stencil_size;         /* bonds per node of the full horizon */
    double alpha;             /* bond-based micromodulus constant (Eq. 17) */
    double m0;                /* full-horizon weighted volume sum omega r^2 dV */
    double Wc;                /* failure threshold G0/delta (0 if off) */
    double dt_max;            /* largest stable velocity-Verlet step for the periodic
                                 operator (2/sqrt(lambda_max/rho)) */
    int64_t workspace_bytes;  /* device memory held by the plan */
    int64_t lds_per_block;    /* LDS bytes a workgroup may use on this device */
} pd_plan_info;

/* Build a plan: validates sizes and padding, samples the kernels on the
 * horizon stencil (FP64), forms their partial spectra and the static
 * embedded-constraint fields (C*chi_B, a*chi_B, m; Eq. 56, 92-94, 97) and
 * allocates workspaces.  Returns PD_EINVAL for inconsistent sizes or
 * padding smaller than the horizon, PD_EUNSUPPORTED for the LPS model in 2D,
 * the nonlinear bond-based model with weights, or grid lengths
 * outside the supported set, PD_ENOMEM / PD_EDEVICE on HIP failures.  On
 * error *out is NULL.  Plans of the nonlinear bond-based model serve
 * pd_force (without W_out) only; the other operations return
 * PD_EUNSUPPORTED for them. */
pd_status pd_plan_create(const pd_grid* grid, const pd_horizon* horizon, const pd_kernel* kernel,
                         const pd_mask* mask, pd_dtype dtype, int flags, void* stream,
                         pd_plan* out);

/* Release every device buffer of the plan (synchronises its stream). NULL is a no-op. */
void pd_plan_destroy(pd_plan plan);

/* Sizes and constants of a plan. */
pd_status pd_plan_query(pd_plan plan, pd_plan_info* info);

/* Internal force density L (Eq. 57/58 for bond-based; Eq. 95-97 for LPS,
 * read with minus signs on the (C*chi) u, P u and (a*chi) u terms, which the
 * derivations imply and which make an affine field's interior force vanish;
 * Eq. 101 with weights; Eq. 21-26 for the nonlinear bond-based model).
 *   u      [dim][body]  displacement
 *   weight NULL for PD_WEIGHT_NONE; uint8 lambda [body] for INTEGRITY;
 *          dtype s [body] for SCALE
 *   L_out  [dim][body]  force density (N/m^3), zero outside chi_B
 *   W_out  [body] strain energy density (Eq. 102) or NULL; bond-based only
 * PD_EINVAL for NULL u/L_out or a weight that does not match the plan. */
pd_status pd_force(pd_plan plan, const void* u, const void* weight, void* L_out, void* W_out,
                   void* stream);

/* Adjoint of pd_force: for a cotangent g_bar on L,
 *   u_bar      [dim][body] = (dL/du)^T g_bar  (= L applied to g_bar; the
 *              operator is symmetric for fixed weights)
 *   weight_bar [body] = d<g_bar, L>/d weight, only for PD_WEIGHT_SCALE
 *              (NULL to skip); bond-based only.
 * Derived from Eq. 46/100 (the paper gives no adjoint). */
pd_status pd_force_adjoint(pd_plan plan, const void* u, const void* weight, const void* g_bar,
                           void* u_bar, void* weight_bar, void* stream);

/* Velocity-Verlet state (caller-owned DEVICE buffers of the plan dtype). */
typedef struct {
    void* u;           /* [dim][body] displacement */
    void* v;           /* [dim][body] velocity */
    void* F;           /* [dim][body] L(u) + b at the current time */
    void* W;           /* [body] strain energy density (INTEGRITY plans), else NULL */
    uint8_t* lambda;   /* [body] integrity (INTEGRITY plans), else NULL */
    void* s;           /* [body] micromodulus scale (SCALE plans), else NULL */
    int64_t step;      /* steps taken; 0 means F (and W) are not yet valid */
    int32_t flags;     /* PD_STATE_* bits (0 for the default) */
} pd_state;

/* pd_state.flags: every step of a pd_verlet_step call reads and writes
 * (v, F), so that a call of n steps equals n calls of one step bit for bit
 * (for callers that replay a trajectory step by step, such as checkpointed
 * adjoints). */
#define PD_STATE_EXACT_STEPS 1

/* Advance nsteps embedded-constraint velocity-Verlet steps (Eq. 67, 83-84):
 *   u <- chi_O [u + dt v + dt^2/(2 rho) F] + (1 - chi_O) w
 *   lambda <- lambda AND [W <= W_c]          (INTEGRITY with G0 > 0)
 *   F' <- L(u) + b   (W' <- W(u))
 *   v <- chi_O [v + dt/(2 rho) (F + F')]
 * When state->step == 0 the initial F (and W) are computed first.  Between
 * the steps of one call without energy_out and without PD_STATE_EXACT_STEPS
 * the half-step velocity v + dt/(2 rho) F is kept in state->v and state->F
 * is left as it was (the same steps regrouped, so inner steps neither read
 * nor write F); on return state->v and state->F hold v and F of the last
 * step.  A call of n steps then equals n calls of one step up to rounding,
 * not bit for bit; on an error return in the middle of such a call
 * state->v may hold the half-step velocity.
 *   b [dim][body] body force density or NULL (zero); w [dim][body] values
 *   on the constrained components or NULL (zero); both time independent.
 *   energy_out HOST FP64 [nsteps][4] or NULL: kinetic, internal
 *   -dV/2 <u, L>, external -dV <u, b>, and the shadow energy
 *   KE + PE + EXT - dt^2/(8 rho) dV |chi_O F|^2 that velocity Verlet
 *   conserves exactly for the linear undamaged operator; FP64 sums.
 * PD_EINVAL if dt <= 0 or dt > dt_max.  PD_ENUMERIC if a new force or
 * velocity value of any step became NaN or infinite: the velocity-update
 * epilogue raises a flag, which the call reads once after its last step (it
 * synchronises the stream for that), and with energy_out also if an energy
 * sum is not finite. */
pd_status pd_verlet_step(pd_plan plan, pd_state* state, const void* b, const void* w, double dt,
                         int nsteps, double* energy_out, void* stream);

/* Reverse-mode sweep of one embedded-constraint velocity-Verlet step (the
 * forward step of Eq. 67 with Eq. 83-84, differentiated by hand; the paper
 * gives no adjoint) with fixed weights, w = 0 and a time-independent body
 * force b.  With c1 = dt/(2 rho), c2 = dt^2/(2 rho), a = chi_O v_bar',
 * ut = chi_O (u_bar' + c1 L a):
 *   u_bar = c1 L a + ut + c2 L ut,   v_bar = a + dt ut,
 *   b_bar += c2 ut + 2 c1 a,
 *   s_bar += d/ds of c1 <a, L(u_n + u_np1)> + c2 <ut, L u_n>.
 *   u_n, u_np1  [dim][body] the states of steps n and n+1
 *   s           [body] micromodulus scale (SCALE plans, else NULL)
 *   u_bar, v_bar [dim][body] in: cotangents of step n+1; out: of step n
 *   s_bar       [body] accumulated (SCALE plans; NULL to skip)
 *   b_bar       [dim][body] accumulated cotangent of b (NULL to skip)
 * All DEVICE buffers of the plan dtype.  PD_EINVAL for NULL states or
 * cotangents; PD_EUNSUPPORTED for INTEGRITY plans.  Uses two
 * force-adjoint evaluations. */
pd_status pd_verlet_adjoint(pd_plan plan, const void* u_n, const void* u_np1, const void* s,
                            void* u_bar, void* v_bar, void* s_bar, void* b_bar, double dt, void* stream);

typedef struct {
    int iters_fp64;        /* FP64 CG iterations (FP64 solves) or FP64 residual
                              replacements (mixed) */
    int iters_fp32;        /* CG iterations with the FP32 operator (mixed) */
    int applies_fp64;      /* FP64 operator applications */
    int applies_fp32;      /* FP32 operator applications */
    double rel_res;        /* final |chi_O (L(u) + b)|_2 / |rhs|_2 in FP64 */
    int precond_applies;   /* preconditioner applications (PD_SOLVE_PRECOND) */
} pd_solve_info;

/* pd_static_solve options (bit flags) */
#define PD_SOLVE_MIXED 1     /* FP32 operator, FP64 vectors / inner products /
                                residual replacement (plan built with PD_PLAN_MIXED) */
#define PD_SOLVE_PRECOND 2   /* spectral preconditioner */

/* Embedded-constraint statics (Eq. 85-89) by conjugate gradients on
 * A = -chi_O L chi_O (symmetric positive definite on the unknowns), to the
 * relative residual rtol.  b, w, u_inout are FP64 DEVICE buffers
 * [dim][body] regardless of the plan dtype; u_inout holds the initial guess
 * on entry and the solution (u = w on constrained components) on exit.
 * options = 0: plain FP64 CG (PD_F64 plan).
 * PD_SOLVE_MIXED (PD_F64 plan created with PD_PLAN_MIXED): CG iterations that
 *   apply the operator in FP32 to a search direction kept in FP32, with the
 *   iterate and residual updated and every inner product accumulated in
 *   FP64, and the residual replaced by the FP64 residual chi_O (L(u) + b)
 *   each time its norm has dropped tenfold and at convergence (refinement
 *   against the FP64 operator).
 * PD_SOLVE_PRECOND: preconditioned CG with z = chi_O M^-1 chi_O r, M the
 *   bond-based operator of the same kernel on the full periodic box without
 *   masks (its symbol Ĉ(0) - Ĉ(k), shifted by a quarter of its mean diagonal
 *   at the first nonzero wavenumber along x so that k = 0 is invertible),
 *   applied by transforms; in FP32 when combined with PD_SOLVE_MIXED.  Not a
 *   method of the paper: an option for the solve only.
 * The call returns when done (the host checks the residual norm of each
 * iteration one iteration late, so one more iteration than needed may run).
 * PD_ENOTCONV when maxit CG iterations did not reach rtol; PD_ENUMERIC when a
 * residual norm is not finite (e.g. a NaN in b); PD_EINVAL for unknown option
 * bits. */
pd_status pd_static_solve(pd_plan plan, const void* b, const void* w, void* u_inout, double rtol,
                          int maxit, int options, pd_solve_info* info, void* stream);

/* pd_static_solve for callers that cannot allocate device memory during the
 * call (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same solve, bit for bit, with its vectors (FP64
 * residual and constraint fields, search direction, operator output,
 * preconditioned residual; FP32 copies for the mixed solve) taken from a
 * 256 MiB device array that the library holds on each GPU it runs on until
 * the process ends, instead of hipMalloc / hipFree per call.  The plan's
 * workspaces are allocated at plan creation as for every other call.
 * Capacity: 40 B per unknown for PD_SOLVE_PRECOND in FP64, 32 B plain FP64,
 * 28 B or 24 B mixed (with or without PD_SOLVE_PRECOND); about 6.7 million
 * unknowns (a 128^3 body in 3D) in every variant.
 * Arguments, results and status codes as pd_static_solve, plus PD_EINVAL
 * when the solve needs more than the array holds, when the current device is
 * not the plan's, or while pass timing (pd_profile_enable) is on.  Every
 * call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (from several host threads or streams) race and must be serialised by the
 * caller.  Nothing in the array needs to start at zero (every vector is
 * written before it is read), so no call clears it. */
pd_status pd_static_solve_noalloc(pd_plan plan, const void* b, const void* w, void* u_inout, double rtol,
                                  int maxit, int options, pd_solve_info* info, void* stream);

/* Damage index (Eq. 12 as Eq. 49/65): d = 1 - chi_B lambda cnt / beta with
 * cnt the number of intact partners within the horizon including the node
 * itself (convolution with the characteristic influence function omega_0,
 * Eq. 48, rounded to the nearest integer) and beta the node's family size
 * inside the body.  lambda uint8 [body], d_out plan dtype [body]. */
pd_status pd_damage_index(pd_plan plan, const uint8_t* lambda, void* d_out, void* stream);

/* Pass timing (measurement support).  While enabled, every kernel launch of
 * the plan (and of its FP32 sub-operator) is bracketed by two hipEvents
 * recorded on the launch stream, together with the pass's algorithmic HBM
 * bytes (what the pass must read and write: its spectral slabs, kernel
 * partial spectra and per-node fields, each once).  pd_profile_read waits
 * for the recorded events, aggregates them by pass name (e.g. "lastconv_4x3":
 * last-axis pass with 4 input and 3 output fields by direct correlation,
 * "lastmul_4x3" in the transform form; "xfwd_3", "ytf_512", "yti_512",
 * "xinv_3": the x and y transform passes), writes up to cap
 * records, sets *n_out to the number of distinct passes and clears the
 * record list.  Enabling adds two event records per launch. */
typedef struct {
    char name[32];
    int64_t launches;
    double total_ms;       /* summed event-measured duration */
    double bytes;          /* summed algorithmic bytes */
} pd_pass_time;

pd_status pd_profile_enable(pd_plan plan, int enable);
pd_status pd_profile_read(pd_plan plan, pd_pass_time* out, int cap, int* n_out);

/* Static description of a status code. */
const char* pd_status_str(pd_status status);

#ifdef __cplusplus
}
#endif

#endif /* PD_FCBM_H */
