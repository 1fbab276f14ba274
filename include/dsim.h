/*
 * dsim.h -- C ABI of the MI355X step-derivative library (gfx950, HIP).
 *
 * One time step of an articulated rigid-body system with frictional point
 * contacts on the ground plane, and its analytical derivatives, for a batch
 * of independent environments of possibly different sizes.
 *
 * The step (Section II.C, eq. 3-5; impulse form, Lam = dt * lambda):
 *     v_f = v + dt M(q)^-1 (tau - b(q, v))
 *     G   = J M^-1 J^T,  g = J v_f (+ phi / dt on normal rows, gap_mode 1)
 *     Lam solves the NCP of Section II.B (eq. NCP) for (G, g, mu)
 *     v+  = v_f + M^-1 J^T Lam
 * and its derivatives (Section III, eq. FD_grads, eq. 7-12, Appendix B and D):
 * d v+ / d(q, v, tau) through the mode-split reduced implicit system, or the
 * vector-Jacobian product of the same derivative (reverse mode, Section III.A).
 *
 * Conventions (fixed):
 *   - spatial layout of the model: see dsim_batch;
 *   - a free-flyer root has q = (position, quaternion x y z w) and
 *     v = (linear, angular) body-frame velocity; derivatives in q are taken
 *     along the tangent perturbation q (+) dq = q * Exp(dq) (n_v columns);
 *   - contacts: world-aligned frame (T1, T2, N) = (x, y, z), N = +z;
 *   - Lam is returned as an impulse (N s); divide by dt for forces;
 *   - gravity, dt and the gap mode travel in dsim_params.
 *
 * Memory and ownership: every pointer in dsim_batch and every array argument
 * is DEVICE memory owned by the caller (the library never allocates or frees
 * device memory, apart from kernel arguments).  Real arrays are float when
 * params->precision == DSIM_F32 and double when DSIM_F64; index arrays are
 * int32.  Buffers must stay valid until the work on `stream` has completed.
 * `stream` is a hipStream_t (NULL = the default stream); all compute calls are
 * asynchronous on it.  The derivative entries (outside graph capture, for a
 * batch without a launch list, and except dsim_step_vjp_noalloc) run part of
 * their work on a second stream
 * that the library creates once per device (default priority), forked from
 * and joined back to `stream` with events: the call's work is complete, and
 * its outputs ready, in `stream`'s order as for any other call.
 *
 * Errors: every call returns 0 (DSIM_SUCCESS) or a negative DSIM_ERR_* code
 * for invalid arguments, unsupported sizes or a failed launch; these are the
 * only synchronous errors.  Numerical trouble in one environment never fails
 * the call: it sets bits in that environment's status word (DSIM_ST_*) and the
 * outputs are still written.
 */
#ifndef DSIM_H
#define DSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DSIM_ABI_VERSION 4

/* return codes */
#define DSIM_SUCCESS 0
#define DSIM_ERR_ARG (-1)        /* null pointer, bad enum, negative size */
#define DSIM_ERR_SIZE (-2)       /* size beyond the supported maxima */
#define DSIM_ERR_LAUNCH (-3)     /* the HIP launch failed */
#define DSIM_ERR_WORKSPACE (-4)  /* workspace smaller than dsim_workspace_bytes */
#define DSIM_ERR_MODEL (-5)      /* dsim_validate_host: non-physical model */
#define DSIM_ERR_DEVICE (-6)     /* no usable gfx950 device */

/* per-environment status bits */
#define DSIM_ST_NCP_NOT_CONVERGED 1  /* FP64 natural-map residual above ncp_tol */
#define DSIM_ST_RANK_DEFICIENT 2     /* reduced system factorised with rank < m */
#define DSIM_ST_MODE_DEGENERATE 4    /* a contact within mode_eps of a mode switch */
#define DSIM_ST_NONFINITE 8          /* a NaN or Inf reached the outputs */
#define DSIM_ST_POLISH_FAILED 16     /* Newton refinement left the mode set */
#define DSIM_ST_SIZE_EXCEEDED 32     /* larger than the launch's max_* sizes: not computed */

/* contact modes written to `mode` (Section III.B) */
#define DSIM_MODE_BREAK 0
#define DSIM_MODE_STICK 1
#define DSIM_MODE_SLIDE 2

/* joint types */
#define DSIM_JOINT_REVOLUTE 0
#define DSIM_JOINT_FREEFLYER 1

/* supported maxima per environment */
#define DSIM_MAX_DOFS 64
#define DSIM_MAX_BODIES 64
#define DSIM_MAX_CONTACTS 21 /* 3 * contacts <= 64 */

typedef enum { DSIM_F64 = 0, DSIM_F32 = 1 } dsim_precision;

/* entry selector for dsim_workspace_bytes / dsim_lds_bytes */
typedef enum {
    DSIM_ENTRY_STEP = 0,
    DSIM_ENTRY_JACOBIAN = 1,
    DSIM_ENTRY_VJP = 2,
    DSIM_ENTRY_STEP_INTEGRATE = 3,
    DSIM_ENTRY_STEP_INTEGRATE_VJP = 4,
    DSIM_ENTRY_VJP_PARAMS = 5,
    DSIM_ENTRY_JACOBIAN_PARAMS = 6
} dsim_entry;

/*
 * A batch of kinematic trees (Section II.C) with point contacts.
 * Per-env ragged data is addressed by prefix offsets (n_env + 1 entries):
 *   bodies of env e are body_off[e] .. body_off[e+1]-1, likewise dofs (v, tau
 *   entries), configuration entries (q) and contacts.
 * Per body (bodies listed parents first inside each env):
 *   parent   int32, local index of the parent body, -1 = world
 *   jtype    int32, DSIM_JOINT_*; a free flyer may only be local body 0
 *   axis     real[3], unit joint axis in the joint frame (revolute)
 *   jrot     real[9], row-major rotation of the joint frame in the parent body
 *            frame (for the root: in the world frame)
 *   jpos     real[3], joint frame origin in the parent body frame
 *   mass     real, > 0
 *   com      real[3], centre of mass in the body frame
 *   inertia  real[6], rotational inertia about the COM in the body frame:
 *            xx yy zz xy xz yz
 * Per contact:
 *   cbody    int32, local body index
 *   cpoint   real[3], contact point in that body's frame
 *   mu       real, friction coefficient >= 0
 *   cradius  real, >= 0 (optional array: NULL means all 0): 0 makes cpoint
 *            a point of the body that touches the plane z = 0; r > 0 makes
 *            it the centre of a sphere of radius r fixed in the body, which
 *            touches the plane at its lowest point (a point that moves
 *            through the body as the body turns: the primitive-plane
 *            collision contribution of Appendix C enters the derivatives)
 * jac_off (n_env + 1 entries) is the prefix sum of n_v^2, the offsets of the
 * per-environment Jacobian blocks (needed by dsim_step_jacobian only; may be
 * NULL otherwise).
 * order (device, optional): when non-NULL, a launch processes only the
 *   n_order environments order[0 .. n_order-1] (indices into 0 .. n_env-1,
 *   in the order the hardware should start them; out-of-range entries are
 *   skipped).  With a sub-list the max_* fields need to bound only the listed
 *   environments: this is how a ragged batch is split into size classes
 *   (each launch sized for its class) and how expensive environments are
 *   started first.
 * pjac_off (device, n_env + 1 entries, optional): the prefix sum of
 *   n_v (7 n_b + n_c), the offsets of the per-environment parameter Jacobians
 *   of dsim_step_jacobian_params (may be NULL otherwise).
 * The max_* fields must bound every processed environment (they size the
 * on-chip buffers); n_env may be 0.
 */
typedef struct dsim_batch {
    int32_t n_env;
    int32_t max_bodies, max_dofs, max_cfg, max_contacts;
    const int32_t *body_off, *dof_off, *cfg_off, *contact_off, *jac_off;
    const int32_t *parent, *jtype, *cbody;
    const void *axis, *jrot, *jpos, *mass, *com, *inertia, *cpoint, *mu;
    int32_t n_order;
    const int32_t* order;
    const int32_t* pjac_off;
    const void* cradius;
} dsim_batch;

typedef struct dsim_params {
    double dt;            /* time step (s), > 0 */
    double gravity[3];    /* world gravity (m/s^2) */
    int32_t gap_mode;     /* 0: every contact touches (g = J v_f);
                             1: g_N += phi/dt with phi = world z of the point,
                             plus the Baumgarte terms of kp, kd (Appendix D) */
    int32_t precision;    /* dsim_precision */
    int32_t ncp_sweeps;   /* block Gauss-Seidel sweeps per round (>= 1) */
    int32_t ncp_rounds;   /* sweep rounds of the solve's first pass, each followed by
                             Newton refinement; an environment they leave unsolved
                             goes to the fallback pass (damped Newton on the
                             natural map, then ADMM, in FP64; Section II.B) */
    int32_t newton_iters; /* Newton iterations per refinement (>= 0) */
    int32_t threads;      /* threads per environment team: 64, 128, 256 or 512 (0 = auto: 128, and
                             512 for the derivative launch when max_dofs >= 24; 64 for the
                             derivative entries' contact-solve and fallback launches) */
    double ncp_tol;       /* relative natural-map residual tolerance */
    double rank_tol;      /* relative pivot tolerance of the reduced factorisation */
    double mode_eps;      /* relative threshold of the mode classification */
    double kp, kd;        /* Baumgarte gains of Appendix D, used in gap mode 1:
                             g_N += phi/dt - kp min(phi/dt, 0) - kd (J v)_N;
                             0 <= kp <= 1, kd >= 0 (defaults 0) */
} dsim_params;

/* fills `p` with the defaults for `precision` */
void dsim_default_params(dsim_params* p, int32_t precision);

int32_t dsim_abi_version(void);

/* sizeof(dsim_batch) for which == 0, sizeof(dsim_params) for which == 1
 * (0 otherwise): lets a binding check its mirror of the structs. */
size_t dsim_struct_size(int32_t which);
const char* dsim_error_string(int32_t code);

/*
 * Host-side validation of a batch whose pointers are HOST memory (no GPU
 * needed): offsets monotone, sizes within the maxima, parents listed first,
 * free flyer only at the root, unit axes and rotations, mass > 0, inertia
 * positive definite and satisfying the triangle inequality, mu >= 0.
 * Returns DSIM_SUCCESS, DSIM_ERR_ARG, DSIM_ERR_SIZE or DSIM_ERR_MODEL; the
 * first offending environment is written to *bad_env when bad_env != NULL.
 */
int32_t dsim_validate_host(const dsim_batch* host_batch, int32_t* bad_env);

/* Checks of the parameter block alone (host). */
int32_t dsim_validate_params(const dsim_params* params);

/* Bytes of device workspace the given entry needs for this batch: 0 for the
 * step entries; for the derivative entries (Jacobian, VJP, parameter
 * gradients and the rollout adjoint), which run the step launches, then the
 * derivative launches, the hand-over between them: each
 * environment's FP64 contact impulses and solver counts (DSIM_WS_ENV_DOUBLES doubles,
 * at the start of the workspace) and a record of the step's
 * quantities that the derivative reads (kinematics, inertias, M^-1, the
 * contact rows, the factorised reduced system, v+ and a+) and of the contact
 * system (G, g, v_f, a_f and the inverses of G's diagonal blocks) that the
 * step's first pass hands from its assembly launch to its contact-solve
 * launch, sized by the batch's max_* fields and the precision (about 42 KB
 * for 31 bodies, 36 dofs and 8 contacts in FP32).  The workspace is the caller's; it must not be
 * shared by calls that may run concurrently. */
size_t dsim_workspace_bytes(const dsim_batch* batch, const dsim_params* params, int32_t entry);

/* The workspace of a derivative entry starts with DSIM_WS_ENV_DOUBLES
 * doubles per environment (environment e at e * DSIM_WS_ENV_DOUBLES): its
 * FP64 contact impulses (3 n_c), then, from index DSIM_WS_WORK, the work its
 * contact solve executed in the call: Gauss-Seidel sweeps of the first pass,
 * Levenberg-Marquardt iterations and damped linear solves, and ADMM
 * iterations of the fallback pass (Section II.B solvers), then 1 if the first
 * pass left the environment to the fallback pass, else 0; as doubles.  Valid
 * after the call completes, until the workspace is reused. */
#define DSIM_WS_ENV_DOUBLES 68
#define DSIM_WS_WORK 63

/* Bytes of on-chip (LDS) storage one environment team uses for `entry`
 * (a dsim_entry).  A call whose team needs more than 160 KiB (the LDS of
 * one gfx950 compute unit) returns DSIM_ERR_SIZE. */
size_t dsim_lds_bytes(const dsim_batch* batch, const dsim_params* params, int32_t entry);

/*
 * The step (eq. 3-5 and the NCP).  Inputs q [sum n_q], v [sum n_v],
 * tau [sum n_v]; outputs v_next [sum n_v], lam [3 * sum n_c] (impulses,
 * (T1 T2 N) per contact), mode [sum n_c] (DSIM_MODE_*), status [n_env].
 * Runs as two launches on `stream`: the solve's first pass over every
 * environment, then its fallback pass, which reads the first pass's lam and
 * status for the environments left unsolved (so the output buffers must not
 * alias the inputs).  The workspace is optional: given one of at least
 * dsim_workspace_bytes(batch, params, DSIM_ENTRY_JACOBIAN) bytes, the step
 * runs as the derivative entries' step launches (the first pass as an
 * assembly launch and a contact-solve launch in a smaller on-chip layout,
 * then the fallback pass from the record they leave in `ws`): the same
 * outputs bit for bit, faster on large batches, and `ws` then holds the
 * FP64 impulses and solver counts described below.  NULL, or fewer bytes,
 * selects the two launches.
 */
int32_t dsim_step(const dsim_batch* batch, const dsim_params* params,
                  const void* q, const void* v, const void* tau,
                  void* v_next, void* lam, int8_t* mode, int32_t* status,
                  void* ws, size_t ws_bytes, void* stream);

/*
 * The step and its full Jacobian (eq. FD_grads with the reduced system of
 * eq. 10 / Appendix B, assembled as in Appendix D).  Besides the dsim_step
 * outputs: dvdq, dvdv, dvdtau, each n_v x n_v row-major per environment,
 * concatenated over environments (offset sum over previous envs of n_v^2).
 * Row i, column j of dvdq is d v+_i / d dq_j for the tangent perturbation.
 */
int32_t dsim_step_jacobian(const dsim_batch* batch, const dsim_params* params,
                           const void* q, const void* v, const void* tau,
                           void* v_next, void* lam, int8_t* mode, int32_t* status,
                           void* dvdq, void* dvdv, void* dvdtau,
                           void* ws, size_t ws_bytes, void* stream);

/*
 * Reverse mode (Section III.A, the adjoint of the implicit system): recomputes
 * the step and returns g_q, g_v, g_tau, the gradients with respect to
 * (dq, v, tau) of gbar . v+ + glam . Lam for gbar = g_vnext [sum n_v] and
 * glam = g_lam [3 sum n_c] (may be NULL: no impulse term).  Also writes the
 * step outputs (v_next, lam, mode, status).  The impulse term uses the
 * derivative of the impulses the library computes; with redundant contacts
 * (a rank-deficient reduced system) the impulses, and so this term, are
 * one of several valid choices, while the v+ term is unique.
 */
int32_t dsim_step_vjp(const dsim_batch* batch, const dsim_params* params,
                      const void* q, const void* v, const void* tau,
                      const void* g_vnext, const void* g_lam,
                      void* v_next, void* lam, int8_t* mode, int32_t* status,
                      void* g_q, void* g_v, void* g_tau,
                      void* ws, size_t ws_bytes, void* stream);

/*
 * dsim_step_vjp in two calls, for a caller that takes the step first and
 * its reverse mode later (an autograd forward and backward): the step
 * (Section II.C) as dsim_step that also keeps, in `ws`, the hand-over the
 * reverse mode reads (ws_bytes at least dsim_workspace_bytes for
 * DSIM_ENTRY_VJP; DSIM_ERR_WORKSPACE otherwise, before any launch) ...
 */
int32_t dsim_step_keep(const dsim_batch* batch, const dsim_params* params,
                       const void* q, const void* v, const void* tau,
                       void* v_next, void* lam, int8_t* mode, int32_t* status,
                       void* ws, size_t ws_bytes, void* stream);

/*
 * ... then the reverse mode of that step (Section III.A, through the
 * implicit contact system) without solving it again: g_q, g_v, g_tau as
 * dsim_step_vjp computes them, bit for bit, for the same batch, params, q,
 * v and tau, reading the kept hand-over from `ws` and the step's modes from
 * `mode` (its output, unchanged); `status` is the step's status output, to
 * which DSIM_ST_NONFINITE is added if a gradient is not finite.  The
 * workspace must not be reused or written between the two calls; several
 * reverse passes may read one kept step.  One launch on `stream`, which
 * must be ordered after the dsim_step_keep call.
 */
int32_t dsim_vjp_kept(const dsim_batch* batch, const dsim_params* params,
                      const void* q, const void* v, const void* tau,
                      const void* g_vnext, const void* g_lam,
                      const int8_t* mode, int32_t* status,
                      void* g_q, void* g_v, void* g_tau,
                      void* ws, size_t ws_bytes, void* stream);

/*
 * ... or the full Jacobian of that step (eq. FD_grads with the reduced
 * system of eq. 10 / Appendix B, assembled as in Appendix D) without solving
 * it again: dvdq, dvdv, dvdtau laid out as in dsim_step_jacobian and equal
 * to its outputs bit for bit, for the same batch, params, q, v and tau
 * (ws_bytes at least dsim_workspace_bytes for DSIM_ENTRY_JACOBIAN, the same
 * size as for DSIM_ENTRY_VJP; `mode` and `status` as in dsim_vjp_kept).
 * One launch on `stream`, ordered after the dsim_step_keep call; it
 * refuses, with DSIM_ERR_SIZE and before any launch, the trees whose
 * derivative layout does not fit on chip, as dsim_step_jacobian does.
 */
int32_t dsim_jacobian_kept(const dsim_batch* batch, const dsim_params* params,
                           const void* q, const void* v, const void* tau,
                           const int8_t* mode, int32_t* status,
                           void* dvdq, void* dvdv, void* dvdtau,
                           void* ws, size_t ws_bytes, void* stream);

/*
 * dsim_step_vjp without a caller workspace and without any allocation, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Arguments, outputs
 * and results are those of dsim_step_vjp; the hand-over between its launches
 * lives in a static device array of dsim_noalloc_scratch_bytes() bytes
 * (64 MiB: about 1590 environments of 31 bodies, 36 dofs and 8 contacts in
 * FP32) that each GPU the library runs on holds until the process ends.  A
 * batch whose hand-over (dsim_workspace_bytes for DSIM_ENTRY_VJP) exceeds it
 * is rejected with DSIM_ERR_WORKSPACE before any device call; DSIM_ERR_DEVICE
 * if the array's address cannot be obtained on the current device.  Every
 * call on a GPU shares that GPU's array, so calls that overlap on one GPU
 * (for instance on two streams) race; calls in stream order do not.
 */
int32_t dsim_step_vjp_noalloc(const dsim_batch* batch, const dsim_params* params,
                              const void* q, const void* v, const void* tau,
                              const void* g_vnext, const void* g_lam,
                              void* v_next, void* lam, int8_t* mode, int32_t* status,
                              void* g_q, void* g_v, void* g_tau, void* stream);

/* Bytes of the static workspace of dsim_step_vjp_noalloc. */
size_t dsim_noalloc_scratch_bytes(void);

/*
 * Reverse mode in the physical parameters as well (derivatives with respect
 * to physical parameters, Section II.D, by the implicit differentiation of
 * the same mode system): everything dsim_step_vjp computes (g_lam as
 * there), plus g_params
 * [7 sum n_b + sum n_c], per environment e at 7 body_off[e] + contact_off[e]:
 *   n_b entries gbar^T dv+/dm_b (body masses; the centre of mass and the
 *     rotational inertia about it held fixed),
 *   6 n_b entries gbar^T dv+/dI_b,k (rotational inertia about the centre of
 *     mass in the body frame, components xx yy zz xy xz yz of each body in
 *     turn, each off-diagonal component moving both symmetric entries),
 *   n_c entries gbar^T dv+/dmu_c (zero for breaking and sticking contacts,
 *     whose equations do not involve mu).
 * Each is a generalised force paired with dt M^-1 P^T gbar, the vector the
 * reverse mode already forms, so the cost over dsim_step_vjp is one pass
 * over the bodies and contacts.  Workspace and errors: as dsim_step_vjp.
 */
int32_t dsim_step_vjp_params(const dsim_batch* batch, const dsim_params* params,
                             const void* q, const void* v, const void* tau,
                             const void* g_vnext, const void* g_lam,
                             void* v_next, void* lam, int8_t* mode, int32_t* status,
                             void* g_q, void* g_v, void* g_tau, void* g_params,
                             void* ws, size_t ws_bytes, void* stream);

/*
 * Forward mode in the physical parameters: everything dsim_step_jacobian
 * computes, plus dvdp, per environment an n_v x (7 n_b + n_c) row-major
 * block at pjac_off[e], its columns in the order of the g_params entries of
 * dsim_step_vjp_params: n_b body masses, 6 n_b rotational inertias, n_c
 * friction coefficients (a friction column is zero unless the contact
 * slides).  The columns are extra right-hand sides of
 * the same reduced system (formed as Q times a generalised force, Q = P M^-1
 * of the Jacobian assembly).  Requires batch->jac_off and batch->pjac_off.
 * Workspace and errors: as dsim_step_jacobian.
 */
int32_t dsim_step_jacobian_params(const dsim_batch* batch, const dsim_params* params,
                                  const void* q, const void* v, const void* tau,
                                  void* v_next, void* lam, int8_t* mode, int32_t* status,
                                  void* dvdq, void* dvdv, void* dvdtau, void* dvdp,
                                  void* ws, size_t ws_bytes, void* stream);

/*
 * The step followed by the position update q_next = q (+) dt v_next
 * (symplectic Euler: the discrete motion of Section II.C advanced in
 * position with the new velocity): a revolute angle adds dt v_next, a free
 * flyer composes its placement with Exp(dt v_next) on the right and
 * renormalises the quaternion.  q_next has the layout of q [sum n_q]; the
 * other outputs are those of dsim_step.
 */
int32_t dsim_step_integrate(const dsim_batch* batch, const dsim_params* params,
                            const void* q, const void* v, const void* tau,
                            void* q_next, void* v_next, void* lam, int8_t* mode, int32_t* status,
                            void* stream);

/*
 * Adjoint of dsim_step_integrate for one step of a rollout (reverse mode of
 * Section III.A chained with the position update): given the adjoints
 * a_qnext [sum n_v] (tangent, at q_next) and a_vnext [sum n_v] of the
 * outputs, recomputes the step at (q, v, tau) and returns the adjoints of the
 * inputs: a_q [sum n_v] (tangent, at q), a_v [sum n_v], g_tau [sum n_v].
 * The step outputs (v_next, lam, mode, status) are written too.
 */
int32_t dsim_step_integrate_vjp(const dsim_batch* batch, const dsim_params* params,
                                const void* q, const void* v, const void* tau,
                                const void* a_qnext, const void* a_vnext,
                                void* v_next, void* lam, int8_t* mode, int32_t* status,
                                void* a_q, void* a_v, void* g_tau,
                                void* ws, size_t ws_bytes, void* stream);

/*
 * dsim_step_integrate_vjp in two calls, for a rollout's reverse sweep over a
 * recomputed segment: the step and position update as dsim_step_integrate
 * (same outputs, bit for bit) that also keeps, in `ws`, the hand-over its
 * adjoint reads (ws_bytes at least dsim_workspace_bytes for
 * DSIM_ENTRY_STEP_INTEGRATE_VJP; DSIM_ERR_WORKSPACE otherwise, and
 * DSIM_ERR_SIZE for a tree whose adjoint does not fit on chip, both before
 * any launch) ...
 */
int32_t dsim_step_integrate_keep(const dsim_batch* batch, const dsim_params* params,
                                 const void* q, const void* v, const void* tau,
                                 void* q_next, void* v_next, void* lam, int8_t* mode, int32_t* status,
                                 void* ws, size_t ws_bytes, void* stream);

/*
 * ... then the adjoint of that step (Section III.A chained with the position
 * update) without solving it again: a_q, a_v, g_tau as
 * dsim_step_integrate_vjp computes them, bit for bit, for the same batch,
 * params, q, v and tau, reading the kept hand-over from `ws` and the step's
 * modes from `mode` (its output, unchanged); `status` is the step's status
 * output, to which DSIM_ST_NONFINITE is added if an adjoint is not finite.
 * One launch on `stream`, ordered after the keeping call; `ws` must not be
 * written in between.
 */
int32_t dsim_step_integrate_vjp_kept(const dsim_batch* batch, const dsim_params* params,
                                     const void* q, const void* v, const void* tau,
                                     const void* a_qnext, const void* a_vnext,
                                     const int8_t* mode, int32_t* status,
                                     void* a_q, void* a_v, void* g_tau,
                                     void* ws, size_t ws_bytes, void* stream);

/*
 * Maps a gradient in the tangent coordinates of q (g_tangent [sum n_v], as
 * returned by the VJP entries) to the stored coordinates of q
 * (g_ambient [sum n_q]): revolute entries copy; a free flyer gets
 * R(quat) g_linear for the position and 2 quat * (g_angular, 0) for the
 * quaternion, so that g_ambient . (d q / d delta) = g_tangent for the
 * perturbation q (+) delta.  Needs only the body offsets and joint types of
 * `batch`; `precision` is a dsim_precision.
 */
int32_t dsim_tangent_to_ambient(const dsim_batch* batch, int32_t precision, const void* q,
                                const void* g_tangent, void* g_ambient, void* stream);

/*
 * The transpose of that map: a gradient on the stored coordinates of q
 * (g_ambient [sum n_q]) -> the tangent adjoint g_tangent [sum n_v] =
 * (d (q (+) delta) / d delta)^T g_ambient at delta = 0, the form the VJP
 * entries take for q_next (for instance a loss gradient on the stored
 * coordinates of q_next from torch autograd).  Revolute entries copy; a
 * free flyer gets R(quat)^T g_p and (w g_v - v x g_v - v g_w) / 2 for a
 * quaternion (v, w) with gradient (g_v, g_w).  The two maps compose to the
 * identity on tangent gradients for unit quaternions.
 */
int32_t dsim_ambient_to_tangent(const dsim_batch* batch, int32_t precision, const void* q,
                                const void* g_ambient, void* g_tangent, void* stream);

/* Description of one status bit (DSIM_ST_*), or "ok" for 0. */
const char* dsim_status_string(int32_t bit);

#ifdef __cplusplus
}
#endif

#endif /* DSIM_H */
