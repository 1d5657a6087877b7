/*
 * dmrod.h -- C ABI of the MI355X implicit Discrete Elastic Rods library (libdmrod.so).
 *
 * The library advances rods and rod networks with the fully implicit backward-Euler
 * step of DisMech (arXiv 2311.18126): stretch, bend and twist energies (Eq. 2-8),
 * elastic force as minus the energy gradient (Eq. 9), optional flat-floor contact and
 * smooth Coulomb friction (Eq. 10-13), the implicit equations of motion (Eq. 14-15)
 * solved by Newton's method with the exact Jacobian (Eq. 16), elastic joints
 * (Elastic Joints subsection) and natural-curvature actuation (Actuation subsection).
 * Every step of the Newton iteration runs in HIP kernels on the GPU in FP64.
 *
 * Conventions shared by every entry point:
 *  - Every function returns a dm_status.  Negative values are errors and leave the
 *    simulation unchanged; the message of the last non-OK status of the calling thread is
 *    available from dm_last_error().  No function aborts, exits or lets a C++ exception out.
 *  - Pointers marked "host" are read or written during the call only; the caller keeps
 *    ownership.  Pointers marked "device" are device memory on the simulation's device,
 *    caller-owned; the library reads/writes them on the simulation's stream and the call
 *    returns after that work completes.
 *  - Units are SI.  Positions are [N][3] row-major doubles; twist angles are per edge.
 *  - A dm_sim is used by one host thread at a time.  Different sims may share a device.
 */
#ifndef DMROD_H
#define DMROD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DM_OK = 0,
  DM_NOT_CONVERGED = 1,        /* warning: some systems did not converge; their state is
                                  left at the start of the failing step and they stop
                                  advancing (see dm_get_stats) */
  DM_ERR_INVALID_ARG = -1,     /* bad pointer, size, index or non-finite input */
  DM_ERR_STATE = -2,           /* call not allowed in this phase (e.g. add after finalize) */
  DM_ERR_HIP = -3,             /* a HIP runtime call failed (message names it) */
  DM_ERR_OOM = -4,             /* device allocation failed */
  DM_ERR_SINGULAR = -5,        /* a Newton linear system had a zero or non-finite pivot;
                                  that system's state is left at the start of the step */
  DM_ERR_UNSUPPORTED = -6      /* topology or option this library does not implement */
} dm_status;

typedef struct dm_sim dm_sim;  /* opaque; created by dm_create, freed by dm_destroy */

/* Simulation-wide settings.  dm_config_default() fills sensible defaults. */
typedef struct {
  double gravity[3];      /* m/s^2, acts on node positions as m_i g (misc. force, Eq. 13 text) */
  double newton_tol;      /* Newton stops when the 2-norm of the residual of Eq. 15 over
                             free DOFs is <= newton_tol (absolute, N and N m mixed) */
  double floor_factor;    /* ...or, after at least one Newton step, when the residual is at or
                             below its FP64 rounding floor and the last step failed to halve
                             it (the floor of stiff or distant systems lies above newton_tol).
                             The floor is floor_factor * eps * || |J| s ||_2 over free rows and
                             columns of the Newton matrix J of the iterate, s_k the step-start
                             magnitude of DOF k's kind (largest |position coordinate| of the
                             system; largest |theta| + pi).  Default 1; 0 disables the rule. */
  int max_iter;           /* Newton iterations per step before DM_NOT_CONVERGED */
  int line_search;        /* 1: halve the Newton step (at most 10 times) until the residual
                             norm decreases (the paper's optional line search) */
  int floor_contact;      /* 1: flat floor z = floor_z with the IMC energy (Eq. 10-11) and
                             friction (Eq. 12-13) on every node */
  double floor_z;         /* floor height [m] */
  double delta;           /* IMC distance tolerance [m]; K1 = 15/delta */
  double nu;              /* slipping tolerance [m/s]; K2 = 15/nu */
  double mu;              /* friction coefficient */
  double k_contact;       /* stiffness multiplying the IMC energy [N/m] */
  double damping;         /* viscous damping eta [1/s]: F = -eta m (x - x_n)/dt */
  int device;             /* HIP device ordinal */
  void* stream;           /* hipStream_t to run on; NULL = the default stream */
  int block_size;         /* threads per system workgroup: 0 = automatic (256; 512 while
                             self-contact is on; dm_autotune's choice once it has run), else
                             64..512, a multiple of 64 */
  int warm_max_iter;      /* Newton iterations allowed to a warm-started solve before it is
                             redone from the step-start state (0 = max_iter) */
  int use_graphs;         /* 1 (default): dm_rollout and the adjoint's recomputation replay one
                             captured HIP graph per checkpoint segment (its one-step launches
                             and tip gathers or state saves) instead of launching them one by
                             one; 0: eager launches */
  /* Device-memory hook (the caller's allocator owns the pages, e.g. a framework's caching
     allocator): when alloc is non-NULL every device buffer of the simulation (its state,
     topology, scratch, checkpoints and trajectory buffers) is obtained by
     alloc(bytes, alloc_ctx), which returns device memory on cfg->device, at least 256-byte
     aligned, or NULL on failure (the call then returns DM_ERR_OOM), and is released by
     free_(ptr, alloc_ctx) (required with alloc) after the simulation's stream has drained:
     when a buffer grows and in dm_destroy.  Both are called on the thread that called the
     library.  NULL (default): hipMalloc / hipFree.  The dm_mlp network keeps its own hipMalloc
     buffers. */
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free_)(void* ptr, void* ctx);
  void* alloc_ctx;
} dm_config;

/* Per-system counters accumulated over the last dm_step call. */
typedef struct {
  int steps_done;         /* time steps completed */
  int newton_iters;       /* Newton iterations summed over those steps */
  int status;             /* dm_status of this system for the call */
  int floor_steps;        /* (sub)steps that ended at the rounding floor (floor_factor), not
                             newton_tol */
  int fallbacks;          /* warm-started steps whose Newton solve failed and was redone
                             from the step-start state (see dm_set_warm_start) */
  int halvings;           /* (sub)steps whose Newton solve failed and were redone as two
                             halves (see dm_set_adaptive) */
  double residual;        /* residual norm at the last Newton iterate */
  double floor_residual_max;  /* largest residual among the floor-ended (sub)steps (0: none) */
  double floor_estimate;      /* the rounding-floor estimate of that (sub)step */
} dm_stats;

void dm_config_default(dm_config* cfg);

/* Create an empty simulation on cfg->device. */
dm_status dm_create(const dm_config* cfg, dm_sim** out);

/* Add a rod of n_nodes >= 2 nodes.  x0 (host, [n_nodes][3]) is both the initial and the
 * undeformed shape (rest edge lengths, and rest curvature unless set).  radius h gives
 * A = pi h^2, I = pi h^4/4, J = pi h^4/2; shear modulus G = E/(2(1+poisson)).
 * Node masses are lumped: half of each incident edge's rho*A*length.  *rod_id receives the
 * rod index (0, 1, ... in order of addition). */
dm_status dm_add_rod(dm_sim* sim, int n_nodes, const double* x0, double radius, double E,
                     double poisson, double density, int* rod_id);

/* Elastic joint: node node_b of rod_b becomes the same node as node_a of rod_a.  Bending
 * and twisting act on every pair of edges meeting there (Elastic Joints subsection); a rod
 * passing through the joint keeps its own stencil there (its natural curvature, actuation
 * and stiffness), and every other pair of edges at the joint gets a joint stencil.
 * Supported topologies: each connected set of rods either is one rod, or meets at a single
 * shared node, which may be an end node or an interior node of each rod in the set (a rod
 * through the joint counts as two branches; at most 8 branches).  Rods joined at two or more
 * different nodes, and closed loops, give DM_ERR_UNSUPPORTED at dm_finalize; a rod joined to
 * itself gives it here. */
dm_status dm_add_joint(dm_sim* sim, int rod_a, int node_a, int rod_b, int node_b);

/* Clamp nodes (all three coordinates) and optionally twist angles of a rod.
 * nodes: host array of n node indices; edges: host array of n_edges edge indices. */
dm_status dm_fix_nodes(dm_sim* sim, int rod, const int* nodes, int n);
dm_status dm_fix_edges(dm_sim* sim, int rod, const int* edges, int n_edges);

/* Natural curvature of a rod's interior nodes 1..N-2 (Actuation subsection), host array
 * [N-2][2] in 1/m along the two material directors.  The integrated value used in Eq. 6 is
 * kbar times the rest Voronoi length.  Allowed before and after finalize. */
dm_status dm_set_natural_curvature(dm_sim* sim, int rod, const double* kbar);

/* Sinusoidal actuation kappa1(t) = A sin(2 pi f t + phi) [1/m] on every interior node of
 * the rod (second component zero), evaluated on the device at the end time of each step. */
dm_status dm_set_actuation_sine(dm_sim* sim, int rod, double A, double f, double phi);

/* Constant external loads: force (host [N][3], N) on the rod's nodes and twisting moment
 * (host [N-1], N m) on its edges.  Either pointer may be NULL. */
dm_status dm_set_external_load(dm_sim* sim, int rod, const double* force, const double* moment);

/* Freeze the topology, build the device layout and upload.  No adds afterwards. */
dm_status dm_finalize(dm_sim* sim);

/* Advance every system by nsteps steps of size dt in one persistent launch.
 * stats: NULL or host array of dm_num_systems() entries.  Returns DM_OK, DM_NOT_CONVERGED
 * or DM_ERR_SINGULAR (the worst over systems), or an error. */
dm_status dm_step(dm_sim* sim, double dt, int nsteps, dm_stats* stats);

/* Time integrator of dm_step and dm_autotune (Time Stepping subsection, which offers
 * backward Euler and implicit midpoint).  DM_BACKWARD_EULER (default): the residual of Eq. 15
 * at the step end.  DM_IMPLICIT_MIDPOINT: q_{n+1} = q_n + dt (qdot_n + qdot_{n+1}) / 2 with
 * M (qdot_{n+1} - qdot_n) = dt F(q_m), q_m = (q_n + q_{n+1}) / 2; solved as the backward-Euler
 * residual over dt / 2 for q_m (the same function values, so newton_tol means the same), then
 * q_{n+1} = 2 q_m - q_n, qdot_{n+1} = 2 (q_{n+1} - q_n) / dt - qdot_n; frames are carried from
 * the step start to q_m for the forces and to q_{n+1} for the commit; damping and friction see
 * (q_{n+1} - q_n) / dt; actuation is evaluated at t + dt / 2.  Applies to later calls; the
 * adjoint (dm_rollout, dm_adjoint) returns DM_ERR_UNSUPPORTED under midpoint.  Unknown
 * scheme: DM_ERR_INVALID_ARG. */
#define DM_BACKWARD_EULER 0
#define DM_IMPLICIT_MIDPOINT 1
dm_status dm_set_integrator(dm_sim* sim, int scheme);

/* Adaptive time stepping of dm_step (offered as an option in the Time Stepping subsection; the
 * rule is not given there).  With max_halvings = L > 0 a step whose Newton solve does not
 * converge (or meets a zero pivot) is redone as two steps of half the size, each of them
 * adaptive in the same way, down to dt / 2^L; a system only fails when a step of dt / 2^L
 * fails, and then stays at the end of its last converged substep.  Substeps are counted in
 * dm_stats.halvings; steps_done counts whole steps.  0 (default) turns it off; values outside
 * 0..20 return DM_ERR_INVALID_ARG.  Applies to later calls; the adjoint (dm_rollout,
 * dm_adjoint) returns DM_ERR_UNSUPPORTED while it is on. */
dm_status dm_set_adaptive(dm_sim* sim, int max_halvings);

/* Number of independent systems (connected rod sets) and the system holding a rod. */
int dm_num_systems(const dm_sim* sim);
int dm_rod_system(const dm_sim* sim, int rod);
int dm_num_rods(const dm_sim* sim);
int dm_rod_nodes(const dm_sim* sim, int rod);

/* State of one rod in its own node/edge order: x [N][3], theta [N-1], v [N][3],
 * theta_dot [N-1]; any pointer may be NULL.  Host memory. */
dm_status dm_get_rod_state(dm_sim* sim, int rod, double* x, double* theta, double* v,
                           double* theta_dot);
dm_status dm_set_rod_state(dm_sim* sim, int rod, const double* x, const double* theta,
                           const double* v, const double* theta_dot);

/* Bulk state in the library's global node/edge numbering (rod after rod, joint nodes
 * once), host or device (on_device != 0) arrays: x [n_nodes][3], theta [n_edges],
 * v [n_nodes][3], theta_dot [n_edges].  Sizes from dm_num_nodes / dm_num_edges.  The
 * global index of rod r's node i is dm_node_index(r, i). */
int dm_num_nodes(const dm_sim* sim);
int dm_num_edges(const dm_sim* sim);
int dm_node_index(const dm_sim* sim, int rod, int node);
int dm_edge_index(const dm_sim* sim, int rod, int edge);
dm_status dm_get_state(dm_sim* sim, double* x, double* theta, double* v, double* theta_dot,
                       int on_device);
dm_status dm_set_state(dm_sim* sim, const double* x, const double* theta, const double* v,
                       const double* theta_dot, int on_device);

/* Full checkpoint: state plus the step-start reference frames, reference twist and time,
 * packed into a caller buffer of dm_checkpoint_size() doubles (host or device). */
size_t dm_checkpoint_size(const dm_sim* sim);
dm_status dm_save_checkpoint(dm_sim* sim, double* buf, int on_device);
dm_status dm_load_checkpoint(dm_sim* sim, const double* buf, int on_device);

/* Natural curvature of every rod at once: kbar is the concatenation, in rod order, of each
 * rod's [N-2][2] array in 1/m (as dm_set_natural_curvature), host or device
 * (on_device != 0, only after finalize). */
dm_status dm_set_natural_curvature_all(dm_sim* sim, const double* kbar, int on_device);

/* Trajectory for the discrete adjoint (gradient-based fitting of natural curvature, which
 * the paper's Real2Sim section does with finite differences, Eq. 20).
 * dm_rollout: nsteps steps of size dt from the current state, each one backward-Euler step
 * solved to the Newton tolerance; a full-state checkpoint is kept (device memory owned by
 * the sim) every ckpt_every steps.  tips receives the position of each rod's last node after
 * every step, [nsteps][n_rods][3], host or device.  A step that does not converge ends the
 * call with its status and no usable trajectory.
 * dm_adjoint: for the last dm_rollout and a loss L of its tip trajectory, takes dL/dtips
 * ([nsteps][n_rods][3], host or device) and writes dL/dkbar, the gradient with respect to
 * every rod's natural curvature in the layout of dm_set_natural_curvature_all (host or
 * device).  It recomputes each checkpoint interval forward, then runs the implicit-function
 * adjoint of every step backward (transposed Newton system, step-start frames and natural
 * curvature differentiated exactly); the sim is back at the rollout's final state after the
 * call.  Both return DM_ERR_UNSUPPORTED for joined rods, floor contact, actuated rods, the
 * implicit-midpoint integrator or adaptive time stepping, and DM_ERR_STATE if dm_adjoint has
 * no completed rollout. */
dm_status dm_rollout(dm_sim* sim, double dt, int nsteps, int ckpt_every, double* tips, int on_device);
dm_status dm_adjoint(dm_sim* sim, const double* dL_dtips, int in_on_device, double* dL_dkbar,
                     int out_on_device);

/* Gradient descent on the natural curvature in the control flow of the Real2Sim algorithm
 * (Alg. 1): per iterate, the sim is reset to its state at the call, the curvature set, the
 * trajectory rolled out (dm_rollout with dt, nsteps, ckpt_every) and the loss
 * L = sum |tip - target|^2 formed on the device; the loop stops when L < tol or after max_iter
 * gradient steps; the step size (alpha0 at first) is halved whenever L rose since the previous
 * iterate; the step is kbar <- kbar - alpha dL/dkbar (Eq. 21) with the gradient from dm_adjoint
 * in place of the forward differences of Eq. 20.  target_tips: [nsteps][n_rods][3] (host or
 * device).  kbar: in the start value, out the fitted one, layout of
 * dm_set_natural_curvature_all (host or device).  losses: NULL or host array of max_iter + 1
 * receiving the loss of every evaluated iterate; n_eval: NULL or their count.  On return the
 * sim holds its starting state and the fitted curvature.  Same restrictions as dm_adjoint;
 * bad step size, tolerance or counts return DM_ERR_INVALID_ARG; a rollout whose Newton solve
 * fails returns its status and leaves the sim's state and curvature unspecified (reload a
 * checkpoint).  The caller's arrays must hold the sizes stated (not checked). */
dm_status dm_fit_natural_curvature(dm_sim* sim, double dt, int nsteps, int ckpt_every, const double* target_tips,
                                   int target_on_device, double alpha0, double tol, int max_iter, double* kbar,
                                   int kbar_on_device, double* losses, int* n_eval);

/* ---- Real2Sim: limb curvatures of quasi-static configurations (Real2Sim section) ----------
 * Limb curvature of a rod: the mean over its interior stencils of the first integrated
 * curvature of Eq. 5 divided by the rest Voronoi length (1/m), at the current state.
 * dm_limb_curvatures: kappa (host [n_rods]) of every rod; 0 for rods of fewer than 3 nodes. */
dm_status dm_limb_curvatures(dm_sim* sim, double* kappa);
/* Gradient of sum_r w[r] kappa_r with respect to each rod's uniform natural curvature (1/m,
 * first material direction, on all its interior stencils) at the current state taken as an
 * equilibrium: the implicit-function adjoint of one more backward-Euler step of dt from it
 * (inertia negligible for a long dt).  w and grad: host [n_rods].  DM_ERR_UNSUPPORTED with floor
 * contact, actuated rods or the midpoint integrator; DM_ERR_SINGULAR for a singular matrix. */
dm_status dm_limb_curvature_gradient(dm_sim* sim, double dt, const double* w, double* grad);
/* Alg. 1 of the Real2Sim section for every system at once, each system's rods being its limbs:
 * for each of n_configs target configurations (targets: host [n_configs][n_rods], limb
 * curvatures in 1/m), alpha = alpha0 and lambda_prev = infinity per system; repeat: set each
 * rod's uniform natural curvature kbar_r, reach the quasi-static configuration by n_settle
 * backward-Euler steps of dt from the current state, lambda = sum over the system's rods of
 * |kappa*_r - kappa_r| (Eq. 19); stop below tol or after max_iter gradient steps; halve alpha if
 * lambda rose; kbar <- kbar - alpha d lambda/d kbar (Eq. 21) with the gradient of
 * dm_limb_curvature_gradient in place of the forward differences of Eq. 20.  kbar starts at 0
 * and carries over between configurations; a system that has stopped is not stepped until the
 * next configuration.  kbar_traj: host [n_configs][n_rods], the fitted kbar after each
 * configuration; steps (host int [n_configs][n_systems]) and losses (host
 * [n_configs][n_systems], the last lambda) may be NULL.  The sim ends in the last configuration
 * with its natural curvature set to the fit.  Same restrictions as the gradient; a failing
 * quasi-static solve returns its status. */
dm_status dm_fit_limb_curvatures(dm_sim* sim, double dt, int n_settle, int n_configs, const double* targets,
                                 double alpha0, double tol, int max_iter, double* kbar_traj, int* steps,
                                 double* losses);

/* Edge-edge self-contact of every rod inside the step (Contact and Friction subsection, Eq.
 * 10-13 applied to pairs of a rod's edges): at every Newton iterate the pairs of each rod's
 * edges with D < 2h + delta are found (two edges closer than 2h + delta along the rest rod are
 * never a pair), their energy k_c E_c(D) joins the elastic energy and their friction (mu, nu)
 * the external forces.  Each rod's Newton matrix is then its band plus every pair's blocks
 * (the contact Hessian and the friction's derivative), held in a dense (4N - 1)^2 matrix per
 * rod that this call allocates (at most 32 GiB for the simulation) and factorised over the
 * half bandwidth the pairs need.  Stick-slip friction may need line search (dm_config) and
 * adaptive halving (dm_set_adaptive).  After dm_finalize; k_c = 0 turns it off; delta > 0,
 * k_c > 0, mu >= 0, nu > 0 otherwise.  DM_ERR_UNSUPPORTED for joined rods, for rods whose
 * self-contact arrays do not fit in 64 KB of LDS (about 400 nodes) or matrices beyond the
 * limit; dm_step then needs the backward-Euler integrator, and the adjoint and the Real2Sim
 * gradient refuse it.  A rod with more than four times as many pairs as edges at some
 * iterate stops there with DM_ERR_UNSUPPORTED.  Without a workgroup size in dm_config (and
 * before any dm_autotune), the step then runs 512 lanes per rod, 256 again when self-contact
 * is turned off. */
dm_status dm_set_self_contact(dm_sim* sim, double delta, double k_c, double mu, double nu);

/* ---- Edge-edge contact (Contact and Friction subsection, Eq. 10-13) ----------------------
 * The Implicit Contact Model between edges: contact energy k_c E_c(D) (Eq. 10, K1 = 15/delta,
 * k_c a stiffness the equation leaves out), D the minimum distance between two edges (as
 * segments), C = h_i + h_j the centreline distance at which contact starts (2h within one rod),
 * contact force -dE/dx (Eq. 11) and friction (Eq. 12-13).  These entry points detect the pairs
 * of a set of edges and evaluate each pair's terms; the implicit step does not use them yet
 * (edge-edge contact couples DOFs outside the banded structure of a rod).
 *
 * Edges are grouped: pairs are only sought inside a group (a scene of rods that may touch);
 * a group holds at most DM_CONTACT_MAX_GROUP_EDGES edges.  Two edges of one rod (same `rod`
 * value) whose rest arclength gap -- arc0 of the later edge minus arc0 + ebar of the earlier --
 * is below h_i + h_j + delta never form a pair (they would touch in the rest shape).  A pair is
 * every other pair of one group with D < h_i + h_j + delta. */
#define DM_CONTACT_MAX_GROUP_EDGES 2048
#define DM_CONTACT_MAX_PAIRS_PER_GROUP 2048
typedef struct dm_contact dm_contact;
/* Tables (host, copied): edges [n_edges][2] node indices into positions [n_nodes][3], rod id
 * [n_edges], arc0 [n_edges] rest arclength of the edge's rod at its first node, ebar
 * [n_edges] rest lengths (> 0), radius [n_edges] (> 0); group_start [n_groups + 1] ascending,
 * 0 .. n_edges, each group's edges contiguous; delta > 0 (m); pair_capacity: pair slots per
 * group, 1 .. DM_CONTACT_MAX_PAIRS_PER_GROUP.  The handle works on `device` and `stream`. */
dm_status dm_contact_create(int device, void* stream, int n_nodes, int n_edges, const int* edges, const int* rod,
                            const double* arc0, const double* ebar, const double* radius, int n_groups,
                            const int* group_start, double delta, int pair_capacity, dm_contact** out);
/* Pairs at positions x [n_nodes][3] (device).  Outputs (device): pairs [n_groups][cap][2] global
 * edge indices i < j, sorted by (i, j) within a group; dst [n_groups][cap][3] = D, s, t (the
 * closest points a + s (b - a) on edge i and c + t (d - c) on edge j; for parallel edges one of
 * the equally close pairs of points); counts [n_groups] pairs per group; total (host, may be
 * NULL) the sum.  A group with more pairs than cap gives DM_ERR_INVALID_ARG: its count is
 * exact, its slots hold an unspecified subset. */
dm_status dm_contact_find(dm_contact* c, const double* x, int* pairs, double* dst, int* counts, int* total);
/* Per pair of the slots of dm_contact_find (pairs, counts as it wrote them), at positions x:
 * energy [n_groups][cap] = k_c E_c(D); grad [n_groups][12][cap], the gradient with respect to
 * the 12 coordinates (edge i's nodes a, b, edge j's c, d, x y z each; component-major per
 * group, so consecutive pairs are consecutive in memory); hess [n_groups][144][cap] (row-major
 * 12 x 12 per pair; NULL to skip); friction [n_groups][12][cap] (NULL to skip) the friction
 * forces of Eq. 12-13 on the four nodes with u the tangential relative velocity of the closest
 * points over the step from x_prev (device [n_nodes][3], the step start; no friction if
 * NULL), dt > 0, mu >= 0, nu > 0.  Slots beyond a group's count are not written.  At D = 0
 * the direction is undefined and the gradient, Hessian and friction are zero. */
dm_status dm_contact_terms(dm_contact* c, const double* x, const double* x_prev, double dt, double k_c, double mu,
                           double nu, const int* pairs, const int* counts, double* energy, double* grad, double* hess,
                           double* friction);
/* Duration in ms of the last detection (which = 0) or terms (1) kernel, from HIP events on the
 * handle's stream. */
double dm_contact_last_ms(const dm_contact* c, int which);
const char* dm_contact_last_error(void);
void dm_contact_destroy(dm_contact* c);

/* ---- Learned warm start of the Newton solve ----------------------------------------------
 * Not part of the paper's method: a small network predicts each node's displacement over a
 * step and the prediction is Newton's initial guess (Eq. 16 is still iterated to newton_tol,
 * and a warm-started step whose solve fails is redone from the step-start state).
 * Network: 26 features per node -> 256 -> 256 -> 3, ReLU, bfloat16 operands with float32
 * accumulation on the matrix cores; parameters are float32 master weights laid out as
 * W1 [256][26], b1 [256], W2 [256][256], b2 [256], W3 [3][256], b3 [3] (dm_mlp_num_params()).
 * Features of node i of a rod (raw, float64, row-major [rows][26]; a missing neighbour at a rod
 * end is replicated): v_{i-1} - v_i, v_{i+1} - v_i, v_i, the velocity change over the last
 * step a_i = v_i - v_prev_i, x_{i-1} - 2 x_i + x_{i+1}, log10 E, radius, mean rest length of the
 * edges at i, the natural curvature at i in 1/m (nearest interior node at the ends), the change
 * of the velocity change j_i = a_i - (v_prev_i - v_prev2_i), and a_{i-1} - 2 a_i + a_{i+1}.
 * Inputs are standardised ((f - mean)/std per feature); the output y is the displacement
 * beyond the third-order extrapolation in units of a per-component scale:
 * dx = dt (v + a + j) + scale * y.  Targets passed to training are raw dx - dt (v + a + j)
 * (float64 [rows][3]).
 * A dm_mlp owns its device buffers; row counts are at most max_rows.  All pointers to
 * features, targets, outputs and gradients are device memory. */
typedef struct dm_mlp dm_mlp;
size_t dm_mlp_num_params(void);
/* Features per row (26). */
int dm_mlp_num_inputs(void);
dm_status dm_mlp_create(int device, void* stream, int max_rows, dm_mlp** out);
/* params: float32 [dm_mlp_num_params()], host or device; resets Adam's moments and step. */
dm_status dm_mlp_set_params(dm_mlp* net, const float* params, int on_device);
dm_status dm_mlp_get_params(dm_mlp* net, float* params, int on_device);
/* Standardisation: host arrays mean [26], std [26], output scale [3] (all std, scale > 0). */
dm_status dm_mlp_set_normalisation(dm_mlp* net, const double* mean, const double* std, const double* scale);
dm_status dm_mlp_get_normalisation(dm_mlp* net, double* mean, double* std, double* scale);
/* Mean and standard deviation of each feature and the root-mean-square of each target
 * component over n >= 2 rows of raw features F [n][26] (device, 16-byte aligned) and targets
 * T [n][3] (device). */
dm_status dm_mlp_fit_normalisation(dm_mlp* net, const double* F, const double* T, int n);
/* Y [n][3] (float32): the network's standardised output for raw features F [n][26]. */
dm_status dm_mlp_forward(dm_mlp* net, const double* F, int n, float* Y);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same forward pass as dm_mlp_forward, bit for
 * bit, with its activations (standardised inputs, both hidden layers, outputs) in a static
 * device array of the library instead of the network's buffers, so the call allocates
 * nothing.  n is limited to DM_MLP_NOALLOC_MAX_ROWS (the array holds that many rows, about
 * 4.5 MB on each GPU the library runs on, kept until the process ends); a larger n returns
 * DM_ERR_INVALID_ARG.  F [n][26] float64 and Y [n][3] float32 are device memory.  Every call
 * on a GPU uses that GPU's one array: calls that overlap on one GPU (other threads, other
 * streams) race.  The array's device address is looked up once per device on the first call. */
#define DM_MLP_NOALLOC_MAX_ROWS 2048
dm_status dm_mlp_forward_noalloc(dm_mlp* net, const double* F, int n, float* Y);
/* Loss = (1/n) sum |y - T/scale|^2 and its gradient with respect to every parameter
 * (float32 [dm_mlp_num_params()], device); loss is a host pointer (may be NULL). */
dm_status dm_mlp_gradients(dm_mlp* net, const double* F, const double* T, int n, float* grads, double* loss);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8, learning rate lr) on that loss. */
dm_status dm_mlp_train_step(dm_mlp* net, const double* F, const double* T, int n, float lr, double* loss);
/* One epoch of such steps without a host wait per step: mini-batches of `batch` rows taken in
 * the order of perm (device int32 [n], indices into the n rows of F [n][26] and T [n][3], both
 * device float64); the last n % batch entries of perm are not used.  mean_loss (host, may be
 * NULL) receives the mean of the batch losses.  1 <= batch <= min(n, max_rows); an index of
 * perm outside 0..n-1 gives DM_ERR_INVALID_ARG (that batch's row is replaced by row 0 and the
 * epoch's steps have still been applied).  Waits for the network's stream before returning. */
dm_status dm_mlp_train_epoch(dm_mlp* net, const double* F, const double* T, const int* perm, int n, int batch,
                             float lr, double* mean_loss);
const char* dm_mlp_last_error(void);
void dm_mlp_destroy(dm_mlp* net);

/* Rows of the simulation's feature matrix: one per rod node (a node shared by k rods appears
 * k times; the prediction of the rod that assembles the node's own terms is used). */
int dm_ws_rows(const dm_sim* sim);
/* Raw features of every row at the current (step-start) state into F [rows][26] (device). */
dm_status dm_ws_features(dm_sim* sim, double* F);
/* Training targets after a step: dt (v_{n+1} - v_n - a_n - j_n) per row into T [rows][3]
 * (device), with v_n, a_n and j_n taken from the step-start features F_prev. */
dm_status dm_ws_targets(dm_sim* sim, const double* F_prev, double dt, double* T);
/* Warm start of dm_step: mode 0 off (Newton from x_n), 1 explicit predictor x_n + dt v_n,
 * 3 the second-order extrapolation x_n + dt (v_n + a_n), 4 the third-order extrapolation
 * x_n + dt (v_n + a_n + j_n), 2 the network on top of the third-order extrapolation (dt is the
 * Newton step; a substep of adaptive halving, or the midpoint state under the implicit-midpoint
 * integrator, takes its share of the network's whole-step correction).
 * Each system guesses at the start of every step inside the same persistent launch (the
 * network runs there on the matrix cores); a guess whose Newton solve fails within
 * warm_max_iter iterations is redone from x_n and counted in dm_stats.fallbacks.  The sim
 * keeps a reference to net, which must outlive its use.  After dm_set_state or
 * dm_load_checkpoint the velocity history is the current velocity (a = j = 0).  Mode 2 with
 * self-contact on is DM_ERR_UNSUPPORTED where the network's activations and the self-contact
 * arrays do not fit together in the workgroup's 64 KB of LDS. */
dm_status dm_set_warm_start(dm_sim* sim, dm_mlp* net, int mode);
/* The guessed displacement x^(0) - x_n of every feature row for a time step dt from the
 * current state under the current warm mode (not 0), into dx [rows][3] (device memory if
 * on_device, else host); the state is not changed.  Under backward Euler that is the guess of
 * the step's end; under the implicit-midpoint integrator the Newton unknown is the midpoint
 * state, and the guess is of it (the Newton step dt / 2, half the network's correction).
 * Rows of clamped or shared nodes are reported too (the step leaves clamped DOFs alone and
 * uses the owning rod's row). */
dm_status dm_ws_predict(dm_sim* sim, double dt, double* dx, int on_device);

/* Autotuner: times the step kernel at each workgroup size (64, 128, 256, 512 threads) over
 * trial_steps steps of size dt from the current state, keeps the fastest, and restores the
 * state afterwards (the last-step velocity change of the warm start is reset).  cache_path
 * (NULL for none) names a text file of "signature block" lines: a signature of the system
 * layout and device found there is used without timing; a new one is appended.  block_out
 * (may be NULL) receives the chosen size. */
dm_status dm_autotune(dm_sim* sim, double dt, int trial_steps, const char* cache_path, int* block_out);

/* Simulation time [s]. */
double dm_time(const dm_sim* sim);

/* Duration [ms] of the last dm_step's kernel, from HIP events recorded on the simulation's
 * stream immediately before and after the launch; and the workgroup size it used. */
double dm_last_kernel_ms(const dm_sim* sim);
int dm_block_size(const dm_sim* sim);

const char* dm_last_error(void);
void dm_destroy(dm_sim* sim);

#ifdef __cplusplus
}
#endif
#endif /* DMROD_H */
