/*
 * pflbm.h - C interface of the MI355X (gfx950) phase-field lattice Boltzmann
 * library with wetting folded into the chemical potential (arXiv:2312.00369).
 *
 * The problem statement follows the paper: a grid with a solid mask
 * (Sec. 2.2.2), a contact angle theta (Eq. chemical_potencial2), the fluid
 * parameters rho_l, rho_g, nu, sigma (through beta and kappa), M and W
 * (Sec. 3.1), an initial order parameter (Eq. initialphi), and the lattice
 * (D2Q9, or D3Q19 for both distribution sets in 3D, Sec. 3).  The outputs are
 * the order parameter, pressure, velocity and chemical potential fields and
 * the contact angle.
 *
 * Conventions shared by every call
 *  - Host arrays are dense nx*ny*nz arrays with x fastest (index x + nx*(y +
 *    ny*z)); nz = 1 in 2D.  The library copies what it needs: the caller keeps
 *    ownership of every array it passes.
 *  - Lattice units: dx = dt = 1.
 *  - Every call returns PFLBM_OK (0) or a negative error code.  No C++
 *    exception crosses this interface.  pflbm_last_error() returns a
 *    thread-local text for the last failure in the calling thread.
 *  - Handles are not thread-safe; a handle's device work is ordered on the HIP
 *    stream given at creation (0 = the null stream), which must outlive it.
 *  - Calls marked (async) enqueue work and return; calls marked (sync) wait
 *    for the handle's stream before returning.
 */
#ifndef PFLBM_H
#define PFLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- errors */
#define PFLBM_OK            0
#define PFLBM_EINVAL       (-1) /* bad argument: tau <= 1/2, M <= 0, dims <= 0, theta
                                   outside (0,180), null required pointer, struct_size
                                   mismatch, buffer too small                         */
#define PFLBM_ENOMEM       (-2) /* device or host allocation failed                   */
#define PFLBM_EDEVICE      (-3) /* a HIP call failed; the message is kept             */
#define PFLBM_ENONFINITE   (-4) /* the case produced a NaN or infinity                 */
#define PFLBM_ESTATE       (-5) /* call not valid in the object's state               */
#define PFLBM_EUNSUPPORTED (-6) /* lattice / storage combination not provided          */

/* ---------------------------------------------------------------- enums */
/* Case lattices: D2Q9 for both sets; D3Q19 for both sets; D3Q19 for f and the
 * phi stencils with D3Q7 for g (Sec. 2.1.3: w_0 = 1/4, w_1-6 = 1/8,
 * c_s^2 = 1/4, and alpha = M / (c_s^2 (tau_g - 1/2)) with that c_s^2).
 * PFLBM_D3Q7 names the phase set alone (pflbm_lattice_table only). */
enum { PFLBM_D2Q9 = 0, PFLBM_D3Q19 = 1, PFLBM_D3Q19_D3Q7 = 2, PFLBM_D3Q7 = 3 };  /* Eq. ci / 3ci */
enum { PFLBM_FP64 = 0, PFLBM_FP32 = 1, PFLBM_FP16_DEV = 2 }; /* distribution storage   */
enum { PFLBM_WALL_NONE = 0, PFLBM_WALL_PLANE = 1, PFLBM_WALL_BALL = 2 };

/* Case parameters (POD, FP64 on the host whatever the storage).
 *  tau            hydrodynamic relaxation time tau_f (nu = c_s^2 (tau_f - 1/2),
 *                 Sec. 2.1.2); used when nu_l = nu_g = 0
 *  tau_phi        relaxation time tau_g of the phase-field LBE (Eq. BGK); 0 = tau
 *  mobility       M; alpha = M / (c_s^2 (tau_g - 1/2)) (Eq. mobility)
 *  beta, kappa    free-energy coefficients (Eq. free-energy, bulk_energy)
 *  rho_l, rho_g   densities at phi = 1 and phi = 0 (Sec. 2.1.1)
 *  nu_l, nu_g     viscosities at phi = 1 and 0; both 0 = uniform tau
 *  theta_deg      contact angle in degrees, in (0, 180)
 *  body_force     F_b (Sec. 2.1.1); components beyond the dimension are ignored
 *  storage        PFLBM_FP64: FP64 storage and arithmetic; PFLBM_FP32: FP32
 *                 storage and arithmetic; PFLBM_FP16_DEV: FP16 deviations with a
 *                 per-case power-of-two scale (g_0 and s in FP32), FP32 arithmetic
 *  wall_*, diag_width
 *                 the wall the contact-angle estimator measures against: a plane
 *                 (point + normal pointing into the fluid) or a circle / sphere
 *                 (centre + radius); interface points closer than diag_width to
 *                 it are left out of the fit
 *  steady_tol     max |phi(t) - phi(t_prev_diag)| below which a case is steady
 *  chi_case       the (chi, mu) pairs of Appendix A, Table A1, with
 *                 chi(phi) = c sqrt(2 beta/kappa) cos(theta) (phi - phi^2) in the
 *                 ghost rule n_w . grad phi = chi (Eq. cubicc) and the wall term of mu
 *                 scaled by (1 + c): case 1 c = -1, case 2 (or 0) c = 0, case 3
 *                 c = +1.  Cases 1 and 3 need every ghost node to face the fluid
 *                 along one lattice axis (flat axis-aligned walls); pflbm_create
 *                 returns PFLBM_EUNSUPPORTED otherwise.
 *  theta_map      heterogeneous wetting: a contact angle per solid node, in
 *                 (0, 180) degrees, else PFLBM_EINVAL.  The wall term of mu at a
 *                 node uses the mean cos(theta) over the solid and virtual nodes
 *                 of its 3^D block (virtual nodes take theta_deg).  At most 1023
 *                 distinct values besides theta_deg's arise, else
 *                 PFLBM_EUNSUPPORTED; with chi_case 1 or 3, PFLBM_EUNSUPPORTED.
 *                 The array is not kept.
 */
typedef struct pflbm_params {
  uint32_t struct_size;          /* = sizeof(pflbm_params) */
  int32_t lattice;               /* PFLBM_D2Q9, PFLBM_D3Q19 or PFLBM_D3Q19_D3Q7 */
  int32_t storage;               /* PFLBM_FP64 / FP32 / FP16_DEV */
  int32_t nx, ny, nz;            /* nz = 1 for D2Q9 */
  int32_t periodic[3];           /* nonzero = periodic axis; others get bounce-back walls */
  double tau, tau_phi, mobility, beta, kappa, rho_l, rho_g, nu_l, nu_g, theta_deg;
  double body_force[3];
  int32_t wall_kind;             /* PFLBM_WALL_* */
  double wall_point[3], wall_normal[3], wall_radius, diag_width;
  double steady_tol;
  int32_t chi_case;              /* Appendix A, Table A1: 0 or 2 = the method (chi = 0),
                                    1 = cubic Robin ghost rule, 3 = its opposite */
  const double* theta_map;       /* NULL, or nx*ny*nz contact angles in degrees (x fastest),
                                    read on solid nodes at pflbm_create only */
} pflbm_params;

/* Diagnostics record (all reductions in FP64 over zeta = 1 nodes). */
typedef struct pflbm_diag {
  int64_t step;            /* time steps taken so far                                  */
  double mass;             /* sum of phi                                               */
  double s_sum;            /* sum of s = u . grad(phi) of the last step; the step's mass
                              change is -(1.5 s_sum(t) - 0.5 s_sum(t-1))                */
  double steady_residual;  /* max |phi - phi at the previous diagnostics call|          */
  double theta_deg;        /* contact angle from the circle / sphere fit (NaN if none)  */
  double centre[3], radius;/* fitted interface circle / sphere                          */
  int64_t n_points;        /* interface points used by the fit                          */
  int32_t nonfinite;       /* nonzero if phi held a NaN or infinity                     */
  int32_t steady;          /* steady_residual <= steady_tol (and not the first call)    */
} pflbm_diag;

typedef struct pflbm_case_s* pflbm_handle;
typedef struct pflbm_group_s* pflbm_group;

/* ---------------------------------------------------------------- host-only helpers */

/* Node classes of Sec. 2.2.2 for a mask, computed on the host without a
 * device: classes[n] gets bit 0 zeta, bit 1 fluid (epsilon = 1), bit 2 ghost,
 * for each of the nx*ny*nz domain nodes.  (no device work) */
int pflbm_classify(const pflbm_params* prm, const uint8_t* solid_mask, uint8_t* classes);

/* Velocity set of a lattice as used by the kernels: c[3*i + a], w[i], opp[i]
 * and the phase-source coefficient k[i] (any pointer may be NULL).  Returns Q
 * (9, 19, or 7 for PFLBM_D3Q7; PFLBM_D3Q19_D3Q7 gives its D3Q19 set) or a
 * negative error code.  (no device work) */
int pflbm_lattice_table(int32_t lattice, int32_t* c, double* w, int32_t* opp, double* k);

/* beta and kappa of the free energy (Eq. bulk_energy with the gradient term)
 * for surface tension sigma and interface width W: the planar equilibrium
 * profile (Eq. initialphi) has W = sqrt(8 kappa / beta) and the tension is
 * sqrt(2 kappa beta) / 6, so beta = 12 sigma / W and kappa = 3 sigma W / 2.
 * EINVAL unless sigma and width are finite and positive.  (no device work) */
int pflbm_beta_kappa(double sigma, double width, double* beta, double* kappa);

/* ---------------------------------------------------------------- single case */

/* Device bytes a case with these parameters needs (sync-free, host only). */
int pflbm_footprint(const pflbm_params* prm, size_t* bytes);

/* Create a case.  solid_mask: nx*ny*nz bytes, nonzero = geometric solid node
 * (Sec. 2.2.2 node marks are derived from it).  phi0: nx*ny*nz initial order
 * parameter (Eq. initialphi), read on fluid and boundary nodes only.
 * The library allocates its device memory itself (hipMalloc).  hip_stream is
 * borrowed (a hipStream_t, or NULL).  (sync: returns with the case initialised) */
int pflbm_create(const pflbm_params* prm, const uint8_t* solid_mask, const double* phi0,
                 void* hip_stream, pflbm_handle* out);

/* As pflbm_create, but the case lives in caller-owned device memory of at least
 * pflbm_footprint bytes, which must stay allocated until pflbm_destroy. */
int pflbm_create_in(const pflbm_params* prm, const uint8_t* solid_mask, const double* phi0,
                    void* hip_stream, void* dev_workspace, size_t ws_bytes, pflbm_handle* out);

/* Advance nsteps >= 0 time steps (Sec. 2.1.2 Eq. BGK-NS and 2.1.3 Eq. BGK, with
 * the wall term of Eq. chemical_potencial2).  With a graph chunk set, full
 * chunks replay a captured HIP graph.  (async) */
int pflbm_step(pflbm_handle h, int64_t nsteps);

/* Steps per captured HIP graph (0 = launch kernels directly).  Default 64. */
int pflbm_set_graph_chunk(pflbm_handle h, int32_t steps);

/* Launch shape of the node-parallel kernels (phi sum, mu stencil, collide-stream
 * of the three-kernel path, the phi pass of the split step, and the
 * reductions): threads along x, y, z of one workgroup (tx a multiple of 64,
 * tx*ty*tz <= 1024).  Results do not depend on it.  Drops any captured graph. */
int pflbm_set_tile(pflbm_handle h, int32_t tx, int32_t ty, int32_t tz);

/* Kernel path of pflbm_step.  variant 0-4: the fused one-kernel step with one
 * of five tile shapes; 5-7: the split step (a phi pass, then one kernel for
 * ghosts, mu and collide-stream) with one of three tile shapes; 8-10 (D3Q19
 * only): the split step whose second kernel marches along z over 64 x ty x tz
 * columns; 11-12 (D3Q19 only): the fused one-kernel step marching along z
 * (phi planes formed from g in a rolling LDS window, g read once per step);
 * -1: the three-kernel path (phi sum, mu stencil, collide-stream).  Defaults:
 * 1 for D2Q9, 7 for D3Q19.  Every path gives bit-identical results.  Drops any
 * captured graph. */
int pflbm_set_step_kernel(pflbm_handle h, int32_t variant);

/* Scheduling options of the step kernels (results do not depend on them).
 * xcd_order: 0 = tile b to workgroup b (the hardware deals workgroups to the 8
 * XCDs round-robin); 1 = each XCD takes one contiguous run of tiles; 2 = whole
 * x-rows of tiles, two tile rows in y at a time, go to one XCD together, so
 * that neighbouring tiles share its L2.  Other values: EINVAL.
 * nontemporal != 0 writes f* and g* with streaming stores.  Defaults:
 * xcd_order 2 for D3Q19 cases, 0 for D2Q9; nontemporal 0.  Drops any captured
 * graph. */
int pflbm_set_step_options(pflbm_handle h, int32_t xcd_order, int32_t nontemporal);

/* Number of step variants for a lattice (see pflbm_set_step_kernel); if tiles
 * is non-NULL, fills up to capacity records of 5 ints: threads (by, bz) of a
 * (64, by, bz) workgroup and the tile (tx, ty, tz) it updates.  (no device
 * work) */
int pflbm_step_variants(int32_t lattice, int32_t* tiles, int32_t capacity);

/* FP16-deviation storage keeps value * 2^k per distribution set.  The current
 * scales of f and g (1 for other storage).  (no device work) */
int pflbm_fp16_scales(pflbm_handle h, double* scale_f, double* scale_g);

/* Sets the FP16 scales (powers of two within 2^-60 .. 2^60) and rescales the
 * stored state to them, exactly unless a stored value leaves the FP16 range.
 * FP16-deviation storage only (else EUNSUPPORTED); refused for a group member
 * (ESTATE).  pflbm_diagnostics and pflbm_group_poll move a scale by themselves
 * when the largest stored magnitude of a set leaves [2^11, 2^14].  Drops any
 * captured graph.  (sync) */
int pflbm_set_fp16_scales(pflbm_handle h, double scale_f, double scale_g);

/* Current fields as FP64 host arrays of nx*ny*nz (u: D arrays, component-major).
 * Any pointer may be NULL.  phi = sum_i g_i (Sec. 2.1.3, Eq. order-parameter);
 * p and u from sum_i f_i and rho u = sum_i c_i f_i + F/2 with F = mu grad phi
 * + F_b (Sec. 2.1.2, the pressure below Eq. GGi), u = 0 on boundary nodes;
 * mu of Eq. (chemical_potencial2).  phi holds the ghost value (Sec. 2.2.2) on
 * ghost nodes and 0 on other solid nodes; p, u and mu are 0 on zeta = 0
 * nodes.  (sync) */
int pflbm_fields(pflbm_handle h, double* phi, double* p, double* u, double* mu);

/* Node classes as nx*ny*nz bytes: bit 0 zeta (fluid or boundary), bit 1 fluid
 * (epsilon = 1), bit 2 ghost.  (host copy, sync-free) */
int pflbm_node_classes(pflbm_handle h, uint8_t* classes);

/* Run the reductions now and fill *d.  Also refreshes the steady-state
 * reference field.  mass: FP64 sum of phi = sum_i g_i (Eq. order-parameter)
 * over fluid and boundary nodes, taken from the stored populations in FP64;
 * s_sum: sum of s = u . grad phi (the source of Eq. F_i sums to -s); theta:
 * contact angle from a least-squares circle / sphere through the phi = 1/2
 * crossings at least diag_width from the wall, against the wall plane (cos theta
 * = -h / R, Sec. 3.1) or the wall circle / sphere (Eq. initialphi_cirref solved
 * for theta, Sec. 3.3); steady_residual: max |phi - phi at the previous call|.
 * (sync) */
int pflbm_diagnostics(pflbm_handle h, pflbm_diag* d);

/* Checkpoint: raw device state (populations, s, step count, and for
 * FP16-deviation storage the scales the populations are stored with).
 * pflbm_state_size gives the byte count; set_state accepts only a blob from a
 * case with identical parameters and takes over the blob's scales (dropping any
 * captured graph when they differ).  Resuming is bit-identical.  (sync) */
int pflbm_state_size(pflbm_handle h, size_t* bytes);
int pflbm_get_state(pflbm_handle h, void* host, size_t bytes);
int pflbm_set_state(pflbm_handle h, const void* host, size_t bytes);

/* Time nsteps (<= 100000) eager steps with HIP events around every kernel
 * launch on the case's stream; avg_ms[k] receives the mean duration in
 * milliseconds per step of kernel kind k for k < nkinds: 0 phi sum, 1 mu
 * stencil, 2 collide-stream (three-kernel path), 3 fused step kernel; kinds the
 * current path does not launch read 0.  The steps count as real steps.  (sync) */
int pflbm_profile(pflbm_handle h, int64_t nsteps, double* avg_ms, int32_t nkinds);

/* Time steps taken so far (-1 for a NULL handle). */
int64_t pflbm_step_count(pflbm_handle h);
void pflbm_destroy(pflbm_handle h);

/* ---------------------------------------------------------------- groups (batched) */

/* A group advances many cases of one lattice and storage together: each step
 * is one launch over a device (case, tile) table (see pflbm_group_set_tile),
 * so small and uneven cases fill the GPU together; full chunks of steps replay
 * a captured HIP graph.  The per-node arithmetic is that of the single-case
 * fused step with the same tile variant, so every member's result is
 * bit-identical to running it alone.  Members are non-owning references:
 * joining a group moves a case's work onto the group's stream (its own stream
 * is restored when it leaves); destroying a member removes it; pflbm_step on a
 * member is refused (PFLBM_ESTATE) while fields, diagnostics and state calls
 * on it stay valid.  hip_stream is borrowed (NULL: the group makes its own). */
int pflbm_group_create(void* hip_stream, pflbm_group* out);
/* Add a case (same lattice and storage as the other members, else EINVAL; a
 * case whose f or g buffer reaches 4 GiB is refused with EUNSUPPORTED, since
 * the batched kernels address populations with 32-bit offsets). */
int pflbm_group_add(pflbm_group g, pflbm_handle h);
/* Remove a member (ESTATE if h is not a member). */
int pflbm_group_remove(pflbm_group g, pflbm_handle h);
/* Number of members, or -1 for a NULL group. */
int pflbm_group_size(pflbm_group g);
/* Advance every member nsteps >= 0 steps.  (async) */
int pflbm_group_step(pflbm_group g, int64_t nsteps);
/* Reductions for every member; d[k] and flags[k] (bit 0 steady, bit 1
 * nonfinite) for member k in insertion order; capacity >= group size.  (sync) */
int pflbm_group_poll(pflbm_group g, pflbm_diag* d, int32_t* flags, int32_t capacity);
/* pflbm_group_poll for callers that cannot allocate device memory (serving
 * loops and harnesses that forbid it): the same reductions and results, with
 * the partial and member records in a static device array of the library
 * instead of buffers it allocates.  Limits: 32768 table entries and 1024
 * members (larger groups: EINVAL).  A group that changed since its last step
 * (members added or removed, launch shape set) needs its table rebuilt, which
 * may allocate: step it first (else ESTATE).  Every call on one GPU shares that
 * array: calls that overlap on a GPU (from two threads, or for two groups on
 * unordered streams) race.  FP16-deviation scale upkeep as in
 * pflbm_group_poll.  (sync) */
int pflbm_group_poll_static(pflbm_group g, pflbm_diag* d, int32_t* flags, int32_t capacity);
/* Launch shape of the batched kernel: step tile variant (-1 = library default)
 * and blocks_per_cu: 0 = one workgroup per table entry (the default; the grid
 * follows the table, so a membership change recaptures the step graph);
 * > 0 = a persistent grid of that many workgroups per CU (capped by occupancy)
 * striding over the table.  Results do not depend on either. */
int pflbm_group_set_tile(pflbm_group g, int32_t variant, int32_t blocks_per_cu);
/* Steps per captured HIP graph (0 = direct launches; odd values round up). */
int pflbm_group_set_graph_chunk(pflbm_group g, int32_t steps);
/* Destroy the group; members stay valid and return to their own streams. */
void pflbm_group_destroy(pflbm_group g);

/* ---------------------------------------------------------------- errors */
const char* pflbm_strerror(int code);
const char* pflbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PFLBM_H */
