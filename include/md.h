/*
 * md.h -- C ABI of the MI355X many-body MD force path (libmd.so).
 *
 * The library evaluates, on one gfx950 GPU and in double precision, the
 * per-timestep force of embedded-atom-model (EAM) and second-moment
 * tight-binding potentials (Hou et al., Section 2, eqs. 1-3):
 *
 *   E_i  = F(rho_i) + 1/2 sum_{j != i} V(r_ij),   rho_i = sum_{j != i} rho(r_ij)
 *   f_i  = -sum_j [(F'(rho_i) + F'(rho_j)) rho'(r_ij) + V'(r_ij)] (x_i - x_j)/r_ij
 *
 * over full Verlet neighbour lists built from periodic linked cells
 * (Section 3.2), driven by velocity Verlet.  Several independent periodic
 * boxes may share one context (the multiple-box scheme of Section 4.4).
 * Around this path: the pressure of eq. (6) and the Berendsen barostat of
 * eq. (5) (md_pressure, md_set_barostat), the electron-gas thermostat of
 * eq. (4) (md_set_thermostat), several atom species with per-type-pair
 * tables (n_types, md_set_types) and frozen atoms (md_set_frozen).
 *
 * Conventions for every entry point
 *   - Units: Angstrom, eV, fs, amu.  All floating point is IEEE double.
 *   - Per-atom input/output buffers are DEVICE pointers owned by the caller,
 *     in the caller's original atom order.  Vectors are packed [N][3]
 *     (x, y, z of atom 0, then atom 1, ...).  The library never frees them.
 *     The per-atom settings of md_set_types and md_set_frozen are HOST
 *     arrays, validated before they are copied.
 *   - `stream` is a hipStream_t passed as void* (NULL: the null stream).
 *     Calls are stream ordered and asynchronous unless stated otherwise.
 *   - Descriptors passed by pointer (md_system, md_potential) and the host
 *     arrays they reference are read during the call only.
 *   - Return value: MD_OK or a negative MD_ERR_* code.  Argument, capacity
 *     and state errors are detected on the host and returned at once.
 *     Conditions found by kernels set bits in a device status word.  List
 *     capacity is never left short: a list build that finds a row longer
 *     than the capacity (or a tile whose halo exceeds its LDS) is noticed
 *     before any pass reads that list -- builds started by a call
 *     (md_build_neighbors, or the first pass after md_set_state) are waited
 *     for and checked; builds decided on the device inside md_step halt the
 *     step sequence there -- and the library then raises the capacity
 *     (taking memory as md_set_max_neighbors does; on a tile overflow the
 *     context moves to the per-atom passes), builds again, and goes on
 *     (md_step completes the halted step and takes the rest), returning
 *     MD_ERR_NLIST_OVERFLOW only when the capacity cannot be raised.
 *     MD_FLAG_NLIST_OVERFLOW then stays set for md_status.  Table-range and
 *     non-finite conditions are returned by the next md_step (as
 *     MD_ERR_TABLE_RANGE, MD_ERR_NONFINITE, once) or read by md_status().
 *   - A context belongs to the device that was current at md_create(); it
 *     allocates its device workspace there, once (or takes it from the
 *     caller's block, md_create_in).  No entry point allocates device memory
 *     after md_create() except md_set_max_neighbors() and the capacity
 *     increase after a list overflow (see above).
 *   - One context must not be used from two host threads at once.
 */
#ifndef MD_H
#define MD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct md_ctx md_ctx;

/* Return codes. */
enum {
    MD_OK = 0,
    MD_ERR_ARG = -1,             /* invalid argument or descriptor                 */
    MD_ERR_BOX = -2,             /* box shorter than twice the force cutoff        */
    MD_ERR_NLIST_OVERFLOW = -3,  /* a neighbour row exceeded the list capacity     */
    MD_ERR_TABLE_RANGE = -4,     /* a table lookup fell outside the tabulated grid */
    MD_ERR_NONFINITE = -5,       /* a coordinate became NaN or infinite            */
    MD_ERR_DEVICE = -6,          /* a HIP runtime call failed                      */
    MD_ERR_STATE = -7,           /* call out of order (e.g. no state set)          */
    MD_ERR_NOMEM = -8,           /* device allocation failed                       */
    MD_ERR_SCRATCH = -9          /* md_forces_static: the system's buffers exceed
                                    the library's static device array            */
};

/* Bits of the device status word (md_status). */
enum {
    MD_FLAG_NLIST_OVERFLOW = 1u,
    MD_FLAG_TABLE_RANGE = 2u,
    MD_FLAG_NONFINITE = 4u,
    MD_FLAG_TILE_OVERFLOW = 8u,  /* a tile's halo exceeded its LDS capacity        */
    MD_FLAG_BOX_RANGE = 16u      /* the barostat would have shrunk a box below its
                                    cell grid (cells narrower than the list radius,
                                    or the list radius >= half the box); that
                                    box was left unscaled                          */
};

/* Potential kinds. */
enum {
    MD_POT_FS = 1,      /* Finnis-Sinclair: params c d c0 c1 c2 A
                           V(r) = (r-c)^2 (c0 + c1 r + c2 r^2) for r < c,
                           rho(r) = (r-d)^2 for r < d, F(rho) = -A sqrt(rho)  */
    MD_POT_SMTB = 2,    /* second-moment tight binding: params A xi p q r0
                           V(r) = 2A exp(-p (r/r0 - 1)),
                           rho(r) = xi^2 exp(-2q (r/r0 - 1)), F(rho) = -sqrt(rho)
                           (the SETB form of Section 4); A, xi, p, q, r0 > 0
                           and V, rho, |V'|, |rho'| within 2^-1000 .. 2^1000
                           on [0, rc], else MD_ERR_ARG                          */
    MD_POT_SPLINE = 3,  /* lookup tables (Section 3.3): for V(r), rho(r), F(rho)
                           each a uniform grid [lo, hi] of n intervals with cubic
                           coefficients (a, b, c, d): S = a + b t + c t^2 + d t^3,
                           t = (x - lo)/h - m in interval m, h = (hi - lo)/n    */
    MD_POT_BSPLINE = 4  /* uniform cubic B-splines: for each function K
                           coefficients theta_0..theta_{K-1} over K-3 intervals
                           of [lo, hi]; S = sum_l theta_{m+l} b_l(t)            */
};

typedef struct {
    int32_t kind;            /* MD_POT_*                                          */
    int32_t n_params;        /* entries of params (FS 6, SMTB 5, else 0)          */
    double rc;               /* force cutoff: pairs with r < rc interact          */
    const double *params;    /* host, analytic parameters                         */
    const double *tab[3];    /* host; V(r), rho(r), F(rho):
                                SPLINE  [n_tab[k]][4] coefficients,
                                BSPLINE [n_tab[k]] coefficients                   */
    int32_t n_tab[3];        /* SPLINE: intervals; BSPLINE: coefficients          */
    double lo[3], hi[3];     /* grid range of each table                          */
    int32_t n_types;         /* species T (eq. 1: V^(ab), rho^(ab) for an atom of
                                type a with a neighbour of type b).  0 or 1: one
                                species.  T in 2..32: SPLINE only; tab[0] holds T*T
                                tables V^(ab) back to back (table a*T + b, each
                                n_tab[0] intervals; V^(ab) = V^(ba) required),
                                tab[1] T*T tables rho^(ab) (the density at an atom
                                of type a contributed by an atom of type b), tab[2]
                                T tables F^(a); the V and rho tables share one
                                grid (lo[0] = lo[1], hi[0] = hi[1], n_tab[0] =
                                n_tab[1]).  Atom types come from md_set_types
                                (default: all 0).                                 */
    const double *rc_pair;   /* host [T*T] or NULL: the cutoff RCUT(a, b) of each
                                pair of types (Sections 3.2-3.3), index a*T + b,
                                symmetric, each in (0, rc]; a pair interacts
                                while r < RCUT(a, b) and is listed while r <
                                min(RCUT(a, b) + skin, box_len/2 - 1e-9).  NULL:
                                rc for every pair.  Several species only.        */
} md_potential;

typedef struct {
    int32_t n_boxes;            /* B >= 1 independent periodic cubic boxes          */
    int32_t max_neighbors;      /* list capacity per atom (rounded up to a multiple
                                   of 8, at most 65528); 0 = estimate from density   */
    const int64_t *box_offset;  /* host [B+1]: atoms of box b are
                                   box_offset[b] .. box_offset[b+1]-1; [0] = 0       */
    const double *box_len;      /* host [B]: edge length of each cubic box           */
    double mass;                /* amu, all atoms                                    */
    double dt;                  /* fs                                                */
    double skin;                /* Verlet skin (Angstrom); the list radius of box b is
                                   min(rc + skin, box_len[b]/2 - 1e-9), and the list is
                                   rebuilt when an atom of the box has moved more than
                                   half of (list radius - rc) since the last build    */
} md_system;

/* Create a context on the current device (Section 3.1: the device-resident
 * arrays of positions, velocities, forces, densities, list counts and the
 * list, with the type and state arrays when used, allocated once; Section
 * 3.3: the potential's tables prepared on the host once and uploaded).
 * Validates the descriptors (MD_ERR_ARG), requires box_len[b] > 2 rc for
 * every box (MD_ERR_BOX), uploads the potential, and allocates all device
 * memory of the context. */
int md_create(const md_system *sys, const md_potential *pot, md_ctx **out);

/* Device bytes a context for these descriptors holds (*bytes): the size of
 * the workspace md_create_in needs.  Host arithmetic only: the descriptors
 * are validated as md_create does and every buffer of such a context is
 * counted, but nothing is allocated, copied or launched on the device, so
 * the query also answers for systems larger than the free device memory. */
int md_workspace_size(const md_system *sys, const md_potential *pot, size_t *bytes);

/* As md_create, but every device buffer of the context (state in cell
 * order, cells, neighbour list, densities, tables, flags, scratch) is carved
 * from the caller's device workspace of `bytes` bytes (256-byte aligned,
 * else MD_ERR_ARG; too small: MD_ERR_NOMEM).  The library then allocates no
 * device memory for this context, ever: md_set_max_neighbors takes a new
 * list from what remains of the workspace (MD_ERR_NOMEM when it does not
 * fit) and the old one is not returned.  The caller frees the workspace
 * after md_destroy. */
int md_create_in(const md_system *sys, const md_potential *pot, void *workspace, size_t bytes,
                 md_ctx **out);

/* Free every device and host resource of the context. */
void md_destroy(md_ctx *ctx);

/* Human-readable text of a return code. */
const char *md_strerror(int code);

/* Replace the potential: same kind, table sizes and cutoff rc as at
 * creation (MD_ERR_ARG otherwise; rc sets the list radius, the cells and the
 * rebuild threshold).  Cutoffs per pair of types may change; the lists are
 * then built again before the next pass. */
int md_set_potential(md_ctx *ctx, const md_potential *pot, void *stream);

/* B-spline potentials only: upload 3K coefficients (device pointer, order
 * V, rho, F) and convert them on the device to per-interval cubics.  A
 * stream-ordered device copy and two kernels, no allocation and no host
 * synchronisation: the call may be captured in a HIP graph. */
int md_set_theta(md_ctx *ctx, const double *theta, void *stream);

/* Load positions pos[N][3] and velocities vel[N][3] (vel may be NULL: zero).
 * The next pass rebuilds the neighbour list first. */
int md_set_state(md_ctx *ctx, const double *pos, const double *vel, void *stream);

/* Bind caller-owned device buffers pos[N][3] and vel[N][3] (original atom
 * order) as the state of record (the paper's device-resident position and
 * velocity arrays of Section 3.1, owned by the caller): the state is loaded
 * from them now, as by md_set_state (vel NULL: zero velocities), and every
 * md_step writes the new positions and velocities back into them (vel NULL:
 * positions only), stream ordered, before it returns; between calls the
 * caller reads them in place.  A caller who writes to the bound buffers binds
 * them again (or calls md_set_state) so that the context takes the change.
 * The buffers must stay valid while bound; pos = vel = NULL unbinds. */
int md_bind(md_ctx *ctx, double *pos, double *vel, void *stream);

/* Copy the current positions and velocities out (either may be NULL).
 * Positions are wrapped into the box at each list build and integrated
 * without wrapping in between. */
int md_get_state(md_ctx *ctx, double *pos, double *vel, void *stream);

/* List build (Section 3.2): wrap positions into each box, bin atoms into
 * cells of edge >= list radius, sort them by (cell, original index) with a
 * counting sort, and build the full neighbour list of every atom (all j != i
 * of the same box within the list radius under the minimum image: x_j - x_i,
 * then the periodic shift, then (dx dx + dy dy) + dz dz with every product
 * and sum rounded on its own, strict <; every pass tests r < rc on the same
 * arithmetic).  Waits for the build; raises the capacity and builds again
 * when a row did not fit. */
int md_build_neighbors(md_ctx *ctx, void *stream);

/* Density pass (Fig. 5, eq. 3) with the embedding fused: rho_i = sum of
 * rho(r_ij) over listed j with r_ij < rc (r_ij < RCUT(a, b) with cutoffs per
 * pair of types).  rho_out[N] may be NULL. */
int md_density(md_ctx *ctx, double *rho_out, void *stream);

/* Embedding pass (eq. 1: F(rho); Section 4: F = -sqrt(rho) for the
 * tight-binding form): F(rho_i) and F'(rho_i) of the last density pass.
 * Either output [N] may be NULL. */
int md_embed(md_ctx *ctx, double *F_out, double *Fp_out, void *stream);

/* Force pass (Fig. 6, eq. 3) after md_density: forces f_out[N][3], per-atom
 * energies e_atom[N] = F(rho_i) + 1/2 sum_j V(r_ij), and per-box energies
 * e_box[B] (deterministic sums).  Any output may be NULL.  When no energy is
 * asked for and the forces of the current state are already computed (after
 * md_step, including md_step(ctx, 0, ...)), no pass runs: f_out receives the
 * forces as the kernel that computed them left them (for several boxes
 * stepped by the persistent multi-box stepper, that stepper's own force
 * evaluation). */
int md_forces(md_ctx *ctx, double *f_out, double *e_atom, double *e_box, void *stream);

/* The time integration of Section 3.3, with velocity Verlet in place of the
 * paper's predictor-corrector and a displacement test in place of its fixed
 * list refresh: nsteps of half kick, drift, conditional list rebuild
 * decided on the device, density + embedding, force, half kick.  Brings the
 * list and forces up to date first if needed (nsteps = 0 does only that,
 * with the kernels that would take the steps).  The steps are captured in
 * HIP graphs of MD_OPT_GRAPH_STEPS steps (and one of the remainder) and
 * replayed (captured again after a change of settings, tiling or list
 * capacity).  Waits for the steps and reads the device status word at the
 * end: a list that outgrew its capacity
 * inside the steps is handled as described at the top (with several boxes
 * in the persistent stepper, the call is taken again from its start state
 * with the larger capacity); MD_ERR_TABLE_RANGE or MD_ERR_NONFINITE report
 * those conditions (the state is then the one the kernels reached). */
int md_step(md_ctx *ctx, int nsteps, void *stream);

/* Kinetic energy per box, ke_box[B] = sum m v^2 / 2 (eV): the kinetic part
 * of the pressure of eq. (6). */
int md_kinetic(md_ctx *ctx, double *ke_box, void *stream);

/* Neighbour rows in original indices: counts[N] and ids[N][max_cols]
 * (row order is the device's summation order; rows longer than max_cols
 * are cut).  Synchronises the stream. */
int md_get_neighbors(md_ctx *ctx, int32_t *counts, int32_t *ids, int32_t max_cols,
                     void *stream);

/* Capacity of the neighbour list per atom. */
int md_max_neighbors(const md_ctx *ctx, int32_t *out);

/* Reallocate the list for a new capacity; the next pass rebuilds it. */
int md_set_max_neighbors(md_ctx *ctx, int32_t max_neighbors);

/* Synchronise the stream, return the device status bits in *flags and clear
 * them.  Also reports counters[0] = list builds and counters[1] = steps
 * since creation (counters may be NULL). */
int md_status(md_ctx *ctx, void *stream, uint32_t *flags, int64_t *counters);

/* Form (3): vector-Jacobian product of the forces and per-box energies with
 * respect to the B-spline coefficients (MD_POT_BSPLINE only).  g[N][3] =
 * dL/df_i, e[B] = dL/dE_b (device); writes gtheta[3K] (device, order V, rho,
 * F).  Recomputes rho, F'(rho) and F''(rho) from the current positions and
 * list; the reduction order is fixed, so results are bitwise reproducible.
 * Contexts with more than 2,730 coefficients per function are refused by
 * md_create (MD_ERR_ARG: the per-atom columns must fit in LDS).  Once the
 * list is current (any earlier pass) the call only launches kernels on the
 * stream, with no allocation or synchronisation, so a forward pass and this
 * call may be captured together in a HIP graph. */
int md_adjoint(md_ctx *ctx, const double *g, const double *e, double *gtheta, void *stream);

/* Instantaneous pressure per box, eq. (6) of Section 2:
 * P_b = (N k_B T + W_b / 3) / V_b with N k_B T = (2/3) E_kin,b.  For a periodic
 * box the sum over atoms f_i . r_i is taken in its pair form
 * W_b = sum over pairs i<j of r_ij . f_ij (r_ij the minimum-image separation,
 * f_ij the pair contribution of eq. (3) to f_i), which the force pass
 * accumulates per atom.  Runs the force pass with energies (as md_forces)
 * and writes p_box[B] (eV/Angstrom^3) and w_box[B] (eV), device pointers,
 * either may be NULL but not both. */
int md_pressure(md_ctx *ctx, double *p_box, double *w_box, void *stream);

/* Berendsen barostat, eq. (5) of Section 2, applied by md_step: after the
 * drift of every step, all coordinates of box b and its edge are multiplied
 * by mu_b = [1 - beta (dt / tau) (p0 - P_b)]^(1/3), P_b the pressure at the
 * end of the previous step (of the current state for the first step).  The
 * paper's eq. (5) is this form with beta = 1 in its units; beta is the
 * coupling compressibility (Angstrom^3/eV), p0 the target (eV/Angstrom^3),
 * tau the coupling time (fs).  tau > 0 switches the barostat on (beta > 0
 * and finite values required, else MD_ERR_ARG); tau <= 0 switches it off.
 * While it is on, md_step uses the merged-box path for several boxes, the
 * list radius of each box stays fixed, and the list is also rebuilt when the
 * strain since the last build could bring a listed-out pair inside the
 * cutoff; a box that would shrink below its cell grid is left unscaled and
 * raises MD_FLAG_BOX_RANGE. */
int md_set_barostat(md_ctx *ctx, double p0, double tau, double beta);

/* Atom states (Section 3.1: some atoms are not allowed to move): frozen is a
 * HOST array [N] in the original atom order, nonzero for an atom that is
 * frozen; NULL (or all zero) frees every atom.  A frozen atom keeps zero
 * velocity through every kick of md_step (its velocity is zeroed at once),
 * so it never moves; it still takes part in the density and force passes
 * and acts on the free atoms.  Refused (MD_ERR_ARG) while the barostat is
 * on, and md_set_barostat refuses to switch on while an atom is frozen: the
 * scaling of eq. (5) would move frozen atoms. */
int md_set_frozen(md_ctx *ctx, const uint8_t *frozen);

/* Species of the atoms (several-species contexts, n_types = T > 1): types is
 * a HOST array [N] in the original atom order with values in [0, T);
 * type_mass a host array [T] of masses (amu, > 0), or NULL for the system
 * mass for every species.  Validated on the host (MD_ERR_ARG on a value out
 * of range, or when the context has one species).  The force of eq. (3)
 * then reads, with a the type of atom i and b that of atom j,
 *   f_i = -sum_j [F^(a)'(rho_i) rho^(ab)'(r) + F^(b)'(rho_j) rho^(ba)'(r)
 *                 + V^(ab)'(r)] (x_i - x_j) / r,
 * and every kick, the friction of md_set_thermostat and the kinetic energy
 * take the mass of the atom's species (in the merged-box kernels and in the
 * persistent multi-box stepper alike). */
int md_set_types(md_ctx *ctx, const int32_t *types, const double *type_mass);

/* Electron-gas thermostat, eq. (4) of Section 2, applied by md_step: each
 * atom feels the friction -(m / tau_t) ((T_i - T_e) / T_i) v_i, with T_i =
 * m v_i^2 / (3 k_B) its instantaneous temperature and T_e (K) the electron
 * temperature; tau_t (fs) is the coupling time.  The friction alone keeps the
 * direction of v_i and relaxes v_i^2 exponentially to 3 k_B T_e / m at rate
 * 2 / tau_t; md_step applies that exact flow over half a step before the
 * first half kick and after the second one of every step (an atom at rest
 * stays at rest).  Every box shares T_e and tau_t.  tau_t > 0 switches the
 * thermostat on (T_e >= 0 and finite required, else MD_ERR_ARG); tau_t <= 0
 * switches it off; a NaN or infinite tau_t is MD_ERR_ARG.  Works with the
 * barostat (the pressure then includes the kinetic term after the flow). */
int md_set_thermostat(md_ctx *ctx, double t_e, double tau_t);

/* Current box edges (host box_len[B]; synchronises stream). */
int md_get_box(md_ctx *ctx, double *box_len, void *stream);

/* Autotuner.  Contexts whose md_step runs the persistent multi-box stepper
 * (several boxes): times the block shapes of the stepper on the context's own
 * boxes (20 steps each after a warm-up): workgroup sizes 256, 512 and 1024,
 * each with one box per workgroup and with packs of small boxes of up to one
 * and two workgroups' worth of atoms, in index and in cell visiting order.
 * Keeps the fastest as MD_OPT_BATCH_BLOCK, MD_OPT_BATCH_PACK and
 * MD_OPT_BATCH_ORDER and writes the workgroup size to *block (host).  The
 * cell grid of each of these boxes is not tuned: it is the grid of cells at
 * least the list radius wide, because each atom's neighbour order (and so
 * the rounding of its sums) follows that grid, and tuning must not change
 * results.  Other contexts that can be tiled (one box, or boxes stepped by
 * the merged-box kernels; not with the barostat): times the passes of a step
 * (density, force with the fused kicks, a tenth of a list build) with the
 * per-atom kernels and with the tiled kernels in each candidate tile shape
 * (a shape whose halo does not fit a tile's LDS on the current state is
 * passed over, and no MD_FLAG_TILE_OVERFLOW is left behind for it),
 * and keeps the fastest as MD_OPT_TILED and MD_OPT_TILE_SHAPE (small systems,
 * with fewer tiles than the GPU has room for, are often faster per atom; the
 * best tile shape depends on the atoms per cell); *block is then the
 * unchanged MD_OPT_BATCH_BLOCK.  Positions and velocities are restored
 * afterwards, and the next md_step rebuilds the lists and recomputes the
 * forces from them: called between md_set_state and the first md_step, the
 * trajectory is bitwise that of an untuned context with the chosen settings
 * (tiled or per-atom passes, tile shape).  Synchronises.  Other contexts are left unchanged. */
int md_autotune(md_ctx *ctx, void *stream, int32_t *block);

/* Benchmarking: launch one pass `reps` times on `stream`, bracketed by HIP
 * events recorded on that stream, and return the mean duration per launch in
 * *avg_ms (synchronises).  Passes: MD_PASS_BUILD (list build), MD_PASS_DENSITY
 * (density + embedding), MD_PASS_FORCE (force + half kick), MD_PASS_KICK_DRIFT,
 * MD_PASS_FORCE_STEP (the force pass as most steps of md_step run it in tiled
 * contexts: force, half kick, and the next step's half kick and drift into the
 * second position buffer; elsewhere the same as MD_PASS_FORCE).  Positions and
 * velocities are restored afterwards, so timing leaves the trajectory
 * unchanged, except that timed list builds leave the state as a list build
 * does (wrapped into the box and re-sorted) and the next pass builds again:
 * timing MD_PASS_BUILD acts as one list rebuild at that point. */
enum {
    MD_PASS_BUILD = 0,
    MD_PASS_DENSITY = 1,
    MD_PASS_FORCE = 2,
    MD_PASS_KICK_DRIFT = 3,
    MD_PASS_FORCE_STEP = 4,
    MD_PASS_PRESSURE = 5   /* force pass with energies and the virial, then the
                              per-box pressure of md_pressure                  */
};
int md_time_pass(md_ctx *ctx, int32_t pass, int32_t reps, void *stream, double *avg_ms);

/* Options. */
enum {
    MD_OPT_BATCHED = 1,     /* multi-box md_step: 1 persistent kernel, a workgroup per
                               box or pack of boxes (Section 4.4's many-box runs)
                               (default when B > 1), 0 the merged-box kernels     */
    MD_OPT_BATCH_BLOCK = 2, /* workgroup size of the persistent kernel (256/512/1024) */
    MD_OPT_USE_GRAPH = 3,   /* md_step replays a captured HIP graph (default 1)     */
    MD_OPT_GRAPH_STEPS = 4, /* steps per captured graph (default 40; in tiled
                               contexts all but the last one or two steps of a
                               graph fuse the next kick and drift into the force
                               pass, with bitwise the same trajectory).  The
                               remainder of an md_step call that is not a
                               multiple runs as one more graph of that many
                               steps (kept for the next call with the same
                               remainder); a single step is launched directly  */
    MD_OPT_TILED = 5,       /* 1: list build, density and force stage each tile's
                               neighbour records in LDS (default where the tiles
                               fit); 0: per-atom kernels gathering from HBM       */
    MD_OPT_BATCH_PACK = 6,  /* persistent kernel: a workgroup takes one box (0, the
                               default) or a pack of consecutive boxes of the
                               size-sorted order holding at most this many atoms
                               together (a larger box still goes alone); 0..65535 */
    MD_OPT_BATCH_ORDER = 7, /* persistent kernel: threads take a pack's atoms in
                               index order (0, default) or in the cell order of
                               the last binning (1).  Neither this nor
                               MD_OPT_BATCH_PACK or MD_OPT_BATCH_BLOCK changes
                               any result: each atom's arithmetic is the same  */
    MD_OPT_TILE_SHAPE = 8,  /* tiled passes: which of the context's candidate
                               tile shapes (cells per tile along each axis)
                               cuts its boxes into tiles, 0 .. MD_OPT_TILE_SHAPES
                               - 1 (0: the planner's choice, the default).  The
                               lists are the same for every shape and each
                               atom's neighbours are visited in the same order;
                               only the atoms of a tile beyond one per thread
                               of its workgroup (at most 64 of them) have their
                               rows summed by 16 lanes, so results differ
                               between shapes in rounding only.  The next pass
                               builds the lists again                          */
    MD_OPT_TILE_SHAPES = 9, /* read only: number of candidate tile shapes (1 for
                               systems of few tiles)                           */
    MD_OPT_TILE_DIMS = 10   /* read only: cells per tile along x, y and z of the
                               current tile shape, x | y << 8 | z << 16 (boxes
                               with fewer than the largest + 2 cells per axis
                               are one tile each); 0 when the context cannot
                               run the tiled passes                            */
};
int md_set_option(md_ctx *ctx, int32_t key, int64_t value);
int md_get_option(const md_ctx *ctx, int32_t key, int64_t *value);

/* For callers that cannot allocate device memory (no hipMalloc of their own
 * and none by the library: tight serving loops, harnesses that forbid
 * allocation).  Forces f_out[N][3], per-atom energies e_atom[N] and per-box
 * energies e_box[B] of the positions pos[N][3] (device pointers, original
 * order; outputs may be NULL), as md_create + md_set_state + md_forces would
 * compute them, with every device buffer (state, cells, list, densities,
 * tables, flags, partial sums) carved from one static array of
 * md_static_bytes() bytes (64 MiB) that the library holds on each device it
 * runs on until the process ends.  The descriptors are validated as by
 * md_create; a system whose buffers exceed the array is refused with
 * MD_ERR_SCRATCH (md_workspace_size gives its size).  Synchronises `stream`
 * before (earlier calls on it may still read the array) and after (the
 * device status word is read): list or tile overflow returns
 * MD_ERR_NLIST_OVERFLOW (raise sys->max_neighbors), a table lookup out of
 * range MD_ERR_TABLE_RANGE, a non-finite coordinate MD_ERR_NONFINITE.  The
 * array is shared by every call on a device and keeps the last call's
 * contents (each call initialises what it reads): calls that overlap on one
 * device, from different streams or host threads, race. */
int md_forces_static(const md_system *sys, const md_potential *pot, const double *pos,
                     double *f_out, double *e_atom, double *e_box, void *stream);
size_t md_static_bytes(void);

#ifdef __cplusplus
}
#endif
#endif /* MD_H */
