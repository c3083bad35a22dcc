// Internal declarations shared by the host ABI (md_api.hip) and the kernel
// files of libmd.so.  Nothing here is part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/md.h"

namespace mdk {

constexpr int kBlock = 256;        // threads per workgroup of the per-atom kernels
// Threads per workgroup of the per-atom pair passes: one wavefront while the
// atoms are too few to give every compute unit several 256-thread workgroups.
inline int atom_block(int64_t n) { return n < 262144 ? 64 : kBlock; }
// Lanes that share the neighbour row of one atom in the per-atom pair passes:
// several while the atoms alone are too few to keep every SIMD busy (each
// lane then waits out a shorter chain of dependent gathers).
constexpr int kRowLanes = 8;
constexpr int64_t kRowSplitAtoms = 262144;
inline int row_lanes(int64_t n) { return n < kRowSplitAtoms ? kRowLanes : 1; }
constexpr int kChunk = 4096;       // atoms per partial sum of the energy reductions
constexpr int kMaxCapacity = 65528; // list entries per atom: a multiple of 8 below 2^16
constexpr int kTileThreads = 1024; // threads of a tiled-pass workgroup (one tile)
constexpr int kHaloCells = 512;    // halo cells a tile may have
constexpr int kTileGlobal = 0, kTileA = 1, kTileB = 2;  // halo modes of a box
constexpr int kTyped = 13;         // kernel kind: spline tables for several species
constexpr int kMaxTypes = 32;      // the type of a neighbour rides in the 5 low bits
                                   // of its (32-byte aligned) row entry

// Per-interval cubic table on a uniform grid: c[4*m + {0,1,2,3}] = a, b, c, d.
struct Table {
    const double *c;
    int n;
    double lo, hi, inv_h;
};

// exp(r) ~ sum_k kExpPoly[k] r^k on |r| <= 0.3466 (just above ln(2)/2, so
// 2^f = exp(f ln 2) for |f| <= 1/2): the degree-10 polynomial interpolating
// exp at the 11 Chebyshev nodes of that interval, computed in 60-digit
// decimal arithmetic; with its coefficients rounded to double its relative
// error is below 3.3e-16 (about three units in the last place).  The leading
// coefficient rounds to exactly 1.
constexpr int kExpDeg = 10;
constexpr double kExpPoly[kExpDeg + 1] = {
    1.0, 1.0000000000000067, 0.5000000000000006, 0.16666666666554406, 0.04166666666657314,
    0.008333333385667814, 0.0013888888932488625, 0.00019841170270400204, 2.480150434696448e-05,
    2.7640180812804505e-06, 2.762635725527078e-07};

// Potential as the kernels see it.  B-spline potentials are converted to
// per-interval tables on the device and evaluated as kind MD_POT_SPLINE.
struct Pot {
    int kind;
    double rc, rc2;
    double c, d, c0, c1, c2, A;        // Finnis-Sinclair
    // SMTB in base 2: V = 2^(av r + bv), rho = 2^(af r + bf), -V' = 2^(av r + bvd),
    // -rho' = 2^(af r + bfd); avn, afn are the slopes of ln V and ln rho
    double av, bv, af, bf, bvd, bfd, avn, afn;
    double ec[kExpDeg + 1];            // kExpPoly[m] ln(2)^m, kernel arguments (scalar registers)
    Table tab[3];                      // V(r), rho(r), F(rho)
    // the force pass's r-grid tables interleaved per interval m (null when the
    // V and rho grids differ): one species [V | rho] (8 doubles), several
    // [V^(ab) | rho^(ab) | rho^(ba) | 0] (16 doubles, index (a nt + b) n + m)
    const double *pair;
    // the same intervals with only what the derivatives need (forces without
    // energies): one species [V_b V_c V_d | rho_b rho_c rho_d] (6 doubles,
    // 48 bytes), several [V^(ab) | rho^(ab) | rho^(ba)] b, c, d and one zero
    // (10 doubles, 80 bytes); null when pair is
    const double *dpair;
    int nt;                            // species; with nt > 1 each Table holds nt*nt (V, rho)
                                       // or nt (F) tables back to back, table a*nt + b
    // cutoffs per pair of types (null: rc for every pair): cut2[a nt + b] =
    // RCUT(a, b)^2, cut2[nt nt + a nt + b] = (RCUT(a, b) + skin)^2
    const double *cut2;
};

// Electron-gas friction of eq. (4) as the kick kernels see it: over half a
// step v^2 -> e v^2 + a along the direction of v, e = exp(-dt / tau_T),
// a = (1 - e) 3 k_B T_e / m in (Angstrom/fs)^2.
struct Thermo {
    double e, a;
    int on;
};

// The friction's exact flow over half a step: with T_i = m v^2 / (3 k_B),
// eq. (4) alone gives d(v^2)/dt = -(2 / tau_T) (v^2 - 3 k_B T_e / m) and keeps
// the direction of v.  An atom at rest has no direction and stays at rest.
__device__ __forceinline__ void friction_flow(const Thermo &th, double &vx, double &vy, double &vz)
{
    double v2 = fma(vz, vz, fma(vy, vy, vx * vx));
    if (v2 > 0.0) {
        double g = sqrt(fma(th.e, v2, th.a)) / sqrt(v2);
        vx *= g;
        vy *= g;
        vz *= g;
    }
}

// Atom state in sorted (cell) order, structure of arrays.
struct State {
    double *x, *y, *z, *vx, *vy, *vz, *fx, *fy, *fz, *xr, *yr, *zr;
    double *xo, *yo, *zo;              // the other position buffer: drift target of a fused force pass
    double *pk;                        // [N][4] packed x, y, z, F'(rho) for neighbour gathers
    int *id;                           // original index of each sorted slot
    double *rho, *Fp, *Femb, *eat;     // density, F'(rho), F(rho), per-atom energy
    double *wat;                       // per-atom virial term sum_j [(F'_i + F'_j) rho' + V'] r
    // several species (null otherwise): type of each slot, type of each
    // original atom, and per type: half-kick factor, friction addend, m / (2 kappa)
    int *type;
    const int *type0;
    const double *tcoef;
    // atom states (null when no atom is frozen): frozen flag of each slot and
    // of each original atom
    unsigned char *frozen;
    const unsigned char *frozen0;
};

// Per-type coefficients (several species): [4 t + k], k as below.
constexpr int kTcKick = 0, kTcFric = 1, kTcHalfM = 2;

// Atom states: a frozen atom keeps zero velocity, so no drift moves it.
__device__ __forceinline__ void hold(const State &st, int i, double &vx, double &vy, double &vz)
{
    if (st.frozen && st.frozen[i]) vx = vy = vz = 0.0;
}

// Half-kick factor and friction addend of atom i: those of its species in
// several-species contexts, else the context's (already in kick and th).
__device__ __forceinline__ void species_kick(const State &st, int i, double &kick, Thermo &th)
{
    if (st.type) {
        const double *c = st.tcoef + 4 * st.type[i];
        kick = c[kTcKick];
        th.a = c[kTcFric];
    }
}

// Per-box geometry (device arrays of length B, box_of of length N).
struct Boxes {
    const double *L, *invL, *rl2, *thr2;
    const int *nc, *cell_off, *atom_off, *box_of;
    const int *tile;                   // per box: tx ty tz gx gy gz tile_cells mode
    const int *tile_off;               // per box: first global tile index [B+1]
    const int *tile_box;               // per global tile: its box
    const int *tile_order;             // per place of the passes' sweep: its tile
};

// Scratch of the list build.
struct Build {
    double *sx, *sy, *sz, *svx, *svy, *svz;
    int *sid;
    int *cell_of, *slot, *cell_count, *cell_start, *tmp, *perm;
    int *bsum;                         // scan block totals [n_cells / 4096 + 2]
    int n_cells;                       // Morton cell slots over all boxes
};

struct NList {
    // [N] per-atom rows: np | ni << 16, pairs without periodic correction at
    // [0, np), pairs across a face at [mn - ni, mn); tiled rows: n | np << 16,
    // the pairs across a face at [np, n)
    int *count;
    int *total;                        // [N]: neighbours found (may exceed mn)
    int *idx;                          // [MN][N], column major (slot-fastest)
    int mn;
    // tiled contexts: the slots of the halo records of tile g, in LDS order,
    // tsrc[g * hmax + k], and their number ttotal[g]; written by each list build
    unsigned *tsrc;
    int *ttotal;
};

// Device words: flags[0] status bits, flags[1] rebuild request,
// flags[2] builds (low), flags[3] steps (low), flags[4] builds (high), flags[5] steps (high),
// flags[6] halt: a list build ran out of row or tile capacity, and every kernel
// of the step sequence does nothing until the host has raised the capacity
// and rebuilt; flags[7] the longest row such a build found; flags[8..9] the
// step counter when md_step began (to tell which step halted).
constexpr int kFlagWords = 16;
constexpr int kHaltWord = 6, kMaxRowWord = 7, kMarkWord = 8;
struct Dev {
    unsigned *flags;
};

struct Ctx;

// Launchers (md_kernels.hip).
void launch_set_state(Ctx &c, const double *pos, const double *vel, hipStream_t s);
void launch_pair_tables(Ctx &c, hipStream_t s);
void launch_refresh_types(Ctx &c, hipStream_t s);
void batched_graph_reset(Ctx &c);

// Context set-up (md_api.hip).  kMeasure counts the workspace bytes only
// (nothing is allocated, copied or launched); kOneShot builds the context in
// `workspace` for one evaluation on `stream` (no capture stream, no graph).
constexpr int kNormal = 0, kMeasure = 1, kOneShot = 2;
int create_context(const md_system *sys, const md_potential *pot, md_ctx **out, void *workspace,
                   size_t workspace_bytes, int mode, hipStream_t stream);

// Device memory of a context (md_api.hip): from hipMalloc, or carved from the
// caller's workspace; sizes are rounded up to 256 bytes.
int ctx_alloc(Ctx &c, void **p, size_t bytes);
void ctx_free(Ctx &c, void *p);
void launch_refresh_frozen(Ctx &c, hipStream_t s);
void launch_get_state(Ctx &c, double *pos, double *vel, hipStream_t s);
void launch_build(Ctx &c, bool gated, hipStream_t s);
void launch_density(Ctx &c, hipStream_t s, bool fp_only = false);  // fp_only: F' alone (tiled)
void launch_embed(Ctx &c, hipStream_t s);
// kick: 0 none, 1 half kick, 2 half kick and the next step's half kick and
// drift into the other position buffer (tiled contexts only)
void launch_force(Ctx &c, bool energy, int kick, hipStream_t s);
void launch_pressure_eval(Ctx &c, hipStream_t s);  // after a force pass with energies
void launch_baro_mu(Ctx &c, hipStream_t s);
void launch_baro_box_scale(Ctx &c, hipStream_t s);
void launch_kick_drift(Ctx &c, hipStream_t s);
void launch_step_end(Ctx &c, hipStream_t s);
void launch_step_mark(Ctx &c, hipStream_t s);
void launch_scatter_scalar(Ctx &c, const double *src, double *dst, hipStream_t s);
void launch_scatter_vec3(Ctx &c, const double *sx, const double *sy, const double *sz,
                         double *dst, hipStream_t s);
void launch_box_sums(Ctx &c, int what, double *out, hipStream_t s);
void launch_get_neighbors(Ctx &c, int32_t *counts, int32_t *ids, int32_t max_cols,
                          hipStream_t s);
void launch_bspline_tables(Ctx &c, const double *theta, hipStream_t s);
void launch_fill_u32(unsigned *p, int n, unsigned v, hipStream_t s);
void launch_clear_bits(Ctx &c, unsigned mask, hipStream_t s);  // status bits off
// Tiled passes (md_tiled.hip).
void tiled_prepare(Ctx &c);
void launch_tile_nlist(Ctx &c, const unsigned *gate, hipStream_t s);
void launch_tile_density(Ctx &c, hipStream_t s, bool fp_only);
void launch_tile_force(Ctx &c, bool energy, int kick, hipStream_t s);
void launch_tile_get_neighbors(Ctx &c, int32_t *counts, int32_t *ids, int32_t cols, hipStream_t s);
void launch_pack_positions(Ctx &c, hipStream_t s);

// Form (2), md_batched.hip.
int batched_prepare(Ctx &c);
int launch_batched_steps(Ctx &c, int nsteps, hipStream_t s);
void batched_invalidate(Ctx &c);
void batched_release(Ctx &c);
// Form (3), md_adjoint.hip.
void launch_adjoint(Ctx &c, const double *g, const double *e, double *gtheta, hipStream_t s);
int adjoint_lanes(int K);
size_t adjoint_scratch_doubles(int64_t N, int K);

struct Ctx {
    int device = 0;
    int64_t N = 0;
    int B = 0;
    double mass = 0, dt = 0, skin = 0;
    Pot pot{};
    int kind_user = 0;                 // kind given at creation (BSPLINE stays BSPLINE here)
    int n_theta = 0;                   // B-spline coefficients per function
    double theta_lo[3]{}, theta_hi[3]{};
    std::vector<int> tab_len;          // doubles per table on the device
    double *tables = nullptr;          // device, 3 tables back to back
    double *theta = nullptr;           // device copy of B-spline coefficients [3K]
    double *pair_tab = nullptr;        // interleaved r-grid tables (Pot::pair)
    double *dpair_tab = nullptr;       // their derivative coefficients (Pot::dpair)
    double *cut_tab = nullptr;         // Pot::cut2 (several species)
    std::vector<double> rc_pair;       // host copy of RCUT(a, b) (empty: rc for every pair)

    // host mirrors of the box geometry
    std::vector<int64_t> box_off;
    std::vector<double> box_len, box_rlist;
    std::vector<int> box_nc, box_cell_off;
    std::vector<int> box_tile;         // per box: tx ty tz gx gy gz tile_cells mode
    int ntiles = 0;
    // tile shapes (cells per tile along x, y, z) md_autotune chooses among:
    // results do not depend on the shape (each atom's neighbours are summed in
    // the same stencil and slot order), only the time does.  Buffers are
    // sized for the largest cell and tile counts among them.
    std::vector<int> tile_shapes;      // 3 per candidate; candidate 0 is the planner's
    int tile_shape = 0;
    int cap_cells = 0, cap_tiles = 0;
    int tile_grid = 1;                 // workgroups of the persistent tiled density pass
    int tile_lanes = 1;                // lanes per atom in the tiled passes (2: few tiles)
    bool tiled = false, tile_feasible = false;
    int hmax = 0;                      // LDS records per tile
    size_t tile_lds = 0;               // dynamic LDS bytes of a tiled-pass workgroup
    int *d_tiles = nullptr;            // tile(8B) | tile_off(B+1) | tile_box(cap) | order(ntiles)
    double *d_boxd = nullptr;          // L | invL | rl2 | thr2, each [B]
    int *d_boxi = nullptr;             // nc | cell_off | atom_off(B+1) | box_of(N)
    Boxes bx{};

    State st{};
    Build bd{};
    NList nl{};
    Dev dev{};

    // energy reductions
    int n_chunks = 0;
    int *d_chunks = nullptr;           // start | end | box_chunk_start(B+1)
    double *d_partial = nullptr;       // [n_chunks]

    // adjoint scratch
    double *adj = nullptr;             // sized at first use
    size_t adj_len = 0;

    // batched persistent kernel (form 2)
    int batch_block = 256;
    int batch_cap = 0;                 // atoms per pack of boxes (0: one box per workgroup)
    int batch_cell_order = 0;          // threads visit atoms in cell order
    bool batched = false;
    bool batch_feasible = false;
    int64_t host_steps = 0;            // steps taken by the persistent kernel
    void *batch = nullptr;             // opaque, owned by md_batched.hip

    // host-side state machine
    bool state_set = false, list_valid = false, density_valid = false, forces_valid = false;
    // caller's buffers bound as the state of record (md_bind): md_step writes back
    double *bound_pos = nullptr, *bound_vel = nullptr;

    // pressure (eq. 6) and Berendsen barostat (eq. 5)
    bool baro_on = false;              // md_step scales coordinates and boxes
    bool baro_mu_valid = false;        // d_baro holds the scale factors of the next step
    double baro_p0 = 0.0, baro_tau = 0.0, baro_beta = 0.0;
    double *d_baro = nullptr;          // per box: mu | strain | rlist | pressure | virial | kinetic | virial sum

    // atom states
    unsigned char *d_frozen = nullptr, *d_frozen0 = nullptr;
    bool any_frozen = false;

    // several species
    int ntypes = 1;
    std::vector<double> type_mass;     // [ntypes]
    int *d_type0 = nullptr, *d_type = nullptr;
    double *d_tcoef = nullptr;         // [4 ntypes]

    // electron-gas thermostat (eq. 4)
    Thermo thermo{1.0, 0.0, 0};
    double thermo_te = 0.0, thermo_tau = 0.0;

    // graph replay of md_step: graphs of graph_steps steps, and one more for
    // the remainder of the last call that was not a multiple of it
    bool use_graph = true;
    int graph_steps = 40;
    hipStream_t cap_stream = nullptr;
    struct StepGraph {
        hipGraphExec_t exec = nullptr;
        int len = 0;                   // steps
        int fused = 0;                 // leading steps with the fused kick and drift
    } graph, tail_graph;

    // allocations to free
    std::vector<void *> allocs;        // device blocks of the context (hipMalloc)
    size_t alloc_bytes = 0;            // bytes handed out by ctx_alloc (256-byte granules)
    char *arena = nullptr;             // caller's workspace (md_create_in): blocks are carved
    size_t arena_size = 0, arena_used = 0;  // from it and never freed
    bool measure = false;              // sizes only: nothing allocated, copied or launched
    bool oneshot = false;              // one evaluation in the static scratch (md_forces_static)
};

}  // namespace mdk

struct md_ctx {
    mdk::Ctx c;
};
