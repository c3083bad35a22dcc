// Host implementation of the C ABI declared in include/md.h.
//
// A context owns one device workspace sized at creation (allocated, or
// carved from the caller's block): the sorted atom state, the cell
// structure, the neighbour list, per-box geometry, tables, partial sums and
// the status word.  Entry points enqueue kernels on the caller's
// stream; md_step replays a captured HIP graph of several velocity-Verlet
// steps in which the list rebuild is decided on the device, so the host
// never waits inside a trajectory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "md_internal.h"

using namespace mdk;

#define HIP_TRY(call)                              \
    do {                                           \
        if ((call) != hipSuccess) return MD_ERR_DEVICE; \
    } while (0)

namespace {

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Device operations of context set-up.  A context that only measures its
// workspace (md_workspace_size) hands out no memory, so they do nothing there.
int h2d(const Ctx &c, void *dst, const void *src, size_t bytes)
{
    if (c.measure) return MD_OK;
    return hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess ? MD_OK : MD_ERR_DEVICE;
}

int zero(const Ctx &c, void *dst, size_t bytes)
{
    if (c.measure) return MD_OK;
    return hipMemset(dst, 0, bytes) == hipSuccess ? MD_OK : MD_ERR_DEVICE;
}

template <class T>
int dev_alloc(Ctx &c, T **p, size_t count)
{
    void *q = nullptr;
    int rc = ctx_alloc(c, &q, (count == 0 ? 1 : count) * sizeof(T));
    *p = static_cast<T *>(q);
    return rc;
}

#define ALLOC(ptr, n)                          \
    do {                                       \
        int rc_ = dev_alloc(c, &(ptr), (n));   \
        if (rc_ != MD_OK) return rc_;          \
    } while (0)

double list_radius(double rc, double skin, double L)
{
    double r = rc + skin, half = 0.5 * L - 1e-9;
    return r < half ? r : half;
}

int cells_per_dim(double L, double rl)
{
    int nc = (int)std::floor(L / rl);
    while (nc > 1 && L / nc < rl) --nc;
    return nc < 1 ? 1 : nc;
}

int check_potential(const md_potential *p)
{
    if (!p || !(p->rc > 0.0)) return MD_ERR_ARG;
    if (p->n_types < 0 || p->n_types > kMaxTypes) return MD_ERR_ARG;
    if (p->rc_pair && p->n_types < 2) return MD_ERR_ARG;
    if (p->n_types > 1) {
        // several species: spline tables, V and rho on one grid
        if (p->kind != MD_POT_SPLINE) return MD_ERR_ARG;
        if (p->lo[0] != p->lo[1] || p->hi[0] != p->hi[1] || p->n_tab[0] != p->n_tab[1])
            return MD_ERR_ARG;
        if (!p->tab[0] || p->n_tab[0] < 1) return MD_ERR_ARG;
        // V^(ab) = V^(ba), coefficient for coefficient
        const int T = p->n_types;
        if (p->rc_pair)
            for (int a = 0; a < T; ++a)
                for (int b = 0; b < T; ++b) {
                    double v = p->rc_pair[a * T + b];
                    if (!(v > 0.0 && v <= p->rc) || v != p->rc_pair[b * T + a]) return MD_ERR_ARG;
                }
        const size_t n0 = 4 * (size_t)p->n_tab[0];
        for (int a = 0; a < T; ++a)
            for (int b = a + 1; b < T; ++b)
                if (std::memcmp(p->tab[0] + (size_t)(a * T + b) * n0,
                                p->tab[0] + (size_t)(b * T + a) * n0, n0 * sizeof(double)) != 0)
                    return MD_ERR_ARG;
    }
    switch (p->kind) {
    case MD_POT_FS: return (p->params && p->n_params >= 6) ? MD_OK : MD_ERR_ARG;
    case MD_POT_SMTB: return (p->params && p->n_params >= 5) ? MD_OK : MD_ERR_ARG;
    case MD_POT_SPLINE:
    case MD_POT_BSPLINE:
        for (int k = 0; k < 3; ++k) {
            int need = p->kind == MD_POT_SPLINE ? 1 : 4;
            if (!p->tab[k] || p->n_tab[k] < need || !(p->hi[k] > p->lo[k])) return MD_ERR_ARG;
        }
        if (p->kind == MD_POT_BSPLINE && (p->n_tab[0] != p->n_tab[1] || p->n_tab[0] != p->n_tab[2]))
            return MD_ERR_ARG;
        // the adjoint keeps 3K coefficient sums per atom in LDS
        if (p->kind == MD_POT_BSPLINE && adjoint_lanes(p->n_tab[0]) == 0) return MD_ERR_ARG;
        return MD_OK;
    }
    return MD_ERR_ARG;
}

void graph_reset(Ctx &c)
{
    for (Ctx::StepGraph *g : {&c.graph, &c.tail_graph}) {
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        *g = Ctx::StepGraph{};
    }
    batched_graph_reset(c);
}

// Analytic constants and device tables of a potential.
int upload_potential(Ctx &c, const md_potential *p, hipStream_t s, bool first)
{
    Pot &q = c.pot;
    q.rc = p->rc;
    q.rc2 = p->rc * p->rc;
    if (p->kind == MD_POT_FS) {
        q.kind = MD_POT_FS;
        q.nt = 1;
        q.pair = q.dpair = nullptr;
        q.c = p->params[0];
        q.d = p->params[1];
        q.c0 = p->params[2];
        q.c1 = p->params[3];
        q.c2 = p->params[4];
        q.A = p->params[5];
    } else if (p->kind == MD_POT_SMTB) {
        q.kind = MD_POT_SMTB;
        q.nt = 1;
        q.pair = q.dpair = nullptr;
        double A = p->params[0], xi = p->params[1], pp = p->params[2], qq = p->params[3],
               r0 = p->params[4];
        if (!(A > 0.0 && xi > 0.0 && r0 > 0.0 && pp > 0.0 && qq > 0.0)) return MD_ERR_ARG;
        // V = 2A exp(-p (r/r0 - 1)) = exp(av r + bv), rho = xi^2 exp(-2q (r/r0 - 1)) =
        // exp(af r + bf); the derivatives as single exponentials, V' = av V =
        // -exp(av r + bv + ln|av|); all four stored in base 2 (times log2 e)
        const long double log2e = 1.442695040888963407359924681001892137L;
        const long double ln2 = 0.693147180559945309417232121458176568L;
        long double av = -(long double)pp / r0, bv = pp + std::log(2.0L * A);
        long double af = -2.0L * qq / r0, bf = 2.0L * qq + 2.0L * std::log((long double)xi);
        long double bvd = bv + std::log(-av), bfd = bf + std::log(-af);
        q.avn = (double)av;
        q.afn = (double)af;
        q.av = (double)(av * log2e);
        q.bv = (double)(bv * log2e);
        q.af = (double)(af * log2e);
        q.bf = (double)(bf * log2e);
        q.bvd = (double)(bvd * log2e);
        q.bfd = (double)(bfd * log2e);
        // the device 2^t assumes |t| <= 1000 for every r in [0, rc]; t is linear in r
        const double slope_offset[4][2] = {{q.av, q.bv}, {q.av, q.bvd}, {q.af, q.bf}, {q.af, q.bfd}};
        for (const auto &so : slope_offset)
            for (double t : {so[1], so[0] * q.rc + so[1]})
                if (!(std::fabs(t) <= 1000.0)) return MD_ERR_ARG;
        static_assert(kExpPoly[0] == 1.0, "leading exp coefficient");
        long double w = 1.0L;
        for (int m = 0; m <= kExpDeg; ++m, w *= ln2) q.ec[m] = (double)(kExpPoly[m] * w);
    } else {
        const int T = std::max(1, (int)p->n_types);
        q.kind = T > 1 ? kTyped : MD_POT_SPLINE;
        // tables per function: T*T for V and rho, T for F (one of each for one species)
        const int per[3] = {T * T, T * T, T};
        if (!first && T != c.ntypes) return MD_ERR_ARG;
        if (first) {
            size_t total = 0;
            c.tab_len.assign(3, 0);
            for (int k = 0; k < 3; ++k) {
                int nint = p->kind == MD_POT_SPLINE ? p->n_tab[k] : p->n_tab[k] - 3;
                c.tab_len[k] = 4 * nint * per[k];
                total += (size_t)c.tab_len[k];
            }
            ALLOC(c.tables, total);
            if (p->kind == MD_POT_BSPLINE) {
                c.n_theta = p->n_tab[0];
                ALLOC(c.theta, 3 * (size_t)c.n_theta);
            }
        } else {
            for (int k = 0; k < 3; ++k) {
                int nint = p->kind == MD_POT_SPLINE ? p->n_tab[k] : p->n_tab[k] - 3;
                if (c.tab_len[k] != 4 * nint * per[k]) return MD_ERR_ARG;
            }
        }
        q.nt = T;
        size_t off = 0;
        for (int k = 0; k < 3; ++k) {
            int nint = c.tab_len[k] / (4 * per[k]);
            q.tab[k].c = c.tables + off;
            q.tab[k].n = nint;
            q.tab[k].lo = p->lo[k];
            q.tab[k].hi = p->hi[k];
            q.tab[k].inv_h = nint / (p->hi[k] - p->lo[k]);
            off += c.tab_len[k];
        }
        // the force pass reads V and rho of one interval together when they share a grid
        const bool shared = q.tab[0].n == q.tab[1].n && p->lo[0] == p->lo[1] && p->hi[0] == p->hi[1];
        // sized at creation for the V grid, so a later potential with shared grids fits
        if (first) {
            ALLOC(c.pair_tab, (size_t)(T > 1 ? 16 : 8) * T * T * q.tab[0].n);
            ALLOC(c.dpair_tab, (size_t)(T > 1 ? 10 : 6) * T * T * q.tab[0].n);
        }
        q.pair = shared ? c.pair_tab : nullptr;
        q.dpair = shared ? c.dpair_tab : nullptr;
        // cutoffs per pair of types: RCUT^2 and (RCUT + skin)^2
        if (first && T > 1) ALLOC(c.cut_tab, 2 * (size_t)T * T);
        c.rc_pair.clear();
        q.cut2 = nullptr;
        if (p->rc_pair) {
            c.rc_pair.assign(p->rc_pair, p->rc_pair + (size_t)T * T);
            std::vector<double> h(2 * (size_t)T * T);
            for (int k = 0; k < T * T; ++k) {
                double r = p->rc_pair[k], rl = r + c.skin;
                h[k] = r * r;
                h[(size_t)T * T + k] = rl * rl;
            }
            if (!c.measure) HIP_TRY(hipStreamSynchronize(s));
            int rh = h2d(c, c.cut_tab, h.data(), h.size() * sizeof(double));
            if (rh != MD_OK) return rh;
            q.cut2 = c.cut_tab;
        }
        if (c.measure) {
            // sizes only
        } else if (p->kind == MD_POT_SPLINE) {
            off = 0;
            for (int k = 0; k < 3; ++k) {
                HIP_TRY(hipMemcpyAsync(c.tables + off, p->tab[k], sizeof(double) * c.tab_len[k],
                                       hipMemcpyHostToDevice, s));
                off += c.tab_len[k];
            }
            launch_pair_tables(c, s);
        } else {
            for (int k = 0; k < 3; ++k)
                HIP_TRY(hipMemcpyAsync(c.theta + (size_t)k * c.n_theta, p->tab[k],
                                       sizeof(double) * c.n_theta, hipMemcpyHostToDevice, s));
            launch_bspline_tables(c, c.theta, s);
        }
        if (!c.measure) HIP_TRY(hipStreamSynchronize(s));
    }
    graph_reset(c);
    c.density_valid = c.forces_valid = false;
    return MD_OK;
}

// The neighbour list at capacity mn; the previous list is released only once
// the new one exists, so a failure leaves the context as it was.
int alloc_list(Ctx &c, int mn)
{
    // rows are stored in groups of four; a multiple of eight also keeps the
    // split of a row's entries over the lanes that share it (entry index
    // modulo the lane count, at most eight) independent of the capacity, so
    // results do not depend on it
    mn = (mn + 7) / 8 * 8;
    if (mn > kMaxCapacity) return MD_ERR_ARG;
    int *idx = nullptr;
    ALLOC(idx, (size_t)mn * c.N);
    int rz = zero(c, idx, sizeof(int) * (size_t)mn * c.N);
    if (rz != MD_OK) return rz;
    ctx_free(c, c.nl.idx);
    c.nl.idx = idx;
    c.nl.mn = mn;
    return MD_OK;
}

// Per-type kick factor, friction addend and m / (2 kappa) (several species),
// uploaded after the device is idle (kernels of any stream may read them).
int upload_type_coef(Ctx &c)
{
    if (c.ntypes < 2) return MD_OK;
    const double kb = 8.617333262e-5;
    const double kappa = 1.602176634e-19 / 1.66053906660e-27 * 1e-10;
    std::vector<double> h(4 * (size_t)c.ntypes, 0.0);
    for (int t = 0; t < c.ntypes; ++t) {
        double m = c.type_mass[t];
        h[4 * t + kTcKick] = 0.5 * c.dt * kappa / m;
        h[4 * t + kTcFric] =
            c.thermo.on ? (1.0 - c.thermo.e) * (3.0 * kb * c.thermo_te * kappa / m) : 0.0;
        h[4 * t + kTcHalfM] = 0.5 * m / kappa;
    }
    if (c.measure) return MD_OK;
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(c.d_tcoef, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
    return MD_OK;
}

// Switch between the tiled and the per-atom passes (as MD_OPT_TILED does).
void set_tiled(Ctx &c, bool v)
{
    if (v == c.tiled) return;
    c.tiled = v;
    graph_reset(c);
    c.list_valid = c.density_valid = c.forces_valid = false;
}

int tile_grid(const Ctx &c, const int s[3], std::vector<int> &bt);
int64_t grid_cells(const Ctx &c, const std::vector<int> &bt, std::vector<int> &cell_off);
void tile_table(const Ctx &c, std::vector<int> &ht);

// Switch to candidate tile shape k: the tile grid, the cell numbering and the
// device tables that describe them (their buffers were sized for every
// candidate at creation); lists and graphs are built again.  The lists do not
// change; results change in rounding only (the rows of the atoms of a tile
// beyond one per thread are summed by several lanes).
int apply_tile_shape(Ctx &c, int k)
{
    if (k < 0 || 3 * (size_t)k >= c.tile_shapes.size()) return MD_ERR_ARG;
    if (k == c.tile_shape) return MD_OK;
    HIP_TRY(hipDeviceSynchronize());
    std::vector<int> bt, co, ht;
    const int nt = tile_grid(c, &c.tile_shapes[3 * (size_t)k], bt);
    const int64_t cells = grid_cells(c, bt, co);
    if (cells < 0 || cells > c.cap_cells || nt > c.cap_tiles) return MD_ERR_ARG;
    c.box_tile = bt;
    c.ntiles = nt;
    c.box_cell_off = co;
    c.bd.n_cells = (int)cells;
    tile_table(c, ht);
    int rc;
    if ((rc = h2d(c, c.d_tiles, ht.data(), ht.size() * sizeof(int))) != MD_OK ||
        (rc = h2d(c, c.d_boxi + c.B, co.data(), sizeof(int) * (size_t)c.B)) != MD_OK)
        return rc;
    c.tile_shape = k;
    if (c.tile_feasible) tiled_prepare(c);
    graph_reset(c);
    c.list_valid = c.density_valid = c.forces_valid = false;
    batched_invalidate(c);
    return MD_OK;
}

// The device status words after the work enqueued on s (waits for it).
int read_flags(Ctx &c, hipStream_t s, unsigned *w)
{
    HIP_TRY(hipMemcpyAsync(w, c.dev.flags, kFlagWords * sizeof(unsigned), hipMemcpyDeviceToHost,
                           s));
    HIP_TRY(hipStreamSynchronize(s));
    return MD_OK;
}

// A list build ran out of capacity (status words w): lift the halt and raise
// the capacity -- the row capacity to the longest row found plus an eighth,
// or, when a tile's halo did not fit LDS, the per-atom passes for the rest of
// the context's life.  The list must then be built again.  MD_FLAG_NLIST_OVERFLOW
// stays set for md_status; MD_FLAG_TILE_OVERFLOW is cleared once handled.
int regrow(Ctx &c, const unsigned *w, hipStream_t s)
{
    launch_fill_u32(c.dev.flags + kHaltWord, 2, 0u, s);
    c.list_valid = c.density_valid = c.forces_valid = false;
    batched_invalidate(c);
    if (w[0] & MD_FLAG_TILE_OVERFLOW) {
        launch_clear_bits(c, MD_FLAG_TILE_OVERFLOW, s);
        set_tiled(c, false);
        c.tile_feasible = false;
    }
    const int need = (int)w[kMaxRowWord];
    if (need > c.nl.mn) {
        if (need > kMaxCapacity) return MD_ERR_NLIST_OVERFLOW;
        int want = std::min(kMaxCapacity, need + need / 8 + 8);
        HIP_TRY(hipStreamSynchronize(s));
        if (alloc_list(c, want) != MD_OK) return MD_ERR_NLIST_OVERFLOW;
        graph_reset(c);
        if (c.B > 1) {
            int rc = batched_prepare(c);
            if (rc != MD_OK) return rc;
        }
    }
    return MD_OK;
}

// A list build from the host: waits for it and, when a row or a tile ran out
// of capacity, raises the capacity and builds again, so that no pass ever
// runs on truncated rows.
int build_checked(Ctx &c, hipStream_t s)
{
    for (int attempt = 0; attempt < 4; ++attempt) {
        launch_build(c, false, s);
        unsigned w[kFlagWords];
        int rc = read_flags(c, s, w);
        if (rc != MD_OK) return rc;
        if (!w[kHaltWord]) {
            c.list_valid = true;
            c.density_valid = c.forces_valid = false;
            batched_invalidate(c);
            return MD_OK;
        }
        if ((rc = regrow(c, w, s)) != MD_OK) return rc;
    }
    return MD_ERR_NLIST_OVERFLOW;
}

// Bring the list, density and forces up to date on stream s.
int ensure_list(Ctx &c, hipStream_t s)
{
    return c.list_valid ? MD_OK : build_checked(c, s);
}

int ensure_density(Ctx &c, hipStream_t s)
{
    int rc = ensure_list(c, s);
    if (rc != MD_OK) return rc;
    if (!c.density_valid) {
        launch_density(c, s);
        c.density_valid = true;
    }
    return MD_OK;
}

#define ENSURE(call)                    \
    do {                                \
        int rc_ = (call);               \
        if (rc_ != MD_OK) return rc_;   \
    } while (0)

// One velocity-Verlet step on stream s.  kick_drift: the step starts with
// the half kick and drift (false when the previous force pass performed
// them); force_mode: 1 the force pass ends with the half kick, 2 it also
// performs the next step's half kick and drift into the second position
// buffer.  The device's rebuild request is counted and cleared right after
// the gated build, before a fused force pass can raise the next one.
// fp_only: the density pass stores F' alone (in tiled contexts; the
// densities and embedding energies of a step inside a sequence are never
// read).  With the barostat (eq. 5) the coordinates and boxes are scaled
// after the drift, and the force pass computes energies and the virial for
// the next pressure (eq. 6) and scale factor.
void launch_step(Ctx &c, hipStream_t s, bool kick_drift, int force_mode, bool fp_only = false)
{
    if (c.baro_on) {
        launch_kick_drift(c, s);
        launch_baro_box_scale(c, s);
        launch_build(c, true, s);
        launch_step_end(c, s);
        launch_density(c, s);
        launch_force(c, true, 1, s);
        launch_pressure_eval(c, s);
        launch_baro_mu(c, s);
        return;
    }
    if (kick_drift) launch_kick_drift(c, s);
    launch_build(c, true, s);
    launch_step_end(c, s);
    launch_density(c, s, fp_only);
    launch_force(c, false, force_mode, s);
}

// One captured graph of nsteps steps.  In tiled contexts without the
// barostat the force pass of a step also performs the next step's half kick
// and drift (the same operations, in the same order, as the separate
// kick-drift kernel) and the steps alternate between the two position
// buffers; the last one or two steps are not fused, so that the state ends
// where it began: in the primary buffer, with velocities at the full step.
int capture_steps(Ctx &c, int nsteps, Ctx::StepGraph &out)
{
    if (out.exec) (void)hipGraphExecDestroy(out.exec);
    out = Ctx::StepGraph{};
    hipGraph_t g = nullptr;
    const State prim = c.st;
    State alt = prim;
    std::swap(alt.x, alt.xo);
    std::swap(alt.y, alt.yo);
    std::swap(alt.z, alt.zo);
    int fused = (c.tiled && !c.baro_on) ? (nsteps % 2 ? nsteps - 1 : nsteps - 2) : 0;
    HIP_TRY(hipStreamBeginCapture(c.cap_stream, hipStreamCaptureModeRelaxed));
    for (int k = 0; k < nsteps; ++k) {
        c.st = (k < fused && k % 2) ? alt : prim;
        // the densities and embedding energies of all but the last step are
        // never read: their density passes store F' alone
        launch_step(c, c.cap_stream, k == 0 || k > fused, k < fused ? 2 : 1, k < nsteps - 1);
    }
    c.st = prim;
    HIP_TRY(hipStreamEndCapture(c.cap_stream, &g));
    hipError_t e = hipGraphInstantiate(&out.exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        out.exec = nullptr;
        return MD_ERR_DEVICE;
    }
    out.len = nsteps;
    out.fused = fused;
    return MD_OK;
}

// nsteps steps: graphs of graph_steps steps, then one graph of the
// remainder (kept for the next call with the same remainder), or with graphs
// off single steps.  *graphs: the full graphs launched; *tail: whether the
// remainder graph was.
int run_steps(Ctx &c, int nsteps, hipStream_t s, int *graphs, bool *tail)
{
    int done = 0;
    *graphs = 0;
    *tail = false;
    if (c.use_graph) {
        if (nsteps >= c.graph_steps && c.graph.len != c.graph_steps)
            ENSURE(capture_steps(c, c.graph_steps, c.graph));
        for (; nsteps - done >= c.graph_steps; done += c.graph_steps, ++*graphs)
            HIP_TRY(hipGraphLaunch(c.graph.exec, s));
        const int rest = nsteps - done;
        if (rest >= 2) {
            if (c.tail_graph.len != rest) ENSURE(capture_steps(c, rest, c.tail_graph));
            HIP_TRY(hipGraphLaunch(c.tail_graph.exec, s));
            *tail = true;
            done = nsteps;
        }
    }
    for (; done < nsteps; ++done) launch_step(c, s, true, 1);
    return MD_OK;
}

// Steps of one box, or of boxes through the merged-box kernels.  A list
// build inside the steps that runs out of capacity halts the step sequence
// on the device (every later kernel of it does nothing); at the end the host
// reads the status, and if the steps halted it raises the capacity, builds
// the list again, completes the halted step (density, force and second half
// kick, and with the barostat the next pressure and scale factor) and takes
// the remaining steps.  The trajectory is the one a context with enough
// capacity from the start would have taken.
int steps_merged(Ctx &c, int nsteps, hipStream_t s)
{
    ENSURE(ensure_list(c, s));
    if (c.baro_on && !c.baro_mu_valid) {
        // pressure of the current state: the first step's scale factor
        ENSURE(ensure_density(c, s));
        launch_force(c, true, 0, s);
        launch_pressure_eval(c, s);
        launch_baro_mu(c, s);
        c.forces_valid = c.baro_mu_valid = true;
    } else if (!c.forces_valid) {
        ENSURE(ensure_density(c, s));
        launch_force(c, false, 0, s);
        c.forces_valid = true;
    }
    int left = nsteps;
    for (int round = 0; left > 0; ++round) {
        if (round > 8) return MD_ERR_NLIST_OVERFLOW;
        launch_step_mark(c, s);
        int graphs = 0;
        bool tail = false;
        ENSURE(run_steps(c, left, s, &graphs, &tail));
        unsigned w[kFlagWords];
        ENSURE(read_flags(c, s, w));
        if (!w[kHaltWord]) break;
        // step k of this run halted at its list build (after its drift)
        const uint64_t now = ((uint64_t)w[5] << 32) | w[3];
        const uint64_t mark = ((uint64_t)w[kMarkWord + 1] << 32) | w[kMarkWord];
        const int k = (int)(now - mark);
        if (k >= left) return MD_ERR_STATE;
        // inside a graph, odd fused steps run on the other position buffer
        int j = -1, fused = 0;
        if (k < graphs * c.graph.len) {
            j = k % c.graph.len;
            fused = c.graph.fused;
        } else if (tail && k < graphs * c.graph.len + c.tail_graph.len) {
            j = k - graphs * c.graph.len;
            fused = c.tail_graph.fused;
        }
        if (j >= 0 && j < fused && j % 2 == 1) {
            const size_t nb = sizeof(double) * (size_t)c.N;
            HIP_TRY(hipMemcpyAsync(c.st.x, c.st.xo, nb, hipMemcpyDeviceToDevice, s));
            HIP_TRY(hipMemcpyAsync(c.st.y, c.st.yo, nb, hipMemcpyDeviceToDevice, s));
            HIP_TRY(hipMemcpyAsync(c.st.z, c.st.zo, nb, hipMemcpyDeviceToDevice, s));
        }
        launch_fill_u32(c.dev.flags + 1, 1, 0u, s);  // its rebuild request
        ENSURE(regrow(c, w, s));
        ENSURE(build_checked(c, s));
        launch_density(c, s);
        if (c.baro_on) {
            launch_force(c, true, 1, s);
            launch_pressure_eval(c, s);
            launch_baro_mu(c, s);
        } else {
            launch_force(c, false, 1, s);
        }
        launch_step_end(c, s);
        left -= k + 1;
    }
    c.list_valid = c.density_valid = c.forces_valid = true;
    batched_invalidate(c);
    return MD_OK;
}

// Steps of several boxes by the persistent stepper.  The start state is kept
// in the merged-box sort scratch (which the stepper does not use); when a
// box's list outgrew the capacity, the state is restored and the call is
// taken again with a capacity for the longest row found.
int steps_batched(Ctx &c, int nsteps, hipStream_t s)
{
    const size_t nb = sizeof(double) * (size_t)c.N;
    double *keep[6] = {c.bd.sx, c.bd.sy, c.bd.sz, c.bd.svx, c.bd.svy, c.bd.svz};
    double *live[6] = {c.st.x, c.st.y, c.st.z, c.st.vx, c.st.vy, c.st.vz};
    for (int k = 0; k < 6; ++k)
        HIP_TRY(hipMemcpyAsync(keep[k], live[k], nb, hipMemcpyDeviceToDevice, s));
    for (int attempt = 0;; ++attempt) {
        ENSURE(launch_batched_steps(c, nsteps, s));
        unsigned w[kFlagWords];
        ENSURE(read_flags(c, s, w));
        if (!w[kMaxRowWord]) break;
        if (attempt == 3) return MD_ERR_NLIST_OVERFLOW;
        for (int k = 0; k < 6; ++k)
            HIP_TRY(hipMemcpyAsync(live[k], keep[k], nb, hipMemcpyDeviceToDevice, s));
        ENSURE(regrow(c, w, s));
    }
    c.host_steps += nsteps;
    // forces in the state arrays match the new positions; the merged-box
    // list and densities do not
    c.list_valid = c.density_valid = false;
    c.forces_valid = true;
    return MD_OK;
}

// Tile grid of every box for one tile shape s (cells per tile along x, y,
// z): per box tx ty tz, tiles per axis, cells per tile and halo mode, in bt;
// returns the number of tiles.  Boxes with at least max(s) + 2 cells per
// axis are cut into tiles (halo mode A), a smaller box is one tile (mode B),
// and without tiling every box is one tile numbered row-major.
int tile_grid(const Ctx &c, const int s[3], std::vector<int> &bt)
{
    const int tmax = std::max(s[0], std::max(s[1], s[2]));
    bt.assign(8 * (size_t)c.B, 0);
    int ntiles = 0;
    for (int b = 0; b < c.B; ++b) {
        int nc = c.box_nc[b];
        int *t = &bt[8 * b];
        if (c.tile_feasible && nc >= tmax + 2) {
            for (int d = 0; d < 3; ++d) {
                t[d] = s[d];
                t[3 + d] = (nc + s[d] - 1) / s[d];
            }
            t[7] = kTileA;
        } else {
            t[0] = t[1] = t[2] = nc;
            t[3] = t[4] = t[5] = 1;
            t[7] = c.tile_feasible ? kTileB : kTileGlobal;
        }
        t[6] = t[0] * t[1] * t[2];
        ntiles += t[3] * t[4] * t[5];
    }
    return ntiles;
}

// Cells of every box (tiles times cells per tile, so a box's cells are
// numbered tile by tile) for the tile grid bt: the first cell of each box in
// cell_off[B + 1]; returns the total, or -1 beyond 2^30.
int64_t grid_cells(const Ctx &c, const std::vector<int> &bt, std::vector<int> &cell_off)
{
    cell_off.assign(c.B + 1, 0);
    int64_t cells = 0;
    for (int b = 0; b < c.B; ++b) {
        const int *t = &bt[8 * b];
        cell_off[b] = (int)cells;
        cells += (int64_t)t[3] * t[4] * t[5] * t[6];
        if (cells >= (int64_t)1 << 30) return -1;
    }
    cell_off[c.B] = (int)cells;
    return cells;
}

// The device tile table: tile(8B) | tile_off(B+1) | tile_box(cap_tiles) |
// order(ntiles).  order is the sweep of the density and force passes: within
// each die's share of the tiles (workgroups go round robin over the dies, and
// the share is cut as in xcd_tile), the full tiles first, then the thinner
// tiles at the upper faces of a box (when its cells per axis are not a
// multiple of the tile's), so that the passes end on short tiles.
void tile_table(const Ctx &c, std::vector<int> &ht)
{
    const int B = c.B;
    ht.assign(8 * (size_t)B + B + 1 + c.ntiles, 0);
    std::copy(c.box_tile.begin(), c.box_tile.end(), ht.begin());
    int g = 0;
    for (int b = 0; b < B; ++b) {
        ht[8 * B + b] = g;
        const int *t = &c.box_tile[8 * b];
        for (int k = 0; k < t[3] * t[4] * t[5]; ++k) ht[9 * B + 1 + g + k] = b;
        g += t[3] * t[4] * t[5];
    }
    ht[9 * B] = g;
    ht.resize(9 * (size_t)B + 1 + c.cap_tiles + c.ntiles, 0);
    int *order = &ht[9 * (size_t)B + 1 + c.cap_tiles];
    std::vector<int> cells(c.ntiles, 0);
    g = 0;
    for (int b = 0; b < B; ++b) {
        const int *t = &c.box_tile[8 * b];
        const int nc = c.box_nc[b], gx = t[3], gy = t[4], gz = t[5];
        for (int k = 0; k < gx * gy * gz; ++k) {
            int kx = k % gx, ky = (k / gx) % gy, kz = k / (gx * gy);
            cells[g + k] = t[7] == kTileA ? std::min(t[0], nc - kx * t[0]) *
                                                std::min(t[1], nc - ky * t[1]) *
                                                std::min(t[2], nc - kz * t[2])
                                          : nc * nc * nc;
        }
        g += gx * gy * gz;
    }
    const int q = c.ntiles / 8, r = c.ntiles % 8;
    for (int x = 0; x < 8; ++x) {
        const int lo = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q, n = q + (x < r);
        for (int k = 0; k < n; ++k) order[lo + k] = lo + k;
        std::stable_sort(order + lo, order + lo + n,
                         [&](int u, int v) { return cells[u] > cells[v]; });
    }
}

// Tile geometry.  Tiles of tx x ty x tz cells are chosen so that a tile
// holds about one 1024-thread workgroup of atoms and its halo (the tile grown
// by one cell) fits the LDS of one workgroup with a 30% margin.  Boxes with at
// least max(t)+2 cells per axis are cut into such tiles (halo mode A); a
// smaller box is one tile holding the whole box (mode B).  Without tiling,
// every box is one tile numbered row-major and the per-atom kernels run.
int plan_tiles(Ctx &c, double per_cell, bool allow)
{
    int max_lds = 0;
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c.device) !=
        hipSuccess)
        return MD_ERR_DEVICE;
    size_t fixed = 8192;  // halo table and scan scratch (static LDS)
    c.hmax = max_lds > (int)fixed ? (int)((max_lds - fixed) / 32) : 0;
    c.tile_lds = (size_t)c.hmax * 32;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c.device) != hipSuccess)
        return MD_ERR_DEVICE;
    // the tile of at most max_atoms atoms (on average) and at most tlim cells
    // per axis with the most atoms whose halo fits in LDS
    auto pick = [&](double max_atoms, int tlim, int out[3], double margin = 1.3) {
        double best_atoms = 0.0;
        out[0] = out[1] = out[2] = 0;
        for (int tz = 1; tz <= tlim; ++tz)
            for (int ty = tz; ty <= tlim; ++ty)
                for (int tx = ty; tx <= tlim; ++tx) {
                    double atoms = tx * ty * tz * per_cell;
                    int halo_cells = (tx + 2) * (ty + 2) * (tz + 2);
                    double halo = halo_cells * per_cell;
                    if (atoms > max_atoms || margin * halo > c.hmax || halo_cells > kHaloCells)
                        continue;
                    if (atoms > best_atoms) {
                        best_atoms = atoms;
                        out[0] = tx;
                        out[1] = ty;
                        out[2] = tz;
                    }
                }
    };
    // tiles of all boxes for a tile shape (a box too small for it is one tile)
    auto count = [&](const int t[3]) {
        int tm = std::max(t[0], std::max(t[1], t[2]));
        long long n = 0;
        for (int b = 0; b < c.B; ++b) {
            int nc = c.box_nc[b];
            n += nc >= tm + 2 ? (long long)((nc + t[0] - 1) / t[0]) * ((nc + t[1] - 1) / t[1]) *
                                    ((nc + t[2] - 1) / t[2])
                              : 1;
        }
        return n;
    };
    int best[3];
    pick(1100.0, 6, best);
    // a system of fewer than two rounds of tiles (one per compute unit) runs
    // half-size tiles, each atom's row shared by two lanes, when that takes
    // fewer rounds of half the length: more compute units work on half rows.
    // Half tiles are no longer along any axis, so no box loses its tiling;
    // larger systems keep the full tiles (their halo overhead would grow).
    c.tile_lanes = 1;
    if (best[0] > 0 && count(best) < 2LL * cus) {
        int half[3];
        pick(550.0, best[0], half);
        long long nf = count(best), nh = half[0] > 0 ? count(half) : nf;
        if ((nh + cus - 1) / cus < 2 * ((nf + cus - 1) / cus)) {
            if (half[0] > 0) {
                best[0] = half[0];
                best[1] = half[1];
                best[2] = half[2];
            }
            c.tile_lanes = 2;
        }
    }
    bool feasible = allow && best[0] > 0;
    int tmax = std::max(best[0], std::max(best[1], best[2]));
    for (int b = 0; b < c.B && feasible; ++b) {
        int nc = c.box_nc[b];
        if (nc >= tmax + 2) continue;
        double nb = (double)(c.box_off[b + 1] - c.box_off[b]);
        if (1.3 * nb > c.hmax || nc * nc * nc > kHaloCells) feasible = false;
    }
    c.tile_feasible = feasible;
    c.tiled = feasible;
    // other shapes for md_autotune (large systems with full tiles): a larger
    // tile with a thinner LDS margin and a smaller one, each kept only when
    // no box changes its halo mode (the tile overflow check guards the
    // thinner margin as it guards every tile)
    c.tile_shapes.assign(best, best + 3);
    if (feasible && c.tile_lanes == 1) {
        int alt[2][3];
        pick(1300.0, 6, alt[0], 1.12);
        pick(900.0, 6, alt[1]);
        for (const auto &s : alt) {
            if (s[0] <= 0) continue;
            bool same = false;
            for (size_t k = 0; k < c.tile_shapes.size(); k += 3)
                same = same || (c.tile_shapes[k] == s[0] && c.tile_shapes[k + 1] == s[1] &&
                                c.tile_shapes[k + 2] == s[2]);
            int tm = std::max(s[0], std::max(s[1], s[2]));
            for (int b = 0; b < c.B && !same; ++b)
                same = (c.box_nc[b] >= tm + 2) != (c.box_nc[b] >= tmax + 2);
            if (!same) c.tile_shapes.insert(c.tile_shapes.end(), s, s + 3);
        }
    }
    c.tile_shape = 0;
    c.ntiles = tile_grid(c, best, c.box_tile);
    return MD_OK;
}

}  // namespace

extern "C" {

const char *md_strerror(int code)
{
    switch (code) {
    case MD_OK: return "ok";
    case MD_ERR_ARG: return "invalid argument";
    case MD_ERR_BOX: return "box edge must exceed twice the force cutoff";
    case MD_ERR_NLIST_OVERFLOW: return "neighbour list capacity exceeded";
    case MD_ERR_TABLE_RANGE: return "table lookup outside the tabulated range";
    case MD_ERR_NONFINITE: return "non-finite coordinate";
    case MD_ERR_DEVICE: return "HIP runtime error";
    case MD_ERR_STATE: return "call out of order";
    case MD_ERR_NOMEM: return "device allocation failed";
    case MD_ERR_SCRATCH: return "system too large for the static device array of md_forces_static";
    }
    return "unknown error";
}

}  // extern "C"

namespace {

// Context set-up.  mode kMeasure: count the workspace bytes only (nothing is
// allocated, copied or launched); kOneShot: the context lives in `workspace`
// for one evaluation on `stream` (no capture stream, no graph).
int create_impl(const md_system *sys, const md_potential *pot, md_ctx **out, void *workspace,
                size_t workspace_bytes, int mode = kNormal, hipStream_t stream = nullptr)
{
    if (!out) return MD_ERR_ARG;
    *out = nullptr;
    if (!sys || sys->n_boxes < 1 || !sys->box_offset || !sys->box_len) return MD_ERR_ARG;
    if (!(sys->mass > 0.0) || !(sys->dt > 0.0) || !(sys->skin >= 0.0)) return MD_ERR_ARG;
    int prc = check_potential(pot);
    if (prc != MD_OK) return prc;
    int B = sys->n_boxes;
    if (sys->box_offset[0] != 0) return MD_ERR_ARG;
    for (int b = 0; b < B; ++b) {
        if (sys->box_offset[b + 1] - sys->box_offset[b] < 2) return MD_ERR_ARG;
        if (!(sys->box_len[b] > 0.0)) return MD_ERR_ARG;
        if (!(0.5 * sys->box_len[b] - 1e-9 > pot->rc)) return MD_ERR_BOX;
    }
    int64_t N = sys->box_offset[B];
    if (N >= (int64_t)1 << 27) return MD_ERR_ARG;  // gathers use 32-bit byte offsets

    md_ctx *h = new (std::nothrow) md_ctx();
    if (!h) return MD_ERR_NOMEM;
    Ctx &c = h->c;
    auto fail = [&](int code) {
        md_destroy(h);
        return code;
    };
    if (workspace) {
        c.arena = static_cast<char *>(workspace);
        c.arena_size = workspace_bytes;
    }
    c.measure = mode == kMeasure;
    c.oneshot = mode == kOneShot;
    if (hipGetDevice(&c.device) != hipSuccess) return fail(MD_ERR_DEVICE);
    c.N = N;
    c.B = B;
    c.mass = sys->mass;
    c.dt = sys->dt;
    c.skin = sys->skin;
    c.kind_user = pot->kind;
    c.batched = false;
    c.box_off.assign(sys->box_offset, sys->box_offset + B + 1);
    c.box_len.assign(sys->box_len, sys->box_len + B);
    c.box_rlist.resize(B);
    c.box_nc.resize(B);
    c.box_cell_off.resize(B + 1);
    double mn_est = 0.0, per_cell = 0.0;
    for (int b = 0; b < B; ++b) {
        double L = c.box_len[b];
        double rl = list_radius(pot->rc, sys->skin, L);
        c.box_rlist[b] = rl;
        int nc = cells_per_dim(L, rl);
        c.box_nc[b] = nc;
        double nb = (double)(c.box_off[b + 1] - c.box_off[b]);
        per_cell = std::max(per_cell, nb / ((double)nc * nc * nc));
        double expect = nb / (L * L * L) * 4.0 / 3.0 * M_PI * rl * rl * rl;
        double est = std::min(nb - 1.0, std::ceil(1.4 * expect + 16.0));
        mn_est = std::max(mn_est, est);
    }
    int rc_t = plan_tiles(c, per_cell, pot->kind != MD_POT_BSPLINE);
    if (rc_t != MD_OK) return fail(rc_t);
    const int64_t cells = grid_cells(c, c.box_tile, c.box_cell_off);
    if (cells < 0) return fail(MD_ERR_ARG);
    c.bd.n_cells = (int)cells;
    // buffers for the largest of the candidate tile shapes
    c.cap_cells = (int)cells;
    c.cap_tiles = c.ntiles;
    for (size_t k = 3; k < c.tile_shapes.size(); k += 3) {
        std::vector<int> bt, co;
        const int nt = tile_grid(c, &c.tile_shapes[k], bt);
        const int64_t nc = grid_cells(c, bt, co);
        if (nc < 0) return fail(MD_ERR_ARG);
        c.cap_cells = std::max(c.cap_cells, (int)nc);
        c.cap_tiles = std::max(c.cap_tiles, nt);
    }
    int mn = sys->max_neighbors > 0 ? sys->max_neighbors : ((int)mn_est + 7) / 8 * 8;
    if (mn < 1) mn = 1;
    if (mn > kMaxCapacity) return fail(MD_ERR_ARG);

    if (mode == kNormal &&
        hipStreamCreateWithFlags(&c.cap_stream, hipStreamNonBlocking) != hipSuccess)
        return fail(MD_ERR_DEVICE);
    hipStream_t s = mode == kNormal ? c.cap_stream : stream;

    // per-box geometry
    int rc;
    if ((rc = dev_alloc(c, &c.d_boxd, 4 * (size_t)B)) != MD_OK) return fail(rc);
    if ((rc = dev_alloc(c, &c.d_boxi, 3 * (size_t)B + 1 + N)) != MD_OK) return fail(rc);
    {
        std::vector<double> hd(4 * (size_t)B);
        std::vector<int> hi(3 * (size_t)B + 1 + N);
        for (int b = 0; b < B; ++b) {
            double L = c.box_len[b], rl = c.box_rlist[b], half = 0.5 * (rl - pot->rc);
            hd[b] = L;
            hd[B + b] = 1.0 / L;
            hd[2 * B + b] = rl * rl;
            hd[3 * B + b] = half * half;
            hi[b] = c.box_nc[b];
            hi[B + b] = c.box_cell_off[b];
        }
        for (int b = 0; b <= B; ++b) hi[2 * B + b] = (int)c.box_off[b];
        for (int b = 0; b < B; ++b)
            for (int64_t i = c.box_off[b]; i < c.box_off[b + 1]; ++i) hi[3 * B + 1 + i] = b;
        if ((rc = h2d(c, c.d_boxd, hd.data(), hd.size() * sizeof(double))) != MD_OK ||
            (rc = h2d(c, c.d_boxi, hi.data(), hi.size() * sizeof(int))) != MD_OK)
            return fail(rc);
        c.bx.L = c.d_boxd;
        c.bx.invL = c.d_boxd + B;
        c.bx.rl2 = c.d_boxd + 2 * B;
        c.bx.thr2 = c.d_boxd + 3 * B;
        c.bx.nc = c.d_boxi;
        c.bx.cell_off = c.d_boxi + B;
        c.bx.atom_off = c.d_boxi + 2 * B;
        c.bx.box_of = c.d_boxi + 3 * B + 1;
    }

    // tile descriptors
    {
        std::vector<int> ht;
        tile_table(c, ht);
        if ((rc = dev_alloc(c, &c.d_tiles, 9 * (size_t)B + 1 + 2 * (size_t)c.cap_tiles)) != MD_OK)
            return fail(rc);
        if ((rc = h2d(c, c.d_tiles, ht.data(), ht.size() * sizeof(int))) != MD_OK)
            return fail(rc);
        c.bx.tile = c.d_tiles;
        c.bx.tile_off = c.d_tiles + 8 * B;
        c.bx.tile_box = c.d_tiles + 9 * B + 1;
        c.bx.tile_order = c.d_tiles + 9 * B + 1 + c.cap_tiles;
        if (c.tile_feasible) {
            tiled_prepare(c);
            if ((rc = dev_alloc(c, &c.nl.tsrc, (size_t)c.cap_tiles * c.hmax)) != MD_OK)
                return fail(rc);
            if ((rc = dev_alloc(c, &c.nl.ttotal, (size_t)c.cap_tiles)) != MD_OK) return fail(rc);
        }
    }

    // atom state and build scratch
    double **dbl[] = {&c.st.x, &c.st.y, &c.st.z, &c.st.xo, &c.st.yo, &c.st.zo, &c.st.vx,
                      &c.st.vy, &c.st.vz, &c.st.fx,
                      &c.st.fy, &c.st.fz, &c.st.xr, &c.st.yr, &c.st.zr, &c.st.rho, &c.st.Fp,
                      &c.st.Femb, &c.st.eat, &c.st.wat, &c.bd.sx, &c.bd.sy, &c.bd.sz, &c.bd.svx,
                      &c.bd.svy, &c.bd.svz};
    for (double **p : dbl)
        if ((rc = dev_alloc(c, p, (size_t)N)) != MD_OK) return fail(rc);
    if ((rc = dev_alloc(c, &c.st.pk, 4 * (size_t)N)) != MD_OK) return fail(rc);
    int **ints[] = {&c.st.id, &c.bd.sid, &c.bd.cell_of, &c.bd.slot, &c.bd.tmp, &c.bd.perm,
                    &c.nl.count, &c.nl.total};
    for (int **p : ints)
        if ((rc = dev_alloc(c, p, (size_t)N)) != MD_OK) return fail(rc);
    const size_t cap = (size_t)c.cap_cells;
    if ((rc = dev_alloc(c, &c.bd.cell_count, cap)) != MD_OK) return fail(rc);
    if ((rc = dev_alloc(c, &c.bd.cell_start, cap + 1)) != MD_OK) return fail(rc);
    if ((rc = dev_alloc(c, &c.bd.bsum, cap / 4096 + 2)) != MD_OK) return fail(rc);
    if ((rc = zero(c, c.bd.cell_count, sizeof(int) * cap)) != MD_OK) return fail(rc);
    if ((rc = alloc_list(c, mn)) != MD_OK) return fail(rc);
    if ((rc = dev_alloc(c, &c.dev.flags, kFlagWords)) != MD_OK) return fail(rc);
    {
        // barostat state per box: mu = 1, strain = 1, list radius, then results
        std::vector<double> hb(7 * (size_t)B, 0.0);
        for (int b = 0; b < B; ++b) {
            hb[b] = 1.0;
            hb[B + b] = 1.0;
            hb[2 * B + b] = c.box_rlist[b];
        }
        if ((rc = dev_alloc(c, &c.d_baro, hb.size())) != MD_OK) return fail(rc);
        if ((rc = h2d(c, c.d_baro, hb.data(), hb.size() * sizeof(double))) != MD_OK)
            return fail(rc);
    }
    if ((rc = zero(c, c.dev.flags, kFlagWords * sizeof(unsigned))) != MD_OK ||
        (rc = zero(c, c.nl.count, sizeof(int) * N)) != MD_OK ||
        (rc = zero(c, c.nl.total, sizeof(int) * N)) != MD_OK)
        return fail(rc);

    // chunks of the fixed-order per-box sums
    {
        std::vector<int> cs, ce, bc(B + 1);
        for (int b = 0; b < B; ++b) {
            bc[b] = (int)cs.size();
            for (int64_t a = c.box_off[b]; a < c.box_off[b + 1]; a += kChunk) {
                cs.push_back((int)a);
                ce.push_back((int)std::min<int64_t>(a + kChunk, c.box_off[b + 1]));
            }
        }
        bc[B] = (int)cs.size();
        c.n_chunks = (int)cs.size();
        std::vector<int> all;
        all.insert(all.end(), cs.begin(), cs.end());
        all.insert(all.end(), ce.begin(), ce.end());
        all.insert(all.end(), bc.begin(), bc.end());
        if ((rc = dev_alloc(c, &c.d_chunks, all.size())) != MD_OK) return fail(rc);
        if ((rc = dev_alloc(c, &c.d_partial, (size_t)c.n_chunks)) != MD_OK) return fail(rc);
        if ((rc = h2d(c, c.d_chunks, all.data(), all.size() * sizeof(int))) != MD_OK)
            return fail(rc);
    }

    // atom states: flags in slot and original order (all free until md_set_frozen)
    if ((rc = dev_alloc(c, &c.d_frozen, (size_t)N)) != MD_OK) return fail(rc);
    if ((rc = dev_alloc(c, &c.d_frozen0, (size_t)N)) != MD_OK) return fail(rc);
    if ((rc = zero(c, c.d_frozen, (size_t)N)) != MD_OK ||
        (rc = zero(c, c.d_frozen0, (size_t)N)) != MD_OK)
        return fail(rc);
    c.ntypes = std::max(1, (int)pot->n_types);
    if (c.ntypes > 1) {
        if ((rc = dev_alloc(c, &c.d_type0, (size_t)N)) != MD_OK) return fail(rc);
        if ((rc = dev_alloc(c, &c.d_type, (size_t)N)) != MD_OK) return fail(rc);
        if ((rc = dev_alloc(c, &c.d_tcoef, 4 * (size_t)c.ntypes)) != MD_OK) return fail(rc);
        if ((rc = zero(c, c.d_type0, sizeof(int) * (size_t)N)) != MD_OK ||
            (rc = zero(c, c.d_type, sizeof(int) * (size_t)N)) != MD_OK)
            return fail(rc);
        c.type_mass.assign(c.ntypes, c.mass);
        c.st.type = c.d_type;
        c.st.type0 = c.d_type0;
        c.st.tcoef = c.d_tcoef;
        if ((rc = upload_type_coef(c)) != MD_OK) return fail(rc);
    }
    if ((rc = upload_potential(c, pot, s, true)) != MD_OK) return fail(rc);
    if (c.kind_user == MD_POT_BSPLINE) {
        size_t nd = adjoint_scratch_doubles(N, c.n_theta);
        if (nd == 0) return fail(MD_ERR_ARG);
        if ((rc = dev_alloc(c, &c.adj, nd)) != MD_OK) return fail(rc);
        c.adj_len = nd;
    }
    if (c.B > 1) {
        if ((rc = batched_prepare(c)) != MD_OK) return fail(rc);
    }
    if (!c.measure && hipStreamSynchronize(s) != hipSuccess) return fail(MD_ERR_DEVICE);
    *out = h;
    return MD_OK;
}

}  // namespace

namespace mdk {

int create_context(const md_system *sys, const md_potential *pot, md_ctx **out, void *workspace,
                   size_t workspace_bytes, int mode, hipStream_t stream)
{
    return create_impl(sys, pot, out, workspace, workspace_bytes, mode, stream);
}

}  // namespace mdk

extern "C" {

int md_create(const md_system *sys, const md_potential *pot, md_ctx **out)
{
    return create_impl(sys, pot, out, nullptr, 0);
}

int md_workspace_size(const md_system *sys, const md_potential *pot, size_t *bytes)
{
    if (!bytes) return MD_ERR_ARG;
    *bytes = 0;
    md_ctx *h = nullptr;
    int rc = create_impl(sys, pot, &h, nullptr, 0, kMeasure);
    if (rc != MD_OK) return rc;
    *bytes = h->c.alloc_bytes;
    md_destroy(h);
    return MD_OK;
}

int md_create_in(const md_system *sys, const md_potential *pot, void *workspace, size_t bytes,
                 md_ctx **out)
{
    if (out) *out = nullptr;
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return MD_ERR_ARG;
    return create_impl(sys, pot, out, workspace, bytes);
}

}  // extern "C"

namespace mdk {

int ctx_alloc(Ctx &c, void **p, size_t bytes)
{
    bytes = (bytes + 255) / 256 * 256;
    if (bytes == 0) bytes = 256;
    if (c.measure) {
        // a stand-in address (never dereferenced): only the size counts
        *p = reinterpret_cast<void *>((uintptr_t)256 + c.alloc_bytes);
    } else if (c.arena) {
        if (bytes > c.arena_size - c.arena_used) return MD_ERR_NOMEM;
        *p = c.arena + c.arena_used;
        c.arena_used += bytes;
    } else {
        void *q = nullptr;
        if (hipMalloc(&q, bytes) != hipSuccess) return MD_ERR_NOMEM;
        c.allocs.push_back(q);
        *p = q;
    }
    c.alloc_bytes += bytes;
    return MD_OK;
}

void ctx_free(Ctx &c, void *p)
{
    if (!p || c.arena || c.measure) return;  // workspace blocks go back with the workspace
    auto it = std::find(c.allocs.begin(), c.allocs.end(), p);
    if (it != c.allocs.end()) {
        (void)hipFree(p);
        c.allocs.erase(it);
    }
}

}  // namespace mdk

extern "C" {

void md_destroy(md_ctx *h)
{
    if (!h) return;
    Ctx &c = h->c;
    graph_reset(c);
    if (c.cap_stream) {
        (void)hipStreamSynchronize(c.cap_stream);
        (void)hipStreamDestroy(c.cap_stream);
    }
    // a measuring context holds no device memory; a one-shot evaluation has
    // synchronised its stream already
    if (!c.measure && !c.oneshot) (void)hipDeviceSynchronize();
    for (void *p : c.allocs) (void)hipFree(p);
    batched_release(c);
    delete h;
}

int md_set_potential(md_ctx *h, const md_potential *pot, void *stream)
{
    if (!h) return MD_ERR_ARG;
    int rc = check_potential(pot);
    if (rc != MD_OK) return rc;
    Ctx &c = h->c;
    if (pot->kind != c.kind_user) return MD_ERR_ARG;
    // the list radius, the cells and the rebuild threshold follow rc
    if (pot->rc != c.pot.rc) return MD_ERR_ARG;
    const std::vector<double> before = c.rc_pair;
    rc = upload_potential(c, pot, as_stream(stream), false);
    if (rc != MD_OK) return rc;
    if (c.rc_pair != before) {
        // cutoffs per pair of types set the list radius of each pair
        c.list_valid = false;
        batched_invalidate(c);
    }
    return MD_OK;
}

int md_set_theta(md_ctx *h, const double *theta, void *stream)
{
    if (!h || !theta) return MD_ERR_ARG;
    Ctx &c = h->c;
    if (c.kind_user != MD_POT_BSPLINE) return MD_ERR_ARG;
    hipStream_t s = as_stream(stream);
    HIP_TRY(hipMemcpyAsync(c.theta, theta, sizeof(double) * 3 * c.n_theta,
                           hipMemcpyDeviceToDevice, s));
    launch_bspline_tables(c, c.theta, s);
    c.density_valid = c.forces_valid = false;
    c.baro_mu_valid = false;
    return MD_OK;
}

int md_set_state(md_ctx *h, const double *pos, const double *vel, void *stream)
{
    if (!h || !pos) return MD_ERR_ARG;
    Ctx &c = h->c;
    launch_set_state(c, pos, vel, as_stream(stream));
    c.state_set = true;
    c.list_valid = c.density_valid = c.forces_valid = false;
    c.baro_mu_valid = false;
    // the persistent stepper's per-box lists and reference positions
    // describe the previous state
    batched_invalidate(c);
    return MD_OK;
}

int md_bind(md_ctx *h, double *pos, double *vel, void *stream)
{
    if (!h) return MD_ERR_ARG;
    Ctx &c = h->c;
    if (!pos) {
        if (vel) return MD_ERR_ARG;
        c.bound_pos = c.bound_vel = nullptr;
        return MD_OK;
    }
    int rc = md_set_state(h, pos, vel, stream);
    if (rc != MD_OK) return rc;
    c.bound_pos = pos;
    c.bound_vel = vel;
    return MD_OK;
}

int md_get_state(md_ctx *h, double *pos, double *vel, void *stream)
{
    if (!h) return MD_ERR_ARG;
    if (!h->c.state_set) return MD_ERR_STATE;
    launch_get_state(h->c, pos, vel, as_stream(stream));
    return MD_OK;
}

int md_build_neighbors(md_ctx *h, void *stream)
{
    if (!h) return MD_ERR_ARG;
    Ctx &c = h->c;
    if (!c.state_set) return MD_ERR_STATE;
    return build_checked(c, as_stream(stream));
}

int md_density(md_ctx *h, double *rho_out, void *stream)
{
    if (!h) return MD_ERR_ARG;
    Ctx &c = h->c;
    if (!c.state_set) return MD_ERR_STATE;
    hipStream_t s = as_stream(stream);
    ENSURE(ensure_list(c, s));
    launch_density(c, s);
    c.density_valid = true;
    c.forces_valid = false;
    if (rho_out) launch_scatter_scalar(c, c.st.rho, rho_out, s);
    return MD_OK;
}

int md_embed(md_ctx *h, double *F_out, double *Fp_out, void *stream)
{
    if (!h) return MD_ERR_ARG;
    Ctx &c = h->c;
    if (!c.state_set) return MD_ERR_STATE;
    hipStream_t s = as_stream(stream);
    ENSURE(ensure_density(c, s));
    launch_embed(c, s);
    if (F_out) launch_scatter_scalar(c, c.st.Femb, F_out, s);
    if (Fp_out) launch_scatter_scalar(c, c.st.Fp, Fp_out, s);
    return MD_OK;
}

int md_forces(md_ctx *h, double *f_out, double *e_atom, double *e_box, void *stream)
{
    if (!h) return MD_ERR_ARG;
    Ctx &c = h->c;
    if (!c.state_set) return MD_ERR_STATE;
    hipStream_t s = as_stream(stream);
    bool energy = e_atom || e_box;
    if (!energy && c.forces_valid) {
        // forces of the current state, as the last force evaluation left them
        if (f_out) launch_scatter_vec3(c, c.st.fx, c.st.fy, c.st.fz, f_out, s);
        return MD_OK;
    }
    ENSURE(ensure_density(c, s));
    launch_force(c, energy, 0, s);
    c.forces_valid = true;
    if (f_out) launch_scatter_vec3(c, c.st.fx, c.st.fy, c.st.fz, f_out, s);
    if (e_atom) launch_scatter_scalar(c, c.st.eat, e_atom, s);
    if (e_box) launch_box_sums(c, 0, e_box, s);
    return MD_OK;
}

int md_step(md_ctx *h, int nsteps, void *stream)
{
    if (!h || nsteps < 0) return MD_ERR_ARG;
    Ctx &c = h->c;
    if (!c.state_set) return MD_ERR_STATE;
    hipStream_t s = as_stream(stream);
    int rc = (c.B > 1 && c.batched && !c.baro_on) ? steps_batched(c, nsteps, s)
                                                  : steps_merged(c, nsteps, s);
    if (rc != MD_OK) return rc;
    if (c.bound_pos) launch_get_state(c, c.bound_pos, c.bound_vel, s);
    // other conditions the kernels found: reported once, here
    unsigned w[kFlagWords];
    ENSURE(read_flags(c, s, w));
    const unsigned report = w[0] & (MD_FLAG_NONFINITE | MD_FLAG_TABLE_RANGE);
    if (report) {
        launch_clear_bits(c, report, s);
        HIP_TRY(hipStreamSynchronize(s));
        return (report & MD_FLAG_NONFINITE) ? MD_ERR_NONFINITE : MD_ERR_TABLE_RANGE;
    }
    return MD_OK;
}

int md_autotune(md_ctx *h, void *stream, int32_t *block)
{
    if (!h || !block) return MD_ERR_ARG;
    Ctx &c = h->c;
    if (!c.state_set) return MD_ERR_STATE;
    *block = c.batch_block;
    if (!(c.B > 1 && c.batched && !c.baro_on)) {
        // md_step runs the single-box passes: keep the faster of the tiled
        // and the per-atom passes for a step (density, force with the fused
        // kicks, a tenth of a list build), timed on the current state
        if (!c.tile_feasible || c.baro_on) return MD_OK;
        // candidates: the per-atom passes (-1) and the tiled passes with each
        // candidate tile shape
        auto cost_of = [&](double &cost) -> int {
            double b = 0.0, d = 0.0, f = 0.0;
            int rc;
            if ((rc = md_time_pass(h, MD_PASS_BUILD, 2, stream, &b)) != MD_OK ||
                (rc = md_time_pass(h, MD_PASS_DENSITY, 10, stream, &d)) != MD_OK ||
                (rc = md_time_pass(h, MD_PASS_FORCE_STEP, 10, stream, &f)) != MD_OK)
                return rc;
            cost = d + f + 0.1 * b;
            return MD_OK;
        };
        const int start = c.tile_shape;
        int best = -1, rc;
        double best_cost = 0.0;
        set_tiled(c, false);
        if ((rc = cost_of(best_cost)) != MD_OK) return rc;
        hipStream_t s = as_stream(stream);
        for (int k = 0; 3 * (size_t)k < c.tile_shapes.size(); ++k) {
            if ((rc = apply_tile_shape(c, k)) != MD_OK) return rc;
            set_tiled(c, true);
            // a shape whose halo does not fit a tile's LDS on this state is no
            // candidate: its build is checked here, and its halt cleared,
            // instead of moving the context to the per-atom passes
            launch_build(c, false, s);
            unsigned w[kFlagWords];
            if ((rc = read_flags(c, s, w)) != MD_OK) return rc;
            // the build sorted the state either way: densities and forces are stale
            c.density_valid = c.forces_valid = false;
            if (w[kHaltWord]) {
                launch_fill_u32(c.dev.flags + kHaltWord, 2, 0u, s);
                launch_clear_bits(c, MD_FLAG_TILE_OVERFLOW, s);
                c.list_valid = false;
                continue;
            }
            c.list_valid = true;
            double cost = 0.0;
            if ((rc = cost_of(cost)) != MD_OK) return rc;
            if (cost <= best_cost) {
                best_cost = cost;
                best = k;
            }
        }
        if ((rc = apply_tile_shape(c, best >= 0 ? best : start)) != MD_OK) return rc;
        set_tiled(c, best >= 0);
        return MD_OK;
    }
    hipStream_t s = as_stream(stream);
    const size_t nb = sizeof(double) * (size_t)c.N;
    double *keep[6] = {c.bd.sx, c.bd.sy, c.bd.sz, c.bd.svx, c.bd.svy, c.bd.svz};
    double *live[6] = {c.st.x, c.st.y, c.st.z, c.st.vx, c.st.vy, c.st.vz};
    // positions and velocities kept in the build scratch (the stepper does not use it)
    for (int k = 0; k < 6; ++k)
        HIP_TRY(hipMemcpyAsync(keep[k], live[k], nb, hipMemcpyDeviceToDevice, s));
    auto restore = [&]() -> int {
        for (int k = 0; k < 6; ++k)
            HIP_TRY(hipMemcpyAsync(live[k], keep[k], nb, hipMemcpyDeviceToDevice, s));
        batched_invalidate(c);
        c.forces_valid = c.list_valid = c.density_valid = false;
        return MD_OK;
    };
    // block shapes: workgroup size x pack capacity (one box, one or two
    // workgroups' worth of atoms) x visiting order
    struct Shape {
        int block, cap, order;
    };
    std::vector<Shape> shapes;
    for (int T : {256, 512, 1024})
        for (int cap : {0, T, 2 * T})
            for (int order : {0, 1}) shapes.push_back({T, cap, order});
    const int reps = 20;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best_ms = 0.0f;
    Shape best{c.batch_block, c.batch_cap, c.batch_cell_order};
    int rc = MD_OK;
    for (const Shape &sh : shapes) {
        if ((rc = restore()) != MD_OK) break;
        c.batch_block = sh.block;
        c.batch_cap = sh.cap;
        c.batch_cell_order = sh.order;
        if ((rc = launch_batched_steps(c, 5, s)) != MD_OK) break;  // lists, forces, first steps
        if (hipEventRecord(e0, s) != hipSuccess) { rc = MD_ERR_DEVICE; break; }
        if ((rc = launch_batched_steps(c, reps, s)) != MD_OK) break;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            rc = MD_ERR_DEVICE;
            break;
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (best_ms == 0.0f || ms < best_ms) {
            best_ms = ms;
            best = sh;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c.batch_block = best.block;
    c.batch_cap = best.cap;
    c.batch_cell_order = best.order;
    int rr = restore();
    HIP_TRY(hipStreamSynchronize(s));
    *block = best.block;
    return rc != MD_OK ? rc : rr;
}

int md_pressure(md_ctx *h, double *p_box, double *w_box, void *stream)
{
    if (!h || (!p_box && !w_box)) return MD_ERR_ARG;
    Ctx &c = h->c;
    if (!c.state_set) return MD_ERR_STATE;
    hipStream_t s = as_stream(stream);
    ENSURE(ensure_density(c, s));
    launch_force(c, true, 0, s);
    c.forces_valid = true;
    launch_pressure_eval(c, s);
    size_t nb = sizeof(double) * (size_t)c.B;
    if (p_box) HIP_TRY(hipMemcpyAsync(p_box, c.d_baro + 3 * c.B, nb, hipMemcpyDeviceToDevice, s));
    if (w_box) HIP_TRY(hipMemcpyAsync(w_box, c.d_baro + 4 * c.B, nb, hipMemcpyDeviceToDevice, s));
    return MD_OK;
}

int md_set_barostat(md_ctx *h, double p0, double tau, double beta)
{
    if (!h) return MD_ERR_ARG;
    Ctx &c = h->c;
    if (tau > 0.0) {
        if (!std::isfinite(p0) || !std::isfinite(tau) || !(beta > 0.0) || !std::isfinite(beta))
            return MD_ERR_ARG;
        if (c.any_frozen) return MD_ERR_ARG;  // scaling would move frozen atoms
        c.baro_on = true;
        c.baro_p0 = p0;
        c.baro_tau = tau;
        c.baro_beta = beta;
    } else if (c.baro_on) {
        // back to fixed boxes: the host takes the current box lengths, and the
        // next pass rebuilds the list without strain
        HIP_TRY(hipDeviceSynchronize());
        HIP_TRY(hipMemcpy(c.box_len.data(), c.d_boxd, sizeof(double) * (size_t)c.B,
                          hipMemcpyDeviceToHost));
        c.baro_on = false;
        c.list_valid = c.density_valid = c.forces_valid = false;
        if (c.B > 1) {
            int rc = batched_prepare(c);
            if (rc != MD_OK) return rc;
        }
    }
    c.baro_mu_valid = false;
    graph_reset(c);
    return MD_OK;
}

int md_set_frozen(md_ctx *h, const uint8_t *frozen)
{
    if (!h) return MD_ERR_ARG;
    Ctx &c = h->c;
    bool any = false;
    if (frozen)
        for (int64_t i = 0; i < c.N && !any; ++i) any = frozen[i] != 0;
    if (any && c.baro_on) return MD_ERR_ARG;
    HIP_TRY(hipDeviceSynchronize());
    if (any) {
        std::vector<unsigned char> f(c.N);
        for (int64_t i = 0; i < c.N; ++i) f[i] = frozen[i] ? 1 : 0;
        HIP_TRY(hipMemcpy(c.d_frozen0, f.data(), (size_t)c.N, hipMemcpyHostToDevice));
        c.st.frozen = c.d_frozen;
        c.st.frozen0 = c.d_frozen0;
        if (c.state_set) {
            // the slots' flags follow their original ids; frozen atoms stop
            launch_refresh_frozen(c, nullptr);
            HIP_TRY(hipDeviceSynchronize());
        }
    } else {
        c.st.frozen = nullptr;
        c.st.frozen0 = nullptr;
    }
    c.any_frozen = any;
    c.baro_mu_valid = false;
    graph_reset(c);
    return MD_OK;
}

int md_set_types(md_ctx *h, const int32_t *types, const double *type_mass)
{
    if (!h || !types) return MD_ERR_ARG;
    Ctx &c = h->c;
    if (c.ntypes < 2) return MD_ERR_ARG;
    for (int64_t i = 0; i < c.N; ++i)
        if (types[i] < 0 || types[i] >= c.ntypes) return MD_ERR_ARG;
    std::vector<double> m(c.ntypes, c.mass);
    if (type_mass)
        for (int t = 0; t < c.ntypes; ++t) {
            if (!(type_mass[t] > 0.0) || !std::isfinite(type_mass[t])) return MD_ERR_ARG;
            m[t] = type_mass[t];
        }
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(c.d_type0, types, sizeof(int) * (size_t)c.N, hipMemcpyHostToDevice));
    c.type_mass = m;
    int rc = upload_type_coef(c);
    if (rc != MD_OK) return rc;
    if (c.state_set) {
        // the slots' species follow their original ids
        launch_refresh_types(c, nullptr);
        HIP_TRY(hipDeviceSynchronize());
    }
    // rows carry the neighbours' species; energies and forces change (and
    // with cutoffs per pair of types, the rows themselves)
    c.list_valid = c.density_valid = c.forces_valid = false;
    batched_invalidate(c);
    c.baro_mu_valid = false;
    graph_reset(c);
    return MD_OK;
}

int md_set_thermostat(md_ctx *h, double t_e, double tau_t)
{
    if (!h) return MD_ERR_ARG;
    Ctx &c = h->c;
    if (std::isnan(tau_t) || std::isinf(tau_t)) return MD_ERR_ARG;
    if (tau_t > 0.0) {
        if (!(t_e >= 0.0) || !std::isfinite(t_e)) return MD_ERR_ARG;
        // v_e^2 = 3 k_B T_e / m in (Angstrom/fs)^2
        const double kb = 8.617333262e-5;
        const double kappa = 1.602176634e-19 / 1.66053906660e-27 * 1e-10;
        double e = std::exp(-c.dt / tau_t);
        double ve2 = 3.0 * kb * t_e * kappa / c.mass;
        c.thermo = Thermo{e, (1.0 - e) * ve2, 1};
        c.thermo_te = t_e;
        c.thermo_tau = tau_t;
    } else {
        c.thermo = Thermo{1.0, 0.0, 0};
        c.thermo_te = c.thermo_tau = 0.0;
    }
    int rc = upload_type_coef(c);
    if (rc != MD_OK) return rc;
    graph_reset(c);
    return MD_OK;
}

int md_get_box(md_ctx *h, double *box_len, void *stream)
{
    if (!h || !box_len) return MD_ERR_ARG;
    Ctx &c = h->c;
    hipStream_t s = as_stream(stream);
    HIP_TRY(hipMemcpyAsync(box_len, c.d_boxd, sizeof(double) * (size_t)c.B,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return MD_OK;
}

int md_kinetic(md_ctx *h, double *ke_box, void *stream)
{
    if (!h || !ke_box) return MD_ERR_ARG;
    if (!h->c.state_set) return MD_ERR_STATE;
    launch_box_sums(h->c, 1, ke_box, as_stream(stream));
    return MD_OK;
}

int md_get_neighbors(md_ctx *h, int32_t *counts, int32_t *ids, int32_t max_cols, void *stream)
{
    if (!h || !counts || !ids || max_cols < 1) return MD_ERR_ARG;
    Ctx &c = h->c;
    if (!c.state_set) return MD_ERR_STATE;
    hipStream_t s = as_stream(stream);
    ENSURE(ensure_list(c, s));
    launch_get_neighbors(c, counts, ids, max_cols, s);
    HIP_TRY(hipStreamSynchronize(s));
    return MD_OK;
}

int md_max_neighbors(const md_ctx *h, int32_t *out)
{
    if (!h || !out) return MD_ERR_ARG;
    *out = h->c.nl.mn;
    return MD_OK;
}

int md_set_max_neighbors(md_ctx *h, int32_t mn)
{
    if (!h || mn < 1) return MD_ERR_ARG;
    Ctx &c = h->c;
    HIP_TRY(hipDeviceSynchronize());
    int rc = alloc_list(c, mn);
    if (rc != MD_OK) return rc;
    graph_reset(c);
    c.list_valid = c.density_valid = c.forces_valid = false;
    if (c.B > 1) {
        rc = batched_prepare(c);
        if (rc != MD_OK) return rc;
    }
    return MD_OK;
}

int md_status(md_ctx *h, void *stream, uint32_t *flags, int64_t *counters)
{
    if (!h) return MD_ERR_ARG;
    Ctx &c = h->c;
    HIP_TRY(hipStreamSynchronize(as_stream(stream)));
    unsigned w[8];
    HIP_TRY(hipMemcpy(w, c.dev.flags, sizeof(w), hipMemcpyDeviceToHost));
    if (flags) *flags = w[0];
    if (counters) {
        counters[0] = ((int64_t)w[4] << 32) | w[2];
        counters[1] = (((int64_t)w[5] << 32) | w[3]) + c.host_steps;
    }
    HIP_TRY(hipMemset(c.dev.flags, 0, sizeof(unsigned)));
    HIP_TRY(hipDeviceSynchronize());
    return MD_OK;
}

int md_adjoint(md_ctx *h, const double *g, const double *e, double *gtheta, void *stream)
{
    if (!h || !g || !e || !gtheta) return MD_ERR_ARG;
    Ctx &c = h->c;
    if (c.kind_user != MD_POT_BSPLINE) return MD_ERR_ARG;
    if (!c.state_set) return MD_ERR_STATE;
    hipStream_t s = as_stream(stream);
    ENSURE(ensure_density(c, s));
    launch_adjoint(c, g, e, gtheta, s);
    return MD_OK;
}

int md_time_pass(md_ctx *h, int32_t pass, int32_t reps, void *stream, double *avg_ms)
{
    if (!h || !avg_ms || reps < 1 || pass < MD_PASS_BUILD || pass > MD_PASS_PRESSURE)
        return MD_ERR_ARG;
    Ctx &c = h->c;
    if (!c.state_set) return MD_ERR_STATE;
    hipStream_t s = as_stream(stream);
    ENSURE(ensure_density(c, s));
    if (!c.forces_valid) {
        launch_force(c, false, 0, s);
        c.forces_valid = true;
    }
    size_t nb = sizeof(double) * (size_t)c.N;
    double *save[6] = {c.bd.sx, c.bd.sy, c.bd.sz, c.bd.svx, c.bd.svy, c.bd.svz};
    double *live[6] = {c.st.x, c.st.y, c.st.z, c.st.vx, c.st.vy, c.st.vz};
    for (int k = 0; k < 6; ++k) HIP_TRY(hipMemcpyAsync(save[k], live[k], nb, hipMemcpyDeviceToDevice, s));
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) {
        switch (pass) {
        case MD_PASS_BUILD: launch_build(c, false, s); break;
        case MD_PASS_DENSITY: launch_density(c, s); break;
        case MD_PASS_FORCE: launch_force(c, false, 1, s); break;
        case MD_PASS_FORCE_STEP: launch_force(c, false, c.tiled ? 2 : 1, s); break;
        case MD_PASS_PRESSURE:
            launch_force(c, true, 0, s);
            launch_pressure_eval(c, s);
            break;
        case MD_PASS_KICK_DRIFT: launch_kick_drift(c, s); break;
        }
    }
    HIP_TRY(hipEventRecord(e1, s));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *avg_ms = ms / reps;
    if (pass == MD_PASS_BUILD) {
        // the build scratch held the saved state; the next pass builds (with
        // the capacity check) on the unchanged positions
        batched_invalidate(c);
        c.list_valid = c.density_valid = c.forces_valid = false;
        return MD_OK;
    }
    for (int k = 0; k < 6; ++k) HIP_TRY(hipMemcpyAsync(live[k], save[k], nb, hipMemcpyDeviceToDevice, s));
    launch_pack_positions(c, s);
    launch_fill_u32(c.dev.flags + 1, 1, 0u, s);
    if (pass == MD_PASS_KICK_DRIFT) launch_force(c, false, 0, s);
    HIP_TRY(hipStreamSynchronize(s));
    return MD_OK;
}

int md_set_option(md_ctx *h, int32_t key, int64_t v)
{
    if (!h) return MD_ERR_ARG;
    Ctx &c = h->c;
    switch (key) {
    case MD_OPT_BATCHED:
        if (v && !c.batch_feasible) return MD_ERR_ARG;
        c.batched = v != 0;
        return MD_OK;
    case MD_OPT_BATCH_BLOCK:
        if (v != 256 && v != 512 && v != 1024) return MD_ERR_ARG;
        c.batch_block = (int)v;
        return MD_OK;
    case MD_OPT_USE_GRAPH:
        c.use_graph = v != 0;
        return MD_OK;
    case MD_OPT_GRAPH_STEPS:
        if (v < 1 || v > 1024) return MD_ERR_ARG;
        c.graph_steps = (int)v;
        graph_reset(c);
        return MD_OK;
    case MD_OPT_TILED:
        if (v && !c.tile_feasible) return MD_ERR_ARG;
        set_tiled(c, v != 0);
        return MD_OK;
    case MD_OPT_BATCH_PACK:
        if (v < 0 || v > 65535) return MD_ERR_ARG;
        c.batch_cap = (int)v;
        return MD_OK;
    case MD_OPT_BATCH_ORDER:
        if (v != 0 && v != 1) return MD_ERR_ARG;
        c.batch_cell_order = (int)v;
        return MD_OK;
    case MD_OPT_TILE_SHAPE:
        if (v < 0 || 3 * (uint64_t)v >= c.tile_shapes.size()) return MD_ERR_ARG;
        return apply_tile_shape(c, (int)v);
    }
    return MD_ERR_ARG;
}

int md_get_option(const md_ctx *h, int32_t key, int64_t *v)
{
    if (!h || !v) return MD_ERR_ARG;
    const Ctx &c = h->c;
    switch (key) {
    case MD_OPT_BATCHED: *v = c.batched; return MD_OK;
    case MD_OPT_BATCH_BLOCK: *v = c.batch_block; return MD_OK;
    case MD_OPT_USE_GRAPH: *v = c.use_graph; return MD_OK;
    case MD_OPT_GRAPH_STEPS: *v = c.graph_steps; return MD_OK;
    case MD_OPT_TILED: *v = c.tiled; return MD_OK;
    case MD_OPT_BATCH_PACK: *v = c.batch_cap; return MD_OK;
    case MD_OPT_BATCH_ORDER: *v = c.batch_cell_order; return MD_OK;
    case MD_OPT_TILE_SHAPE: *v = c.tile_shape; return MD_OK;
    case MD_OPT_TILE_SHAPES: *v = (int64_t)(c.tile_shapes.size() / 3); return MD_OK;
    case MD_OPT_TILE_DIMS: {
        const int *d = &c.tile_shapes[3 * (size_t)c.tile_shape];
        *v = c.tile_feasible ? (int64_t)d[0] | (int64_t)d[1] << 8 | (int64_t)d[2] << 16 : 0;
        return MD_OK;
    }
    }
    return MD_ERR_ARG;
}

}  // extern "C"
