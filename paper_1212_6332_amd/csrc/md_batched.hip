// Form (2): many small independent periodic boxes stepped by one persistent
// kernel.
//
// The paper runs many small boxes in one job by merging them into one large
// box whose cells are offset box by box (Section 4.4).  Here each workgroup
// takes whole boxes from a queue (largest first) and advances a box through
// all requested velocity-Verlet steps before taking the next one.  A box's
// positions (and F'(rho)) stay in LDS for the whole launch; the phases of a
// step (kick + drift, optional list rebuild, density + embedding, force +
// kick) are separated by workgroup barriers only, since no box spans two
// workgroups.  The rebuild (wrap, bin, in-cell order by local index, stencil
// scan) runs inside the workgroup on LDS data, and each box decides its own
// rebuilds.  Neighbour rows hold 16-bit local indices in groups of four per
// atom (one 8-byte load per group, the next group in flight while the
// current one is evaluated), slot-fastest.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "md_device.h"
#include "md_internal.h"

namespace mdk {

namespace {

constexpr double kKappa = 1.602176634e-19 / 1.66053906660e-27 * 1e-10;
constexpr int kMaxSteps = 100;  // steps per launch (bounds one launch's duration)

struct BBox {
    double L, invL, rl2, thr2;
    int nc, n, off, ncell;
};

struct BArgs {
    State st;
    const BBox *boxes;
    const int *order;
    int B;
    unsigned *queue;
    uint16_t *list;   // per box: [mn][n] at off * mn
    int *count;       // [N]
    int mn;
    Pot pot;
    double kick, dt;
    Thermo th;        // friction of eq. (4)
    int nsteps;
    int mode;         // bit 0: rebuild every box first; bit 1: compute forces first
    unsigned *flags;
    int nmax;
};

struct Batch {
    BBox *boxes = nullptr;
    int *order = nullptr;
    unsigned *queue = nullptr;
    uint16_t *list = nullptr;
    int *count = nullptr;
    int nmax = 0, cmax = 0, grid = 0;
    size_t lds = 0;
    int list_mn = 0;          // capacity the list storage was sized for
    bool list_valid = false;
    bool prepared = false;    // later calls keep the caller's MD_OPT_BATCHED choice
    hipGraphExec_t graph = nullptr;  // one captured launch of kMaxSteps steady steps
    int graph_block = 0;             // workgroup size it was captured with
};

using namespace dev;

// Entry m of local atom i in a box of n atoms: group m / 4 of the atom,
// groups of all atoms of the box contiguous (the capacity is a multiple of 4).
__device__ __forceinline__ size_t row16_off(int m, int i, int n)
{
    return (((size_t)(m >> 2) * n + i) << 2) + (m & 3);
}

// Visit the c entries of local atom i: one 8-byte load per group of four,
// group q + 1 in flight while group q is evaluated.
template <class Body>
__device__ __forceinline__ void for_row16(const uint16_t *__restrict__ lst, int i, int n, int c,
                                          Body &&body)
{
    if (c <= 0) return;
    const uint2 *g = reinterpret_cast<const uint2 *>(lst) + i;
    const int ng = (c + 3) >> 2;
    uint2 cur = g[0];
    for (int q = 0; q < ng; ++q) {
        const uint2 nxt = q + 1 < ng ? g[(size_t)(q + 1) * n] : cur;
        const int m = min(4, c - 4 * q);
        const unsigned e[4] = {cur.x & 0xffffu, cur.x >> 16, cur.y & 0xffffu, cur.y >> 16};
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (u < m) body((int)e[u]);
        cur = nxt;
    }
}

template <int KIND, int T>
__global__ __launch_bounds__(T) void k_batched(BArgs a)
{
    extern __shared__ double smem[];
    const int nmax = a.nmax;
    double *X = smem, *Y = smem + nmax, *Z = smem + 2 * nmax, *FP = smem + 3 * nmax;
    // rebuild scratch aliases FP (F' is recomputed after every rebuild)
    uint16_t *cell_of = reinterpret_cast<uint16_t *>(FP);
    uint16_t *slot = cell_of + nmax, *tmp = slot + nmax, *srt = tmp + nmax;
    int *cstart = reinterpret_cast<int *>(smem + 4 * nmax);
    __shared__ int s_box;
    __shared__ unsigned s_flag[2];
    const int tid = threadIdx.x;
    const Pot &pot = a.pot;

    for (;;) {
        if (tid == 0) s_box = (int)atomicAdd(a.queue, 1u);
        __syncthreads();
        const int k = s_box;
        __syncthreads();
        if (k >= a.B) break;
        const BBox bx = a.boxes[a.order[k]];
        const int n = bx.n, off = bx.off, nc = bx.nc;
        const double L = bx.L, invL = bx.invL;
        double *gx = a.st.x + off, *gy = a.st.y + off, *gz = a.st.z + off;
        double *vx = a.st.vx + off, *vy = a.st.vy + off, *vz = a.st.vz + off;
        double *fx = a.st.fx + off, *fy = a.st.fy + off, *fz = a.st.fz + off;
        double *xr = a.st.xr + off, *yr = a.st.yr + off, *zr = a.st.zr + off;
        const unsigned char *frz = a.st.frozen ? a.st.frozen + off : nullptr;
        uint16_t *lst = a.list + (size_t)off * a.mn;
        int *cnt = a.count + off;
        unsigned bad = 0;
        for (int i = tid; i < n; i += T) {
            X[i] = gx[i];
            Y[i] = gy[i];
            Z[i] = gz[i];
        }
        if (tid < 2) s_flag[tid] = 0u;
        __syncthreads();

        auto rebuild = [&]() {
#pragma clang fp contract(off)
            for (int c = tid; c <= bx.ncell; c += T) cstart[c] = 0;
            __syncthreads();
            const double ncL = nc * invL;
            for (int i = tid; i < n; i += T) {
                double x = wrap1(X[i], L), y = wrap1(Y[i], L), z = wrap1(Z[i], L);
                X[i] = x;
                Y[i] = y;
                Z[i] = z;
                int c = (cell_coord(z, ncL, nc) * nc + cell_coord(y, ncL, nc)) * nc +
                        cell_coord(x, ncL, nc);
                cell_of[i] = (uint16_t)c;
                slot[i] = (uint16_t)atomicAdd(&cstart[c], 1);
            }
            __syncthreads();
            if (tid == 0) {
                int run = 0;
                for (int c = 0; c < bx.ncell; ++c) {
                    int t = cstart[c];
                    cstart[c] = run;
                    run += t;
                }
                cstart[bx.ncell] = run;
            }
            __syncthreads();
            for (int i = tid; i < n; i += T) tmp[cstart[cell_of[i]] + slot[i]] = (uint16_t)i;
            __syncthreads();
            // deterministic order inside each cell: ascending local index
            for (int q = tid; q < n; q += T) {
                int p = tmp[q], c = cell_of[p];
                int s = cstart[c], e = cstart[c + 1], rank = 0;
                for (int m = s; m < e; ++m) rank += tmp[m] < p;
                srt[s + rank] = (uint16_t)p;
            }
            __syncthreads();
            for (int i = tid; i < n; i += T) {
                double xi = X[i], yi = Y[i], zi = Z[i];
                xr[i] = xi;
                yr[i] = yi;
                zr[i] = zi;
                int c = cell_of[i];
                int cx = c % nc, cy = (c / nc) % nc, cz = c / (nc * nc);
                int sx[3], sy[3], sz[3];
                int kx = stencil_1d(cx, nc, sx), ky = stencil_1d(cy, nc, sy),
                    kz = stencil_1d(cz, nc, sz);
                int m = 0;
                for (int u = 0; u < kz; ++u)
                    for (int v = 0; v < ky; ++v)
                        for (int w = 0; w < kx; ++w) {
                            int cc = (sz[u] * nc + sy[v]) * nc + sx[w];
                            for (int q = cstart[cc]; q < cstart[cc + 1]; ++q) {
                                int j = srt[q];
                                if (j == i) continue;
                                double dx = X[j] - xi, dy = Y[j] - yi, dz = Z[j] - zi;
                                dx = dx - rint(dx * invL) * L;
                                dy = dy - rint(dy * invL) * L;
                                dz = dz - rint(dz * invL) * L;
                                double r2 = (dx * dx + dy * dy) + dz * dz;
                                if (r2 < bx.rl2) {
                                    if (m < a.mn) lst[row16_off(m, i, n)] = (uint16_t)j;
                                    ++m;
                                }
                            }
                        }
                cnt[i] = m;
                if (m > a.mn) {
                    // recorded for the host, which redoes the call with a
                    // larger capacity (the merged-box halt word stays clear)
                    bad |= MD_FLAG_NLIST_OVERFLOW;
                    atomicMax(a.flags + kMaxRowWord, (unsigned)m);
                }
            }
            __syncthreads();
        };

        auto density = [&]() {
            for (int i = tid; i < n; i += T) {
                double xi = X[i], yi = Y[i], zi = Z[i];
                int c = min(cnt[i], a.mn);
                double rho = 0.0;
                for_row16(lst, i, n, c, [&](int j) {
                    double dx = min_image(X[j] - xi, L, invL);
                    double dy = min_image(Y[j] - yi, L, invL);
                    double dz = min_image(Z[j] - zi, L, invL);
                    double r2 = dist2(dx, dy, dz);
                    if (r2 < pot.rc2) rho += dens<KIND>(pot, r2 * rsqrt_nr(r2), bad);
                });
                double F, Fp;
                embed<KIND>(pot, rho, F, Fp, bad);
                FP[i] = Fp;
            }
            __syncthreads();
        };

        auto force = [&](bool kick) {
            for (int i = tid; i < n; i += T) {
                double xi = X[i], yi = Y[i], zi = Z[i], fpi = FP[i];
                int c = min(cnt[i], a.mn);
                double ax = 0.0, ay = 0.0, az = 0.0;
                for_row16(lst, i, n, c, [&](int j) {
                    double dx = min_image(X[j] - xi, L, invL);
                    double dy = min_image(Y[j] - yi, L, invL);
                    double dz = min_image(Z[j] - zi, L, invL);
                    double r2 = dist2(dx, dy, dz);
                    if (r2 < pot.rc2) {
                        double inv_r = rsqrt_nr(r2), dfr, v, dv;
                        pair_terms<KIND>(pot, r2 * inv_r, dfr, v, dv, bad);
                        double coef = fma(fpi + FP[j], dfr, dv) * inv_r;
                        ax = fma(coef, dx, ax);
                        ay = fma(coef, dy, ay);
                        az = fma(coef, dz, az);
                    }
                });
                fx[i] = ax;
                fy[i] = ay;
                fz[i] = az;
                if (kick) {
                    double ux = fma(a.kick, ax, vx[i]);
                    double uy = fma(a.kick, ay, vy[i]);
                    double uz = fma(a.kick, az, vz[i]);
                    if (a.th.on) friction_flow(a.th, ux, uy, uz);
                    if (frz && frz[i]) ux = uy = uz = 0.0;
                    vx[i] = ux;
                    vy[i] = uy;
                    vz[i] = uz;
                }
            }
            __syncthreads();
        };

        if (a.mode & 1) rebuild();
        if (a.mode & 2) {
            density();
            force(false);
        }
        for (int s = 0; s < a.nsteps; ++s) {
            unsigned *flag = &s_flag[s & 1];
            for (int i = tid; i < n; i += T) {
                double ux = vx[i], uy = vy[i], uz = vz[i];
                if (a.th.on) friction_flow(a.th, ux, uy, uz);
                ux = fma(a.kick, fx[i], ux);
                uy = fma(a.kick, fy[i], uy);
                uz = fma(a.kick, fz[i], uz);
                if (frz && frz[i]) ux = uy = uz = 0.0;
                vx[i] = ux;
                vy[i] = uy;
                vz[i] = uz;
                double x = fma(a.dt, ux, X[i]), y = fma(a.dt, uy, Y[i]), z = fma(a.dt, uz, Z[i]);
                X[i] = x;
                Y[i] = y;
                Z[i] = z;
                double ddx = x - xr[i], ddy = y - yr[i], ddz = z - zr[i];
                double d2 = fma(ddz, ddz, fma(ddy, ddy, ddx * ddx));
                if (d2 > bx.thr2) atomicOr(flag, 1u);
                if (!isfinite(d2)) bad |= MD_FLAG_NONFINITE;
            }
            __syncthreads();
            const bool need = *flag != 0u;
            // the other flag was last read one step ago; clear it for the next step
            if (tid == 0) s_flag[(s + 1) & 1] = 0u;
            if (need) rebuild();
            density();
            force(true);
        }
        for (int i = tid; i < n; i += T) {
            gx[i] = X[i];
            gy[i] = Y[i];
            gz[i] = Z[i];
        }
        if (bad) atomicOr(a.flags, bad);
        __syncthreads();
    }
}

__global__ void k_reset_queue(unsigned *q) { *q = 0u; }

template <int KIND>
void launch_kind(Ctx &c, const BArgs &a, hipStream_t s)
{
    Batch &b = *static_cast<Batch *>(c.batch);
    switch (c.batch_block) {
    case 1024: k_batched<KIND, 1024><<<b.grid, 1024, b.lds, s>>>(a); break;
    case 512: k_batched<KIND, 512><<<b.grid, 512, b.lds, s>>>(a); break;
    default: k_batched<KIND, 256><<<b.grid, 256, b.lds, s>>>(a); break;
    }
}

template <int KIND, int T>
int occupancy(size_t lds)
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batched<KIND, T>, T, lds) !=
        hipSuccess)
        return 0;
    return blocks;
}

template <int KIND>
int occupancy_for(int T, size_t lds)
{
    if (T == 1024) return occupancy<KIND, 1024>(lds);
    if (T == 512) return occupancy<KIND, 512>(lds);
    return occupancy<KIND, 256>(lds);
}

template <int KIND, int T>
void allow_lds(size_t lds)
{
    (void)hipFuncSetAttribute((const void *)k_batched<KIND, T>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

}  // namespace

int batched_prepare(Ctx &c)
{
    Batch *b = static_cast<Batch *>(c.batch);
    if (!b) {
        b = new Batch();
        c.batch = b;
    }
    if (c.ntypes > 1) {
        // the persistent stepper evaluates one species
        c.batch_feasible = c.batched = false;
        return MD_OK;
    }
    int nmax = 0, cmax = 0;
    for (int i = 0; i < c.B; ++i) {
        nmax = std::max<int>(nmax, (int)(c.box_off[i + 1] - c.box_off[i]));
        cmax = std::max(cmax, c.box_nc[i] * c.box_nc[i] * c.box_nc[i]);
    }
    b->nmax = nmax;
    b->cmax = cmax;
    b->lds = sizeof(double) * 4 * (size_t)nmax + sizeof(int) * (size_t)(cmax + 2);
    int max_lds = 0;
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c.device) !=
        hipSuccess)
        return MD_ERR_DEVICE;
    // 16-bit local indices; LDS must hold one box
    bool feasible = nmax <= 65535 && cmax <= 65535 && b->lds <= (size_t)max_lds;
    c.batch_feasible = feasible;
    c.batched = b->prepared ? (c.batched && feasible) : feasible;
    b->prepared = true;
    if (!feasible) return MD_OK;
    if (b->lds > 65536) {
        if (c.pot.kind == MD_POT_FS) {
            allow_lds<MD_POT_FS, 256>(b->lds);
            allow_lds<MD_POT_FS, 512>(b->lds);
            allow_lds<MD_POT_FS, 1024>(b->lds);
        } else if (c.pot.kind == MD_POT_SMTB) {
            allow_lds<MD_POT_SMTB, 256>(b->lds);
            allow_lds<MD_POT_SMTB, 512>(b->lds);
            allow_lds<MD_POT_SMTB, 1024>(b->lds);
        } else {
            allow_lds<MD_POT_SPLINE, 256>(b->lds);
            allow_lds<MD_POT_SPLINE, 512>(b->lds);
            allow_lds<MD_POT_SPLINE, 1024>(b->lds);
        }
    }
    if (!b->boxes) {
        void *p[4];
        const size_t bytes[4] = {sizeof(BBox) * c.B, sizeof(int) * c.B, sizeof(unsigned) * 4,
                                 sizeof(int) * (size_t)c.N};
        for (int k = 0; k < 4; ++k) {
            int rc = ctx_alloc(c, &p[k], bytes[k]);
            if (rc != MD_OK) return rc;
        }
        b->boxes = static_cast<BBox *>(p[0]);
        b->order = static_cast<int *>(p[1]);
        b->queue = static_cast<unsigned *>(p[2]);
        b->count = static_cast<int *>(p[3]);
    }
    {
        // per-box descriptors from the current box edges (the barostat changes them)
        std::vector<BBox> hb(c.B);
        for (int i = 0; i < c.B; ++i) {
            double L = c.box_len[i], rl = c.box_rlist[i], half = 0.5 * (rl - c.pot.rc);
            hb[i] = BBox{L, 1.0 / L, rl * rl, half * half, c.box_nc[i],
                         (int)(c.box_off[i + 1] - c.box_off[i]), (int)c.box_off[i],
                         c.box_nc[i] * c.box_nc[i] * c.box_nc[i]};
        }
        std::vector<int> order(c.B);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(),
                         [&](int x, int y) { return hb[x].n > hb[y].n; });
        if (!c.measure && (hipMemcpy(b->boxes, hb.data(), sizeof(BBox) * c.B, hipMemcpyHostToDevice) !=
                hipSuccess ||
            hipMemcpy(b->order, order.data(), sizeof(int) * c.B, hipMemcpyHostToDevice) !=
                hipSuccess))
            return MD_ERR_DEVICE;
    }
    // list storage follows the capacity (reallocated when it changes)
    if (!b->list || b->list_mn != c.nl.mn) {
        void *p = nullptr;
        int rc = ctx_alloc(c, &p, sizeof(uint16_t) * (size_t)c.N * c.nl.mn);
        if (rc != MD_OK) {
            // no room for a list of the new capacity: the merged-box kernels step
            c.batch_feasible = c.batched = false;
            return rc;
        }
        ctx_free(c, b->list);
        b->list = static_cast<uint16_t *>(p);
        b->list_mn = c.nl.mn;
    }
    b->list_valid = false;
    return MD_OK;
}

void batched_invalidate(Ctx &c)
{
    if (c.batch) static_cast<Batch *>(c.batch)->list_valid = false;
}

void batched_graph_reset(Ctx &c)
{
    Batch *b = static_cast<Batch *>(c.batch);
    if (b && b->graph) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
        b->graph_block = 0;
    }
}

void batched_release(Ctx &c)
{
    batched_graph_reset(c);
    delete static_cast<Batch *>(c.batch);
    c.batch = nullptr;
}

int launch_batched_steps(Ctx &c, int nsteps, hipStream_t s)
{
    Batch &b = *static_cast<Batch *>(c.batch);
    int T = c.batch_block;
    int kind = c.pot.kind;
    int occ = kind == MD_POT_FS ? occupancy_for<MD_POT_FS>(T, b.lds)
              : kind == MD_POT_SMTB ? occupancy_for<MD_POT_SMTB>(T, b.lds)
                                    : occupancy_for<MD_POT_SPLINE>(T, b.lds);
    int cus = 0;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c.device);
    b.grid = std::max(1, std::min(c.B, std::max(1, occ) * std::max(1, cus)));
    BArgs a{};
    a.st = c.st;
    a.boxes = b.boxes;
    a.order = b.order;
    a.B = c.B;
    a.queue = b.queue;
    a.list = b.list;
    a.count = b.count;
    a.mn = c.nl.mn;
    a.pot = c.pot;
    a.kick = 0.5 * c.dt * kKappa / c.mass;
    a.dt = c.dt;
    a.th = c.thermo;
    a.flags = c.dev.flags;
    a.nmax = b.nmax;
    auto launch = [&](int k, int mode, hipStream_t st) {
        a.nsteps = k;
        a.mode = mode;
        k_reset_queue<<<1, 1, 0, st>>>(b.queue);
        if (kind == MD_POT_FS) launch_kind<MD_POT_FS>(c, a, st);
        else if (kind == MD_POT_SMTB) launch_kind<MD_POT_SMTB>(c, a, st);
        else launch_kind<MD_POT_SPLINE>(c, a, st);
    };
    int done = 0;
    const int mode = (b.list_valid ? 0 : 1) | (c.forces_valid ? 0 : 2);
    if (mode != 0) {
        // the first launch rebuilds the boxes' lists and/or computes forces first
        int k = std::min(kMaxSteps, nsteps);
        launch(k, mode, s);
        done = k;
    }
    if (c.use_graph && nsteps - done >= kMaxSteps) {
        // full chunks replay one captured launch (reset + persistent kernel)
        if (!b.graph || b.graph_block != T) {
            batched_graph_reset(c);
            hipGraph_t g = nullptr;
            bool ok = hipStreamBeginCapture(c.cap_stream, hipStreamCaptureModeRelaxed) == hipSuccess;
            if (ok) {
                launch(kMaxSteps, 0, c.cap_stream);
                ok = hipStreamEndCapture(c.cap_stream, &g) == hipSuccess && g != nullptr;
            }
            if (ok && hipGraphInstantiate(&b.graph, g, nullptr, nullptr, 0) != hipSuccess)
                b.graph = nullptr;
            if (g) (void)hipGraphDestroy(g);
            b.graph_block = b.graph ? T : 0;
        }
        if (b.graph)
            for (; done + kMaxSteps <= nsteps; done += kMaxSteps)
                if (hipGraphLaunch(b.graph, s) != hipSuccess) return MD_ERR_DEVICE;
    }
    while (done < nsteps) {
        int k = std::min(kMaxSteps, nsteps - done);
        launch(k, 0, s);
        done += k;
    }
    if (hipGetLastError() != hipSuccess) return MD_ERR_DEVICE;
    b.list_valid = true;
    return MD_OK;
}

}  // namespace mdk
