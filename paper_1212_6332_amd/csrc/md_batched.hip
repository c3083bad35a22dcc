// Form (2): many small independent periodic boxes stepped by one persistent
// kernel.
//
// The paper runs many small boxes in one job by merging them into one large
// box whose cells are offset box by box (Section 4.4).  Here each workgroup
// takes a pack of whole boxes from a queue (largest packs first) and advances
// them through all requested velocity-Verlet steps before taking the next
// pack.  A pack is one box, or several consecutive small boxes of the
// size-sorted box order whose atoms together stay within a capacity, so that
// small boxes do not leave most of a workgroup idle.  The pack's positions
// (and F'(rho)) stay in LDS for the whole launch; the phases of a step (kick +
// drift, list rebuild of the boxes that need one, density + embedding, force +
// kick) are separated by workgroup barriers only, since no box spans two
// workgroups.  The rebuild (wrap, bin, in-cell order by local index, stencil
// scan) runs inside the workgroup on LDS data, and each box decides its own
// rebuilds.  Neighbour rows hold 16-bit local indices in groups of four per
// atom (one 8-byte load per group, the next group in flight while the
// current one is evaluated), slot-fastest.  Threads take the pack's atoms in
// index order or, as an option, in the cell order of the last binning (so
// that the lanes of a wavefront hold nearby atoms); neither the packing nor
// the visiting order changes any atom's arithmetic.  Several species use the
// per-type-pair tables, cutoffs and masses of the merged-box kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <type_traits>
#include <vector>

#include "md_device.h"
#include "md_internal.h"

namespace mdk {

namespace {

constexpr double kKappa = 1.602176634e-19 / 1.66053906660e-27 * 1e-10;
constexpr int kMaxSteps = 100;  // steps per launch (bounds one launch's duration)
constexpr int kPackBoxes = 64;  // boxes per pack at most

struct BBox {
    double L, invL, rl2, thr2;
    int nc, n, off, ncell;
};

// Boxes order[first, first + nbox) of the size-sorted order: natoms atoms and
// cells cell-table entries (ncell + 1 per box) in LDS.
struct BPack {
    int first, nbox, natoms, cells;
};

struct BArgs {
    State st;
    const BBox *boxes;
    const int *order;
    const BPack *packs;
    int npacks;
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
    int smax, cmax;   // atoms and cell-table entries of the largest pack
    int cell_order;   // threads visit atoms in the cell order of the last binning
};

// Tuning of the stepper: workgroup size, pack capacity (atoms; 0: one box
// per workgroup), visiting order.  The key of a captured launch.
struct BConf {
    int block = 256, cap = 0, cell_order = 0;
    bool operator==(const BConf &o) const
    {
        return block == o.block && cap == o.cap && cell_order == o.cell_order;
    }
};

struct Batch {
    BBox *boxes = nullptr;
    int *order = nullptr;
    BPack *packs = nullptr;
    unsigned *queue = nullptr;
    uint16_t *list = nullptr;
    int *count = nullptr;
    int npacks = 0, smax = 0, cmax = 0, grid = 0;
    int packed_cap = -1;      // capacity the packs were formed for
    size_t lds = 0;
    int list_mn = 0;          // capacity the list storage was sized for
    bool list_valid = false;
    bool prepared = false;    // later calls keep the caller's MD_OPT_BATCHED choice
    std::vector<BBox> hb;     // host copies
    std::vector<int> horder;
    hipGraphExec_t graph = nullptr;  // one captured launch of kMaxSteps steady steps
    BConf graph_conf;                // configuration it was captured with
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

// LDS of one pack: X, Y, Z, F' (doubles) for smax atoms, the cell table
// (cmax ints), the visiting order (uint16), the box of each atom and, with
// several species, its type (bytes).  The rebuild's cell-of, slot, scatter
// and sorted arrays (uint16 each) alias F', which every step recomputes.
__host__ __device__ inline size_t pack_lds_bytes(int smax, int cmax)
{
    size_t b = 32 * (size_t)smax + 4 * (size_t)cmax + 2 * (size_t)smax + 2 * (size_t)smax;
    return (b + 15) & ~(size_t)15;
}

// The kernel's static LDS (the pack's box descriptors, prefix tables and
// rebuild flags), with a margin for alignment: the dynamic part may take
// what the device allows per workgroup minus this.
constexpr size_t kStaticLds = sizeof(BBox) * kPackBoxes + sizeof(int) * 2 * (kPackBoxes + 1) +
                              sizeof(unsigned) * (2 * kPackBoxes + 2) + sizeof(int) + 256;

template <int KIND, int T>
__global__ __launch_bounds__(T) void k_batched(BArgs a)
{
    constexpr bool TYPED = KIND == kTyped;
    extern __shared__ double smem[];
    const int smax = a.smax;
    double *X = smem, *Y = smem + smax, *Z = smem + 2 * smax, *FP = smem + 3 * smax;
    int *cstart = reinterpret_cast<int *>(smem + 4 * smax);
    uint16_t *visit = reinterpret_cast<uint16_t *>(cstart + a.cmax);
    uint8_t *bof = reinterpret_cast<uint8_t *>(visit + smax);
    uint8_t *ty = bof + smax;
    uint16_t *cell_of = reinterpret_cast<uint16_t *>(FP);
    uint16_t *slot = cell_of + smax, *tmp = slot + smax, *srt = tmp + smax;
    __shared__ BBox s_bx[kPackBoxes];
    __shared__ int s_aoff[kPackBoxes + 1], s_coff[kPackBoxes + 1];
    __shared__ unsigned s_need[2][kPackBoxes], s_any[2];
    __shared__ int s_pack;
    const int tid = threadIdx.x;
    const Pot &pot = a.pot;
    const State &st = a.st;

    for (;;) {
        if (tid == 0) s_pack = (int)atomicAdd(a.queue, 1u);
        __syncthreads();
        const int k = s_pack;
        __syncthreads();
        if (k >= a.npacks) break;
        const BPack pk = a.packs[k];
        const int K = pk.nbox, S = pk.natoms;
        if (tid < K) s_bx[tid] = a.boxes[a.order[pk.first + tid]];
        if (tid < kPackBoxes) s_need[0][tid] = s_need[1][tid] = 0u;
        if (tid < 2) s_any[tid] = 0u;
        __syncthreads();
        if (tid == 0) {
            int na = 0, nc = 0;
            for (int b = 0; b < K; ++b) {
                s_aoff[b] = na;
                s_coff[b] = nc;
                na += s_bx[b].n;
                nc += s_bx[b].ncell + 1;
            }
            s_aoff[K] = na;
            s_coff[K] = nc;
        }
        __syncthreads();
        unsigned bad = 0;
        for (int p = tid; p < S; p += T) {
            int lo = 0, hi = K - 1;  // box holding pack atom p
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (s_aoff[mid] <= p) lo = mid;
                else hi = mid - 1;
            }
            bof[p] = (uint8_t)lo;
            visit[p] = (uint16_t)p;
            const int g = s_bx[lo].off + (p - s_aoff[lo]);
            X[p] = st.x[g];
            Y[p] = st.y[g];
            Z[p] = st.z[g];
            if constexpr (TYPED) ty[p] = (uint8_t)st.type[g];
        }
        __syncthreads();

        // Counting sort of the atoms of the boxes with need[b] set (all boxes
        // for need == nullptr) into their cells, ascending local index inside
        // a cell: srt[aoff + k] is the box-local index of the k-th atom in
        // cell order.  commit: the wrapped positions become the state.
        auto sort_cells = [&](const unsigned *need, bool commit) {
            for (int b = 0; b < K; ++b)
                if (!need || need[b])
                    for (int c = tid; c <= s_bx[b].ncell; c += T) cstart[s_coff[b] + c] = 0;
            __syncthreads();
            for (int p = tid; p < S; p += T) {
                const int b = bof[p];
                if (need && !need[b]) continue;
                const BBox &bx = s_bx[b];
                double x = wrap1(X[p], bx.L), y = wrap1(Y[p], bx.L), z = wrap1(Z[p], bx.L);
                if (commit) {
                    X[p] = x;
                    Y[p] = y;
                    Z[p] = z;
                }
                const int nc = bx.nc;
                const double ncL = nc * bx.invL;
                int c = (cell_coord(z, ncL, nc) * nc + cell_coord(y, ncL, nc)) * nc +
                        cell_coord(x, ncL, nc);
                cell_of[p] = (uint16_t)c;
                slot[p] = (uint16_t)atomicAdd(&cstart[s_coff[b] + c], 1);
            }
            __syncthreads();
            if (tid < K && (!need || need[tid])) {
                int *cs = cstart + s_coff[tid];
                int run = 0;
                for (int c = 0; c < s_bx[tid].ncell; ++c) {
                    int t = cs[c];
                    cs[c] = run;
                    run += t;
                }
                cs[s_bx[tid].ncell] = run;
            }
            __syncthreads();
            for (int p = tid; p < S; p += T) {
                const int b = bof[p];
                if (need && !need[b]) continue;
                tmp[s_aoff[b] + cstart[s_coff[b] + cell_of[p]] + slot[p]] =
                    (uint16_t)(p - s_aoff[b]);
            }
            __syncthreads();
            for (int q = tid; q < S; q += T) {
                const int b = bof[q];
                if (need && !need[b]) continue;
                const int base = s_aoff[b];
                const int pl = tmp[q];
                const int c = cell_of[base + pl];
                const int s0 = cstart[s_coff[b] + c], s1 = cstart[s_coff[b] + c + 1];
                int rank = 0;
                for (int m = s0; m < s1; ++m) rank += tmp[base + m] < pl;
                srt[base + s0 + rank] = (uint16_t)pl;
            }
            __syncthreads();
            if (a.cell_order) {
                for (int q = tid; q < S; q += T) {
                    const int b = bof[q];
                    if (!need || need[b]) visit[q] = (uint16_t)(s_aoff[b] + srt[q]);
                }
                __syncthreads();
            }
        };

        auto rebuild = [&](const unsigned *need) {
#pragma clang fp contract(off)
            sort_cells(need, true);
            for (int q = tid; q < S; q += T) {
                const int p = visit[q], b = bof[p];
                if (need && !need[b]) continue;
                const BBox &bx = s_bx[b];
                const int base = s_aoff[b], i = p - base, n = bx.n, nc = bx.nc;
                const int *cs = cstart + s_coff[b];
                const double L = bx.L, invL = bx.invL;
                double xi = X[p], yi = Y[p], zi = Z[p];
                st.xr[bx.off + i] = xi;
                st.yr[bx.off + i] = yi;
                st.zr[bx.off + i] = zi;
                // several species: the list radius of each pair of types
                const double *rl2row = nullptr;
                if constexpr (TYPED)
                    if (pot.cut2) rl2row = pot.cut2 + pot.nt * pot.nt + ty[p] * pot.nt;
                uint16_t *lst = a.list + (size_t)bx.off * a.mn;
                int c = cell_of[p];
                int cx = c % nc, cy = (c / nc) % nc, cz = c / (nc * nc);
                int sx[3], sy[3], sz[3];
                int kx = stencil_1d(cx, nc, sx), ky = stencil_1d(cy, nc, sy),
                    kz = stencil_1d(cz, nc, sz);
                int m = 0;
                for (int u = 0; u < kz; ++u)
                    for (int v = 0; v < ky; ++v)
                        for (int w = 0; w < kx; ++w) {
                            int cc = (sz[u] * nc + sy[v]) * nc + sx[w];
                            for (int q2 = cs[cc]; q2 < cs[cc + 1]; ++q2) {
                                int j = srt[base + q2];
                                if (j == i) continue;
                                double dx = X[base + j] - xi, dy = Y[base + j] - yi,
                                       dz = Z[base + j] - zi;
                                dx = dx - rint(dx * invL) * L;
                                dy = dy - rint(dy * invL) * L;
                                dz = dz - rint(dz * invL) * L;
                                double r2 = (dx * dx + dy * dy) + dz * dz;
                                bool in = r2 < bx.rl2;
                                if constexpr (TYPED)
                                    if (rl2row) in = r2 < fmin(rl2row[ty[base + j]], bx.rl2);
                                if (in) {
                                    if (m < a.mn) lst[row16_off(m, i, n)] = (uint16_t)j;
                                    ++m;
                                }
                            }
                        }
                a.count[bx.off + i] = m;
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
            for (int q = tid; q < S; q += T) {
                const int p = visit[q], b = bof[p];
                const BBox &bx = s_bx[b];
                const int base = s_aoff[b], i = p - base;
                const double L = bx.L, invL = bx.invL;
                double xi = X[p], yi = Y[p], zi = Z[p];
                const int ai = TYPED ? ty[p] : 0;
                const double *cr = (TYPED && pot.cut2) ? pot.cut2 + ai * pot.nt : nullptr;
                int c = min(a.count[bx.off + i], a.mn);
                double rho = 0.0;
                for_row16(a.list + (size_t)bx.off * a.mn, i, bx.n, c, [&](int j) {
                    double dx = min_image(X[base + j] - xi, L, invL);
                    double dy = min_image(Y[base + j] - yi, L, invL);
                    double dz = min_image(Z[base + j] - zi, L, invL);
                    double r2 = dist2(dx, dy, dz);
                    if constexpr (TYPED) {
                        const int tj = ty[base + j];
                        if (r2 < (cr ? cr[tj] : pot.rc2))
                            rho += dens_typed(pot, r2 * rsqrt_nr(r2), ai, tj, bad);
                    } else {
                        if (r2 < pot.rc2) rho += dens<KIND>(pot, r2 * rsqrt_nr(r2), bad);
                    }
                });
                double F, Fp;
                if constexpr (TYPED)
                    embed_typed(pot, rho, ai, F, Fp, bad);
                else
                    embed<KIND>(pot, rho, F, Fp, bad);
                FP[p] = Fp;
            }
            __syncthreads();
        };

        // Half kick factor and friction of the atom at pack slot p.
        auto kick_of = [&](int p, double &ki, Thermo &thi) {
            ki = a.kick;
            thi = a.th;
            if constexpr (TYPED) {
                const double *tc = st.tcoef + 4 * ty[p];
                ki = tc[kTcKick];
                thi.a = tc[kTcFric];
            }
        };

        auto force = [&](bool kick) {
            for (int q = tid; q < S; q += T) {
                const int p = visit[q], b = bof[p];
                const BBox &bx = s_bx[b];
                const int base = s_aoff[b], i = p - base, g = bx.off + i;
                const double L = bx.L, invL = bx.invL;
                double xi = X[p], yi = Y[p], zi = Z[p], fpi = FP[p];
                const int ai = TYPED ? ty[p] : 0;
                const double *cr = (TYPED && pot.cut2) ? pot.cut2 + ai * pot.nt : nullptr;
                int c = min(a.count[g], a.mn);
                double ax = 0.0, ay = 0.0, az = 0.0;
                for_row16(a.list + (size_t)bx.off * a.mn, i, bx.n, c, [&](int j) {
                    double dx = min_image(X[base + j] - xi, L, invL);
                    double dy = min_image(Y[base + j] - yi, L, invL);
                    double dz = min_image(Z[base + j] - zi, L, invL);
                    double r2 = dist2(dx, dy, dz);
                    double coef;
                    if constexpr (TYPED) {
                        const int tj = ty[base + j];
                        if (!(r2 < (cr ? cr[tj] : pot.rc2))) return;
                        double inv_r = rsqrt_nr(r2), dab, dba, dv;
                        pair_derivs_typed(pot, r2 * inv_r, ai, tj, dab, dba, dv, bad);
                        coef = fma(fpi, dab, fma(FP[base + j], dba, dv)) * inv_r;
                    } else {
                        if (!(r2 < pot.rc2)) return;
                        double inv_r = rsqrt_nr(r2), dfr, dv;
                        pair_derivs<KIND>(pot, r2 * inv_r, dfr, dv, bad);
                        coef = fma(fpi + FP[base + j], dfr, dv) * inv_r;
                    }
                    ax = fma(coef, dx, ax);
                    ay = fma(coef, dy, ay);
                    az = fma(coef, dz, az);
                });
                st.fx[g] = ax;
                st.fy[g] = ay;
                st.fz[g] = az;
                if (kick) {
                    double ki;
                    Thermo thi;
                    kick_of(p, ki, thi);
                    double ux = fma(ki, ax, st.vx[g]);
                    double uy = fma(ki, ay, st.vy[g]);
                    double uz = fma(ki, az, st.vz[g]);
                    if (thi.on) friction_flow(thi, ux, uy, uz);
                    if (st.frozen && st.frozen[g]) ux = uy = uz = 0.0;
                    st.vx[g] = ux;
                    st.vy[g] = uy;
                    st.vz[g] = uz;
                }
            }
            __syncthreads();
        };

        if (a.cell_order) sort_cells(nullptr, false);  // visiting order only
        if (a.mode & 1) rebuild(nullptr);
        if (a.mode & 2) {
            density();
            force(false);
        }
        for (int s = 0; s < a.nsteps; ++s) {
            unsigned *need = s_need[s & 1];
            for (int q = tid; q < S; q += T) {
                const int p = visit[q], b = bof[p];
                const BBox &bx = s_bx[b];
                const int g = bx.off + (p - s_aoff[b]);
                double ki;
                Thermo thi;
                kick_of(p, ki, thi);
                double ux = st.vx[g], uy = st.vy[g], uz = st.vz[g];
                if (thi.on) friction_flow(thi, ux, uy, uz);
                ux = fma(ki, st.fx[g], ux);
                uy = fma(ki, st.fy[g], uy);
                uz = fma(ki, st.fz[g], uz);
                if (st.frozen && st.frozen[g]) ux = uy = uz = 0.0;
                st.vx[g] = ux;
                st.vy[g] = uy;
                st.vz[g] = uz;
                double x = fma(a.dt, ux, X[p]), y = fma(a.dt, uy, Y[p]), z = fma(a.dt, uz, Z[p]);
                X[p] = x;
                Y[p] = y;
                Z[p] = z;
                double ddx = x - st.xr[g], ddy = y - st.yr[g], ddz = z - st.zr[g];
                double d2 = fma(ddz, ddz, fma(ddy, ddy, ddx * ddx));
                if (d2 > bx.thr2 && !need[b]) {
                    atomicOr(&need[b], 1u);
                    atomicOr(&s_any[s & 1], 1u);
                }
                if (!isfinite(d2)) bad |= MD_FLAG_NONFINITE;
            }
            __syncthreads();
            const bool any = s_any[s & 1] != 0u;
            // the other flags were last read one step ago; clear them for the next step
            if (tid < kPackBoxes) s_need[(s + 1) & 1][tid] = 0u;
            if (tid == 0) s_any[(s + 1) & 1] = 0u;
            if (any) rebuild(need);
            density();
            force(true);
        }
        for (int p = tid; p < S; p += T) {
            const int b = bof[p];
            const int g = s_bx[b].off + (p - s_aoff[b]);
            st.x[g] = X[p];
            st.y[g] = Y[p];
            st.z[g] = Z[p];
        }
        if (bad) atomicOr(a.flags, bad);
        __syncthreads();
    }
}

__global__ void k_reset_queue(unsigned *q) { *q = 0u; }

template <int KIND>
void launch_kind(const Batch &b, int T, const BArgs &a, hipStream_t s)
{
    switch (T) {
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

template <int KIND>
void allow_lds(size_t lds)
{
    (void)hipFuncSetAttribute((const void *)k_batched<KIND, 256>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipFuncSetAttribute((const void *)k_batched<KIND, 512>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipFuncSetAttribute((const void *)k_batched<KIND, 1024>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <class F>
auto by_kind(int kind, F &&f)
{
    switch (kind) {
    case MD_POT_FS: return f(std::integral_constant<int, MD_POT_FS>{});
    case MD_POT_SMTB: return f(std::integral_constant<int, MD_POT_SMTB>{});
    case kTyped: return f(std::integral_constant<int, kTyped>{});
    default: return f(std::integral_constant<int, MD_POT_SPLINE>{});
    }
}

// Packs for capacity cap over the size-sorted order: a box starts a pack and
// the boxes after it join while the pack's atoms stay within cap (and LDS
// and the 8-bit box index allow); packs are then queued largest first.
void form_packs(const std::vector<BBox> &hb, const std::vector<int> &order, int cap,
                size_t max_lds, std::vector<BPack> &packs, int &smax, int &cmax)
{
    packs.clear();
    smax = cmax = 0;
    const int B = (int)order.size();
    for (int i = 0; i < B;) {
        const BBox &f = hb[order[i]];
        BPack p{i, 1, f.n, f.ncell + 1};
        for (++i; i < B && p.nbox < kPackBoxes; ++i) {
            const BBox &x = hb[order[i]];
            const int na = p.natoms + x.n, nc = p.cells + x.ncell + 1;
            if (na > cap || pack_lds_bytes(na, nc) > max_lds) break;
            p.natoms = na;
            p.cells = nc;
            ++p.nbox;
        }
        packs.push_back(p);
        smax = std::max(smax, p.natoms);
        cmax = std::max(cmax, p.cells);
    }
    std::stable_sort(packs.begin(), packs.end(),
                     [](const BPack &x, const BPack &y) { return x.natoms > y.natoms; });
}

}  // namespace

int batched_prepare(Ctx &c)
{
    Batch *b = static_cast<Batch *>(c.batch);
    if (!b) {
        b = new Batch();
        c.batch = b;
    }
    int max_lds = 0;
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c.device) !=
        hipSuccess)
        return MD_ERR_DEVICE;
    int nmax = 0, cmax = 0;
    for (int i = 0; i < c.B; ++i) {
        nmax = std::max<int>(nmax, (int)(c.box_off[i + 1] - c.box_off[i]));
        cmax = std::max(cmax, c.box_nc[i] * c.box_nc[i] * c.box_nc[i]);
    }
    // 16-bit local indices and cells, 8-bit species; LDS must hold one box
    bool feasible = nmax <= 65535 && cmax < 65535 && c.ntypes <= 256 &&
                    pack_lds_bytes(nmax, cmax + 1) + kStaticLds <= (size_t)max_lds;
    c.batch_feasible = feasible;
    c.batched = b->prepared ? (c.batched && feasible) : feasible;
    b->prepared = true;
    if (!feasible) return MD_OK;
    if (!b->boxes) {
        void *p[5];
        const size_t bytes[5] = {sizeof(BBox) * c.B, sizeof(int) * c.B, sizeof(BPack) * c.B,
                                 sizeof(unsigned) * 4, sizeof(int) * (size_t)c.N};
        for (int k = 0; k < 5; ++k) {
            int rc = ctx_alloc(c, &p[k], bytes[k]);
            if (rc != MD_OK) return rc;
        }
        b->boxes = static_cast<BBox *>(p[0]);
        b->order = static_cast<int *>(p[1]);
        b->packs = static_cast<BPack *>(p[2]);
        b->queue = static_cast<unsigned *>(p[3]);
        b->count = static_cast<int *>(p[4]);
    }
    {
        // per-box descriptors from the current box edges (the barostat changes them)
        b->hb.resize(c.B);
        for (int i = 0; i < c.B; ++i) {
            double L = c.box_len[i], rl = c.box_rlist[i], half = 0.5 * (rl - c.pot.rc);
            b->hb[i] = BBox{L, 1.0 / L, rl * rl, half * half, c.box_nc[i],
                            (int)(c.box_off[i + 1] - c.box_off[i]), (int)c.box_off[i],
                            c.box_nc[i] * c.box_nc[i] * c.box_nc[i]};
        }
        b->horder.resize(c.B);
        std::iota(b->horder.begin(), b->horder.end(), 0);
        std::stable_sort(b->horder.begin(), b->horder.end(),
                         [&](int x, int y) { return b->hb[x].n > b->hb[y].n; });
        if (!c.measure &&
            (hipMemcpy(b->boxes, b->hb.data(), sizeof(BBox) * c.B, hipMemcpyHostToDevice) !=
                 hipSuccess ||
             hipMemcpy(b->order, b->horder.data(), sizeof(int) * c.B, hipMemcpyHostToDevice) !=
                 hipSuccess))
            return MD_ERR_DEVICE;
        b->packed_cap = -1;   // packs formed again at the next launch
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
    }
}

void batched_release(Ctx &c)
{
    batched_graph_reset(c);
    delete static_cast<Batch *>(c.batch);
    c.batch = nullptr;
}

// Packs for the context's capacity (formed again when it changed), LDS size
// and grid for the workgroup size.
static int batched_configure(Ctx &c, Batch &b, hipStream_t s)
{
    int max_lds = 0, cus = 0;
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c.device) !=
            hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c.device) != hipSuccess)
        return MD_ERR_DEVICE;
    if (b.packed_cap != c.batch_cap) {
        std::vector<BPack> packs;
        form_packs(b.hb, b.horder, c.batch_cap, (size_t)max_lds - kStaticLds, packs, b.smax,
                   b.cmax);
        b.npacks = (int)packs.size();
        b.lds = pack_lds_bytes(b.smax, b.cmax);
        // earlier launches (on any stream) may still read the packs
        (void)s;
        if (hipDeviceSynchronize() != hipSuccess ||
            hipMemcpy(b.packs, packs.data(), sizeof(BPack) * packs.size(),
                      hipMemcpyHostToDevice) != hipSuccess)
            return MD_ERR_DEVICE;
        b.packed_cap = c.batch_cap;
        if (b.lds > 65536) by_kind(c.pot.kind, [&](auto k) { allow_lds<decltype(k)::value>(b.lds); });
    }
    const int occ = by_kind(c.pot.kind, [&](auto k) {
        return occupancy_for<decltype(k)::value>(c.batch_block, b.lds);
    });
    b.grid = std::max(1, std::min(b.npacks, std::max(1, occ) * std::max(1, cus)));
    return MD_OK;
}

int launch_batched_steps(Ctx &c, int nsteps, hipStream_t s)
{
    Batch &b = *static_cast<Batch *>(c.batch);
    int rc = batched_configure(c, b, s);
    if (rc != MD_OK) return rc;
    const BConf conf{c.batch_block, c.batch_cap, c.batch_cell_order};
    BArgs a{};
    a.st = c.st;
    a.boxes = b.boxes;
    a.order = b.order;
    a.packs = b.packs;
    a.npacks = b.npacks;
    a.queue = b.queue;
    a.list = b.list;
    a.count = b.count;
    a.mn = c.nl.mn;
    a.pot = c.pot;
    a.kick = 0.5 * c.dt * kKappa / c.mass;
    a.dt = c.dt;
    a.th = c.thermo;
    a.flags = c.dev.flags;
    a.smax = b.smax;
    a.cmax = b.cmax;
    a.cell_order = c.batch_cell_order;
    auto launch = [&](int k, int mode, hipStream_t st) {
        a.nsteps = k;
        a.mode = mode;
        k_reset_queue<<<1, 1, 0, st>>>(b.queue);
        by_kind(c.pot.kind, [&](auto kk) { launch_kind<decltype(kk)::value>(b, conf.block, a, st); });
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
        if (!b.graph || !(b.graph_conf == conf)) {
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
            if (b.graph) b.graph_conf = conf;
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
