// Tiled passes: the neighbour records a workgroup needs are staged in LDS.
//
// Cells are numbered tile by tile, so the atoms of a tile of tx x ty x tz
// cells are one contiguous range of sorted slots.  One 1024-thread
// workgroup owns one tile.  It first stages the records of the tile's halo
// -- the tile's cells plus one layer of cells around them (the union of the
// 27-cell stencils of Fig. 3) -- from HBM/L2 into LDS, then every thread
// evaluates its atoms' neighbour rows against LDS.  The paper stages list
// candidates in shared memory the same way (Fig. 3, spos); here the density
// and force passes do it too, which turns their scattered global gathers
// (the limiting cost of the per-atom kernels) into LDS reads.
//
// Two halo modes, fixed per box:
//  A  (boxes with at least max(t)+2 cells per axis): the halo is the tile
//     grown by one cell; a halo cell past a face of the box is the cell on
//     the far side of the box, whose pairs with the tile's atoms cross that
//     face.
//  B  (small boxes): one tile is the whole box, staged once.
// Records hold the wrapped coordinates in both modes.  The list build puts
// the pairs that need no periodic correction at the front of a row and the
// pairs that cross a face at its back (as the per-atom rows do); the passes
// take the minimum image for the back part only.  Every kernel therefore
// forms x_j - x_i first and adds the periodic shift after it, and tests the
// cutoff on the separately rounded square of that separation, so the set of
// interacting pairs is the same whichever kernel evaluates a pair.
// Rows hold the byte offsets of halo records in the LDS record array
// (record index times 32), so the passes address a record with no
// arithmetic; with several species the neighbour's species rides in the
// five low bits of its entry.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "md_device.h"
#include "md_internal.h"

namespace mdk {

namespace {

using namespace dev;

constexpr int kT = kTileThreads;

struct Tile {
    int b, nc, mode;
    double L, invL;
    int ox, oy, oz;   // first cell of the tile
    int hx, hy, hz;   // halo extent in cells
    int s0, s1;       // slot range of the tile
    int nh;           // halo cells
};

constexpr int kNoShift = 1 | (1 << 2) | (1 << 4);  // shift code of an unshifted cell

// Shared halo table: per halo cell, LDS offset, first slot, image shift code.
// Its 256-byte alignment (and size) keeps the record array behind it aligned,
// so each record's 16-byte halves are aligned for 128-bit LDS reads.
struct alignas(256) HaloLds {
    int off[kHaloCells + 1];
    int start[kHaloCells];
    int shift[kHaloCells];   // (sx+1) | (sy+1) << 2 | (sz+1) << 4, s in {-1, 0, 1}
    int wsum[16];
    int total;
};

// Tile of workgroup b of a one-workgroup-per-tile launch of G workgroups:
// workgroups are dispatched round robin over the 8 dies, and the workgroups
// of one die take one contiguous eighth of the tiles (neighbouring tiles share
// halo cells, which then pass through one L2), in the sweep order `order`
// (null: tile index order).
__device__ __forceinline__ int xcd_tile(int b, int G, const int *order)
{
    const int X = 8;
    int q = G / X, r = G % X, k = b % X, w = b / X;
    const int p = (k < r) ? k * (q + 1) + w : r * (q + 1) + (k - r) * q + w;
    return order ? order[p] : p;
}

__device__ __forceinline__ void tile_setup(const Boxes &bx, const Build &bd, int g, Tile &t)
{
    int b = bx.tile_box[g];
    const int *tg = bx.tile + 8 * b;
    int tx = tg[0], ty = tg[1], tz = tg[2], gx = tg[3], gy = tg[4], tc = tg[6];
    t.b = b;
    t.mode = tg[7];
    t.nc = bx.nc[b];
    t.L = bx.L[b];
    t.invL = bx.invL[b];
    int lin = g - bx.tile_off[b];
    int Tx = lin % gx, Ty = (lin / gx) % gy, Tz = lin / (gx * gy);
    t.ox = Tx * tx;
    t.oy = Ty * ty;
    t.oz = Tz * tz;
    if (t.mode == kTileA) {
        t.hx = min(tx, t.nc - t.ox) + 2;
        t.hy = min(ty, t.nc - t.oy) + 2;
        t.hz = min(tz, t.nc - t.oz) + 2;
    } else {
        t.hx = t.hy = t.hz = t.nc;
    }
    t.nh = t.hx * t.hy * t.hz;
    int first = bx.cell_off[b] + lin * tc;
    t.s0 = bd.cell_start[first];
    t.s1 = bd.cell_start[first + tc];
}

// Exclusive scan over the 1024 threads of the block (one value each).
__device__ __forceinline__ int block_scan(int v, HaloLds &H)
{
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int incl = v;
    for (int off = 1; off < 64; off <<= 1) {
        int u = __shfl_up(incl, off);
        if (lane >= off) incl += u;
    }
    if (lane == 63) H.wsum[w] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int k = 0; k < 16; ++k) {
            int x = H.wsum[k];
            H.wsum[k] = run;
            run += x;
        }
        H.total = run;
    }
    __syncthreads();
    return H.wsum[w] + incl - v;
}

// Halo table of a tile (all threads).
__device__ __forceinline__ void halo_table(const Tile &t, const Boxes &bx, const Build &bd,
                                           HaloLds &H)
{
    int h = threadIdx.x;
    int cnt = 0;
    if (h < t.nh) {
        int ix = h % t.hx, iy = (h / t.hx) % t.hy, iz = h / (t.hx * t.hy);
        int cx, cy, cz, code;
        if (t.mode == kTileA) {
            int ux = t.ox + ix - 1, uy = t.oy + iy - 1, uz = t.oz + iz - 1;
            int sx = ux < 0 ? -1 : (ux >= t.nc ? 1 : 0);
            int sy = uy < 0 ? -1 : (uy >= t.nc ? 1 : 0);
            int sz = uz < 0 ? -1 : (uz >= t.nc ? 1 : 0);
            cx = ux - sx * t.nc;
            cy = uy - sy * t.nc;
            cz = uz - sz * t.nc;
            code = (sx + 1) | ((sy + 1) << 2) | ((sz + 1) << 4);
        } else {
            cx = ix;
            cy = iy;
            cz = iz;
            code = 1 | (1 << 2) | (1 << 4);
        }
        int c = cell_id(bx, t.b, cx, cy, cz);
        int s = bd.cell_start[c];
        cnt = bd.cell_start[c + 1] - s;
        H.start[h] = s;
        H.shift[h] = code;
    }
    int off = block_scan(cnt, H);
    if (h < t.nh) H.off[h] = off;
    if (h == 0) H.off[t.nh] = H.total;
    __syncthreads();
}

__device__ __forceinline__ double shift_of(int code, int axis, double L)
{
    return (double)(((code >> (2 * axis)) & 3) - 1) * L;
}

// Stage the halo records: x, y, z (+ F') at 32 bytes per record, at the
// wrapped coordinates.  Every thread copies records k = tid, tid + 1024, ...;
// its loads are all issued before the first LDS store, so a tile pays about
// one memory round trip for its whole halo.  The slot of each record goes to
// src_out, from which the passes stage the same records again.
template <bool WITH_FP>
__device__ __forceinline__ void stage(const Tile &t, const State &st, const HaloLds &H,
                                      double *rec, int hmax, unsigned *flags,
                                      unsigned *src_out = nullptr)
{
    constexpr int R = 6;  // records per thread per round (hmax <= R * 1024 per round)
    int total = min(H.total, hmax);
    for (int base = 0; base < total; base += R * kT) {
        double vx[R], vy[R], vz[R], vf[R];
        int kk[R], ty[R];
#pragma unroll
        for (int u = 0; u < R; ++u) {
            int k = base + u * kT + (int)threadIdx.x;
            kk[u] = k;
            if (k < total) {
                int lo = 0, hi = t.nh - 1;  // halo cell holding record k
                while (lo < hi) {
                    int mid = (lo + hi + 1) >> 1;
                    if (H.off[mid] <= k) lo = mid;
                    else hi = mid - 1;
                }
                int j = H.start[lo] + (k - H.off[lo]);
                if (src_out) src_out[k] = (unsigned)j;
                vx[u] = st.x[j];
                vy[u] = st.y[j];
                vz[u] = st.z[j];
                if constexpr (WITH_FP) vf[u] = st.Fp[j];
                else ty[u] = st.type ? st.type[j] : 0;
            }
        }
#pragma unroll
        for (int u = 0; u < R; ++u) {
            if (kk[u] < total) {
                double *r = rec + 4 * (size_t)kk[u];
                r[0] = vx[u];
                r[1] = vy[u];
                r[2] = vz[u];
                if constexpr (WITH_FP) r[3] = vf[u];
                else reinterpret_cast<int *>(r + 3)[0] = ty[u];
            }
        }
    }
    if (threadIdx.x == 0 && H.total > hmax) raise_overflow(flags, MD_FLAG_TILE_OVERFLOW, 0);
    __syncthreads();
}

// Stage the halo records of tile g from its source list (written by the list
// build): one coalesced load of the list, then the gathers.
template <bool WITH_FP>
__device__ __forceinline__ void stage_list(int g, const State &st, const NList &nl, double *rec,
                                           int hmax)
{
    constexpr int R = 6;  // records per thread per round (hmax <= R * 1024 per round)
    const int total = min(nl.ttotal[g], hmax);
    const unsigned *src = nl.tsrc + (size_t)g * hmax;
    for (int base = 0; base < total; base += R * kT) {
        double vx[R], vy[R], vz[R], vf[R];
        int kk[R];
#pragma unroll
        for (int u = 0; u < R; ++u) {
            int k = base + u * kT + (int)threadIdx.x;
            kk[u] = k;
            if (k < total) {
                int j = (int)src[k];
                vx[u] = st.x[j];
                vy[u] = st.y[j];
                vz[u] = st.z[j];
                if constexpr (WITH_FP) vf[u] = st.Fp[j];
            }
        }
#pragma unroll
        for (int u = 0; u < R; ++u) {
            if (kk[u] < total) {
                double *r = rec + 4 * (size_t)kk[u];
                r[0] = vx[u];
                r[1] = vy[u];
                r[2] = vz[u];
                if constexpr (WITH_FP) r[3] = vf[u];
            }
        }
    }
    __syncthreads();
}

// Halo cell of a local cell coordinate (tile-relative, -1..extent).
__device__ __forceinline__ int halo_index(const Tile &t, int ix, int iy, int iz)
{
    return ((iz + 1) * t.hy + (iy + 1)) * t.hx + (ix + 1);
}

// ---------------------------------------------------------------- list build

// Row layout: the pairs that need no periodic correction at entries [0, np),
// then the pairs that cross a face of the box at [np, n); count = n | np << 16.
// While the row is built the crossing pairs go to its back, [mn - nb, mn);
// `close` moves them behind the others.
struct RowFill {
    int np = 0, nb = 0, total = 0;
    __device__ __forceinline__ void put(int *__restrict__ idx, int i, int N, int mn, bool plain,
                                        int e)
    {
        if (np + nb < mn) idx[nl_off(plain ? np++ : mn - 1 - nb++, i, N)] = e;
    }
    // entries move down (np <= mn - nb), so each is read before it is overwritten
    __device__ __forceinline__ int close(int *__restrict__ idx, int i, int N, int mn)
    {
        for (int k = 0; k < nb; ++k) idx[nl_off(np + k, i, N)] = idx[nl_off(mn - nb + k, i, N)];
        return (np + nb) | (np << 16);
    }
};

// Candidates [k0, k1) of one stencil cell against atom i, 32 at a time: first
// a hit mask with no branch per candidate, then one store per hit, in
// ascending record order.  The record kself (the atom itself) is never
// listed.  SHIFT adds the cell's periodic image shift to the difference,
// (x_j - x_i) + s, as the minimum image convention rounds it; its pairs go to
// the back of the row.  An entry is the record's byte offset, with the
// record's species (staged in its fourth slot) in the five low bits when
// `typed`.
__device__ __forceinline__ int row_entry(const double *rec, int k, bool typed)
{
    int e = k << 5;
    if (typed) e |= reinterpret_cast<const int *>(rec + 4 * (size_t)k + 3)[0];
    return e;
}

// Several species with cutoffs per pair of types: a hit within the box's
// list radius stays only within its own pair's, rl2row[type_j] (the atom's
// row of the (RCUT + skin)^2 table; null: no per-pair radius).
__device__ __forceinline__ bool pair_listed(const double *rec, int k, double r2, double rl2,
                                            const double *rl2row)
{
    if (!rl2row) return true;
    int tj = reinterpret_cast<const int *>(rec + 4 * (size_t)k + 3)[0];
    return r2 < fmin(rl2row[tj], rl2);
}

template <bool SHIFT>
__device__ __forceinline__ void list_cell(const double *rec, int k0, int k1, int kself,
                                          double xi, double yi, double zi, double sx, double sy,
                                          double sz, double rl2, const double *rl2row,
                                          int *__restrict__ idx, int i, int N, int mn, bool typed,
                                          RowFill &row)
{
#pragma clang fp contract(off)
    for (int c0 = k0; c0 < k1; c0 += 32) {
        const int m = min(32, k1 - c0);
        const double *r = rec + 4 * c0;
        unsigned mask = 0u;
#pragma unroll 2
        for (int q = 0; q < m; ++q, r += 4) {
            double dx = r[0] - xi, dy = r[1] - yi, dz = r[2] - zi;
            if constexpr (SHIFT) {
                dx = dx + sx;
                dy = dy + sy;
                dz = dz + sz;
            }
            mask |= (dist2(dx, dy, dz) < rl2 ? 1u : 0u) << q;
        }
        unsigned d = (unsigned)(kself - c0);
        if (d < 32u) mask &= ~(1u << d);
        while (mask) {
            int q = __ffs(mask) - 1;
            mask &= mask - 1u;
            if (rl2row) {
                const double *r = rec + 4 * (c0 + q);
                double dx = r[0] - xi, dy = r[1] - yi, dz = r[2] - zi;
                if constexpr (SHIFT) {
                    dx = dx + sx;
                    dy = dy + sy;
                    dz = dz + sz;
                }
                if (!pair_listed(rec, c0 + q, dist2(dx, dy, dz), rl2, rl2row)) continue;
            }
            ++row.total;
            row.put(idx, i, N, mn, !SHIFT, row_entry(rec, c0 + q, typed));
        }
    }
}

__global__ __launch_bounds__(kT) void k_tile_nlist(const unsigned *gate, int N, State st, Boxes bx,
                                                   Build bd, NList nl, int hmax,
                                                   const double *rl2p, int nt, unsigned *flags)
{
#pragma clang fp contract(off)
    if (skip(gate)) return;
    extern __shared__ __attribute__((aligned(256))) double rec[];
    __shared__ HaloLds H;
    Tile t;
    const int g = xcd_tile(blockIdx.x, gridDim.x, nullptr);
    tile_setup(bx, bd, g, t);
    halo_table(t, bx, bd, H);
    stage<false>(t, st, H, rec, hmax, flags, nl.tsrc + (size_t)g * hmax);
    if (threadIdx.x == 0) nl.ttotal[g] = H.total;
    const double L = t.L, invL = t.invL, rl2 = bx.rl2[t.b];
    const int mn = nl.mn, nc = t.nc;
    const double ncL = nc * invL;
    const bool typed = st.type != nullptr;
    unsigned bad = 0;
    int worst = 0;  // longest row of this thread's atoms
    for (int i = t.s0 + threadIdx.x; i < t.s1; i += kT) {
        double xi = st.x[i], yi = st.y[i], zi = st.z[i];
        int cx = cell_coord(xi, ncL, nc), cy = cell_coord(yi, ncL, nc), cz = cell_coord(zi, ncL, nc);
        const double *rl2row = rl2p ? rl2p + st.type[i] * nt : nullptr;
        RowFill row;
        if (t.mode == kTileA) {
            int lx = cx - t.ox, ly = cy - t.oy, lz = cz - t.oz;
            int hs = halo_index(t, lx, ly, lz);
            int kself = H.off[hs] + (i - H.start[hs]);
            // squared distance from the atom to the lower and upper faces of
            // its cell along each axis; a stencil cell whose box is farther
            // than the list radius cannot hold a neighbour (tested with a
            // relative margin so that rounding never drops a pair)
            double w = L / nc;
            double gx0 = xi - cx * w, gy0 = yi - cy * w, gz0 = zi - cz * w;
            double ex[3] = {gx0 * gx0, 0.0, (w - gx0) * (w - gx0)};
            double ey[3] = {gy0 * gy0, 0.0, (w - gy0) * (w - gy0)};
            double ez[3] = {gz0 * gz0, 0.0, (w - gz0) * (w - gz0)};
            double reach = rl2 * (1.0 + 1e-6);
            for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx_ = -1; dx_ <= 1; ++dx_) {
                        if (ex[dx_ + 1] + ey[dy + 1] + ez[dz + 1] > reach) continue;
                        int h = halo_index(t, lx + dx_, ly + dy, lz + dz);
                        int code = H.shift[h];
                        int k0 = H.off[h], k1 = min(H.off[h + 1], hmax);
                        if (code == kNoShift)
                            list_cell<false>(rec, k0, k1, kself, xi, yi, zi, 0.0, 0.0, 0.0, rl2,
                                             rl2row, nl.idx, i, N, mn, typed, row);
                        else
                            list_cell<true>(rec, k0, k1, -1, xi, yi, zi, shift_of(code, 0, L),
                                            shift_of(code, 1, L), shift_of(code, 2, L), rl2,
                                            rl2row, nl.idx, i, N, mn, typed, row);
                    }
        } else {
            int kself = H.off[(cz * nc + cy) * nc + cx] + (i - H.start[(cz * nc + cy) * nc + cx]);
            int ux[3], uy[3], uz[3];
            int kx = stencil_1d(cx, nc, ux), ky = stencil_1d(cy, nc, uy), kz = stencil_1d(cz, nc, uz);
            for (int a = 0; a < kz; ++a)
                for (int bb = 0; bb < ky; ++bb)
                    for (int c = 0; c < kx; ++c) {
                        int h = (uz[a] * nc + uy[bb]) * nc + ux[c];
                        int k0 = H.off[h], k1 = min(H.off[h + 1], hmax);
                        for (int k = k0; k < k1; ++k) {
                            if (k == kself) continue;
                            const double *r = rec + 4 * k;
                            double dx = r[0] - xi, dy2 = r[1] - yi, dz2 = r[2] - zi;
                            double kx_ = rint(dx * invL), ky_ = rint(dy2 * invL),
                                   kz_ = rint(dz2 * invL);
                            dx = dx - kx_ * L;
                            dy2 = dy2 - ky_ * L;
                            dz2 = dz2 - kz_ * L;
                            double r2 = dist2(dx, dy2, dz2);
                            if (r2 < rl2 && pair_listed(rec, k, r2, rl2, rl2row)) {
                                row.put(nl.idx, i, N, mn, kx_ == 0.0 && ky_ == 0.0 && kz_ == 0.0,
                                        row_entry(rec, k, typed));
                                ++row.total;
                            }
                        }
                    }
        }
        nl.count[i] = row.close(nl.idx, i, N, mn);
        nl.total[i] = row.total;
        worst = max(worst, row.total);
    }
    if (worst > mn) raise_overflow(flags, MD_FLAG_NLIST_OVERFLOW, worst);
    raise_flags(flags, bad);
}

// ---------------------------------------------------------------- passes

// Visit the n1 entries of the row of slot i (record byte offsets) four at a
// time, one 16-byte load per group: groups part, part + S, ... (S lanes share
// a row).  While one group is evaluated, the next is already in flight; the
// two registers alternate roles (the loop body is unrolled by two) so that no
// register copy at the back edge waits for a load.  The four records of a
// group are read from LDS together (entries past the end of the row read
// record 0 and are dropped), then each pair inside the cutoff goes to
// body(dx, dy, dz, r2, F'_j, type_j).  With IMG, entries from np on (pairs
// across a face of the box) take the minimum image.  WITH_FP reads F'_j.
template <bool IMG, bool TYPED, bool WITH_FP, int S, class Body>
__device__ __forceinline__ void for_row(const int *__restrict__ idx, int i, int N, int n1, int np,
                                        int part, const double *rec, double xi, double yi,
                                        double zi, double L, double invL, double rc2,
                                        const double *cut2row, Body &&body)
{
    if (n1 <= 0) return;
    const int4 *g = reinterpret_cast<const int4 *>(idx) + i;
    const int ng = (n1 + 3) >> 2;
    const char *base = reinterpret_cast<const char *>(rec);
    auto group = [&](const int4 &c, int q) {
        const int m = n1 - 4 * q, mp = np - 4 * q;
        const int kk[4] = {c.x, c.y, c.z, c.w};
        unsigned off[4];
        int tj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            unsigned o = (unsigned)kk[u];
            // entries past the end of the row are not this build's: record 0, species 0
            tj[u] = (TYPED && u < m) ? (int)(o & 31u) : 0;
            if constexpr (TYPED) o &= ~31u;
            off[u] = u < m ? o : 0u;
        }
        double2 A[4];
        double zj[4], fj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double2 *r = reinterpret_cast<const double2 *>(base + off[u]);
            A[u] = r[0];
            if constexpr (WITH_FP) {
                double2 B = r[1];
                zj[u] = B.x;
                fj[u] = B.y;
            } else {
                zj[u] = reinterpret_cast<const double *>(r + 1)[0];
                fj[u] = 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            double dx = A[u].x - xi, dy = A[u].y - yi, dz = zj[u] - zi;
            if (IMG && u >= mp) {
                dx = min_image(dx, L, invL);
                dy = min_image(dy, L, invL);
                dz = min_image(dz, L, invL);
            }
            const double r2 = dist2(dx, dy, dz);
            // several species with cutoffs per pair of types: RCUT(a, b)^2
            const double c2 = (TYPED && cut2row) ? cut2row[tj[u]] : rc2;
            if (u < m && r2 < c2) body(dx, dy, dz, r2, fj[u], tj[u]);
        }
    };
    // Every load is unconditional (past the end of the row it re-reads the
    // row's last group, already in cache): with a fixed number of loads per
    // iteration the wait before a group can leave the later load in flight.
    auto load = [&](int q) { return g[(size_t)min(q, ng - 1) * N]; };
    const int qa = S == 1 ? 0 : part;  // one lane per row: the loop counter stays uniform
    int4 a = load(qa);
    int4 b = load(qa + S);
    for (int q = qa; q < ng; q += 2 * S) {
        group(a, q);
        a = load(q + 2 * S);
        group(b, q + S);
        b = load(q + 3 * S);
    }
}

// The whole row of slot i.  The minimum image is compiled in only for the
// wavefronts that hold an atom with pairs across a face of the box.
template <bool TYPED, bool WITH_FP, int S, class Body>
__device__ __forceinline__ void for_row_all(const NList &nl, int i, int N, int part,
                                            const double *rec, double xi, double yi, double zi,
                                            double L, double invL, double rc2,
                                            const double *cut2row, Body &&body)
{
    const unsigned w = (unsigned)nl.count[i];
    const int n1 = (int)(w & 0xffffu), np = (int)(w >> 16);
    if (__any(np < n1))
        for_row<true, TYPED, WITH_FP, S>(nl.idx, i, N, n1, np, part, rec, xi, yi, zi, L, invL,
                                         rc2, cut2row, body);
    else
        for_row<false, TYPED, WITH_FP, S>(nl.idx, i, N, n1, np, part, rec, xi, yi, zi, L, invL,
                                          rc2, cut2row, body);
}

// The value of the lane that DPP control CTRL names (within a row of 16).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// Sum over the P lanes (1, 2, 4, 8 or 16, adjacent and aligned) that share
// the row of one atom, by a butterfly of DPP exchanges within a row of 16
// lanes: lane k with k ^ 1 (quad_perm [1, 0, 3, 2]), then with k ^ 2
// (quad_perm [2, 3, 0, 1]), then the two quads of each half row
// (row_half_mirror), then the two halves (row_mirror).  Each step adds two
// values that are equal across the lanes of each side, so every lane ends
// with the same sum, in the same order of additions.
template <int P>
__device__ __forceinline__ double lanes_sum(double v)
{
    static_assert(P == 1 || P == 2 || P == 4 || P == 8 || P == 16, "lanes per row");
    if constexpr (P >= 2) v += dpp_f64<0xB1>(v);
    if constexpr (P >= 4) v += dpp_f64<0x4E>(v);
    if constexpr (P >= 8) v += dpp_f64<0x141>(v);
    if constexpr (P >= 16) v += dpp_f64<0x140>(v);
    return v;
}

template <int V>
struct Lanes {
    static constexpr int value = V;
};

// The atoms of a tile, atom(lanes, slot, lane of the row): P lanes on each
// row (one, or two in systems of few tiles).  With one lane per row, a tile
// of n atoms, kT < n <= 1.5 kT, runs its first kT atoms one per thread and
// the surplus e = n - kT with S lanes on each row, S the largest of 16, 8, 4
// and 2 with e S <= kT: a second pass over the surplus atoms then costs every
// wavefront about 1/S of a row, where one lane per row would cost the
// wavefronts holding them a whole row while the others wait.  The analytic
// kinds take only S = 16 (e <= 64; more variants cost their kernels
// registers), larger surpluses one lane per row.  Only these rows are summed
// in another order (per lane, then across the S lanes), so results depend on
// the tiling in rounding only.
template <int KIND>
constexpr bool kAllSurplus = KIND == MD_POT_SPLINE || KIND == kTyped;

template <int P, bool ALL, class Atom>
__device__ __forceinline__ void tile_atoms(const Tile &t, Atom &&atom)
{
    const int n = t.s1 - t.s0, tid = (int)threadIdx.x;
    const int e = n - kT;
    if (P == 1 && e > 0 && (ALL ? 2 * e : 16 * e) <= kT) {
        atom(Lanes<1>{}, t.s0 + tid, 0);
        auto surplus = [&](auto lanes) {
            constexpr int S = decltype(lanes)::value;
            const int i = t.s0 + kT + tid / S;
            if (i < t.s1) atom(lanes, i, tid % S);
        };
        if (16 * e <= kT) {
            surplus(Lanes<16>{});
        } else if constexpr (ALL) {
            if (8 * e <= kT) surplus(Lanes<8>{});
            else if (4 * e <= kT) surplus(Lanes<4>{});
            else surplus(Lanes<2>{});
        }
        return;
    }
    for (int i = t.s0 + tid / P; i < t.s1; i += kT / P)
        atom(Lanes<P>{}, i, P == 1 ? 0 : tid % P);
}

// Tile m of persistent workgroup b (of P), or -1.  Workgroups are dispatched
// round robin over the 8 XCDs; the workgroups of one XCD sweep one contiguous
// eighth of the tiles together (in the sweep order of the tile table), so
// neighbouring tiles (which share halo cells) are staged through the same L2
// at about the same time.
__device__ __forceinline__ int tile_at(int b, int m, int P, int G, const int *order)
{
    if (P % 8 == 0) {
        int x = b % 8, Q = P / 8;
        int q = G / 8, r = G % 8;
        int lo = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q, hi = lo + q + (x < r);
        int g = lo + b / 8 + m * Q;
        return g < hi ? order[g] : -1;
    }
    int g = b + m * P;
    return g < G ? order[g] : -1;
}

// Persistent driver of the tiled passes: each workgroup takes its tiles in
// turn.  Each wave fetches its share of the next tile's halo (source list,
// then the gathers) as soon as its own rows of the current tile are done,
// while slower waves of the workgroup are still evaluating; after a barrier
// the records go to LDS.
template <bool WITH_FP, class Rows>
__device__ __forceinline__ void run_tiles(int G, const State &st, const Boxes &bx, const Build &bd,
                                          const NList &nl, double *rec, int hmax, Rows &&rows)
{
    constexpr int R = 5;  // records per thread: hmax <= R * 1024
    const int P = gridDim.x, tid = threadIdx.x;
    int m = 0;
    int g = tile_at(blockIdx.x, 0, P, G, bx.tile_order);
    if (g < 0) return;
    Tile t;
    tile_setup(bx, bd, g, t);
    stage_list<WITH_FP>(g, st, nl, rec, hmax);
    while (true) {
        const int gn = tile_at(blockIdx.x, m + 1, P, G, bx.tile_order);
        Tile tn = t;
        int totn = 0;
        if (gn >= 0) {
            tile_setup(bx, bd, gn, tn);
            totn = min(nl.ttotal[gn], hmax);
        }
        rows(t);
        const unsigned *src = nl.tsrc + (size_t)max(gn, 0) * hmax;
        unsigned e[R];
#pragma unroll
        for (int u = 0; u < R; ++u) e[u] = src[min(u * kT + tid, hmax - 1)];
        double px[R], py[R], pz[R], pf[R];
#pragma unroll
        for (int u = 0; u < R; ++u) {
            int k = u * kT + tid;
            if (k < totn) {
                int j = (int)e[u];
                px[u] = st.x[j];
                py[u] = st.y[j];
                pz[u] = st.z[j];
                if constexpr (WITH_FP) pf[u] = st.Fp[j];
            }
        }
        __syncthreads();
        if (gn < 0) break;
#pragma unroll
        for (int u = 0; u < R; ++u) {
            int k = u * kT + tid;
            if (k < totn) {
                double *r = rec + 4 * (size_t)k;
                r[0] = px[u];
                r[1] = py[u];
                r[2] = pz[u];
                if constexpr (WITH_FP) r[3] = pf[u];
            }
        }
        __syncthreads();
        t = tn;
        ++m;
    }
}

// P lanes per atom (1, or 2 for systems of few tiles): lane `part` takes
// the row groups part, part + P, ...; the sums are combined before the
// epilogue, which the first lane alone performs.
template <int KIND, int P>
__global__ __launch_bounds__(kT) void k_tile_density(int N, int G, State st, Boxes bx, Build bd,
                                                     NList nl, Pot pot_arg, int hmax,
                                                     unsigned *flags, int fp_only)
{
    extern __shared__ __attribute__((aligned(256))) double rec[];
    if (halted(flags)) return;
    const Pot pot = pinned(pot_arg);
    unsigned bad = 0;
    run_tiles<false>(G, st, bx, bd, nl, rec, hmax, [&](const Tile &t) {
        tile_atoms<P, kAllSurplus<KIND>>(t, [&](auto lanes, int i, int part) {
            constexpr int S = decltype(lanes)::value;
            double xi = st.x[i], yi = st.y[i], zi = st.z[i];
            double rho = 0.0;
            const int ai = KIND == kTyped ? st.type[i] : 0;
            auto body = [&](double, double, double, double r2, double, int tj) {
                if constexpr (KIND == kTyped)
                    rho += dens_typed(pot, r2 * rsqrt_nr(r2), ai, tj, bad);
                else
                    rho += dens<KIND>(pot, r2 * rsqrt_nr(r2), bad);
            };
            const double *cr = (KIND == kTyped && pot.cut2) ? pot.cut2 + ai * pot.nt : nullptr;
            for_row_all<KIND == kTyped, false, S>(nl, i, N, part, rec, xi, yi, zi, t.L, t.invL,
                                                  pot.rc2, cr, body);
            rho = lanes_sum<S>(rho);
            if (S > 1 && part != 0) return;
            double F, Fp;
            if constexpr (KIND == kTyped)
                embed_typed(pot, rho, ai, F, Fp, bad);
            else
                embed<KIND>(pot, rho, F, Fp, bad);
            // inside a sequence of steps only F' is read (by the force pass)
            st.Fp[i] = Fp;
            if (!fp_only) {
                st.rho[i] = rho;
                st.Femb[i] = F;
            }
        });
    });
    raise_flags(flags, bad);
}

// MODE 0: forces only; 1: forces and the half kick v += kick f; 2: also the
// next step's half kick and drift, x' = x + dt (v + kick f) into the other
// position buffer, with the rebuild test of the kick-drift kernel.
template <int KIND, bool ENERGY, int MODE, int P>
__global__ __launch_bounds__(kT) void k_tile_force(int N, int G, State st, Boxes bx, Build bd,
                                                   NList nl, Pot pot_arg, int hmax, double kick,
                                                   double dt, Thermo th, unsigned *flags)
{
    extern __shared__ __attribute__((aligned(256))) double rec[];
    if (halted(flags)) return;
    const Pot pot = pinned(pot_arg);
    // without the energy, SMTB accumulates the negated force (see pair_coef)
    constexpr double sg = ENERGY ? 1.0 : kForceSign<KIND>;
    unsigned bad = 0;
    bool need = false;
    // one workgroup per tile (with the persistent driver the fused variant
    // needs more registers than it gains)
    {
        const int g = xcd_tile(blockIdx.x, gridDim.x, bx.tile_order);
        Tile t;
        tile_setup(bx, bd, g, t);
        stage_list<true>(g, st, nl, rec, hmax);
        const double thr2 = bx.thr2[t.b];
        tile_atoms<P, kAllSurplus<KIND>>(t, [&](auto lanes, int i, int part) {
            constexpr int S = decltype(lanes)::value;
            double xi = st.x[i], yi = st.y[i], zi = st.z[i];
            double fpi = st.Fp[i];
            // the epilogue's inputs are loaded before the row, so their
            // latency hides behind it
            double v0x = 0.0, v0y = 0.0, v0z = 0.0, rx = 0.0, ry = 0.0, rz = 0.0;
            if constexpr (MODE >= 1) {
                v0x = st.vx[i];
                v0y = st.vy[i];
                v0z = st.vz[i];
            }
            if constexpr (MODE == 2) {
                rx = st.xr[i];
                ry = st.yr[i];
                rz = st.zr[i];
            }
            double ax = 0.0, ay = 0.0, az = 0.0, ep = 0.0, wv = 0.0;
            const int ai = KIND == kTyped ? st.type[i] : 0;
            auto body = [&](double dx, double dy, double dz, double r2, double fpj, int tj) {
                {
                    double inv_r = rsqrt_nr(r2);
                    // f_i += [(F'_i + F'_j) rho'(r) + V'(r)] (x_j - x_i) / r; with
                    // several species [F'_i rho^(ab)'(r) + F'_j rho^(ba)'(r) + V^(ab)'(r)]
                    double coef;
                    if constexpr (KIND == kTyped) {
                        double dab, dba, v, dv;
                        if constexpr (ENERGY)
                            pair_terms_typed(pot, r2 * inv_r, ai, tj, dab, dba, v, dv, bad);
                        else
                            pair_derivs_typed(pot, r2 * inv_r, ai, tj, dab, dba, dv, bad);
                        coef = fma(fpi, dab, fma(fpj, dba, dv)) * inv_r;
                        if constexpr (ENERGY) {
                            ep += v;
                            wv = fma(coef, r2, wv);
                        }
                    } else if constexpr (ENERGY) {
                        double dfr, v, dv;
                        pair_terms<KIND>(pot, r2 * inv_r, dfr, v, dv, bad);
                        coef = fma(fpi + fpj, dfr, dv) * inv_r;
                        ep += v;
                        wv = fma(coef, r2, wv);  // virial term [(F'_i + F'_j) rho' + V'] r
                    } else {
                        coef = pair_coef<KIND>(pot, r2 * inv_r, fpi + fpj, bad) * inv_r;
                    }
                    ax = fma(coef, dx, ax);
                    ay = fma(coef, dy, ay);
                    az = fma(coef, dz, az);
                }
            };
            const double *cr = (KIND == kTyped && pot.cut2) ? pot.cut2 + ai * pot.nt : nullptr;
            for_row_all<KIND == kTyped, true, S>(nl, i, N, part, rec, xi, yi, zi, t.L, t.invL,
                                                 pot.rc2, cr, body);
            ax = lanes_sum<S>(ax);
            ay = lanes_sum<S>(ay);
            az = lanes_sum<S>(az);
            if constexpr (ENERGY) {
                ep = lanes_sum<S>(ep);
                wv = lanes_sum<S>(wv);
            }
            if (S > 1 && part != 0) return;
            ax *= sg;
            ay *= sg;
            az *= sg;
            // with the next kick fused (MODE 2) the forces go straight into
            // the velocities: the next force pass overwrites them before any
            // kernel reads them (a sequence of steps ends with an unfused one)
            if constexpr (MODE != 2) {
                st.fx[i] = ax;
                st.fy[i] = ay;
                st.fz[i] = az;
            }
            if constexpr (ENERGY) {
                st.eat[i] = fma(0.5, ep, st.Femb[i]);
                st.wat[i] = wv;
            }
            if constexpr (MODE >= 1) {
                double ki = kick;
                Thermo thi = th;
                species_kick(st, i, ki, thi);
                double vx = fma(ki, ax, v0x);
                double vy = fma(ki, ay, v0y);
                double vz = fma(ki, az, v0z);
                if (thi.on) friction_flow(thi, vx, vy, vz);
                hold(st, i, vx, vy, vz);
                if constexpr (MODE == 2) {
                    if (thi.on) friction_flow(thi, vx, vy, vz);
                    vx = fma(ki, ax, vx);
                    vy = fma(ki, ay, vy);
                    vz = fma(ki, az, vz);
                    hold(st, i, vx, vy, vz);
                    double x = fma(dt, vx, xi), y = fma(dt, vy, yi), z = fma(dt, vz, zi);
                    st.xo[i] = x;
                    st.yo[i] = y;
                    st.zo[i] = z;
                    double ddx = x - rx, ddy = y - ry, ddz = z - rz;
                    double d2 = fma(ddz, ddz, fma(ddy, ddy, ddx * ddx));
                    need = need || d2 > thr2;
                    if (!isfinite(d2)) bad |= MD_FLAG_NONFINITE;
                }
                st.vx[i] = vx;
                st.vy[i] = vy;
                st.vz[i] = vz;
            }
        });
    }
    if constexpr (MODE == 2) {
        // one request per wavefront, and none once the flag is already raised
        if (__any(need) && (threadIdx.x & 63) == 0 &&
            __atomic_load_n(flags + 1, __ATOMIC_RELAXED) == 0u)
            atomicOr(flags + 1, 1u);
    }
    raise_flags(flags, bad);
}

// Rows in original indices: LDS index -> halo cell (binary search) -> slot.
__global__ __launch_bounds__(kT) void k_tile_get_neighbors(int N, State st, Boxes bx, Build bd,
                                                           NList nl, int32_t *counts, int32_t *ids,
                                                           int cols)
{
    __shared__ HaloLds H;
    Tile t;
    tile_setup(bx, bd, blockIdx.x, t);
    halo_table(t, bx, bd, H);
    for (int i = t.s0 + threadIdx.x; i < t.s1; i += kT) {
        int o = st.id[i];
        counts[o] = nl.total[i];
        int m = min(min(nl.count[i] & 0xffff, nl.mn), cols);
        for (int q = 0; q < m; ++q) {
            int k = nl.idx[nl_off(q, i, N)] >> 5;
            int lo = 0, hi = t.nh - 1;
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (H.off[mid] <= k) lo = mid;
                else hi = mid - 1;
            }
            int j = H.start[lo] + (k - H.off[lo]);
            ids[(size_t)o * cols + q] = st.id[j];
        }
    }
}

template <int KIND, int P>
void force_launch(Ctx &c, bool energy, int mode, double k, hipStream_t s)
{
    const int N = (int)c.N, G = c.ntiles;
    size_t lds = c.tile_lds;
    double dt = c.dt;
#define MDK_FORCE(E, M) \
    k_tile_force<KIND, E, M, P><<<G, kT, lds, s>>>(N, G, c.st, c.bx, c.bd, c.nl, c.pot, c.hmax, k, dt, c.thermo, c.dev.flags)
    if (energy && mode > 0)
        MDK_FORCE(true, 1);
    else if (energy)
        MDK_FORCE(true, 0);
    else if (mode == 2)
        MDK_FORCE(false, 2);
    else if (mode == 1)
        MDK_FORCE(false, 1);
    else
        MDK_FORCE(false, 0);
#undef MDK_FORCE
}

template <class F>
void allow(F *f, size_t lds)
{
    (void)hipFuncSetAttribute((const void *)f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

}  // namespace

static constexpr double kKappaT = 1.602176634e-19 / 1.66053906660e-27 * 1e-10;

template <int KIND, int P>
static void allow_kind(size_t lds)
{
    allow(k_tile_density<KIND, P>, lds);
    allow(k_tile_force<KIND, true, 1, P>, lds);
    allow(k_tile_force<KIND, true, 0, P>, lds);
    allow(k_tile_force<KIND, false, 1, P>, lds);
    allow(k_tile_force<KIND, false, 0, P>, lds);
    allow(k_tile_force<KIND, false, 2, P>, lds);
}

template <int P>
static void allow_passes(size_t lds)
{
    allow_kind<MD_POT_FS, P>(lds);
    allow_kind<MD_POT_SMTB, P>(lds);
    allow_kind<MD_POT_SPLINE, P>(lds);
    allow_kind<kTyped, P>(lds);
}

void tiled_prepare(Ctx &c)
{
    size_t lds = c.tile_lds;
    // persistent grid of the density pass: as many workgroups as can be resident
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_tile_density<MD_POT_SMTB, 1>, kT,
                                                     lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c.device) != hipSuccess ||
        cus < 1)
        cus = 1;
    c.tile_grid = std::max(1, std::min(c.ntiles, per_cu * cus));
    allow(k_tile_nlist, lds);
    allow_passes<1>(lds);
    allow_passes<2>(lds);
}

void launch_tile_nlist(Ctx &c, const unsigned *gate, hipStream_t s)
{
    const double *rl2p = c.pot.cut2 ? c.pot.cut2 + (size_t)c.pot.nt * c.pot.nt : nullptr;
    k_tile_nlist<<<c.ntiles, kT, c.tile_lds, s>>>(gate, (int)c.N, c.st, c.bx, c.bd, c.nl, c.hmax,
                                                  rl2p, c.pot.nt, c.dev.flags);
}

template <int L>
static void tile_density_lanes(Ctx &c, hipStream_t s, int fp_only)
{
    const int N = (int)c.N, P = c.tile_grid, G = c.ntiles;
    switch (c.pot.kind) {
    case MD_POT_FS: k_tile_density<MD_POT_FS, L><<<P, kT, c.tile_lds, s>>>(N, G, c.st, c.bx, c.bd, c.nl, c.pot, c.hmax, c.dev.flags, fp_only); break;
    case MD_POT_SMTB: k_tile_density<MD_POT_SMTB, L><<<P, kT, c.tile_lds, s>>>(N, G, c.st, c.bx, c.bd, c.nl, c.pot, c.hmax, c.dev.flags, fp_only); break;
    case kTyped: k_tile_density<kTyped, L><<<P, kT, c.tile_lds, s>>>(N, G, c.st, c.bx, c.bd, c.nl, c.pot, c.hmax, c.dev.flags, fp_only); break;
    default: k_tile_density<MD_POT_SPLINE, L><<<P, kT, c.tile_lds, s>>>(N, G, c.st, c.bx, c.bd, c.nl, c.pot, c.hmax, c.dev.flags, fp_only); break;
    }
}

void launch_tile_density(Ctx &c, hipStream_t s, bool fp_only)
{
    if (c.tile_lanes == 2) tile_density_lanes<2>(c, s, fp_only);
    else tile_density_lanes<1>(c, s, fp_only);
}

template <int L>
static void tile_force_lanes(Ctx &c, bool energy, int mode, hipStream_t s)
{
    double k = 0.5 * c.dt * kKappaT / c.mass;
    switch (c.pot.kind) {
    case MD_POT_FS: force_launch<MD_POT_FS, L>(c, energy, mode, k, s); break;
    case MD_POT_SMTB: force_launch<MD_POT_SMTB, L>(c, energy, mode, k, s); break;
    case kTyped: force_launch<kTyped, L>(c, energy, mode, k, s); break;
    default: force_launch<MD_POT_SPLINE, L>(c, energy, mode, k, s); break;
    }
}

void launch_tile_force(Ctx &c, bool energy, int mode, hipStream_t s)
{
    if (c.tile_lanes == 2) tile_force_lanes<2>(c, energy, mode, s);
    else tile_force_lanes<1>(c, energy, mode, s);
}

void launch_tile_get_neighbors(Ctx &c, int32_t *counts, int32_t *ids, int32_t cols, hipStream_t s)
{
    k_tile_get_neighbors<<<c.ntiles, kT, 0, s>>>((int)c.N, c.st, c.bx, c.bd, c.nl, counts, ids, cols);
}

}  // namespace mdk
