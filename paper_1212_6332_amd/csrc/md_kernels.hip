// Per-atom kernels of the many-body MD force path on gfx950 (CDNA4).
//
// Layout: every per-atom array is structure-of-arrays FP64 in cell-sorted
// order, so that a 64-lane wavefront reads 64 consecutive atoms (coalesced)
// and the neighbours of those atoms lie in a few nearby cells (cache
// friendly gathers).  The neighbour list is stored slot-fastest in groups
// of four entries (entry n of slot i at ((n / 4) N + i) 4 + n % 4), so one
// 16-byte load returns four neighbours of an atom and 64 consecutive atoms
// read 1 KiB contiguously.  Lists are full (each pair stored twice): the
// force on atom i is gathered by the thread of atom i alone, with no
// scatter and no floating-point atomics, which makes every pass
// deterministic.
//
// Passes follow Hou et al.: density (Fig. 5) with the embedding of
// Section 4 fused into its epilogue, then force (Fig. 6, eq. 3), with the
// cutoff re-checked for every listed pair (the list radius exceeds rc by
// the skin).  Binning and the counting sort replace the host-side linked
// lists and sort of Section 3.2; the list build scans the (deduplicated)
// 27-cell stencil of Fig. 3.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "md_device.h"
#include "md_internal.h"

namespace mdk {

namespace {

using namespace dev;

constexpr int kXcds = 8;

// Workgroups are dispatched to the 8 XCDs round robin.  Renumber them so
// that each XCD works on one contiguous eighth of the (cell-sorted) atoms;
// the neighbour gathers of a workgroup then mostly hit its own XCD's L2.
__device__ __forceinline__ int xcd_block(int b, int G)
{
    int q = G / kXcds, r = G % kXcds, k = b % kXcds, w = b / kXcds;
    return (k < r) ? k * (q + 1) + w : r * (q + 1) + (k - r) * q + w;
}

__device__ __forceinline__ int atom_index()
{
    return xcd_block((int)blockIdx.x, (int)gridDim.x) * (int)blockDim.x + (int)threadIdx.x;
}

// Gather with a 32-bit byte offset from a uniform base pointer (the compiler
// then issues scalar-base global loads; atom counts stay below 2^29).
__device__ __forceinline__ double ldg(const double *__restrict__ base, unsigned j)
{
    return *reinterpret_cast<const double *>(reinterpret_cast<const char *>(base) + (j << 3));
}

// Packed neighbour record j: (x, y) and (z, F') as two 16-byte loads from
// one 32-byte record (one cache line), 32-bit byte offsets (N < 2^27).
__device__ __forceinline__ double2 ldpk(const double *__restrict__ pk, unsigned j, unsigned half)
{
    return *reinterpret_cast<const double2 *>(reinterpret_cast<const char *>(pk) + (j << 5) +
                                              (half << 4));
}

__device__ __forceinline__ double ldpk_z(const double *__restrict__ pk, unsigned j)
{
    return *reinterpret_cast<const double *>(reinterpret_cast<const char *>(pk) + (j << 5) + 16);
}

// Neighbour row of slot i: `np` pairs that need no periodic correction at
// rows [0, np), `ni` pairs that cross the box boundary at rows [mn - ni, mn).
struct Row {
    int np, ni;
};

__device__ __forceinline__ Row row_of(const NList &nl, int i)
{
    unsigned w = (unsigned)nl.count[i];
    return Row{(int)(w & 0xffffu), (int)(w >> 16)};
}

// Visit rows n0, n0 + S, ... below n1 of the column of slot i.  Software
// pipelined: while pair n is evaluated, the record of pair n+S and the index
// of pair n+2S are already in flight.  Each pair costs one coalesced index
// load and two 16-byte loads from one 32-byte record.
template <bool IMG, bool FPJ, int S = 1, class Body>
__device__ __forceinline__ void for_pairs(const int *__restrict__ idx, int i, int N, int n0, int n1,
                                          const double *__restrict__ pk, double xi, double yi,
                                          double zi, double L, double invL, Body &&body)
{
    if (n0 >= n1) return;
    unsigned j = (unsigned)idx[nl_off(n0, i, N)];
    unsigned jn = (n0 + S < n1) ? (unsigned)idx[nl_off(n0 + S, i, N)] : j;
    double2 a = ldpk(pk, j, 0);
    double2 b;
    if constexpr (FPJ) b = ldpk(pk, j, 1);
    else b.x = ldpk_z(pk, j);
    unsigned jc = j;
    for (int n = n0; n < n1; n += S) {
        unsigned jnn = (n + 2 * S < n1) ? (unsigned)idx[nl_off(n + 2 * S, i, N)] : jn;
        double2 an = ldpk(pk, jn, 0);
        double2 bn;
        if constexpr (FPJ) bn = ldpk(pk, jn, 1);
        else bn.x = ldpk_z(pk, jn);
        double dx = a.x - xi, dy = a.y - yi, dz = b.x - zi;
        if constexpr (IMG) {
            dx = min_image(dx, L, invL);
            dy = min_image(dy, L, invL);
            dz = min_image(dz, L, invL);
        }
        body(dx, dy, dz, FPJ ? b.y : 0.0, jc);
        jc = jn;
        jn = jnn;
        a = an;
        b = bn;
    }
}

// P lanes share the row of one atom (P a power of two dividing 64, lanes of
// an atom adjacent): lane `part` takes the rows congruent to part modulo P,
// which keeps the four-entry groups of the list layout coalesced.
template <int P>
struct RowLanes {
    int i, part;
    __device__ __forceinline__ RowLanes(int t) : i(t / P), part(t % P) {}
    // first row of this lane at or above n
    __device__ __forceinline__ int first(int n) const { return n + ((part - n) & (P - 1)); }
};

// Sum over the P lanes of an atom by a fixed butterfly: every lane ends
// with the same value, whatever the lane.
template <int P>
__device__ __forceinline__ double lanes_sum(double v)
{
    for (int o = 1; o < P; o <<= 1) v += __shfl_xor(v, o);
    return v;
}

template <bool MULTI>
__device__ __forceinline__ void box_geom(const Boxes &bx, int i, double L1, double invL1,
                                         double &L, double &invL)
{
    if constexpr (MULTI) {
        int b = bx.box_of[i];
        L = bx.L[b];
        invL = bx.invL[b];
    } else {
        L = L1;
        invL = invL1;
    }
}

// ---------------------------------------------------------------- state I/O

__global__ void k_set_state(int N, const double *__restrict__ pos, const double *__restrict__ vel,
                            State st)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    st.x[i] = pos[3 * (size_t)i];
    st.y[i] = pos[3 * (size_t)i + 1];
    st.z[i] = pos[3 * (size_t)i + 2];
    st.vx[i] = vel ? vel[3 * (size_t)i] : 0.0;
    st.vy[i] = vel ? vel[3 * (size_t)i + 1] : 0.0;
    st.vz[i] = vel ? vel[3 * (size_t)i + 2] : 0.0;
    st.id[i] = i;
    if (st.type) st.type[i] = st.type0[i];
    if (st.frozen) {
        st.frozen[i] = st.frozen0[i];
        if (st.frozen0[i]) st.vx[i] = st.vy[i] = st.vz[i] = 0.0;
    }
}

// Frozen flag of every slot from its original id; frozen atoms stop.
__global__ void k_refresh_frozen(int N, State st)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    unsigned char f = st.frozen0[st.id[i]];
    st.frozen[i] = f;
    if (f) st.vx[i] = st.vy[i] = st.vz[i] = 0.0;
}

// Species of every slot from its original id.
__global__ void k_refresh_types(int N, State st)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    st.type[i] = st.type0[st.id[i]];
}

__global__ void k_get_state(int N, State st, double *__restrict__ pos, double *__restrict__ vel)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    size_t o = 3 * (size_t)st.id[i];
    if (pos) {
        pos[o] = st.x[i];
        pos[o + 1] = st.y[i];
        pos[o + 2] = st.z[i];
    }
    if (vel) {
        vel[o] = st.vx[i];
        vel[o + 1] = st.vy[i];
        vel[o + 2] = st.vz[i];
    }
}

__global__ void k_scatter_scalar(int N, const int *__restrict__ id, const double *__restrict__ src,
                                 double *__restrict__ dst)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) dst[id[i]] = src[i];
}

__global__ void k_scatter_vec3(int N, const int *__restrict__ id, const double *__restrict__ sx,
                               const double *__restrict__ sy, const double *__restrict__ sz,
                               double *__restrict__ dst)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    size_t o = 3 * (size_t)id[i];
    dst[o] = sx[i];
    dst[o + 1] = sy[i];
    dst[o + 2] = sz[i];
}

__global__ void k_pack_positions(int N, State st)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    reinterpret_cast<double2 *>(st.pk)[2 * (size_t)i] = make_double2(st.x[i], st.y[i]);
    st.pk[4 * (size_t)i + 2] = st.z[i];
}

__global__ void k_fill_u32(unsigned *p, int n, unsigned v)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------- list build

// Binning: wrap into the box, find the cell (numbered tile by tile),
// count atoms per cell.  Consecutive slots mostly share a cell (the state is
// sorted from the previous build), so each run of equal cells in a
// wavefront takes its slots with one atomic add.
__global__ __launch_bounds__(kBlock) void k_bin(const unsigned *gate, int N, State st, Boxes bx,
                                                Build bd, unsigned *flags)
{
    if (skip(gate)) return;
    // grid-stride over blocks of atoms (a capped grid keeps the launch cheap
    // in steps that skip the build); whole blocks iterate together, so the
    // wavefront ballots below always see consecutive atoms
    for (int b0 = blockIdx.x * blockDim.x; b0 < N; b0 += gridDim.x * blockDim.x) {
    int i = b0 + threadIdx.x;
    bool valid = i < N;
    int cell = -1;
    if (valid) {
        int b = bx.box_of[i];
        double L = bx.L[b];
        int nc = bx.nc[b];
        double x = st.x[i], y = st.y[i], z = st.z[i];
        if (!(isfinite(x) && isfinite(y) && isfinite(z))) {
            atomicOr(flags, (unsigned)MD_FLAG_NONFINITE);
            x = y = z = 0.0;
        }
        x = wrap1(x, L);
        y = wrap1(y, L);
        z = wrap1(z, L);
        st.x[i] = x;
        st.y[i] = y;
        st.z[i] = z;
        double ncL = nc * bx.invL[b];
        cell = cell_id(bx, b, cell_coord(x, ncL, nc), cell_coord(y, ncL, nc),
                       cell_coord(z, ncL, nc));
        bd.cell_of[i] = cell;
    }
    int lane = threadIdx.x & 63;
    int prev = __shfl_up(cell, 1);
    bool head = valid && (lane == 0 || prev != cell);
    unsigned long long heads = __ballot(head);
    unsigned long long nvalid = __popcll(__ballot(valid));
    unsigned long long upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
    unsigned long long below = heads & upto;
    int leader = below ? 63 - __clzll(below) : 0;
    unsigned long long after = heads & ~upto;
    int end = after ? __ffsll(after) - 1 : 64;
    if (end > (int)nvalid) end = (int)nvalid;
    int base = 0;
    if (head) base = atomicAdd(&bd.cell_count[cell], end - lane);
    base = __shfl(base, leader);
    if (valid) bd.slot[i] = base + (lane - leader);
    }
}

// Exclusive scan of the per-cell counts in two passes: per-block scans of
// kScanCells cells, then the offsets of the earlier blocks added.
constexpr int kScanCells = 4096;  // cells per scan block (1024 threads x 4)

// Exclusive scan of one value per thread over a 1024-thread block; returns
// the block total in *total.
__device__ __forceinline__ int block_scan_1024(int v, int *total)
{
    __shared__ int wsum[16];
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int incl = v;
    for (int off = 1; off < 64; off <<= 1) {
        int u = __shfl_up(incl, off);
        if (lane >= off) incl += u;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int k = 0; k < 16; ++k) {
            int t = wsum[k];
            wsum[k] = run;
            run += t;
        }
        *total = run;
    }
    __syncthreads();
    return wsum[w] + incl - v;
}

// The counts are cleared once read, so that the next build starts from zero
// (they are zero at creation) without a clearing pass of its own.
__global__ __launch_bounds__(1024) void k_scan_local(const unsigned *gate, int C,
                                                     int *__restrict__ cnt,
                                                     int *__restrict__ start, int *__restrict__ bsum)
{
    if (skip(gate)) return;
    __shared__ int tot;
    int c0 = blockIdx.x * kScanCells + threadIdx.x * 4;
    int v[4], s = 0;
    for (int k = 0; k < 4; ++k) {
        v[k] = (c0 + k < C) ? cnt[c0 + k] : 0;
        if (c0 + k < C) cnt[c0 + k] = 0;
        s += v[k];
    }
    int run = block_scan_1024(s, &tot);
    for (int k = 0; k < 4; ++k) {
        if (c0 + k < C) start[c0 + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Each workgroup adds the totals of the scan blocks before its own cells
// (a kBlock-cell workgroup lies inside one scan block), summed by its first
// wavefront; the last workgroup also writes the grand total at start[C].
__global__ __launch_bounds__(kBlock) void k_scan_add(const unsigned *gate, int C, int nb,
                                                     int *__restrict__ start,
                                                     const int *__restrict__ bsum)
{
    if (skip(gate)) return;
    __shared__ int off;
    const int c0 = blockIdx.x * blockDim.x, c = c0 + threadIdx.x;
    if (threadIdx.x < 64) {
        const int j = c0 / kScanCells;
        const bool last = blockIdx.x == gridDim.x - 1;
        int before = 0, all = 0;
        for (int k = threadIdx.x; k < nb; k += 64) {
            int v = bsum[k];
            if (k < j) before += v;
            all += v;
        }
        for (int o = 32; o > 0; o >>= 1) {
            before += __shfl_xor(before, o);
            all += __shfl_xor(all, o);
        }
        if (threadIdx.x == 0) {
            off = before;
            if (last) start[C] = all;
        }
    }
    __syncthreads();
    if (c < C) start[c] += off;
}

// Counting sort, first half: place every atom in its cell's segment (order inside a
// cell is not yet deterministic).
__global__ void k_scatter(const unsigned *gate, int N, Build bd)
{
    if (skip(gate)) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x)
        bd.tmp[bd.cell_start[bd.cell_of[i]] + bd.slot[i]] = i;
}

// Counting sort, second half: order each cell by original index.  The rank of an atom
// is the number of atoms of its cell with a smaller original index.
__global__ void k_rank(const unsigned *gate, int N, State st, Build bd)
{
    if (skip(gate)) return;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < N; q += gridDim.x * blockDim.x) {
        int p = bd.tmp[q];
        int c = bd.cell_of[p];
        int s = bd.cell_start[c], e = bd.cell_start[c + 1];
        int mine = st.id[p];
        int rank = 0;
        for (int k = s; k < e; ++k) rank += st.id[bd.tmp[k]] < mine;
        bd.perm[s + rank] = p;
    }
}

__global__ void k_gather(const unsigned *gate, int N, State st, Build bd)
{
    if (skip(gate)) return;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < N; q += gridDim.x * blockDim.x) {
        int p = bd.perm[q];
        bd.sx[q] = st.x[p];
        bd.sy[q] = st.y[p];
        bd.sz[q] = st.z[p];
        bd.svx[q] = st.vx[p];
        bd.svy[q] = st.vy[p];
        bd.svz[q] = st.vz[p];
        bd.sid[q] = st.id[p];
    }
}

__global__ void k_commit(const unsigned *gate, int N, State st, Build bd)
{
    if (skip(gate)) return;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < N; q += gridDim.x * blockDim.x) {
        double x = bd.sx[q], y = bd.sy[q], z = bd.sz[q];
        st.x[q] = x;
        st.y[q] = y;
        st.z[q] = z;
        reinterpret_cast<double2 *>(st.pk)[2 * (size_t)q] = make_double2(x, y);
        st.pk[4 * (size_t)q + 2] = z;
        st.xr[q] = x;
        st.yr[q] = y;
        st.zr[q] = z;
        st.vx[q] = bd.svx[q];
        st.vy[q] = bd.svy[q];
        st.vz[q] = bd.svz[q];
        st.id[q] = bd.sid[q];
        if (st.type) st.type[q] = st.type0[bd.sid[q]];
        if (st.frozen) st.frozen[q] = st.frozen0[bd.sid[q]];
    }
}

// Full list of slot i.  r^2 = (dx*dx + dy*dy) + dz*dz with separate
// roundings (no contraction) so that membership is reproducible exactly; the
// periodic correction is one exact addition of +-L, as in the minimum image.
// With three or more cells per axis the correction is known per stencil cell;
// with one or two cells every cell is in the stencil and the minimum image is
// taken per pair.  Pairs without correction go to the front of the row, the
// others to its back.
__global__ __launch_bounds__(kBlock) void k_nlist(const unsigned *gate, int N, State st, Boxes bx,
                                                  Build bd, NList nl, const double *rl2p, int nt,
                                                  unsigned *flags)
{
#pragma clang fp contract(off)
    if (skip(gate)) return;
    int i = atom_index();
    if (i >= N) return;
    int b = bx.box_of[i];
    double L = bx.L[b], invL = bx.invL[b], rl2 = bx.rl2[b];
    int nc = bx.nc[b], coff = bx.cell_off[b];
    const double *__restrict__ X = st.x;
    const double *__restrict__ Y = st.y;
    const double *__restrict__ Z = st.z;
    double xi = X[i], yi = Y[i], zi = Z[i];
    double ncL = nc * invL;
    int cx = cell_coord(xi, ncL, nc), cy = cell_coord(yi, ncL, nc), cz = cell_coord(zi, ncL, nc);
    const int mn = nl.mn;
    int np = 0, ni = 0, total = 0;
    // several species with cutoffs per pair of types: the pair's own list
    // radius, (RCUT + skin)^2 (never above the box's)
    const double *rl2row = rl2p ? rl2p + st.type[i] * nt : nullptr;
    auto listed = [&](int j, double r2) {
        return !rl2row || r2 < fmin(rl2row[st.type[j]], rl2);
    };
    auto add = [&](int j, bool plain) {
        if (np + ni < mn) {
            if (plain)
                nl.idx[nl_off(np++, i, N)] = j;
            else
                nl.idx[nl_off(mn - 1 - (ni++), i, N)] = j;
        }
        ++total;
    };
    if (nc >= 3) {
        // the 27 cells in ascending cell order: rows come out ascending in
        // the neighbour's slot, so the lanes of a wavefront gather nearby
        // records at the same row
        int ux[3], uy[3], uz[3];
        double hx[3], hy[3], hz[3];
        stencil_shift(cx, nc, L, ux, hx);
        stencil_shift(cy, nc, L, uy, hy);
        stencil_shift(cz, nc, L, uz, hz);
        int key[27];
        for (int a = 0; a < 3; ++a)
            for (int bb = 0; bb < 3; ++bb)
                for (int c = 0; c < 3; ++c)
                    key[(a * 3 + bb) * 3 + c] = ((cell_id(bx, b, ux[c], uy[bb], uz[a]) - coff) << 5) |
                                                ((a * 3 + bb) * 3 + c);
        for (int k = 1; k < 27; ++k) {
            int v = key[k], m = k - 1;
            while (m >= 0 && key[m] > v) {
                key[m + 1] = key[m];
                --m;
            }
            key[m + 1] = v;
        }
        for (int k = 0; k < 27; ++k) {
            int t = key[k] & 31;
            int a = t / 9, bb = (t / 3) % 3, c = t % 3;
            int cell = coff + (key[k] >> 5);
            int s = bd.cell_start[cell], e = bd.cell_start[cell + 1];
            double sx = hx[c], sy = hy[bb], sz = hz[a];
            if (sx == 0.0 && sy == 0.0 && sz == 0.0) {
                for (int j = s; j < e; ++j) {
                    double2 p2 = ldpk(st.pk, (unsigned)j, 0);
                    double dx = p2.x - xi;
                    double dy = p2.y - yi;
                    double dz = ldpk_z(st.pk, (unsigned)j) - zi;
                    double r2 = (dx * dx + dy * dy) + dz * dz;
                    if (r2 < rl2 && j != i && listed(j, r2)) add(j, true);
                }
            } else {
                for (int j = s; j < e; ++j) {
                    double2 p2 = ldpk(st.pk, (unsigned)j, 0);
                    double dx = (p2.x - xi) + sx;
                    double dy = (p2.y - yi) + sy;
                    double dz = (ldpk_z(st.pk, (unsigned)j) - zi) + sz;
                    double r2 = (dx * dx + dy * dy) + dz * dz;
                    if (r2 < rl2 && listed(j, r2)) add(j, false);
                }
            }
        }
    } else {
        int ux[3], uy[3], uz[3];
        int kx = stencil_1d(cx, nc, ux), ky = stencil_1d(cy, nc, uy), kz = stencil_1d(cz, nc, uz);
        for (int a = 0; a < kz; ++a)
            for (int bb = 0; bb < ky; ++bb)
                for (int c = 0; c < kx; ++c) {
                    int cell = cell_id(bx, b, ux[c], uy[bb], uz[a]);
                    int s = bd.cell_start[cell], e = bd.cell_start[cell + 1];
                    for (int j = s; j < e; ++j) {
                        if (j == i) continue;
                        double2 p2 = ldpk(st.pk, (unsigned)j, 0);
                        double dx = p2.x - xi;
                        double dy = p2.y - yi;
                        double dz = ldpk_z(st.pk, (unsigned)j) - zi;
                        double kx_ = rint(dx * invL), ky_ = rint(dy * invL), kz_ = rint(dz * invL);
                        dx = dx - kx_ * L;
                        dy = dy - ky_ * L;
                        dz = dz - kz_ * L;
                        double r2 = (dx * dx + dy * dy) + dz * dz;
                        if (r2 < rl2 && listed(j, r2))
                            add(j, kx_ == 0.0 && ky_ == 0.0 && kz_ == 0.0);
                    }
                }
    }
    nl.count[i] = np | (ni << 16);
    nl.total[i] = total;
    if (total > mn) raise_overflow(flags, MD_FLAG_NLIST_OVERFLOW, total);
}

// ---------------------------------------------------------------- passes

// Density pass with the embedding fused: rho_i over listed neighbours with
// r < rc, then F(rho_i) and F'(rho_i).
template <int KIND, bool MULTI, int P>
__global__ __launch_bounds__(kBlock) void k_density(int N, State st, Boxes bx, NList nl, Pot pot,
                                                    double L1, double invL1, unsigned *flags)
{
    if (halted(flags)) return;
    const RowLanes<P> rl(atom_index());
    const int i = rl.i;
    if (i >= N) return;
    double L, invL;
    box_geom<MULTI>(bx, i, L1, invL1, L, invL);
    const double *__restrict__ pk = st.pk;
    double xi = st.x[i], yi = st.y[i], zi = st.z[i];
    Row rw = row_of(nl, i);
    unsigned bad = 0;
    double rho = 0.0;
    const int ai = KIND == kTyped ? st.type[i] : 0;
    // several species with cutoffs per pair of types: RCUT(a, b)^2
    const double *cr = (KIND == kTyped && pot.cut2) ? pot.cut2 + ai * pot.nt : nullptr;
    auto body = [&](double dx, double dy, double dz, double, unsigned j) {
        double r2 = dev::dist2(dx, dy, dz);
        if (r2 < (cr ? cr[st.type[j]] : pot.rc2)) {
            if constexpr (KIND == kTyped)
                rho += dens_typed(pot, r2 * rsqrt_nr(r2), ai, st.type[j], bad);
            else
                rho += dens<KIND>(pot, r2 * rsqrt_nr(r2), bad);
        }
    };
    for_pairs<false, false, P>(nl.idx, i, N, rl.part, rw.np, pk, xi, yi, zi, L, invL, body);
    for_pairs<true, false, P>(nl.idx, i, N, rl.first(nl.mn - rw.ni), nl.mn, pk, xi, yi, zi, L,
                              invL, body);
    rho = lanes_sum<P>(rho);
    if (rl.part != 0) {
        raise_flags(flags, bad);
        return;
    }
    double F, Fp;
    if constexpr (KIND == kTyped)
        embed_typed(pot, rho, ai, F, Fp, bad);
    else
        embed<KIND>(pot, rho, F, Fp, bad);
    st.rho[i] = rho;
    st.Femb[i] = F;
    st.Fp[i] = Fp;
    st.pk[4 * (size_t)i + 3] = Fp;
    raise_flags(flags, bad);
}

template <int KIND>
__global__ void k_embed(int N, State st, Pot pot, unsigned *flags)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    unsigned bad = 0;
    double F, Fp;
    if constexpr (KIND == kTyped)
        embed_typed(pot, st.rho[i], st.type[i], F, Fp, bad);
    else
        embed<KIND>(pot, st.rho[i], F, Fp, bad);
    st.Femb[i] = F;
    st.Fp[i] = Fp;
    raise_flags(flags, bad);
}

// Force pass (eq. 3) gathered per atom, optionally fused with the second
// half kick of velocity Verlet (and after it the half-step friction flow of
// eq. (4)).
template <int KIND, bool MULTI, bool ENERGY, bool KICK, int P>
__global__ __launch_bounds__(kBlock) void k_force(int N, State st, Boxes bx, NList nl, Pot pot,
                                                  double L1, double invL1, double kick,
                                                  Thermo th, unsigned *flags)
{
    if (halted(flags)) return;
    const RowLanes<P> rl(atom_index());
    const int i = rl.i;
    if (i >= N) return;
    double L, invL;
    box_geom<MULTI>(bx, i, L1, invL1, L, invL);
    const double *__restrict__ pk = st.pk;
    double xi = st.x[i], yi = st.y[i], zi = st.z[i];
    double fpi = st.Fp[i];
    Row rw = row_of(nl, i);
    unsigned bad = 0;
    double ax = 0.0, ay = 0.0, az = 0.0, ep = 0.0, wv = 0.0;
    const int ai = KIND == kTyped ? st.type[i] : 0;
    // several species with cutoffs per pair of types: RCUT(a, b)^2
    const double *cr = (KIND == kTyped && pot.cut2) ? pot.cut2 + ai * pot.nt : nullptr;
    auto body = [&](double dx, double dy, double dz, double fpj, unsigned j) {
        double r2 = dev::dist2(dx, dy, dz);
        if (r2 < (cr ? cr[st.type[j]] : pot.rc2)) {
            double inv_r = rsqrt_nr(r2);
            double coef, v;
            if constexpr (KIND == kTyped) {
                // [F'_i rho^(ab)'(r) + F'_j rho^(ba)'(r) + V^(ab)'(r)] / r
                double dab, dba, dv;
                if constexpr (ENERGY)
                    pair_terms_typed(pot, r2 * inv_r, ai, st.type[j], dab, dba, v, dv, bad);
                else
                    pair_derivs_typed(pot, r2 * inv_r, ai, st.type[j], dab, dba, dv, bad);
                coef = fma(fpi, dab, fma(fpj, dba, dv)) * inv_r;
            } else {
                // [(F'_i + F'_j) rho'(r) + V'(r)] / r
                double dfr, dv;
                if constexpr (ENERGY)
                    pair_terms<KIND>(pot, r2 * inv_r, dfr, v, dv, bad);
                else
                    pair_derivs<KIND>(pot, r2 * inv_r, dfr, dv, bad);
                coef = fma(fpi + fpj, dfr, dv) * inv_r;
            }
            // f_i += coef (x_j - x_i)
            ax = fma(coef, dx, ax);
            ay = fma(coef, dy, ay);
            az = fma(coef, dz, az);
            if constexpr (ENERGY) {
                ep += v;
                wv = fma(coef, r2, wv);  // [(F'_i + F'_j) rho' + V'] r
            }
        }
    };
    for_pairs<false, true, P>(nl.idx, i, N, rl.part, rw.np, pk, xi, yi, zi, L, invL, body);
    for_pairs<true, true, P>(nl.idx, i, N, rl.first(nl.mn - rw.ni), nl.mn, pk, xi, yi, zi, L,
                             invL, body);
    ax = lanes_sum<P>(ax);
    ay = lanes_sum<P>(ay);
    az = lanes_sum<P>(az);
    if constexpr (ENERGY) {
        ep = lanes_sum<P>(ep);
        wv = lanes_sum<P>(wv);
    }
    if (rl.part != 0) {
        raise_flags(flags, bad);
        return;
    }
    st.fx[i] = ax;
    st.fy[i] = ay;
    st.fz[i] = az;
    if constexpr (ENERGY) {
        st.eat[i] = fma(0.5, ep, st.Femb[i]);
        st.wat[i] = wv;
    }
    if constexpr (KICK) {
        species_kick(st, i, kick, th);
        double vx = fma(kick, ax, st.vx[i]);
        double vy = fma(kick, ay, st.vy[i]);
        double vz = fma(kick, az, st.vz[i]);
        if (th.on) friction_flow(th, vx, vy, vz);
        hold(st, i, vx, vy, vz);
        st.vx[i] = vx;
        st.vy[i] = vy;
        st.vz[i] = vz;
    }
    raise_flags(flags, bad);
}

// First half of a velocity-Verlet step: the half-step friction flow of
// eq. (4) when the thermostat is on, v += (dt/2) a; x += dt v; request a list
// rebuild when an atom has moved more than half the skin since the last build.
template <bool MULTI, bool PACK>
__global__ __launch_bounds__(kBlock) void k_kick_drift(int N, State st, Boxes bx, double kick,
                                                       double dt, double thr2_1, Thermo th,
                                                       unsigned *flags)
{
    if (halted(flags)) return;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    bool need = false, bad = false;
    if (i < N) {
        species_kick(st, i, kick, th);
        double vx = st.vx[i], vy = st.vy[i], vz = st.vz[i];
        if (th.on) friction_flow(th, vx, vy, vz);
        vx = fma(kick, st.fx[i], vx);
        vy = fma(kick, st.fy[i], vy);
        vz = fma(kick, st.fz[i], vz);
        hold(st, i, vx, vy, vz);
        double x = fma(dt, vx, st.x[i]);
        double y = fma(dt, vy, st.y[i]);
        double z = fma(dt, vz, st.z[i]);
        st.vx[i] = vx;
        st.vy[i] = vy;
        st.vz[i] = vz;
        st.x[i] = x;
        st.y[i] = y;
        st.z[i] = z;
        if constexpr (PACK) {
            reinterpret_cast<double2 *>(st.pk)[2 * (size_t)i] = make_double2(x, y);
            st.pk[4 * (size_t)i + 2] = z;
        }
        double ddx = x - st.xr[i], ddy = y - st.yr[i], ddz = z - st.zr[i];
        double d2 = fma(ddz, ddz, fma(ddy, ddy, ddx * ddx));
        double thr2 = MULTI ? bx.thr2[bx.box_of[i]] : thr2_1;
        need = d2 > thr2;
        bad = !isfinite(d2);
    }
    // one request per wavefront, and none once the flag is already raised
    if (__any(need) && (threadIdx.x & 63) == 0 &&
        __atomic_load_n(flags + 1, __ATOMIC_RELAXED) == 0u)
        atomicOr(flags + 1, 1u);
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flags, (unsigned)MD_FLAG_NONFINITE);
}

// End of a replayed step: count the build if one happened, clear the request.
__global__ void k_step_end(unsigned *flags)
{
    if (halted(flags)) return;
    unsigned b = flags[1] ? 1u : 0u;
    unsigned lo = flags[2] + b;
    if (lo < flags[2]) flags[4] += 1u;
    flags[2] = lo;
    unsigned s = flags[3] + 1u;
    if (s == 0u) flags[5] += 1u;
    flags[3] = s;
    flags[1] = 0u;
}

// Step counter at the start of md_step.
__global__ void k_step_mark(unsigned *flags)
{
    flags[kMarkWord] = flags[3];
    flags[kMarkWord + 1] = flags[5];
}

__global__ void k_count_build(unsigned *flags)
{
    unsigned lo = flags[2] + 1u;
    if (lo == 0u) flags[4] += 1u;
    flags[2] = lo;
}

// ---------------------------------------------------------------- reductions

// Fixed-order sums per box: chunk partials (one workgroup per chunk of at
// most kChunk atoms of one box) then one thread per box over its chunks.
__global__ __launch_bounds__(kBlock) void k_chunk_sums(int what, State st, double half_m_over_k,
                                                       const int *__restrict__ cstart,
                                                       const int *__restrict__ cend,
                                                       double *__restrict__ partial)
{
    __shared__ double red[kBlock];
    int c = blockIdx.x;
    int s = cstart[c], e = cend[c];
    double acc = 0.0;
    for (int i = s + threadIdx.x; i < e; i += blockDim.x) {
        if (what == 0) {
            acc += st.eat[i];
        } else if (what == 2) {
            acc += st.wat[i];
        } else {
            double vx = st.vx[i], vy = st.vy[i], vz = st.vz[i];
            double hm = st.type ? st.tcoef[4 * st.type[i] + kTcHalfM] : half_m_over_k;
            acc += hm * fma(vz, vz, fma(vy, vy, vx * vx));
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[c] = red[0];
}

__global__ void k_box_sums(int B, const int *__restrict__ box_chunk, const double *__restrict__ partial,
                           double *__restrict__ out)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double s = 0.0;
    for (int c = box_chunk[b]; c < box_chunk[b + 1]; ++c) s += partial[c];
    out[b] = s;
}

// ---------------------------------------------------------------- pressure, barostat

// Eq. (6) per box from the kinetic energy K and the per-atom virial sum S
// (W = -S/2, the pair form of sum_i f_i . r_i): P = (2 K + W) / (3 V).
// d_baro layout per box: mu | strain | rlist | pressure | virial | kinetic | virial sum.
__global__ void k_pressure_eval(int B, const double *__restrict__ L, double *__restrict__ baro)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double w = -0.5 * baro[6 * B + b], k = baro[5 * B + b], l = L[b];
    baro[4 * B + b] = w;
    baro[3 * B + b] = (2.0 * k + w) / (3.0 * (l * l * l));
}

// Eq. (5): mu = [1 - beta (dt / tau) (P0 - P)]^(1/3) for the next step.
__global__ void k_baro_mu(int B, double p0, double beta_dt_tau, double *__restrict__ baro)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    baro[b] = cbrt(1.0 - beta_dt_tau * (p0 - baro[3 * B + b]));
}

// Box update of a barostat step: L *= mu, the strain since the last build
// s *= mu and the rebuild threshold ((r_list - rc) - |1 - s| r_list) / 2
// (negative: rebuild at once).  A box that would shrink below its cell grid
// keeps its size (mu = 1) and raises MD_FLAG_BOX_RANGE.  The rebuild request
// of the kick-drift kernel is withdrawn: it is decided again on the scaled
// coordinates.
__global__ void k_baro_box(int B, double rc, double *__restrict__ boxd, const int *__restrict__ nc,
                           double *__restrict__ baro, unsigned *flags)
{
    if (halted(flags)) return;
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b == 0) flags[1] = 0u;
    if (b >= B) return;
    double *L = boxd, *invL = boxd + B, *thr2 = boxd + 3 * B;
    double mu = baro[b], rl = baro[2 * B + b], Ln = L[b] * mu;
    if (!(Ln >= nc[b] * rl * (1.0 + 1e-12) && rl < 0.5 * Ln)) {
        mu = 1.0;
        Ln = L[b];
        atomicOr(flags, (unsigned)MD_FLAG_BOX_RANGE);
    }
    baro[b] = mu;
    L[b] = Ln;
    invL[b] = 1.0 / Ln;
    double st = baro[B + b] * mu;
    baro[B + b] = st;
    double half = 0.5 * ((rl - rc) - fabs(1.0 - st) * rl);
    thr2[b] = half < 0.0 ? -1.0 : half * half;
}

// Scale coordinates and reference positions by their box's mu and decide the
// rebuild on the scaled coordinates.
template <bool PACK>
__global__ __launch_bounds__(kBlock) void k_baro_scale(int N, State st, Boxes bx,
                                                       const double *__restrict__ baro,
                                                       unsigned *flags)
{
    if (halted(flags)) return;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    bool need = false;
    if (i < N) {
        int b = bx.box_of[i];
        double mu = baro[b];
        double x = st.x[i] * mu, y = st.y[i] * mu, z = st.z[i] * mu;
        double xr = st.xr[i] * mu, yr = st.yr[i] * mu, zr = st.zr[i] * mu;
        st.x[i] = x;
        st.y[i] = y;
        st.z[i] = z;
        st.xr[i] = xr;
        st.yr[i] = yr;
        st.zr[i] = zr;
        if constexpr (PACK) {
            reinterpret_cast<double2 *>(st.pk)[2 * (size_t)i] = make_double2(x, y);
            st.pk[4 * (size_t)i + 2] = z;
        }
        double ddx = x - xr, ddy = y - yr, ddz = z - zr;
        double d2 = fma(ddz, ddz, fma(ddy, ddy, ddx * ddx));
        need = d2 > bx.thr2[b];
    }
    if (__any(need) && (threadIdx.x & 63) == 0 &&
        __atomic_load_n(flags + 1, __ATOMIC_RELAXED) == 0u)
        atomicOr(flags + 1, 1u);
}

// After a list build: no strain since the build, the plain half-skin test.
__global__ void k_baro_rebuilt(const unsigned *gate, int B, double rc, double *__restrict__ boxd,
                               double *__restrict__ baro)
{
    if (skip(gate)) return;
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double half = 0.5 * (baro[2 * B + b] - rc);
    baro[B + b] = 1.0;
    boxd[3 * B + b] = half * half;
}

// ---------------------------------------------------------------- neighbours out

__global__ void k_get_neighbors(int N, State st, NList nl, int32_t *counts, int32_t *ids, int cols)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int o = st.id[i];
    Row rw = row_of(nl, i);
    counts[o] = nl.total[i];
    int m = 0;
    for (int n = 0; n < rw.np && m < cols; ++n)
        ids[(size_t)o * cols + (m++)] = st.id[nl.idx[nl_off(n, i, N)]];
    for (int n = nl.mn - rw.ni; n < nl.mn && m < cols; ++n)
        ids[(size_t)o * cols + (m++)] = st.id[nl.idx[nl_off(n, i, N)]];
}

// ---------------------------------------------------------------- B-spline

// Uniform cubic B-spline -> per-interval cubic in t: on interval m
// S(t) = sum_l theta_{m+l} b_l(t) with the standard pieces
// b0 = (1-t)^3/6, b1 = (3t^3 - 6t^2 + 4)/6, b2 = (-3t^3 + 3t^2 + 3t + 1)/6, b3 = t^3/6.
__global__ void k_bspline_tables(int K, const double *__restrict__ theta, double *__restrict__ tab)
{
    int nint = K - 3;
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= 3 * nint) return;
    int f = g / nint, m = g % nint;
    const double *th = theta + f * K + m;
    double t0 = th[0], t1 = th[1], t2 = th[2], t3 = th[3];
    double *o = tab + (size_t)f * nint * 4 + 4 * m;
    o[0] = (t0 + 4.0 * t1 + t2) / 6.0;
    o[1] = (t2 - t0) / 2.0;
    o[2] = (t0 - 2.0 * t1 + t2) / 2.0;
    o[3] = (-t0 + 3.0 * t1 - 3.0 * t2 + t3) / 6.0;
}

// Interleaved r-grid tables of the force pass (Pot::pair): thread g fills
// interval m of table pair ab = g / n.
__global__ void k_pair_tables(int n, int T, const double *__restrict__ V,
                              const double *__restrict__ R, double *__restrict__ out,
                              double *__restrict__ dout)
{
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= T * T * n) return;
    int ab = g / n, m = g % n;
    const double *v = V + 4 * (size_t)g, *rab = R + 4 * (size_t)g;
    if (T == 1) {
        double *o = out + 8 * (size_t)m, *d = dout + 6 * (size_t)m;
        for (int k = 0; k < 4; ++k) {
            o[k] = v[k];
            o[4 + k] = rab[k];
        }
        for (int k = 1; k < 4; ++k) {
            d[k - 1] = v[k];
            d[2 + k] = rab[k];
        }
        return;
    }
    int a = ab / T, b = ab % T;
    const double *rba = R + 4 * ((size_t)(b * T + a) * n + m);
    double *o = out + 16 * (size_t)g, *d = dout + 10 * (size_t)g;
    for (int k = 0; k < 4; ++k) {
        o[k] = v[k];
        o[4 + k] = rab[k];
        o[8 + k] = rba[k];
        o[12 + k] = 0.0;
    }
    for (int k = 1; k < 4; ++k) {
        d[k - 1] = v[k];
        d[2 + k] = rab[k];
        d[5 + k] = rba[k];
    }
    d[9] = 0.0;
}

inline int grid_for(int64_t n, int block = kBlock) { return (int)((n + block - 1) / block); }

constexpr int kGatedBlocks = 2048;  // grid cap of the sort's atom loops (8 per CU)

template <int KIND, bool MULTI>
void density_t(Ctx &c, hipStream_t s)
{
    int blk = atom_block(c.N);
    int N = (int)c.N;
    double L = c.box_len[0], iL = 1.0 / c.box_len[0];
    if (row_lanes(c.N) == kRowLanes)
        k_density<KIND, MULTI, kRowLanes><<<grid_for(c.N * kRowLanes, blk), blk, 0, s>>>(
            N, c.st, c.bx, c.nl, c.pot, L, iL, c.dev.flags);
    else
        k_density<KIND, MULTI, 1><<<grid_for(c.N, blk), blk, 0, s>>>(N, c.st, c.bx, c.nl, c.pot,
                                                                      L, iL, c.dev.flags);
}

template <int KIND, bool MULTI, int P>
void force_p(Ctx &c, bool energy, bool kick, int blk, hipStream_t s)
{
    double k = 0.5 * c.dt * (1.602176634e-19 / 1.66053906660e-27 * 1e-10) / c.mass;
    double L = c.box_len[0], iL = 1.0 / c.box_len[0];
    int g = grid_for(c.N * P, blk);
    int N = (int)c.N;
    if (energy && kick)
        k_force<KIND, MULTI, true, true, P><<<g, blk, 0, s>>>(N, c.st, c.bx, c.nl, c.pot, L, iL, k, c.thermo, c.dev.flags);
    else if (energy)
        k_force<KIND, MULTI, true, false, P><<<g, blk, 0, s>>>(N, c.st, c.bx, c.nl, c.pot, L, iL, k, c.thermo, c.dev.flags);
    else if (kick)
        k_force<KIND, MULTI, false, true, P><<<g, blk, 0, s>>>(N, c.st, c.bx, c.nl, c.pot, L, iL, k, c.thermo, c.dev.flags);
    else
        k_force<KIND, MULTI, false, false, P><<<g, blk, 0, s>>>(N, c.st, c.bx, c.nl, c.pot, L, iL, k, c.thermo, c.dev.flags);
}

template <int KIND, bool MULTI>
void force_t(Ctx &c, bool energy, bool kick, hipStream_t s)
{
    int blk = atom_block(c.N);
    if (row_lanes(c.N) == kRowLanes)
        force_p<KIND, MULTI, kRowLanes>(c, energy, kick, blk, s);
    else
        force_p<KIND, MULTI, 1>(c, energy, kick, blk, s);
}

}  // namespace

// Acceleration unit (eV/Angstrom)/amu -> Angstrom/fs^2.
static constexpr double kKappa = 1.602176634e-19 / 1.66053906660e-27 * 1e-10;

__global__ void k_clear_bits(unsigned *flags, unsigned mask) { flags[0] &= ~mask; }

void launch_clear_bits(Ctx &c, unsigned mask, hipStream_t s)
{
    k_clear_bits<<<1, 1, 0, s>>>(c.dev.flags, mask);
}

void launch_fill_u32(unsigned *p, int n, unsigned v, hipStream_t s)
{
    k_fill_u32<<<grid_for(n), kBlock, 0, s>>>(p, n, v);
}

void launch_pack_positions(Ctx &c, hipStream_t s)
{
    k_pack_positions<<<grid_for(c.N), kBlock, 0, s>>>((int)c.N, c.st);
}

void launch_refresh_frozen(Ctx &c, hipStream_t s)
{
    k_refresh_frozen<<<grid_for(c.N), kBlock, 0, s>>>((int)c.N, c.st);
}

void launch_refresh_types(Ctx &c, hipStream_t s)
{
    k_refresh_types<<<grid_for(c.N), kBlock, 0, s>>>((int)c.N, c.st);
}

void launch_set_state(Ctx &c, const double *pos, const double *vel, hipStream_t s)
{
    k_set_state<<<grid_for(c.N), kBlock, 0, s>>>((int)c.N, pos, vel, c.st);
}

void launch_get_state(Ctx &c, double *pos, double *vel, hipStream_t s)
{
    k_get_state<<<grid_for(c.N), kBlock, 0, s>>>((int)c.N, c.st, pos, vel);
}

void launch_build(Ctx &c, bool gated, hipStream_t s)
{
    const unsigned *gate = gated ? c.dev.flags : nullptr;
    int N = (int)c.N;
    int C = c.bd.n_cells;
    // the per-cell counts are zero here: set at creation, cleared by every scan
    // the atom loops of the sort are grid-stride over a capped grid: in the
    // replayed steps that skip the build, launching them costs less
    const int gN = std::min(grid_for(N), kGatedBlocks);
    k_bin<<<gN, kBlock, 0, s>>>(gate, N, c.st, c.bx, c.bd, c.dev.flags);
    int nb = (C + kScanCells - 1) / kScanCells;
    k_scan_local<<<nb, 1024, 0, s>>>(gate, C, c.bd.cell_count, c.bd.cell_start, c.bd.bsum);
    k_scan_add<<<grid_for(C), kBlock, 0, s>>>(gate, C, nb, c.bd.cell_start, c.bd.bsum);
    k_scatter<<<gN, kBlock, 0, s>>>(gate, N, c.bd);
    k_rank<<<gN, kBlock, 0, s>>>(gate, N, c.st, c.bd);
    k_gather<<<gN, kBlock, 0, s>>>(gate, N, c.st, c.bd);
    k_commit<<<gN, kBlock, 0, s>>>(gate, N, c.st, c.bd);
    if (c.tiled)
        launch_tile_nlist(c, gate, s);
    else
        k_nlist<<<grid_for(N, atom_block(N)), atom_block(N), 0, s>>>(
            gate, N, c.st, c.bx, c.bd, c.nl,
            c.pot.cut2 ? c.pot.cut2 + (size_t)c.pot.nt * c.pot.nt : nullptr, c.pot.nt, c.dev.flags);
    if (c.baro_on)
        k_baro_rebuilt<<<grid_for(c.B), kBlock, 0, s>>>(gate, c.B, c.pot.rc, c.d_boxd, c.d_baro);
    if (!gated) k_count_build<<<1, 1, 0, s>>>(c.dev.flags);
}

void launch_density(Ctx &c, hipStream_t s, bool fp_only)
{
    if (c.tiled) {
        launch_tile_density(c, s, fp_only);
        return;
    }
    // with the barostat the box lengths live on the device only
    bool multi = c.B > 1 || c.baro_on;
    switch (c.pot.kind) {
    case MD_POT_FS: multi ? density_t<MD_POT_FS, true>(c, s) : density_t<MD_POT_FS, false>(c, s); break;
    case MD_POT_SMTB: multi ? density_t<MD_POT_SMTB, true>(c, s) : density_t<MD_POT_SMTB, false>(c, s); break;
    case kTyped: multi ? density_t<kTyped, true>(c, s) : density_t<kTyped, false>(c, s); break;
    default: multi ? density_t<MD_POT_SPLINE, true>(c, s) : density_t<MD_POT_SPLINE, false>(c, s); break;
    }
}

void launch_embed(Ctx &c, hipStream_t s)
{
    int g = grid_for(c.N);
    switch (c.pot.kind) {
    case MD_POT_FS: k_embed<MD_POT_FS><<<g, kBlock, 0, s>>>((int)c.N, c.st, c.pot, c.dev.flags); break;
    case MD_POT_SMTB: k_embed<MD_POT_SMTB><<<g, kBlock, 0, s>>>((int)c.N, c.st, c.pot, c.dev.flags); break;
    case kTyped: k_embed<kTyped><<<g, kBlock, 0, s>>>((int)c.N, c.st, c.pot, c.dev.flags); break;
    default: k_embed<MD_POT_SPLINE><<<g, kBlock, 0, s>>>((int)c.N, c.st, c.pot, c.dev.flags); break;
    }
}

void launch_force(Ctx &c, bool energy, int kick_mode, hipStream_t s)
{
    if (c.tiled) {
        launch_tile_force(c, energy, kick_mode, s);
        return;
    }
    bool kick = kick_mode > 0;  // fused drifts are captured for tiled contexts only
    bool multi = c.B > 1 || c.baro_on;
    switch (c.pot.kind) {
    case MD_POT_FS: multi ? force_t<MD_POT_FS, true>(c, energy, kick, s) : force_t<MD_POT_FS, false>(c, energy, kick, s); break;
    case MD_POT_SMTB: multi ? force_t<MD_POT_SMTB, true>(c, energy, kick, s) : force_t<MD_POT_SMTB, false>(c, energy, kick, s); break;
    case kTyped: multi ? force_t<kTyped, true>(c, energy, kick, s) : force_t<kTyped, false>(c, energy, kick, s); break;
    default: multi ? force_t<MD_POT_SPLINE, true>(c, energy, kick, s) : force_t<MD_POT_SPLINE, false>(c, energy, kick, s); break;
    }
}

void launch_kick_drift(Ctx &c, hipStream_t s)
{
    double k = 0.5 * c.dt * kKappa / c.mass;
    double h = 0.5 * (c.box_rlist[0] - c.pot.rc);
    // the packed neighbour records feed only the per-atom kernels
    int g = grid_for(c.N), N = (int)c.N;
    bool multi = c.B > 1 || c.baro_on;
    if (multi && c.tiled)
        k_kick_drift<true, false><<<g, kBlock, 0, s>>>(N, c.st, c.bx, k, c.dt, 0.0, c.thermo, c.dev.flags);
    else if (multi)
        k_kick_drift<true, true><<<g, kBlock, 0, s>>>(N, c.st, c.bx, k, c.dt, 0.0, c.thermo, c.dev.flags);
    else if (c.tiled)
        k_kick_drift<false, false><<<g, kBlock, 0, s>>>(N, c.st, c.bx, k, c.dt, h * h, c.thermo, c.dev.flags);
    else
        k_kick_drift<false, true><<<g, kBlock, 0, s>>>(N, c.st, c.bx, k, c.dt, h * h, c.thermo, c.dev.flags);
}

void launch_step_end(Ctx &c, hipStream_t s) { k_step_end<<<1, 1, 0, s>>>(c.dev.flags); }

void launch_step_mark(Ctx &c, hipStream_t s) { k_step_mark<<<1, 1, 0, s>>>(c.dev.flags); }

void launch_scatter_scalar(Ctx &c, const double *src, double *dst, hipStream_t s)
{
    k_scatter_scalar<<<grid_for(c.N), kBlock, 0, s>>>((int)c.N, c.st.id, src, dst);
}

void launch_scatter_vec3(Ctx &c, const double *sx, const double *sy, const double *sz, double *dst,
                         hipStream_t s)
{
    k_scatter_vec3<<<grid_for(c.N), kBlock, 0, s>>>((int)c.N, c.st.id, sx, sy, sz, dst);
}

void launch_box_sums(Ctx &c, int what, double *out, hipStream_t s)
{
    const int *cs = c.d_chunks, *ce = c.d_chunks + c.n_chunks, *bc = c.d_chunks + 2 * c.n_chunks;
    k_chunk_sums<<<c.n_chunks, kBlock, 0, s>>>(what, c.st, 0.5 * c.mass / kKappa, cs, ce, c.d_partial);
    k_box_sums<<<grid_for(c.B), kBlock, 0, s>>>(c.B, bc, c.d_partial, out);
}

void launch_pressure_eval(Ctx &c, hipStream_t s)
{
    launch_box_sums(c, 1, c.d_baro + 5 * c.B, s);
    launch_box_sums(c, 2, c.d_baro + 6 * c.B, s);
    k_pressure_eval<<<grid_for(c.B), kBlock, 0, s>>>(c.B, c.d_boxd, c.d_baro);
}

void launch_baro_mu(Ctx &c, hipStream_t s)
{
    k_baro_mu<<<grid_for(c.B), kBlock, 0, s>>>(c.B, c.baro_p0, c.baro_beta * c.dt / c.baro_tau,
                                              c.d_baro);
}

void launch_baro_box_scale(Ctx &c, hipStream_t s)
{
    k_baro_box<<<grid_for(c.B), kBlock, 0, s>>>(c.B, c.pot.rc, c.d_boxd, c.bx.nc, c.d_baro,
                                               c.dev.flags);
    if (c.tiled)
        k_baro_scale<false><<<grid_for(c.N), kBlock, 0, s>>>((int)c.N, c.st, c.bx, c.d_baro, c.dev.flags);
    else
        k_baro_scale<true><<<grid_for(c.N), kBlock, 0, s>>>((int)c.N, c.st, c.bx, c.d_baro, c.dev.flags);
}

void launch_get_neighbors(Ctx &c, int32_t *counts, int32_t *ids, int32_t max_cols, hipStream_t s)
{
    if (c.tiled) {
        launch_tile_get_neighbors(c, counts, ids, max_cols, s);
        return;
    }
    k_get_neighbors<<<grid_for(c.N), kBlock, 0, s>>>((int)c.N, c.st, c.nl, counts, ids, max_cols);
}

void launch_bspline_tables(Ctx &c, const double *theta, hipStream_t s)
{
    int K = c.n_theta;
    k_bspline_tables<<<grid_for(3 * (K - 3)), kBlock, 0, s>>>(K, theta, c.tables);
    launch_pair_tables(c, s);
}

void launch_pair_tables(Ctx &c, hipStream_t s)
{
    if (!c.pot.pair) return;
    const int n = c.pot.tab[0].n, T = c.pot.nt;
    k_pair_tables<<<grid_for((int64_t)T * T * n), kBlock, 0, s>>>(n, T, c.pot.tab[0].c,
                                                                 c.pot.tab[1].c, c.pair_tab,
                                                                 c.dpair_tab);
}

}  // namespace mdk
