// Device helpers shared by the kernel files of libmd.so: potential
// evaluation (eq. 1 forms and lookup tables), distance arithmetic, cell and
// tile geometry.  All functions are inline device code.
#pragma once

#include <hip/hip_runtime.h>

#include "md_internal.h"

namespace mdk {
namespace dev {

// ---------------------------------------------------------------- arithmetic

// Minimum image of a separation component: d - L * rint(d / L).  For the
// separations that can be listed (|d| < L/2 after the correction) this
// equals subtracting or adding L once, exactly.
__device__ __forceinline__ double min_image(double d, double L, double invL)
{
    return fma(-L, rint(d * invL), d);
}

// Squared distance of a pair as the cutoff tests take it: (dx dx + dy dy) +
// dz dz with every product and sum rounded separately.  Every pass decides
// r < rc (and the list build r < r_list) from this value, so the set of
// interacting pairs does not depend on which kernel evaluates a pair.
__device__ __forceinline__ double dist2(double dx, double dy, double dz)
{
#pragma clang fp contract(off)
    return (dx * dx + dy * dy) + dz * dz;
}

// 1/sqrt(a), a > 0: the hardware estimate y (relative error about 5e-8)
// refined by one third-order step: with e = 1 - a y^2,
// 1/sqrt(a) = y (1 - e)^(-1/2) = y (1 + e/2 + 3 e^2/8 + O(e^3)).
__device__ __forceinline__ double rsqrt_nr(double a)
{
    double y = __builtin_amdgcn_rsq(a);
    double e = fma(-a * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

// 2^t on the vector ALU alone, for |t| <= 1000 (the host checks that the
// arguments of a potential stay in that range): t = k + f with k the nearest
// integer and |f| <= 1/2, 2^f = exp(f ln2) by the polynomial kExpPoly in
// f ln2 (its coefficients are stored premultiplied by powers of ln 2), then
// 2^t = 2^k 2^f.  k comes from adding 1.5 * 2^52 to t: the sum rounds t to an
// integer, which the low 32 bits of the result then hold in two's complement;
// f = t - k is exact.  Exponentials exp(a r + b) of the pair terms are taken
// as 2^(a' r + b') with a' = a log2(e), b' = b log2(e) folded on the host.
__device__ __forceinline__ double exp2_fast(double t, const Pot &p)
{
    const double shifter = 6755399441055744.0;  // 1.5 * 2^52
    double s = t + shifter;
    int k = __double2loint(s);
    double f = t - (s - shifter);
    double q = fma(p.ec[kExpDeg], f, p.ec[kExpDeg - 1]);
#pragma unroll
    for (int m = kExpDeg - 2; m >= 1; --m) q = fma(q, f, p.ec[m]);
    q = fma(q, f, 1.0);
    return ldexp(q, k);
}

// ---------------------------------------------------------------- potential

// The vector ALU takes at most one scalar-register operand per instruction,
// so fma(a, r, b) with a and b both uniform needs one of them copied into a
// vector register.  Pinning the additive constants of the pair terms in
// vector registers once, before a loop over pairs, keeps that copy out of
// the loop.  (The empty asm only forces the value into a vector register.)
__device__ __forceinline__ void pin_vector(double &v) { asm volatile("" : "+v"(v)); }

__device__ __forceinline__ Pot pinned(const Pot &p)
{
    Pot q = p;
    if (q.kind == MD_POT_SMTB) {
        pin_vector(q.bv);
        pin_vector(q.bf);
        pin_vector(q.bvd);
        pin_vector(q.bfd);
        pin_vector(q.ec[kExpDeg - 1]);
    }
    return q;
}

__device__ __forceinline__ void table_eval(const Table &t, double x, double &s, double &ds,
                                           unsigned &bad)
{
    double u = (x - t.lo) * t.inv_h;
    int m = (int)floor(u);
    if (!(x >= t.lo && x <= t.hi)) bad |= MD_FLAG_TABLE_RANGE;
    m = m < 0 ? 0 : (m > t.n - 1 ? t.n - 1 : m);
    double tt = u - (double)m;
    const double2 *p = reinterpret_cast<const double2 *>(t.c + 4 * m);
    double2 ab = p[0], cd = p[1];
    s = fma(tt, fma(tt, fma(tt, cd.y, cd.x), ab.y), ab.x);
    ds = fma(tt, fma(tt, 3.0 * cd.y, 2.0 * cd.x), ab.y) * t.inv_h;
}

// Density contribution rho(r).
template <int KIND>
__device__ __forceinline__ double dens(const Pot &p, double r, unsigned &bad)
{
    if constexpr (KIND == MD_POT_FS) {
        double u = r - p.d;
        return r < p.d ? u * u : 0.0;
    } else if constexpr (KIND == MD_POT_SMTB) {
        return exp2_fast(fma(p.af, r, p.bf), p);
    } else {
        double s, ds;
        table_eval(p.tab[1], r, s, ds, bad);
        return s;
    }
}

// rho'(r), V(r), V'(r).
template <int KIND>
__device__ __forceinline__ void pair_terms(const Pot &p, double r, double &dfr, double &v,
                                           double &dv, unsigned &bad)
{
    if constexpr (KIND == MD_POT_FS) {
        double u = r - p.d;
        dfr = r < p.d ? 2.0 * u : 0.0;
        double w = r - p.c;
        double poly = fma(r, fma(r, p.c2, p.c1), p.c0);
        double dpoly = fma(2.0 * p.c2, r, p.c1);
        bool in = r < p.c;
        v = in ? w * w * poly : 0.0;
        dv = in ? w * fma(w, dpoly, 2.0 * poly) : 0.0;
    } else if constexpr (KIND == MD_POT_SMTB) {
        double ef = exp2_fast(fma(p.af, r, p.bf), p);
        double ev = exp2_fast(fma(p.av, r, p.bv), p);
        dfr = p.afn * ef;
        v = ev;
        dv = p.avn * ev;
    } else if (p.pair) {
        // one interval of V and rho, 64 contiguous bytes
        const Table &t = p.tab[0];
        double u = (r - t.lo) * t.inv_h;
        int m = (int)floor(u);
        if (!(r >= t.lo && r <= t.hi)) bad |= MD_FLAG_TABLE_RANGE;
        m = m < 0 ? 0 : (m > t.n - 1 ? t.n - 1 : m);
        double tt = u - (double)m;
        const double2 *c = reinterpret_cast<const double2 *>(p.pair + 8 * (size_t)m);
        double2 va = c[0], vb = c[1], fa = c[2], fb = c[3];
        v = fma(tt, fma(tt, fma(tt, vb.y, vb.x), va.y), va.x);
        dv = fma(tt, fma(tt, 3.0 * vb.y, 2.0 * vb.x), va.y) * t.inv_h;
        dfr = fma(tt, fma(tt, 3.0 * fb.y, 2.0 * fb.x), fa.y) * t.inv_h;
    } else {
        double s;
        table_eval(p.tab[1], r, s, dfr, bad);
        table_eval(p.tab[0], r, v, dv, bad);
    }
}

// Force coefficient of one pair without the energy, up to a sign fixed per
// kind: (F'_i + F'_j) rho'(r) + V'(r) = kSign * returned value.  For SMTB
// both derivatives are negative single exponentials, so the kernel takes
// exp(af r + bfd) and exp(av r + bvd) and negates the sum once per atom.
template <int KIND>
constexpr double kForceSign = KIND == MD_POT_SMTB ? -1.0 : 1.0;

// Several species: interval and local coordinate of x on a grid shared by
// the tables of one kind.
__device__ __forceinline__ double table_locate(const Table &t, double x, int &m, unsigned &bad)
{
    double u = (x - t.lo) * t.inv_h;
    m = (int)floor(u);
    if (!(x >= t.lo && x <= t.hi)) bad |= MD_FLAG_TABLE_RANGE;
    m = m < 0 ? 0 : (m > t.n - 1 ? t.n - 1 : m);
    return u - (double)m;
}

// rho'(r) and V'(r) alone (forces without energies): for tables on a shared
// grid from the derivative interval (b, c, d of each cubic, 48 bytes: three
// 16-byte loads instead of four), with the arithmetic of pair_terms.
template <int KIND>
__device__ __forceinline__ void pair_derivs(const Pot &p, double r, double &dfr, double &dv,
                                            unsigned &bad)
{
    if constexpr (KIND == MD_POT_SPLINE) {
        if (p.dpair) {
            const Table &t = p.tab[0];
            int m;
            const double tt = table_locate(t, r, m, bad);
            const double2 *c = reinterpret_cast<const double2 *>(p.dpair + 6 * (size_t)m);
            const double2 vb = c[0], vd = c[1], rc = c[2];  // (Vb, Vc) (Vd, Rb) (Rc, Rd)
            dv = fma(tt, fma(tt, 3.0 * vd.x, 2.0 * vb.y), vb.x) * t.inv_h;
            dfr = fma(tt, fma(tt, 3.0 * rc.y, 2.0 * rc.x), vd.y) * t.inv_h;
            return;
        }
    }
    double v;
    pair_terms<KIND>(p, r, dfr, v, dv, bad);
}

template <int KIND>
__device__ __forceinline__ double pair_coef(const Pot &p, double r, double fpij, unsigned &bad)
{
    if constexpr (KIND == MD_POT_SMTB) {
        double e1 = exp2_fast(fma(p.af, r, p.bfd), p);
        double e2 = exp2_fast(fma(p.av, r, p.bvd), p);
        return fma(fpij, e1, e2);
    } else {
        double dfr, dv;
        pair_derivs<KIND>(p, r, dfr, dv, bad);
        return fma(fpij, dfr, dv);
    }
}

// The coefficients of table idx of a kind at interval m (several species).
__device__ __forceinline__ void table_cubic(const Table &t, int idx, int m, double tt, double &s,
                                            double &ds)
{
    const double2 *p = reinterpret_cast<const double2 *>(t.c + 4 * ((size_t)idx * t.n + m));
    double2 ab = p[0], cd = p[1];
    s = fma(tt, fma(tt, fma(tt, cd.y, cd.x), ab.y), ab.x);
    ds = fma(tt, fma(tt, 3.0 * cd.y, 2.0 * cd.x), ab.y) * t.inv_h;
}

// rho^(ab)(r): density at an atom of type a contributed by one of type b.
__device__ __forceinline__ double dens_typed(const Pot &p, double r, int a, int b, unsigned &bad)
{
    int m;
    double tt = table_locate(p.tab[1], r, m, bad), s, ds;
    table_cubic(p.tab[1], a * p.nt + b, m, tt, s, ds);
    return s;
}

// rho^(ab)'(r), rho^(ba)'(r), V^(ab)(r), V^(ab)'(r) on the shared r grid,
// from the interleaved table (one 128-byte line per pair and interval).
__device__ __forceinline__ void pair_terms_typed(const Pot &p, double r, int a, int b,
                                                 double &dab, double &dba, double &v, double &dv,
                                                 unsigned &bad)
{
    int m;
    const Table &t = p.tab[0];
    double tt = table_locate(t, r, m, bad);
    const double2 *c =
        reinterpret_cast<const double2 *>(p.pair + 16 * ((size_t)(a * p.nt + b) * t.n + m));
    double2 va = c[0], vb = c[1], aa = c[2], ab = c[3], ba = c[4], bb = c[5];
    v = fma(tt, fma(tt, fma(tt, vb.y, vb.x), va.y), va.x);
    dv = fma(tt, fma(tt, 3.0 * vb.y, 2.0 * vb.x), va.y) * t.inv_h;
    dab = fma(tt, fma(tt, 3.0 * ab.y, 2.0 * ab.x), aa.y) * t.inv_h;
    dba = fma(tt, fma(tt, 3.0 * bb.y, 2.0 * bb.x), ba.y) * t.inv_h;
}

// rho^(ab)'(r), rho^(ba)'(r), V^(ab)'(r) alone (forces without energies),
// from the derivative interval (b, c, d of the three cubics, 80 bytes: five
// 16-byte loads instead of six), with the arithmetic of pair_terms_typed.
__device__ __forceinline__ void pair_derivs_typed(const Pot &p, double r, int a, int b,
                                                  double &dab, double &dba, double &dv,
                                                  unsigned &bad)
{
    if (!p.dpair) {
        double v;
        pair_terms_typed(p, r, a, b, dab, dba, v, dv, bad);
        return;
    }
    int m;
    const Table &t = p.tab[0];
    const double tt = table_locate(t, r, m, bad);
    const double2 *c =
        reinterpret_cast<const double2 *>(p.dpair + 10 * ((size_t)(a * p.nt + b) * t.n + m));
    // (Vb, Vc) (Vd, Ab) (Ac, Ad) (Bb, Bc) (Bd, 0): A = rho^(ab), B = rho^(ba)
    const double2 c0 = c[0], c1 = c[1], c2 = c[2];
    dv = fma(tt, fma(tt, 3.0 * c1.x, 2.0 * c0.y), c0.x) * t.inv_h;
    dab = fma(tt, fma(tt, 3.0 * c2.y, 2.0 * c2.x), c1.y) * t.inv_h;
    if (a == b) {
        dba = dab;   // the same table: the lanes of such pairs skip its last two loads
    } else {
        const double2 c3 = c[3], c4 = c[4];
        dba = fma(tt, fma(tt, 3.0 * c4.x, 2.0 * c3.y), c3.x) * t.inv_h;
    }
}

// F^(a)(rho), F^(a)'(rho).
__device__ __forceinline__ void embed_typed(const Pot &p, double rho, int a, double &F, double &Fp,
                                            unsigned &bad)
{
    int m;
    double tt = table_locate(p.tab[2], rho, m, bad);
    table_cubic(p.tab[2], a, m, tt, F, Fp);
}

// F(rho), F'(rho).
template <int KIND>
__device__ __forceinline__ void embed(const Pot &p, double rho, double &F, double &Fp,
                                      unsigned &bad)
{
    if constexpr (KIND == MD_POT_FS || KIND == MD_POT_SMTB) {
        double A = (KIND == MD_POT_FS) ? p.A : 1.0;
        if (rho > 0.0) {
            double s = sqrt(rho);
            F = -A * s;
            Fp = -0.5 * A / s;
        } else {
            F = 0.0;
            Fp = 0.0;
        }
    } else {
        table_eval(p.tab[2], rho, F, Fp, bad);
    }
}

// ---------------------------------------------------------------- cells

__device__ __forceinline__ double wrap1(double x, double L)
{
    while (x < 0.0) x += L;
    while (x >= L) x -= L;
    return x;
}

// Cell of a wrapped coordinate along one axis.
__device__ __forceinline__ int cell_coord(double x, double ncL, int nc)
{
    int c = (int)(x * ncL);
    return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

// Distinct cells {c-1, c, c+1} modulo nc along one axis.
__device__ __forceinline__ int stencil_1d(int c, int nc, int out[3])
{
    if (nc == 1) {
        out[0] = 0;
        return 1;
    }
    if (nc == 2) {
        out[0] = 0;
        out[1] = 1;
        return 2;
    }
    out[0] = c == 0 ? nc - 1 : c - 1;
    out[1] = c;
    out[2] = c == nc - 1 ? 0 : c + 1;
    return 3;
}

// Neighbour cells along one axis for three or more cells, with the periodic
// shift that brings x_j - x_i to the minimum image: +L for the cell past the
// upper end (wrapped to 0), -L for the cell past the lower end.
__device__ __forceinline__ void stencil_shift(int c, int nc, double L, int cell[3], double sh[3])
{
    cell[0] = c == 0 ? nc - 1 : c - 1;
    sh[0] = c == 0 ? -L : 0.0;
    cell[1] = c;
    sh[1] = 0.0;
    cell[2] = c == nc - 1 ? 0 : c + 1;
    sh[2] = c == nc - 1 ? L : 0.0;
}

// Cells are numbered tile by tile: a box's cells are grouped in tiles of
// tx x ty x tz cells (row-major over the tile grid, row-major inside a tile),
// so the atoms of one tile are contiguous once sorted by cell.
__device__ __forceinline__ int cell_id(const Boxes &bx, int b, int cx, int cy, int cz)
{
    const int *g = bx.tile + 8 * b;  // tx ty tz gx gy gz tile_cells mode
    int tx = g[0], ty = g[1], tz = g[2], gx = g[3], gy = g[4], tc = g[6];
    int Tx = cx / tx, Ty = cy / ty, Tz = cz / tz;
    int lx = cx - Tx * tx, ly = cy - Ty * ty, lz = cz - Tz * tz;
    return bx.cell_off[b] + ((Tz * gy + Ty) * gx + Tx) * tc + (lz * ty + ly) * tx + lx;
}

// Neighbour-list layout: rows come in groups of four per slot, group-major
// and slot-fastest, so that one 16-byte load returns four neighbours of an
// atom and 64 consecutive slots read 1 KiB contiguously.  The capacity is a
// multiple of four.
__device__ __forceinline__ size_t nl_off(int r, int i, int N)
{
    return (((size_t)(r >> 2) * N + i) << 2) + (r & 3);
}

// Build kernels run unconditionally (gate == nullptr) or only when the device
// rebuild request is set and the step sequence is not halted (inside
// replayed steps).
__device__ __forceinline__ bool skip(const unsigned *gate)
{
    return gate && (gate[1] == 0u || gate[kHaltWord] != 0u);
}

// The step sequence is halted: a list build ran out of capacity.
__device__ __forceinline__ bool halted(const unsigned *flags) { return flags[kHaltWord] != 0u; }

// A list build found a row of `total` entries beyond the capacity (or a tile
// beyond its LDS): record it and halt the step sequence.
__device__ __forceinline__ void raise_overflow(unsigned *flags, unsigned bit, int total)
{
    atomicOr(flags, bit);
    if (total > 0) atomicMax(flags + kMaxRowWord, (unsigned)total);
    atomicOr(flags + kHaltWord, 1u);
}

__device__ __forceinline__ void raise_flags(unsigned *flags, unsigned bad)
{
    if (bad) atomicOr(flags, bad);
}

}  // namespace dev
}  // namespace mdk
