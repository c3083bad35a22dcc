// Form (3): vector-Jacobian product of the forces f_i (eq. 3) and per-box
// energies E_b (eq. 2) with respect to uniform cubic B-spline coefficients
// of V(r) (phi), rho(r) (f) and F(rho).
//
// Varying the three functions at fixed positions in eqs. (2)-(3) gives, with
// u_ij = (x_i - x_j)/r_ij, c_ij = g_i . u_ij, g_i = dL/df_i, e = dL/dE_b:
//   s_i      = sum_j f'(r_ij) (g_i - g_j) . u_ij
//   lambda_i = e F'(rho_i) - F''(rho_i) s_i
//   dL/dphi_k = sum_{i->j} [ e/2 B_k(r) - B'_k(r) c_ij ]
//   dL/df_k   = sum_{i->j} [ lambda_i B_k(r) - (F'_i + F'_j) B'_k(r) c_ij ]
//   dL/dF_k   = sum_i [ e C_k(rho_i) - C'_k(rho_i) s_i ]
// Every term is gathered on the side of atom i (full lists), so no atom
// receives a scatter.  The only reduction is into the 3K coefficients: the
// lanes that share the row of atom i add its terms, in row order, to one LDS
// column per atom, the columns of a workgroup are summed in atom order, and
// the workgroup partials by a fixed tree -- a fixed order, so results are
// bitwise reproducible with no floating-point atomics.
// F'(rho) and F''(rho) are re-evaluated from the density once per atom, never
// taken from the forward pass.
#include <hip/hip_runtime.h>

#include <cmath>

#include "md_device.h"
#include "md_internal.h"

namespace mdk {

namespace {

using dev::min_image;

// Interval m and local t of x on a table grid (same grid as the B-spline).
__device__ __forceinline__ void locate(const Table &t, double x, int &m, double &tt)
{
    double u = (x - t.lo) * t.inv_h;
    int k = (int)floor(u);
    k = k < 0 ? 0 : (k > t.n - 1 ? t.n - 1 : k);
    m = k;
    tt = u - (double)k;
}

// B-spline pieces b_l(t) and db_l/dx = b_l'(t) inv_h on one interval.
__device__ __forceinline__ void basis(double t, double inv_h, double b[4], double db[4])
{
    double s = 1.0 - t;
    b[0] = s * s * s * (1.0 / 6.0);
    b[1] = (t * t * (3.0 * t - 6.0) + 4.0) * (1.0 / 6.0);
    b[2] = (t * (t * (-3.0 * t + 3.0) + 3.0) + 1.0) * (1.0 / 6.0);
    b[3] = t * t * t * (1.0 / 6.0);
    db[0] = -0.5 * s * s * inv_h;
    db[1] = t * (1.5 * t - 2.0) * inv_h;
    db[2] = (t * (-1.5 * t + 1.0) + 0.5) * inv_h;
    db[3] = 0.5 * t * t * inv_h;
}

// Table value, first and second derivative (per-interval cubic).
__device__ __forceinline__ void table_eval2(const Table &t, double x, double &s, double &ds,
                                            double &dds)
{
    int m;
    double tt;
    locate(t, x, m, tt);
    const double *c = t.c + 4 * m;
    s = fma(tt, fma(tt, fma(tt, c[3], c[2]), c[1]), c[0]);
    ds = fma(tt, fma(tt, 3.0 * c[3], 2.0 * c[2]), c[1]) * t.inv_h;
    dds = fma(6.0 * c[3], tt, 2.0 * c[2]) * t.inv_h * t.inv_h;
}

__global__ void k_adj_gather(int N, const int *__restrict__ id, const double *__restrict__ g,
                             double *__restrict__ gs)
{
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N) return;
    size_t o = 3 * (size_t)id[q];
    gs[q] = g[o];
    gs[N + q] = g[o + 1];
    gs[2 * N + q] = g[o + 2];
}

// s_i, lambda_i and F'(rho_i); P lanes share the row of atom i, taking the
// rows congruent to their part modulo P, and are summed by a fixed butterfly.
template <int P>
__global__ __launch_bounds__(kBlock) void k_adj_s(int N, State st, Boxes bx, NList nl, Pot pot,
                                                  const double *__restrict__ gs,
                                                  const double *__restrict__ e,
                                                  double *__restrict__ sv, double *__restrict__ lam,
                                                  double *__restrict__ fpv)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    int i = t / P, part = t % P;
    if (i >= N) return;
    int b = bx.box_of[i];
    double L = bx.L[b], invL = bx.invL[b];
    const double *gx = gs, *gy = gs + N, *gz = gs + 2 * N;
    double xi = st.x[i], yi = st.y[i], zi = st.z[i];
    double gxi = gx[i], gyi = gy[i], gzi = gz[i];
    unsigned w = (unsigned)nl.count[i];
    int np = (int)(w & 0xffffu), n1 = nl.mn - (int)(w >> 16);
    double s = 0.0;
    for (int n = part; n < nl.mn; n += P) {
        if (n >= np && n < n1) n = n1 + ((part - n1) & (P - 1));  // boundary-crossing part
        if (n >= nl.mn) break;
        int j = nl.idx[dev::nl_off(n, i, N)];
        double dx = min_image(st.x[j] - xi, L, invL);
        double dy = min_image(st.y[j] - yi, L, invL);
        double dz = min_image(st.z[j] - zi, L, invL);
        double r2 = dev::dist2(dx, dy, dz);
        if (r2 >= pot.rc2) continue;
        double r = sqrt(r2);
        double f, df, ddf;
        table_eval2(pot.tab[1], r, f, df, ddf);
        // (g_i - g_j) . u_ij with u_ij = -(dx, dy, dz)/r
        double proj = fma(gzi - gz[j], dz, fma(gyi - gy[j], dy, (gxi - gx[j]) * dx));
        s -= df * proj / r;
    }
    for (int o = 1; o < P; o <<= 1) s += __shfl_xor(s, o);
    if (part != 0) return;
    double F, Fp, Fpp;
    table_eval2(pot.tab[2], st.rho[i], F, Fp, Fpp);
    sv[i] = s;
    lam[i] = e[b] * Fp - Fpp * s;
    fpv[i] = Fp;
}

// Coefficient gradients.  A workgroup is one wavefront: A = 64 / P atoms,
// P lanes per atom, one LDS column of 3K per atom.  Lane `part` evaluates the
// entries q = part, part + P, ... of its atom's row; the P lanes then add
// their contributions to the column in P ordered phases, so the column
// receives the row in entry order, exactly as one lane walking the row would.
// Sharing a column keeps the LDS per workgroup small enough for several
// workgroups per compute unit, and P lanes shorten each lane's chain of
// dependent gathers P times.
template <int P>
__global__ __launch_bounds__(64) void k_adj_theta(int N, int K, State st, Boxes bx, NList nl,
                                                  Pot pot, const double *__restrict__ gs,
                                                  const double *__restrict__ e,
                                                  const double *__restrict__ sv,
                                                  const double *__restrict__ lam,
                                                  const double *__restrict__ fpv,
                                                  double *__restrict__ partial)
{
    constexpr int A = 64 / P;
    extern __shared__ double acc[];  // [3K][A]
    const int lane = threadIdx.x, a = lane / P, part = lane % P;
    for (int k = lane; k < 3 * K * A; k += 64) acc[k] = 0.0;
    const int i = blockIdx.x * A + a;
    const bool atom = i < N;
    int cnt = 0, np = 0, n1 = 0, b = 0;
    double L = 1.0, invL = 1.0, eb = 0.0, xi = 0.0, yi = 0.0, zi = 0.0;
    double gxi = 0.0, gyi = 0.0, gzi = 0.0, lami = 0.0, fpi = 0.0;
    if (atom) {
        b = bx.box_of[i];
        L = bx.L[b];
        invL = bx.invL[b];
        eb = e[b];
        xi = st.x[i];
        yi = st.y[i];
        zi = st.z[i];
        gxi = gs[i];
        gyi = gs[N + i];
        gzi = gs[2 * N + i];
        lami = lam[i];
        fpi = fpv[i];
        unsigned cw = (unsigned)nl.count[i];
        // entries [0, np) and [n1, mn) of the row, numbered q = 0 .. np + ni - 1
        np = (int)(cw & 0xffffu);
        int ni = (int)(cw >> 16);
        n1 = nl.mn - ni;
        cnt = np + ni;
    }
    __syncthreads();
    double bb[4], db[4];
    for (int q0 = 0; __syncthreads_or(q0 + part < cnt); q0 += P) {
        const int q = q0 + part;
        bool live = false;
        int m0 = 0, m1 = 0;
        double c0[4], c1[4];
        if (q < cnt) {
            int n = q < np ? q : n1 + (q - np);
            int j = nl.idx[dev::nl_off(n, i, N)];
            double dx = min_image(st.x[j] - xi, L, invL);
            double dy = min_image(st.y[j] - yi, L, invL);
            double dz = min_image(st.z[j] - zi, L, invL);
            double r2 = dev::dist2(dx, dy, dz);
            if (r2 < pot.rc2) {
                live = true;
                double r = sqrt(r2);
                double cij = -fma(gzi, dz, fma(gyi, dy, gxi * dx)) / r;
                double t;
                locate(pot.tab[0], r, m0, t);
                basis(t, pot.tab[0].inv_h, bb, db);
                for (int l = 0; l < 4; ++l) c0[l] = fma(0.5 * eb, bb[l], -db[l] * cij);
                locate(pot.tab[1], r, m1, t);
                basis(t, pot.tab[1].inv_h, bb, db);
                double w = (fpi + fpv[j]) * cij;
                for (int l = 0; l < 4; ++l) c1[l] = fma(lami, bb[l], -db[l] * w);
            }
        }
        for (int ph = 0; ph < P; ++ph) {
            if (live && part == ph) {
                for (int l = 0; l < 4; ++l) acc[(m0 + l) * A + a] += c0[l];
                for (int l = 0; l < 4; ++l) acc[(K + m1 + l) * A + a] += c1[l];
            }
            __syncthreads();
        }
    }
    if (atom && part == 0) {
        int m;
        double t;
        locate(pot.tab[2], st.rho[i], m, t);
        basis(t, pot.tab[2].inv_h, bb, db);
        double si = sv[i];
        for (int l = 0; l < 4; ++l) acc[(2 * K + m + l) * A + a] += fma(eb, bb[l], -db[l] * si);
    }
    __syncthreads();
    for (int k = lane; k < 3 * K; k += 64) {
        double s = 0.0;
        for (int c = 0; c < A; ++c) s += acc[k * A + c];
        partial[(size_t)blockIdx.x * 3 * K + k] = s;
    }
}

// One workgroup per coefficient: lane t sums partials t, t + kBlock, ... in
// order, then the lanes are combined by a fixed tree.
__global__ __launch_bounds__(kBlock) void k_adj_reduce(int nblk, int K3,
                                                       const double *__restrict__ partial,
                                                       double *__restrict__ out)
{
    __shared__ double red[kBlock];
    int k = blockIdx.x, t = threadIdx.x;
    double s = 0.0;
    for (int w = t; w < nblk; w += kBlock) s += partial[(size_t)w * K3 + k];
    red[t] = s;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (t < off) red[t] += red[t + off];
        __syncthreads();
    }
    if (t == 0) out[k] = red[0];
}

}  // namespace

// Lanes per atom of the coefficient kernel: the fewest (at least eight) that
// keep the columns of its 64 / P atoms within 32 KiB of LDS, else one atom
// per workgroup with up to 64 KiB; 0 when even that does not fit.
int adjoint_lanes(int K)
{
    for (int p = 8; p <= 64; p *= 2)
        if ((size_t)3 * K * (64 / p) * sizeof(double) <= 32768) return p;
    return (size_t)3 * K * sizeof(double) <= 65536 ? 64 : 0;
}

// Workgroups of the coefficient kernel.
static int64_t adjoint_blocks(int64_t N, int P) { return (N + 64 / P - 1) / (64 / P); }

size_t adjoint_scratch_doubles(int64_t N, int K)
{
    int p = adjoint_lanes(K);
    if (p == 0) return 0;
    return 6 * (size_t)N + (size_t)adjoint_blocks(N, p) * 3 * (size_t)K;
}

void launch_adjoint(Ctx &c, const double *g, const double *e, double *gtheta, hipStream_t s)
{
    int N = (int)c.N, K = c.n_theta, P = adjoint_lanes(K);
    double *gs = c.adj, *sv = c.adj + 3 * (size_t)N, *lam = c.adj + 4 * (size_t)N;
    double *fpv = c.adj + 5 * (size_t)N, *partial = c.adj + 6 * (size_t)N;
    int blk = atom_block(N), g1 = (N + blk - 1) / blk;
    k_adj_gather<<<g1, blk, 0, s>>>(N, c.st.id, g, gs);
    if (row_lanes(N) == kRowLanes)
        k_adj_s<kRowLanes><<<(int)(((int64_t)N * kRowLanes + blk - 1) / blk), blk, 0, s>>>(
            N, c.st, c.bx, c.nl, c.pot, gs, e, sv, lam, fpv);
    else
        k_adj_s<1><<<g1, blk, 0, s>>>(N, c.st, c.bx, c.nl, c.pot, gs, e, sv, lam, fpv);
    int nblk = (int)adjoint_blocks(N, P);
    size_t lds = (size_t)3 * K * (64 / P) * sizeof(double);
    switch (P) {
    case 8: k_adj_theta<8><<<nblk, 64, lds, s>>>(N, K, c.st, c.bx, c.nl, c.pot, gs, e, sv, lam, fpv, partial); break;
    case 16: k_adj_theta<16><<<nblk, 64, lds, s>>>(N, K, c.st, c.bx, c.nl, c.pot, gs, e, sv, lam, fpv, partial); break;
    case 32: k_adj_theta<32><<<nblk, 64, lds, s>>>(N, K, c.st, c.bx, c.nl, c.pot, gs, e, sv, lam, fpv, partial); break;
    default: k_adj_theta<64><<<nblk, 64, lds, s>>>(N, K, c.st, c.bx, c.nl, c.pot, gs, e, sv, lam, fpv, partial); break;
    }
    k_adj_reduce<<<3 * K, kBlock, 0, s>>>(nblk, 3 * K, partial, gtheta);
}

}  // namespace mdk
