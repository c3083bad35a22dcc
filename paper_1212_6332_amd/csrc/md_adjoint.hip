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
// row of atom i is split over kAdjParts lanes, each lane accumulates its
// share of the row into a private LDS column, the columns of a workgroup are
// summed in lane order, and the workgroup partials by a fixed tree -- a fixed
// order, so results are bitwise reproducible with no floating-point atomics.
// F'(rho) and F''(rho) are re-evaluated from the density once per atom, never
// taken from the forward pass.
#include <hip/hip_runtime.h>

#include <cmath>

#include "md_device.h"
#include "md_internal.h"

namespace mdk {

namespace {

__device__ __forceinline__ double min_image(double d, double L, double invL)
{
    return fma(-L, rint(d * invL), d);
}

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

// Lanes that share the neighbour row of one atom in the coefficient kernel.
constexpr int kAdjParts = 4;

// s_i, lambda_i and F'(rho_i).
__global__ __launch_bounds__(kBlock) void k_adj_s(int N, State st, Boxes bx, NList nl, Pot pot,
                                                  const double *__restrict__ gs,
                                                  const double *__restrict__ e,
                                                  double *__restrict__ sv, double *__restrict__ lam,
                                                  double *__restrict__ fpv)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int b = bx.box_of[i];
    double L = bx.L[b], invL = bx.invL[b];
    const double *gx = gs, *gy = gs + N, *gz = gs + 2 * N;
    double xi = st.x[i], yi = st.y[i], zi = st.z[i];
    double gxi = gx[i], gyi = gy[i], gzi = gz[i];
    unsigned w = (unsigned)nl.count[i];
    int np = (int)(w & 0xffffu), n1 = nl.mn - (int)(w >> 16);
    double s = 0.0;
    for (int n = 0; n < nl.mn; ++n) {
        if (n == np) n = n1;  // skip to the boundary-crossing part of the row
        if (n >= nl.mn) break;
        int j = nl.idx[dev::nl_off(n, i, N)];
        double dx = min_image(st.x[j] - xi, L, invL);
        double dy = min_image(st.y[j] - yi, L, invL);
        double dz = min_image(st.z[j] - zi, L, invL);
        double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        if (r2 >= pot.rc2) continue;
        double r = sqrt(r2);
        double f, df, ddf;
        table_eval2(pot.tab[1], r, f, df, ddf);
        // (g_i - g_j) . u_ij with u_ij = -(dx, dy, dz)/r
        double proj = fma(gzi - gz[j], dz, fma(gyi - gy[j], dy, (gxi - gx[j]) * dx));
        s -= df * proj / r;
    }
    double F, Fp, Fpp;
    table_eval2(pot.tab[2], st.rho[i], F, Fp, Fpp);
    sv[i] = s;
    lam[i] = e[b] * Fp - Fpp * s;
    fpv[i] = Fp;
}

// Coefficient gradients: W lanes per workgroup, each with an LDS column of
// 3K; the kAdjParts lanes of one atom take every kAdjParts-th entry of its
// row, the first of them also the embedding term.
template <int W>
__global__ __launch_bounds__(W) void k_adj_theta(int N, int K, State st, Boxes bx, NList nl,
                                                 Pot pot, const double *__restrict__ gs,
                                                 const double *__restrict__ e,
                                                 const double *__restrict__ sv,
                                                 const double *__restrict__ lam,
                                                 const double *__restrict__ fpv,
                                                 double *__restrict__ partial)
{
    extern __shared__ double acc[];  // [3K][W]
    int lane = threadIdx.x;
    for (int k = 0; k < 3 * K; ++k) acc[k * W + lane] = 0.0;
    int part = lane % kAdjParts;
    int i = blockIdx.x * (W / kAdjParts) + lane / kAdjParts;
    if (i < N) {
        int b = bx.box_of[i];
        double L = bx.L[b], invL = bx.invL[b];
        double eb = e[b];
        const double *gx = gs, *gy = gs + N, *gz = gs + 2 * N;
        double xi = st.x[i], yi = st.y[i], zi = st.z[i];
        double gxi = gx[i], gyi = gy[i], gzi = gz[i];
        double lami = lam[i], fpi = fpv[i];
        unsigned cw = (unsigned)nl.count[i];
        // entries [0, np) and [n1, mn) of the row, numbered q = 0 .. np + ni - 1
        int np = (int)(cw & 0xffffu), ni = (int)(cw >> 16), n1 = nl.mn - ni;
        double bb[4], db[4];
        for (int q = part; q < np + ni; q += kAdjParts) {
            int n = q < np ? q : n1 + (q - np);
            int j = nl.idx[dev::nl_off(n, i, N)];
            double dx = min_image(st.x[j] - xi, L, invL);
            double dy = min_image(st.y[j] - yi, L, invL);
            double dz = min_image(st.z[j] - zi, L, invL);
            double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
            if (r2 >= pot.rc2) continue;
            double r = sqrt(r2);
            double cij = -fma(gzi, dz, fma(gyi, dy, gxi * dx)) / r;
            int m;
            double t;
            locate(pot.tab[0], r, m, t);
            basis(t, pot.tab[0].inv_h, bb, db);
            for (int l = 0; l < 4; ++l)
                acc[(m + l) * W + lane] += fma(0.5 * eb, bb[l], -db[l] * cij);
            locate(pot.tab[1], r, m, t);
            basis(t, pot.tab[1].inv_h, bb, db);
            double w = (fpi + fpv[j]) * cij;
            for (int l = 0; l < 4; ++l)
                acc[(K + m + l) * W + lane] += fma(lami, bb[l], -db[l] * w);
        }
        if (part == 0) {
            int m;
            double t;
            locate(pot.tab[2], st.rho[i], m, t);
            basis(t, pot.tab[2].inv_h, bb, db);
            double si = sv[i];
            for (int l = 0; l < 4; ++l)
                acc[(2 * K + m + l) * W + lane] += fma(eb, bb[l], -db[l] * si);
        }
    }
    __syncthreads();
    for (int k = lane; k < 3 * K; k += W) {
        double s = 0.0;
        for (int l = 0; l < W; ++l) s += acc[k * W + l];
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

// Lanes per workgroup of the coefficient kernel: 3K W doubles must fit in 64 KiB.
int adjoint_lanes(int K)
{
    for (int w = 32; w >= 8; w /= 2)
        if ((size_t)3 * K * w * sizeof(double) <= 65536) return w;
    return 0;
}

// Workgroups of the coefficient kernel.
static int64_t adjoint_blocks(int64_t N, int W) { return (N + W / kAdjParts - 1) / (W / kAdjParts); }

size_t adjoint_scratch_doubles(int64_t N, int K)
{
    int w = adjoint_lanes(K);
    if (w == 0) return 0;
    return 6 * (size_t)N + (size_t)adjoint_blocks(N, w) * 3 * (size_t)K;
}

void launch_adjoint(Ctx &c, const double *g, const double *e, double *gtheta, hipStream_t s)
{
    int N = (int)c.N, K = c.n_theta, W = adjoint_lanes(K);
    double *gs = c.adj, *sv = c.adj + 3 * (size_t)N, *lam = c.adj + 4 * (size_t)N;
    double *fpv = c.adj + 5 * (size_t)N, *partial = c.adj + 6 * (size_t)N;
    int blk = atom_block(N), g1 = (N + blk - 1) / blk;
    k_adj_gather<<<g1, blk, 0, s>>>(N, c.st.id, g, gs);
    k_adj_s<<<g1, blk, 0, s>>>(N, c.st, c.bx, c.nl, c.pot, gs, e, sv, lam, fpv);
    int nblk = (int)adjoint_blocks(N, W);
    size_t lds = (size_t)3 * K * W * sizeof(double);
    if (W == 32)
        k_adj_theta<32><<<nblk, 32, lds, s>>>(N, K, c.st, c.bx, c.nl, c.pot, gs, e, sv, lam, fpv, partial);
    else if (W == 16)
        k_adj_theta<16><<<nblk, 16, lds, s>>>(N, K, c.st, c.bx, c.nl, c.pot, gs, e, sv, lam, fpv, partial);
    else
        k_adj_theta<8><<<nblk, 8, lds, s>>>(N, K, c.st, c.bx, c.nl, c.pot, gs, e, sv, lam, fpv, partial);
    k_adj_reduce<<<3 * K, kBlock, 0, s>>>(nblk, 3 * K, partial, gtheta);
}

}  // namespace mdk
