// Adjoint (vector-Jacobian product) of one frozen-link-speed VLBM step
// (arXiv 2609.10639, Sec. III) and of the equilibrium initialisation.
//
// Forward map f^n -> f^{n+1} with c fixed (so no reprojection):
//   W = sum_i f_i; closure and flux Q_alpha(W) (Eq. 10); sensor j_k, s, theta,
//   box filters, beta (Eqs. 28-35, with the global normalisers M_k);
//   f*_i = f_i + 2 beta (f^eq_i(W) - f_i) (Eqs. 20, 22); f^{n+1}_i(x) = f*_i(x - e_i).
// Given lam = dJ/df^{n+1}, the passes below accumulate dJ/df^n:
//   P1  per cell: W, velocity, flux -> scratch; exact grid maxima of |Q_alpha,k|
//   P2  per cell: j_k, s, theta, dilatation, vorticity -> scratch; first
//       maximiser of every |Q_alpha,k| in (alpha, y, x) order
//   P3  per cell: lam* (the transposed streaming of lam), beta, dJ/dbeta,
//       the seeds of the box-filtered activity and Ducros ratio
//   P4  per cell: transposed box filter, derivatives of s and theta, dJ/dj_k,
//       d/ddil, d/dvort; per-block partial sums for dJ/dM_k
//   P5  per cell: transposed central differences -> dJ/dQ and dJ/du, plus the
//       direct equilibrium terms, through the closure -> dJ/dW; lam^n
//   P6  one block: dJ/dM_k added at the first maximiser of each |Q_alpha,k|
// Non-smooth points: d clip/dx = 1 on (0,1), 0 elsewhere; d sqrt(s)/ds := 0 at 0.
// Every neighbour index follows the forward boundary rule (periodic wrap or
// clamped ghost), and each transposed stencil sums over exactly the cells
// whose forward stencil reached the current one.
#include <algorithm>

#include "vlbm_adjoint_math.hpp"
#include "vlbm_aux.hpp"

namespace vlbm {

constexpr int kAdjBlock = 256;

__device__ __forceinline__ int nb1(int i, int d, int n, int lo, int hi)
{
    int j = i + d;
    if (j < 0) return lo == 0 ? j + n : 0;
    if (j >= n) return hi == 0 ? j - n : n - 1;
    return j;
}

template <int D>
struct Geo {
    int nx, ny, bc[4];
    __device__ __forceinline__ int nbx(int x, int d) const { return nb1(x, d, nx, bc[0], bc[1]); }
    __device__ __forceinline__ int nby(int y, int d) const { return D == 2 ? nb1(y, d, ny, bc[2], bc[3]) : y; }
    // cell reached from (x, y) by the offset (ox, oy) under the boundary rule
    __device__ __forceinline__ int cell(int x, int y, int ox, int oy) const
    {
        return nby(y, oy) * nx + nbx(x, ox);
    }
};

template <int D>
__device__ __forceinline__ Geo<D> make_geo(const KParams& p)
{
    Geo<D> g;
    g.nx = p.nx;
    g.ny = p.ny;
    for (int i = 0; i < 4; ++i) g.bc[i] = p.bc[i];
    return g;
}

constexpr int EX[4] = {1, -1, 0, 0};
constexpr int EY[4] = {0, 0, 1, -1};

// scratch field layout (arithmetic type C, ncell each)
//   aux1: Q[a][k] at a*NK+k, then u[a] at D*NK+a          (D*NK + D fields)
//   aux2: j[k] at k, then s, theta, dil, vort              (NK + 4 fields)
//   aux3: seed_s, seed_theta, beta                         (3 fields)
//   aux4: jbar[k] at k, then dilbar, vortbar               (NK + 2 fields)
template <int D>
struct AuxLayout {
    static constexpr int NK = D + 2;
    static constexpr int A1 = 0, N1 = D * NK + D;
    static constexpr int A2 = N1, N2 = NK + 4;
    static constexpr int A3 = A2 + N2, N3 = 3;
    static constexpr int A4 = A3 + N3, N4 = NK + 2;
    static constexpr int TOTAL = A4 + N4;
};

// maximum over the copies of field j of a norms array (kRedCopies copies, kRedStride apart)
__device__ __forceinline__ double norm_max(const double* norms, int j)
{
    double v = norms[j];
    for (int i = 1; i < kRedCopies; ++i) v = fmax(v, norms[i * kRedStride + j]);
    return v;
}

template <typename S, typename C>
__device__ __forceinline__ void load_cell(const S* f, long long plane, int Q, int NK, long long c, C* out)
{
    for (int j = 0; j < Q * NK; ++j) out[j] = (C)f[j * plane + c];
}

// ---------------------------------------------------------------- P1
template <typename S, typename C, int EOS, int D>
__global__ void __launch_bounds__(kAdjBlock) k_adj_p1(KParams p, const S* __restrict__ f, C* __restrict__ aux,
                                                       double* __restrict__ qpart)
{
    using L = AuxLayout<D>;
    constexpr int NK = D + 2, Q = 2 * D;
    const long long ncell = (long long)p.nx * p.ny;
    const Gas<C> g = make_gas<C>(p);
    double mx[4] = {0, 0, 0, 0};
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < ncell;
         c += (long long)gridDim.x * blockDim.x) {
        C fv[16], W[4] = {0, 0, 0, 0};
        load_cell<S, C>(f, p.plane, Q, NK, c, fv);
        for (int i = 0; i < Q; ++i)
            for (int k = 0; k < NK; ++k) W[k] += fv[i * NK + k];
        C u[2], e, P, Qf[2][4];
        closure<C, EOS, D>(g, W, u, e, P, Qf);
        for (int a = 0; a < D; ++a) {
            for (int k = 0; k < NK; ++k) {
                aux[(L::A1 + a * NK + k) * ncell + c] = Qf[a][k];
                mx[k] = fmax(mx[k], (double)fabs(Qf[a][k]));
            }
            aux[(L::A1 + D * NK + a) * ncell + c] = u[a];
        }
    }
    // block maximum into qpart[blockIdx] (no same-address atomics); k_adj_qmax folds the blocks
    __shared__ double sh[kAdjBlock / 64][4];
    for (int k = 0; k < NK; ++k) {
        const double v = wave_max(mx[k]);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < NK) {
        double v = sh[0][threadIdx.x];
        for (int w = 1; w < kAdjBlock / 64; ++w) v = fmax(v, sh[w][threadIdx.x]);
        qpart[blockIdx.x * 4 + threadIdx.x] = v;
    }
}

// qmax[k] = max over the blocks of P1 (one workgroup)
__global__ void __launch_bounds__(kAdjBlock) k_adj_qmax(int NK, int nparts, const double* __restrict__ qpart,
                                                         double* __restrict__ qmax)
{
    __shared__ double sh[4][kAdjBlock];
    double acc[4] = {0, 0, 0, 0};
    for (int b = threadIdx.x; b < nparts; b += kAdjBlock)
        for (int k = 0; k < NK; ++k) acc[k] = fmax(acc[k], qpart[b * 4 + k]);
    for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = kAdjBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = fmax(sh[k][threadIdx.x], sh[k][threadIdx.x + s]);
        __syncthreads();
    }
    if ((int)threadIdx.x < NK) qmax[threadIdx.x] = sh[threadIdx.x][0];
}

// ---------------------------------------------------------------- P2
template <typename C, int D, int SENSOR>
__global__ void __launch_bounds__(kAdjBlock) k_adj_p2(KParams p, const double* __restrict__ norms, C* __restrict__ aux,
                                                       const double* __restrict__ qmax,
                                                       unsigned long long* __restrict__ argmax)
{
    using L = AuxLayout<D>;
    constexpr int NK = D + 2;
    const Geo<D> G = make_geo<D>(p);
    const long long ncell = (long long)p.nx * p.ny;
    const C inv2c = (C)(0.5 / p.c_fixed);   // the gate's differences in lattice units (dt = dx/c)
    C invM[4];
    for (int k = 0; k < NK; ++k) {
        const double M = norm_max(norms, 1 + k);
        invM[k] = M > 0.0 ? (C)(1.0 / M) : (C)0;
    }
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < ncell;
         c += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(c % p.nx), y = (int)(c / p.nx);
        // first maximiser of |Q_alpha,k| in (alpha, y, x) order
        for (int a = 0; a < D; ++a)
            for (int k = 0; k < NK; ++k)
                if ((double)fabs(aux[(L::A1 + a * NK + k) * ncell + c]) == qmax[k])
                    atomicMin(&argmax[k], (unsigned long long)(a * ncell + c));
        C acc = 0;
        for (int k = 0; k < NK; ++k) {
            C j = 0;
            for (int a = 0; a < D; ++a) {
                const int cp = G.cell(x, y, EX[2 * a], EY[2 * a]), cm = G.cell(x, y, -EX[2 * a], -EY[2 * a]);
                j += (C)0.5 * (aux[(L::A1 + a * NK + k) * ncell + cp] - aux[(L::A1 + a * NK + k) * ncell + cm]);
            }
            aux[(L::A2 + k) * ncell + c] = j;
            const C sh = j * invM[k];
            acc += sh * sh;
        }
        const C s = acc > (C)0 ? sqrt(acc / (C)NK) : (C)0;
        C th = 0, dil = 0, vort = 0;
        if constexpr (SENSOR == 2 && D == 2) {
            const C* ux = aux + (L::A1 + D * NK + 0) * ncell;
            const C* uy = aux + (L::A1 + D * NK + 1) * ncell;
            const int xp = G.cell(x, y, 1, 0), xm = G.cell(x, y, -1, 0), yp = G.cell(x, y, 0, 1), ym = G.cell(x, y, 0, -1);
            dil = (ux[xp] - ux[xm]) * inv2c + (uy[yp] - uy[ym]) * inv2c;
            vort = (uy[xp] - uy[xm]) * inv2c - (ux[yp] - ux[ym]) * inv2c;
            th = dil * dil / (dil * dil + vort * vort + (C)p.eps_theta);
        }
        aux[(L::A2 + NK + 0) * ncell + c] = s;
        aux[(L::A2 + NK + 1) * ncell + c] = th;
        aux[(L::A2 + NK + 2) * ncell + c] = dil;
        aux[(L::A2 + NK + 3) * ncell + c] = vort;
    }
}

// separable (1/4, 1/2, 1/4) filter of field `a` at (x, y), boundary rule applied
template <typename C, int D>
__device__ __forceinline__ C box_at(const Geo<D>& G, const C* a, int x, int y)
{
    auto sx = [&](int yy) {
        return (C)0.25 * a[yy * G.nx + G.nbx(x, -1)] + (C)0.5 * a[yy * G.nx + x] + (C)0.25 * a[yy * G.nx + G.nbx(x, 1)];
    };
    if (D == 1) return sx(y);
    return (C)0.25 * sx(G.nby(y, -1)) + (C)0.5 * sx(y) + (C)0.25 * sx(G.nby(y, 1));
}

// transposed filter: sum over the cells whose filter reached (x, y)
template <typename C, int D>
__device__ __forceinline__ C box_t_at(const Geo<D>& G, const C* a, int x, int y)
{
    auto wx = [&](int from, int to) {   // weight of column `to` in the x-filter at column `from`
        return (G.nbx(from, -1) == to ? (C)0.25 : (C)0) + (from == to ? (C)0.5 : (C)0) +
               (G.nbx(from, 1) == to ? (C)0.25 : (C)0);
    };
    auto wy = [&](int from, int to) {
        return (G.nby(from, -1) == to ? (C)0.25 : (C)0) + (from == to ? (C)0.5 : (C)0) +
               (G.nby(from, 1) == to ? (C)0.25 : (C)0);
    };
    C acc = 0;
    const int dys = D == 2 ? 1 : 0;
    // candidate rows/columns: every cell whose stencil can reach (x, y); with
    // wrap-around on tiny periodic grids the same cell may appear twice, so
    // candidates are de-duplicated
    int xs[3], ys[3], nxs = 0, nys = 0;
    for (int d = -1; d <= 1; ++d) {
        const int cxx = (x + d + G.nx) % G.nx;
        bool dup = false;
        for (int q = 0; q < nxs; ++q) dup |= xs[q] == cxx;
        if (!dup) xs[nxs++] = cxx;
    }
    for (int d = -dys; d <= dys; ++d) {
        const int cyy = D == 2 ? (y + d + G.ny) % G.ny : y;
        bool dup = false;
        for (int q = 0; q < nys; ++q) dup |= ys[q] == cyy;
        if (!dup) ys[nys++] = cyy;
    }
    for (int qy = 0; qy < nys; ++qy) {
        const C wyv = D == 2 ? wy(ys[qy], y) : (C)1;
        if (wyv == (C)0) continue;
        for (int qx = 0; qx < nxs; ++qx) {
            const C wxv = wx(xs[qx], x);
            if (wxv != (C)0) acc += wyv * wxv * a[ys[qy] * G.nx + xs[qx]];
        }
    }
    return acc;
}

// lam*_i(x,y) = sum of lam_i over the cells whose streaming source is (x, y)
template <typename S, typename C, int D>
__device__ __forceinline__ C lam_star(const Geo<D>& G, const S* lam, long long plane, int i, int k, int x, int y)
{
    constexpr int NK = D + 2;
    const int ex = EX[i], ey = EY[i];
    C acc = 0;
    // candidates x' = x + d*ex, y' = y + d*ey for d in {-1, 0, 1}; source of x' is nb(x', -e_i)
    int seen[3], ns = 0;
    for (int d = -1; d <= 1; ++d) {
        int xx = x + d * ex, yy = y + d * ey;
        if (ex) xx = (xx + G.nx) % G.nx;
        if (ey) yy = (yy + G.ny) % G.ny;
        const int cc = yy * G.nx + xx;
        bool dup = false;
        for (int q = 0; q < ns; ++q) dup |= seen[q] == cc;
        if (dup) continue;
        seen[ns++] = cc;
        if (G.cell(xx, yy, -ex, -ey) == y * G.nx + x) acc += (C)lam[(long long)(i * NK + k) * plane + cc];
    }
    return acc;
}

// transposed central difference along axis (ax, ay): sum over cells z with
// nb(z, +e) == w of a(z), minus the same for nb(z, -e) == w
template <typename C, int D>
__device__ __forceinline__ C diff_t(const Geo<D>& G, const C* a, int x, int y, int ex, int ey)
{
    C acc = 0;
    int seen[3], ns = 0;
    const int w = y * G.nx + x;
    for (int d = -1; d <= 1; ++d) {
        int xx = x + d * ex, yy = y + d * ey;
        if (ex) xx = (xx + G.nx) % G.nx;
        if (ey) yy = (yy + G.ny) % G.ny;
        const int cc = yy * G.nx + xx;
        bool dup = false;
        for (int q = 0; q < ns; ++q) dup |= seen[q] == cc;
        if (dup) continue;
        seen[ns++] = cc;
        if (G.cell(xx, yy, ex, ey) == w) acc += a[cc];
        if (G.cell(xx, yy, -ex, -ey) == w) acc -= a[cc];
    }
    return acc;
}

// ---------------------------------------------------------------- P3
template <typename S, typename C, int EOS, int D, int SENSOR>
__global__ void __launch_bounds__(kAdjBlock) k_adj_p3(KParams p, const S* __restrict__ f, const S* __restrict__ lam,
                                                       C* __restrict__ aux)
{
    using L = AuxLayout<D>;
    constexpr int NK = D + 2, Q = 2 * D;
    const Geo<D> G = make_geo<D>(p);
    const long long ncell = (long long)p.nx * p.ny;
    const C inv2c = (C)(0.5 / p.c_fixed);
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < ncell;
         c += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(c % p.nx), y = (int)(c / p.nx);
        C beta = (C)p.beta_const, sbar = 0, thbar = 1, X = 0;
        if constexpr (SENSOR != 0) {
            sbar = box_at<C, D>(G, aux + (L::A2 + NK + 0) * ncell, x, y);
            if constexpr (SENSOR == 2 && D == 2) thbar = box_at<C, D>(G, aux + (L::A2 + NK + 1) * ncell, x, y);
            X = (C)p.c_sensor * sbar * thbar;
            const C chi = X < (C)0 ? (C)0 : (X > (C)1 ? (C)1 : X);
            beta = (C)p.beta_max - (C)(p.beta_max - p.beta_min) * chi;
        }
        C seed_s = 0, seed_t = 0;
        if constexpr (SENSOR != 0) {
            if (X > (C)0 && X < (C)1) {
                C fv[16], W[4] = {0, 0, 0, 0};
                load_cell<S, C>(f, p.plane, Q, NK, c, fv);
                for (int i = 0; i < Q; ++i)
                    for (int k = 0; k < NK; ++k) W[k] += fv[i * NK + k];
                C betabar = 0;
                for (int i = 0; i < Q; ++i) {
                    const int a = i / 2;
                    const C sg = (i & 1) ? (C)-1 : (C)1;
                    for (int k = 0; k < NK; ++k) {
                        const C feq = W[k] / (C)(2 * D) + sg * aux[(L::A1 + a * NK + k) * ncell + c] * inv2c;
                        betabar += (C)2 * (feq - fv[i * NK + k]) * lam_star<S, C, D>(G, lam, p.plane, i, k, x, y);
                    }
                }
                const C chibar = -(C)(p.beta_max - p.beta_min) * betabar;
                seed_s = (C)p.c_sensor * thbar * chibar;
                seed_t = (C)p.c_sensor * sbar * chibar;
            }
        }
        aux[(L::A3 + 0) * ncell + c] = seed_s;
        aux[(L::A3 + 1) * ncell + c] = seed_t;
        aux[(L::A3 + 2) * ncell + c] = beta;
    }
}

// ---------------------------------------------------------------- P4
template <typename C, int D, int SENSOR>
__global__ void __launch_bounds__(kAdjBlock) k_adj_p4(KParams p, const double* __restrict__ norms, C* __restrict__ aux,
                                                       double* __restrict__ partials)
{
    using L = AuxLayout<D>;
    constexpr int NK = D + 2;
    const Geo<D> G = make_geo<D>(p);
    const long long ncell = (long long)p.nx * p.ny;
    C invM[4];
    for (int k = 0; k < NK; ++k) {
        const double M = norm_max(norms, 1 + k);
        invM[k] = M > 0.0 ? (C)(1.0 / M) : (C)0;
    }
    C mpart[4] = {0, 0, 0, 0};
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < ncell;
         c += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(c % p.nx), y = (int)(c / p.nx);
        C jb[4] = {0, 0, 0, 0}, dilb = 0, vortb = 0;
        if constexpr (SENSOR != 0) {
            const C sadj = box_t_at<C, D>(G, aux + (L::A3 + 0) * ncell, x, y);
            const C s = aux[(L::A2 + NK + 0) * ncell + c];
            if (s > (C)0) {
                for (int k = 0; k < NK; ++k) {
                    const C shat = aux[(L::A2 + k) * ncell + c] * invM[k];
                    const C shbar = sadj * shat / ((C)NK * s);   // d s / d s_hat_k = s_hat_k/(NK s)
                    jb[k] = shbar * invM[k];
                    mpart[k] -= shbar * shat * invM[k];            // d s_hat_k / d M_k = -s_hat_k/M_k
                }
            }
            if constexpr (SENSOR == 2 && D == 2) {
                const C tadj = box_t_at<C, D>(G, aux + (L::A3 + 1) * ncell, x, y);
                const C dil = aux[(L::A2 + NK + 2) * ncell + c], vort = aux[(L::A2 + NK + 3) * ncell + c];
                const C den = dil * dil + vort * vort + (C)p.eps_theta;
                const C iden2 = (C)1 / (den * den);
                dilb = tadj * (C)2 * dil * (vort * vort + (C)p.eps_theta) * iden2;
                vortb = -tadj * (C)2 * vort * dil * dil * iden2;
            }
        }
        for (int k = 0; k < NK; ++k) aux[(L::A4 + k) * ncell + c] = jb[k];
        aux[(L::A4 + NK + 0) * ncell + c] = dilb;
        aux[(L::A4 + NK + 1) * ncell + c] = vortb;
    }
    // fixed-order block reduction of the normaliser adjoint partial sums
    __shared__ double sh[4][kAdjBlock];
    for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = (double)mpart[k];
    __syncthreads();
    for (int s = kAdjBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; ++k) partials[blockIdx.x * 4 + k] = sh[k][0];
}

// ---------------------------------------------------------------- P5
template <typename S, typename C, int EOS, int D, int SENSOR>
__global__ void __launch_bounds__(kAdjBlock) k_adj_p5(KParams p, const S* __restrict__ f, const S* __restrict__ lam,
                                                       const C* __restrict__ aux, S* __restrict__ lam_out)
{
    using L = AuxLayout<D>;
    constexpr int NK = D + 2, Q = 2 * D;
    const Geo<D> G = make_geo<D>(p);
    const long long ncell = (long long)p.nx * p.ny;
    const Gas<C> g = make_gas<C>(p);
    const C inv2c = (C)(0.5 / p.c_fixed);
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < ncell;
         c += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(c % p.nx), y = (int)(c / p.nx);
        const C beta = aux[(L::A3 + 2) * ncell + c];
        C fv[16], W[4] = {0, 0, 0, 0}, ls[16];
        load_cell<S, C>(f, p.plane, Q, NK, c, fv);
        for (int i = 0; i < Q; ++i)
            for (int k = 0; k < NK; ++k) {
                W[k] += fv[i * NK + k];
                ls[i * NK + k] = lam_star<S, C, D>(G, lam, p.plane, i, k, x, y);
            }
        // direct terms of the equilibrium: f^eq_i = W/(2D) + sign_i Q_a/(2c)
        C Wb[4] = {0, 0, 0, 0}, Qb[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}}, ub[2] = {0, 0};
        const C tb = (C)2 * beta;
        for (int k = 0; k < NK; ++k) {
            C sum = 0;
            for (int i = 0; i < Q; ++i) sum += ls[i * NK + k];
            Wb[k] = tb * sum / (C)(2 * D);
            for (int a = 0; a < D; ++a) Qb[a][k] = tb * (ls[(2 * a) * NK + k] - ls[(2 * a + 1) * NK + k]) * inv2c;
        }
        // sensor terms: transposed central differences of jbar, dilbar, vortbar
        if constexpr (SENSOR != 0) {
            for (int a = 0; a < D; ++a)
                for (int k = 0; k < NK; ++k)
                    Qb[a][k] += (C)0.5 * diff_t<C, D>(G, aux + (L::A4 + k) * ncell, x, y, EX[2 * a], EY[2 * a]);
            if constexpr (SENSOR == 2 && D == 2) {
                const C* dilb = aux + (L::A4 + NK + 0) * ncell;
                const C* vortb = aux + (L::A4 + NK + 1) * ncell;
                ub[0] = (diff_t<C, D>(G, dilb, x, y, 1, 0) - diff_t<C, D>(G, vortb, x, y, 0, 1)) * inv2c;
                ub[1] = (diff_t<C, D>(G, dilb, x, y, 0, 1) + diff_t<C, D>(G, vortb, x, y, 1, 0)) * inv2c;
            }
        }
        closure_adj<C, EOS, D>(g, W, Qb, ub, Wb);
        for (int i = 0; i < Q; ++i)
            for (int k = 0; k < NK; ++k)
                lam_out[(long long)(i * NK + k) * p.plane + c] = (S)(((C)1 - tb) * ls[i * NK + k] + Wb[k]);
    }
}

// ---------------------------------------------------------------- P6
template <typename S, typename C, int EOS, int D>
__global__ void __launch_bounds__(kAdjBlock) k_adj_p6(KParams p, const S* __restrict__ f, const double* __restrict__ partials, int nparts,
                         const unsigned long long* __restrict__ argmax, S* __restrict__ lam_out)
{
    constexpr int NK = D + 2, Q = 2 * D;
    // M-bar_k = sum of the P4 block partials: fixed assignment to threads and a
    // fixed tree, so the sum is deterministic
    __shared__ double sh[4][kAdjBlock];
    {
        double acc[4] = {0, 0, 0, 0};
        for (int b = threadIdx.x; b < nparts; b += kAdjBlock)
            for (int k = 0; k < NK; ++k) acc[k] += partials[b * 4 + k];
        for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = acc[k];
        __syncthreads();
        for (int s = kAdjBlock / 2; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s)
                for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
            __syncthreads();
        }
    }
    if (threadIdx.x != 0) return;
    const long long ncell = (long long)p.nx * p.ny;
    const Gas<C> g = make_gas<C>(p);
    for (int k = 0; k < NK; ++k) {
        const double Mb = sh[k][0];
        if (Mb == 0.0 || argmax[k] == ~0ull) continue;
        const int a = (int)(argmax[k] / (unsigned long long)ncell);
        const long long c = (long long)(argmax[k] % (unsigned long long)ncell);
        C fv[16], W[4] = {0, 0, 0, 0};
        load_cell<S, C>(f, p.plane, Q, NK, c, fv);
        for (int i = 0; i < Q; ++i)
            for (int kk = 0; kk < NK; ++kk) W[kk] += fv[i * NK + kk];
        C u[2], e, P, Qf[2][4];
        closure<C, EOS, D>(g, W, u, e, P, Qf);
        C Qb[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}}, ub[2] = {0, 0}, Wb[4] = {0, 0, 0, 0};
        Qb[a][k] = (C)Mb * (Qf[a][k] > (C)0 ? (C)1 : (Qf[a][k] < (C)0 ? (C)-1 : (C)0));
        closure_adj<C, EOS, D>(g, W, Qb, ub, Wb);
        for (int i = 0; i < Q; ++i)
            for (int kk = 0; kk < NK; ++kk) {
                S* dst = lam_out + (long long)(i * NK + kk) * p.plane + c;
                *dst = (S)((C)*dst + Wb[kk]);
            }
    }
}

__global__ void k_adj_reset(double* qmax, unsigned long long* argmax)
{
    if (threadIdx.x < 4) {
        qmax[threadIdx.x] = 0.0;
        argmax[threadIdx.x] = ~0ull;
    }
}

// ---------------------------------------------------------------- init adjoint
// W0bar = (d f^eq(W0; c)/d W0)^T lam0 = sum_i lam0_i/(2D) + closure adjoint of
// Qbar_a = (lam0_{a+} - lam0_{a-})/(2c).
template <typename S, typename C, int EOS, int D>
__global__ void k_init_adj(KParams p, const double* __restrict__ W0, const S* __restrict__ lam0,
                           double* __restrict__ W0bar)
{
    constexpr int NK = D + 2, Q = 2 * D;
    const long long ncell = (long long)p.nx * p.ny;
    const Gas<C> g = make_gas<C>(p);
    const C inv2c = (C)(0.5 / p.c_fixed);
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < ncell;
         c += (long long)gridDim.x * blockDim.x) {
        C W[4], Wb[4] = {0, 0, 0, 0}, Qb[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}}, ub[2] = {0, 0};
        for (int k = 0; k < NK; ++k) W[k] = (C)W0[k * ncell + c];
        for (int k = 0; k < NK; ++k) {
            C sum = 0;
            for (int i = 0; i < Q; ++i) sum += (C)lam0[(long long)(i * NK + k) * p.plane + c];
            Wb[k] = sum / (C)(2 * D);
            for (int a = 0; a < D; ++a)
                Qb[a][k] = ((C)lam0[(long long)((2 * a) * NK + k) * p.plane + c] -
                            (C)lam0[(long long)((2 * a + 1) * NK + k) * p.plane + c]) * inv2c;
        }
        closure_adj<C, EOS, D>(g, W, Qb, ub, Wb);
        for (int k = 0; k < NK; ++k) W0bar[k * ncell + c] = (double)Wb[k];
    }
}

// ---------------------------------------------------------------- launchers

size_t adjoint_partials_count(const KParams& p)
{
    long long n = ((long long)p.nx * p.ny + kAdjBlock - 1) / kAdjBlock;
    return (size_t)(n > 2048 ? 2048 : n);
}

size_t adjoint_aux_elems(const KParams& p)
{
    return (size_t)AuxLayout<2>::TOTAL * (size_t)p.nx * (size_t)p.ny;
}

template <typename S, typename C, int EOS, int D, int SENSOR>
static hipError_t adj_t(const KParams& p, const void* f_n, const double* norms, const void* lam_np1, void* lam_n,
                        const AdjScratch& sc, hipStream_t st)
{
    const int nb = (int)adjoint_partials_count(p);
    const S* f = (const S*)f_n;
    const S* lam = (const S*)lam_np1;
    S* lo = (S*)lam_n;
    C* aux = (C*)sc.aux;
    hipLaunchKernelGGL(k_adj_reset, dim3(1), dim3(64), 0, st, sc.qmax, sc.argmax);
    // P1 block maxima go through the partials buffer, which P4 reuses afterwards
    hipLaunchKernelGGL((k_adj_p1<S, C, EOS, D>), dim3(nb), dim3(kAdjBlock), 0, st, p, f, aux, sc.partials);
    hipLaunchKernelGGL(k_adj_qmax, dim3(1), dim3(kAdjBlock), 0, st, D + 2, nb, (const double*)sc.partials, sc.qmax);
    hipLaunchKernelGGL((k_adj_p2<C, D, SENSOR>), dim3(nb), dim3(kAdjBlock), 0, st, p, norms, aux,
                       (const double*)sc.qmax, sc.argmax);
    hipLaunchKernelGGL((k_adj_p3<S, C, EOS, D, SENSOR>), dim3(nb), dim3(kAdjBlock), 0, st, p, f, lam, aux);
    hipLaunchKernelGGL((k_adj_p4<C, D, SENSOR>), dim3(nb), dim3(kAdjBlock), 0, st, p, norms, aux, sc.partials);
    hipLaunchKernelGGL((k_adj_p5<S, C, EOS, D, SENSOR>), dim3(nb), dim3(kAdjBlock), 0, st, p, f, lam,
                       (const C*)aux, lo);
    if (SENSOR != 0)
        hipLaunchKernelGGL((k_adj_p6<S, C, EOS, D>), dim3(1), dim3(kAdjBlock), 0, st, p, f, (const double*)sc.partials, nb,
                           (const unsigned long long*)sc.argmax, lo);
    return hipGetLastError();
}

template <typename S, typename C>
static hipError_t adj_prec(const KParams& p, const void* f_n, const double* norms, const void* lam_np1, void* lam_n,
                           const AdjScratch& sc, hipStream_t st)
{
#define VLBM_ADJ(E, DD, SN)                                                                           \
    if (p.eos == E && p.dim == DD && p.sensor == SN)                                                 \
        return adj_t<S, C, E, DD, SN>(p, f_n, norms, lam_np1, lam_n, sc, st);
    VLBM_ADJ(0, 2, 0) VLBM_ADJ(0, 2, 1) VLBM_ADJ(0, 2, 2) VLBM_ADJ(1, 2, 0) VLBM_ADJ(1, 2, 1) VLBM_ADJ(1, 2, 2)
    VLBM_ADJ(0, 1, 0) VLBM_ADJ(0, 1, 1) VLBM_ADJ(1, 1, 0) VLBM_ADJ(1, 1, 1)
#undef VLBM_ADJ
    return hipErrorInvalidValue;
}

hipError_t launch_adjoint_step(const KParams& p, int prec, const void* f_n, const double* norms_n,
                               const void* lam_np1, void* lam_n, const AdjScratch& sc, hipStream_t st)
{
    switch (prec) {
    case PREC_FP64: return adj_prec<double, double>(p, f_n, norms_n, lam_np1, lam_n, sc, st);
    case PREC_FP32: return adj_prec<float, float>(p, f_n, norms_n, lam_np1, lam_n, sc, st);
    case PREC_FP32_MIXED: return adj_prec<float, double>(p, f_n, norms_n, lam_np1, lam_n, sc, st);
    }
    return hipErrorInvalidValue;
}

template <typename S, typename C>
static hipError_t init_adj_prec(const KParams& p, const double* W0, long long ncell, const void* lam0, double* W0bar,
                                hipStream_t st)
{
    const unsigned grid = (unsigned)std::min<long long>((ncell + 255) / 256, 4096);
#define VLBM_IADJ(E, DD)                                                                                       \
    if (p.eos == E && p.dim == DD) {                                                                           \
        hipLaunchKernelGGL((k_init_adj<S, C, E, DD>), dim3(grid), dim3(256), 0, st, p, W0, (const S*)lam0, W0bar); \
        return hipGetLastError();                                                                              \
    }
    VLBM_IADJ(0, 2) VLBM_IADJ(1, 2) VLBM_IADJ(0, 1) VLBM_IADJ(1, 1)
#undef VLBM_IADJ
    return hipErrorInvalidValue;
}

hipError_t launch_init_adjoint(const KParams& p, int prec, const double* W0, long long ncell, const void* lam0,
                               double* W0bar, hipStream_t st)
{
    switch (prec) {
    case PREC_FP64: return init_adj_prec<double, double>(p, W0, ncell, lam0, W0bar, st);
    case PREC_FP32: return init_adj_prec<float, float>(p, W0, ncell, lam0, W0bar, st);
    case PREC_FP32_MIXED: return init_adj_prec<float, double>(p, W0, ncell, lam0, W0bar, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace vlbm
