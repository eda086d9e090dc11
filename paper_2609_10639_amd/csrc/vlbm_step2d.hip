// Fused D2Q4 VLBM time step for gfx950 (arXiv 2609.10639, Sec. III).
//
// One wavefront owns a strip of 58 output columns and marches up a segment of
// rows.  Its 64 lanes hold 64 consecutive columns (3 halo columns on each
// side); x-neighbour values move between lanes through the LDS crossbar
// (ds_bpermute), y-neighbour values are the previous rows kept in registers.
// For the row R entering the strip the pipeline runs, within one iteration:
//   A  row R    load the 16 populations (SoA planes, coalesced), reproject to
//               the new link speed (Eqs. 38-40), moments W, primitives, EOS
//               pressure, flux Q_x, Q_y (Eq. 10), x-parts of the central
//               differences of Q and u;
//   B  row R-1  flux-divergence jump j_k (Eqs. 28-29), normalised activity s
//               (Eqs. 30-31), Ducros ratio theta (Eqs. 32-33), x-pass of the box filter;
//   C  row R-2  y-pass of the box filter, beta (Eqs. 34-35), over-relaxation
//               towards the vector equilibrium (Eqs. 20, 22);
//   D  row R-3  pull-streaming (Eq. 21) of the four directions into the new
//               populations, store, and the reductions of the new state
//               (s_max of Eq. 36, M_k of Eq. 30) that the next step needs.
// Every population is read once and written once per step; halo rows and
// columns are re-read from L2.
#include "vlbm_common.hpp"

namespace vlbm {

constexpr int kStripW = 58;  // output columns per wavefront (64 lanes - 2*3 halo)

template <typename T>
__device__ __forceinline__ T shfl(T v, int src)
{
    return __shfl(v, src, 64);
}

template <typename T>
__device__ __forceinline__ void reproject4(T* f, T r)
{
    // Eq. 40 with J_alpha = c_old (f_alpha+ - f_alpha-) and K = c_old^2 (S_x - S_y)
    // held fixed, in terms of r = c_old/c_new, for each component k.
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const T sx = f[0 * 4 + k] + f[1 * 4 + k], dxv = f[0 * 4 + k] - f[1 * 4 + k];
        const T sy = f[2 * 4 + k] + f[3 * 4 + k], dyv = f[2 * 4 + k] - f[3 * 4 + k];
        const T w = sx + sy;
        const T kk = r * r * (sx - sy);
        const T a = (T)0.25 * (w + kk), b = (T)0.25 * (w - kk);
        const T hx = (T)0.5 * r * dxv, hy = (T)0.5 * r * dyv;
        f[0 * 4 + k] = a + hx;
        f[1 * 4 + k] = a - hx;
        f[2 * 4 + k] = b + hy;
        f[3 * 4 + k] = b - hy;
    }
}

// W, velocity, pressure and the two directional fluxes of one cell.
template <typename T, int EOS>
__device__ __forceinline__ void cell_flux(const Gas<T>& g, const T* f, T* W, T& ux, T& uy, T& e, T* qx, T* qy)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) W[k] = (f[0 * 4 + k] + f[1 * 4 + k]) + (f[2 * 4 + k] + f[3 * 4 + k]);
    const T irho = (T)1 / W[0];
    ux = W[1] * irho;
    uy = W[2] * irho;
    e = W[3] * irho - (T)0.5 * (ux * ux + uy * uy);
    const T P = eos_pressure<T, EOS>(g, W[0], e);
    const T h = W[3] + P;
    qx[0] = W[1];
    qx[1] = W[1] * ux + P;
    qx[2] = W[1] * uy;
    qx[3] = h * ux;
    qy[0] = W[2];
    qy[1] = W[2] * ux;
    qy[2] = W[2] * uy + P;
    qy[3] = h * uy;
}

template <typename T, int EOS, int SENSOR>
__global__ void __launch_bounds__(64) k_step_d2q4(const KParams P, const KStep S, const T* __restrict__ fin,
                                                  T* __restrict__ fout)
{
    double c_old, c_new, t, dt;
    bool last;
    if (!step_clock(P, S, c_old, c_new, t, dt, last)) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) write_clock(S, t, dt, c_new, last);

    const Gas<T> g = make_gas<T>(P);
    const bool reproj = (c_old != c_new);
    const T r = (T)(c_old / c_new);
    const T inv2c = (T)(0.5 / c_new);
    T invM[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double M = S.red_in[1 + k];
        invM[k] = M > 0.0 ? (T)(1.0 / M) : (T)0;
    }
    const T inv2dx = (T)(0.5 / P.dx);
    const T bmin = (T)P.beta_min, bmax = (T)P.beta_max, csen = (T)P.c_sensor, eps = (T)P.eps_theta;
    const T bconst = (T)P.beta_const;

    const int nx = P.nx, ny = P.ny;
    const long long plane = P.plane;
    const int lane = threadIdx.x;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int strip = tile % P.nstrips, seg = tile / P.nstrips;
    const int X = strip * kStripW - 3 + lane;
    int cx = X;
    if (X < 0) cx = P.bc[0] == 0 ? wrap_index(X, nx) : 0;
    else if (X >= nx) cx = P.bc[1] == 0 ? wrap_index(X, nx) : nx - 1;
    int lnb = lane - 1, rnb = lane + 1;
    if (P.bc[0] == 1 && X == 0) lnb = lane;
    if (P.bc[1] == 1 && X == nx - 1) rnb = lane;
    lnb = max(lnb, 0);
    rnb = min(rnb, 63);
    const bool owner = lane >= 3 && lane < 3 + kStripW && X < nx;

    const bool clo = P.bc[2] == 1, chi = P.bc[3] == 1;
    const int y0 = seg * P.seg_h;
    const int y1 = min(y0 + P.seg_h, ny);
    const int Rb = clo ? max(y0 - 3, 0) : y0 - 3;
    const int Re = chi ? min(y1 + 2, ny - 1) : y1 + 2;

    // row histories (see the file header for the pipeline)
    T f1[16], f2[16];            // reprojected populations, rows R-1, R-2
    T qy1[4], qy2[4];            // Q_y, rows R-1, R-2
    T ux1 = 0, uy1 = 0, ux2 = 0, uy2 = 0;
    T jx1[4], dil1 = 0, vor1 = 0;  // x-parts of j_k, dilatation, vorticity, row R-1
    T ss2 = 0, st2 = 0, ss3 = 0, st3 = 0;  // S_x[s], S_x[theta], rows R-2, R-3
    T xp1[4], xm1[4];            // populations arriving from -x / +x neighbours, row R-3
    T yp1[4], yp2[4];            // f*_{+y}, rows R-3, R-4
    T ym1[4];                    // f*_{-y}, row R-3
#pragma unroll
    for (int j = 0; j < 16; ++j) f1[j] = f2[j] = (T)0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        qy1[k] = qy2[k] = jx1[k] = xp1[k] = xm1[k] = yp1[k] = yp2[k] = ym1[k] = (T)0;
    }

    double red_s = 0.0, red_M[4] = {0.0, 0.0, 0.0, 0.0};
    int errbits = 0;

    for (int R = Rb; R <= y1 + 2; ++R) {
        // ---------------- stage A: row R
        T fa[16], qya[4], jxa[4];
        T uxa = 0, uya = 0, dila = 0, vora = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) qya[k] = jxa[k] = (T)0;
#pragma unroll
        for (int j = 0; j < 16; ++j) fa[j] = (T)0;
        if (R <= Re) {
            const int mrow = (R < 0 || R >= ny) ? wrap_index(R, ny) : R;
            const long long base = (long long)mrow * nx + cx;
#pragma unroll
            for (int j = 0; j < 16; ++j) fa[j] = fin[j * plane + base];
            if (reproj) reproject4(fa, r);
            if constexpr (SENSOR != 0) {
                T W[4], qxa[4], e;
                cell_flux<T, EOS>(g, fa, W, uxa, uya, e, qxa, qya);
#pragma unroll
                for (int k = 0; k < 4; ++k) jxa[k] = (T)0.5 * (shfl(qxa[k], rnb) - shfl(qxa[k], lnb));
                if constexpr (SENSOR == 2) {
                    dila = (shfl(uxa, rnb) - shfl(uxa, lnb)) * inv2dx;   // d u_x / dx
                    vora = (shfl(uya, rnb) - shfl(uya, lnb)) * inv2dx;   // d u_y / dx
                }
            }
        }

        // ---------------- stage B: row q = R-1
        const int q = R - 1;
        T ssq = 0, stq = 0;
        if constexpr (SENSOR != 0) {
            if (q >= Rb && q <= Re) {
                const bool qlo = clo && q == 0, qhi = chi && q == ny - 1;
                T acc = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const T qn = qhi ? qy1[k] : qya[k];
                    const T qp = qlo ? qy1[k] : qy2[k];
                    const T jk = jx1[k] + (T)0.5 * (qn - qp);
                    const T sh = jk * invM[k];
                    acc += sh * sh;
                }
                const T sq = sqrt(acc * (T)0.25);
                ssq = (T)0.25 * shfl(sq, lnb) + (T)0.5 * sq + (T)0.25 * shfl(sq, rnb);
                if constexpr (SENSOR == 2) {
                    const T uxn = qhi ? ux1 : uxa, uxp = qlo ? ux1 : ux2;
                    const T uyn = qhi ? uy1 : uya, uyp = qlo ? uy1 : uy2;
                    const T dil = dil1 + (uyn - uyp) * inv2dx;
                    const T vor = vor1 - (uxn - uxp) * inv2dx;
                    const T d2 = dil * dil;
                    const T th = d2 / (d2 + vor * vor + eps);
                    stq = (T)0.25 * shfl(th, lnb) + (T)0.5 * th + (T)0.25 * shfl(th, rnb);
                }
            }
        }

        // ---------------- stage C: row p = R-2
        const int p = R - 2;
        T fs[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) fs[j] = (T)0;
        T xpa[4], xma[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) xpa[k] = xma[k] = (T)0;
        if (p >= Rb && p <= Re) {
            T beta = bconst;
            if constexpr (SENSOR != 0) {
                const bool plo = clo && p == 0, phi = chi && p == ny - 1;
                const T sn = phi ? ss2 : ssq, sp = plo ? ss2 : ss3;
                const T sbar = (T)0.25 * sp + (T)0.5 * ss2 + (T)0.25 * sn;
                T thbar = (T)1;
                if constexpr (SENSOR == 2) {
                    const T tn = phi ? st2 : stq, tp = plo ? st2 : st3;
                    thbar = (T)0.25 * tp + (T)0.5 * st2 + (T)0.25 * tn;
                }
                T chiv = csen * sbar * thbar;
                chiv = chiv < (T)0 ? (T)0 : (chiv > (T)1 ? (T)1 : chiv);
                beta = bmax - (bmax - bmin) * chiv;
            }
            if (S.probe) {
                if (owner && p >= y0 && p < y1) S.beta_out[(long long)p * nx + X] = (double)beta;
            } else {
                T W[4], qx[4], qy[4], ux, uy, e;
                cell_flux<T, EOS>(g, f2, W, ux, uy, e, qx, qy);
                const T tb = (T)2 * beta;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const T w4 = (T)0.25 * W[k];
                    const T ax = qx[k] * inv2c, ay = qy[k] * inv2c;
                    fs[0 * 4 + k] = f2[0 * 4 + k] + tb * ((w4 + ax) - f2[0 * 4 + k]);
                    fs[1 * 4 + k] = f2[1 * 4 + k] + tb * ((w4 - ax) - f2[1 * 4 + k]);
                    fs[2 * 4 + k] = f2[2 * 4 + k] + tb * ((w4 + ay) - f2[2 * 4 + k]);
                    fs[3 * 4 + k] = f2[3 * 4 + k] + tb * ((w4 - ay) - f2[3 * 4 + k]);
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    xpa[k] = shfl(fs[0 * 4 + k], lnb);   // +x population arriving from x-1
                    xma[k] = shfl(fs[1 * 4 + k], rnb);   // -x population arriving from x+1
                }
            }
        }

        // ---------------- stage D: row o = R-3
        const int o = R - 3;
        if (!S.probe && o >= y0 && o < y1) {
            const bool olo = clo && o == 0, ohi = chi && o == ny - 1;
            T gn[16];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                gn[0 * 4 + k] = xp1[k];
                gn[1 * 4 + k] = xm1[k];
                gn[2 * 4 + k] = olo ? yp1[k] : yp2[k];
                gn[3 * 4 + k] = ohi ? ym1[k] : fs[3 * 4 + k];
            }
            if (owner) {
                const long long base = (long long)o * nx + X;
#pragma unroll
                for (int j = 0; j < 16; ++j) fout[j * plane + base] = gn[j];
                T W[4], qx[4], qy[4], ux, uy, e;
                cell_flux<T, EOS>(g, gn, W, ux, uy, e, qx, qy);
                const T cs2 = eos_cs2<T, EOS>(g, W[0], e);
                errbits |= eos_check<T, EOS>(g, W[0], e, cs2);
                const T cs = sqrt(cs2 > (T)0 ? cs2 : (T)0);
                red_s = fmax(red_s, (double)(fmax(fabs(ux), fabs(uy)) + cs));
#pragma unroll
                for (int k = 0; k < 4; ++k) red_M[k] = fmax(red_M[k], (double)fmax(fabs(qx[k]), fabs(qy[k])));
            }
        }

        // ---------------- shift the row histories
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            f2[j] = f1[j];
            f1[j] = fa[j];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            qy2[k] = qy1[k];
            qy1[k] = qya[k];
            jx1[k] = jxa[k];
            xp1[k] = xpa[k];
            xm1[k] = xma[k];
            yp2[k] = yp1[k];
            yp1[k] = fs[2 * 4 + k];
            ym1[k] = fs[3 * 4 + k];
        }
        ux2 = ux1; ux1 = uxa;
        uy2 = uy1; uy1 = uya;
        dil1 = dila;
        vor1 = vora;
        ss3 = ss2; ss2 = ssq;
        st3 = st2; st2 = stq;
    }
    if (!S.probe) wave_publish(S, red_s, red_M, 4, errbits);
}

// ------------------------------------------------------------------ launcher

template <typename T>
static hipError_t launch_t(const KParams& p, const KStep& s, const void* fin, void* fout, hipStream_t st)
{
    const dim3 grid(p.nstrips * p.nsegs), block(64);
    const T* in = (const T*)fin;
    T* out = (T*)fout;
#define VLBM_CASE(E, SN)                                                                  \
    if (p.eos == E && p.sensor == SN) {                                                   \
        hipLaunchKernelGGL((k_step_d2q4<T, E, SN>), grid, block, 0, st, p, s, in, out); \
        return hipGetLastError();                                                         \
    }
    VLBM_CASE(0, 0) VLBM_CASE(0, 1) VLBM_CASE(0, 2) VLBM_CASE(1, 0) VLBM_CASE(1, 1) VLBM_CASE(1, 2)
#undef VLBM_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_step_d2q4(const KParams& p, const KStep& s, bool fp32, const void* fin, void* fout,
                            hipStream_t st)
{
    return fp32 ? launch_t<float>(p, s, fin, fout, st) : launch_t<double>(p, s, fin, fout, st);
}

}  // namespace vlbm

namespace vlbm {

int step_d2q4_blocks_per_cu(const KParams& p, bool fp32)
{
    int nb = 0;
    hipError_t e;
    if (fp32) {
        e = p.eos == 0 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_step_d2q4<float, 0, 2>, 64, 0)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_step_d2q4<float, 1, 2>, 64, 0);
    } else {
        e = p.eos == 0 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_step_d2q4<double, 0, 2>, 64, 0)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_step_d2q4<double, 1, 2>, 64, 0);
    }
    return e == hipSuccess ? nb : 0;
}

}  // namespace vlbm
