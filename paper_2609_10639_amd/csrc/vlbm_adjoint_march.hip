// Fused adjoint of one frozen-link-speed D2Q4 step (arXiv 2609.10639, Sec. III
// with c fixed), in a single march over the rows.
//
// Forward map f^n -> f^{n+1} (c fixed, so no reprojection):
//   W = sum_i f_i; closure and flux Q_alpha(W) (Eq. 10);
//   j_k = 1/2 sum_alpha [Q_alpha,k(x+e_alpha) - Q_alpha,k(x-e_alpha)],
//   s = sqrt(sum_k (j_k/M_k)^2 / 4), theta = dil^2/(dil^2 + vort^2 + eps),
//   s-bar, theta-bar by the separable (1/4, 1/2, 1/4) filter, X = C s-bar theta-bar,
//   beta = beta_max - (beta_max - beta_min) clip(X, 0, 1) (Eqs. 28-35);
//   f*_i = f_i + beta g_i with g_i = 2 (f^eq_i - f_i) (Eqs. 20, 22);
//   f^{n+1}_i(x) = f*_i(x - e_i) (Eq. 21; periodic wrap or clamped ghost).
// Given lam = dJ/df^{n+1}, one wavefront owns a strip of columns and marches a
// segment of rows; at row R it
//   L  loads f(R) and lam(R); W, Q, u; g; the transposed streaming of lam
//      (lam*_i(x) = sum of lam_i over the cells whose source is x) as far as it
//      is known, accumulating dJ/dbeta = sum_i g_i lam*_i of rows R and R-1;
//   A  accumulates the partial sums of j_k, dilatation and vorticity;
//   B  completes s and theta of row R-1 and filters them along x;
//   C  row R-2: beta and the seeds dJ/ds-bar = C theta-bar chi-bar,
//      dJ/dtheta-bar = C s-bar chi-bar (chi-bar = -(beta_max - beta_min)
//      dJ/dbeta where 0 < X < 1), the transposed x-filter, pushed into the
//      transposed y-filter of rows R-3..R-1;
//   D  row R-3: dJ/ds and dJ/dtheta complete -> dJ/dj_k, dJ/ddil, dJ/dvort,
//      the normaliser adjoint (partial sums of dJ/dM_k), transposed central
//      differences along x, pushed along y into rows R-4..R-2;
//   E  row R-4: lam*(R-4) (re-read from cache), the direct equilibrium terms
//      and the sensor terms through the closure transpose -> lam^n(R-4).
// Each wavefront records its dJ/dM_k partial sums and the first maximiser of
// every |Q_alpha,k| over its cells; k_adjm_fix folds the records and adds the
// normaliser term at the maximisers.
// Non-smooth points: d clip/dX = 1 on (0, 1), 0 elsewhere; d sqrt(s)/ds := 0 at
// s = 0; the M_k sub-gradient goes to the first maximiser in (alpha, y, x) order.
#include <mutex>

#include "vlbm_adjoint_math.hpp"
#include "vlbm_aux.hpp"
#include "vlbm_planes.hpp"

namespace vlbm {

constexpr int kRecDoubles = 12;   // per wavefront: dJ/dM_k (4), max |Q| (4), its cell index (4)

template <typename S, typename C, int EOS, int SENSOR>
struct AdjMarch {
    const KParams& P;
    Planes fin, lin, lout;      // f^n, lam^{n+1}, lam^n
    C (*wr)[4][64];             // W of the last five rows (LDS ring)
    C (*hr)[9][64];             // j_k, dil, vort, s and the x-filtered s and theta of the last three
                                // completed rows (LDS ring): written when row R-1 completes, read by
                                // stage C (rows R-2, R-3) and stage D (row R-3)
    Gas<C> g;
    C inv2c, invM[4], csen, bspan, bmax, eps;   // inv2c = 1/(2c) also scales the gate's differences
    int nx, ny, y0, y1, Rb, Re;
    long long ncell;
    bool clo, chi;              // clamped y-low / y-high boundaries
    int lane, X;
    bool kl, kr;       // the left / right neighbour is the cell itself (clamped edge)
    unsigned colx;
    bool owner, atL, atR;       // atL / atR: the clamped first / last column

    // sensor forward: partial sums of rows R+1 (n), R, R-1 (older rows live in hr)
    C Jn[4], J0[4], J1[4];
    C Dn, D0, D1, Vn, V0, V1;
    // dJ/dbeta of rows R (partial), R-1, R-2; g_{+y} and lam_{-y} of row R-1
    C bb0, bb1, bb2, gyp[4], lym[4];
    C bq1, bq2;                 // beta of rows R-3, R-4
    // transposed y-filter of the seeds: rows R-3, R-2, R-1
    C SAm, SA0, SAp, TBm, TB0, TBp;
    // transposed y-differences: rows R-4, R-3, R-2; x-parts of row R-4
    C QYm[4], QY0[4], QYp[4], UXm, UX0, UXp, UYm, UY0, UYp;
    C QXh[4], UXh, UYh;
    double mbar[4];
    C amax[4];
    double aidx[4];

    __device__ __forceinline__ bool row_ok(int r) const { return !(clo && r < 0) && !(chi && r > ny - 1); }
    __device__ __forceinline__ int hslot(int r) const { return (r - Rb + 3) % 3; }   // r >= Rb - 3
    __device__ __forceinline__ unsigned row_off(int r) const
    {
        const int m = (r < 0 || r >= ny) ? wrap_index(r, ny) : r;
        return ((unsigned)m * (unsigned)nx + colx) * (unsigned)sizeof(S);
    }
    // transposed central difference along x: sum_x a(x) ([nb(x,+1)=z] - [nb(x,-1)=z])
    __device__ __forceinline__ C tdiff_x(C a) const
    {
        const C l = from_left(a, false), r = from_right(a, false);
        return (atL ? -a : l) + (atR ? a : -r);
    }
    // transposed (1/4, 1/2, 1/4) filter along x
    __device__ __forceinline__ C tbox_x(C a) const
    {
        const C l = from_left(a, false), r = from_right(a, false);
        return (C)0.25 * (atL ? a : l) + (C)0.5 * a + (C)0.25 * (atR ? a : r);
    }

    __device__ __forceinline__ void iter(int R)
    {
        const bool rowR = R <= Re && row_ok(R);
        // ================= L: row R
        C qx[4] = {0, 0, 0, 0}, qy[4] = {0, 0, 0, 0}, ux = 0, uy = 0;
        C gy_p[4] = {0, 0, 0, 0}, ly_m[4] = {0, 0, 0, 0};
        bb0 = 0;
        if (rowR) {
            const unsigned off = row_off(R);
            C fv[16], lv[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                fv[j] = (C)bload(fin, j, off, S());
                lv[j] = (C)bload(lin, j, off, S());
            }
            C W[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) W[k] = (fv[k] + fv[4 + k]) + (fv[8 + k] + fv[12 + k]);
            const int slot = (R - Rb) % 5;
#pragma unroll
            for (int k = 0; k < 4; ++k) wr[slot][k][lane] = W[k];
            const C irho = (C)1 / W[0];
            ux = W[1] * irho;
            uy = W[2] * irho;
            const C e = W[3] * irho - (C)0.5 * (ux * ux + uy * uy);
            const C Pp = eos_pressure<C, EOS>(g, W[0], e);
            const C h = W[3] + Pp;
            qx[0] = W[1]; qx[1] = W[1] * ux + Pp; qx[2] = W[1] * uy; qx[3] = h * ux;
            qy[0] = W[2]; qy[1] = W[2] * ux; qy[2] = W[2] * uy + Pp; qy[3] = h * uy;
            // first maximiser of |Q_alpha,k| over the cells this wavefront owns
            if (owner && R >= y0 && R < y1) {
                const double cidx = (double)R * (double)nx + (double)X;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    // selects, not branches: a branchy update let the optimiser
                    // keep one of these in scratch memory
                    const C vx = fabs(qx[k]), vy = fabs(qy[k]);
                    const bool tx = vx > amax[k];
                    amax[k] = tx ? vx : amax[k];
                    aidx[k] = tx ? cidx : aidx[k];
                    const double iy = (double)ncell + cidx;
                    const bool ty = vy > amax[k] || (vy == amax[k] && iy < aidx[k]);
                    amax[k] = ty ? vy : amax[k];
                    aidx[k] = ty ? iy : aidx[k];
                }
            }
            if constexpr (SENSOR != 0) {
                // g_i = 2 (f^eq_i - f_i); lam* along x from the neighbour columns
                C bx = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const C w4 = (C)0.25 * W[k];
                    const C gxp = (C)2 * (w4 + qx[k] * inv2c - fv[k]);
                    const C gxm = (C)2 * (w4 - qx[k] * inv2c - fv[4 + k]);
                    const C gyy = (C)2 * (w4 + qy[k] * inv2c - fv[8 + k]);
                    const C gym = (C)2 * (w4 - qy[k] * inv2c - fv[12 + k]);
                    const C lpr = from_right(lv[k], false);
                    const C lml = from_left(lv[4 + k], false);
                    const C lsxp = (atR ? (C)0 : lpr) + (atL ? lv[k] : (C)0);
                    const C lsxm = (atL ? (C)0 : lml) + (atR ? lv[4 + k] : (C)0);
                    bx += gxp * lsxp + gxm * lsxm;
                    // lam*_{-y}(R) = lam_{-y}(R-1) [not below a clamped bottom] + lam_{-y}(R) at a clamped top
                    const C lsym = ((clo && R == 0) ? (C)0 : lym[k]) + ((chi && R == ny - 1) ? lv[12 + k] : (C)0);
                    bx += gym * lsym;
                    // lam*_{+y}(R-1) = lam_{+y}(R) (+ lam_{+y}(0) itself when R-1 is a clamped bottom row)
                    if (!(clo && R == 0)) bb1 += gyp[k] * lv[8 + k];
                    if (clo && R == 0) bx += gyy * lv[8 + k];
                    gy_p[k] = gyy;
                    ly_m[k] = lv[12 + k];
                }
                bb0 = bx;
            }
        }

        // ================= A: partial sums of j, dilatation, vorticity (row R)
        if constexpr (SENSOR != 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) Jn[k] = 0;
            Dn = Vn = 0;
            if (rowR) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const C hq = (C)0.5 * qy[k];
                    J1[k] += hq;
                    // flux and velocity come from the loaded column alone: the lane beyond a
                    // clamped edge loaded the edge column, so no edge select is needed
                    J0[k] += (C)0.5 * (from_right(qx[k], false) - from_left(qx[k], false));
                    Jn[k] = -hq;
                    if (clo && R == 0) J0[k] -= hq;
                    if (chi && R == ny - 1) J0[k] += hq;
                }
                if constexpr (SENSOR == 2) {
                    const C hx = ux * inv2c, hy = uy * inv2c;   // lattice units (dt = dx/c)
                    D1 += hy;
                    V1 -= hx;
                    D0 += (from_right(ux, false) - from_left(ux, false)) * inv2c;
                    V0 += (from_right(uy, false) - from_left(uy, false)) * inv2c;
                    Dn = -hy;
                    Vn = hx;
                    if (clo && R == 0) { D0 -= hy; V0 += hx; }
                    if (chi && R == ny - 1) { D0 += hy; V0 -= hx; }
                }
            }
        }

        // ================= B: s, theta of row R-1, filtered along x
        C s1 = 0, Ss1 = 0, Th1 = 0;
        if constexpr (SENSOR != 0) {
            if (row_ok(R - 1)) {
                C acc = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const C sh = J1[k] * invM[k];
                    acc = fma(sh, sh, acc);
                }
                s1 = acc > (C)0 ? sqrt(acc * (C)0.25) : (C)0;
                const int hs = hslot(R - 1);
#pragma unroll
                for (int k = 0; k < 4; ++k) hr[hs][k][lane] = J1[k];
                hr[hs][4][lane] = D1;
                hr[hs][5][lane] = V1;
                hr[hs][6][lane] = s1;
                Ss1 = (C)0.25 * from_left(s1, kl) + (C)0.5 * s1 + (C)0.25 * from_right(s1, kr);
                if constexpr (SENSOR == 2) {
                    const C d2 = D1 * D1;
                    const C th = d2 / (fma(V1, V1, d2) + eps);
                    Th1 = (C)0.25 * from_left(th, kl) + (C)0.5 * th + (C)0.25 * from_right(th, kr);
                }
                hr[hs][7][lane] = Ss1;
                hr[hs][8][lane] = Th1;
            }
        }

        // ================= C: beta and the seeds of row p = R-2
        C bnew = (C)P.beta_const;
        if constexpr (SENSOR != 0) {
            const int p = R - 2;
            if (row_ok(p)) {
                const int h2 = hslot(p), h3 = hslot(p - 1);
                const C Ss2 = hr[h2][7][lane], Th2 = hr[h2][8][lane];
                const bool pb = clo && p == 0, pt = chi && p == ny - 1;
                // row p-1 below a clamped bottom is never read (its slot may hold older rows)
                const C Ss3 = pb ? Ss2 : hr[h3][7][lane], Th3 = pb ? Th2 : hr[h3][8][lane];
                const C sm = pb ? Ss2 : Ss3, sp = pt ? Ss2 : Ss1;
                const C sbar = (C)0.25 * sm + (C)0.5 * Ss2 + (C)0.25 * sp;
                C thbar = (C)1;
                if constexpr (SENSOR == 2) {
                    const C tm = pb ? Th2 : Th3, tp = pt ? Th2 : Th1;
                    thbar = (C)0.25 * tm + (C)0.5 * Th2 + (C)0.25 * tp;
                }
                const C Xv = csen * sbar * thbar;
                const C chiv = fmin(fmax(Xv, (C)0), (C)1);
                bnew = bmax - bspan * chiv;
                const C chibar = (Xv > (C)0 && Xv < (C)1) ? -bspan * bb2 : (C)0;
                const C ax = tbox_x(csen * thbar * chibar);
                const C qa = (C)0.25 * ax;
                SAm += pb ? (C)0 : qa;
                SA0 += (C)0.5 * ax + (pb ? qa : (C)0) + (pt ? qa : (C)0);
                SAp += pt ? (C)0 : qa;
                if constexpr (SENSOR == 2) {
                    const C bx = tbox_x(csen * sbar * chibar);
                    const C qb = (C)0.25 * bx;
                    TBm += pb ? (C)0 : qb;
                    TB0 += (C)0.5 * bx + (pb ? qb : (C)0) + (pt ? qb : (C)0);
                    TBp += pt ? (C)0 : qb;
                }
            }
        }

        // ================= D: row q = R-3: dJ/dj, dJ/ddil, dJ/dvort; transposed differences
        C QX[4] = {0, 0, 0, 0}, UXx = 0, UYx = 0;
        if constexpr (SENSOR != 0) {
            const int q = R - 3;
            if (row_ok(q)) {
                const int hs = hslot(q);
                const C s3 = hr[hs][6][lane];
                C jb[4] = {0, 0, 0, 0};
                if (s3 > (C)0) {
                    const C f4s = SAm / ((C)4 * s3);
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const C shat = hr[hs][k][lane] * invM[k];
                        const C shb = f4s * shat;   // d s / d s_hat_k = s_hat_k / (4 s)
                        jb[k] = shb * invM[k];
                        if (owner && q >= y0 && q < y1) mbar[k] -= (double)(shb * shat * invM[k]);
                    }
                }
                C dilb = 0, vortb = 0;
                if constexpr (SENSOR == 2) {
                    const C D3 = hr[hs][4][lane], V3 = hr[hs][5][lane];
                    const C den = D3 * D3 + V3 * V3 + eps;
                    const C iden2 = (C)1 / (den * den);
                    dilb = TBm * (C)2 * D3 * (V3 * V3 + eps) * iden2;
                    vortb = -TBm * (C)2 * V3 * D3 * D3 * iden2;
                }
                const bool bot = clo && q == 0, top = chi && q == ny - 1;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    QX[k] = (C)0.5 * tdiff_x(jb[k]);
                    const C hj = (C)0.5 * jb[k];
                    QYp[k] += top ? (C)0 : hj;
                    QY0[k] += (top ? hj : (C)0) - (bot ? hj : (C)0);
                    QYm[k] -= bot ? (C)0 : hj;
                }
                if constexpr (SENSOR == 2) {
                    // u_x-bar = (T_x dil-bar - T_y vort-bar)/(2c), u_y-bar = (T_y dil-bar + T_x vort-bar)/(2c)
                    UXx = inv2c * tdiff_x(dilb);
                    UYx = inv2c * tdiff_x(vortb);
                    const C vx = -inv2c * vortb, dy = inv2c * dilb;
                    UXp += top ? (C)0 : vx;
                    UYp += top ? (C)0 : dy;
                    UX0 += (top ? vx : (C)0) - (bot ? vx : (C)0);
                    UY0 += (top ? dy : (C)0) - (bot ? dy : (C)0);
                    UXm -= bot ? (C)0 : vx;
                    UYm -= bot ? (C)0 : dy;
                }
            }
        }

        // ================= E: lam^n of row o = R-4
        const int o = R - 4;
        if (o >= y0 && o < y1 && row_ok(o)) {
            const C beta = SENSOR != 0 ? bq2 : (C)P.beta_const;
            const unsigned offo = row_off(o);
            const bool bot = clo && o == 0, top = chi && o == ny - 1;
            const unsigned offu = top ? offo : row_off(o + 1), offd = bot ? offo : row_off(o - 1);
            C ls[16];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const C lp = (C)bload(lin, k, offo, S()), lm = (C)bload(lin, 4 + k, offo, S());
                const C lpr = from_right(lp, false), lml = from_left(lm, false);
                ls[k] = (atR ? (C)0 : lpr) + (atL ? lp : (C)0);
                ls[4 + k] = (atL ? (C)0 : lml) + (atR ? lm : (C)0);
                const C lyu = (C)bload(lin, 8 + k, offu, S()), lyd = (C)bload(lin, 12 + k, offd, S());
                ls[8 + k] = top ? (C)0 : lyu;
                ls[12 + k] = bot ? (C)0 : lyd;
                if (bot) ls[8 + k] += (C)bload(lin, 8 + k, offo, S());
                if (top) ls[12 + k] += (C)bload(lin, 12 + k, offo, S());
            }
            const int slot = (o - Rb) % 5;
            C W[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) W[k] = wr[slot][k][lane];
            const C tb = (C)2 * beta;
            C Wb[4], Qb[2][4], ub[2];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                Wb[k] = tb * (C)0.25 * ((ls[k] + ls[4 + k]) + (ls[8 + k] + ls[12 + k]));
                Qb[0][k] = tb * (ls[k] - ls[4 + k]) * inv2c + QXh[k];      // direct + x-differences of j-bar
                Qb[1][k] = tb * (ls[8 + k] - ls[12 + k]) * inv2c + QYm[k]; // direct + y-differences of j-bar
            }
            ub[0] = UXh + UXm;
            ub[1] = UYh + UYm;
            closure_adj<C, EOS, 2>(g, W, Qb, ub, Wb);
            if (owner) {
                const C om = (C)1 - tb;
#pragma unroll
                for (int j = 0; j < 16; ++j) bstore(lout, j, offo, (S)(om * ls[j] + Wb[j & 3]));
            }
        }

        // ================= shift the row histories
        if constexpr (SENSOR != 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                J1[k] = J0[k]; J0[k] = Jn[k];
                QYm[k] = QY0[k]; QY0[k] = QYp[k]; QYp[k] = 0;
                QXh[k] = QX[k];
                gyp[k] = gy_p[k];
                lym[k] = ly_m[k];
            }
            D1 = D0; D0 = Dn;
            V1 = V0; V0 = Vn;
            bb2 = bb1; bb1 = bb0;
            bq2 = bq1; bq1 = bnew;
            SAm = SA0; SA0 = SAp; SAp = 0;
            TBm = TB0; TB0 = TBp; TBp = 0;
            UXm = UX0; UX0 = UXp; UXp = 0;
            UYm = UY0; UY0 = UYp; UYp = 0;
            UXh = UXx;
            UYh = UYx;
        }
    }
};

// XPER: both x edges periodic (no clamped column): the edge selects fold away.
template <typename S, typename C, int EOS, int SENSOR, bool XPER>
__global__ void __launch_bounds__(64) k_adj_march(const KParams P, const S* __restrict__ f, const double* __restrict__ norms,
                                                  const S* __restrict__ lam, S* __restrict__ lam_out,
                                                  double* __restrict__ rec)
{
    __shared__ C wring[5][4][64];
    __shared__ C hring[3][9][64];
    AdjMarch<S, C, EOS, SENSOR> m{P};
    m.fin = make_planes(f, (unsigned)P.plane);
    m.lin = make_planes(lam, (unsigned)P.plane);
    m.lout = make_planes((const S*)lam_out, (unsigned)P.plane);
    m.wr = wring;
    m.hr = hring;
    // rows before the first completed one read as zeros (each lane owns its column)
#pragma unroll
    for (int sl = 0; sl < 3; ++sl)
#pragma unroll
        for (int v = 0; v < 9; ++v) hring[sl][v][threadIdx.x] = (C)0;
    m.g = make_gas<C>(P);
    m.inv2c = (C)(0.5 / P.c_fixed);
    // M_k of the state, the maximum over the norms' copies: lane i reads copy
    // i and a wave maximum folds them (one read per field, not a chain of
    // dependent reads over the copies)
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double M = wave_max_dpp(lane < kRedCopies ? norms[lane * kRedStride + 1 + k] : 0.0);
        m.invM[k] = M > 0.0 ? (C)(1.0 / M) : (C)0;
    }
    m.csen = (C)P.c_sensor;
    m.bspan = (C)(P.beta_max - P.beta_min);
    m.bmax = (C)P.beta_max;
    m.eps = (C)P.eps_theta;
    m.nx = P.nx;
    m.ny = P.ny;
    m.ncell = (long long)P.nx * P.ny;
    m.lane = threadIdx.x;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int strip = tile % P.nstrips, seg = tile / P.nstrips;
    const int halo = (64 - P.strip_w) / 2;
    m.X = strip * P.strip_w - halo + m.lane;
    int cx = m.X;
    if (m.X < 0) cx = P.bc[0] == 0 ? wrap_index(m.X, m.nx) : 0;
    else if (m.X >= m.nx) cx = P.bc[1] == 0 ? wrap_index(m.X, m.nx) : m.nx - 1;
    m.colx = (unsigned)cx;
    m.atL = !XPER && P.bc[0] == 1 && m.X == 0;
    m.atR = !XPER && P.bc[1] == 1 && m.X == m.nx - 1;
    m.kl = m.atL;
    m.kr = m.atR;
    m.owner = m.lane >= halo && m.lane < halo + P.strip_w && m.X < m.nx;
    m.clo = P.bc[2] == 1;
    m.chi = P.bc[3] == 1;
    m.y0 = seg * P.seg_h;
    m.y1 = min(m.y0 + P.seg_h, m.ny);
    m.Rb = m.clo ? max(m.y0 - 4, 0) : m.y0 - 4;
    m.Re = m.chi ? min(m.y1 + 3, m.ny - 1) : m.y1 + 3;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        m.Jn[k] = m.J0[k] = m.J1[k] = 0;
        m.QYm[k] = m.QY0[k] = m.QYp[k] = m.QXh[k] = 0;
        m.gyp[k] = m.lym[k] = 0;
        m.mbar[k] = 0.0;
        m.amax[k] = (C)-1;
        m.aidx[k] = 0.0;
    }
    m.Dn = m.D0 = m.D1 = m.Vn = m.V0 = m.V1 = 0;
    m.bb0 = m.bb1 = m.bb2 = 0;
    m.bq1 = m.bq2 = (C)P.beta_const;
    m.SAm = m.SA0 = m.SAp = m.TBm = m.TB0 = m.TBp = 0;
    m.UXm = m.UX0 = m.UXp = m.UYm = m.UY0 = m.UYp = m.UXh = m.UYh = 0;

    for (int R = m.Rb; R <= m.y1 + 3; ++R) m.iter(R);

    // per-wavefront record: dJ/dM_k (sum over lanes, fixed tree), and the
    // first maximiser of |Q_alpha,k| (largest value, then smallest index)
    double* out = rec + (size_t)blockIdx.x * kRecDoubles;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double mb = m.mbar[k];
        double v = (double)m.amax[k], ix = m.aidx[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            mb += __shfl_xor(mb, o, 64);
            const double v2 = __shfl_xor(v, o, 64), i2 = __shfl_xor(ix, o, 64);
            if (v2 > v || (v2 == v && i2 < ix)) { v = v2; ix = i2; }
        }
        if (m.lane == 0) {
            out[k] = mb;
            out[4 + k] = v;
            out[8 + k] = ix;
        }
    }
}

// Folds the per-wavefront records (sum of dJ/dM_k; max |Q_alpha,k| with the
// smallest flat index among equal maxima) and adds the normaliser term
// dJ/dM_k * sign(Q_alpha,k) at each maximiser, through the closure transpose,
// to lam^n.  One workgroup of 1024 threads: each folds its records, the waves combine theirs by
// shuffles and the 16 wave results are folded in wave order, so the sums have
// a fixed order.  Threads 0-3 evaluate the four components' terms in parallel;
// thread 0 then applies them to lam in component order (two components may
// share a maximiser).
constexpr int kFixThreads = 1024;

// Wave-wide sum and minimum by DPP row shifts (as wave_max_dpp): lanes whose
// source lies outside their 16-lane row add 0 / keep their own value; the
// four row results are read from lanes 15, 31, 47 and 63.  Whole wave active.
template <int CTRL>
__device__ __forceinline__ double dpp_shr(double v, bool zero_fill)
{
    const long long b = __double_as_longlong(v);
    const int lo = (int)b, hi = (int)(b >> 32);
    int lo2, hi2;
    if (zero_fill) {
        lo2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xf, 0xf, true);
        hi2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xf, 0xf, true);
    } else {
        lo2 = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xf, 0xf, false);
        hi2 = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xf, 0xf, false);
    }
    return __longlong_as_double(((long long)hi2 << 32) | (unsigned int)lo2);
}
__device__ __forceinline__ double row_lane(double v, int r)
{
    const long long b = __double_as_longlong(v);
    const int l = __builtin_amdgcn_readlane((int)b, r), h = __builtin_amdgcn_readlane((int)(b >> 32), r);
    return __longlong_as_double(((long long)h << 32) | (unsigned int)l);
}
__device__ __forceinline__ double wave_sum_dpp(double v)
{
    v += dpp_shr<0x111>(v, true);
    v += dpp_shr<0x112>(v, true);
    v += dpp_shr<0x114>(v, true);
    v += dpp_shr<0x118>(v, true);
    return ((row_lane(v, 15) + row_lane(v, 31)) + row_lane(v, 47)) + row_lane(v, 63);
}
__device__ __forceinline__ double wave_min_dpp(double v)
{
    v = fmin(v, dpp_shr<0x111>(v, false));
    v = fmin(v, dpp_shr<0x112>(v, false));
    v = fmin(v, dpp_shr<0x114>(v, false));
    v = fmin(v, dpp_shr<0x118>(v, false));
    return fmin(fmin(row_lane(v, 15), row_lane(v, 31)), fmin(row_lane(v, 47), row_lane(v, 63)));
}

template <typename S, typename C, int EOS>
__global__ void __launch_bounds__(kFixThreads) k_adjm_fix(KParams p, const S* __restrict__ f,
                                                          const double* __restrict__ rec, int nrec,
                                                          S* __restrict__ lam_out)
{
    constexpr int NW = kFixThreads / 64;
    __shared__ double wm[NW][4], wv[NW][4], wi[NW][4];
    __shared__ C wb[4][4];
    __shared__ long long wc[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double a[4] = {0, 0, 0, 0}, v[4] = {-1, -1, -1, -1}, ix[4] = {0, 0, 0, 0};
    for (int b = threadIdx.x; b < nrec; b += kFixThreads) {
        const double* r = rec + (size_t)b * kRecDoubles;
        double rr[kRecDoubles];
#pragma unroll
        for (int j = 0; j < kRecDoubles; ++j) rr[j] = r[j];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            a[k] += rr[k];
            if (rr[4 + k] > v[k] || (rr[4 + k] == v[k] && rr[8 + k] < ix[k])) {
                v[k] = rr[4 + k];
                ix[k] = rr[8 + k];
            }
        }
    }
    // wave folds by DPP: the sum of dJ/dM_k, the largest |Q| (records with no
    // cell hold -1), and the first cell holding it
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        a[k] = wave_sum_dpp(a[k]);
        const double vm = -wave_min_dpp(-v[k]);
        ix[k] = wave_min_dpp(v[k] == vm ? ix[k] : HUGE_VAL);
        v[k] = vm;
    }
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            wm[wave][k] = a[k];
            wv[wave][k] = v[k];
            wi[wave][k] = ix[k];
        }
    __syncthreads();
    const long long ncell = (long long)p.nx * p.ny;
    if (threadIdx.x < 4) {
        const int k = threadIdx.x;
        double Mb = 0.0, vm = -1.0, im = 0.0;
        for (int w = 0; w < NW; ++w) {
            Mb += wm[w][k];
            if (wv[w][k] > vm || (wv[w][k] == vm && wi[w][k] < im)) {
                vm = wv[w][k];
                im = wi[w][k];
            }
        }
        wc[k] = -1;
        if (Mb != 0.0 && vm >= 0.0) {
            const long long id = (long long)im;
            const int al = (int)(id / ncell);
            const long long c = id % ncell;
            const Gas<C> g = make_gas<C>(p);
            C W[4] = {0, 0, 0, 0};
            for (int i = 0; i < 4; ++i)
                for (int kk = 0; kk < 4; ++kk) W[kk] += (C)f[(long long)(i * 4 + kk) * p.plane + c];
            C u[2], e, P, Qf[2][4];
            closure<C, EOS, 2>(g, W, u, e, P, Qf);
            // seed Q_bar at (al, k) only; selects keep every array index static
            C Qb[2][4], ub[2] = {0, 0}, Wb[4] = {0, 0, 0, 0};
#pragma unroll
            for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
                for (int k2 = 0; k2 < 4; ++k2) {
                    const C q = Qf[a2][k2];
                    const C sg = q > (C)0 ? (C)1 : (q < (C)0 ? (C)-1 : (C)0);
                    Qb[a2][k2] = (a2 == al && k2 == k) ? (C)Mb * sg : (C)0;
                }
            closure_adj<C, EOS, 2>(g, W, Qb, ub, Wb);
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) wb[k][kk] = Wb[kk];
            wc[k] = c;
        }
    }
    __syncthreads();
    // one thread per population plane: the terms of components that share a
    // maximiser are summed in component order, then each distinct cell is read
    // and written once (all loads issued before the stores)
    if (threadIdx.x >= 16) return;
    const int plane = threadIdx.x, kk = plane & 3;
    bool use[4];
    C add[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        bool first = wc[k] >= 0;
#pragma unroll
        for (int k2 = 0; k2 < k; ++k2) first = first && wc[k2] != wc[k];
        C a = (C)0;
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2)
            if (k2 >= k && wc[k2] == wc[k]) a += wb[k2][kk];
        use[k] = first;
        add[k] = a;
    }
    S* base = lam_out + (long long)plane * p.plane;
    S old[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) old[k] = base[use[k] ? wc[k] : 0];   // cell 0 stands in when unused
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (use[k]) base[wc[k]] = (S)((C)old[k] + add[k]);
}

int adjoint_march_records(const KParams& p) { return p.nstrips * p.nsegs; }

bool adjoint_march_supported(const KParams& p)
{
    return p.dim == 2 && (64 - p.strip_w) / 2 >= 4 && p.e_off == 0.0;
}

template <typename S, typename C>
static hipError_t march_t(const KParams& p, const void* f_n, const double* norms, const void* lam_np1, void* lam_n,
                          double* rec, hipStream_t st)
{
    const int nb = adjoint_march_records(p);
    const S* f = (const S*)f_n;
    const S* lam = (const S*)lam_np1;
    S* lo = (S*)lam_n;
#define VLBM_AM(E, SN)                                                                                         \
    if (p.eos == E && p.sensor == SN) {                                                                        \
        if (p.bc[0] == 0)                                                                                      \
            hipLaunchKernelGGL((k_adj_march<S, C, E, SN, true>), dim3(nb), dim3(64), 0, st, p, f, norms, lam, lo, rec); \
        else                                                                                                   \
            hipLaunchKernelGGL((k_adj_march<S, C, E, SN, false>), dim3(nb), dim3(64), 0, st, p, f, norms, lam, lo, rec); \
        if (SN != 0) hipLaunchKernelGGL((k_adjm_fix<S, C, E>), dim3(1), dim3(kFixThreads), 0, st, p, f, rec, nb, lo);  \
        return hipGetLastError();                                                                              \
    }
    VLBM_AM(0, 0) VLBM_AM(0, 1) VLBM_AM(0, 2) VLBM_AM(1, 0) VLBM_AM(1, 1) VLBM_AM(1, 2)
#undef VLBM_AM
    return hipErrorInvalidValue;
}

hipError_t launch_adjoint_march(const KParams& p, int prec, const void* f_n, const double* norms_n,
                                const void* lam_np1, void* lam_n, double* rec, hipStream_t st)
{
    switch (prec) {
    case PREC_FP64: return march_t<double, double>(p, f_n, norms_n, lam_np1, lam_n, rec, st);
    case PREC_FP32: return march_t<float, float>(p, f_n, norms_n, lam_np1, lam_n, rec, st);
    case PREC_FP32_MIXED: return march_t<float, double>(p, f_n, norms_n, lam_np1, lam_n, rec, st);
    }
    return hipErrorInvalidValue;
}

// Scratch of the allocation-free adjoint step: the per-wavefront records of the
// march (kRecDoubles each) in a file-scope device array, which every GPU the
// library runs on holds until the process ends.  Host code never passes the
// array's name to a kernel: it passes the device address that
// hipGetSymbolAddress returns for the GPU at hand, looked up once per device.
static __device__ __align__(256) double scratch[kStaticMarchRecords * kRecDoubles];

constexpr int kMaxDevices = 64;

hipError_t adjm_static_scratch(int device, double** out)
{
    static std::mutex mu;
    static double* addr[kMaxDevices] = {};
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) {
            const hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        addr[device] = static_cast<double*>(p);
    }
    *out = addr[device];
    return hipSuccess;
}

}  // namespace vlbm
