// Fused D2Q4 VLBM time step for gfx950 (arXiv 2609.10639, Sec. III).
//
// One wavefront owns a strip of output columns and marches up a segment of
// rows.  The strip is 56 columns; the 64 lanes hold 64 consecutive columns
// centred on it, 4 halo lanes on each side (the stencil chain needs 3 halo
// columns and streaming one more).  56 columns are three and a half 128-byte
// lines in FP64 and one and three quarters in FP32; the strips that share a
// line write their parts of it in the same row sweep and the parts merge in L2
// (measured faster than 48-column strips, whose whole lines cost a third more
// halo loads).  x-neighbour values move between lanes by DPP wavefront shifts
// or through the LDS crossbar; the raw populations of the last three rows sit
// in a per-wave LDS ring; the per-row partial sums that later rows complete
// sit in registers.  The march is unrolled by three so that every row slot
// (LDS ring and register histories alike) is a compile-time index.
//
// Iteration R (front row R) runs, in this order:
//   issue the global loads of row R+DEPTH (DEPTH rows stay in flight: one with
//               FP64 storage on large grids, else two);
//   C  row R-3  y-pass of the box filter, beta (Eqs. 34-35), reprojection to
//               the new link speed (Eqs. 38-40) of the populations read back
//               from LDS, over-relaxation towards the vector equilibrium
//               (Eqs. 20, 22), streaming (Eq. 21) as stores into the rows
//               R-4..R-2 of the new populations, and the reductions of the
//               new state (s_max of Eq. 36, M_k of Eq. 30) for the next step;
//   A  row R    moments W (of the un-reprojected populations: reprojection
//               leaves W unchanged), primitives, EOS pressure, flux (Eq. 10),
//               x-parts of the central differences of Q and u, completion of
//               the y-differences of row R-1; the raw row is parked in LDS;
//   B  row R-1  flux-divergence jump j_k (Eqs. 28-29), normalised activity s
//               (Eqs. 30-31), Ducros ratio theta (Eqs. 32-33), x-pass of the
//               box filter.
// Every population is read once from HBM and written once; halo rows and
// columns are re-read through L2.  S is the storage type of the populations,
// C the arithmetic type.
#include <algorithm>
#include <cstdlib>

#include "vlbm_planes.hpp"

namespace vlbm {


// +x equilibrium of a pinned x-low ghost, then -x of a pinned x-high ghost, at
// this step's link speed (written once per workgroup before the march).
__shared__ double vlbm_pin_lds[8];

// The LDS ring keeps lanes kRingLo .. kRingLo + kRingW - 1 only: stage C needs
// the raw populations of the lanes whose post-collision populations stream into
// owned columns, lanes halo-1 .. 64-halo, within that span for strips of at
// most 56 columns (halo >= 4).
constexpr int kRingLo = 3, kRingW = 58;

// XPER: both x edges periodic (no clamped column, no pinned ghost), so the
// neighbour moves need no edge selects.
template <typename S, typename C, int EOS, int SENSOR, int DEPTH_, bool XPER>
struct March {
    // uniform
    const KParams& P;
    const KStep& St;
    Planes in, out;
    S (*ring)[16][kRingW];
    Gas<C> g;
    C r, inv2c, invM[4];   // inv2c = 1/(2c): also scales the velocity differences of the gate
    C eoff;            // energy gauge of the stored populations (physical e = e_stored + eoff)
    int nx, ny, y0, y1, Rb, Re;
    bool clo, chi;
    // per lane
    int lane, X;
    int lnb, rnb;      // lanes of the x-1 / x+1 neighbours (the own lane at a clamped edge)
    bool kl, kr;       // clamped x edge: the left / right neighbour is the cell itself
    int rl;            // this lane's ring column (clamped; lanes outside the span never write)
    unsigned colx;     // column loaded by this lane
    bool owner;
    // row-indexed histories, slot = (row - Rb) % 3
    C J[3][4], Dl[3], Vo[3];   // partial sums of j_k, dilatation, vorticity
    C Ss[3], Sth[3];           // S_x[s], S_x[theta]
    C yprev[4], wpend[4];      // f*_{+y} of the last collided row, pending moments of the row below
    // Rows in flight: with DEPTH 1 buf[0] holds the loads of row R+1 while row R
    // is processed; with DEPTH 2 three buffers rotate with the unrolled phase,
    // row R in buf[PH] and the loads of rows R+1 and R+2 in the other two, so
    // twice the bytes are in flight per wavefront.  FP32 storage always has the
    // registers for it; with FP64 storage it costs the second wavefront per SIMD
    // (255 VGPRs and up to 14 AGPRs), which pays only on grids too small to fill
    // the second one anyway.
    static constexpr int DEPTH = DEPTH_;
    S buf[DEPTH == 2 ? 3 : 1][16];
    // x-neighbour values: DPP wavefront shifts (VALU) where a wavefront runs
    // alone on its SIMD and the march is latency-bound (two rows in flight),
    // the LDS crossbar (ds_bpermute) where two FP64 wavefronts share the VALU
    // (measured: 1024^2 FP64 +4.5 % with DPP, 4096^2 FP64 -1.8 %)
    static constexpr bool kDpp = DEPTH == 2;
    template <typename T>
    __device__ __forceinline__ T left(T v) const
    {
        if constexpr (kDpp && XPER) return dpp_move<kDppWaveShr1>(v);
        else if constexpr (kDpp) return from_left(v, kl);
        else return shfl(v, lnb);
    }
    template <typename T>
    __device__ __forceinline__ T right(T v) const
    {
        if constexpr (kDpp && XPER) return dpp_move<kDppWaveShl1>(v);
        else if constexpr (kDpp) return from_right(v, kr);
        else return shfl(v, rnb);
    }
    // the same for a value computed from the loaded column alone: the lane
    // beyond a clamped edge loaded the edge column, so it already holds the
    // clamped neighbour's value and no select is needed
    template <typename T>
    __device__ __forceinline__ T left_col(T v) const
    {
        if constexpr (kDpp) return dpp_move<kDppWaveShr1>(v);
        else return shfl(v, lnb);
    }
    template <typename T>
    __device__ __forceinline__ T right_col(T v) const
    {
        if constexpr (kDpp) return dpp_move<kDppWaveShl1>(v);
        else return shfl(v, rnb);
    }
    // reductions of the new state: maxima, and the admissibility witnesses
    C red_s, red_M[4];
    int ebits;                 // admissibility of the new state: ERR_NONHYP | ERR_NONFINITE

    __device__ __forceinline__ void reduce(const C* w)
    {
        const C irho = fast_rcp(w[0]);
        const C vx = w[1] * irho, vy = w[2] * irho;
        const C ee = w[3] * irho - (C)0.5 * (vx * vx + vy * vy) + eoff;
        const C PP = eos_pressure<C, EOS>(g, w[0], ee);
        const C cs2 = eos_cs2<C, EOS>(g, w[0], ee);
        ebits |= eos_check<C, EOS>(g, w[0], ee, cs2);
        red_s = fmax(red_s, fmax(fabs(vx), fabs(vy)) + fast_sqrt(cs2));
        const C h = fma(eoff, w[0], w[3]) + PP;   // physical rho E + P
        red_M[0] = fmax(red_M[0], fmax(fabs(w[1]), fabs(w[2])));
        red_M[1] = fmax(red_M[1], fmax(fabs(w[1] * vx + PP), fabs(w[2] * vx)));
        red_M[2] = fmax(red_M[2], fmax(fabs(w[1] * vy), fabs(w[2] * vy + PP)));
        red_M[3] = fmax(red_M[3], fmax(fabs(h * vx), fabs(h * vy)));
    }

    // issue the 16 population loads of row R (periodic rows wrap) into dst
    __device__ __forceinline__ void load_row(int R, S* dst)
    {
        const int mrow = (R < 0 || R >= ny) ? wrap_index(R, ny) : R;
        const unsigned off = ((unsigned)mrow * (unsigned)nx + colx) * (unsigned)sizeof(S);
#pragma unroll
        for (int j = 0; j < 16; ++j) dst[j] = bload(in, j, off, S());
    }

    // one row of the march; PH = (R - Rb) % 3.  Software-pipelined: the loads
    // of row R+1 are in flight while row R is processed.
    template <int PH>
    __device__ __forceinline__ void iter(int R)
    {
        constexpr int cR = PH, cR1 = (PH + 2) % 3, cR2 = (PH + 1) % 3, cR3 = PH, cR4 = (PH + 2) % 3;
        // ---------------- row R arrived during the previous rows; issue the loads of row
        // R+DEPTH.  The load is unconditional (past the last row it re-reads row Re, in
        // bounds): a conditional load would merge into the buffer through copies that wait
        // for the data at once.
        const bool hasA = R <= Re;
        S fa1[16];
        if constexpr (DEPTH == 1) {
#pragma unroll
            for (int j = 0; j < 16; ++j) fa1[j] = buf[0][j];
            load_row(min(R + 1, Re), buf[0]);
        } else {
            load_row(min(R + 2, Re), buf[(PH + 2) % 3]);
        }
        const S(&fa)[16] = DEPTH == 1 ? fa1 : buf[DEPTH == 1 ? 0 : PH];

        // ---------------- stage C: row p = R-3 (LDS slot cR3)
        const int p = R - 3;
        if (p >= Rb && p >= y0 - 1 && p <= y1 && p <= Re) {
            const bool plo = clo && p == 0, phi = chi && p == ny - 1;
            C beta = (C)P.beta_const;
            if constexpr (SENSOR != 0) {
                if (plo) { Ss[cR4] = Ss[cR3]; Sth[cR4] = Sth[cR3]; }
                if (phi) { Ss[cR2] = Ss[cR3]; Sth[cR2] = Sth[cR3]; }
                const C sbar = (C)0.25 * Ss[cR4] + (C)0.5 * Ss[cR3] + (C)0.25 * Ss[cR2];
                C thbar = (C)1;
                if constexpr (SENSOR == 2) thbar = (C)0.25 * Sth[cR4] + (C)0.5 * Sth[cR3] + (C)0.25 * Sth[cR2];
                const C chiv = fmin(fmax((C)P.c_sensor * sbar * thbar, (C)0), (C)1);
                beta = (C)P.beta_max - (C)(P.beta_max - P.beta_min) * chiv;
            }
            if (St.probe) {
                if (owner && p >= y0 && p < y1) St.beta_out[(long long)p * nx + X] = (double)beta;
            } else {
                // Reprojection to the new link speed (Eq. 40, holding W, J_alpha =
                // c_old (f_a+ - f_a-) and K = c_old^2 (S_x - S_y)) and relaxation
                // f* = (1 - 2 beta) f + 2 beta f^eq (Eqs. 20, 22) in moment form:
                //   f*_{x+-} = W/4 + mu (S_x - S_y) +- (nu D_x + tau Q_x),
                //   f*_{y+-} = W/4 - mu (S_x - S_y) +- (nu D_y + tau Q_y),
                // mu = (1 - 2 beta) r^2/4, nu = (1 - 2 beta) r/2, tau = 2 beta/(2 c).
                C Sx[4], Dx[4], Sy[4], Dy[4], W[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const C a0 = (C)ring[cR3][0 * 4 + k][rl], a1 = (C)ring[cR3][1 * 4 + k][rl];
                    const C a2 = (C)ring[cR3][2 * 4 + k][rl], a3 = (C)ring[cR3][3 * 4 + k][rl];
                    Sx[k] = a0 + a1;
                    Dx[k] = a0 - a1;
                    Sy[k] = a2 + a3;
                    Dy[k] = a2 - a3;
                    W[k] = Sx[k] + Sy[k];
                }
                const C irho = fast_rcp(W[0]);
                const C ux = W[1] * irho, uy = W[2] * irho;
                const C e = W[3] * irho - (C)0.5 * (ux * ux + uy * uy) + eoff;
                const C Pp = eos_pressure<C, EOS>(g, W[0], e);
                const C h = W[3] + Pp;   // stored gauge: the energy flux is Q_E - eoff Q_rho
                const C qx[4] = {W[1], W[1] * ux + Pp, W[1] * uy, h * ux};
                const C qy[4] = {W[2], W[2] * ux, W[2] * uy + Pp, h * uy};
                const C om = (C)1 - (C)2 * beta;
                const C mu = om * (C)0.25 * r * r, nu = om * (C)0.5 * r, tau = (C)2 * beta * inv2c;
                C gx[8], fyp[4], fym[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const C a = (C)0.25 * W[k], m = mu * (Sx[k] - Sy[k]);
                    const C cx = fma(nu, Dx[k], tau * qx[k]), cy = fma(nu, Dy[k], tau * qy[k]);
                    const C ap = a + m, am = a - m;
                    gx[k] = left(ap + cx);       // +x population arriving from x-1
                    gx[4 + k] = right(ap - cx);   // -x population arriving from x+1
                    fyp[k] = am + cy;
                    fym[k] = am - cy;
                }
                // a pinned x edge: its ghost's equilibrium streams in instead (nx >= 4:
                // X == 0 and X == nx - 1 are distinct columns).  Applied as a second
                // store and in the pending moments, after the streaming stores.
                const bool pin_lo = !XPER && P.bc[0] == 2 && X == 0, pin_hi = !XPER && P.bc[1] == 2 && X == nx - 1;
                // streaming stores (pull semantics: a clamped ghost repeats the edge cell)
                if (owner) {
                    const unsigned col = (unsigned)X * (unsigned)sizeof(S);
                    const unsigned rowb = (unsigned)nx * (unsigned)sizeof(S);
                    if (p >= y0 && p < y1) {
                        const unsigned b = (unsigned)p * rowb + col;
#pragma unroll
                        for (int j = 0; j < 8; ++j) bstore(out, j, b, (S)gx[j]);
                        if (pin_lo)
#pragma unroll
                            for (int k = 0; k < 4; ++k) bstore(out, k, b, (S)(C)vlbm_pin_lds[k]);
                        if (pin_hi)
#pragma unroll
                            for (int k = 0; k < 4; ++k) bstore(out, 4 + k, b, (S)(C)vlbm_pin_lds[4 + k]);
                        if (plo)
#pragma unroll
                            for (int k = 0; k < 4; ++k) bstore(out, 8 + k, b, (S)fyp[k]);
                        if (phi)
#pragma unroll
                            for (int k = 0; k < 4; ++k) bstore(out, 12 + k, b, (S)fym[k]);
                    }
                    if (p + 1 >= y0 && p + 1 < y1) {
                        const unsigned b = (unsigned)(p + 1) * rowb + col;
#pragma unroll
                        for (int k = 0; k < 4; ++k) bstore(out, 8 + k, b, (S)fyp[k]);
                    }
                    if (p - 1 >= y0 && p - 1 < y1) {
                        const unsigned b = (unsigned)(p - 1) * rowb + col;
#pragma unroll
                        for (int k = 0; k < 4; ++k) bstore(out, 12 + k, b, (S)fym[k]);
                    }
                }
                // reductions of the new state: row p-1 completes with f*_{-y}(p)
                if (owner && p - 1 >= y0 && p - 1 < y1) {
                    C w[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) w[k] = wpend[k] + fym[k];
                    reduce(w);
                }
                if (plo)
#pragma unroll
                    for (int k = 0; k < 4; ++k) yprev[k] = fyp[k];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const C gl = pin_lo ? (C)vlbm_pin_lds[k] : gx[k];
                    const C gr = pin_hi ? (C)vlbm_pin_lds[4 + k] : gx[4 + k];
                    wpend[k] = (gl + gr) + yprev[k];
                    yprev[k] = fyp[k];
                }
                if (phi && owner && p >= y0 && p < y1) {
                    C w[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) w[k] = wpend[k] + fym[k];
                    reduce(w);
                }
            }
        }

        // ---------------- stage A: row R (LDS slot cR)
        if (hasA) {
            if (lane >= kRingLo && lane < kRingLo + kRingW)
#pragma unroll
                for (int j = 0; j < 16; ++j) ring[cR][j][rl] = fa[j];
            if constexpr (SENSOR != 0) {
                C W[4];
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    W[k] = ((C)fa[0 * 4 + k] + (C)fa[1 * 4 + k]) + ((C)fa[2 * 4 + k] + (C)fa[3 * 4 + k]);
                const C irho = fast_rcp(W[0]);
                const C ux = W[1] * irho, uy = W[2] * irho;
                const C e = W[3] * irho - (C)0.5 * (ux * ux + uy * uy) + eoff;
                const C Pp = eos_pressure<C, EOS>(g, W[0], e);
                const C h = W[3] + Pp;
                const C qx[4] = {W[1], W[1] * ux + Pp, W[1] * uy, h * ux};
                const C hq[4] = {(C)0.5 * W[2], (C)0.5 * W[2] * ux, (C)0.5 * (W[2] * uy + Pp), (C)0.5 * h * uy};
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    J[cR1][k] += hq[k];                                             // completes row R-1
                    J[cR][k] += (C)0.5 * (right_col(qx[k]) - left_col(qx[k]));   // x-part of row R
                    J[cR2][k] = -hq[k];                                             // starts row R+1
                }
                C hx = 0, hy = 0;
                if constexpr (SENSOR == 2) {
                    // dilatation and vorticity in lattice units: (u(x+e) - u(x-e))/(2c),
                    // i.e. dt times the central difference (dt = dx/c)
                    hx = ux * inv2c;
                    hy = uy * inv2c;
                    Dl[cR1] += hy;
                    Vo[cR1] -= hx;
                    Dl[cR] += (right_col(ux) - left_col(ux)) * inv2c;
                    Vo[cR] += (right_col(uy) - left_col(uy)) * inv2c;
                    Dl[cR2] = -hy;
                    Vo[cR2] = hx;
                }
                if (clo && R == 0) {   // clamped: the row below row 0 is row 0
#pragma unroll
                    for (int k = 0; k < 4; ++k) J[cR][k] -= hq[k];
                    if constexpr (SENSOR == 2) { Dl[cR] -= hy; Vo[cR] += hx; }
                }
                if (chi && R == ny - 1) {   // clamped: the row above the top row is itself
#pragma unroll
                    for (int k = 0; k < 4; ++k) J[cR][k] += hq[k];
                    if constexpr (SENSOR == 2) { Dl[cR] += hy; Vo[cR] -= hx; }
                }
            }
        }

        // ---------------- stage B: row q = R-1 (slot cR1)
        if constexpr (SENSOR != 0) {
            const int q = R - 1;
            if (q >= Rb && q <= Re && q >= y0 - 2 && q <= y1 + 1) {
                C acc = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    // energy activity of the physical flux: j_E = j_E,stored + eoff j_rho
                    const C jk = k == 3 ? fma(eoff, J[cR1][0], J[cR1][3]) : J[cR1][k];
                    const C sh = jk * invM[k];
                    acc = fma(sh, sh, acc);
                }
                const C sq = fast_sqrt(acc * (C)0.25);
                Ss[cR1] = (C)0.25 * left(sq) + (C)0.5 * sq + (C)0.25 * right(sq);
                if constexpr (SENSOR == 2) {
                    const C d2 = Dl[cR1] * Dl[cR1];
                    const C th = d2 * fast_rcp(fma(Vo[cR1], Vo[cR1], d2) + (C)P.eps_theta);
                    Sth[cR1] = (C)0.25 * left(th) + (C)0.5 * th + (C)0.25 * right(th);
                }
            }
        }
    }
};

// Dynamic LDS: one 3-row ring of raw populations per wavefront.
extern __shared__ __align__(16) unsigned char vlbm_step_lds[];

// A workgroup holds P.wpg wavefronts on adjacent strips of the same segment.
// They march in step (one barrier per row), so the halo lines that
// neighbouring strips both read are fetched from HBM once and served to the
// second reader from the caches.
template <typename S, typename C, int EOS, int SENSOR, int DEPTH, bool XPER>
// up to 8 wavefronts a workgroup with FP32 storage and arithmetic (512 threads,
// at most 256 VGPRs a wavefront: the FP32 kernel holds about 145), 4 otherwise
__global__ void __launch_bounds__(sizeof(S) == 4 && sizeof(C) == 4 ? 512 : 256) k_step_d2q4(const KParams P, const KStep St, const S* __restrict__ fin,
                                                   S* __restrict__ fout)
{
    const int wave = threadIdx.x >> 6;
    S (*ring)[16][kRingW] = reinterpret_cast<S (*)[16][kRingW]>(vlbm_step_lds) + 3 * wave;

    // The march's geometry and its first rows' loads come first, then the
    // reductions of the current state and the clock logic: none depends on
    // another, so their memory latencies overlap.
    March<S, C, EOS, SENSOR, DEPTH, XPER> m{P, St};
    m.in = make_planes(fin, (unsigned)P.plane);
    m.out = make_planes((const S*)fout, (unsigned)P.plane);
    m.ring = ring;
    m.nx = P.nx;
    m.ny = P.ny;
    m.lane = threadIdx.x & 63;
    m.rl = min(max(m.lane - kRingLo, 0), kRingW - 1);
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int group = tile % P.ngroups, seg = tile / P.ngroups;
    const int strip = group * P.wpg + wave;   // past the last strip: a wavefront that owns nothing
    const int halo = (64 - P.strip_w) / 2;
    m.X = strip * P.strip_w - halo + m.lane;
    int cx = m.X;
    if (m.X < 0) cx = P.bc[0] == 0 ? wrap_index(m.X, m.nx) : 0;
    else if (m.X >= m.nx) cx = P.bc[1] == 0 ? wrap_index(m.X, m.nx) : m.nx - 1;
    m.colx = (unsigned)cx;
    m.kl = P.bc[0] != 0 && m.X == 0;   // outflow and pinned edges clamp the stencils
    m.kr = P.bc[1] != 0 && m.X == m.nx - 1;
    m.lnb = m.kl ? m.lane : max(m.lane - 1, 0);
    m.rnb = m.kr ? m.lane : min(m.lane + 1, 63);
    m.owner = m.lane >= halo && m.lane < halo + P.strip_w && m.X < m.nx && strip < P.nstrips;
    m.clo = P.bc[2] == 1;
    m.chi = P.bc[3] == 1;
    m.y0 = seg * P.seg_h;
    m.y1 = min(m.y0 + P.seg_h, m.ny);
    m.Rb = m.clo ? max(m.y0 - 3, 0) : m.y0 - 3;
    m.Re = m.chi ? min(m.y1 + 2, m.ny - 1) : m.y1 + 2;
    if (m.Rb <= m.Re) {
        m.load_row(m.Rb, m.buf[0]);
        if constexpr (decltype(m)::DEPTH == 2) m.load_row(min(m.Rb + 1, m.Re), m.buf[1]);
    }

    double R[5];   // s_max, M_k of the current state
    red_fold_wave<5>(St, R);
    double c_old, c_new, t, dt;
    bool last;
    if (!step_clock(P, St, R[0], c_old, c_new, t, dt, last)) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) write_clock(St, t, dt, c_new, last);
    if (blockIdx.x == 0 && threadIdx.x < 64 && !St.frozen) clear_reductions(St, threadIdx.x);

    if (P.bc[0] == 2 || P.bc[1] == 2) {
        if (threadIdx.x < 2 && P.bc[threadIdx.x] == 2) {
            C pe[4];
            pinned_feq<C, EOS>(P, make_gas<C>(P), (int)threadIdx.x, (C)(0.5 / c_new), (C)P.e_off, pe);
#pragma unroll
            for (int k = 0; k < 4; ++k) vlbm_pin_lds[4 * threadIdx.x + k] = (double)pe[k];
        }
        __syncthreads();
    }

    m.g = make_gas<C>(P);
    // c_old == c_new gives r = 1: the reprojection is then the identity
    m.r = (C)(c_old / c_new);
    m.inv2c = (C)(0.5 / c_new);
#pragma unroll
    for (int k = 0; k < 4; ++k) m.invM[k] = R[1 + k] > 0.0 ? (C)(1.0 / R[1 + k]) : (C)0;
    m.eoff = (C)P.e_off;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        m.Dl[s] = m.Vo[s] = m.Ss[s] = m.Sth[s] = (C)0;
#pragma unroll
        for (int k = 0; k < 4; ++k) m.J[s][k] = (C)0;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) m.yprev[k] = m.wpend[k] = m.red_M[k] = (C)0;
    m.red_s = (C)0;
    m.ebits = 0;

    const int Rlast = m.y1 + 3;
    // every wavefront of the workgroup runs the same rows (same segment), so the
    // barriers are reached uniformly
    for (int R = m.Rb; R <= Rlast; R += 3) {
        m.template iter<0>(R);
        __syncthreads();
        if (R + 1 <= Rlast) {
            m.template iter<1>(R + 1);
            __syncthreads();
        }
        if (R + 2 <= Rlast) {
            m.template iter<2>(R + 2);
            __syncthreads();
        }
    }
    if (!St.probe) {
        double M[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) M[k] = (double)m.red_M[k];
        int bits = 0;
        bits |= m.ebits;
        if (!isfinite(m.red_s)) bits |= ERR_NONFINITE;
        wave_publish(St, (double)m.red_s, M, 4, bits);
    }
}

// ------------------------------------------------------------------ launchers

template <typename S, typename C, int DEPTH>
static hipError_t launch_t(const KParams& p, const KStep& s, const void* fin, void* fout, hipStream_t st)
{
    const dim3 grid(p.ngroups * p.nsegs), block(64 * p.wpg);
    const size_t lds = (size_t)p.wpg * 3 * 16 * kRingW * sizeof(S);
    const S* in = (const S*)fin;
    S* out = (S*)fout;
#define VLBM_CASE(E, SN)                                                                                     \
    if (p.eos == E && p.sensor == SN) {                                                                    \
        if (p.bc[0] == 0)                                                                                  \
            hipLaunchKernelGGL((k_step_d2q4<S, C, E, SN, DEPTH, true>), grid, block, lds, st, p, s, in, out);  \
        else                                                                                               \
            hipLaunchKernelGGL((k_step_d2q4<S, C, E, SN, DEPTH, false>), grid, block, lds, st, p, s, in, out); \
        return hipGetLastError();                                                                          \
    }
    VLBM_CASE(0, 0) VLBM_CASE(0, 1) VLBM_CASE(0, 2) VLBM_CASE(1, 0) VLBM_CASE(1, 1) VLBM_CASE(1, 2)
#undef VLBM_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_step_d2q4(const KParams& p, const KStep& s, int prec, const void* fin, void* fout, hipStream_t st)
{
    switch (prec) {
    case PREC_FP64:
        return p.deep ? launch_t<double, double, 2>(p, s, fin, fout, st) : launch_t<double, double, 1>(p, s, fin, fout, st);
    case PREC_FP32: return launch_t<float, float, 2>(p, s, fin, fout, st);
    case PREC_FP32_MIXED: return launch_t<float, double, 2>(p, s, fin, fout, st);
    }
    return hipErrorInvalidValue;
}

// Measurement aid: the step's memory access pattern with none of its
// arithmetic.  Same grid, tiling (strips with their halo lanes, segments with
// their 3-row halos, wpg wavefronts marching in step, XCD remapping), buffer
// addressing and two rows of loads in flight; every row's 16 planes are loaded
// and the owned cells' values are stored where the step stores post-collision
// populations: the x planes into the same row (moved one lane across the
// wavefront, as streaming moves them), the +y planes into the row above, the -y
// planes into the row below.  It bounds what the step's own access pattern can
// move through HBM.
template <typename S>
__global__ void __launch_bounds__(sizeof(S) == 4 ? 512 : 256) k_march_probe(const KParams P, const S* __restrict__ fin, S* __restrict__ fout)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const Planes in = make_planes(fin, (unsigned)P.plane), out = make_planes((const S*)fout, (unsigned)P.plane);
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int group = tile % P.ngroups, seg = tile / P.ngroups;
    const int strip = group * P.wpg + wave;
    const int halo = (64 - P.strip_w) / 2;
    const int X = strip * P.strip_w - halo + lane;
    int cx = X;
    if (X < 0) cx = P.bc[0] == 0 ? wrap_index(X, P.nx) : 0;
    else if (X >= P.nx) cx = P.bc[1] == 0 ? wrap_index(X, P.nx) : P.nx - 1;
    const bool owner = lane >= halo && lane < halo + P.strip_w && X < P.nx && strip < P.nstrips;
    const bool clo = P.bc[2] == 1, chi = P.bc[3] == 1;
    const int y0 = seg * P.seg_h, y1 = min(y0 + P.seg_h, P.ny);
    const int Rb = clo ? max(y0 - 3, 0) : y0 - 3, Re = chi ? min(y1 + 2, P.ny - 1) : y1 + 2;
    const unsigned rowb = (unsigned)P.nx * (unsigned)sizeof(S), col = (unsigned)X * (unsigned)sizeof(S);
    S buf[3][16];
    auto load_row = [&](int R, S* dst) {
        const int mrow = (R < 0 || R >= P.ny) ? wrap_index(R, P.ny) : R;
        const unsigned off = (unsigned)mrow * rowb + (unsigned)cx * (unsigned)sizeof(S);
#pragma unroll
        for (int j = 0; j < 16; ++j) dst[j] = bload(in, j, off, S());
    };
    auto row = [&](int R, S* cur) {
        if (P.wpg > 1) __syncthreads();
        S gx[8];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            gx[k] = dpp_move<kDppWaveShr1>(cur[k]);
            gx[4 + k] = dpp_move<kDppWaveShl1>(cur[4 + k]);
        }
        if (!owner) return;
        if (R >= y0 && R < y1)
#pragma unroll
            for (int j = 0; j < 8; ++j) bstore(out, j, (unsigned)R * rowb + col, gx[j]);
        if (R + 1 >= y0 && R + 1 < y1)
#pragma unroll
            for (int k = 0; k < 4; ++k) bstore(out, 8 + k, (unsigned)(R + 1) * rowb + col, cur[8 + k]);
        if (R - 1 >= y0 && R - 1 < y1)
#pragma unroll
            for (int k = 0; k < 4; ++k) bstore(out, 12 + k, (unsigned)(R - 1) * rowb + col, cur[12 + k]);
    };
    load_row(Rb, buf[0]);
    load_row(min(Rb + 1, Re), buf[1]);
    // unrolled by three so that the buffer index is a compile-time constant; the
    // loads are unconditional (past the last row they re-read row Re, in bounds)
    for (int R = Rb; R <= Re; R += 3) {
        load_row(min(R + 2, Re), buf[2]);
        row(R, buf[0]);
        if (R + 1 <= Re) {
            load_row(min(R + 3, Re), buf[0]);
            row(R + 1, buf[1]);
        }
        if (R + 2 <= Re) {
            load_row(min(R + 4, Re), buf[1]);
            row(R + 2, buf[2]);
        }
    }
}

hipError_t launch_march_probe(const KParams& p, bool fp32, const void* fin, void* fout, hipStream_t st)
{
    const dim3 grid(p.ngroups * p.nsegs), block(64 * p.wpg);
    if (fp32)
        hipLaunchKernelGGL(k_march_probe<float>, grid, block, 0, st, p, (const float*)fin, (float*)fout);
    else
        hipLaunchKernelGGL(k_march_probe<double>, grid, block, 0, st, p, (const double*)fin, (double*)fout);
    return hipGetLastError();
}

int step_d2q4_blocks_per_cu(const KParams& p, int prec)
{
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
    const int bs = 64 * p.wpg;
    const size_t l8 = (size_t)p.wpg * 3 * 16 * kRingW * 8, l4 = l8 / 2;
    switch (prec) {
    case PREC_FP64:
        e = p.deep ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_step_d2q4<double, double, 0, 2, 2, false>, bs, l8)
                   : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_step_d2q4<double, double, 0, 2, 1, false>, bs, l8);
        break;
    case PREC_FP32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_step_d2q4<float, float, 0, 2, 2, false>, bs, l4); break;
    case PREC_FP32_MIXED: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_step_d2q4<float, double, 0, 2, 2, false>, bs, l4); break;
    }
    return e == hipSuccess ? nb : 0;
}


// rows per segment of the D2Q4 march: enough wavefronts to fill every CU
// once at the kernel's occupancy, without a partial second round
static int choose_seg_h(const KParams& p, int prec)
{
    if (const char* env = getenv("VLBM_SEG_H")) {
        const int v = atoi(env);
        if (v > 0) return std::min(v, p.ny);
    }
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
            cus = prop.multiProcessorCount;
    }
    int per_cu = step_d2q4_blocks_per_cu(p, prec);
    if (per_cu <= 0) per_cu = 8 / p.wpg > 0 ? 8 / p.wpg : 1;
    const long long resident = (long long)cus * per_cu;   // workgroups resident at once
    long long nsegs = std::max(1LL, resident / p.ngroups);
    int h = (int)((p.ny + nsegs - 1) / nsegs);
    // at least 10 rows: shorter segments spend more on their 6 halo rows than
    // the extra wavefronts win (measured on MI355X at 512^2 and 1024^2, where
    // 10-11 rows beat 16 by 9-20 % and 8 rows lose again).  FP64 frozen-speed
    // contexts keep 16: the adjoint rollout replays them beside the FP64 adjoint
    // march, which then finds free slots (end to end 3.4 -> 3.1 at 1024^2).
    int hmin = prec == PREC_FP64 && p.retarget_every == 0 ? 16 : 10;
    if (const char* env = getenv("VLBM_SEG_MIN")) hmin = std::max(1, atoi(env));
    h = std::max(h, hmin);
    return std::min(h, p.ny);
}

void configure_d2q4(KParams& p, int prec)
{
    // D2Q4 strips of 56 columns (4 halo lanes a side); measured faster than 48
    // columns (three whole FP64 lines, but 16 halo lanes), and than 32
    p.strip_w = 56;
    if (const char* env = getenv("VLBM_STRIP_W")) {
        const int v = atoi(env);
        if (v >= 8 && v <= 56 && v % 2 == 0) p.strip_w = v;   // the step's LDS ring covers halos >= 4
    }
    p.nstrips = (p.nx + p.strip_w - 1) / p.strip_w;
    // FP64 below 1.5M cells: two rows of loads in flight per wavefront at one
    // wavefront per SIMD, where too few strips x segments exist to fill a second
    // (measured on MI355X: 512^2 and 1024^2 3-8 % faster; 1280^2 and 1536^2
    // 1.5 % slower, 2048^2 5 %, 4096^2 14 %).  Not for frozen-speed contexts:
    // they serve the adjoint rollout, whose replay runs beside the FP64 adjoint
    // march, and a wavefront holding more than half of a SIMD's registers
    // (255 VGPRs and 14 AGPRs) cannot share it with one of the march's (248).
    const long long cells = p.nx * (long long)p.ny;
    const bool small = cells < (1LL << 22);
    p.deep = prec == PREC_FP64 && cells < 3 * (1LL << 19) && p.retarget_every != 0;
    if (const char* env = getenv("VLBM_DEEP")) p.deep = prec == PREC_FP64 && atoi(env) != 0;
    // adjacent strips per workgroup (measured on MI355X): 2 FP64 wavefronts
    // (22 KB of LDS ring each), 1 with two rows in flight; with FP32 storage 4
    // on large grids, where the shared halo lines save HBM traffic, and 1 below
    // 4M cells, where the march is latency-bound and the per-row barrier costs
    // more than it saves.  FP32 arithmetic: 8, one workgroup a CU (87 KB of
    // LDS) whose eight strips share their halo lines, against three of 4, with
    // the strips narrowed below to spread the columns evenly (Riemann
    // configuration 3 under Sensor B, fractions of 8 TB/s: 4096^2 58.6 against
    // 56.1 %, 2896^2 55.0 / 53.8, 2560^2 53.9 / 52.7, 2048^2 47.8 / 45.7; the
    // dense-gas extrusion at 2048^2 46.1 / 44.8; 5, 6, 10 and 12 slower at
    // 4096^2).  The FP64 arithmetic of the mixed form loses with 8 (52.1
    // against 54.7 %).
    p.wpg = prec == PREC_FP64 ? (p.deep ? 1 : 2) : (small ? 1 : (prec == PREC_FP32 ? 8 : 4));
    if (const char* env = getenv("VLBM_WPG")) {
        const int v = atoi(env);
        if (v >= 1 && v <= (prec == PREC_FP32 ? 8 : 4)) p.wpg = v;
    }
    // 8 FP32 strips a workgroup: as few workgroups as 56-column strips need,
    // then the narrowest strips (a multiple of 4 columns, so that every
    // workgroup's span starts on a 128-byte line) that still cover the grid,
    // which spreads the columns evenly over the workgroups (4096^2: 52-column
    // strips, 58.6 against 57.5 % of 8 TB/s; 48 columns 58.3 %, and 50 and 54,
    // off the line grid, 56.1 and 56.5 %)
    if (p.wpg == 8 && !getenv("VLBM_STRIP_W")) {
        const int ng = (p.nx + 8 * 56 - 1) / (8 * 56);
        const int sw = ((p.nx + 8 * ng - 1) / (8 * ng) + 3) / 4 * 4;
        if (sw >= 40 && sw <= 56) {
            p.strip_w = sw;
            p.nstrips = (p.nx + p.strip_w - 1) / p.strip_w;
        }
    }
    p.wpg = std::min(p.wpg, p.nstrips);
    p.ngroups = (p.nstrips + p.wpg - 1) / p.wpg;
    p.seg_h = p.ny;
    p.nsegs = 1;
    if (p.dim == 2) {
        p.seg_h = choose_seg_h(p, prec);
        p.nsegs = (p.ny + p.seg_h - 1) / p.seg_h;
    }

}

}  // namespace vlbm
