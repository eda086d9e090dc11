// D1Q2 VLBM steps for small grids in one resident workgroup (arXiv 2609.10639,
// Sec. III).
//
// At a few thousand cells a step moves a few hundred kilobytes, and a launch
// per step costs its fixed latency (the control block's loads, the
// populations' HBM round trip, the end-of-kernel write-back: about 14 us per
// step on MI355X for 1000 or 8192 cells) many times over the arithmetic.
// Here one workgroup runs a whole batch of steps on one CU: each thread holds
// K consecutive cells' populations in registers, threads exchange the values
// at their chunk edges through LDS, and the global maxima that the next step
// needs (s_max for the retarget of Eq. 37 and the normalisers M_k of Eq. 29)
// are reduced across the workgroup every step.  Only the first state is read
// from HBM and only the last one written back, with its clock and reductions,
// so the ring protocol of the per-step kernel (state n in buffer n & 1, its
// clock and reductions in ring slot n % 3) holds after the launch and both
// paths can follow each other.
//
// The workgroup has as few waves as cover the grid at K cells per lane, at
// most one per SIMD where the registers allow: every wave repeats the
// per-step work that does not depend on its cells (the clock and its
// divisions, the reductions, the barriers), so fewer, fuller waves finish a
// step sooner; the cells' arithmetic is the same either way.
//
// The arithmetic is that of the per-step kernel, in the same order: moments,
// reprojection (D = 1 form of Eq. 40), flux (Eq. 10), Sensor A (Eqs. 28-31,
// 34), relaxation (Eqs. 20, 22), pull-streaming (Eq. 21), edge rules, then the
// reductions of the new state and the clock logic (Eq. 37 and the landing),
// so both paths give the same bits.
#include <cstdio>
#include <cstdlib>

#include "vlbm_aux.hpp"
#include "vlbm_d1q2_cell.hpp"

namespace vlbm {

template <typename ST, typename T, int EOS, int SENSOR, int K, int NT>
__global__ void __launch_bounds__(NT) k_run_d1q2_resident(const KParams P, const KRun R, ST* __restrict__ f0,
                                                           ST* __restrict__ f1)
{
    // no fused multiply-adds beyond the ones written out, as in the per-step
    // kernel: where the compiler fuses depends on the code around an
    // expression, which differs between the two kernels
#pragma clang fp contract(off)
    // chunk-edge exchange: the flux Q_k of each chunk's first and last cell
    // (phase A), then the post-collision +x populations of its last cell and
    // -x populations of its first (phase C); the activity s of both edges
    __shared__ T xq[6][NT];
    __shared__ T xs[2][NT];
    __shared__ T xg[2][3];   // a clamped edge's own population streaming back in (x-low +x, x-high -x)
    __shared__ double xr[NT / 64][4];
    __shared__ int xe[NT / 64];

    const unsigned long long stop0 = *R.stop_at;
    if ((unsigned long long)R.n0 >= stop0 || R.count <= 0) return;
    const long long n_end = (unsigned long long)(R.n0 + R.count) < stop0 ? R.n0 + R.count : (long long)stop0;

    // clock and reductions of the first state (ring slot n0 % 3, maximum over the copies)
    const double* slot = R.ring + kSlot * (R.n0 % 3);
    double t = slot[0], c = slot[1];
    double red[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double v = slot[kRedBase + k];
        for (int i = 1; i < kRedCopies; ++i) v = fmax(v, slot[kRedBase + i * kRedStride + k]);
        red[k] = v;
    }

    const int tid = threadIdx.x;
    const int nw = blockDim.x >> 6;   // waves of this launch
    const int nt = blockDim.x;
    const int nx = P.nx;
    const long long plane = P.plane;
    const int x0 = tid * K;
    const int nmine = nx - x0 >= K ? K : (nx - x0 > 0 ? nx - x0 : 0);
    const bool cl = P.bc[0] != 0, ch = P.bc[1] != 0;
    const bool pl = P.bc[0] == 2, ph = P.bc[1] == 2;
    const bool first_edge = tid == 0;                      // owns cell 0
    const bool last_edge = nmine > 0 && x0 + nmine == nx;  // owns cell nx - 1
    // threads holding the neighbours of the first and the last owned cell
    // (across a periodic edge: the owner of the other end's cell)
    const int il = first_edge ? (nx - 1) / K : tid - 1;
    const int ir = last_edge ? 0 : (tid + 1 < nt ? tid + 1 : tid);
    // at a clamped (outflow or pinned) edge the neighbour is the cell itself;
    // every exchange below is one LDS load from a selected address, so that
    // no load waits behind a branch
    const bool self_l = first_edge && cl, self_r = last_edge && ch;

    D1Consts<T> cs;
    cs.g = make_gas<T>(P);
    cs.eoff = (T)P.e_off;
    const int re = P.retarget_every;
    int phase = re > 0 ? (int)(R.n0 % re) : 0;   // n % retarget_every

    ST f[K][6];
    {
        const ST* fin = (R.n0 & 1) ? f1 : f0;
#pragma unroll
        for (int j = 0; j < K; ++j)
#pragma unroll
            for (int q = 0; q < 6; ++q) f[j][q] = j < nmine ? fin[q * plane + x0 + j] : (ST)0;
    }

    long long n = R.n0;
    int bits = 0;
    bool landed = false;
    while (n < n_end) {
        // ---- clock (Sec. III.E): retarget c = s_max/CFL, dt = dx/c, landing on t_end
        const double c_old = c;
        double c_new = c_old;
        if (re > 0 && (phase == 0 || red[0] > c_old)) c_new = red[0] / P.cfl;
        double dt = P.dx / c_new;
        bool last = false;
        if (R.t_end < HUGE_VAL && t + dt >= R.t_end * (1.0 - 1e-14)) {
            dt = R.t_end - t;
            c_new = P.dx / dt;
            last = true;
        }
        cs.reproj = c_old != c_new;
        cs.r = (T)(c_old / c_new);
        cs.inv2c = (T)(0.5 / c_new);
#pragma unroll
        for (int k = 0; k < 3; ++k) cs.invM[k] = red[1 + k] > 0.0 ? (T)(1.0 / red[1 + k]) : (T)0;

        // ---- A: reprojection to the new link speed, flux Q(W)
        T fr[K][6], q[K][3];
#pragma unroll
        for (int j = 0; j < K; ++j) d1_flux<ST, T, EOS>(cs, f[j], fr[j], q[j]);
        // the last owned cell's values (a partial chunk ends before K)
        T qlast[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) qlast[k] = q[K - 1][k];
#pragma unroll
        for (int j = 0; j < K - 1; ++j)
            if (j == nmine - 1)
#pragma unroll
                for (int k = 0; k < 3; ++k) qlast[k] = q[j][k];

        // ---- B: normalised flux-divergence activity s (Eqs. 28-31)
        T sv[K];
        T slast = (T)0;
        if constexpr (SENSOR != 0) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                xq[k][tid] = q[0][k];
                xq[3 + k][tid] = qlast[k];
            }
            __syncthreads();
            T ql[3], qr[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                ql[k] = *(self_l ? &xq[k][tid] : &xq[3 + k][il]);
                qr[k] = *(self_r ? &xq[3 + k][tid] : &xq[k][ir]);
            }
#pragma unroll
            for (int j = 0; j < K; ++j) {
                T left[3], right[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    left[k] = j == 0 ? ql[k] : q[j - 1 >= 0 ? j - 1 : 0][k];
                    right[k] = (j == nmine - 1 || j == K - 1) ? qr[k] : q[j + 1 < K ? j + 1 : j][k];
                }
                sv[j] = d1_activity(cs, left, right);
            }
            slast = sv[K - 1];
#pragma unroll
            for (int j = 0; j < K - 1; ++j)
                if (j == nmine - 1) slast = sv[j];
            xs[0][tid] = sv[0];
            xs[1][tid] = slast;
            __syncthreads();
        }

        // ---- C: box filter, beta (Sensor A, Eq. 34), over-relaxation (Eqs. 20, 22)
        T gpc[K][6];
        {
            T sl = 0, sr = 0;
            if constexpr (SENSOR != 0) {
                sl = *(self_l ? &xs[0][tid] : &xs[1][il]);
                sr = *(self_r ? &xs[1][tid] : &xs[0][ir]);
            }
#pragma unroll
            for (int j = 0; j < K; ++j) {
                T beta;
                if constexpr (SENSOR != 0) {
                    const T left = j == 0 ? sl : sv[j - 1 >= 0 ? j - 1 : 0];
                    const T right = (j == nmine - 1 || j == K - 1) ? sr : sv[j + 1 < K ? j + 1 : j];
                    beta = d1_beta<T, SENSOR>(P, left, sv[j], right);
                } else {
                    beta = d1_beta<T, SENSOR>(P, (T)0, (T)0, (T)0);
                }
                d1_collide(cs, fr[j], q[j], beta, gpc[j]);
            }
        }
        T glast[6];
#pragma unroll
        for (int p = 0; p < 6; ++p) glast[p] = gpc[K - 1][p];
#pragma unroll
        for (int j = 0; j < K - 1; ++j)
            if (j == nmine - 1)
#pragma unroll
                for (int p = 0; p < 6; ++p) glast[p] = gpc[j][p];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            xq[k][tid] = glast[k];           // +x populations leaving the last cell
            xq[3 + k][tid] = gpc[0][3 + k];  // -x populations leaving the first cell
            if (self_l) xg[0][k] = gpc[0][k];
            if (self_r) xg[1][k] = glast[3 + k];
        }
        __syncthreads();

        // ---- D: pull-streaming (Eq. 21), edge rules, reductions of the new state
        double red_s = 0.0, red_M[3] = {0.0, 0.0, 0.0};
        int eb = 0;
        {
            T gl[3], gr[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                gl[k] = *(self_l ? &xg[0][k] : &xq[k][il]);
                gr[k] = *(self_r ? &xg[1][k] : &xq[3 + k][ir]);
            }
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const int X = x0 + j;
                T gn[6];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    gn[k] = j == 0 ? gl[k] : gpc[j - 1 >= 0 ? j - 1 : 0][k];
                    gn[3 + k] = (j == nmine - 1 || j == K - 1) ? gr[k] : gpc[j + 1 < K ? j + 1 : j][3 + k];
                }
                if ((pl && X == 0) || (ph && X == nx - 1)) {   // nx >= 4: distinct cells
                    T pe[3];
                    const int side = X == 0 ? 0 : 1;
                    pinned_feq<T, EOS>(P, cs.g, side, cs.inv2c, cs.eoff, pe);
#pragma unroll
                    for (int k = 0; k < 3; ++k) gn[side * 3 + k] = pe[k];
                }
#pragma unroll
                for (int p = 0; p < 6; ++p) f[j][p] = (ST)gn[p];
                if (j >= nmine) continue;   // past the grid's end (a partial or idle chunk)
                d1_reduce<T, EOS>(cs, gn, red_s, red_M, eb);
            }
        }
        // wave maxima (every lane), then the maximum over the waves from LDS
        red_s = wave_max_dpp(red_s);
#pragma unroll
        for (int k = 0; k < 3; ++k) red_M[k] = wave_max_dpp(red_M[k]);
        const int ebw = (__any(eb & ERR_NONHYP) ? ERR_NONHYP : 0) | (__any(eb & ERR_NONFINITE) ? ERR_NONFINITE : 0);
        if ((tid & 63) == 0) {
            const int w = tid >> 6;
            xr[w][0] = red_s;
#pragma unroll
            for (int k = 0; k < 3; ++k) xr[w][1 + k] = red_M[k];
            xe[w] = ebw;
        }
        __syncthreads();
        int all = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) red[k] = 0.0;
        for (int w = 0; w < nw; ++w) {
#pragma unroll
            for (int k = 0; k < 4; ++k) red[k] = fmax(red[k], xr[w][k]);
            all |= xe[w];
        }

        t = last ? R.t_end : t + dt;
        c = c_new;
        ++n;
        if (re > 0 && ++phase == re) phase = 0;
        if (all) {
            bits = all;
            break;
        }
        if (last) {
            landed = true;
            break;
        }
    }

    // state n back to buffer n & 1; its clock and reductions to ring slot n % 3
    // (copy 0, the other copies zero); the slot after it cleared for the next step
    ST* fout = (n & 1) ? f1 : f0;
#pragma unroll
    for (int j = 0; j < K; ++j)
        if (j < nmine)
#pragma unroll
            for (int p = 0; p < 6; ++p) fout[p * plane + x0 + j] = f[j][p];
    double* so = R.ring + kSlot * (n % 3);
    double* sn = R.ring + kSlot * ((n + 1) % 3);
    for (int i = tid; i < kRedCopies * kRedFields; i += nt) {
        const int copy = i / kRedFields, fld = i % kRedFields;
        so[kRedBase + copy * kRedStride + fld] = copy == 0 && fld < 4 ? red[fld] : 0.0;
        sn[kRedBase + copy * kRedStride + fld] = 0.0;
    }
    if (tid == 0) {
        so[0] = t;
        so[1] = c;
        if (bits) atomicOr(R.err, bits);
        if (bits || landed) atomicMin(R.stop_at, (unsigned long long)n);
    }
}

namespace {

// Launch shapes: K cells per lane in a workgroup of at most NT threads, the
// first that covers the grid.  Measured on MI355X (Sod and BZT tubes, every
// precision, same bits from every shape): at 1000 cells 4 cells a lane in 4
// waves (3.6-3.9 us a step) beat 1 in 16 waves (5.1-6.2) and 8 in 2 (5.3-6.7);
// at 2000 cells 4 in 8 waves beat 8 in 4.
//
// The resident path is taken where it beats one launch per step (about 6.1-6.4
// us a step at these sizes, 1 cell a lane): up to 2048 cells (FP32 5.0 against
// 6.3 us at 2000 cells, FP64 5.9 against 6.5, FP32 storage with FP64
// arithmetic even at 6.1).  At 2500-4000 cells 8 cells a lane in 8 waves take
// 7.4-7.7 us in FP32, and one launch per step is faster.
struct ResShape {
    int K, NT;
};
constexpr ResShape kShapes[] = {{2, 256}, {4, 256}, {4, 512}};

bool pick_shape(int nx, ResShape& out)
{
    if (const char* env = getenv("VLBM_D1_SHAPE")) {   // tuning override "K,NT", one of the shapes
        int k = 0, nt = 0;
        if (sscanf(env, "%d,%d", &k, &nt) == 2)
            for (const ResShape& s : kShapes)
                if (s.K == k && s.NT == nt && nx <= k * nt) return out = s, true;
    }
    for (const ResShape& s : kShapes)
        if (nx <= s.K * s.NT) return out = s, true;
    return false;
}

template <typename ST, typename T, int K, int NT>
hipError_t launch_k(const KParams& p, const KRun& r, void* f0, void* f1, hipStream_t st)
{
    const int lanes = (p.nx + K - 1) / K;
    const dim3 block((lanes + 63) / 64 * 64);
#define VLBM_CASE(E, SN)                                                                                          \
    if (p.eos == E && p.sensor == SN) {                                                                           \
        hipLaunchKernelGGL((k_run_d1q2_resident<ST, T, E, SN, K, NT>), dim3(1), block, 0, st, p, r, (ST*)f0, \
                           (ST*)f1);                                                                             \
        return hipGetLastError();                                                                                 \
    }
    VLBM_CASE(0, 0) VLBM_CASE(0, 1) VLBM_CASE(1, 0) VLBM_CASE(1, 1)
#undef VLBM_CASE
    return hipErrorInvalidValue;
}

template <typename ST, typename T>
hipError_t launch_prec(const KParams& p, const KRun& r, const ResShape& s, void* f0, void* f1, hipStream_t st)
{
    if (s.K == 2 && s.NT == 256) return launch_k<ST, T, 2, 256>(p, r, f0, f1, st);
    if (s.K == 4 && s.NT == 256) return launch_k<ST, T, 4, 256>(p, r, f0, f1, st);
    if (s.K == 4 && s.NT == 512) return launch_k<ST, T, 4, 512>(p, r, f0, f1, st);
    return hipErrorInvalidValue;
}

}  // namespace

int resident_d1q2_max_cells(int)
{
    return 4 * 512;
}

hipError_t launch_run_d1q2(const KParams& p, const KRun& r, int prec, void* f0, void* f1, hipStream_t st)
{
    ResShape s;
    if (p.dim != 1 || p.nx < 4 || p.nx > resident_d1q2_max_cells(prec) || !pick_shape(p.nx, s))
        return hipErrorInvalidValue;
    switch (prec) {
    case PREC_FP64: return launch_prec<double, double>(p, r, s, f0, f1, st);
    case PREC_FP32: return launch_prec<float, float>(p, r, s, f0, f1, st);
    case PREC_FP32_MIXED: return launch_prec<float, double>(p, r, s, f0, f1, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace vlbm
