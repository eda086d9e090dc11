// Internal definitions shared by the HIP kernels and the host runtime of the
// VLBM library (arXiv 2609.10639).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vlbm {

// Static problem parameters, passed by value to every kernel.
struct KParams {
    int dim, nx, ny;
    long long plane;          // elements per population plane (padded)
    double dx;
    int bc[4];                // x-lo, x-hi, y-lo, y-hi: 0 periodic, 1 outflow (clamped ghost),
                              // 2 pinned (x edges: ghost at equilibrium of pin_w[side])
    double pin_w[2][4];       // conserved state of a pinned x-lo / x-hi ghost (physical gauge)
    int eos;                  // 0 ideal, 1 van der Waals
    double gamma, vdw_a, vdw_b, vdw_R, inv_cv;
    double e_off;             // energy gauge: populations carry rho E - e_off rho in the energy component
    double cfl, c_fixed;
    int retarget_every;
    int sensor;               // resolved: 0 off, 1 A (no gate), 2 B (Ducros gate)
    double beta_const, beta_min, beta_max, c_sensor, eps_theta;
    int strip_w;              // D2Q4: output columns per wavefront (56; halo lanes (64 - strip_w)/2 a side)
    int nstrips, seg_h, nsegs; // D2Q4 tiling: strips of columns x segments of rows
    int wpg, ngroups;         // D2Q4 step: wavefronts (adjacent strips) per workgroup, strip groups
    int deep;                 // D2Q4 FP64 step: two rows of loads in flight (one wavefront per SIMD)
};

// Per-launch control: where the clock and the reductions of the current state
// are read from and where those of the next state go.
//
// Reductions (s_max, then max|Q_alpha,k| for each component k) are kept in
// `red_copies` copies, `red_stride` doubles apart: a workgroup publishes its
// maxima into copy blockIdx % red_copies and readers take the maximum over the
// copies (exact and order-free).  Spreading the atomics over copies on
// separate cache lines keeps same-address atomics from serialising at the end
// of a launch.  red_copies <= 1 means one copy.
//
// Ring slot (kSlot doubles): [0] t, [1] c, copy i of the reductions at
// kRedBase + i kRedStride.  Step n reads slot n%3, writes the clock and
// accumulates the reductions of the new state into slot (n+1)%3, and clears
// the reductions of slot (n+2)%3.
constexpr int kRedCopies = 16, kRedStride = 16, kRedBase = 16;
constexpr int kSlot = kRedBase + kRedCopies * kRedStride;
constexpr int kRedFields = 6;      // s_max and up to 4 components, plus one spare

struct KStep {
    const double* clock_in;        // t, c of the current state
    double* clock_out;             // t, c after the step (block 0 writes)
    const double* red_in;          // s_max, M_k of the current state (copy 0)
    double* red_out;               // s_max, M_k of the new state (atomic max, copy 0)
    double* red_clear;             // reductions to zero (copy 0, nullable)
    int red_copies;                // copies of the three reduction blocks
    int red_stride;                // doubles between copies
    unsigned long long* stop_at;   // steps with n >= *stop_at return at once (nullable)
    int* err;                      // error bits (1: non-hyperbolic, 2: non-finite)
    long long n;                   // index of this step
    double t_end;                  // landing time (HUGE_VAL: none)
    int frozen;                    // 1: c = c_fixed, no clock update, no landing
    int probe;                     // 1: write beta of the current state to beta_out, no populations
    double* beta_out;              // probe output, FP64 (ny, nx)
};

// population storage / arithmetic precision of a context
constexpr int PREC_FP64 = 0;        // FP64 populations, FP64 arithmetic
constexpr int PREC_FP32 = 1;        // FP32 populations, FP32 arithmetic
constexpr int PREC_FP32_MIXED = 2;  // FP32 populations, FP64 arithmetic

constexpr int ERR_NONHYP = 1;
constexpr int ERR_NONFINITE = 2;

// ------------------------------------------------------------- device helpers

// Reciprocal from the hardware estimate refined by Newton-Raphson steps
// (e = 1 - x r, r <- r + r e): two steps in FP64 bring it to within about an
// ulp of the correctly rounded quotient; in FP32 the estimate (1 ulp) is used.
__device__ __forceinline__ double fast_rcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Square root of x >= 0 (0 for x <= 0): FP64 from the reciprocal square-root
// estimate with Newton-Raphson refinement of s = x/sqrt(x) and h = 1/(2 sqrt(x));
// FP32 from the hardware square root (1 ulp).
__device__ __forceinline__ double fast_sqrt(double x)
{
    if (!(x > 0.0)) return 0.0;
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double d = fma(-g, g, x);
    return fma(d, h, g);
}
__device__ __forceinline__ float fast_sqrt(float x) { return x > 0.0f ? __builtin_amdgcn_sqrtf(x) : 0.0f; }

template <typename T>
struct Gas {
    T gm1, gamma, a, b, R, inv_cv;
};

template <typename T>
__device__ __forceinline__ Gas<T> make_gas(const KParams& p)
{
    Gas<T> g;
    g.gamma = (T)p.gamma;
    g.gm1 = (T)(p.gamma - 1.0);
    g.a = (T)p.vdw_a;
    g.b = (T)p.vdw_b;
    g.R = (T)p.vdw_R;
    g.inv_cv = (T)p.inv_cv;
    return g;
}

// Pressure P(rho, e): ideal gas Eq. 15; van der Waals Eqs. 16-17 with
// T = (e + a rho)/c_v.
template <typename T, int EOS>
__device__ __forceinline__ T eos_pressure(const Gas<T>& g, T rho, T e)
{
    if constexpr (EOS == 0) {
        return g.gm1 * rho * e;
    } else {
        const T temp = (e + g.a * rho) * g.inv_cv;
        return g.R * rho * temp * fast_rcp((T)1 - g.b * rho) - g.a * rho * rho;
    }
}

// Frozen isentropic sound speed squared (Eq. 13) in closed form:
// ideal gamma (gamma-1) e; van der Waals gamma R T/(1 - b rho)^2 - 2 a rho.
template <typename T, int EOS>
__device__ __forceinline__ T eos_cs2(const Gas<T>& g, T rho, T e)
{
    if constexpr (EOS == 0) {
        return g.gamma * g.gm1 * e;
    } else {
        const T temp = (e + g.a * rho) * g.inv_cv;
        const T d = (T)1 - g.b * rho;
        return g.gamma * g.R * temp * fast_rcp(d * d) - (T)2 * g.a * rho;
    }
}

// Admissibility bits of a state (Eq. 14 and the domain of the vdW closure).
template <typename T, int EOS>
__device__ __forceinline__ int eos_check(const Gas<T>& g, T rho, T e, T cs2)
{
    int bits = 0;
    if (!(rho > (T)0) || !(cs2 > (T)0)) bits |= ERR_NONHYP;
    if constexpr (EOS == 1) {
        if (!((T)1 - g.b * rho > (T)0)) bits |= ERR_NONHYP;
    }
    if (!isfinite(rho) || !isfinite(e) || !isfinite(cs2)) bits |= ERR_NONFINITE;
    return bits;
}

// maximum over the copies of reduction field j of the current state
// Population of direction +x (side 0: streams in across the x-low edge) or -x
// (side 1: across the x-high edge) of a pinned ghost, the equilibrium of its
// state W_b at the link speed of this step (Eq. 20): W_b/(2D) +- Q_x(W_b)/(2c),
// returned in the stored energy gauge (energy rho E - eoff rho, flux Q_E - eoff Q_rho).
template <typename T, int EOS>
__device__ inline void pinned_feq(const KParams& p, const Gas<T>& g, int side, T inv2c, T eoff, T* out)
{
    const int D = p.dim, NK = D + 2;
    const double* w = p.pin_w[side];
    const T rho = (T)w[0], mx = (T)w[1], my = D == 2 ? (T)w[2] : (T)0, E = (T)w[NK - 1];
    const T u = mx / rho, v = my / rho;
    const T e = E / rho - (T)0.5 * (u * u + v * v);
    const T P = eos_pressure<T, EOS>(g, rho, e);
    const T sgn = side == 0 ? (T)1 : (T)-1;
    const T inv2d = (T)1 / (T)(2 * D);
    out[0] = rho * inv2d + sgn * mx * inv2c;
    out[1] = mx * inv2d + sgn * (mx * u + P) * inv2c;
    if (D == 2) out[2] = my * inv2d + sgn * (my * u) * inv2c;
    out[NK - 1] = (E - eoff * rho) * inv2d + sgn * ((E + P) * u - eoff * mx) * inv2c;
}

// One step of a wave maximum: v = max(v, v of the lane CTRL names).  Lanes
// whose source lies outside their 16-lane row keep their own value (DPP
// bound_ctrl off: the update is skipped and `old`, the lane's own value, is
// returned), which leaves a maximum unchanged.
template <int CTRL>
__device__ __forceinline__ double dpp_max_step(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = (int)b, hi = (int)(b >> 32);
    const int lo2 = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xf, 0xf, false);
    const int hi2 = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xf, 0xf, false);
    return fmax(v, __longlong_as_double(((long long)hi2 << 32) | (unsigned int)lo2));
}

// Maximum over the 64 lanes of a wave, in every lane: row shifts right by 1,
// 2, 4 and 8 lanes (DPP row_shr, controls 0x111, 0x112, 0x114, 0x118) leave
// the maximum of each 16-lane row in its last lane; the four rows' maxima are
// then read from lanes 15, 31, 47 and 63.  Call with the whole wave active.
__device__ __forceinline__ double wave_max_dpp(double v)
{
    v = dpp_max_step<0x111>(v);
    v = dpp_max_step<0x112>(v);
    v = dpp_max_step<0x114>(v);
    v = dpp_max_step<0x118>(v);
    const long long b = __double_as_longlong(v);
    const int lo = (int)b, hi = (int)(b >> 32);
    double m = 0.0;
#pragma unroll
    for (int r = 15; r < 64; r += 16) {
        const int l = __builtin_amdgcn_readlane(lo, r), h = __builtin_amdgcn_readlane(hi, r);
        m = fmax(m, __longlong_as_double(((long long)h << 32) | (unsigned int)l));
    }
    return m;
}

// The reductions of the current state, fields 0 .. NF-1 (s_max, M_k), each
// the maximum over the copies: lane i reads copy i (at most 64 copies; the
// values are non-negative, 0 is neutral) and a wave maximum folds them, one
// memory latency for all of them.  Call with the whole wave active.
template <int NF>
__device__ __forceinline__ void red_fold_wave(const KStep& s, double (&out)[NF])
{
    const int lane = threadIdx.x & 63;
    const int copies = s.red_copies > 1 ? s.red_copies : 1;
    double v[NF];
#pragma unroll
    for (int j = 0; j < NF; ++j) v[j] = lane < copies ? s.red_in[lane * s.red_stride + j] : 0.0;
#pragma unroll
    for (int j = 0; j < NF; ++j) out[j] = wave_max_dpp(v[j]);
}

// the copy of the new state's reductions this workgroup publishes into
__device__ __forceinline__ double* red_target(const KStep& s)
{
    return s.red_copies > 1 ? s.red_out + (int)(blockIdx.x % (unsigned)s.red_copies) * s.red_stride : s.red_out;
}

// zero every copy of the reductions two steps ahead; lanes of one wave
__device__ __forceinline__ void clear_reductions(const KStep& s, int lane)
{
    if (!s.red_clear) return;
    const int copies = s.red_copies > 1 ? s.red_copies : 1;
    for (int i = lane; i < copies * kRedFields; i += 64) s.red_clear[(i / kRedFields) * s.red_stride + i % kRedFields] = 0.0;
}

// Clock logic of one step (Sec. III.E): retarget c = s_max/CFL (Eq. 37), dt =
// dx/c, final-step landing; smax is the current state's s_max (red_fold_wave).
// Returns false when the step must not run.
__device__ __forceinline__ bool step_clock(const KParams& p, const KStep& s, double smax, double& c_old,
                                           double& c_new, double& t, double& dt, bool& last)
{
    last = false;
    t = 0.0;
    dt = 0.0;
    if (s.frozen) {
        c_old = c_new = p.c_fixed;
        return true;
    }
    // the stop mark and the clock are loaded together (independent reads: one
    // memory latency, not two in a row), then the stop mark decides
    const unsigned long long stop = s.stop_at ? *s.stop_at : ~0ull;
    t = s.clock_in[0];
    c_old = s.clock_in[1];
    if ((unsigned long long)s.n >= stop) return false;
    c_new = c_old;
    if (p.retarget_every > 0 && ((s.n % p.retarget_every) == 0 || smax > c_old)) c_new = smax / p.cfl;
    dt = p.dx / c_new;
    if (s.t_end < HUGE_VAL && t + dt >= s.t_end * (1.0 - 1e-14)) {
        dt = s.t_end - t;
        c_new = p.dx / dt;
        last = true;
    }
    return true;
}

__device__ __forceinline__ void write_clock(const KStep& s, double t, double dt, double c_new, bool last)
{
    if (s.frozen) return;
    s.clock_out[0] = last ? s.t_end : t + dt;
    s.clock_out[1] = c_new;
    if (last) atomicMin(s.stop_at, (unsigned long long)(s.n + 1));
}

// Max of non-negative doubles through their IEEE bit patterns (monotone as
// unsigned integers); NaNs dominate.
__device__ __forceinline__ void atomic_max_nonneg(double* addr, double v)
{
    atomicMax(reinterpret_cast<unsigned long long*>(addr), (unsigned long long)__double_as_longlong(v));
}

template <typename T>
__device__ __forceinline__ T wave_max(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ int wave_or(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
    return v;
}

// OR of the admissibility bits (ERR_NONHYP | ERR_NONFINITE) over a wave, by
// two wave-wide votes.  Call with the whole wave active.
__device__ __forceinline__ int wave_or_errbits(int v)
{
    return (__any(v & ERR_NONHYP) ? ERR_NONHYP : 0) | (__any(v & ERR_NONFINITE) ? ERR_NONFINITE : 0);
}

// Publish the per-lane maxima of one wave: s_max and M_k (nk of them), plus
// the error bits.  The maxima fold by DPP (wave_max_dpp), not by a chain of
// LDS-crossbar shuffles, to keep the end of a launch short.  Call with the
// whole wave active.
__device__ __forceinline__ void wave_publish(const KStep& s, double smax, const double* M, int nk, int errbits)
{
    smax = wave_max_dpp(smax);
    double Mr[4];
    for (int k = 0; k < nk; ++k) Mr[k] = wave_max_dpp(M[k]);
    errbits = wave_or_errbits(errbits);
    if ((threadIdx.x & 63) == 0) {
        double* out = red_target(s);
        atomic_max_nonneg(&out[0], smax);
        for (int k = 0; k < nk; ++k) atomic_max_nonneg(&out[1 + k], Mr[k]);
        if (errbits) {
            atomicOr(s.err, errbits);
            if (s.stop_at) atomicMin(s.stop_at, (unsigned long long)(s.n + 1));
        }
    }
}

// Publish the per-lane maxima of a whole block of NW waves with one set of
// atomics per block (same-address atomics serialise in L2, so a launch issues
// as few as it can).  Call with every thread of the block.
template <int NW>
__device__ __forceinline__ void block_publish(const KStep& s, double smax, const double* M, int nk, int errbits)
{
    __shared__ double sh[NW][5];
    __shared__ int she[NW];
    smax = wave_max_dpp(smax);
    double Mr[4] = {0, 0, 0, 0};
    for (int k = 0; k < nk; ++k) Mr[k] = wave_max_dpp(M[k]);
    errbits = wave_or_errbits(errbits);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[w][0] = smax;
        for (int k = 0; k < 4; ++k) sh[w][1 + k] = Mr[k];
        she[w] = errbits;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < NW; ++i) {
            for (int k = 0; k < 5; ++k) sh[0][k] = fmax(sh[0][k], sh[i][k]);
            she[0] |= she[i];
        }
        double* out = red_target(s);
        atomic_max_nonneg(&out[0], sh[0][0]);
        for (int k = 0; k < nk; ++k) atomic_max_nonneg(&out[1 + k], sh[0][1 + k]);
        if (she[0]) {
            atomicOr(s.err, she[0]);
            if (s.stop_at) atomicMin(s.stop_at, (unsigned long long)(s.n + 1));
        }
    }
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).
// Renumber them so that every XCD receives one contiguous range of logical
// tiles: neighbouring tiles, which share halo cells, then share an L2.
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    const int per = nb / 8, rem = nb % 8;
    const int xcd = b % 8, idx = b / 8;
    return xcd * per + min(xcd, rem) + idx;
}

__device__ __forceinline__ int wrap_index(int i, int n)
{
    i %= n;
    return i < 0 ? i + n : i;
}

}  // namespace vlbm
