// Fused D1Q2 VLBM time step for gfx950 (arXiv 2609.10639, Sec. III).
//
// A 256-thread workgroup processes tiles of consecutive cells (grid-stride over
// the tiles): 256 cells with FP64 arithmetic, 512 with FP32 arithmetic, whose
// cells carry half the bytes, so that the fixed cost of a tile (four barriers,
// the halo) is spread over as many bytes (FP32: +4 %).  At most 1024
// workgroups with FP64 storage, 4096 with FP32 storage and FP64 arithmetic,
// 2048 with FP32 (measured best on MI355X).  It stages the
// cells of a tile plus a 3-cell halo in LDS and runs the step in four
// barrier-separated phases:
//   A  load the 6 populations (SoA planes, coalesced), reproject to the new
//      link speed (Sec. III.E, D = 1 form of Eq. 40), flux Q(W) (Eq. 10);
//   B  normalised flux-divergence activity s (Eqs. 28-31);
//   C  box filter, beta (Sensor A, Eq. 34), over-relaxation (Eqs. 20, 22);
//   D  pull-streaming (Eq. 21), store, and the reductions of the new state.
#include <cstdlib>

#include "vlbm_common.hpp"

namespace vlbm {

constexpr int kBlock1 = 256;   // threads per workgroup
constexpr int kHalo1 = 3;
constexpr int kGrid1 = 1024;   // blocks per launch, FP64 storage (4 per CU); each strides over the tiles
constexpr int kGrid1F = 4096;  // the same with FP32 storage (16 per CU), for tiles of 256 cells

template <typename ST, typename T, int EOS, int SENSOR, int TILE>
__global__ void __launch_bounds__(kBlock1) k_step_d1q2(const KParams P, const KStep S, const ST* __restrict__ fin,
                                                       ST* __restrict__ fout)
{
    // no fused multiply-adds beyond the ones written out: the resident kernel
    // (vlbm_resident1d.hip) runs the same arithmetic and so gives the same bits
#pragma clang fp contract(off)
    constexpr int kSlots1 = TILE + 2 * kHalo1;
    constexpr int NS = (kSlots1 + kBlock1 - 1) / kBlock1;   // slot sets per thread, the last one partial
    static_assert(TILE % kBlock1 == 0, "whole output cells per thread");
    __shared__ T sf[6][kSlots1];   // reprojected populations, plane i*3+k (arithmetic type)
    __shared__ T sq[3][kSlots1];   // flux Q_k
    __shared__ T sa[kSlots1];      // activity s
    __shared__ T sg[6][kSlots1];   // post-collision populations

    double c_old, c_new, t, dt;
    bool last;
    if (!step_clock(P, S, c_old, c_new, t, dt, last)) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) write_clock(S, t, dt, c_new, last);
    if (blockIdx.x == 0 && threadIdx.x < 64 && !S.frozen) clear_reductions(S, threadIdx.x);

    const Gas<T> g = make_gas<T>(P);
    const bool reproj = (c_old != c_new);
    const T r = (T)(c_old / c_new);
    const T inv2c = (T)(0.5 / c_new);
    const T eoff = (T)P.e_off;   // energy gauge of the stored populations (physical e = e_stored + eoff)
    T invM[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double M = red_fold(S, 1 + k);
        invM[k] = M > 0.0 ? (T)(1.0 / M) : (T)0;
    }
    const int nx = P.nx;
    const long long plane = P.plane;
    // outflow and pinned edges clamp every neighbour index; a pinned edge then
    // replaces the population streaming in across it by its ghost's equilibrium
    const bool cl = P.bc[0] != 0, ch = P.bc[1] != 0;
    const bool pl = P.bc[0] == 2, ph = P.bc[1] == 2;
    const int ntiles = (nx + TILE - 1) / TILE;

    // reductions of the new state over every tile this block visits
    double red_s = 0.0, red_M[3] = {0.0, 0.0, 0.0};
    int errbits = 0;

    // slot s of tile t holds cell X = t TILE - 3 + s; neighbours follow the boundary rule
    auto cell_of = [&](int X) {
        if (X < 0) return cl ? 0 : wrap_index(X, nx);
        if (X >= nx) return ch ? nx - 1 : wrap_index(X, nx);
        return X;
    };
    // Each thread owns slots threadIdx.x + h kBlock1 (h < NS; the last set only
    // for the first kSlots1 - (NS - 1) kBlock1 threads).  With FP32 storage the
    // populations of its slots of the next tile are loaded while the current
    // tile is processed (measured +8 %; with FP64 storage the extra registers
    // cost more than they hide, -4 %).  The loads are unconditional (past the
    // last tile the last tile is re-read, in bounds; a thread without a slot in
    // the last set re-reads its first), so they never merge through copies that
    // wait at once.
    constexpr bool kAhead = sizeof(ST) == 4;
    const bool two = threadIdx.x + (NS - 1) * kBlock1 < kSlots1;   // owns a slot of the last set
    ST pre[NS][6];
    auto load_slots = [&](int t) {
#pragma unroll
        for (int h = 0; h < NS; ++h) {
            const int sl = threadIdx.x + h * kBlock1;
            const bool full = h < NS - 1;
            if (full || kAhead || two) {
                const int c = cell_of(t * TILE - kHalo1 + (full || two ? sl : (int)threadIdx.x));
#pragma unroll
                for (int j = 0; j < 6; ++j) pre[h][j] = fin[j * plane + c];
            }
        }
    };
    if (kAhead && (int)blockIdx.x < ntiles) load_slots(blockIdx.x);

    // grid-stride over tiles of TILE cells: few blocks, one set of atomics each
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int x0 = tile * TILE;
        auto left_of = [&](int s) { return (cl && x0 - kHalo1 + s == 0) ? s : s - 1; };
        auto right_of = [&](int s) { return (ch && x0 - kHalo1 + s == nx - 1) ? s : s + 1; };
        if (!kAhead) load_slots(tile);
        ST cur[NS][6];
#pragma unroll
        for (int h = 0; h < NS; ++h)
#pragma unroll
            for (int j = 0; j < 6; ++j) cur[h][j] = pre[h][j];
        if (kAhead) load_slots(min(tile + (int)gridDim.x, ntiles - 1));

        // ---- A
#pragma unroll
        for (int h = 0; h < NS; ++h) {
            if (h == NS - 1 && !two) break;
            const int s = threadIdx.x + h * kBlock1;
            T f[6];
#pragma unroll
            for (int j = 0; j < 6; ++j) f[j] = (T)cur[h][j];
            if (reproj) {
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const T sm = f[k] + f[3 + k], df = f[k] - f[3 + k];
                    const T a = (T)0.5 * sm, b = (T)0.5 * r * df;
                    f[k] = a + b;
                    f[3 + k] = a - b;
                }
            }
#pragma unroll
            for (int j = 0; j < 6; ++j) sf[j][s] = f[j];
            const T rho = f[0] + f[3], m = f[1] + f[4], E = f[2] + f[5];
            const T u = m / rho;
            const T e = E / rho - (T)0.5 * u * u + eoff;
            const T Pp = eos_pressure<T, EOS>(g, rho, e);
            sq[0][s] = m;
            sq[1][s] = m * u + Pp;
            sq[2][s] = (E + Pp) * u;
        }
        __syncthreads();
        // ---- B
        if constexpr (SENSOR != 0) {
            for (int s = threadIdx.x + 1; s < kSlots1 - 1; s += kBlock1) {
                const int sl = left_of(s), sr = right_of(s);
                T acc = 0, j0 = 0;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    T jk = (T)0.5 * (sq[k][sr] - sq[k][sl]);
                    if (k == 0) j0 = jk;
                    if (k == 2) jk = fma(eoff, j0, jk);   // physical energy flux: Q_E,stored + eoff Q_rho
                    const T sh = jk * invM[k];
                    acc += sh * sh;
                }
                sa[s] = sqrt(acc / (T)3);
            }
            __syncthreads();
        }
        // ---- C
        for (int s = threadIdx.x + 2; s < kSlots1 - 2; s += kBlock1) {
            T beta = (T)P.beta_const;
            if constexpr (SENSOR != 0) {
                const T sbar = (T)0.25 * sa[left_of(s)] + (T)0.5 * sa[s] + (T)0.25 * sa[right_of(s)];
                T chiv = (T)P.c_sensor * sbar;
                chiv = chiv < (T)0 ? (T)0 : (chiv > (T)1 ? (T)1 : chiv);
                beta = (T)P.beta_max - (T)(P.beta_max - P.beta_min) * chiv;
            }
            const int X = x0 - kHalo1 + s;
            if (S.probe) {
                if (s >= kHalo1 && s < kHalo1 + TILE && X < nx) S.beta_out[X] = (double)beta;
                continue;
            }
            const T tb = (T)2 * beta;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const T w2 = (T)0.5 * (sf[k][s] + sf[3 + k][s]);
                const T a = sq[k][s] * inv2c;
                sg[k][s] = sf[k][s] + tb * ((w2 + a) - sf[k][s]);
                sg[3 + k][s] = sf[3 + k][s] + tb * ((w2 - a) - sf[3 + k][s]);
            }
        }
        __syncthreads();
        // ---- D
#pragma unroll
        for (int h = 0; h < TILE / kBlock1; ++h) {
            if (S.probe) break;
            const int s = kHalo1 + threadIdx.x + h * kBlock1;
            const int X = x0 + threadIdx.x + h * kBlock1;
            if (X < nx) {
                const int sl = left_of(s), sr = right_of(s);
                T gn[6];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    gn[k] = sg[k][sl];
                    gn[3 + k] = sg[3 + k][sr];
                }
                if ((pl && X == 0) || (ph && X == nx - 1)) {   // nx >= 4: distinct cells
                    T pe[3];
                    const int side = X == 0 ? 0 : 1;
                    pinned_feq<T, EOS>(P, g, side, inv2c, eoff, pe);
#pragma unroll
                    for (int k = 0; k < 3; ++k) gn[side * 3 + k] = pe[k];
                }
#pragma unroll
                for (int j = 0; j < 6; ++j) fout[j * plane + X] = (ST)gn[j];
                const T rho = gn[0] + gn[3], m = gn[1] + gn[4], E = gn[2] + gn[5];
                const T u = m / rho;
                const T e = E / rho - (T)0.5 * u * u + eoff;
                const T Pp = eos_pressure<T, EOS>(g, rho, e);
                const T cs2 = eos_cs2<T, EOS>(g, rho, e);
                errbits |= eos_check<T, EOS>(g, rho, e, cs2);
                red_s = fmax(red_s, (double)(fabs(u) + sqrt(cs2 > (T)0 ? cs2 : (T)0)));
                red_M[0] = fmax(red_M[0], (double)fabs(m));
                red_M[1] = fmax(red_M[1], (double)fabs(m * u + Pp));
                red_M[2] = fmax(red_M[2], (double)fabs((fma(eoff, rho, E) + Pp) * u));
            }
        }
        __syncthreads();   // the next tile overwrites sf, sq, sa and sg
    }
    if (!S.probe) block_publish<kBlock1 / 64>(S, red_s, red_M, 3, errbits);
}

template <typename ST, typename T, int TILE>
static hipError_t launch_t(const KParams& p, const KStep& s, const void* fin, void* fout, hipStream_t st)
{
    const int ntiles = (p.nx + TILE - 1) / TILE;
    int gmax = sizeof(ST) == 4 ? kGrid1F * 256 / TILE : kGrid1;   // FP32 tiles of 512: 2048 blocks
    if (const char* env = getenv("VLBM_D1_GRID")) {   // tuning override
        const int v = atoi(env);
        if (v >= 64 && v <= 65536) gmax = v;
    }
    const dim3 grid(ntiles < gmax ? ntiles : gmax), block(kBlock1);
    const ST* in = (const ST*)fin;
    ST* out = (ST*)fout;
#define VLBM_CASE(E, SN)                                                                            \
    if (p.eos == E && p.sensor == SN) {                                                             \
        hipLaunchKernelGGL((k_step_d1q2<ST, T, E, SN, TILE>), grid, block, 0, st, p, s, in, out); \
        return hipGetLastError();                                                                   \
    }
    VLBM_CASE(0, 0) VLBM_CASE(0, 1) VLBM_CASE(1, 0) VLBM_CASE(1, 1)
#undef VLBM_CASE
    return hipErrorInvalidValue;
}

// cells per tile: 512 with FP32 arithmetic, 256 with FP64 (VLBM_D1_TILE overrides, for tuning)
template <typename ST, typename T>
static hipError_t launch_tiled(const KParams& p, const KStep& s, const void* fin, void* fout, hipStream_t st)
{
    int tile = sizeof(T) == 4 ? 512 : 256;
    if (const char* env = getenv("VLBM_D1_TILE")) {
        const int v = atoi(env);
        if (v == 256 || v == 512) tile = v;
    }
    return tile == 512 ? launch_t<ST, T, 512>(p, s, fin, fout, st) : launch_t<ST, T, 256>(p, s, fin, fout, st);
}

hipError_t launch_step_d1q2(const KParams& p, const KStep& s, int prec, const void* fin, void* fout, hipStream_t st)
{
    switch (prec) {
    case PREC_FP64: return launch_tiled<double, double>(p, s, fin, fout, st);
    case PREC_FP32: return launch_tiled<float, float>(p, s, fin, fout, st);
    case PREC_FP32_MIXED: return launch_tiled<float, double>(p, s, fin, fout, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace vlbm
