// Fused D1Q2 VLBM time step for gfx950 (arXiv 2609.10639, Sec. III).
//
// A wavefront updates a tile of consecutive cells.  Each lane holds V cells:
// on large grids V = 16 bytes over the storage size (4 with FP32 storage, 2
// with FP64), so that every population plane is read and written with one
// 16-byte access per lane and the wavefront's loads of a plane are one
// contiguous 1 KB stream; smaller grids take fewer cells a lane (launch_prec).
// The stencil chain of a step (flux, activity, box filter, streaming) reaches
// 3 cells to each side; HL = ceil(3/V) halo lanes at each end of the
// wavefront load those cells and repeat their arithmetic, and the other
// 64 - 2 HL lanes own their cells.  Neighbour values move between lanes by
// DPP wavefront shifts: no LDS and no barrier.  Workgroups of 4 wavefronts
// stride over the tiles with the next tile's loads in flight.
//
// Per cell, in the order the oracle follows: reprojection to the new link
// speed and the flux (Eq. 40, Eq. 10), the normalised activity (Eqs. 28-31),
// beta (Sensor A, Eq. 34, box-filtered), over-relaxation (Eqs. 20, 22),
// pull-streaming (Eq. 21) with the edge rules, and the reductions of the new
// state (s_max, M_k) for the next step.  The per-cell arithmetic is shared
// with the resident kernel (vlbm_d1q2_cell.hpp), so both give the same bits.
#include <algorithm>
#include <cstdint>
#include <cstdlib>

#include "vlbm_d1q2_cell.hpp"
#include "vlbm_planes.hpp"

namespace vlbm {

constexpr int kBlock1 = 256;   // threads per workgroup: 4 wavefronts, each on its own tiles
// Most workgroups per launch, grid-striding over the tiles, every wavefront
// taking the same number of tiles (measured on MI355X at 2^26 cells, Sensor A,
// in fractions of 8 TB/s):
//   FP64 storage, 65536: 68 % (64 % at 16384, 66 % at 32768, 67 % at 131072);
//   FP32 storage, 32768: 62 % (59 % at 8192, 60 % at 16384, 49 % at 131072,
//     where each wavefront takes a single tile and nothing is prefetched);
//   FP32 storage with FP64 arithmetic, 2048: 56 % (56 % at 4096, 55 % at 8192,
//     49 % at 32768).
template <typename ST, typename T>
constexpr long long grid_cap()
{
    return sizeof(ST) == 8 ? 65536 : (sizeof(T) == 8 ? 2048 : 32768);
}

// V cells per lane, read and written as one V-element vector access per plane.
template <typename ST, typename T, int EOS, int SENSOR, int V>
__global__ void __launch_bounds__(kBlock1) k_step_d1q2(const KParams P, const KStep S, const ST* __restrict__ fin,
                                                       ST* __restrict__ fout)
{
    // no fused multiply-adds beyond the ones written out: the resident kernel
    // (vlbm_resident1d.hip) runs the same arithmetic and so gives the same bits
#pragma clang fp contract(off)
    constexpr int HL = (3 + V - 1) / V;        // halo lanes at each end
    constexpr int WO = (64 - 2 * HL) * V;      // cells a tile owns
    typedef ST VT __attribute__((ext_vector_type(V)));

    const int nx = P.nx;
    const long long plane = P.plane;
    // outflow and pinned edges clamp every neighbour to the edge cell itself; a
    // pinned edge then replaces the population streaming in across it by its
    // ghost's equilibrium; periodic edges wrap
    const bool cl = P.bc[0] != 0, ch = P.bc[1] != 0;
    const bool pl = P.bc[0] == 2, ph = P.bc[1] == 2;
    const int lane = threadIdx.x & 63;
    const bool own_lane = lane >= HL && lane < 64 - HL;
    const int ntiles = (nx + WO - 1) / WO;
    const int nwaves = (int)gridDim.x * (kBlock1 / 64);
    // FP32 storage: every XCD takes one contiguous range of workgroups, so the
    // lines that neighbouring tiles' halo lanes share are fetched once (reads
    // 1.065 -> 1.001 of the algorithmic bytes at 2^26 cells, 61.7 -> 62.4 % of
    // 8 TB/s).  FP64 storage keeps dispatch order: the same renumbering cut
    // its reads to 1.000 but measured 66 % against 68 %.
    const int wg = sizeof(ST) == 4 ? xcd_tile((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
    const int wave = wg * (kBlock1 / 64) + (int)(threadIdx.x >> 6);

    double red_s = 0.0, red_M[3] = {0.0, 0.0, 0.0};
    int errbits = 0;

    // The lane's V cells of tile t, plane by plane: one 16-byte load a plane
    // where they lie inside the grid, else cell by cell through the edge rule
    // (clamped or wrapped).  Past the last tile the last tile is re-read, in
    // bounds, so that the prefetch is unconditional.
    auto load_tile = [&](int tile, ST (&d)[V][6]) {
        const int X0 = tile * WO - HL * V + lane * V;
        if (X0 >= 0 && X0 + V <= nx) {
#pragma unroll
            for (int p = 0; p < 6; ++p) {
                const VT v = *reinterpret_cast<const VT*>(fin + p * plane + X0);
#pragma unroll
                for (int j = 0; j < V; ++j) d[j][p] = v[j];
            }
        } else {
#pragma unroll
            for (int j = 0; j < V; ++j) {
                const int X = X0 + j;
                const int c = X < 0 ? (cl ? 0 : wrap_index(X, nx)) : (X >= nx ? (ch ? nx - 1 : wrap_index(X, nx)) : X);
#pragma unroll
                for (int p = 0; p < 6; ++p) d[j][p] = fin[p * plane + c];
            }
        }
    };

    // the next tile's loads are in flight while a tile is processed (two
    // tiles ahead measured no faster: the registers cost a wavefront per SIMD)
    ST nxt[V][6];
    if (wave < ntiles) load_tile(wave, nxt);

    // the control reads (reductions, clock) after the first tile's loads:
    // none depends on another, so their memory latencies overlap
    double R[4];   // s_max, M_k of the current state
    red_fold_wave<4>(S, R);
    double c_old, c_new, t, dt;
    bool last;
    if (!step_clock(P, S, R[0], c_old, c_new, t, dt, last)) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) write_clock(S, t, dt, c_new, last);
    if (blockIdx.x == 0 && threadIdx.x < 64 && !S.frozen) clear_reductions(S, threadIdx.x);

    D1Consts<T> cs;
    cs.g = make_gas<T>(P);
    cs.eoff = (T)P.e_off;
    cs.reproj = c_old != c_new;
    cs.r = (T)(c_old / c_new);
    cs.inv2c = (T)(0.5 / c_new);
#pragma unroll
    for (int k = 0; k < 3; ++k) cs.invM[k] = R[1 + k] > 0.0 ? (T)(1.0 / R[1 + k]) : (T)0;
    for (int tile = wave; tile < ntiles; tile += nwaves) {
        ST cur[V][6];
#pragma unroll
        for (int j = 0; j < V; ++j)
#pragma unroll
            for (int p = 0; p < 6; ++p) cur[j][p] = nxt[j][p];
        load_tile(min(tile + nwaves, ntiles - 1), nxt);
        const int X0 = tile * WO - HL * V + lane * V;
        // a clamped grid edge: the neighbour of the edge cell is the cell itself
        bool selfL[V], selfR[V];
#pragma unroll
        for (int j = 0; j < V; ++j) {
            selfL[j] = cl && X0 + j == 0;
            selfR[j] = ch && X0 + j == nx - 1;
        }

        // ---- reprojection and flux
        T fr[V][6], q[V][3];
#pragma unroll
        for (int j = 0; j < V; ++j) d1_flux<ST, T, EOS>(cs, cur[j], fr[j], q[j]);

        // ---- activity, beta
        T beta[V];
        if constexpr (SENSOR != 0) {
            T qL[3], qR[3];   // flux of the left lane's last cell and of the right lane's first
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                qL[k] = dpp_move<kDppWaveShr1>(q[V - 1][k]);
                qR[k] = dpp_move<kDppWaveShl1>(q[0][k]);
            }
            T sv[V];
#pragma unroll
            for (int j = 0; j < V; ++j) {
                T left[3], right[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    left[k] = selfL[j] ? q[j][k] : (j > 0 ? q[j > 0 ? j - 1 : 0][k] : qL[k]);
                    right[k] = selfR[j] ? q[j][k] : (j < V - 1 ? q[j < V - 1 ? j + 1 : j][k] : qR[k]);
                }
                sv[j] = d1_activity(cs, left, right);
            }
            const T sL = dpp_move<kDppWaveShr1>(sv[V - 1]), sR = dpp_move<kDppWaveShl1>(sv[0]);
#pragma unroll
            for (int j = 0; j < V; ++j) {
                const T left = selfL[j] ? sv[j] : (j > 0 ? sv[j > 0 ? j - 1 : 0] : sL);
                const T right = selfR[j] ? sv[j] : (j < V - 1 ? sv[j < V - 1 ? j + 1 : j] : sR);
                beta[j] = d1_beta<T, SENSOR>(P, left, sv[j], right);
            }
        } else {
#pragma unroll
            for (int j = 0; j < V; ++j) beta[j] = d1_beta<T, SENSOR>(P, (T)0, (T)0, (T)0);
        }
        if (S.probe) {   // beta of the current state only
            if (own_lane)
#pragma unroll
                for (int j = 0; j < V; ++j)
                    if (X0 + j >= 0 && X0 + j < nx) S.beta_out[X0 + j] = (double)beta[j];
            continue;
        }

        // ---- over-relaxation
        T gp[V][6];
#pragma unroll
        for (int j = 0; j < V; ++j) d1_collide(cs, fr[j], q[j], beta[j], gp[j]);

        // ---- pull-streaming, edge rules, reductions of the new state, stores
        T gL[3], gR[3];   // +x populations leaving the left lane's last cell, -x leaving the right lane's first
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            gL[k] = dpp_move<kDppWaveShr1>(gp[V - 1][k]);
            gR[k] = dpp_move<kDppWaveShl1>(gp[0][3 + k]);
        }
        ST out[V][6];
#pragma unroll
        for (int j = 0; j < V; ++j) {
            const int X = X0 + j;
            T gn[6];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                gn[k] = selfL[j] ? gp[j][k] : (j > 0 ? gp[j > 0 ? j - 1 : 0][k] : gL[k]);
                gn[3 + k] = selfR[j] ? gp[j][3 + k] : (j < V - 1 ? gp[j < V - 1 ? j + 1 : j][3 + k] : gR[k]);
            }
            if ((pl && X == 0) || (ph && X == nx - 1)) {   // nx >= 4: distinct cells
                T pe[3];
                const int side = X == 0 ? 0 : 1;
                pinned_feq<T, EOS>(P, cs.g, side, cs.inv2c, cs.eoff, pe);
#pragma unroll
                for (int k = 0; k < 3; ++k) gn[side * 3 + k] = pe[k];
            }
#pragma unroll
            for (int p = 0; p < 6; ++p) out[j][p] = (ST)gn[p];
            if (own_lane && X >= 0 && X < nx) d1_reduce<T, EOS>(cs, gn, red_s, red_M, errbits);
        }
        if (own_lane) {
            if (X0 + V <= nx) {
#pragma unroll
                for (int p = 0; p < 6; ++p) {
                    VT v;
#pragma unroll
                    for (int j = 0; j < V; ++j) v[j] = out[j][p];
                    // FP64 storage: non-temporal stores, 68 % against 66 % of
                    // 8 TB/s; with FP32 storage they measured 1-2 points slower
                    if constexpr (sizeof(ST) == 8)
                        __builtin_nontemporal_store(v, reinterpret_cast<VT*>(fout + p * plane + X0));
                    else
                        *reinterpret_cast<VT*>(fout + p * plane + X0) = v;
                }
            } else {
#pragma unroll
                for (int j = 0; j < V; ++j)
                    if (X0 + j < nx)
#pragma unroll
                        for (int p = 0; p < 6; ++p) fout[p * plane + X0 + j] = out[j][p];
            }
        }
    }
    if (!S.probe) block_publish<kBlock1 / 64>(S, red_s, red_M, 3, errbits);
}

template <typename ST, typename T, int V>
static hipError_t launch_v(const KParams& p, const KStep& s, const void* fin, void* fout, hipStream_t st)
{
    constexpr int HL = (3 + V - 1) / V, WO = (64 - 2 * HL) * V;
    const long long ntiles = (p.nx + WO - 1) / WO;
    long long gmax = grid_cap<ST, T>();
    if (const char* env = getenv("VLBM_D1_GRID")) {   // tuning override
        const int v = atoi(env);
        if (v >= 64 && v <= (1 << 20)) gmax = v;
    }
    // tiles a wavefront takes, then as many workgroups as give every wavefront
    // that many: no wavefront is left with one tile more than the others
    const long long need = (ntiles + kBlock1 / 64 - 1) / (kBlock1 / 64);
    const long long per = (need + gmax - 1) / gmax;
    const long long blocks = (need + per - 1) / per;
    const dim3 grid((unsigned)blocks), block(kBlock1);
    const ST* in = (const ST*)fin;
    ST* out = (ST*)fout;
#define VLBM_CASE(E, SN)                                                                       \
    if (p.eos == E && p.sensor == SN) {                                                        \
        hipLaunchKernelGGL((k_step_d1q2<ST, T, E, SN, V>), grid, block, 0, st, p, s, in, out); \
        return hipGetLastError();                                                              \
    }
    VLBM_CASE(0, 0) VLBM_CASE(0, 1) VLBM_CASE(1, 0) VLBM_CASE(1, 1)
#undef VLBM_CASE
    return hipErrorInvalidValue;
}

// Cells per lane (measured on MI355X, one launch per step; every width gives
// the same bits):
//   1 cell on grids of at most 2048 one-cell tiles (58 cells each, 1.2e5
//     cells): the chain of arithmetic each lane runs in series is shortest.
//     8192 cells: FP64 7.52 -> 6.37 us a step, FP32 7.00 -> 6.20, FP32
//     storage with FP64 arithmetic 7.39 -> 6.01; 65536 cells 4-7 % faster;
//     262144 cells 2-8 % slower.
//   Otherwise 16 bytes of each plane (2 cells with FP64 storage, 4 with FP32),
//   except with FP32 storage on grids that need less than the chip's width
//   of 4-cell tiles (248 cells each), where 2 cells halve each lane's work:
//     FP32 arithmetic below 1024 such tiles (2.5e5 cells; at 2^19 cells 4
//       cells a lane are 10 % faster);
//     FP64 arithmetic, whose 4-cell form holds 200-235 VGPRs, below 65536
//       such tiles (1.6e7 cells: 2^22 cells 59.0 -> 54.5 us; the two are even
//       at 2^24, and at 2^25 4 cells a lane are 5 % faster).
// The environment variable VLBM_D1_LANE_CELLS (1, 2, or 4 with FP32 storage)
// fixes the choice.
template <typename ST, typename T>
static int lane_cells(long long nx)
{
    int v;
    if (nx <= 2048LL * 58) v = 1;
    else if (sizeof(ST) == 8) v = 2;
    else v = (nx + 247) / 248 < (sizeof(T) == 8 ? 65536 : 1024) ? 2 : 4;
    if (const char* env = getenv("VLBM_D1_LANE_CELLS")) {
        const int e = atoi(env);
        if (e == 1 || e == 2 || (e == 4 && sizeof(ST) == 4)) v = e;
    }
    return v;
}

template <typename ST, typename T>
static hipError_t launch_prec(const KParams& p, const KStep& s, const void* fin, void* fout, hipStream_t st)
{
    switch (lane_cells<ST, T>(p.nx)) {
    case 1: return launch_v<ST, T, 1>(p, s, fin, fout, st);
    case 2: return launch_v<ST, T, 2>(p, s, fin, fout, st);
    default:
        if constexpr (sizeof(ST) == 4) return launch_v<ST, T, 4>(p, s, fin, fout, st);
        return hipErrorInvalidValue;
    }
}

hipError_t launch_step_d1q2(const KParams& p, const KStep& s, int prec, const void* fin, void* fout, hipStream_t st)
{
    // the 16-byte accesses need 16-byte aligned planes (a plane holds a
    // multiple of 64 elements): the library's buffers are, and populations
    // handed to the raw entry points must be
    if ((reinterpret_cast<uintptr_t>(fin) | reinterpret_cast<uintptr_t>(fout)) & 15) return hipErrorInvalidValue;
    switch (prec) {
    case PREC_FP64: return launch_prec<double, double>(p, s, fin, fout, st);
    case PREC_FP32: return launch_prec<float, float>(p, s, fin, fout, st);
    case PREC_FP32_MIXED: return launch_prec<float, double>(p, s, fin, fout, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace vlbm
