// The per-cell arithmetic of a D1Q2 step (arXiv 2609.10639, Sec. III), shared
// by the per-step kernel (vlbm_step1d.hip) and the resident kernel
// (vlbm_resident1d.hip).  Both gather a cell's neighbour values their own way
// (DPP shifts across a wavefront, LDS between the lanes of a workgroup) and
// call these functions on them, so both compute the same bits.  Fused
// multiply-adds occur only where written out: where the compiler would fuse
// depends on the surrounding code, which differs between the two kernels.
// Not part of the public ABI.
#pragma once

#include "vlbm_common.hpp"

namespace vlbm {

// Constants of one step, the same for every cell.
template <typename T>
struct D1Consts {
    Gas<T> g;
    T eoff;       // energy gauge of the stored populations (physical e = e_stored + eoff)
    T r;          // c_old / c_new
    T inv2c;      // 1 / (2 c_new)
    T invM[3];    // 1 / M_k of the current state (0 where M_k = 0)
    bool reproj;  // c_new != c_old
};

// Populations of one cell, plane i*3 + k (direction i = +x, -x; component k):
// reprojection to the new link speed (D = 1 form of Eq. 40, holding W and
// J = c (f+ - f-)) and the flux Q(W) (Eq. 10) of the reprojected state.
template <typename ST, typename T, int EOS>
__device__ __forceinline__ void d1_flux(const D1Consts<T>& c, const ST (&f)[6], T (&fr)[6], T (&q)[3])
{
#pragma clang fp contract(off)
#pragma unroll
    for (int p = 0; p < 6; ++p) fr[p] = (T)f[p];
    if (c.reproj) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const T sm = fr[k] + fr[3 + k], df = fr[k] - fr[3 + k];
            const T a = (T)0.5 * sm, b = (T)0.5 * c.r * df;
            fr[k] = a + b;
            fr[3 + k] = a - b;
        }
    }
    const T rho = fr[0] + fr[3], m = fr[1] + fr[4], E = fr[2] + fr[5];
    const T u = m / rho;
    const T e = E / rho - (T)0.5 * u * u + c.eoff;
    const T Pp = eos_pressure<T, EOS>(c.g, rho, e);
    q[0] = m;
    q[1] = m * u + Pp;
    q[2] = (E + Pp) * u;
}

// Normalised flux-divergence activity s of a cell (Eqs. 28-31) from the flux
// of its left and right neighbours.
template <typename T>
__device__ __forceinline__ T d1_activity(const D1Consts<T>& c, const T (&ql)[3], const T (&qr)[3])
{
#pragma clang fp contract(off)
    T acc = 0, j0 = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        T jk = (T)0.5 * (qr[k] - ql[k]);
        if (k == 0) j0 = jk;
        if (k == 2) jk = fma(c.eoff, j0, jk);   // physical energy flux: Q_E,stored + eoff Q_rho
        const T sh = jk * c.invM[k];
        acc += sh * sh;
    }
    return sqrt(acc / (T)3);
}

// beta of a cell: Sensor A (Eq. 34) on the box-filtered activity, or the
// constant beta with the sensor off.
template <typename T, int SENSOR>
__device__ __forceinline__ T d1_beta(const KParams& P, T sl, T s, T sr)
{
#pragma clang fp contract(off)
    T beta = (T)P.beta_const;
    if constexpr (SENSOR != 0) {
        const T sbar = (T)0.25 * sl + (T)0.5 * s + (T)0.25 * sr;
        T chiv = (T)P.c_sensor * sbar;
        chiv = chiv < (T)0 ? (T)0 : (chiv > (T)1 ? (T)1 : chiv);
        beta = (T)P.beta_max - (T)(P.beta_max - P.beta_min) * chiv;
    }
    return beta;
}

// Over-relaxation towards the vector equilibrium (Eqs. 20, 22):
// g = f + 2 beta (f^eq - f), f^eq_+- = W/2 +- Q/(2c).
template <typename T>
__device__ __forceinline__ void d1_collide(const D1Consts<T>& c, const T (&fr)[6], const T (&q)[3], T beta,
                                           T (&g)[6])
{
#pragma clang fp contract(off)
    const T tb = (T)2 * beta;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const T w2 = (T)0.5 * (fr[k] + fr[3 + k]);
        const T a = q[k] * c.inv2c;
        g[k] = fr[k] + tb * ((w2 + a) - fr[k]);
        g[3 + k] = fr[3 + k] + tb * ((w2 - a) - fr[3 + k]);
    }
}

// Reductions of a cell of the new state (its streamed populations gn): the
// running maxima s_max (Eq. 36) and M_k (Eq. 30), and the admissibility bits.
template <typename T, int EOS>
__device__ __forceinline__ void d1_reduce(const D1Consts<T>& c, const T (&gn)[6], double& red_s, double (&red_M)[3],
                                          int& eb)
{
#pragma clang fp contract(off)
    const T rho = gn[0] + gn[3], m = gn[1] + gn[4], E = gn[2] + gn[5];
    const T u = m / rho;
    const T e = E / rho - (T)0.5 * u * u + c.eoff;
    const T Pp = eos_pressure<T, EOS>(c.g, rho, e);
    const T cs2 = eos_cs2<T, EOS>(c.g, rho, e);
    eb |= eos_check<T, EOS>(c.g, rho, e, cs2);
    red_s = fmax(red_s, (double)(fabs(u) + sqrt(cs2 > (T)0 ? cs2 : (T)0)));
    red_M[0] = fmax(red_M[0], (double)fabs(m));
    red_M[1] = fmax(red_M[1], (double)fabs(m * u + Pp));
    red_M[2] = fmax(red_M[2], (double)fabs((fma(c.eoff, rho, E) + Pp) * u));
}

}  // namespace vlbm
