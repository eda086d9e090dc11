// Closure of one cell and its transpose (vector-Jacobian product), shared by
// the adjoint kernels of the VLBM library.  Not part of the public ABI.
#pragma once

#include "vlbm_common.hpp"

namespace vlbm {

// EOS partial derivatives P_rho (at fixed e) and P_e (at fixed rho) of
// Eqs. 15-17, for the closure adjoint.
template <typename C, int EOS>
__device__ __forceinline__ void eos_partials(const Gas<C>& g, C rho, C e, C& Prho, C& Pe)
{
    if constexpr (EOS == 0) {
        Prho = g.gm1 * e;
        Pe = g.gm1 * rho;
    } else {
        const C temp = (e + g.a * rho) * g.inv_cv;
        const C id = (C)1 / ((C)1 - g.b * rho);
        Prho = g.R * temp * id + g.R * rho * temp * g.b * id * id + g.R * rho * g.a * g.inv_cv * id - (C)2 * g.a * rho;
        Pe = g.R * rho * g.inv_cv * id;
    }
}

// Closure of one cell: velocity, internal energy, pressure, flux Q[a][k].
template <typename C, int EOS, int D>
__device__ __forceinline__ void closure(const Gas<C>& g, const C* W, C* u, C& e, C& P, C (*Q)[4])
{
    const C rho = W[0];
    C ke = 0;
    for (int a = 0; a < D; ++a) {
        u[a] = W[1 + a] / rho;
        ke += u[a] * u[a];
    }
    e = W[D + 1] / rho - (C)0.5 * ke;
    P = eos_pressure<C, EOS>(g, rho, e);
    for (int a = 0; a < D; ++a) {
        Q[a][0] = W[1 + a];
        for (int b = 0; b < D; ++b) Q[a][1 + b] = W[1 + a] * u[b] + (a == b ? P : (C)0);
        Q[a][D + 1] = (W[D + 1] + P) * u[a];
    }
}

// Wbar += (d Q/d W)^T Qbar + (d u/d W)^T ubar at the state W.
template <typename C, int EOS, int D>
__device__ __forceinline__ void closure_adj(const Gas<C>& g, const C* W, C (*Qb)[4], const C* ub_in, C* Wb)
{
    const C rho = W[0], Et = W[D + 1];
    C u[2] = {0, 0}, ke = 0;
    for (int a = 0; a < D; ++a) {
        u[a] = W[1 + a] / rho;
        ke += u[a] * u[a];
    }
    const C e = Et / rho - (C)0.5 * ke;
    const C P = eos_pressure<C, EOS>(g, rho, e);
    C mb[2] = {0, 0}, ub[2] = {ub_in[0], D == 2 ? ub_in[1] : (C)0};
    C Pb = 0, Etb = 0, rhob = 0;
    for (int a = 0; a < D; ++a) {
        mb[a] += Qb[a][0];
        for (int b = 0; b < D; ++b) {
            mb[a] += Qb[a][1 + b] * u[b];
            ub[b] += Qb[a][1 + b] * W[1 + a];
        }
        Pb += Qb[a][1 + a];
        Etb += Qb[a][D + 1] * u[a];
        Pb += Qb[a][D + 1] * u[a];
        ub[a] += Qb[a][D + 1] * (Et + P);
    }
    C Prho, Pe;
    eos_partials<C, EOS>(g, rho, e, Prho, Pe);
    rhob += Pb * Prho;
    const C eb = Pb * Pe;
    Etb += eb / rho;
    rhob -= eb * Et / (rho * rho);
    for (int a = 0; a < D; ++a) ub[a] -= eb * u[a];
    for (int a = 0; a < D; ++a) {
        mb[a] += ub[a] / rho;
        rhob -= ub[a] * u[a] / rho;
    }
    Wb[0] += rhob;
    for (int a = 0; a < D; ++a) Wb[1 + a] += mb[a];
    Wb[D + 1] += Etb;
}

}  // namespace vlbm
