/* Reference finite-volume solver for the compressible Euler equations with a
 * generic EOS: TEST INFRASTRUCTURE ONLY (an independent numerical method used
 * to produce reference solutions where no closed form exists, as the paper
 * does for its 1-D and 2-D benchmarks, Sec. IV.B-IV.F).
 *
 * Method (the paper's description of its reference solver):
 *   * cell averages of W = (rho, rho u[, rho v], rho E) on a uniform grid;
 *   * MUSCL reconstruction of the primitive variables (rho, u[, v], P) with the
 *     minmod limiter, giving left and right states at every face;
 *   * Rusanov (local Lax-Friedrichs) flux with the wave speed
 *     max(|u_n| + c_s) of the two states;
 *   * Heun's two-stage Runge-Kutta (strong-stability-preserving RK2);
 *   * dt = CFL dx / max(|u_a| + c_s), the last step shortened to land on t_end;
 *   * boundaries: outflow (two zero-gradient ghost cells), periodic, or (x
 *     edges) pinned: both ghost cells hold a fixed state W_b (the inflow edge
 *     of the shock-vortex problem, Sec. IV.H);
 *   * 2-D by summing the x and y face fluxes of each stage.
 * EOS (Sec. II.C): ideal P = (gamma-1) rho e, or van der Waals
 * P = R rho T/(1 - b rho) - a rho^2 with e = c_v T - a rho, c_v = R/(gamma-1);
 * sound speed c_s^2 = P_rho + P P_e/rho^2.  This file shares no code with the
 * VLBM oracle or the GPU library.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int dim, nx, ny;
    double dx;
    int bc[4];          /* x-low, x-high, y-low, y-high: 0 periodic, 1 outflow, 2 pinned (x only) */
    double bc_state[2][4]; /* conserved W_b of a pinned x-low / x-high edge */
    int eos;            /* 0 ideal, 1 van der Waals */
    double gamma, a, b, R;
    double cfl;
} ms_config;

#define NG 2

static double pressure(const ms_config* c, double rho, double e)
{
    if (c->eos == 0) return (c->gamma - 1.0) * rho * e;
    const double cv = c->R / (c->gamma - 1.0);
    const double T = (e + c->a * rho) / cv;
    return c->R * rho * T / (1.0 - c->b * rho) - c->a * rho * rho;
}

static double energy_from_p(const ms_config* c, double rho, double P)
{
    if (c->eos == 0) return P / ((c->gamma - 1.0) * rho);
    const double cv = c->R / (c->gamma - 1.0);
    const double T = (P + c->a * rho * rho) * (1.0 - c->b * rho) / (c->R * rho);
    return cv * T - c->a * rho;
}

static double sound2(const ms_config* c, double rho, double e)
{
    double Pr, Pe;
    if (c->eos == 0) {
        Pr = (c->gamma - 1.0) * e;
        Pe = (c->gamma - 1.0) * rho;
    } else {
        const double cv = c->R / (c->gamma - 1.0);
        const double T = (e + c->a * rho) / cv;
        const double g = 1.0 - c->b * rho;
        /* P = R rho T/g - a rho^2 with T = (e + a rho)/c_v */
        Pr = c->R * T / g + c->R * rho * (c->a / cv) / g + c->R * rho * T * c->b / (g * g) - 2.0 * c->a * rho;
        Pe = c->R * rho / (cv * g);
    }
    const double P = pressure(c, rho, e);
    return Pr + P * Pe / (rho * rho);
}

static double minmod(double p, double q)
{
    if (p * q <= 0.0) return 0.0;
    return fabs(p) < fabs(q) ? p : q;
}

/* primitive (rho, u, v, P) -> flux along direction a (0: x, 1: y) and its
 * conserved state, NK = dim + 2 components */
static void phys_flux(const ms_config* c, int a, const double* q, double* W, double* F)
{
    const int D = c->dim;
    const double rho = q[0], P = q[D + 1];
    double ke = 0.0;
    for (int b = 0; b < D; ++b) ke += 0.5 * q[1 + b] * q[1 + b];
    const double E = energy_from_p(c, rho, P) + ke;
    W[0] = rho;
    for (int b = 0; b < D; ++b) W[1 + b] = rho * q[1 + b];
    W[D + 1] = rho * E;
    const double un = q[1 + a];
    F[0] = rho * un;
    for (int b = 0; b < D; ++b) F[1 + b] = rho * q[1 + b] * un + (a == b ? P : 0.0);
    F[D + 1] = (rho * E + P) * un;
}

static double wave_speed(const ms_config* c, int a, const double* q)
{
    const int D = c->dim;
    const double rho = q[0], P = q[D + 1];
    const double e = energy_from_p(c, rho, P);
    const double cs2 = sound2(c, rho, e);
    return fabs(q[1 + a]) + sqrt(cs2 > 0.0 ? cs2 : 0.0);
}

/* ghost-padded layout: component k of cell (i, j) (i in [-NG, nx+NG)) */
typedef struct {
    int px, py;          /* padded sizes */
    double* q;           /* primitive variables, NK planes */
} prim_t;

static int wrap(int i, int n) { return ((i % n) + n) % n; }

static void to_primitives(const ms_config* c, const double* W, prim_t* p)
{
    const int D = c->dim, NK = D + 2, nx = c->nx, ny = c->ny;
    const int gy = D == 2 ? NG : 0;
    const long long pl = (long long)p->px * p->py;
#pragma omp parallel for
    for (int jj = 0; jj < p->py; ++jj)
        for (int ii = 0; ii < p->px; ++ii) {
            int i = ii - NG, j = jj - gy;
            const int side = i < 0 ? 0 : (i >= nx ? 1 : -1);
            if (side >= 0 && c->bc[side] == 2) {
                const double* w = c->bc_state[side];
                double ke = 0.0;
                for (int b = 0; b < D; ++b) ke += 0.5 * w[1 + b] * w[1 + b] / (w[0] * w[0]);
                double* q = p->q + (long long)jj * p->px + ii;
                q[0] = w[0];
                for (int b = 0; b < D; ++b) q[(1 + b) * pl] = w[1 + b] / w[0];
                q[(D + 1) * pl] = pressure(c, w[0], w[D + 1] / w[0] - ke);
                continue;
            }
            if (i < 0) i = c->bc[0] == 0 ? wrap(i, nx) : 0;
            if (i >= nx) i = c->bc[1] == 0 ? wrap(i, nx) : nx - 1;
            if (D == 2) {
                if (j < 0) j = c->bc[2] == 0 ? wrap(j, ny) : 0;
                if (j >= ny) j = c->bc[3] == 0 ? wrap(j, ny) : ny - 1;
            } else {
                j = 0;
            }
            const long long cell = (long long)j * nx + i, n = (long long)nx * ny;
            const double rho = W[cell];
            double ke = 0.0, u[2] = {0.0, 0.0};
            for (int b = 0; b < D; ++b) {
                u[b] = W[(1 + b) * n + cell] / rho;
                ke += 0.5 * u[b] * u[b];
            }
            const double e = W[(D + 1) * n + cell] / rho - ke;
            double* q = p->q + (long long)jj * p->px + ii;
            q[0] = rho;
            for (int b = 0; b < D; ++b) q[(1 + b) * pl] = u[b];
            q[(D + 1) * pl] = pressure(c, rho, e);
        }
    (void)NK;
}

/* dW/dt = -(1/dx) sum_a [F_a(upper face) - F_a(lower face)] into rhs, from the
 * face fluxes (written to fbuf first, so the sums are in a fixed order) */
static void residual(const ms_config* c, const prim_t* p, double* fbuf, double* rhs)
{
    const int D = c->dim, NK = D + 2, nx = c->nx, ny = c->ny;
    const int gy = D == 2 ? NG : 0;
    const long long pl = (long long)p->px * p->py, n = (long long)nx * ny;
    memset(rhs, 0, sizeof(double) * NK * n);
    for (int a = 0; a < D; ++a) {
        const int sx = a == 0 ? 1 : 0, sy = a == 1 ? 1 : 0;
        const int nfx = a == 0 ? nx + 1 : nx, nfy = a == 1 ? ny + 1 : ny;
        const long long nf = (long long)nfx * nfy;
#pragma omp parallel for
        for (long long f = 0; f < nf; ++f) {
            const int fi = (int)(f % nfx), fj = (int)(f / nfx);
            /* face between cells (fi - sx, fj - sy) and (fi, fj) */
            const int iR = fi + NG, jR = fj + gy, iL = iR - sx, jL = jR - sy;
            double qL[4], qR[4];
            for (int k = 0; k < NK; ++k) {
                const double* q = p->q + k * pl;
                const double cL = q[(long long)jL * p->px + iL];
                const double cLm = q[(long long)(jL - sy) * p->px + iL - sx];
                const double cR = q[(long long)jR * p->px + iR];
                const double cRp = q[(long long)(jR + sy) * p->px + iR + sx];
                qL[k] = cL + 0.5 * minmod(cL - cLm, cR - cL);
                qR[k] = cR - 0.5 * minmod(cR - cL, cRp - cR);
            }
            double WL[4], WR[4], FL[4], FR[4];
            phys_flux(c, a, qL, WL, FL);
            phys_flux(c, a, qR, WR, FR);
            const double s = fmax(wave_speed(c, a, qL), wave_speed(c, a, qR));
            for (int k = 0; k < NK; ++k) fbuf[k * nf + f] = 0.5 * (FL[k] + FR[k]) - 0.5 * s * (WR[k] - WL[k]);
        }
#pragma omp parallel for
        for (long long cell = 0; cell < n; ++cell) {
            const int i = (int)(cell % nx), j = (int)(cell / nx);
            const long long lo = (long long)j * nfx + i, hi = lo + (a == 0 ? 1 : nfx);
            for (int k = 0; k < NK; ++k) rhs[k * n + cell] -= (fbuf[k * nf + hi] - fbuf[k * nf + lo]) / c->dx;
        }
    }
}

static double max_speed(const ms_config* c, const prim_t* p)
{
    const int D = c->dim, nx = c->nx, ny = c->ny, gy = D == 2 ? NG : 0;
    const long long pl = (long long)p->px * p->py;
    double smax = 0.0;
#pragma omp parallel for reduction(max : smax)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double q[4];
            for (int k = 0; k < D + 2; ++k) q[k] = p->q[k * pl + (long long)(j + gy) * p->px + i + NG];
            for (int a = 0; a < D; ++a) {
                const double s = wave_speed(c, a, q);
                if (s > smax) smax = s;
            }
        }
    return smax;
}

/* Advance W (FP64, (dim+2, ny, nx)) in place to t_end.  Returns the steps
 * taken, or -1 on a non-positive density or pressure / non-finite value. */
long ms_run(const ms_config* c, double* W, double t_end)
{
    const int D = c->dim, NK = D + 2;
    const long long n = (long long)c->nx * c->ny;
    prim_t p;
    p.px = c->nx + 2 * NG;
    p.py = D == 2 ? c->ny + 2 * NG : 1;
    p.q = (double*)malloc(sizeof(double) * NK * p.px * p.py);
    double* r1 = (double*)malloc(sizeof(double) * NK * n);
    double* r2 = (double*)malloc(sizeof(double) * NK * n);
    double* W1 = (double*)malloc(sizeof(double) * NK * n);
    const long long nfmax = (long long)(c->nx + 1) * (c->ny + 1);
    double* fb = (double*)malloc(sizeof(double) * NK * nfmax);
    double t = 0.0;
    long steps = 0;
    int bad = 0;
    while (t < t_end && !bad) {
        to_primitives(c, W, &p);
        double dt = c->cfl * c->dx / max_speed(c, &p);
        if (t + dt >= t_end * (1.0 - 1e-14)) dt = t_end - t;
        residual(c, &p, fb, r1);
        for (long long i = 0; i < NK * n; ++i) W1[i] = W[i] + dt * r1[i];
        to_primitives(c, W1, &p);
        residual(c, &p, fb, r2);
        for (long long i = 0; i < NK * n; ++i) W[i] = 0.5 * (W[i] + W1[i] + dt * r2[i]);
        for (long long i = 0; i < n; ++i)
            if (!(W[i] > 0.0) || !isfinite(W[(D + 1) * n + i])) bad = 1;
        t = (t + dt >= t_end * (1.0 - 1e-14)) ? t_end : t + dt;
        ++steps;
    }
    free(p.q);
    free(r1);
    free(r2);
    free(W1);
    free(fb);
    return bad ? -1 : steps;
}

/* Thermodynamic state at (rho, P): out = (e, P(rho, e), c_s^2).  Exposed so the
 * tests can pin this file's EOS against the paper's printed worked values. */
void ms_state(const ms_config* c, double rho, double P, double* out)
{
    const double e = energy_from_p(c, rho, P);
    out[0] = e;
    out[1] = pressure(c, rho, e);
    out[2] = sound2(c, rho, e);
}
