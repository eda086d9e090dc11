/*
 * Plain FP64 CPU oracle of the vectorial lattice Boltzmann (VLBM) time step
 * (Hosseini & Karlin, arXiv 2609.10639).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product library never does, and the two share no code, headers or tables.
 *
 * Every quantity is a separate full-grid array and every sub-step is its own
 * sweep over the grid, in the order the paper states them:
 *   moments (Sec. III.A, W = sum_i f_i under Eq. 22)
 *   -> EOS closure (Sec. II.C, Eqs. 13, 15-17)
 *   -> s_max (Sec. III.E, Eq. 36) -> retarget (Eq. 37, final-step landing)
 *   -> reprojection at the new link speed (Eqs. 38-40)
 *   -> flux Q(W) (Sec. II.B, Eq. 10)
 *   -> sensor: flux-divergence jump, normalisation, activity, box filter,
 *      Ducros gate, beta (Sec. III.D, Eqs. 28-35)
 *   -> over-relaxation towards the vector equilibrium (Eqs. 20, 22)
 *   -> exact transport (Eq. 21) -> clock update.
 *
 * Readings of points the paper leaves open (all shared with the GPU path by
 * specification, never by code):
 *   - initial populations are the equilibrium at c0 = s_max(W0)/CFL;
 *   - the landing step shortens dt to t_end - t and therefore retargets the
 *     link speed to c = dx/dt (reprojecting), triggered when
 *     t + dt >= t_end (1 - 1e-14); t is then set to t_end exactly;
 *   - a normaliser M_k == 0 gives s_hat_k = 0;
 *   - outflow = edge-replicated ghost cell: every neighbour index (streaming
 *     source, central differences, box filter) is clamped into the grid;
 *     periodic wraps.  s_max and M_k run over interior cells only;
 *   - pinned x edge (the shock-vortex inflow of Sec. IV.H): the ghost cell
 *     holds a fixed state W_b at equilibrium, so the populations that stream
 *     in across that edge are f^eq_i(W_b) at the current link speed (Eq. 20);
 *     the sensor's stencils treat the edge like an outflow edge;
 *   - with retarget_every = K > 1 a retarget is forced whenever s_max > c;
 *   - the Ducros ratio (Eq. 33) takes dilatation and vorticity in lattice
 *     units, dt times their central differences (dt = dx/c at the step's
 *     link speed), so that its regulariser eps is a dimensionless number and
 *     beta does not depend on the units of time or length, like every other
 *     ratio of the sensor (Eqs. 29-31).
 *
 * Directions: i = 0 (+x), 1 (-x), 2 (+y), 3 (-y).  Components:
 * k = 0 rho, 1..D momentum, D+1 total energy rho*E.
 * Populations: f[(i*NK + k)*ncell + cell], cell = y*nx + x.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_LANDED 1
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ENONHYP (-4)
#define ORC_ENONFINITE (-5)

typedef struct {
    int dim;              /* 1 or 2 */
    long nx, ny;          /* ny == 1 when dim == 1 */
    double dx;            /* uniform spacing, dy == dx */
    int bc[4];            /* xlo, xhi, ylo, yhi: 0 periodic, 1 outflow, 2 pinned (x edges only) */
    double bc_state[2][4];/* conserved state W_b held at the x-low / x-high edge when pinned */
    int eos;              /* 0 ideal gas, 1 van der Waals */
    double gamma, vdw_a, vdw_b, vdw_R;
    double cfl;
    int retarget_every;   /* 0: link speed frozen at c_fixed */
    double c_fixed;
    int sensor;           /* 0 off (beta_const), 1 A, 2 B, 3 auto (A in 1-D, B in 2-D) */
    double beta_const, beta_min, beta_max, c_sensor, eps_theta;
} orc_config;

typedef struct {
    orc_config cfg;
    int D, Q, NK;
    long ncell;
    double *f, *fs;                 /* populations, post-collision populations */
    double *W, *u, *e, *P, *cs2;    /* moments and closure */
    double *flux;                   /* Q_alpha,k: [alpha][k][cell] */
    double *s, *theta, *tmp, *sbar, *thetabar, *beta;
    double c, t;
    long n;
    double pin_Q[2][2][4];          /* Euler flux Q_alpha,k of each pinned edge state */
} orc_state;

/* ------------------------------------------------------------------ EOS */

/* Pressure P(rho, e).  Ideal gas: Eq. 15.  van der Waals: Eqs. 16-17 with
 * T = (e + a rho)/c_v and gamma := 1 + R/c_v (Sec. II.C). */
static double eos_P(const orc_config* g, double rho, double e)
{
    if (g->eos == 0) return (g->gamma - 1.0) * rho * e;
    double cv = g->vdw_R / (g->gamma - 1.0);
    double T = (e + g->vdw_a * rho) / cv;
    return g->vdw_R * rho * T / (1.0 - g->vdw_b * rho) - g->vdw_a * rho * rho;
}

/* Partial derivatives P_rho = (dP/drho)_e and P_e = (dP/de)_rho, written out
 * from the same expressions as eos_P. */
static void eos_partials(const orc_config* g, double rho, double e, double* Prho, double* Pe)
{
    if (g->eos == 0) {
        *Prho = (g->gamma - 1.0) * e;
        *Pe = (g->gamma - 1.0) * rho;
        return;
    }
    double a = g->vdw_a, b = g->vdw_b, R = g->vdw_R;
    double cv = R / (g->gamma - 1.0);
    double T = (e + a * rho) / cv;
    double dTdrho = a / cv;                  /* at fixed e */
    double den = 1.0 - b * rho;
    /* d/drho [R rho T/(1-b rho)] = R T/den + R rho T b/den^2 + R rho dT/drho/den */
    *Prho = R * T / den + R * rho * T * b / (den * den) + R * rho * dTdrho / den - 2.0 * a * rho;
    *Pe = R * rho / (cv * den);
}

/* Frozen isentropic sound speed squared, Eq. 13: c_s^2 = P_rho + P P_e / rho^2. */
static double eos_cs2(const orc_config* g, double rho, double e)
{
    double Prho, Pe;
    eos_partials(g, rho, e, &Prho, &Pe);
    double P = eos_P(g, rho, e);
    return Prho + P * Pe / (rho * rho);
}

/* Admissibility (Eq. 14 and the domain of the vdW closure). */
static int eos_admissible(const orc_config* g, double rho, double e, double cs2)
{
    if (!isfinite(rho) || !isfinite(e) || !isfinite(cs2)) return ORC_ENONFINITE;
    if (!(rho > 0.0)) return ORC_ENONHYP;
    if (g->eos == 1 && !(1.0 - g->vdw_b * rho > 0.0)) return ORC_ENONHYP;
    if (!(cs2 > 0.0)) return ORC_ENONHYP;
    return ORC_OK;
}

/* ------------------------------------------------------------ indexing */

static long nb_index(long i, long d, long n, int bc_lo, int bc_hi)
{
    long j = i + d;
    if (j < 0) return bc_lo == 0 ? j + n : 0;
    if (j >= n) return bc_hi == 0 ? j - n : n - 1;
    return j;
}

/* cell index of the neighbour of (x,y) at offset (dx,dy) */
static long nb_cell(const orc_state* s, long x, long y, long ox, long oy)
{
    const orc_config* g = &s->cfg;
    long xx = nb_index(x, ox, g->nx, g->bc[0], g->bc[1]);
    long yy = (s->D == 2) ? nb_index(y, oy, g->ny, g->bc[2], g->bc[3]) : 0;
    return yy * g->nx + xx;
}

/* unit lattice vector of direction i along axis a */
static int evec(int i, int a)
{
    static const int E[4][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}};
    return E[i][a];
}

#define F(st, i, k, c) ((st)->f[((long)(i) * (st)->NK + (k)) * (st)->ncell + (c)])
#define FS(st, i, k, c) ((st)->fs[((long)(i) * (st)->NK + (k)) * (st)->ncell + (c)])
#define WV(st, k, c) ((st)->W[(long)(k) * (st)->ncell + (c)])
#define UV(st, a, c) ((st)->u[(long)(a) * (st)->ncell + (c)])
#define FLX(st, a, k, c) ((st)->flux[((long)(a) * (st)->NK + (k)) * (st)->ncell + (c)])

/* Euler flux Q_alpha(W_b) (Eq. 10) of a pinned edge state, both axes; the
 * state must be admissible. */
static int pin_flux(const orc_config* g, const double* Wb, double Q[2][4])
{
    const int D = g->dim;
    const double rho = Wb[0];
    if (!(rho > 0.0)) return ORC_ENONHYP;
    double u[2] = {0.0, 0.0}, ke = 0.0;
    for (int a = 0; a < D; ++a) {
        u[a] = Wb[1 + a] / rho;
        ke += 0.5 * u[a] * u[a];
    }
    const double e = Wb[D + 1] / rho - ke;
    const double P = eos_P(g, rho, e);
    int st = eos_admissible(g, rho, e, eos_cs2(g, rho, e));
    if (st != ORC_OK) return st;
    if (!isfinite(P)) return ORC_ENONFINITE;
    for (int a = 0; a < D; ++a) {
        Q[a][0] = rho * u[a];
        for (int b = 0; b < D; ++b) Q[a][1 + b] = rho * u[a] * u[b] + (a == b ? P : 0.0);
        Q[a][D + 1] = (Wb[D + 1] + P) * u[a];
    }
    return ORC_OK;
}

/* ---------------------------------------------------------- lifecycle */

int orc_create(const orc_config* cfg, orc_state** out)
{
    if (!cfg || !out) return ORC_EINVAL;
    if (cfg->dim != 1 && cfg->dim != 2) return ORC_EINVAL;
    if (cfg->nx < 3 || (cfg->dim == 2 && cfg->ny < 3) || (cfg->dim == 1 && cfg->ny != 1)) return ORC_EINVAL;
    if (!(cfg->dx > 0)) return ORC_EINVAL;
    for (int i = 0; i < 4; ++i)
        if (cfg->bc[i] < 0 || cfg->bc[i] > (i < 2 ? 2 : 1)) return ORC_EINVAL;
    double pin_Q[2][2][4] = {{{0}}};
    for (int side = 0; side < 2; ++side) {
        if (cfg->bc[side] != 2) continue;
        if (pin_flux(cfg, cfg->bc_state[side], pin_Q[side]) != ORC_OK) return ORC_EINVAL;
    }
    orc_state* s = (orc_state*)calloc(1, sizeof(orc_state));
    if (!s) return ORC_ENOMEM;
    s->cfg = *cfg;
    memcpy(s->pin_Q, pin_Q, sizeof(pin_Q));
    s->D = cfg->dim;
    s->Q = 2 * cfg->dim;          /* Q = 2^D = 2D for D <= 2 (Sec. III.A) */
    s->NK = cfg->dim + 2;
    s->ncell = cfg->nx * cfg->ny;
    long nf = (long)s->Q * s->NK * s->ncell;
    s->f = (double*)calloc(nf, sizeof(double));
    s->fs = (double*)calloc(nf, sizeof(double));
    s->W = (double*)calloc((long)s->NK * s->ncell, sizeof(double));
    s->u = (double*)calloc((long)s->D * s->ncell, sizeof(double));
    s->e = (double*)calloc(s->ncell, sizeof(double));
    s->P = (double*)calloc(s->ncell, sizeof(double));
    s->cs2 = (double*)calloc(s->ncell, sizeof(double));
    s->flux = (double*)calloc((long)s->D * s->NK * s->ncell, sizeof(double));
    s->s = (double*)calloc(s->ncell, sizeof(double));
    s->theta = (double*)calloc(s->ncell, sizeof(double));
    s->tmp = (double*)calloc(s->ncell, sizeof(double));
    s->sbar = (double*)calloc(s->ncell, sizeof(double));
    s->thetabar = (double*)calloc(s->ncell, sizeof(double));
    s->beta = (double*)calloc(s->ncell, sizeof(double));
    if (!s->f || !s->fs || !s->W || !s->u || !s->e || !s->P || !s->cs2 || !s->flux || !s->s ||
        !s->theta || !s->tmp || !s->sbar || !s->thetabar || !s->beta) {
        free(s);
        return ORC_ENOMEM;
    }
    *out = s;
    return ORC_OK;
}

void orc_destroy(orc_state* s)
{
    if (!s) return;
    free(s->f); free(s->fs); free(s->W); free(s->u); free(s->e); free(s->P); free(s->cs2);
    free(s->flux); free(s->s); free(s->theta); free(s->tmp); free(s->sbar); free(s->thetabar);
    free(s->beta);
    free(s);
}

/* ------------------------------------------------------ sub-step sweeps */

/* W = sum_i f_i (Sec. III.A, below Eq. 22). */
static void sweep_moments(orc_state* s)
{
    for (int k = 0; k < s->NK; ++k) {
#pragma omp parallel for
        for (long c = 0; c < s->ncell; ++c) {
            double acc = 0.0;
            for (int i = 0; i < s->Q; ++i) acc += F(s, i, k, c);
            WV(s, k, c) = acc;
        }
    }
}

/* Primitive variables and EOS closure from W (Eqs. 1, 2, 13, 15-17).
 * Returns the first error status found (ORC_OK if admissible everywhere). */
static int sweep_closure(orc_state* s)
{
    int err = ORC_OK;
#pragma omp parallel for reduction(min : err)
    for (long c = 0; c < s->ncell; ++c) {
        double rho = WV(s, 0, c);
        double ke = 0.0;
        for (int a = 0; a < s->D; ++a) {
            double ua = WV(s, 1 + a, c) / rho;
            UV(s, a, c) = ua;
            ke += 0.5 * ua * ua;
        }
        double e = WV(s, s->D + 1, c) / rho - ke;   /* E = e + |u|^2/2, Eq. 1 */
        s->e[c] = e;
        s->P[c] = eos_P(&s->cfg, rho, e);
        s->cs2[c] = eos_cs2(&s->cfg, rho, e);
        int st = eos_admissible(&s->cfg, rho, e, s->cs2[c]);
        if (!isfinite(s->P[c]) && st == ORC_OK) st = ORC_ENONFINITE;
        if (st < err) err = st;
    }
    return err;
}

/* s_max = max_x max_alpha (|u_alpha| + c_s)  (Eq. 36). */
static double sweep_smax(orc_state* s)
{
    double m = 0.0;
#pragma omp parallel for reduction(max : m)
    for (long c = 0; c < s->ncell; ++c) {
        double cs = sqrt(s->cs2[c]);
        for (int a = 0; a < s->D; ++a) {
            double v = fabs(UV(s, a, c)) + cs;
            if (v > m) m = v;
        }
    }
    return m;
}

/* Euler flux Q_alpha(W) (Eq. 10): (rho u_a, rho u_a u + P e_a, (rho E + P) u_a). */
static void sweep_flux(orc_state* s)
{
    int D = s->D;
#pragma omp parallel for
    for (long c = 0; c < s->ncell; ++c) {
        double rho = WV(s, 0, c), rE = WV(s, D + 1, c), P = s->P[c];
        for (int a = 0; a < D; ++a) {
            double ua = UV(s, a, c);
            FLX(s, a, 0, c) = rho * ua;
            for (int b = 0; b < D; ++b)
                FLX(s, a, 1 + b, c) = rho * ua * UV(s, b, c) + (a == b ? P : 0.0);
            FLX(s, a, D + 1, c) = (rE + P) * ua;
        }
    }
}

/* Reprojection at a new link speed (Eqs. 38-40): hold W, J_alpha and (2-D) K,
 * evaluated with the old speed, and rebuild the populations at the new one. */
static void sweep_reproject(orc_state* s, double c_old, double c_new)
{
    int D = s->D, Q = s->Q, NK = s->NK;
#pragma omp parallel for
    for (long c = 0; c < s->ncell; ++c) {
        for (int k = 0; k < NK; ++k) {
            double W = 0.0, J[2] = {0.0, 0.0}, K = 0.0;
            for (int i = 0; i < Q; ++i) {
                double fi = F(s, i, k, c);
                W += fi;
                for (int a = 0; a < D; ++a) J[a] += c_old * evec(i, a) * fi;      /* Eq. 38 */
                if (D == 2) {
                    double cx = c_old * evec(i, 0), cy = c_old * evec(i, 1);
                    K += (cx * cx - cy * cy) * fi;                             /* Eq. 39 */
                }
            }
            for (int i = 0; i < Q; ++i) {
                double cdotJ = 0.0;
                for (int a = 0; a < D; ++a) cdotJ += c_new * evec(i, a) * J[a];
                double fi = W / Q + cdotJ / (2.0 * c_new * c_new);                  /* Eq. 40 */
                if (D == 2) {
                    double cx = c_new * evec(i, 0), cy = c_new * evec(i, 1);
                    fi += (cx * cx - cy * cy) * K / (4.0 * c_new * c_new * c_new * c_new);
                }
                F(s, i, k, c) = fi;
            }
        }
    }
}

/* Box filter S: separable (1/4, 1/2, 1/4) along x, then along y (Sec. III.D). */
static void box_filter(orc_state* s, const double* in, double* out)
{
    const orc_config* g = &s->cfg;
#pragma omp parallel for
    for (long c = 0; c < s->ncell; ++c) {
        long x = c % g->nx, y = c / g->nx;
        s->tmp[c] = 0.25 * in[nb_cell(s, x, y, -1, 0)] + 0.5 * in[c] + 0.25 * in[nb_cell(s, x, y, 1, 0)];
    }
    if (s->D == 1) {
        memcpy(out, s->tmp, sizeof(double) * s->ncell);
        return;
    }
#pragma omp parallel for
    for (long c = 0; c < s->ncell; ++c) {
        long x = c % g->nx, y = c / g->nx;
        out[c] = 0.25 * s->tmp[nb_cell(s, x, y, 0, -1)] + 0.5 * s->tmp[c] + 0.25 * s->tmp[nb_cell(s, x, y, 0, 1)];
    }
}

static int sensor_mode(const orc_state* s)
{
    if (s->cfg.sensor == 3) return s->D == 1 ? 1 : 2;
    return s->cfg.sensor;
}

/* Relaxation coefficient beta(x) from the current flux field (Sec. III.D):
 * j_k = dx (div Q)_k by central differences (Eqs. 28-29), normalised by the
 * domain-and-direction maximum of |Q_alpha,k| (Eq. 30), combined by an L2
 * average (Eq. 31), box-filtered, gated (2-D, Sensor B) by the Ducros ratio
 * of dilatation and vorticity (Eqs. 32-33), and mapped to beta (Eqs. 34-35). */
static void sweep_beta(orc_state* s)
{
    const orc_config* g = &s->cfg;
    int D = s->D, NK = s->NK;
    int mode = sensor_mode(s);
    if (mode == 0) {
        for (long c = 0; c < s->ncell; ++c) s->beta[c] = g->beta_const;
        return;
    }
    double M[4] = {0, 0, 0, 0};
    for (int k = 0; k < NK; ++k) {
        double m = 0.0;
        for (int a = 0; a < D; ++a)
            for (long c = 0; c < s->ncell; ++c) {
                double v = fabs(FLX(s, a, k, c));
                if (v > m) m = v;
            }
        M[k] = m;
    }
#pragma omp parallel for
    for (long c = 0; c < s->ncell; ++c) {
        long x = c % g->nx, y = c / g->nx;
        double acc = 0.0;
        for (int k = 0; k < NK; ++k) {
            double j = 0.0;
            for (int a = 0; a < D; ++a) {
                long cp = nb_cell(s, x, y, evec(2 * a, 0), evec(2 * a, 1));
                long cm = nb_cell(s, x, y, -evec(2 * a, 0), -evec(2 * a, 1));
                /* dx * (dQ/dx_a) with (Q(x+e)-Q(x-e))/(2 dx): dx cancels */
                j += 0.5 * (FLX(s, a, k, cp) - FLX(s, a, k, cm));
            }
            double sh = (M[k] > 0.0) ? j / M[k] : 0.0;
            acc += sh * sh;
        }
        s->s[c] = sqrt(acc / NK);
    }
    box_filter(s, s->s, s->sbar);

    int gate = (mode == 2 && D == 2);
    if (gate) {
#pragma omp parallel for
        for (long c = 0; c < s->ncell; ++c) {
            long x = c % g->nx, y = c / g->nx;
            long xp = nb_cell(s, x, y, 1, 0), xm = nb_cell(s, x, y, -1, 0);
            long yp = nb_cell(s, x, y, 0, 1), ym = nb_cell(s, x, y, 0, -1);
            /* central differences (Eq. 32) times the time step dt = dx/c:
             * dilatation and vorticity in lattice units, so that eps is a
             * dimensionless number (reading of Eq. 33) */
            double dt = g->dx / s->c;
            double h2 = 2.0 * g->dx;
            double dux_dx = (UV(s, 0, xp) - UV(s, 0, xm)) / h2;
            double duy_dy = (UV(s, 1, yp) - UV(s, 1, ym)) / h2;
            double duy_dx = (UV(s, 1, xp) - UV(s, 1, xm)) / h2;
            double dux_dy = (UV(s, 0, yp) - UV(s, 0, ym)) / h2;
            double dil = dt * (dux_dx + duy_dy);
            double vort = dt * (duy_dx - dux_dy);
            s->theta[c] = dil * dil / (dil * dil + vort * vort + g->eps_theta);
        }
        box_filter(s, s->theta, s->thetabar);
    } else {
        for (long c = 0; c < s->ncell; ++c) s->thetabar[c] = 1.0;
    }
    for (long c = 0; c < s->ncell; ++c) {
        double chi = g->c_sensor * s->sbar[c] * s->thetabar[c];
        if (chi < 0.0) chi = 0.0;
        if (chi > 1.0) chi = 1.0;
        s->beta[c] = g->beta_max - (g->beta_max - g->beta_min) * chi;
    }
}

/* Over-relaxation f* = 2 beta f^eq(W) + (1 - 2 beta) f (Eq. 22) with the vector
 * equilibrium f^eq_i = W/(2D) + c_i . Q(W)/(2 c^2) (Eq. 20). */
static void sweep_collide(orc_state* s)
{
    int D = s->D, Q = s->Q, NK = s->NK;
    double c = s->c;
#pragma omp parallel for
    for (long cell = 0; cell < s->ncell; ++cell) {
        double b = s->beta[cell];
        for (int i = 0; i < Q; ++i)
            for (int k = 0; k < NK; ++k) {
                double cdotQ = 0.0;
                for (int a = 0; a < D; ++a) cdotQ += c * evec(i, a) * FLX(s, a, k, cell);
                double feq = WV(s, k, cell) / (2.0 * D) + cdotQ / (2.0 * c * c);
                FS(s, i, k, cell) = 2.0 * b * feq + (1.0 - 2.0 * b) * F(s, i, k, cell);
            }
    }
}

/* Exact transport f_i(x, t + dt) = f*_i(x - dt c_i) (Eq. 21): a one-cell pull.
 * A source beyond a pinned x edge is that edge's ghost at equilibrium,
 * f^eq_i(W_b) = W_b/(2D) + c_i . Q(W_b)/(2 c^2) (Eq. 20). */
static void sweep_stream(orc_state* s)
{
    const orc_config* g = &s->cfg;
    const int D = s->D;
    for (int i = 0; i < s->Q; ++i)
        for (int k = 0; k < s->NK; ++k) {
#pragma omp parallel for
            for (long c = 0; c < s->ncell; ++c) {
                long x = c % g->nx, y = c / g->nx;
                long xs = x - evec(i, 0);
                int side = xs < 0 ? 0 : (xs >= g->nx ? 1 : -1);
                if (side >= 0 && g->bc[side] == 2) {
                    double cdotQ = 0.0;
                    for (int a = 0; a < D; ++a) cdotQ += s->c * evec(i, a) * s->pin_Q[side][a][k];
                    F(s, i, k, c) = g->bc_state[side][k] / (2.0 * D) + cdotQ / (2.0 * s->c * s->c);
                    continue;
                }
                long src = nb_cell(s, x, y, -evec(i, 0), -evec(i, 1));
                F(s, i, k, c) = FS(s, i, k, src);
            }
        }
}

/* ------------------------------------------------------------- API */

/* f = f^eq(W0; c0) with c0 = s_max(W0)/CFL (or the frozen c_fixed). */
int orc_init(orc_state* s, const double* W0)
{
    memcpy(s->W, W0, sizeof(double) * s->NK * s->ncell);
    int err = sweep_closure(s);
    if (err != ORC_OK) return err;
    double smax = sweep_smax(s);
    s->c = (s->cfg.retarget_every == 0) ? s->cfg.c_fixed : smax / s->cfg.cfl;
    if (!(s->c > 0.0) || !isfinite(s->c)) return ORC_EINVAL;
    sweep_flux(s);
    int D = s->D;
    for (int i = 0; i < s->Q; ++i)
        for (int k = 0; k < s->NK; ++k)
            for (long c = 0; c < s->ncell; ++c) {
                double cdotQ = 0.0;
                for (int a = 0; a < D; ++a) cdotQ += s->c * evec(i, a) * FLX(s, a, k, c);
                F(s, i, k, c) = WV(s, k, c) / (2.0 * D) + cdotQ / (2.0 * s->c * s->c);
            }
    s->t = 0.0;
    s->n = 0;
    return ORC_OK;
}

/* One time step towards t_end (INFINITY for no cap).  Returns ORC_LANDED on
 * the step that lands on t_end, ORC_OK otherwise, or an error status (state
 * left as it was before the step). */
int orc_step(orc_state* s, double t_end)
{
    const orc_config* g = &s->cfg;
    sweep_moments(s);
    int err = sweep_closure(s);
    if (err != ORC_OK) return err;
    double smax = sweep_smax(s);

    double c_new = s->c;
    if (g->retarget_every > 0 && ((s->n % g->retarget_every) == 0 || smax > s->c)) c_new = smax / g->cfl;
    double dt = g->dx / c_new;
    int last = 0;
    if (t_end < INFINITY && s->t + dt >= t_end * (1.0 - 1e-14)) {
        dt = t_end - s->t;
        c_new = g->dx / dt;
        last = 1;
    }
    if (c_new != s->c) {
        sweep_reproject(s, s->c, c_new);
        s->c = c_new;
    }
    sweep_flux(s);
    sweep_beta(s);
    sweep_collide(s);
    sweep_stream(s);
    s->t = last ? t_end : s->t + dt;
    s->n += 1;
    return last ? ORC_LANDED : ORC_OK;
}

int orc_run_to_time(orc_state* s, double t_end, long max_steps, long* steps)
{
    long k = 0;
    int st = ORC_OK;
    while (s->t < t_end && k < max_steps) {
        st = orc_step(s, t_end);
        if (st < 0) break;
        ++k;
        if (st == ORC_LANDED) break;
    }
    if (steps) *steps = k;
    return st < 0 ? st : ORC_OK;
}

/* beta field the next step would use, from the current populations. */
int orc_beta(orc_state* s, double* out)
{
    sweep_moments(s);
    int err = sweep_closure(s);
    if (err != ORC_OK) return err;
    sweep_flux(s);
    sweep_beta(s);
    memcpy(out, s->beta, sizeof(double) * s->ncell);
    return ORC_OK;
}

int orc_get_W(orc_state* s, double* out)
{
    sweep_moments(s);
    memcpy(out, s->W, sizeof(double) * s->NK * s->ncell);
    return ORC_OK;
}

int orc_get_f(const orc_state* s, double* out)
{
    memcpy(out, s->f, sizeof(double) * s->Q * s->NK * s->ncell);
    return ORC_OK;
}

int orc_set_f(orc_state* s, const double* in)
{
    memcpy(s->f, in, sizeof(double) * s->Q * s->NK * s->ncell);
    return ORC_OK;
}

void orc_get_clock(const orc_state* s, double* t, double* c, long* n)
{
    *t = s->t;
    *c = s->c;
    *n = s->n;
}

void orc_set_clock(orc_state* s, double t, double c, long n)
{
    s->t = t;
    s->c = c;
    s->n = n;
}

/* Reproject the stored populations to link speed c_new (Eqs. 38-40). */
void orc_reproject(orc_state* s, double c_new)
{
    sweep_reproject(s, s->c, c_new);
    s->c = c_new;
}

/* Conserved totals sum_x W(x) dx^D with compensated (Neumaier) summation. */
int orc_totals(orc_state* s, double* out)
{
    sweep_moments(s);
    double vol = s->D == 1 ? s->cfg.dx : s->cfg.dx * s->cfg.dx;
    for (int k = 0; k < s->NK; ++k) {
        double sum = 0.0, comp = 0.0;
        for (long c = 0; c < s->ncell; ++c) {
            double v = WV(s, k, c);
            double t = sum + v;
            if (fabs(sum) >= fabs(v)) comp += (sum - t) + v;
            else comp += (v - t) + sum;
            sum = t;
        }
        out[k] = (sum + comp) * vol;
    }
    return ORC_OK;
}

/* Pointwise EOS evaluation for checks: P, c_s^2, P_rho, P_e. */
void orc_eos(const orc_config* g, double rho, double e, double* out4)
{
    double Prho, Pe;
    eos_partials(g, rho, e, &Prho, &Pe);
    out4[0] = eos_P(g, rho, e);
    out4[1] = eos_cs2(g, rho, e);
    out4[2] = Prho;
    out4[3] = Pe;
}

/* Fundamental derivative Gamma = 1 + (rho/c_s)(d c_s/d rho)_s (Eq. 46).
 * Along an isentrope de = (P/rho^2) drho, so
 * (d c_s^2/d rho)_s = (d c_s^2/d rho)_e + (P/rho^2)(d c_s^2/d e)_rho, and
 * Gamma = 1 + rho/(2 c_s^2) (d c_s^2/d rho)_s.  The two partials are taken
 * by central differences of eos_cs2 (a diagnostic, not part of the step). */
double orc_gamma_fundamental(const orc_config* g, double rho, double e)
{
    double hr = 1e-5 * rho, he = 1e-5 * fabs(e) + 1e-8;
    double dr = (eos_cs2(g, rho + hr, e) - eos_cs2(g, rho - hr, e)) / (2.0 * hr);
    double de = (eos_cs2(g, rho, e + he) - eos_cs2(g, rho, e - he)) / (2.0 * he);
    double P = eos_P(g, rho, e);
    double cs2 = eos_cs2(g, rho, e);
    return 1.0 + rho / (2.0 * cs2) * (dr + P / (rho * rho) * de);
}

/* Vector equilibrium of one state for identity checks: W[NK] -> feq[Q][NK]. */
void orc_equilibrium(const orc_config* g, double c, const double* W, double* feq)
{
    int D = g->dim, NK = D + 2, Q = 2 * D;
    double rho = W[0], ke = 0.0, u[2] = {0, 0};
    for (int a = 0; a < D; ++a) {
        u[a] = W[1 + a] / rho;
        ke += 0.5 * u[a] * u[a];
    }
    double e = W[D + 1] / rho - ke;
    double P = eos_P(g, rho, e);
    double flux[2][4];
    for (int a = 0; a < D; ++a) {
        flux[a][0] = rho * u[a];
        for (int b = 0; b < D; ++b) flux[a][1 + b] = rho * u[a] * u[b] + (a == b ? P : 0.0);
        flux[a][D + 1] = (W[D + 1] + P) * u[a];
    }
    for (int i = 0; i < Q; ++i)
        for (int k = 0; k < NK; ++k) {
            double cdotQ = 0.0;
            for (int a = 0; a < D; ++a) cdotQ += c * evec(i, a) * flux[a][k];
            feq[i * NK + k] = W[k] / (2.0 * D) + cdotQ / (2.0 * c * c);
        }
}

/* threads the OpenMP loops of this library use (1 without OpenMP) */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
