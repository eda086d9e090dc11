// Host runtime of the VLBM library: configuration checks, device buffers,
// the clock/reduction ring and the batched step loop behind the C ABI of
// include/vlbm.h.
//
// Device state
//   f[2]       two population buffers; state n lives in f[n & 1]
//   ring       3 slots of kSlot doubles: [t, c] and kRedCopies copies of the
//              reductions [s_max, M_0..M_{D+1}]; state n has its clock and
//              reductions in slot n % 3
//   stop_at    launches with index >= stop_at return immediately (landing or
//              an inadmissible state), so a batch never overruns
//   err        admissibility bits of the state stop_at
// The host launches steps in batches without synchronising, then reads the
// control block back once per batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <string>

#include "../../include/vlbm.h"
#include "vlbm_aux.hpp"

using namespace vlbm;

static_assert(kRedCopies * kRedStride == VLBM_NORMS_LEN, "norms arrays hold the reduction copies");

// pinned host mirror: the three ring slots, then scratch for totals and checkpoints
constexpr int kHostAux = 3 * kSlot;

struct vlbm_ctx {
    vlbm_config cfg;
    KParams kp;
    int D, Q, NK, nplanes;
    int prec;      // PREC_*
    bool fp32;     // populations stored as FP32
    size_t esize;
    long long ncell, plane;
    void* f[2] = {nullptr, nullptr};
    double* ring = nullptr;
    unsigned long long* stop_at = nullptr;
    int* err = nullptr;
    double* scratchW = nullptr;    // (NK, ncell) FP64
    double* scratchB = nullptr;    // (ncell) FP64
    double* partials = nullptr;    // totals partials
    double* norms_scratch = nullptr;
    double* host = nullptr;        // pinned readback: ring (3 kSlot), then kHostAux scratch doubles
    unsigned long long* host_u = nullptr;
    int* raw_err = nullptr;
    AdjScratch adj{};
    bool adj_march = false;        // fused single-march adjoint (D2Q4)
    bool resident = false;         // D1Q2 batches in one resident workgroup (small grids)
    hipStream_t stream;
    int device = 0;                // current device at creation: where the buffers live
    long long n = 0;
    double t = 0.0, c = 0.0;
    bool initialised = false;
    std::string msg;
};

namespace {

vlbm_status fail(vlbm_ctx* ctx, vlbm_status st, const std::string& m)
{
    if (ctx) ctx->msg = m;
    return st;
}

vlbm_status hip_fail(vlbm_ctx* ctx, hipError_t e, const char* where)
{
    return fail(ctx, VLBM_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(ctx, expr)                                      \
    do {                                                       \
        hipError_t e_ = (expr);                                \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr); \
    } while (0)

vlbm_status err_status(int bits)
{
    if (bits & ERR_NONFINITE) return VLBM_ENONFINITE;
    if (bits & ERR_NONHYP) return VLBM_ENONHYPERBOLIC;
    return VLBM_OK;
}

vlbm_status sync_readback(vlbm_ctx* ctx)
{
    HIPCHK(ctx, hipMemcpyAsync(ctx->host, ctx->ring, 3 * kSlot * sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(ctx->host_u, ctx->stop_at, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync((char*)(ctx->host_u + 1), ctx->err, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return VLBM_OK;
}

hipError_t launch_one(vlbm_ctx* ctx, long long n, double t_end)
{
    KStep s{};
    double* slot = ctx->ring + kSlot * (n % 3);
    double* next = ctx->ring + kSlot * ((n + 1) % 3);
    double* after = ctx->ring + kSlot * ((n + 2) % 3);
    s.clock_in = slot;
    s.clock_out = next;
    s.red_in = slot + kRedBase;
    s.red_out = next + kRedBase;
    s.red_clear = after + kRedBase;
    s.red_copies = kRedCopies;
    s.red_stride = kRedStride;
    s.stop_at = ctx->stop_at;
    s.err = ctx->err;
    s.n = n;
    s.t_end = t_end;
    const void* fin = ctx->f[n & 1];
    void* fout = ctx->f[(n + 1) & 1];
    return ctx->D == 2 ? launch_step_d2q4(ctx->kp, s, ctx->prec, fin, fout, ctx->stream)
                       : launch_step_d1q2(ctx->kp, s, ctx->prec, fin, fout, ctx->stream);
}

// steps per launch of the resident D1Q2 kernel: bounds one launch's duration
// (about 20 ms at 2048 cells) without a measurable cost per launch
constexpr long long kResidentChunk = 4096;

// launch `count` steps from the host's step index, read back, update the mirror
vlbm_status run_batch(vlbm_ctx* ctx, long long count, double t_end, long long* executed)
{
    const long long n0 = ctx->n;
    if (ctx->resident) {
        for (long long k = 0; k < count; k += kResidentChunk) {
            KRun r{ctx->ring, ctx->stop_at, ctx->err, n0 + k, std::min(kResidentChunk, count - k), t_end};
            HIPCHK(ctx, launch_run_d1q2(ctx->kp, r, ctx->prec, ctx->f[0], ctx->f[1], ctx->stream));
        }
    } else {
        for (long long k = 0; k < count; ++k) HIPCHK(ctx, launch_one(ctx, n0 + k, t_end));
    }
    vlbm_status st = sync_readback(ctx);
    if (st != VLBM_OK) return st;
    const unsigned long long stop = ctx->host_u[0];
    int bits;
    memcpy(&bits, (char*)(ctx->host_u + 1), sizeof(int));
    long long nn = n0 + count;
    if (stop != ~0ull && (long long)stop < nn) nn = (long long)stop;
    ctx->n = nn;
    const double* slot = ctx->host + kSlot * (nn % 3);
    ctx->t = slot[0];
    ctx->c = slot[1];
    *executed = nn - n0;
    if (bits) {
        char buf[160];
        snprintf(buf, sizeof buf, "inadmissible state (bits %d) at step %lld", bits, nn);
        return fail(ctx, err_status(bits), buf);
    }
    return VLBM_OK;
}

// Elements per population plane: the cells rounded up to 64, plus 1 KB.  Without
// the extra kilobyte the planes of a power-of-two grid start a power of two
// apart, and the 16 row streams of the D2Q4 march meet in the same HBM
// channels (measured on MI355X at 4096^2: FP64 +4.5 %, FP32 +2 %; D1Q2 +2 %;
// 512 B and 1.5 KB did about as well, 4 KB was slower).
long long padded_plane(long long ncell, long long esize)
{
    return (ncell + 63) / 64 * 64 + 1024 / esize;
}

bool check_config(const vlbm_config* c, std::string& why)
{
    if (c->dim != 1 && c->dim != 2) return why = "dim must be 1 or 2", false;
    if (c->nx < 4 || c->nx > (1LL << 30)) return why = "nx out of range", false;
    if (c->dim == 1 && c->ny != 1) return why = "ny must be 1 in 1-D", false;
    if (c->dim == 2 && (c->ny < 4 || c->ny > (1LL << 30))) return why = "ny out of range", false;
    if (c->nx * c->ny > (1LL << 31)) return why = "grid too large", false;
    if (!(c->dx > 0) || !std::isfinite(c->dx)) return why = "dx must be positive", false;
    for (int i = 0; i < 4; ++i) {
        const bool pinned_ok = i < 2 && c->bc[i] == VLBM_BC_PINNED;
        if (c->bc[i] != VLBM_BC_PERIODIC && c->bc[i] != VLBM_BC_OUTFLOW && !pinned_ok)
            return why = "bad boundary kind (pinned is for x edges only)", false;
    }
    if ((c->bc[0] == VLBM_BC_PERIODIC) != (c->bc[1] == VLBM_BC_PERIODIC))
        return why = "periodic x needs both x sides periodic", false;
    if (c->dim == 2 && (c->bc[2] == VLBM_BC_PERIODIC) != (c->bc[3] == VLBM_BC_PERIODIC))
        return why = "periodic y needs both y sides periodic", false;
    if (c->eos != VLBM_EOS_IDEAL && c->eos != VLBM_EOS_VDW) return why = "bad eos", false;
    if (!(c->gamma > 1.0)) return why = "gamma must exceed 1", false;
    if (c->eos == VLBM_EOS_VDW && (!(c->vdw_R > 0) || c->vdw_a < 0 || c->vdw_b < 0))
        return why = "bad van der Waals constants", false;
    if (!std::isfinite(c->e_offset)) return why = "e_offset must be finite", false;
    for (int side = 0; side < 2; ++side) {
        if (c->bc[side] != VLBM_BC_PINNED) continue;
        const double* w = c->bc_state[side];
        const int NK = c->dim + 2;
        for (int k = 0; k < NK; ++k)
            if (!std::isfinite(w[k])) return why = "pinned state must be finite", false;
        if (!(w[0] > 0)) return why = "pinned state needs rho > 0", false;
        double ke = 0.0;
        for (int a = 0; a < c->dim; ++a) ke += 0.5 * w[1 + a] * w[1 + a] / w[0];
        const double e = (w[NK - 1] - ke) / w[0];   // specific internal energy
        // positive pressure (ideal) / temperature and co-volume (van der Waals, Eqs. 16-17)
        if (c->eos == VLBM_EOS_IDEAL && !(e > 0)) return why = "pinned state needs e > 0", false;
        if (c->eos == VLBM_EOS_VDW && (!(e + c->vdw_a * w[0] > 0) || !(c->vdw_b * w[0] < 1)))
            return why = "pinned state needs T > 0 and b rho < 1", false;
    }
    if (c->retarget_every < 0) return why = "retarget_every must be >= 0", false;
    if (c->retarget_every > 0 && !(c->cfl > 0 && c->cfl <= 1.0)) return why = "cfl must be in (0, 1]", false;
    if (c->retarget_every == 0 && !(c->c_fixed > 0)) return why = "c_fixed must be positive", false;
    if (c->sensor < 0 || c->sensor > 3) return why = "bad sensor", false;
    auto okb = [](double b) { return b > 0.0 && b <= 1.0; };
    if (c->sensor == VLBM_SENSOR_OFF && !okb(c->beta_const)) return why = "beta_const must be in (0, 1]", false;
    if (c->sensor != VLBM_SENSOR_OFF &&
        (!okb(c->beta_min) || !okb(c->beta_max) || c->beta_min > c->beta_max || !(c->c_sensor >= 0) ||
         !(c->eps_theta > 0)))
        return why = "bad sensor constants", false;
    if (c->precision != VLBM_FP64 && c->precision != VLBM_FP32 && c->precision != VLBM_FP32_MIXED)
        return why = "bad precision", false;
    if (c->dim == 2) {
        // the D2Q4 marches address four planes from one buffer resource with
        // 32-bit offsets: 4 padded planes must fit in 4 GiB.  A plane holds the
        // cells rounded up to 64 plus 1 KB, so the largest grids are 2^27 - 128
        // cells in FP64 and 2^28 - 256 with FP32 storage
        const long long esize = c->precision == VLBM_FP64 ? 8 : 4;
        const long long plane = padded_plane(c->nx * c->ny, esize);
        if (4 * plane * esize > (1LL << 32))
            return why = "grid too large for the D2Q4 kernels' 32-bit offsets (at most 2^27 - 128 cells in FP64, "
                         "2^28 - 256 with FP32 storage)",
                   false;
    }
    return true;
}

}  // namespace

extern "C" {

vlbm_status vlbm_check_config(const vlbm_config* cfg)
{
    std::string why;
    return cfg && check_config(cfg, why) ? VLBM_OK : VLBM_EINVAL;
}

vlbm_status vlbm_create(const vlbm_config* cfg, vlbm_ctx** out)
{
    if (!cfg || !out) return VLBM_EINVAL;
    *out = nullptr;
    std::string why;
    if (!check_config(cfg, why)) {
        fprintf(stderr, "vlbm_create: %s\n", why.c_str());
        return VLBM_EINVAL;
    }
    vlbm_ctx* ctx = new vlbm_ctx();
    ctx->cfg = *cfg;
    if (hipGetDevice(&ctx->device) != hipSuccess) {
        delete ctx;
        return VLBM_EDEVICE;
    }
    ctx->stream = (hipStream_t)cfg->stream;
    ctx->D = cfg->dim;
    ctx->Q = 2 * cfg->dim;
    ctx->NK = cfg->dim + 2;
    ctx->nplanes = ctx->Q * ctx->NK;
    ctx->prec = cfg->precision == VLBM_FP32 ? PREC_FP32 : cfg->precision == VLBM_FP32_MIXED ? PREC_FP32_MIXED : PREC_FP64;
    ctx->fp32 = ctx->prec != PREC_FP64;
    ctx->esize = ctx->fp32 ? 4 : 8;
    ctx->ncell = cfg->nx * cfg->ny;
    ctx->plane = padded_plane(ctx->ncell, ctx->esize);

    KParams& p = ctx->kp;
    p.dim = cfg->dim;
    p.nx = (int)cfg->nx;
    p.ny = (int)cfg->ny;
    p.plane = ctx->plane;
    p.dx = cfg->dx;
    for (int i = 0; i < 4; ++i) p.bc[i] = cfg->bc[i];
    for (int side = 0; side < 2; ++side)
        for (int k = 0; k < 4; ++k) p.pin_w[side][k] = cfg->bc[side] == VLBM_BC_PINNED ? cfg->bc_state[side][k] : 0.0;
    p.eos = cfg->eos;
    p.gamma = cfg->gamma;
    p.vdw_a = cfg->vdw_a;
    p.vdw_b = cfg->vdw_b;
    p.vdw_R = cfg->eos == VLBM_EOS_VDW ? cfg->vdw_R : 1.0;
    p.inv_cv = (cfg->gamma - 1.0) / p.vdw_R;
    p.e_off = cfg->e_offset;
    p.cfl = cfg->cfl;
    p.c_fixed = cfg->c_fixed;
    p.retarget_every = cfg->retarget_every;
    int sensor = cfg->sensor;
    if (sensor == VLBM_SENSOR_AUTO) sensor = cfg->dim == 1 ? VLBM_SENSOR_A : VLBM_SENSOR_B;
    if (cfg->dim == 1 && sensor == VLBM_SENSOR_B) sensor = VLBM_SENSOR_A;   // no vorticity in 1-D
    p.sensor = sensor;
    p.beta_const = cfg->beta_const;
    p.beta_min = cfg->beta_min;
    p.beta_max = cfg->beta_max;
    p.c_sensor = cfg->c_sensor;
    p.eps_theta = cfg->eps_theta;
    configure_d2q4(p, ctx->prec);   // the D2Q4 march's tiling (vlbm_step2d.hip)

    const size_t fbytes = (size_t)ctx->nplanes * ctx->plane * ctx->esize;
    bool ok = hipMalloc(&ctx->f[0], fbytes) == hipSuccess && hipMalloc(&ctx->f[1], fbytes) == hipSuccess &&
              hipMalloc(&ctx->ring, 3 * kSlot * sizeof(double)) == hipSuccess &&
              hipMalloc(&ctx->stop_at, sizeof(unsigned long long)) == hipSuccess &&
              hipMalloc(&ctx->err, sizeof(int)) == hipSuccess &&
              hipMalloc(&ctx->raw_err, sizeof(int)) == hipSuccess &&
              hipMalloc(&ctx->scratchW, (size_t)ctx->NK * ctx->ncell * sizeof(double)) == hipSuccess &&
              hipMalloc(&ctx->scratchB, (size_t)ctx->ncell * sizeof(double)) == hipSuccess &&
              hipMalloc(&ctx->partials, (size_t)totals_nparts(ctx->ncell) * 4 * sizeof(double) + 64) == hipSuccess &&
              hipMalloc(&ctx->norms_scratch, 16 * sizeof(double)) == hipSuccess &&
              hipHostMalloc((void**)&ctx->host, (kHostAux + kSlot + 16) * sizeof(double)) == hipSuccess &&
              hipHostMalloc((void**)&ctx->host_u, 4 * sizeof(unsigned long long)) == hipSuccess;
    if (ok && cfg->retarget_every == 0) {
        // adjoint scratch only for frozen-speed contexts (the raw entry points)
        ok = hipMalloc(&ctx->adj.aux, adjoint_aux_elems(p) * sizeof(double)) == hipSuccess &&
             hipMalloc(&ctx->adj.partials, adjoint_partials_count(p) * 4 * sizeof(double) + 64) == hipSuccess &&
             hipMalloc(&ctx->adj.qmax, 8 * sizeof(double)) == hipSuccess &&
             hipMalloc(&ctx->adj.argmax, 8 * sizeof(unsigned long long)) == hipSuccess &&
             hipMalloc(&ctx->adj.rec, (size_t)std::max(adjoint_march_records(p), 1) * 12 * sizeof(double)) ==
                 hipSuccess;
        // the fused adjoint march is used where it applies (D2Q4, halo >= 4 columns,
        // physical energy gauge); VLBM_ADJ_MULTIPASS=1 selects the multi-pass form
        const char* mp = getenv("VLBM_ADJ_MULTIPASS");
        ctx->adj_march = adjoint_march_supported(p) && !(mp && atoi(mp) != 0);
    }
    if (!ok) {
        vlbm_destroy(ctx);
        return VLBM_ENOMEM;
    }
    // D1Q2 grids that one workgroup holds run their batches in it (VLBM_D1_RESIDENT=0:
    // one launch per step, as on larger grids)
    ctx->resident = cfg->dim == 1 && p.nx <= resident_d1q2_max_cells(ctx->prec);
    if (const char* env = getenv("VLBM_D1_RESIDENT")) ctx->resident = ctx->resident && atoi(env) != 0;
    if (launch_reset_ctl(ctx->ring, ctx->stop_at, ctx->err, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess) {
        vlbm_destroy(ctx);
        return VLBM_EDEVICE;
    }
    *out = ctx;
    return VLBM_OK;
}

void vlbm_destroy(vlbm_ctx* ctx)
{
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    for (void* p : {ctx->f[0], ctx->f[1], (void*)ctx->ring, (void*)ctx->stop_at, (void*)ctx->err,
                    (void*)ctx->raw_err, (void*)ctx->scratchW, (void*)ctx->scratchB, (void*)ctx->partials,
                    (void*)ctx->norms_scratch, ctx->adj.aux, (void*)ctx->adj.partials, (void*)ctx->adj.qmax,
                    (void*)ctx->adj.argmax, (void*)ctx->adj.rec})
        if (p) (void)hipFree(p);
    if (ctx->host) (void)hipHostFree(ctx->host);
    if (ctx->host_u) (void)hipHostFree(ctx->host_u);
    delete ctx;
}

vlbm_status vlbm_init(vlbm_ctx* ctx, const double* W0, int32_t W0_on_device)
{
    if (!ctx || !W0) return fail(ctx, VLBM_EINVAL, "null argument");
    const size_t wbytes = (size_t)ctx->NK * ctx->ncell * sizeof(double);
    HIPCHK(ctx, hipMemcpyAsync(ctx->scratchW, W0, wbytes,
                               W0_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, launch_reset_ctl(ctx->ring, ctx->stop_at, ctx->err, ctx->stream));
    HIPCHK(ctx, launch_init(ctx->kp, ctx->fp32, ctx->scratchW, ctx->ncell, ctx->ring, ctx->ring + kRedBase,
                            kRedCopies, kRedStride, ctx->err, ctx->cfg.retarget_every == 0, ctx->f[0], ctx->stream));
    vlbm_status st = sync_readback(ctx);
    if (st != VLBM_OK) return st;
    int bits;
    memcpy(&bits, (char*)(ctx->host_u + 1), sizeof(int));
    ctx->n = 0;
    ctx->t = ctx->host[0];
    ctx->c = ctx->host[1];
    ctx->initialised = false;
    if (bits) return fail(ctx, err_status(bits), "initial state not admissible");
    if (!(ctx->c > 0) || !std::isfinite(ctx->c)) return fail(ctx, VLBM_EINVAL, "initial link speed not positive");
    ctx->initialised = true;
    return VLBM_OK;
}

vlbm_status vlbm_step(vlbm_ctx* ctx, int64_t nsteps, double t_end_cap, int64_t* steps_taken)
{
    if (steps_taken) *steps_taken = 0;
    if (!ctx || nsteps < 0) return fail(ctx, VLBM_EINVAL, "bad argument");
    if (!ctx->initialised) return fail(ctx, VLBM_EINVAL, "not initialised");
    if (std::isnan(t_end_cap)) return fail(ctx, VLBM_EINVAL, "t_end_cap is NaN");
    if (ctx->t >= t_end_cap) return VLBM_EDONE;
    if (nsteps == 0) return VLBM_OK;
    HIPCHK(ctx, launch_reset_stop(ctx->stop_at, ctx->err, ctx->stream));
    long long done = 0;
    vlbm_status st = run_batch(ctx, nsteps, std::isinf(t_end_cap) ? HUGE_VAL : t_end_cap, &done);
    if (steps_taken) *steps_taken = done;
    return st;
}

vlbm_status vlbm_run_to_time(vlbm_ctx* ctx, double t_end, int64_t* steps_taken)
{
    if (steps_taken) *steps_taken = 0;
    if (!ctx || !std::isfinite(t_end)) return fail(ctx, VLBM_EINVAL, "bad argument");
    if (!ctx->initialised) return fail(ctx, VLBM_EINVAL, "not initialised");
    if (ctx->t >= t_end) return VLBM_EDONE;
    long long total = 0;
    HIPCHK(ctx, launch_reset_stop(ctx->stop_at, ctx->err, ctx->stream));
    while (ctx->t < t_end) {
        // steps left at the current time step, plus a margin; extra launches
        // after the landing step return at once
        const double dt = ctx->cfg.dx / ctx->c;
        double est = std::ceil((t_end - ctx->t) / dt);
        long long batch = (long long)std::min(std::max(est * 1.05 + 4.0, 1.0), 8192.0);
        long long done = 0;
        vlbm_status st = run_batch(ctx, batch, t_end, &done);
        total += done;
        if (st != VLBM_OK) {
            if (steps_taken) *steps_taken = total;
            return st;
        }
        if (done < batch) break;   // landed
    }
    if (steps_taken) *steps_taken = total;
    return VLBM_OK;
}

vlbm_status vlbm_conserved_totals(vlbm_ctx* ctx, double* out)
{
    if (!ctx || !out) return fail(ctx, VLBM_EINVAL, "null argument");
    if (!ctx->initialised) return fail(ctx, VLBM_EINVAL, "not initialised");
    double* dout = ctx->norms_scratch;
    HIPCHK(ctx, launch_totals(ctx->D, ctx->plane, ctx->ncell, ctx->fp32, ctx->kp.e_off, ctx->f[ctx->n & 1], ctx->partials, dout,
                              ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(ctx->host + kHostAux, dout, ctx->NK * sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    const double vol = ctx->D == 1 ? ctx->cfg.dx : ctx->cfg.dx * ctx->cfg.dx;
    for (int k = 0; k < ctx->NK; ++k) out[k] = ctx->host[kHostAux + k] * vol;
    return VLBM_OK;
}

vlbm_status vlbm_get_W(vlbm_ctx* ctx, double* out, int32_t out_on_device)
{
    if (!ctx || !out) return fail(ctx, VLBM_EINVAL, "null argument");
    if (!ctx->initialised) return fail(ctx, VLBM_EINVAL, "not initialised");
    double* dst = out_on_device ? out : ctx->scratchW;
    HIPCHK(ctx, launch_moments(ctx->D, ctx->plane, ctx->ncell, ctx->fp32, ctx->kp.e_off, ctx->f[ctx->n & 1], dst, ctx->stream));
    if (!out_on_device)
        HIPCHK(ctx, hipMemcpyAsync(out, dst, (size_t)ctx->NK * ctx->ncell * sizeof(double), hipMemcpyDeviceToHost,
                                   ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return VLBM_OK;
}

vlbm_status vlbm_get_beta(vlbm_ctx* ctx, double* out, int32_t out_on_device)
{
    if (!ctx || !out) return fail(ctx, VLBM_EINVAL, "null argument");
    if (!ctx->initialised) return fail(ctx, VLBM_EINVAL, "not initialised");
    KParams p = ctx->kp;
    p.c_fixed = ctx->c;
    KStep s{};
    double* slot = ctx->ring + kSlot * (ctx->n % 3);
    s.clock_in = slot;
    s.red_in = slot + kRedBase;
    s.red_copies = kRedCopies;
    s.red_stride = kRedStride;
    s.red_out = ctx->norms_scratch;
    s.err = ctx->raw_err;
    s.frozen = 1;
    s.probe = 1;
    s.beta_out = out_on_device ? out : ctx->scratchB;
    s.t_end = HUGE_VAL;
    const void* fin = ctx->f[ctx->n & 1];
    HIPCHK(ctx, ctx->D == 2 ? launch_step_d2q4(p, s, ctx->prec, fin, nullptr, ctx->stream)
                            : launch_step_d1q2(p, s, ctx->prec, fin, nullptr, ctx->stream));
    if (!out_on_device)
        HIPCHK(ctx, hipMemcpyAsync(out, ctx->scratchB, (size_t)ctx->ncell * sizeof(double), hipMemcpyDeviceToHost,
                                   ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return VLBM_OK;
}

vlbm_status vlbm_get_f(vlbm_ctx* ctx, void* out, int32_t out_on_device)
{
    if (!ctx || !out) return fail(ctx, VLBM_EINVAL, "null argument");
    if (!ctx->initialised) return fail(ctx, VLBM_EINVAL, "not initialised");
    const size_t bytes = (size_t)ctx->nplanes * ctx->ncell * ctx->esize;
    if (out_on_device) {
        HIPCHK(ctx, launch_unpad(ctx->D, ctx->plane, ctx->ncell, ctx->fp32, ctx->kp.e_off, ctx->f[ctx->n & 1], out,
                                 ctx->stream));
    } else {
        void* tmp = ctx->f[(ctx->n + 1) & 1];   // the spare buffer is free between steps
        HIPCHK(ctx, launch_unpad(ctx->D, ctx->plane, ctx->ncell, ctx->fp32, ctx->kp.e_off, ctx->f[ctx->n & 1], tmp,
                                 ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(out, tmp, bytes, hipMemcpyDeviceToHost, ctx->stream));
    }
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return VLBM_OK;
}

vlbm_status vlbm_get_clock(vlbm_ctx* ctx, double* t, double* c, int64_t* n)
{
    if (!ctx) return VLBM_EINVAL;
    if (t) *t = ctx->t;
    if (c) *c = ctx->c;
    if (n) *n = ctx->n;
    return VLBM_OK;
}

// Checkpoint layout: a header naming the context it was taken from, the
// populations, the ring slot of the current state (clock and reductions), the
// step count.
struct CkptHeader {
    char magic[8];
    int64_t version, dim, nx, ny, precision, plane, nplanes;
};
static_assert(sizeof(CkptHeader) == 64, "checkpoint header is 64 bytes");
constexpr int64_t kCkptVersion = 1;

static CkptHeader ckpt_header(const vlbm_ctx* ctx)
{
    CkptHeader h{};
    memcpy(h.magic, "VLBMCKPT", 8);
    h.version = kCkptVersion;
    h.dim = ctx->D;
    h.nx = ctx->cfg.nx;
    h.ny = ctx->cfg.ny;
    h.precision = ctx->cfg.precision;
    h.plane = ctx->plane;
    h.nplanes = ctx->nplanes;
    return h;
}

size_t vlbm_state_bytes(const vlbm_ctx* ctx)
{
    if (!ctx) return 0;
    return sizeof(CkptHeader) + (size_t)ctx->nplanes * ctx->plane * ctx->esize + (kSlot + 8) * sizeof(double);
}

vlbm_status vlbm_save(vlbm_ctx* ctx, void* buf, size_t bytes)
{
    if (!ctx || !buf) return fail(ctx, VLBM_EINVAL, "null argument");
    if (!ctx->initialised) return fail(ctx, VLBM_EINVAL, "not initialised");
    if (bytes < vlbm_state_bytes(ctx)) return fail(ctx, VLBM_EINVAL, "checkpoint buffer smaller than vlbm_state_bytes");
    const size_t hb = sizeof(CkptHeader), fb = (size_t)ctx->nplanes * ctx->plane * ctx->esize;
    char* b = (char*)buf;
    // header and step count staged in pinned host memory
    double* stage = ctx->host + kHostAux;
    const CkptHeader h = ckpt_header(ctx);
    memcpy(stage, &h, hb);
    stage[hb / sizeof(double)] = (double)ctx->n;
    HIPCHK(ctx, hipMemcpyAsync(b, stage, hb, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(b + hb, ctx->f[ctx->n & 1], fb, hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(b + hb + fb, ctx->ring + kSlot * (ctx->n % 3), kSlot * sizeof(double),
                               hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(b + hb + fb + kSlot * sizeof(double), stage + hb / sizeof(double), sizeof(double),
                               hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return VLBM_OK;
}

vlbm_status vlbm_restore(vlbm_ctx* ctx, const void* buf, size_t bytes)
{
    if (!ctx || !buf) return fail(ctx, VLBM_EINVAL, "null argument");
    if (bytes < vlbm_state_bytes(ctx)) return fail(ctx, VLBM_EINVAL, "checkpoint buffer smaller than vlbm_state_bytes");
    const size_t hb = sizeof(CkptHeader), fb = (size_t)ctx->nplanes * ctx->plane * ctx->esize;
    const char* b = (const char*)buf;
    double* stage = ctx->host + kHostAux;
    HIPCHK(ctx, hipMemcpyAsync(stage, b, hb, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    CkptHeader h;
    memcpy(&h, stage, hb);
    const CkptHeader want = ckpt_header(ctx);
    if (memcmp(&h, &want, hb) != 0)
        return fail(ctx, VLBM_EINVAL, "checkpoint taken from a context of another grid, lattice or precision");
    HIPCHK(ctx, hipMemcpyAsync(stage, b + hb + fb, (kSlot + 1) * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    const double t = stage[0], c = stage[1], nd = stage[kSlot];
    if (!(nd >= 0) || nd != std::floor(nd) || !std::isfinite(t) || !(c > 0) || !std::isfinite(c))
        return fail(ctx, VLBM_EINVAL, "corrupt checkpoint");
    const long long n = (long long)nd;
    HIPCHK(ctx, launch_reset_ctl(ctx->ring, ctx->stop_at, ctx->err, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(ctx->f[n & 1], b + hb, fb, hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(ctx->ring + kSlot * (n % 3), b + hb + fb, kSlot * sizeof(double),
                               hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    ctx->n = n;
    ctx->t = t;
    ctx->c = c;
    ctx->initialised = true;
    return VLBM_OK;
}

int64_t vlbm_plane_elems(const vlbm_ctx* ctx) { return ctx ? ctx->plane : 0; }

size_t vlbm_population_bytes(const vlbm_ctx* ctx)
{
    return ctx ? (size_t)ctx->nplanes * ctx->plane * ctx->esize : 0;
}

// ------------------------------------------------------------------ raw entry points

static vlbm_status need_frozen(vlbm_ctx* ctx)
{
    if (!ctx) return VLBM_EINVAL;
    if (ctx->cfg.retarget_every != 0) return fail(ctx, VLBM_EINVAL, "raw entry points need retarget_every == 0");
    return VLBM_OK;
}

// the adjoint kernels work in the physical energy gauge, with periodic and
// outflow edges
static vlbm_status need_adjoint_support(vlbm_ctx* ctx)
{
    if (ctx->cfg.e_offset != 0.0) return fail(ctx, VLBM_EINVAL, "the adjoint entry points need e_offset == 0");
    if (ctx->cfg.bc[0] == VLBM_BC_PINNED || ctx->cfg.bc[1] == VLBM_BC_PINNED)
        return fail(ctx, VLBM_EINVAL, "the adjoint entry points do not cover pinned edges");
    return VLBM_OK;
}

vlbm_status vlbm_raw_init(vlbm_ctx* ctx, const double* W0, void* f0, double* norms0)
{
    if (vlbm_status st = need_frozen(ctx)) return st;
    if (!W0 || !f0 || !norms0) return fail(ctx, VLBM_EINVAL, "null argument");
    HIPCHK(ctx, launch_zero(norms0, VLBM_NORMS_LEN, ctx->stream));
    HIPCHK(ctx, launch_init(ctx->kp, ctx->fp32, W0, ctx->ncell, ctx->norms_scratch, norms0, kRedCopies, kRedStride,
                            ctx->raw_err, 1, f0, ctx->stream));
    return VLBM_OK;
}

vlbm_status vlbm_raw_step(vlbm_ctx* ctx, const void* f_in, const double* norms_in, void* f_out, double* norms_out)
{
    if (vlbm_status st = need_frozen(ctx)) return st;
    if (!f_in || !f_out || !norms_in || !norms_out) return fail(ctx, VLBM_EINVAL, "null argument");
    if (((uintptr_t)f_in | (uintptr_t)f_out) & 15) return fail(ctx, VLBM_EINVAL, "populations must be 16-byte aligned");
    HIPCHK(ctx, launch_zero(norms_out, VLBM_NORMS_LEN, ctx->stream));
    KStep s{};
    s.red_in = norms_in;
    s.red_out = norms_out;
    s.red_copies = kRedCopies;
    s.red_stride = kRedStride;
    s.err = ctx->raw_err;
    s.frozen = 1;
    s.t_end = HUGE_VAL;
    HIPCHK(ctx, ctx->D == 2 ? launch_step_d2q4(ctx->kp, s, ctx->prec, f_in, f_out, ctx->stream)
                            : launch_step_d1q2(ctx->kp, s, ctx->prec, f_in, f_out, ctx->stream));
    return VLBM_OK;
}

vlbm_status vlbm_raw_adjoint_step(vlbm_ctx* ctx, const void* f_n, const double* norms_n, const void* lam_np1,
                                  void* lam_n)
{
    if (vlbm_status st = need_frozen(ctx)) return st;
    if (vlbm_status st = need_adjoint_support(ctx)) return st;
    if (!f_n || !norms_n || !lam_np1 || !lam_n) return fail(ctx, VLBM_EINVAL, "null argument");
    if (lam_np1 == lam_n) return fail(ctx, VLBM_EINVAL, "lam_np1 and lam_n must differ");
    if (ctx->adj_march)
        HIPCHK(ctx, launch_adjoint_march(ctx->kp, ctx->prec, f_n, norms_n, lam_np1, lam_n, ctx->adj.rec, ctx->stream));
    else
        HIPCHK(ctx, launch_adjoint_step(ctx->kp, ctx->prec, f_n, norms_n, lam_np1, lam_n, ctx->adj, ctx->stream));
    return VLBM_OK;
}

vlbm_status vlbm_raw_adjoint_step_static(vlbm_ctx* ctx, const void* f_n, const double* norms_n, const void* lam_np1,
                                         void* lam_n)
{
    if (vlbm_status st = need_frozen(ctx)) return st;
    if (vlbm_status st = need_adjoint_support(ctx)) return st;
    if (!f_n || !norms_n || !lam_np1 || !lam_n) return fail(ctx, VLBM_EINVAL, "null argument");
    if (lam_np1 == lam_n) return fail(ctx, VLBM_EINVAL, "lam_np1 and lam_n must differ");
    if (!ctx->adj_march)
        return fail(ctx, VLBM_EINVAL, "the allocation-free adjoint step covers the fused D2Q4 march only");
    const int need = adjoint_march_records(ctx->kp);
    if (need > kStaticMarchRecords) {
        char buf[200];
        snprintf(buf, sizeof buf,
                 "the grid's tiling needs %d march records, the static scratch of the allocation-free adjoint step "
                 "holds %d",
                 need, kStaticMarchRecords);
        return fail(ctx, VLBM_EINVAL, buf);
    }
    double* rec = nullptr;
    HIPCHK(ctx, adjm_static_scratch(ctx->device, &rec));
    HIPCHK(ctx, launch_adjoint_march(ctx->kp, ctx->prec, f_n, norms_n, lam_np1, lam_n, rec, ctx->stream));
    return VLBM_OK;
}

vlbm_status vlbm_raw_init_adjoint(vlbm_ctx* ctx, const double* W0, const void* lam0, double* W0bar)
{
    if (vlbm_status st = need_frozen(ctx)) return st;
    if (vlbm_status st = need_adjoint_support(ctx)) return st;
    if (!W0 || !lam0 || !W0bar) return fail(ctx, VLBM_EINVAL, "null argument");
    HIPCHK(ctx, launch_init_adjoint(ctx->kp, ctx->prec, W0, ctx->ncell, lam0, W0bar, ctx->stream));
    return VLBM_OK;
}

vlbm_status vlbm_raw_moments(vlbm_ctx* ctx, const void* f, double* W)
{
    if (!ctx || !f || !W) return fail(ctx, VLBM_EINVAL, "null argument");
    HIPCHK(ctx, launch_moments(ctx->D, ctx->plane, ctx->ncell, ctx->fp32, ctx->kp.e_off, f, W, ctx->stream));
    return VLBM_OK;
}

vlbm_status vlbm_raw_moments_adjoint(vlbm_ctx* ctx, const double* Wbar, void* lam)
{
    if (!ctx || !Wbar || !lam) return fail(ctx, VLBM_EINVAL, "null argument");
    if (vlbm_status st = need_adjoint_support(ctx)) return st;
    HIPCHK(ctx, launch_moments_adj(ctx->D, ctx->plane, ctx->ncell, ctx->fp32, Wbar, lam, ctx->stream));
    return VLBM_OK;
}

const char* vlbm_last_error(const vlbm_ctx* ctx) { return ctx ? ctx->msg.c_str() : "null context"; }

vlbm_status vlbm_copy_probe(const void* src, void* dst, size_t bytes, void* stream, int32_t mode)
{
    if (!src || !dst || bytes % 16 != 0 || (mode != 0 && mode != 1)) return VLBM_EINVAL;
    return launch_copy_probe(src, dst, bytes, mode, (hipStream_t)stream) == hipSuccess ? VLBM_OK : VLBM_EDEVICE;
}

size_t vlbm_copy_probe_read_bytes(size_t bytes) { return read_probe_out_bytes(bytes); }

vlbm_status vlbm_probe_march(vlbm_ctx* ctx, int32_t nlaunch)
{
    if (!ctx || nlaunch < 0) return fail(ctx, VLBM_EINVAL, "bad argument");
    if (ctx->D != 2) return fail(ctx, VLBM_EINVAL, "the march probe is the D2Q4 step's access pattern");
    if (!ctx->initialised) return fail(ctx, VLBM_EINVAL, "not initialised");
    const void* fin = ctx->f[ctx->n & 1];
    void* spare = ctx->f[(ctx->n + 1) & 1];   // free between steps
    for (int i = 0; i < nlaunch; ++i) HIPCHK(ctx, launch_march_probe(ctx->kp, ctx->fp32, fin, spare, ctx->stream));
    return VLBM_OK;
}

}  // extern "C"
