// Internal launcher declarations of the VLBM library (not part of the ABI).
#pragma once

#include "vlbm_common.hpp"

namespace vlbm {

hipError_t launch_step_d2q4(const KParams& p, const KStep& s, int prec, const void* fin, void* fout, hipStream_t st);
hipError_t launch_step_d1q2(const KParams& p, const KStep& s, int prec, const void* fin, void* fout, hipStream_t st);
int step_d2q4_blocks_per_cu(const KParams& p, int prec);
// Tiling of the D2Q4 march for a context (strip width, wavefronts per
// workgroup, rows of loads in flight, segment height; the measured choices
// with their environment overrides).  Needs dim, nx, ny and retarget_every of p;
// sets strip_w, nstrips, deep, wpg, ngroups, seg_h and nsegs (one segment of
// ny rows for D1Q2).
void configure_d2q4(KParams& p, int prec);

// A batch of D1Q2 steps in one resident workgroup (vlbm_resident1d.hip), for
// grids of at most resident_d1q2_max_cells cells: steps n0 .. n0 + count - 1,
// stopping early at a landing or an inadmissible state (then stop_at = the
// index of the state reached, and err holds its bits), or not at all when n0 >=
// stop_at.  State n0 is read from f0 or f1 (n0 & 1), its clock and reductions
// from ring slot n0 % 3; the state reached goes to buffer n & 1 and ring slot n % 3.
struct KRun {
    double* ring;                  // 3 slots of kSlot doubles
    unsigned long long* stop_at;
    int* err;
    long long n0, count;
    double t_end;                  // landing time (HUGE_VAL: none)
};
int resident_d1q2_max_cells(int prec);
hipError_t launch_run_d1q2(const KParams& p, const KRun& r, int prec, void* f0, void* f1, hipStream_t st);
// measurement aid: the D2Q4 step's loads and stores without its arithmetic
hipError_t launch_march_probe(const KParams& p, bool fp32, const void* fin, void* fout, hipStream_t st);

hipError_t launch_reset_ctl(double* ring, unsigned long long* stop_at, int* err, hipStream_t st);
hipError_t launch_reset_stop(unsigned long long* stop_at, int* err, hipStream_t st);
hipError_t launch_zero(double* p, int n, hipStream_t st);
// reductions of W0 into `copies` copies at red0 (stride apart), then the clock
// (t = 0, c0) at clock0 and f = f^eq(W0; c0)
hipError_t launch_init(const KParams& p, bool fp32, const double* W, long long ncell, double* clock0, double* red0,
                       int copies, int stride, int* err, int frozen, void* f, hipStream_t st);
// moments, totals and the population copy return the physical energy gauge
// (e_off: the gauge shift of the stored populations, KParams::e_off)
hipError_t launch_moments(int D, long long plane, long long ncell, bool fp32, double e_off, const void* f, double* W,
                          hipStream_t st);
hipError_t launch_moments_adj(int D, long long plane, long long ncell, bool fp32, const double* Wbar, void* lam,
                              hipStream_t st);
int totals_nparts(long long ncell);
hipError_t launch_totals(int D, long long plane, long long ncell, bool fp32, double e_off, const void* f,
                         double* partials, double* out, hipStream_t st);
hipError_t launch_copy_probe(const void* src, void* dst, size_t bytes, int mode, hipStream_t st);
size_t read_probe_out_bytes(size_t bytes);
hipError_t launch_unpad(int D, long long plane, long long ncell, bool fp32, double e_off, const void* f, void* out,
                        hipStream_t st);

// adjoint (vlbm_adjoint.hip)
struct AdjScratch {
    void* aux;                   // per-cell intermediate fields (adjoint_aux_elems, 8 bytes each)
    double* partials;            // per-block partial sums of the normaliser adjoint (4 per block)
    double* qmax;                // grid maxima of |Q_alpha,k| (4)
    unsigned long long* argmax;  // first maximiser of each |Q_alpha,k| (4)
    double* rec;                 // fused D2Q4 adjoint: per-wavefront records (adjoint_march_records x 12)
};
size_t adjoint_partials_count(const KParams& p);
size_t adjoint_aux_elems(const KParams& p);
hipError_t launch_adjoint_step(const KParams& p, int prec, const void* f_n, const double* norms_n,
                               const void* lam_np1, void* lam_n, const AdjScratch& sc, hipStream_t st);
// fused single-march adjoint of a D2Q4 step (vlbm_adjoint_march.hip): the same
// map as launch_adjoint_step, in one pass over f, lam_np1 and lam_n plus a
// one-workgroup fix-up of the normaliser term
int adjoint_march_records(const KParams& p);
bool adjoint_march_supported(const KParams& p);
hipError_t launch_adjoint_march(const KParams& p, int prec, const void* f_n, const double* norms_n,
                                const void* lam_np1, void* lam_n, double* rec, hipStream_t st);
// records of the march that the allocation-free adjoint step's static scratch
// holds (12 doubles each: 384 KiB), and that scratch's device address on
// `device` (looked up on the first call for that device)
constexpr int kStaticMarchRecords = 4096;
hipError_t adjm_static_scratch(int device, double** out);
hipError_t launch_init_adjoint(const KParams& p, int prec, const double* W0, long long ncell, const void* lam0,
                               double* W0bar, hipStream_t st);

}  // namespace vlbm
