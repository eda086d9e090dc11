// Auxiliary kernels of the VLBM library: control-block reset, initial state
// (reductions of W0 and the equilibrium populations), conserved totals,
// moments and layout copies.
#include "vlbm_aux.hpp"

#include <algorithm>

namespace vlbm {

__global__ void k_reset_ctl(double* ring, unsigned long long* stop_at, int* err)
{
    const int i = threadIdx.x;
    for (int j = i; j < 3 * kSlot; j += blockDim.x) ring[j] = 0.0;
    if (i == 0) {
        *stop_at = ~0ull;
        *err = 0;
    }
}

__global__ void k_reset_stop(unsigned long long* stop_at, int* err)
{
    if (threadIdx.x == 0) {
        *stop_at = ~0ull;
        *err = 0;
    }
}

__global__ void k_zero(double* p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// primitive closure of one FP64 cell of W (component stride `cs`)
template <int EOS>
__device__ __forceinline__ void prim_cell(const Gas<double>& g, int D, const double* W, long long cs, double& rho,
                                          double* u, double& e, double& P, double& E)
{
    rho = W[0];
    const double irho = 1.0 / rho;
    double ke = 0.0;
    for (int a = 0; a < D; ++a) {
        u[a] = W[(1 + a) * cs] * irho;
        ke += u[a] * u[a];
    }
    E = W[(D + 1) * cs];
    e = E * irho - 0.5 * ke;
    P = eos_pressure<double, EOS>(g, rho, e);
}

// Reductions of the initial state: s_max (Eq. 36) and M_k (Eq. 30) into the
// `copies` copies at red_out (stride doubles apart); admissibility bits into err.
template <int EOS>
__global__ void __launch_bounds__(256) k_init_reduce(KParams p, const double* __restrict__ W, long long ncell,
                                                     double* red_out, int copies, int stride, int* err)
{
    const Gas<double> g = make_gas<double>(p);
    const int D = p.dim;
    double smax = 0.0, M[4] = {0, 0, 0, 0};
    int bits = 0;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < ncell;
         c += (long long)gridDim.x * blockDim.x) {
        double rho, u[2] = {0, 0}, e, P, E;
        prim_cell<EOS>(g, D, W + c, ncell, rho, u, e, P, E);
        const double cs2 = eos_cs2<double, EOS>(g, rho, e);
        bits |= eos_check<double, EOS>(g, rho, e, cs2);
        const double cs = sqrt(cs2 > 0.0 ? cs2 : 0.0);
        for (int a = 0; a < D; ++a) {
            smax = fmax(smax, fabs(u[a]) + cs);
            const double m = W[(1 + a) * ncell + c];
            M[0] = fmax(M[0], fabs(m));
            for (int b = 0; b < D; ++b) M[1 + b] = fmax(M[1 + b], fabs(m * u[b] + (a == b ? P : 0.0)));
            M[D + 1] = fmax(M[D + 1], fabs((E + P) * u[a]));
        }
    }
    KStep s{};
    s.red_out = red_out;
    s.red_copies = copies;
    s.red_stride = stride;
    s.err = err;
    block_publish<4>(s, smax, M, D + 2, bits);
}

// f = f^eq(W0; c0) (Eq. 20); c0 = s_max/CFL from the reductions of W0 (or
// c_fixed).  Block 0 writes the clock (t = 0, c0) to clock0.  The energy component is stored in
// the shifted gauge: W_E - e_off W_rho and Q_E - e_off Q_rho (linear in W, Q).
template <typename T, int EOS>
__global__ void k_init_eq(KParams p, const double* __restrict__ W, long long ncell, double* clock0,
                          const double* red0, int copies, int stride, int frozen, T* __restrict__ f)
{
    double smax = red0[0];
    for (int i = 1; i < copies; ++i) smax = fmax(smax, red0[i * stride]);
    const double c0 = frozen ? p.c_fixed : smax / p.cfl;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        clock0[0] = 0.0;
        clock0[1] = c0;
    }
    const Gas<double> g = make_gas<double>(p);
    const int D = p.dim, NK = D + 2;
    const double inv2c = 0.5 / c0, w = 1.0 / (2.0 * D);
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < ncell;
         c += (long long)gridDim.x * blockDim.x) {
        double rho, u[2] = {0, 0}, e, P, E;
        prim_cell<EOS>(g, D, W + c, ncell, rho, u, e, P, E);
        for (int a = 0; a < D; ++a) {
            const double m = W[(1 + a) * ncell + c];
            double q[4], wv[4];
            q[0] = m;
            for (int b = 0; b < D; ++b) q[1 + b] = m * u[b] + (a == b ? P : 0.0);
            q[D + 1] = (E + P) * u[a] - p.e_off * m;
            for (int k = 0; k <= D; ++k) wv[k] = W[k * ncell + c];
            wv[D + 1] = E - p.e_off * rho;
            for (int k = 0; k < NK; ++k) {
                const double wk = w * wv[k];
                f[((2 * a) * NK + k) * p.plane + c] = (T)(wk + q[k] * inv2c);
                f[((2 * a + 1) * NK + k) * p.plane + c] = (T)(wk - q[k] * inv2c);
            }
        }
    }
}

// W = sum_i f_i in FP64, (NK, ncell), back in the physical energy gauge
template <typename T>
__global__ void k_moments(int D, long long plane, long long ncell, double e_off, const T* __restrict__ f,
                          double* __restrict__ W)
{
    const int NK = D + 2, Q = 2 * D;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < ncell;
         c += (long long)gridDim.x * blockDim.x) {
        double rho = 0.0;
        for (int k = 0; k < NK; ++k) {
            double acc = 0.0;
            for (int i = 0; i < Q; ++i) acc += (double)f[(i * NK + k) * plane + c];
            if (k == 0) rho = acc;
            if (k == NK - 1) acc += e_off * rho;
            W[k * ncell + c] = acc;
        }
    }
}

// lam_i = Wbar for every direction i (adjoint of k_moments)
template <typename T>
__global__ void k_moments_adj(int D, long long plane, long long ncell, const double* __restrict__ Wbar,
                              T* __restrict__ lam)
{
    const int NK = D + 2, Q = 2 * D;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < ncell;
         c += (long long)gridDim.x * blockDim.x)
        for (int k = 0; k < NK; ++k) {
            const T v = (T)Wbar[k * ncell + c];
            for (int i = 0; i < Q; ++i) lam[(i * NK + k) * plane + c] = v;
        }
}

// Deterministic FP64 totals: each block sums a fixed set of cells with a fixed
// tree; a second single-block pass sums the block partials in order.
constexpr int kTotBlock = 256;

template <typename T>
__global__ void __launch_bounds__(kTotBlock) k_totals_partial(int D, long long plane, long long ncell,
                                                               const T* __restrict__ f, double* partials)
{
    __shared__ double sh[4][kTotBlock];
    const int NK = D + 2, Q = 2 * D;
    double acc[4] = {0, 0, 0, 0};
    for (long long c = blockIdx.x * (long long)kTotBlock + threadIdx.x; c < ncell;
         c += (long long)gridDim.x * kTotBlock)
        for (int k = 0; k < NK; ++k) {
            double w = 0.0;
            for (int i = 0; i < Q; ++i) w += (double)f[(i * NK + k) * plane + c];
            acc[k] += w;
        }
    for (int k = 0; k < NK; ++k) sh[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = kTotBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < NK; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < NK; ++k) partials[blockIdx.x * 4 + k] = sh[k][0];
}

__global__ void __launch_bounds__(kTotBlock) k_totals_final(int NK, int nparts, double e_off, const double* partials,
                                                             double* out)
{
    __shared__ double sh[4][kTotBlock];
    double acc[4] = {0, 0, 0, 0};
    for (int b = threadIdx.x; b < nparts; b += kTotBlock)
        for (int k = 0; k < NK; ++k) acc[k] += partials[b * 4 + k];
    for (int k = 0; k < NK; ++k) sh[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = kTotBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < NK; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int k = 0; k < NK; ++k) out[k] = sh[k][0];
        out[NK - 1] += e_off * sh[0][0];
    }
}

// populations without plane padding, physical energy gauge:
// out[i][k][cell] = f[(i NK + k) plane + cell] (+ e_off f_i,rho for the energy component)
template <typename T>
__global__ void k_unpad(int D, long long plane, long long ncell, double e_off, const T* __restrict__ f,
                        T* __restrict__ out)
{
    const int NK = D + 2, Q = 2 * D;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < ncell;
         c += (long long)gridDim.x * blockDim.x)
        for (int i = 0; i < Q; ++i)
            for (int k = 0; k < NK; ++k) {
                const int j = i * NK + k;
                T v = f[j * plane + c];
                if (k == NK - 1 && e_off != 0.0) v = (T)((double)v + e_off * (double)f[i * NK * plane + c]);
                out[j * ncell + c] = v;
            }
}

// ------------------------------------------------------------------ launchers

static unsigned grid_for(long long n, int block)
{
    long long g = (n + block - 1) / block;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (unsigned)g;
}

hipError_t launch_reset_ctl(double* ring, unsigned long long* stop_at, int* err, hipStream_t st)
{
    hipLaunchKernelGGL(k_reset_ctl, dim3(1), dim3(256), 0, st, ring, stop_at, err);
    return hipGetLastError();
}

hipError_t launch_reset_stop(unsigned long long* stop_at, int* err, hipStream_t st)
{
    hipLaunchKernelGGL(k_reset_stop, dim3(1), dim3(64), 0, st, stop_at, err);
    return hipGetLastError();
}

hipError_t launch_zero(double* p, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero, dim3((n + 63) / 64), dim3(64), 0, st, p, n);
    return hipGetLastError();
}

// the reduction kernels stride over the cells with few blocks: one set of
// same-address atomics per block
static unsigned reduce_grid(long long ncell) { return std::min(grid_for(ncell, 256), 1024u); }

hipError_t launch_init(const KParams& p, bool fp32, const double* W, long long ncell, double* clock0, double* red0,
                       int copies, int stride, int* err, int frozen, void* f, hipStream_t st)
{
    const unsigned grid = grid_for(ncell, 256);
    if (p.eos == 0)
        hipLaunchKernelGGL(k_init_reduce<0>, dim3(reduce_grid(ncell)), dim3(256), 0, st, p, W, ncell, red0, copies,
                           stride, err);
    else
        hipLaunchKernelGGL(k_init_reduce<1>, dim3(reduce_grid(ncell)), dim3(256), 0, st, p, W, ncell, red0, copies,
                           stride, err);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
#define VLBM_INIT(T, E)                                                                                   \
    hipLaunchKernelGGL((k_init_eq<T, E>), dim3(grid), dim3(256), 0, st, p, W, ncell, clock0, (const double*)red0, \
                       copies, stride, frozen, (T*)f)
    if (fp32) {
        if (p.eos == 0) VLBM_INIT(float, 0); else VLBM_INIT(float, 1);
    } else {
        if (p.eos == 0) VLBM_INIT(double, 0); else VLBM_INIT(double, 1);
    }
#undef VLBM_INIT
    return hipGetLastError();
}

hipError_t launch_moments(int D, long long plane, long long ncell, bool fp32, double e_off, const void* f, double* W,
                          hipStream_t st)
{
    const unsigned grid = grid_for(ncell, 256);
    if (fp32)
        hipLaunchKernelGGL(k_moments<float>, dim3(grid), dim3(256), 0, st, D, plane, ncell, e_off, (const float*)f,
                           W);
    else
        hipLaunchKernelGGL(k_moments<double>, dim3(grid), dim3(256), 0, st, D, plane, ncell, e_off,
                           (const double*)f, W);
    return hipGetLastError();
}

hipError_t launch_moments_adj(int D, long long plane, long long ncell, bool fp32, const double* Wbar, void* lam,
                              hipStream_t st)
{
    const unsigned grid = grid_for(ncell, 256);
    if (fp32)
        hipLaunchKernelGGL(k_moments_adj<float>, dim3(grid), dim3(256), 0, st, D, plane, ncell, Wbar, (float*)lam);
    else
        hipLaunchKernelGGL(k_moments_adj<double>, dim3(grid), dim3(256), 0, st, D, plane, ncell, Wbar, (double*)lam);
    return hipGetLastError();
}

int totals_nparts(long long ncell)
{
    return (int)grid_for(ncell, kTotBlock) > 1024 ? 1024 : (int)grid_for(ncell, kTotBlock);
}

hipError_t launch_totals(int D, long long plane, long long ncell, bool fp32, double e_off, const void* f,
                         double* partials, double* out, hipStream_t st)
{
    const int nparts = totals_nparts(ncell);
    if (fp32)
        hipLaunchKernelGGL(k_totals_partial<float>, dim3(nparts), dim3(kTotBlock), 0, st, D, plane, ncell,
                           (const float*)f, partials);
    else
        hipLaunchKernelGGL(k_totals_partial<double>, dim3(nparts), dim3(kTotBlock), 0, st, D, plane, ncell,
                           (const double*)f, partials);
    hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(kTotBlock), 0, st, D + 2, nparts, e_off, partials, out);
    return hipGetLastError();
}

hipError_t launch_unpad(int D, long long plane, long long ncell, bool fp32, double e_off, const void* f, void* out,
                        hipStream_t st)
{
    const unsigned grid = grid_for(ncell, 256);
    if (fp32)
        hipLaunchKernelGGL(k_unpad<float>, dim3(grid), dim3(256), 0, st, D, plane, ncell, e_off, (const float*)f,
                           (float*)out);
    else
        hipLaunchKernelGGL(k_unpad<double>, dim3(grid), dim3(256), 0, st, D, plane, ncell, e_off, (const double*)f,
                           (double*)out);
    return hipGetLastError();
}

// Measurement aids.  Copy: grid-stride, 16 bytes per lane with non-temporal
// loads and stores (the fastest plain copy measured on MI355X: 65536
// workgroups of 512 threads, 5.7 TB/s; four independent loads in flight per
// lane measured slower, 5.2 TB/s).
__global__ void __launch_bounds__(512) k_copy_probe(const double2* __restrict__ a, double2* __restrict__ b, size_t n)
{
    typedef double d2v __attribute__((ext_vector_type(2)));
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const d2v v = __builtin_nontemporal_load((const d2v*)(a + i));
        __builtin_nontemporal_store(v, (d2v*)(b + i));
    }
}

// Read-only stream: four independent 16-byte non-temporal loads in flight per
// lane, folded into an XOR per workgroup (the read rate of the memory system
// without a write stream: 6.2 TB/s measured on MI355X with 8192 workgroups of
// 256 threads).  Workgroup b writes its 16-byte XOR to b[blockIdx].
constexpr int kReadBlocks = 8192, kReadThreads = 256;
__global__ void __launch_bounds__(kReadThreads) k_read_probe(const ulonglong2* __restrict__ a, ulonglong2* __restrict__ b,
                                                             size_t n)
{
    typedef unsigned long long u2v __attribute__((ext_vector_type(2)));
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    u2v acc = {0ull, 0ull};
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += 4 * stride) {
        u2v v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const size_t j = i + k * stride;
            v[k] = j < n ? __builtin_nontemporal_load((const u2v*)(a + j)) : u2v{0ull, 0ull};
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) acc ^= v[k];
    }
    __shared__ unsigned long long sh[2][kReadThreads];
    sh[0][threadIdx.x] = acc.x;
    sh[1][threadIdx.x] = acc.y;
    __syncthreads();
    for (int o = kReadThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sh[0][threadIdx.x] ^= sh[0][threadIdx.x + o];
            sh[1][threadIdx.x] ^= sh[1][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) b[blockIdx.x] = make_ulonglong2(sh[0][0], sh[1][0]);
}

size_t read_probe_out_bytes(size_t bytes)
{
    const size_t n = bytes / 16;
    return std::min<size_t>(kReadBlocks, (n + kReadThreads - 1) / kReadThreads) * 16;
}

hipError_t launch_copy_probe(const void* src, void* dst, size_t bytes, int mode, hipStream_t st)
{
    const size_t n = bytes / 16;
    if (n == 0) return hipSuccess;
    if (mode == 1) {
        const size_t blocks = read_probe_out_bytes(bytes) / 16;
        hipLaunchKernelGGL(k_read_probe, dim3((unsigned)blocks), dim3(kReadThreads), 0, st, (const ulonglong2*)src,
                           (ulonglong2*)dst, n);
        return hipGetLastError();
    }
    const size_t blocks = std::min<size_t>(65536, (n + 511) / 512);
    hipLaunchKernelGGL(k_copy_probe, dim3((unsigned)blocks), dim3(512), 0, st, (const double2*)src, (double2*)dst, n);
    return hipGetLastError();
}

}  // namespace vlbm
