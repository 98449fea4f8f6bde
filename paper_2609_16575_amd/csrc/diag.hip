// diag.hip -- FP64 diagnostics reductions (Sec. 3.3 of KEMPIC-3D: energy,
// Gauss's law, discrete continuity).  Every reduction writes one FP64
// partial per workgroup into its slot; k_final_reduce then sums (or takes the
// max of) each slot in a fixed order, so results do not depend on timing.
#include "internal.hpp"

namespace empic {

namespace {

// backward-difference divergence of an E-located field at node (i,j,k)
template <typename T>
__device__ inline double div_node(const GridP &g, const T *Fx, const T *Fy, const T *Fz, int i,
                                  int j, int k) {
    const long long sy = g.ext[0], sz = (long long)g.ext[0] * g.ext[1];
    const long long p = i + sy * j + sz * k;
    const int idx[3] = {i, j, k};
    const T *F[3] = {Fx, Fy, Fz};
    const long long st[3] = {1, sy, sz};
    double s = 0.0;
    for (int a = 0; a < 3; ++a) {
        double fm;
        if (idx[a] == 0) {
            fm = g.bc[a] == EMPIC_BC_PERIODIC ? (double)F[a][p + (long long)(g.n[a] - 1) * st[a]]
                                              : 0.0;
        } else {
            fm = (double)F[a][p - st[a]];
        }
        s += ((double)F[a][p] - fm) * g.inv_d[a];
    }
    return s;
}

template <typename T>
__global__ void k_gauss(GridP g, const T *Ex, const T *Ey, const T *Ez, const double *rho,
                        double rho_bg, double *partials) {
    __shared__ double sm[16];
    const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    double mx = 0.0, s2 = 0.0;
    for (int k = blockIdx.z; k < g.ext[2]; k += gridDim.z)
        for (int j = blockIdx.y * blockDim.y + threadIdx.y; j < g.ext[1]; j += gridDim.y * blockDim.y)
            for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < g.ext[0];
                 i += gridDim.x * blockDim.x) {
                const long long p = i + (long long)g.ext[0] * (j + (long long)g.ext[1] * k);
                const double r = div_node(g, Ex, Ey, Ez, i, j, k) - rho[p] - rho_bg;
                mx = fmax(mx, fabs(r));
                s2 += r * r;
            }
    const double a = block_reduce<true>(mx, sm);
    const double b = block_reduce<false>(s2, sm);
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        partials[Q_GMAX * PSTRIDE + bid] = a;
        partials[Q_G2 * PSTRIDE + bid] = b;
    }
}

template <typename T>
__global__ void k_continuity(GridP g, const T *Jx, const T *Jy, const T *Jz, const double *rho_now,
                             const double *rho_prev, double *partials) {
    __shared__ double sm[16];
    const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    double mx = 0.0, rm = 0.0;
    for (int k = blockIdx.z; k < g.ext[2]; k += gridDim.z)
        for (int j = blockIdx.y * blockDim.y + threadIdx.y; j < g.ext[1]; j += gridDim.y * blockDim.y)
            for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < g.ext[0];
                 i += gridDim.x * blockDim.x) {
                const long long p = i + (long long)g.ext[0] * (j + (long long)g.ext[1] * k);
                // rho^{n+1} - rho^n + dt div J^{n+1/2}, on every node but those
                // of the faces of a walled axis: a particle that leaves through
                // the wall takes its charge out of the grid there
                const int idx[3] = {i, j, k};
                bool face = false;
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    face = face || (g.bc[a] != EMPIC_BC_PERIODIC && (idx[a] == 0 || idx[a] == g.n[a]));
                const double r =
                    face ? 0.0 : rho_now[p] - rho_prev[p] + g.dt * div_node(g, Jx, Jy, Jz, i, j, k);
                mx = fmax(mx, fabs(r));
                rm = fmax(rm, fabs(rho_now[p]));
            }
    const double a = block_reduce<true>(mx, sm);
    const double b = block_reduce<true>(rm, sm);
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        partials[Q_CMAX * PSTRIDE + bid] = a;
        partials[Q_RMAX * PSTRIDE + bid] = b;
    }
}

__global__ void k_final_reduce(const double *partials, double *result) {
    __shared__ double sm[16];
    const int q = blockIdx.x;
    const bool mx = slot_is_max(q);
    double v = 0.0;
    for (int i = threadIdx.x; i < PSTRIDE; i += blockDim.x) {
        const double x = partials[(long long)q * PSTRIDE + i];
        v = mx ? fmax(v, x) : v + x;
    }
    const double r = mx ? block_reduce<true>(v, sm) : block_reduce<false>(v, sm);
    if (threadIdx.x == 0) result[q] = r;
}

// grid-stride FP64 products, one partial per workgroup, then a fixed-order sum
__global__ void k_dot_f64(const float *a, const float *b, long long n, double *partials) {
    __shared__ double sm[16];
    double v = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        v += (double)a[i] * (double)b[i];
    const double r = block_reduce<false>(v, sm);
    if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

__global__ void k_sum_partials(const double *partials, int n, double *out) {
    __shared__ double sm[16];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v += partials[i];
    const double r = block_reduce<false>(v, sm);
    if (threadIdx.x == 0) *out = r;
}

__global__ void k_absmax_f64(const double *x, long long n, double *out) {
    __shared__ double sm[16];
    double m = 0.0;
    for (long long i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, fabs(x[i]));
    const double r = block_reduce<true>(m, sm);
    if (threadIdx.x == 0) *out = r;
}

__global__ void k_zero_f64(double *p, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

}  // namespace

void launch_zero_f64(double *p, long long n, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_f64, dim3(1024), dim3(256), 0, s, p, n);
}

template <typename T>
void launch_gauss(const GridP &g, T *const E[3], const double *rho, double rho_bg,
                  double *partials, hipStream_t s) {
    hipLaunchKernelGGL(k_gauss<T>, reduction_grid(g), dim3(64, 4), 0, s, g, E[0], E[1], E[2], rho,
                       rho_bg, partials);
}

template <typename T>
void launch_continuity(const GridP &g, T *const J[3], const double *rho_now,
                       const double *rho_prev, double *partials, hipStream_t s) {
    hipLaunchKernelGGL(k_continuity<T>, reduction_grid(g), dim3(64, 4), 0, s, g, J[0], J[1], J[2],
                       rho_now, rho_prev, partials);
}

void launch_absmax_f64(const double *x, long long n, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_absmax_f64, dim3(1), dim3(1024), 0, s, x, n, out);
}

void launch_dot_f64(const float *a, const float *b, long long n, double *partials,
                    double *result, hipStream_t s) {
    hipLaunchKernelGGL(k_dot_f64, dim3(RED_BLOCKS), dim3(256), 0, s, a, b, n, partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, partials, RED_BLOCKS, result);
}

void launch_final_reduce(const double *partials, double *result, hipStream_t s) {
    hipLaunchKernelGGL(k_final_reduce, dim3(NQ), dim3(256), 0, s, partials, result);
}

template void launch_gauss<float>(const GridP &, float *const[3], const double *, double,
                                  double *, hipStream_t);
template void launch_gauss<double>(const GridP &, double *const[3], const double *, double,
                                   double *, hipStream_t);
template void launch_continuity<float>(const GridP &, float *const[3], const double *,
                                       const double *, double *, hipStream_t);
template void launch_continuity<double>(const GridP &, double *const[3], const double *,
                                        const double *, double *, hipStream_t);

}  // namespace empic
