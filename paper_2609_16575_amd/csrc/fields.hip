// fields.hip -- Yee FDTD kernels for gfx950 (Sec. 2.3 of KEMPIC-3D).
//
// One thread per grid point, x fastest across a wavefront so that every
// component load and store is coalesced; a thread updates all three
// components at its point.  Periodic neighbours wrap; on a walled (absorbing
// or PEC) axis the validity rules below keep every neighbour inside the
// stored array.
//
// Bytes per cell (FP32): Faraday reads E, B (24) and writes B, Bbar (24) and
// zeroes J (12); Ampere reads E, B, J (36) and writes E (12).
#include <cmath>
#include <utility>

#include "internal.hpp"

namespace empic {

namespace {

struct Pt {
    int idx[3];
    long long p;
    long long st[3];  // strides
};

__device__ inline bool make_point(const GridP &g, Pt &q) {
    q.idx[0] = blockIdx.x * blockDim.x + threadIdx.x;
    q.idx[1] = blockIdx.y * blockDim.y + threadIdx.y;
    q.idx[2] = blockIdx.z;
    if (q.idx[0] >= g.ext[0] || q.idx[1] >= g.ext[1]) return false;
    q.st[0] = 1;
    q.st[1] = g.ext[0];
    q.st[2] = (long long)g.ext[0] * g.ext[1];
    q.p = q.idx[0] + q.st[1] * q.idx[1] + q.st[2] * q.idx[2];
    return true;
}

// offset of the +1 / -1 neighbour along axis a (periodic wrap)
__device__ inline long long up(const GridP &g, const Pt &q, int a) {
    return (g.bc[a] == EMPIC_BC_PERIODIC && q.idx[a] == g.n[a] - 1) ? -(long long)(g.n[a] - 1) * q.st[a]
                                                                   : q.st[a];
}
__device__ inline long long dn(const GridP &g, const Pt &q, int a) {
    return (g.bc[a] == EMPIC_BC_PERIODIC && q.idx[a] == 0) ? (long long)(g.n[a] - 1) * q.st[a]
                                                           : -q.st[a];
}

// A component half-staggered along walled axis a has n values: entry n is padding.
__device__ inline bool valid_B(const GridP &g, const Pt &q, int c) {
    for (int a = 0; a < 3; ++a)
        if (g.bc[a] != EMPIC_BC_PERIODIC && a != c && q.idx[a] == g.n[a]) return false;
    return true;
}
// E_c updated by Ampere: valid and not tangential on a walled face (those
// belong to the Mur or PEC condition).
__device__ inline bool ampere_E(const GridP &g, const Pt &q, int c) {
    for (int a = 0; a < 3; ++a) {
        if (g.bc[a] == EMPIC_BC_PERIODIC) continue;
        if (a == c && q.idx[a] == g.n[a]) return false;
        if (a != c && (q.idx[a] == 0 || q.idx[a] == g.n[a])) return false;
    }
    return true;
}

template <typename T>
__global__ void k_faraday(GridP g, const T *__restrict__ Ex, const T *__restrict__ Ey,
                          const T *__restrict__ Ez, T *__restrict__ Bx, T *__restrict__ By,
                          T *__restrict__ Bz, T *__restrict__ Bbx, T *__restrict__ Bby,
                          T *__restrict__ Bbz, T *__restrict__ Jx, T *__restrict__ Jy,
                          T *__restrict__ Jz, unsigned long long *__restrict__ Jfx,
                          unsigned long long *__restrict__ Jfy, unsigned long long *__restrict__ Jfz,
                          unsigned *__restrict__ fb_reset, int write_B) {
    Pt q;
    if (!make_point(g, q)) return;
    const long long p = q.p;
    if (fb_reset && p == 0) {  // the out-of-window counts of the coming push
        fb_reset[0] = 0u;
        fb_reset[1] = 0u;
        fb_reset[2] = 0u;
    }
    if (Jx) {
        Jx[p] = T(0);
        Jy[p] = T(0);
        Jz[p] = T(0);
    }
    if (Jfx) {  // the fixed-point current of the FP32 path
        Jfx[p] = 0ull;
        Jfy[p] = 0ull;
        Jfz[p] = 0ull;
    }
    // evaluated in FP64 and rounded once per stored value (see k_ampere)
    const double dt = g.dt;
    const double ix = g.inv_d[0], iy = g.inv_d[1], iz = g.inv_d[2];
    // B^{n+1/2} = B^{n-1/2} - dt curl E^n (forward differences); Bbar = average
    if (valid_B(g, q, 0)) {
        const double curl = ((double)Ez[p + up(g, q, 1)] - (double)Ez[p]) * iy -
                            ((double)Ey[p + up(g, q, 2)] - (double)Ey[p]) * iz;
        const double old = (double)Bx[p], nw = old - dt * curl;
        if (write_B) Bx[p] = (T)nw;
        Bbx[p] = (T)(0.5 * (old + nw));
    } else {
        Bbx[p] = T(0);
    }
    if (valid_B(g, q, 1)) {
        const double curl = ((double)Ex[p + up(g, q, 2)] - (double)Ex[p]) * iz -
                            ((double)Ez[p + up(g, q, 0)] - (double)Ez[p]) * ix;
        const double old = (double)By[p], nw = old - dt * curl;
        if (write_B) By[p] = (T)nw;
        Bby[p] = (T)(0.5 * (old + nw));
    } else {
        Bby[p] = T(0);
    }
    if (valid_B(g, q, 2)) {
        const double curl = ((double)Ey[p + up(g, q, 0)] - (double)Ey[p]) * ix -
                            ((double)Ex[p + up(g, q, 1)] - (double)Ex[p]) * iy;
        const double old = (double)Bz[p], nw = old - dt * curl;
        if (write_B) Bz[p] = (T)nw;
        Bbz[p] = (T)(0.5 * (old + nw));
    } else {
        Bbz[p] = T(0);
    }
}

// J in units of 1/jscale (int64, exact sums of the deposit) -> T, one rounding
template <typename T>
__device__ __forceinline__ T j_from_fixed(long long x, double jinv) {
    return (T)((double)x * jinv);
}

// With Jf (the FP32 path): J is first formed from the fixed-point sums and
// written out, at every point, then used.
template <typename T>
__global__ void k_ampere(GridP g, T *__restrict__ Ex, T *__restrict__ Ey, T *__restrict__ Ez,
                         const T *__restrict__ Bx, const T *__restrict__ By,
                         const T *__restrict__ Bz, T *__restrict__ Jx, T *__restrict__ Jy,
                         T *__restrict__ Jz, const long long *__restrict__ Jfx,
                         const long long *__restrict__ Jfy, const long long *__restrict__ Jfz,
                         double jinv) {
    Pt q;
    if (!make_point(g, q)) return;
    const long long p = q.p;
    // Evaluated in FP64 and rounded once per stored value: in FP32 the
    // rounding of J, of curl - J and of the two-part update add up coherently
    // on a quiet plasma (every cell of a wave front rounds alike).  The kernel
    // is bound by memory, and gfx950 issues FP64 at the FP32 (unpacked) rate.
    double jx, jy, jz;
    if (Jfx) {
        jx = (double)Jfx[p] * jinv;
        jy = (double)Jfy[p] * jinv;
        jz = (double)Jfz[p] * jinv;
        Jx[p] = (T)jx;
        Jy[p] = (T)jy;
        Jz[p] = (T)jz;
    } else {
        jx = (double)Jx[p];
        jy = (double)Jy[p];
        jz = (double)Jz[p];
    }
    const double dt = g.dt;
    const double ix = g.inv_d[0], iy = g.inv_d[1], iz = g.inv_d[2];
    // E^{n+1} = E^n + dt curl B^{n+1/2} - dt J^{n+1/2} (backward differences)
    if (ampere_E(g, q, 0)) {
        const double curl = ((double)Bz[p] - (double)Bz[p + dn(g, q, 1)]) * iy -
                            ((double)By[p] - (double)By[p + dn(g, q, 2)]) * iz;
        Ex[p] = (T)((double)Ex[p] + dt * (curl - jx));
    }
    if (ampere_E(g, q, 1)) {
        const double curl = ((double)Bx[p] - (double)Bx[p + dn(g, q, 2)]) * iz -
                            ((double)Bz[p] - (double)Bz[p + dn(g, q, 0)]) * ix;
        Ey[p] = (T)((double)Ey[p] + dt * (curl - jy));
    }
    if (ampere_E(g, q, 2)) {
        const double curl = ((double)By[p] - (double)By[p + dn(g, q, 0)]) * ix -
                            ((double)Bx[p] - (double)Bx[p + dn(g, q, 1)]) * iy;
        Ez[p] = (T)((double)Ez[p] + dt * (curl - jz));
    }
}

// Six arrays of n floats copied in one launch (the fields of a state)
struct Copy6 {
    const float *src[6];
    float *dst[6];
};

__global__ void k_copy6(Copy6 c, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
#pragma unroll
        for (int a = 0; a < 6; ++a) c.dst[a][i] = c.src[a][i];
    }
}

// J = the fixed-point sums converted (before the current filter)
__global__ void k_j_from_fixed(GridP g, float *__restrict__ Jx, float *__restrict__ Jy,
                               float *__restrict__ Jz, const long long *__restrict__ Jfx,
                               const long long *__restrict__ Jfy,
                               const long long *__restrict__ Jfz, double jinv) {
    Pt q;
    if (!make_point(g, q)) return;
    const long long p = q.p;
    Jx[p] = j_from_fixed<float>(Jfx[p], jinv);
    Jy[p] = j_from_fixed<float>(Jfy[p], jinv);
    Jz[p] = j_from_fixed<float>(Jfz[p], jinv);
}

// ---------------------------------------------------------------------------
// First-order Mur faces (READING of the boundary module: tangential E on the
// faces of an absorbing axis).  planes[a][c'][q][point], q = index 0, 1, n-1,
// n along a, point = i_b1 + ext[b1] * i_b2 over the other two axes.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_mur_save(GridP g, int a, T *Ex, T *Ey, T *Ez, T *planes, long long pstride) {
    const int b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;
    const long long npt = (long long)g.ext[b1] * g.ext[b2];
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t >= npt) return;
    const int i1 = (int)(t % g.ext[b1]), i2 = (int)(t / g.ext[b1]);
    T *E[3] = {Ex, Ey, Ez};
    long long st[3] = {1, g.ext[0], (long long)g.ext[0] * g.ext[1]};
    const int qidx[4] = {0, 1, g.n[a] - 1, g.n[a]};
    int ci = 0;
    for (int c = 0; c < 3; ++c) {
        if (c == a) continue;
        for (int qq = 0; qq < 4; ++qq) {
            const long long p = st[b1] * i1 + st[b2] * i2 + st[a] * qidx[qq];
            planes[(((long long)a * 2 + ci) * 4 + qq) * pstride + t] = E[c][p];
        }
        ++ci;
    }
}

template <typename T>
__global__ void k_mur_apply(GridP g, int a, T *Ex, T *Ey, T *Ez, const T *planes,
                            long long pstride) {
    const int b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;
    const long long npt = (long long)g.ext[b1] * g.ext[b2];
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t >= npt) return;
    const int i1 = (int)(t % g.ext[b1]), i2 = (int)(t / g.ext[b1]);
    T *E[3] = {Ex, Ey, Ez};
    long long st[3] = {1, g.ext[0], (long long)g.ext[0] * g.ext[1]};
    const T coef = (T)((g.dt - g.d[a]) / (g.dt + g.d[a]));
    int ci = 0;
    for (int c = 0; c < 3; ++c) {
        if (c == a) continue;
        const T *pl = planes + ((long long)a * 2 + ci) * 4 * pstride;
        const long long base = st[b1] * i1 + st[b2] * i2;
        // face at index 0: E_0^{n+1} = E_1^n + coef (E_1^{n+1} - E_0^n)
        E[c][base] = pl[1 * pstride + t] + coef * (E[c][base + st[a]] - pl[0 * pstride + t]);
        // face at index n: E_n^{n+1} = E_{n-1}^n + coef (E_{n-1}^{n+1} - E_n^n)
        const long long pn = base + st[a] * g.n[a];
        E[c][pn] = pl[2 * pstride + t] + coef * (E[c][pn - st[a]] - pl[3 * pstride + t]);
        ++ci;
    }
}

// Soft current sheet J_y on x-node plane i_s (READING of the external-source
// module), applied to E after Ampere: E_y -= dt J_sheet(t^{n+1/2}).
template <typename T>
__global__ void k_laser(GridP g, T *Ey, empic_laser_desc L, double t_half) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    const int cy = g.n[1];                                              // E_y half along y
    const int cz = g.bc[2] != EMPIC_BC_PERIODIC ? g.n[2] + 1 : g.n[2];  // node along z
    if (j >= cy || k >= cz) return;
    if (g.bc[0] != EMPIC_BC_PERIODIC && (L.i_s == 0 || L.i_s == g.n[0])) return;
    if (g.bc[2] != EMPIC_BC_PERIODIC && (k == 0 || k == g.n[2])) return;
    const double y = ((double)j + 0.5) * g.d[1];
    const double z = (double)k * g.d[2];
    const double ry2 = L.slab ? 0.0 : (y - L.yc) * (y - L.yc);
    const double r2 = ry2 + (z - L.zc) * (z - L.zc);
    const double tt = t_half - L.t0;
    const double einc = L.a0 * exp(-r2 / (L.w0 * L.w0)) *
                        exp(-2.0 * log(2.0) * tt * tt / (L.tau * L.tau)) * sin(L.omega0 * tt);
    const double Jy = -2.0 * einc / g.d[0];
    const long long p = L.i_s + (long long)g.ext[0] * (j + (long long)g.ext[1] * k);
    Ey[p] -= (T)(g.dt * Jy);
}

// Perfectly conducting walls: tangential E on both faces of axis a set to
// zero (after Ampere, which leaves them alone).  One thread per face point.
template <typename T>
__global__ void k_pec(GridP g, int a, T *Ex, T *Ey, T *Ez) {
    const int b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t >= (long long)g.ext[b1] * g.ext[b2]) return;
    int idx[3];
    idx[b1] = (int)(t % g.ext[b1]);
    idx[b2] = (int)(t / g.ext[b1]);
    const long long st[3] = {1, g.ext[0], (long long)g.ext[0] * g.ext[1]};
    T *E[3] = {Ex, Ey, Ez};
    for (int side = 0; side < 2; ++side) {
        idx[a] = side ? g.n[a] : 0;
        const long long p = idx[0] + st[1] * idx[1] + st[2] * idx[2];
        E[b1][p] = T(0);
        E[b2][p] = T(0);
    }
}

// Waveguide port (hard source): E_comp = e0 sin(pi s/L) g(t) sin(omega t) on
// the node plane of axis P.axis, s the component's position along
// P.prof_axis, with the amplitude factor computed on the host in FP64.
template <typename T>
__global__ void k_port(GridP g, T *Ec, empic_port_desc P, double amp) {
    const int a = P.axis, c = P.comp, pa = P.prof_axis;
    const int b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;
    // E_c holds ext values along a transverse axis, n where it is
    // half-staggered on a walled axis (entry n is padding)
    const int n1 = (g.bc[b1] == EMPIC_BC_PERIODIC || c != b1) ? g.ext[b1] : g.n[b1];
    const int n2 = (g.bc[b2] == EMPIC_BC_PERIODIC || c != b2) ? g.ext[b2] : g.n[b2];
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t >= (long long)n1 * n2) return;
    int idx[3];
    idx[a] = P.plane;
    idx[b1] = (int)(t % n1);
    idx[b2] = (int)(t / n1);
    const double s = ((double)idx[pa] + (c == pa ? 0.5 : 0.0)) * g.d[pa];
    const double L = g.n[pa] * g.d[pa];
    const long long p = idx[0] + (long long)g.ext[0] * (idx[1] + (long long)g.ext[1] * idx[2]);
    const double sw = fmin(s, L - s);  // sin(pi s/L) from the nearer wall: exactly 0 on both
    Ec[p] = (T)(amp * sin(3.14159265358979323846 * sw / L));
}

// One pass of the current filter along axis ax: dst = a src[-1] + b src + a src[+1]
// per component on its own sub-grid; periodic axes wrap, on a walled axis
// values beyond the stored ones (entry n of a half-cell component is
// padding) count as zero.
template <typename T>
__global__ void k_filter_pass(GridP g, int ax, const T *__restrict__ s0, const T *__restrict__ s1,
                              const T *__restrict__ s2, T *__restrict__ d0, T *__restrict__ d1,
                              T *__restrict__ d2, T a, T b) {
    Pt q;
    if (!make_point(g, q)) return;
    const T *src[3] = {s0, s1, s2};
    T *dst[3] = {d0, d1, d2};
    const long long p = q.p;
    const bool per = g.bc[ax] == EMPIC_BC_PERIODIC;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        // stored values of component c along every axis
        bool valid = true;
        for (int a2 = 0; a2 < 3; ++a2)
            if (g.bc[a2] != EMPIC_BC_PERIODIC && a2 == c && q.idx[a2] == g.n[a2]) valid = false;
        if (!valid) {
            dst[c][p] = T(0);
            continue;
        }
        const int L = (!per && ax == c) ? g.n[ax] : g.ext[ax];
        const int i = q.idx[ax];
        T lo = T(0), hi = T(0);
        if (i > 0) lo = src[c][p - q.st[ax]];
        else if (per) lo = src[c][p + (long long)(L - 1) * q.st[ax]];
        if (i < L - 1) hi = src[c][p + q.st[ax]];
        else if (per) hi = src[c][p - (long long)(L - 1) * q.st[ax]];
        dst[c][p] = a * lo + b * src[c][p] + a * hi;
    }
}

// Moving window: every value moves `cells` planes toward index 0 along axis
// ax; values that would come from beyond the stored ones are zero (the new
// front planes); padding entries stay zero.  isB selects the B staggering.
template <typename T>
__global__ void k_window_shift(GridP g, int ax, int cells, int isB, const T *__restrict__ s0,
                               const T *__restrict__ s1, const T *__restrict__ s2,
                               T *__restrict__ d0, T *__restrict__ d1, T *__restrict__ d2) {
    Pt q;
    if (!make_point(g, q)) return;
    const T *src[3] = {s0, s1, s2};
    T *dst[3] = {d0, d1, d2};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        bool pad = false;
        for (int b = 0; b < 3; ++b) {
            const bool half = isB ? (b != c) : (b == c);
            if (g.bc[b] != EMPIC_BC_PERIODIC && half && q.idx[b] == g.n[b]) pad = true;
        }
        const bool half_ax = isB ? (ax != c) : (ax == c);
        const int L = (g.bc[ax] != EMPIC_BC_PERIODIC && half_ax) ? g.n[ax] : g.ext[ax];
        const int m = q.idx[ax];
        dst[c][q.p] = (!pad && m + cells < L) ? src[c][q.p + (long long)cells * q.st[ax]] : T(0);
    }
}

// FP64 partial sums of |E|^2 and B^{n-1/2}.B^{n+1/2} (B^{n+1/2} formed on the fly)
template <typename T>
__global__ void k_field_energy(GridP g, const T *__restrict__ Ex, const T *__restrict__ Ey,
                               const T *__restrict__ Ez, const T *__restrict__ Bx,
                               const T *__restrict__ By, const T *__restrict__ Bz,
                               double *partials) {
    __shared__ double sm[16];
    double ee = 0.0, bb = 0.0;
    const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    const T dt = (T)g.dt;
    const T ix = (T)g.inv_d[0], iy = (T)g.inv_d[1], iz = (T)g.inv_d[2];
    for (int k = blockIdx.z; k < g.ext[2]; k += gridDim.z)
        for (int j = blockIdx.y * blockDim.y + threadIdx.y; j < g.ext[1]; j += gridDim.y * blockDim.y)
            for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < g.ext[0];
                 i += gridDim.x * blockDim.x) {
                Pt q;
                q.idx[0] = i;
                q.idx[1] = j;
                q.idx[2] = k;
                q.st[0] = 1;
                q.st[1] = g.ext[0];
                q.st[2] = (long long)g.ext[0] * g.ext[1];
                const long long p = i + q.st[1] * j + q.st[2] * k;
                ee += (double)Ex[p] * Ex[p] + (double)Ey[p] * Ey[p] + (double)Ez[p] * Ez[p];
                if (valid_B(g, q, 0)) {
                    const T c = (Ez[p + up(g, q, 1)] - Ez[p]) * iy - (Ey[p + up(g, q, 2)] - Ey[p]) * iz;
                    bb += (double)Bx[p] * (double)(Bx[p] - dt * c);
                }
                if (valid_B(g, q, 1)) {
                    const T c = (Ex[p + up(g, q, 2)] - Ex[p]) * iz - (Ez[p + up(g, q, 0)] - Ez[p]) * ix;
                    bb += (double)By[p] * (double)(By[p] - dt * c);
                }
                if (valid_B(g, q, 2)) {
                    const T c = (Ey[p + up(g, q, 0)] - Ey[p]) * ix - (Ex[p + up(g, q, 1)] - Ex[p]) * iy;
                    bb += (double)Bz[p] * (double)(Bz[p] - dt * c);
                }
            }
    const double se = block_reduce<false>(ee, sm);
    const double sb = block_reduce<false>(bb, sm);
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        partials[Q_EE * PSTRIDE + bid] = se;
        partials[Q_BB * PSTRIDE + bid] = sb;
    }
}

dim3 point_grid(const GridP &g) { return dim3((g.ext[0] + 63) / 64, (g.ext[1] + 3) / 4, g.ext[2]); }

}  // namespace

// Grid of the (64, 4) point reductions: every kernel strides over all three
// axes, and gx * gy * gz <= PSTRIDE keeps one partial slot per workgroup.
dim3 reduction_grid(const GridP &g) {
    int gx = (g.ext[0] + 63) / 64;
    if (gx > 64) gx = 64;
    int gy = (g.ext[1] + 3) / 4;
    if (gy > PSTRIDE / gx) gy = PSTRIDE / gx;
    int gz = PSTRIDE / (gx * gy);
    if (gz > g.ext[2]) gz = g.ext[2];
    if (gz < 1) gz = 1;
    return dim3(gx, gy, gz);
}

template <typename T>
void launch_faraday(const GridP &g, T *const E[3], T *const B[3], T *const Bbar[3],
                    T *const J[3], unsigned long long *const Jf[3], bool write_B, hipStream_t s,
                    unsigned *fb_reset) {
    hipLaunchKernelGGL(k_faraday<T>, point_grid(g), dim3(64, 4), 0, s, g, E[0], E[1], E[2], B[0],
                       B[1], B[2], Bbar[0], Bbar[1], Bbar[2], J ? J[0] : nullptr,
                       J ? J[1] : nullptr, J ? J[2] : nullptr, Jf ? Jf[0] : nullptr,
                       Jf ? Jf[1] : nullptr, Jf ? Jf[2] : nullptr, fb_reset, write_B ? 1 : 0);
}

template <typename T>
void launch_ampere(const GridP &g, T *const E[3], T *const B[3], T *const J[3],
                   const long long *const Jf[3], double jinv, hipStream_t s) {
    hipLaunchKernelGGL(k_ampere<T>, point_grid(g), dim3(64, 4), 0, s, g, E[0], E[1], E[2], B[0],
                       B[1], B[2], J[0], J[1], J[2], Jf ? Jf[0] : nullptr, Jf ? Jf[1] : nullptr,
                       Jf ? Jf[2] : nullptr, jinv);
}

void launch_copy6(const float *const src[6], float *const dst[6], long long n, hipStream_t s) {
    Copy6 c;
    for (int a = 0; a < 6; ++a) {
        c.src[a] = src[a];
        c.dst[a] = dst[a];
    }
    long long nb = (n + 255) / 256;
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_copy6, dim3((unsigned)nb), dim3(256), 0, s, c, n);
}

void launch_j_from_fixed(const GridP &g, float *const J[3], const long long *const Jf[3],
                         double jinv, hipStream_t s) {
    hipLaunchKernelGGL(k_j_from_fixed, point_grid(g), dim3(64, 4), 0, s, g, J[0], J[1], J[2],
                       Jf[0], Jf[1], Jf[2], jinv);
}

template <typename T>
void launch_mur_save(const GridP &g, T *const E[3], T *planes, long long pstride, hipStream_t s) {
    for (int a = 0; a < 3; ++a) {
        if (g.bc[a] != EMPIC_BC_ABSORBING) continue;
        const int b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;
        const long long npt = (long long)g.ext[b1] * g.ext[b2];
        hipLaunchKernelGGL(k_mur_save<T>, dim3((unsigned)((npt + 255) / 256)), dim3(256), 0, s, g,
                           a, E[0], E[1], E[2], planes, pstride);
    }
}

template <typename T>
void launch_mur_apply(const GridP &g, T *const E[3], const T *planes, long long pstride,
                      hipStream_t s) {
    for (int a = 0; a < 3; ++a) {
        if (g.bc[a] != EMPIC_BC_ABSORBING) continue;
        const int b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;
        const long long npt = (long long)g.ext[b1] * g.ext[b2];
        hipLaunchKernelGGL(k_mur_apply<T>, dim3((unsigned)((npt + 255) / 256)), dim3(256), 0, s,
                           g, a, E[0], E[1], E[2], planes, pstride);
    }
}

template <typename T>
void launch_filter(const GridP &g, T *const F[3], T *const tmp[3], int passes, int compensate,
                   hipStream_t s) {
    T *cur[3] = {F[0], F[1], F[2]}, *oth[3] = {tmp[0], tmp[1], tmp[2]};
    for (int ax = 0; ax < 3; ++ax)
        for (int k = 0; k < passes + (compensate ? 1 : 0); ++k) {
            const bool comp = k == passes;
            const T a = comp ? T(-0.25) : T(0.25), b = comp ? T(1.5) : T(0.5);
            hipLaunchKernelGGL(k_filter_pass<T>, point_grid(g), dim3(64, 4), 0, s, g, ax, cur[0],
                               cur[1], cur[2], oth[0], oth[1], oth[2], a, b);
            for (int c = 0; c < 3; ++c) std::swap(cur[c], oth[c]);
        }
    if (cur[0] != F[0])
        for (int c = 0; c < 3; ++c)
            (void)hipMemcpyAsync(F[c], cur[c], (size_t)g.V * sizeof(T), hipMemcpyDeviceToDevice, s);
}

template <typename T>
void launch_window_shift(const GridP &g, T *const F[3], T *const tmp[3], int ax, int cells,
                         bool isB, hipStream_t s) {
    hipLaunchKernelGGL(k_window_shift<T>, point_grid(g), dim3(64, 4), 0, s, g, ax, cells,
                       isB ? 1 : 0, F[0], F[1], F[2], tmp[0], tmp[1], tmp[2]);
    for (int c = 0; c < 3; ++c)
        (void)hipMemcpyAsync(F[c], tmp[c], (size_t)g.V * sizeof(T), hipMemcpyDeviceToDevice, s);
}

template <typename T>
void launch_pec(const GridP &g, T *const E[3], hipStream_t s) {
    for (int a = 0; a < 3; ++a) {
        if (g.bc[a] != EMPIC_BC_PEC) continue;
        const int b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;
        const long long npt = (long long)g.ext[b1] * g.ext[b2];
        hipLaunchKernelGGL(k_pec<T>, dim3((unsigned)((npt + 255) / 256)), dim3(256), 0, s, g, a,
                           E[0], E[1], E[2]);
    }
}

template <typename T>
void launch_port(const GridP &g, T *const E[3], const empic_port_desc &P, double t,
                 hipStream_t s) {
    const double amp = P.e0 * (1.0 - std::exp(-t / P.tau)) * std::sin(P.omega * t);
    const int a = P.axis;
    const int b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;
    const long long npt = (long long)g.ext[b1] * g.ext[b2];
    hipLaunchKernelGGL(k_port<T>, dim3((unsigned)((npt + 255) / 256)), dim3(256), 0, s, g,
                       E[P.comp], P, amp);
}

template <typename T>
void launch_laser(const GridP &g, T *const E[3], const empic_laser_desc &L, double t_half,
                  hipStream_t s) {
    const int cz = g.bc[2] != EMPIC_BC_PERIODIC ? g.n[2] + 1 : g.n[2];
    hipLaunchKernelGGL(k_laser<T>, dim3((g.n[1] + 63) / 64, cz), dim3(64), 0, s, g, E[1], L,
                       t_half);
}

template <typename T>
void launch_field_energy(const GridP &g, T *const E[3], T *const B[3], double *partials,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_field_energy<T>, reduction_grid(g), dim3(64, 4), 0, s, g, E[0], E[1],
                       E[2], B[0], B[1], B[2], partials);
}

#define EMPIC_INST(T)                                                                          \
    template void launch_faraday<T>(const GridP &, T *const[3], T *const[3], T *const[3],      \
                                    T *const[3], unsigned long long *const[3], bool,           \
                                    hipStream_t, unsigned *);                                  \
    template void launch_ampere<T>(const GridP &, T *const[3], T *const[3], T *const[3],       \
                                   const long long *const[3], double, hipStream_t);            \
    template void launch_mur_save<T>(const GridP &, T *const[3], T *, long long, hipStream_t); \
    template void launch_mur_apply<T>(const GridP &, T *const[3], const T *, long long,        \
                                      hipStream_t);                                            \
    template void launch_laser<T>(const GridP &, T *const[3], const empic_laser_desc &, double, \
                                  hipStream_t);                                                \
    template void launch_pec<T>(const GridP &, T *const[3], hipStream_t);                      \
    template void launch_window_shift<T>(const GridP &, T *const[3], T *const[3], int, int,    \
                                         bool, hipStream_t);                                   \
    template void launch_filter<T>(const GridP &, T *const[3], T *const[3], int, int,          \
                                   hipStream_t);                                               \
    template void launch_port<T>(const GridP &, T *const[3], const empic_port_desc &, double,  \
                                 hipStream_t);                                                 \
    template void launch_field_energy<T>(const GridP &, T *const[3], T *const[3], double *,    \
                                         hipStream_t);
EMPIC_INST(float)
EMPIC_INST(double)
#undef EMPIC_INST

}  // namespace empic
