// push_f64.hip -- plain FP64 particle step for gfx950: global FP64 positions,
// unsorted, one thread per particle, fields gathered straight from global
// memory and the ZigZag current scattered with global FP64 atomics
// (hardware global_atomic_add_f64).  Same operations, in the same order, as
// the paper's cycle (Sec. 2.4-2.5): staggered CIC gather of E^n and of the
// centred B^n, relativistic Boris push, x += dt u/gamma, ZigZag deposit.
//
// Bytes per particle: 48 read + 48 written (+ 8 with a per-particle weight).
#include "internal.hpp"

namespace empic {

namespace {

// linear index of (i,j,k); periodic axes wrap, absorbing axes give -1 outside
__device__ inline long long at64(const GridP &g, long long i, long long j, long long k) {
    long long p[3] = {i, j, k};
    for (int a = 0; a < 3; ++a) {
        if (g.bc[a] == EMPIC_BC_PERIODIC) {
            const long long n = g.n[a];
            p[a] = ((p[a] % n) + n) % n;
        } else if (p[a] < 0 || p[a] >= g.ext[a]) {
            return -1;
        }
    }
    return p[0] + (long long)g.ext[0] * (p[1] + (long long)g.ext[1] * p[2]);
}

// staggered CIC interpolation of one component (stag[a] = 1: half-cell)
__device__ inline double gather_one(const GridP &g, const double *__restrict__ F,
                                    const int sx, const int sy, const int sz, const double xi[3]) {
    const int st[3] = {sx, sy, sz};
    long long i0[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        const double t = xi[a] - 0.5 * st[a];
        const double fl = floor(t);
        i0[a] = (long long)fl;
        f[a] = t - fl;
    }
    double s = 0.0;
    for (int oz = 0; oz < 2; ++oz)
        for (int oy = 0; oy < 2; ++oy)
            for (int ox = 0; ox < 2; ++ox) {
                const long long ip = at64(g, i0[0] + ox, i0[1] + oy, i0[2] + oz);
                if (ip < 0) continue;
                const double w = (ox ? f[0] : 1.0 - f[0]) * (oy ? f[1] : 1.0 - f[1]) *
                                 (oz ? f[2] : 1.0 - f[2]);
                s += w * F[ip];
            }
    return s;
}

struct F64Fields {
    const double *E[3];
    const double *Bb[3];
    double *J[3];
};

__device__ inline void gather_all(const GridP &g, const F64Fields &f, const double xi[3],
                                  double Ep[3], double Bp[3]) {
    Ep[0] = gather_one(g, f.E[0], 1, 0, 0, xi);
    Ep[1] = gather_one(g, f.E[1], 0, 1, 0, xi);
    Ep[2] = gather_one(g, f.E[2], 0, 0, 1, xi);
    Bp[0] = gather_one(g, f.Bb[0], 0, 1, 1, xi);
    Bp[1] = gather_one(g, f.Bb[1], 1, 0, 1, xi);
    Bp[2] = gather_one(g, f.Bb[2], 1, 1, 0, xi);
}

// relativistic Boris (standard t/s rotation), r = q dt / (2 m)
__device__ inline void boris(double u[3], const double E[3], const double B[3], double r) {
    double um[3], t[3], s[3], up[3], upl[3];
    for (int a = 0; a < 3; ++a) um[a] = u[a] + r * E[a];
    const double gm = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
    for (int a = 0; a < 3; ++a) t[a] = r * B[a] / gm;
    const double tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    for (int a = 0; a < 3; ++a) s[a] = 2.0 * t[a] / (1.0 + tt);
    up[0] = um[0] + (um[1] * t[2] - um[2] * t[1]);
    up[1] = um[1] + (um[2] * t[0] - um[0] * t[2]);
    up[2] = um[2] + (um[0] * t[1] - um[1] * t[0]);
    upl[0] = um[0] + (up[1] * s[2] - up[2] * s[1]);
    upl[1] = um[1] + (up[2] * s[0] - up[0] * s[2]);
    upl[2] = um[2] + (up[0] * s[1] - up[1] * s[0]);
    for (int a = 0; a < 3; ++a) u[a] = upl[a] + r * E[a];
}

__device__ inline void add_edge(const GridP &g, double *J, int c, long long i, long long j,
                                long long k, double v) {
    const long long ip = at64(g, i, j, k);
    if (ip < 0) return;
    const long long p[3] = {i, j, k};
    if (g.bc[c] != EMPIC_BC_PERIODIC && p[c] >= g.n[c]) return;  // half-cell padding
    atomicAdd(J + ip, v);
}

// one straight segment inside one cell: line integral of the bilinear weights
__device__ inline void deposit_segment(const GridP &g, const F64Fields &f, const long long cell[3],
                                       const double s[3], const double e[3], double qsp) {
    const double dV = g.d[0] * g.d[1] * g.d[2];
    double dxi[3], W[3];
    for (int a = 0; a < 3; ++a) {
        dxi[a] = e[a] - s[a];
        W[a] = 0.5 * (s[a] + e[a]) - (double)cell[a];
    }
    for (int c = 0; c < 3; ++c) {
        const int b1 = (c + 1) % 3, b2 = (c + 2) % 3;
        const double amp = qsp * dxi[c] * g.d[c] / (g.dt * dV);
        const double cross = dxi[b1] * dxi[b2] / 12.0;
        for (int o2 = 0; o2 < 2; ++o2)
            for (int o1 = 0; o1 < 2; ++o1) {
                const double w1 = o1 ? W[b1] : 1.0 - W[b1];
                const double w2 = o2 ? W[b2] : 1.0 - W[b2];
                const double sg = (o1 == o2) ? 1.0 : -1.0;
                long long p[3] = {cell[0], cell[1], cell[2]};
                p[b1] += o1;
                p[b2] += o2;
                add_edge(g, f.J[c], c, p[0], p[1], p[2], amp * (w1 * w2 + sg * cross));
            }
    }
}

// ZigZag: relay point per axis, two segments each inside one cell
__device__ inline void zigzag(const GridP &g, const F64Fields &f, const double xi1[3],
                              const double xi2[3], double qsp) {
    long long c1[3], c2[3];
    double xr[3];
    for (int a = 0; a < 3; ++a) {
        const long long i1 = (long long)floor(xi1[a]);
        const long long i2 = (long long)floor(xi2[a]);
        const double lo = (double)((i1 < i2 ? i1 : i2) + 1);
        const double hi = (double)(i1 > i2 ? i1 : i2);
        const double mid = 0.5 * (xi1[a] + xi2[a]);
        xr[a] = fmin(lo, fmax(hi, mid));
        c1[a] = i1;
        c2[a] = i2;
    }
    deposit_segment(g, f, c1, xi1, xr, qsp);
    deposit_segment(g, f, c2, xr, xi2, qsp);
}

template <bool DRY>
__global__ __launch_bounds__(256) void k_push_f64(GridP g, F64Fields f, SpeciesP sp,
                                                  long long count, uint32_t *fault,
                                                  double *partial) {
    __shared__ double sm[16];
    const double r = sp.q * g.dt / (2.0 * sp.m);
    double *X = (double *)sp.pos[0], *Y = (double *)sp.pos[1], *Z = (double *)sp.pos[2];
    double *UX = (double *)sp.u[0], *UY = (double *)sp.u[1], *UZ = (double *)sp.u[2];
    const double *W = (const double *)sp.w;
    double L[3];
    for (int a = 0; a < 3; ++a) L[a] = g.n[a] * g.d[a];
    double ksum = 0.0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < count; p += stride) {
        double pos[3] = {X[p], Y[p], Z[p]};
        if (isnan(pos[0])) continue;  // removed by an absorbing face
        const double wp = (sp.per_particle_w && W) ? W[p] : sp.w_species;
        double xi1[3], Ep[3], Bp[3];
        for (int a = 0; a < 3; ++a) xi1[a] = pos[a] / g.d[a];
        gather_all(g, f, xi1, Ep, Bp);
        double un[3] = {UX[p], UY[p], UZ[p]};
        boris(un, Ep, Bp, r);
        const double uu = un[0] * un[0] + un[1] * un[1] + un[2] * un[2];
        const double gm = sqrt(1.0 + uu);
        if (DRY) {
            ksum += wp * sp.m * uu / (gm + 1.0);
            continue;
        }
        if (!isfinite(gm)) atomicOr(fault, (uint32_t)EMPIC_FAULT_NONFINITE);
        double xi2[3];
        for (int a = 0; a < 3; ++a) {
            xi2[a] = xi1[a] + g.dt * un[a] / (gm * g.d[a]);
            if (fabs(xi2[a] - xi1[a]) >= 1.0) atomicOr(fault, (uint32_t)EMPIC_FAULT_FAST);
        }
        zigzag(g, f, xi1, xi2, sp.q * wp);
        bool dead = false;
        for (int a = 0; a < 3; ++a) {
            double x = pos[a] + g.dt * un[a] / gm;
            if (g.bc[a] == EMPIC_BC_PERIODIC) {
                if (x >= L[a]) x -= L[a];
                if (x < 0.0) {
                    x += L[a];
                    if (x >= L[a]) x = 0.0;
                }
            } else if (x < 0.0 || x >= L[a]) {
                dead = true;
            }
            pos[a] = x;
        }
        X[p] = dead ? __builtin_nan("") : pos[0];
        Y[p] = pos[1];
        Z[p] = pos[2];
        UX[p] = un[0];
        UY[p] = un[1];
        UZ[p] = un[2];
    }
    if (DRY) {
        const double s = block_reduce<false>(ksum, sm);
        if (threadIdx.x == 0) partial[blockIdx.x] = s;
    }
}

__global__ void k_kinetic_f64(SpeciesP sp, long long count, double *partial) {
    __shared__ double sm[16];
    const double *UX = (const double *)sp.u[0], *UY = (const double *)sp.u[1],
                 *UZ = (const double *)sp.u[2], *X = (const double *)sp.pos[0];
    const double *W = (const double *)sp.w;
    double ksum = 0.0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < count; p += stride) {
        if (isnan(X[p])) continue;
        const double uu = UX[p] * UX[p] + UY[p] * UY[p] + UZ[p] * UZ[p];
        const double wp = (sp.per_particle_w && W) ? W[p] : sp.w_species;
        ksum += wp * sp.m * uu / (sqrt(1.0 + uu) + 1.0);
    }
    const double s = block_reduce<false>(ksum, sm);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// CIC charge density at nodes, rho += (q w / dV) prod_a w_a
__global__ void k_rho_f64(GridP g, SpeciesP sp, long long count, double *rho) {
    const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (p >= count) return;
    const double *X = (const double *)sp.pos[0], *Y = (const double *)sp.pos[1],
                 *Z = (const double *)sp.pos[2];
    const double *W = (const double *)sp.w;
    if (isnan(X[p])) return;
    const double dV = g.d[0] * g.d[1] * g.d[2];
    const double qsp = sp.q * ((sp.per_particle_w && W) ? W[p] : sp.w_species);
    const double pos[3] = {X[p], Y[p], Z[p]};
    long long i0[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        const double t = pos[a] / g.d[a];
        const double fl = floor(t);
        i0[a] = (long long)fl;
        f[a] = t - fl;
    }
    for (int oz = 0; oz < 2; ++oz)
        for (int oy = 0; oy < 2; ++oy)
            for (int ox = 0; ox < 2; ++ox) {
                const long long ip = at64(g, i0[0] + ox, i0[1] + oy, i0[2] + oz);
                if (ip < 0) continue;
                const double wt = (ox ? f[0] : 1.0 - f[0]) * (oy ? f[1] : 1.0 - f[1]) *
                                  (oz ? f[2] : 1.0 - f[2]);
                atomicAdd(rho + ip, qsp / dV * wt);
            }
}

__global__ void k_load_f64(GridP g, SpeciesP sp, long long count, const double *pos,
                           const double *u, const double *w, const int32_t *ids, uint32_t *fault) {
    const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (p >= count) return;
    for (int a = 0; a < 3; ++a) {
        const double x = pos[3 * p + a];
        if (!(x >= 0.0 && x < g.n[a] * g.d[a])) atomicOr(fault, (uint32_t)EMPIC_FAULT_CELL);
        ((double *)sp.pos[a])[p] = x;
        ((double *)sp.u[a])[p] = u[3 * p + a];
    }
    if (sp.id) sp.id[p] = ids ? ids[p] : (int32_t)p;
    if (sp.w && w) ((double *)sp.w)[p] = w[p];
}

__global__ void k_store_f64(SpeciesP sp, long long count, double *pos, double *u, int32_t *ids) {
    const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (p >= count) return;
    const bool dead = isnan(((const double *)sp.pos[0])[p]);
    for (int a = 0; a < 3; ++a) {
        pos[3 * p + a] = ((const double *)sp.pos[a])[p];
        u[3 * p + a] = ((const double *)sp.u[a])[p];
    }
    if (ids) ids[p] = dead ? -1 : (sp.id ? sp.id[p] : (int32_t)p);
}

inline unsigned nblk(long long n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

void launch_push_f64(const GridP &g, double *const E[3], double *const Bbar[3],
                     double *const J[3], const SpeciesP &sp, long long count, uint32_t *fault,
                     hipStream_t s) {
    if (count <= 0) return;
    F64Fields f{{E[0], E[1], E[2]}, {Bbar[0], Bbar[1], Bbar[2]}, {J[0], J[1], J[2]}};
    hipLaunchKernelGGL(k_push_f64<false>, dim3(nblk(count, 256)), dim3(256), 0, s, g, f, sp,
                       count, fault, nullptr);
}

void launch_dry_push_f64(const GridP &g, double *const E[3], double *const Bbar[3],
                         const SpeciesP &sp, long long count, double *partial_slot,
                         uint32_t *fault, hipStream_t s) {
    F64Fields f{{E[0], E[1], E[2]}, {Bbar[0], Bbar[1], Bbar[2]}, {nullptr, nullptr, nullptr}};
    hipLaunchKernelGGL(k_push_f64<true>, dim3(RED_BLOCKS), dim3(256), 0, s, g, f, sp, count,
                       fault, partial_slot);
}

void launch_kinetic_f64(const SpeciesP &sp, long long count, double *partial_slot,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_kinetic_f64, dim3(RED_BLOCKS), dim3(256), 0, s, sp, count, partial_slot);
}

void launch_rho_f64(const GridP &g, const SpeciesP &sp, long long count, double *rho,
                    hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_rho_f64, dim3(nblk(count, 256)), dim3(256), 0, s, g, sp, count, rho);
}

void launch_load_f64(const GridP &g, const SpeciesP &sp, long long count, const double *pos,
                     const double *u, const double *w, const int32_t *ids, uint32_t *fault,
                     hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_load_f64, dim3(nblk(count, 256)), dim3(256), 0, s, g, sp, count, pos, u,
                       w, ids, fault);
}

void launch_store_f64(const SpeciesP &sp, long long count, double *pos, double *u, int32_t *ids,
                      hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_store_f64, dim3(nblk(count, 256)), dim3(256), 0, s, sp, count, pos, u,
                       ids);
}

}  // namespace empic
