// adjoint.hip -- discrete adjoint (vector-Jacobian product) of one FP32 PIC
// step on a periodic grid, for the differentiable runs.
//
// The forward step from state (E, B, x, u) is
//   B' = B - dt Cf E,  Bbar = (B + B')/2,  E_p = G_E(x) E,  B_p = G_B(x) Bbar,
//   u' = Boris(u, E_p, B_p),  x' = x + dt u'/gamma',  J = Z(x, x'),
//   E' = E + dt Cb B' - dt J,
// with Cf / Cb the forward / backward difference curls of the Yee scheme
// (Sec. 2.3; on a periodic grid Cf^T = Cb).  Given the adjoints of
// (E', B', x', u') the kernels below return those of (E, B, x, u):
//   k_adj_particles: per particle, recompute the forward in FP32 from the saved
//     state, then reverse it: the ZigZag deposit adjoint gathers -dt lam_E' on
//     the edges the particle touched (Sec. 2.5), the position and Boris adjoints
//     follow, and the gather adjoint scatters lam_Ep, lam_Bp onto the Yee
//     sub-grids (float atomics) while its derivative in x adds to lam_x;
//   k_adj_bprime: lam_B'_t = lam_B' + dt Cf lam_E' + lam_Bbar / 2,
//                 lam_B = lam_B'_t + lam_Bbar / 2;
//   k_adj_e:      lam_E = lam_E' + lam_Egather - dt Cb lam_B'_t.
// Derivatives are taken inside the current piece of each piecewise map (the
// relay-point branch and the interpolation corners are frozen).  Position
// adjoints are per unit length (global coordinates).
#include "internal.hpp"

namespace empic {

namespace {

__device__ __forceinline__ float rcpf_(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ int pwrap(int x, int n) {
    int m = x % n;
    return m < 0 ? m + n : m;
}
__device__ __forceinline__ long long gidx(const GridP &g, int i, int j, int k) {
    return pwrap(i, g.n[0]) + (long long)g.ext[0] * (pwrap(j, g.n[1]) + (long long)g.ext[1] * pwrap(k, g.n[2]));
}

// trilinear value of F at corner (i0,j0,k0) + (fx,fy,fz), and its gradient in f
__device__ void tri_val_grad(const GridP &g, const float *F, int i0, int j0, int k0, float fx,
                             float fy, float fz, float &val, float grad[3]) {
    float v[8];
#pragma unroll
    for (int o = 0; o < 8; ++o) v[o] = F[gidx(g, i0 + (o & 1), j0 + ((o >> 1) & 1), k0 + (o >> 2))];
    const float gx = 1.f - fx, gy = 1.f - fy, gz = 1.f - fz;
    val = gz * (gy * (gx * v[0] + fx * v[1]) + fy * (gx * v[2] + fx * v[3])) +
          fz * (gy * (gx * v[4] + fx * v[5]) + fy * (gx * v[6] + fx * v[7]));
    grad[0] = gz * (gy * (v[1] - v[0]) + fy * (v[3] - v[2])) +
              fz * (gy * (v[5] - v[4]) + fy * (v[7] - v[6]));
    grad[1] = gz * (gx * (v[2] - v[0]) + fx * (v[3] - v[1])) +
              fz * (gx * (v[6] - v[4]) + fx * (v[7] - v[5]));
    grad[2] = gy * (gx * (v[4] - v[0]) + fx * (v[5] - v[1])) +
              fy * (gx * (v[6] - v[2]) + fx * (v[7] - v[3]));
}

__device__ void tri_scatter(const GridP &g, float *lF, int i0, int j0, int k0, float fx, float fy,
                            float fz, float l) {
    if (l == 0.f) return;
    const float gx = 1.f - fx, gy = 1.f - fy, gz = 1.f - fz;
    const float w[8] = {gx * gy * gz, fx * gy * gz, gx * fy * gz, fx * fy * gz,
                        gx * gy * fz, fx * gy * fz, gx * fy * fz, fx * fy * fz};
#pragma unroll
    for (int o = 0; o < 8; ++o)
        atomicAdd(lF + gidx(g, i0 + (o & 1), j0 + ((o >> 1) & 1), k0 + (o >> 2)), l * w[o]);
}

__device__ __forceinline__ void half_idx(float o, int c, int &h, float &f) {
    if (o < 0.5f) {
        h = c - 1;
        f = o + 0.5f;
    } else {
        h = c;
        f = o - 0.5f;
    }
}

// adjoint of one straight segment inside cell (ci,cj,ck) (global cell index),
// given per axis its midpoint W relative to that cell and its displacement D:
// accumulates d/ds and d/de (cell units) of sum_edges lJ . J_segment, with
// D = e - s and W = (s + e)/2 - cell.
__device__ void segment_vjp(const GridP &g, const float *const lJ[3], int ci, int cj, int ck,
                            const float W[3], const float D[3], const float ampc[3], float ls[3],
                            float le[3]) {
    float lD[3] = {0.f, 0.f, 0.f}, lW[3] = {0.f, 0.f, 0.f};
    const int cell[3] = {ci, cj, ck};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int b1 = (c + 1) % 3, b2 = (c + 2) % 3;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int o1 = q & 1, o2 = q >> 1;
            int p[3] = {cell[0], cell[1], cell[2]};
            p[b1] += o1;
            p[b2] += o2;
            const float lam = lJ[c][gidx(g, p[0], p[1], p[2])];
            const float w1 = o1 ? W[b1] : 1.f - W[b1];
            const float w2 = o2 ? W[b2] : 1.f - W[b2];
            const float sg = (o1 == o2) ? 1.f : -1.f;
            const float weight = w1 * w2 + sg * D[b1] * D[b2] * (1.f / 12.f);
            lD[c] += lam * ampc[c] * weight;
            const float k = lam * ampc[c] * D[c];
            lW[b1] += k * (o1 ? 1.f : -1.f) * w2;
            lW[b2] += k * w1 * (o2 ? 1.f : -1.f);
            lD[b1] += k * sg * D[b2] * (1.f / 12.f);
            lD[b2] += k * sg * D[b1] * (1.f / 12.f);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        ls[a] += -lD[a] + 0.5f * lW[a];
        le[a] += lD[a] + 0.5f * lW[a];
    }
}

struct AdjArgs {
    GridP g;
    const float *E[3];
    const float *Bb[3];
    const float *lJsrc[3];  // adjoint of E^{n+1}; lam_J = -dt * it
    float *lEg[3];          // accumulated adjoint of E^n through the gather
    float *lBb[3];          // accumulated adjoint of Bbar
    float dtd[3];
    float inv_d[3];
    float dt;
};

struct AdjSpecies {
    const uint32_t *cell;
    const float *pos[3];
    const float *u[3];
    const float *w;
    float *lx[3];
    float *lu[3];
    const int32_t *count;
    float r;
    float qc[3];
};

__global__ __launch_bounds__(256) void k_adj_particles(AdjArgs A, AdjSpecies S) {
    const GridP &g = A.g;
    const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (p >= *S.count) return;
    const uint32_t c = S.cell[p];
    if (c == DEAD) return;
    const int ci = cell_i(c), cj = cell_j(c), ck = cell_k(c);
    const float o[3] = {S.pos[0][p], S.pos[1][p], S.pos[2][p]};
    const float u0[3] = {S.u[0][p], S.u[1][p], S.u[2][p]};
    const float wq = S.w ? S.w[p] : 1.f;
    // ---- forward recompute: gather (value and d/d offset) ----
    int hx, hy, hz;
    float fx, fy, fz;
    half_idx(o[0], ci, hx, fx);
    half_idx(o[1], cj, hy, fy);
    half_idx(o[2], ck, hz, fz);
    const int idx[6][3] = {{hx, cj, ck}, {ci, hy, ck}, {ci, cj, hz},
                           {ci, hy, hz}, {hx, cj, hz}, {hx, hy, ck}};
    const float fr[6][3] = {{fx, o[1], o[2]}, {o[0], fy, o[2]}, {o[0], o[1], fz},
                            {o[0], fy, fz}, {fx, o[1], fz}, {fx, fy, o[2]}};
    float F6[6], G6[6][3];
#pragma unroll
    for (int q = 0; q < 6; ++q)
        tri_val_grad(g, q < 3 ? A.E[q] : A.Bb[q - 3], idx[q][0], idx[q][1], idx[q][2], fr[q][0],
                     fr[q][1], fr[q][2], F6[q], G6[q]);
    const float Ep[3] = {F6[0], F6[1], F6[2]}, Bp[3] = {F6[3], F6[4], F6[5]};
    // ---- Boris forward (keeping intermediates) ----
    const float r = S.r;
    float um[3], t[3], s[3], up[3], un[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) um[a] = fmaf(r, Ep[a], u0[a]);
    const float gm = sqrtf(fmaf(um[0], um[0], fmaf(um[1], um[1], fmaf(um[2], um[2], 1.f))));
    const float igm = rcpf_(gm);
#pragma unroll
    for (int a = 0; a < 3; ++a) t[a] = r * Bp[a] * igm;
    const float tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    const float den = 1.f + tt;
    const float sf = 2.f * rcpf_(den);
#pragma unroll
    for (int a = 0; a < 3; ++a) s[a] = sf * t[a];
    up[0] = um[0] + (um[1] * t[2] - um[2] * t[1]);
    up[1] = um[1] + (um[2] * t[0] - um[0] * t[2]);
    up[2] = um[2] + (um[0] * t[1] - um[1] * t[0]);
    un[0] = um[0] + (up[1] * s[2] - up[2] * s[1]) + r * Ep[0];
    un[1] = um[1] + (up[2] * s[0] - up[0] * s[2]) + r * Ep[1];
    un[2] = um[2] + (up[0] * s[1] - up[1] * s[0]) + r * Ep[2];
    const float gn = sqrtf(fmaf(un[0], un[0], fmaf(un[1], un[1], fmaf(un[2], un[2], 1.f))));
    const float ign = rcpf_(gn);
    float dx[3], e[3];
    int dc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        dx[a] = un[a] * ign * A.dtd[a];
        e[a] = o[a] + dx[a];
        dc[a] = e[a] >= 1.f ? 1 : (e[a] < 0.f ? -1 : 0);
    }
    // ---- deposit adjoint: lam_J = -dt lam_E' on the touched edges ----
    const float ampc[3] = {S.qc[0] * wq, S.qc[1] * wq, S.qc[2] * wq};
    float l1[3] = {0.f, 0.f, 0.f}, l2[3] = {0.f, 0.f, 0.f};
    if ((dc[0] | dc[1] | dc[2]) == 0) {
        // one straight segment; midpoint and displacement from the unrounded dx
        const float W[3] = {fmaf(0.5f, dx[0], o[0]), fmaf(0.5f, dx[1], o[1]),
                            fmaf(0.5f, dx[2], o[2])};
        segment_vjp(g, A.lJsrc, ci, cj, ck, W, dx, ampc, l1, l2);
    } else {
        float WA[3], DA[3], WB[3], DB[3], dr[3], lsA[3] = {0.f, 0.f, 0.f},
              leA[3] = {0.f, 0.f, 0.f}, lsB[3] = {0.f, 0.f, 0.f}, leB[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (dc[a] == 0) {  // relay at the mid-point: derivative 1/2 in both ends
                DA[a] = DB[a] = 0.5f * dx[a];
                WA[a] = fmaf(0.25f, dx[a], o[a]);
                WB[a] = fmaf(0.75f, dx[a], o[a]);
                dr[a] = 0.5f;
            } else {           // relay on the crossed face: constant
                const float xr = dc[a] > 0 ? 1.f : 0.f;
                DA[a] = xr - o[a];
                WA[a] = 0.5f * (o[a] + xr);
                DB[a] = e[a] - xr;
                WB[a] = 0.5f * (xr + e[a]) - (float)dc[a];
                dr[a] = 0.f;
            }
        }
        segment_vjp(g, A.lJsrc, ci, cj, ck, WA, DA, ampc, lsA, leA);
        segment_vjp(g, A.lJsrc, ci + dc[0], cj + dc[1], ck + dc[2], WB, DB, ampc, lsB, leB);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float lr = leA[a] + lsB[a];
            l1[a] = lsA[a] + lr * dr[a];
            l2[a] = leB[a] + lr * dr[a];
        }
    }
    // lam_J = -dt lam_E': the segment adjoints were taken with lam_E', scale now
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        l1[a] *= -A.dt;
        l2[a] *= -A.dt;
    }
    // ---- position chain: x' = x + dt v', xi1 = x/d, xi2 = x/d + dt v'/d ----
    float lxn[3], lv[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float lxp = S.lx[a][p];
        lxn[a] = lxp + (l1[a] + l2[a]) * A.inv_d[a];
        lv[a] = A.dt * (lxp + l2[a] * A.inv_d[a]);
    }
    const float uv = un[0] * lv[0] + un[1] * lv[1] + un[2] * lv[2];
    const float ign3 = ign * ign * ign;
    float lupl[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) lupl[a] = S.lu[a][p] + lv[a] * ign - un[a] * uv * ign3;
    // ---- Boris adjoint ----
    float lE[3], lB[3], lum[3], lup[3], ls[3], lt[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lE[a] = r * lupl[a];
        lum[a] = lupl[a];
    }
    lup[0] = s[1] * lupl[2] - s[2] * lupl[1];
    lup[1] = s[2] * lupl[0] - s[0] * lupl[2];
    lup[2] = s[0] * lupl[1] - s[1] * lupl[0];
    ls[0] = lupl[1] * up[2] - lupl[2] * up[1];
    ls[1] = lupl[2] * up[0] - lupl[0] * up[2];
    ls[2] = lupl[0] * up[1] - lupl[1] * up[0];
    lum[0] += lup[0] + (t[1] * lup[2] - t[2] * lup[1]);
    lum[1] += lup[1] + (t[2] * lup[0] - t[0] * lup[2]);
    lum[2] += lup[2] + (t[0] * lup[1] - t[1] * lup[0]);
    lt[0] = lup[1] * um[2] - lup[2] * um[1];
    lt[1] = lup[2] * um[0] - lup[0] * um[2];
    lt[2] = lup[0] * um[1] - lup[1] * um[0];
    const float tls = t[0] * ls[0] + t[1] * ls[1] + t[2] * ls[2];
    const float iden = rcpf_(den);
#pragma unroll
    for (int a = 0; a < 3; ++a) lt[a] += 2.f * ls[a] * iden - 4.f * t[a] * tls * iden * iden;
    float tlt = 0.f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lB[a] = r * lt[a] * igm;
        tlt += t[a] * lt[a];
    }
    const float lgm = -tlt * igm;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lum[a] += lgm * um[a] * igm;
        lE[a] += r * lum[a];
    }
    // ---- gather adjoint: scatter onto the sub-grids, derivative in x ----
    const float l6[6] = {lE[0], lE[1], lE[2], lB[0], lB[1], lB[2]};
    float dxi[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        tri_scatter(g, q < 3 ? A.lEg[q] : A.lBb[q - 3], idx[q][0], idx[q][1], idx[q][2], fr[q][0],
                    fr[q][1], fr[q][2], l6[q]);
#pragma unroll
        for (int a = 0; a < 3; ++a) dxi[a] += l6[q] * G6[q][a];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        S.lx[a][p] = lxn[a] + dxi[a] * A.inv_d[a];
        S.lu[a][p] = lum[a];
    }
}

// periodic neighbour offsets
__device__ inline long long nb(const GridP &g, int i, int j, int k, int a, int dir) {
    int p[3] = {i, j, k};
    p[a] += dir;
    return gidx(g, p[0], p[1], p[2]);
}

__global__ void k_adj_bprime(GridP g, const float *lEx, const float *lEy, const float *lEz,
                             float *lBx, float *lBy, float *lBz, const float *lbx,
                             const float *lby, const float *lbz, float *tx, float *ty, float *tz) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y * blockDim.y + threadIdx.y,
              k = blockIdx.z;
    if (i >= g.n[0] || j >= g.n[1]) return;
    const long long p = gidx(g, i, j, k);
    const float *lE[3] = {lEx, lEy, lEz};
    float *lB[3] = {lBx, lBy, lBz};
    const float *lb[3] = {lbx, lby, lbz};
    float *tB[3] = {tx, ty, tz};
    const float dt = (float)g.dt;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
        const float curl = (lE[a2][nb(g, i, j, k, a1, 1)] - lE[a2][p]) * (float)g.inv_d[a1] -
                           (lE[a1][nb(g, i, j, k, a2, 1)] - lE[a1][p]) * (float)g.inv_d[a2];
        const float t = lB[c][p] + dt * curl + 0.5f * lb[c][p];
        tB[c][p] = t;
        lB[c][p] = t + 0.5f * lb[c][p];
    }
}

__global__ void k_adj_e(GridP g, float *lEx, float *lEy, float *lEz, const float *gx,
                        const float *gy, const float *gz, const float *tx, const float *ty,
                        const float *tz) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y * blockDim.y + threadIdx.y,
              k = blockIdx.z;
    if (i >= g.n[0] || j >= g.n[1]) return;
    const long long p = gidx(g, i, j, k);
    float *lE[3] = {lEx, lEy, lEz};
    const float *ge[3] = {gx, gy, gz};
    const float *tB[3] = {tx, ty, tz};
    const float dt = (float)g.dt;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
        const float curl = (tB[a2][p] - tB[a2][nb(g, i, j, k, a1, -1)]) * (float)g.inv_d[a1] -
                           (tB[a1][p] - tB[a1][nb(g, i, j, k, a2, -1)]) * (float)g.inv_d[a2];
        lE[c][p] = lE[c][p] + ge[c][p] - dt * curl;
    }
}

// a sort moves the particle in slot perm[j] to slot j; its adjoint moves the
// slot adjoints back.  Pass 1 copies them aside and clears them, pass 2
// writes each to the slot its particle came from.
struct Lam6 {
    float *p[6];
};

__global__ void k_sort_vjp_stash(Lam6 lam, Lam6 tmp, long long cap) {
    const long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (j >= cap) return;
#pragma unroll
    for (int a = 0; a < 6; ++a) {
        tmp.p[a][j] = lam.p[a][j];
        lam.p[a][j] = 0.f;
    }
}

__global__ void k_sort_vjp_scatter(Lam6 lam, Lam6 tmp, const int32_t *perm, long long cap) {
    const long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (j >= cap) return;
    const int32_t q = perm[j];
    if (q < 0 || q >= cap) return;
#pragma unroll
    for (int a = 0; a < 6; ++a) lam.p[a][q] = tmp.p[a][j];
}

__global__ void k_zero_f32(float *p, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = 0.f;
}

}  // namespace

void launch_step_vjp(const GridP &g, float *const E[3], float *const Bbar[3],
                     float *const lE[3], float *const lB[3], float *const lEg[3],
                     float *const lBb[3], float *const tB[3], const SpeciesP *sp,
                     float *const (*lx)[3], float *const (*lu)[3], int nsp, hipStream_t s) {
    for (int a = 0; a < 3; ++a) {
        hipLaunchKernelGGL(k_zero_f32, dim3(1024), dim3(256), 0, s, lEg[a], g.V);
        hipLaunchKernelGGL(k_zero_f32, dim3(1024), dim3(256), 0, s, lBb[a], g.V);
    }
    AdjArgs A;
    A.g = g;
    for (int a = 0; a < 3; ++a) {
        A.E[a] = E[a];
        A.Bb[a] = Bbar[a];
        A.lJsrc[a] = lE[a];
        A.lEg[a] = lEg[a];
        A.lBb[a] = lBb[a];
        A.dtd[a] = (float)(g.dt / g.d[a]);
        A.inv_d[a] = (float)(1.0 / g.d[a]);
    }
    A.dt = (float)g.dt;
    const double dV = g.d[0] * g.d[1] * g.d[2];
    for (int i = 0; i < nsp; ++i) {
        AdjSpecies S;
        S.cell = sp[i].cell;
        for (int a = 0; a < 3; ++a) {
            S.pos[a] = (const float *)sp[i].pos[a];
            S.u[a] = (const float *)sp[i].u[a];
            S.lx[a] = lx[i][a];
            S.lu[a] = lu[i][a];
        }
        S.w = (sp[i].per_particle_w && sp[i].w) ? (const float *)sp[i].w : nullptr;
        S.count = sp[i].count;
        S.r = (float)(sp[i].q * g.dt / (2.0 * sp[i].m));
        const double w = sp[i].per_particle_w ? 1.0 : sp[i].w_species;
        for (int a = 0; a < 3; ++a) S.qc[a] = (float)(sp[i].q * w * g.d[a] / (g.dt * dV));
        if (sp[i].capacity > 0)
            hipLaunchKernelGGL(k_adj_particles, dim3((unsigned)((sp[i].capacity + 255) / 256)),
                               dim3(256), 0, s, A, S);
    }
    const dim3 grid((g.n[0] + 63) / 64, (g.n[1] + 3) / 4, g.n[2]);
    hipLaunchKernelGGL(k_adj_bprime, grid, dim3(64, 4), 0, s, g, lE[0], lE[1], lE[2], lB[0], lB[1],
                       lB[2], lBb[0], lBb[1], lBb[2], tB[0], tB[1], tB[2]);
    hipLaunchKernelGGL(k_adj_e, grid, dim3(64, 4), 0, s, g, lE[0], lE[1], lE[2], lEg[0], lEg[1],
                       lEg[2], tB[0], tB[1], tB[2]);
}

void launch_sort_vjp(const int32_t *perm, long long cap, float *const lx[3], float *const lu[3],
                     float *const scratch[6], hipStream_t s) {
    if (cap <= 0) return;
    Lam6 lam, tmp;
    for (int a = 0; a < 3; ++a) {
        lam.p[a] = lx[a];
        lam.p[3 + a] = lu[a];
    }
    for (int a = 0; a < 6; ++a) tmp.p[a] = scratch[a];
    const unsigned nb = (unsigned)((cap + 255) / 256);
    hipLaunchKernelGGL(k_sort_vjp_stash, dim3(nb), dim3(256), 0, s, lam, tmp, cap);
    hipLaunchKernelGGL(k_sort_vjp_scatter, dim3(nb), dim3(256), 0, s, lam, tmp, perm, cap);
}

}  // namespace empic
