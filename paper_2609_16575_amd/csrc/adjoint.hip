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
//   k_adj_particles (pass 1): one workgroup per tile of the particle sort,
//     like the step's fused kernel.  Per particle it re-computes the forward
//     step with the step kernel's own arithmetic (gather from the staged E,
//     Bbar window, Boris, move), then reverses it: the ZigZag deposit adjoint
//     gathers -dt lam_E' on the edges the particle touched (Sec. 2.5) from a
//     staged lam_E' window, the position and Boris adjoints follow, and the
//     gather's derivative in x adds to lam_x.  lam_Ep, lam_Bp go to per-slot
//     scratch, with a per-tile exponent bounding them.
//   k_adj_scatter (pass 2): the gather adjoint, i.e. lam_Ep, lam_Bp scattered
//     onto the six Yee sub-grids, accumulated per tile in an LDS window in
//     int64 fixed point scaled by the tile's exponent (integer LDS atomics are
//     an order of magnitude cheaper than float ones here), then added to
//     global memory once per tile.  Lanes of a wave take particles in
//     different cells, so that they seldom hit one LDS word together.
//   k_adj_fallback: particles that drifted out of their tile window since the
//     sort, through global memory.
//   k_adj_bprime: lam_B'_t = lam_B' + dt Cf lam_E' + lam_Bbar / 2,
//                 lam_B = lam_B'_t + lam_Bbar / 2;
//   k_adj_e:      lam_E = lam_E' + lam_Egather - dt Cb lam_B'_t.
// Derivatives are taken inside the current piece of each piecewise map (the
// relay-point branch and the interpolation corners are frozen).  Position
// adjoints are per unit length (global coordinates).
#include "internal.hpp"
#include "pic_math.hpp"

namespace empic {

namespace {

constexpr int ADJ_THREADS = 256;   // particle pass
constexpr int SCAT_THREADS = 512;  // scatter pass
constexpr int APPT = 1;            // particles per thread and pass-1 iteration
constexpr int SPPT = 4;            // consecutive particles per thread in pass 2
constexpr int EB = 31;             // fixed point: contributions below 2^EB
typedef float vfA __attribute__((ext_vector_type(APPT)));
typedef uint32_t vuA __attribute__((ext_vector_type(APPT)));
typedef float vfS __attribute__((ext_vector_type(SPPT)));
typedef uint32_t vuS __attribute__((ext_vector_type(SPPT)));
constexpr int NO_EXP = -100000;

__device__ __forceinline__ int pwrap(int x, int n) {
    int m = x % n;
    return m < 0 ? m + n : m;
}

// ---- field and lam_E' access: the tile's LDS windows or global memory --------
template <class TL>
struct LdsAcc {
    const float *sF;  // 6 x FW3: E0..2, Bbar0..2
    const float *sL;  // 3 x JW3: lam_E'
    __device__ float F(int q, int i, int j, int k) const {
        return sF[q * TL::FW3 + i + TL::FWX * (j + TL::FWY * k)];
    }
    __device__ float L(int c, int i, int j, int k) const {
        return sL[c * TL::JW3 + i + TL::JWX * (j + TL::JWY * k)];
    }
};

struct GlobAcc {
    int n0, n1, n2, e0, e1;
    const float *E[3];
    const float *Bb[3];
    const float *lJ[3];
    __device__ long long idx(int i, int j, int k) const {
        return pwrap(i, n0) + (long long)e0 * (pwrap(j, n1) + (long long)e1 * pwrap(k, n2));
    }
    __device__ float F(int q, int i, int j, int k) const {
        return (q < 3 ? E[q] : Bb[q - 3])[idx(i, j, k)];
    }
    __device__ float L(int c, int i, int j, int k) const { return lJ[c][idx(i, j, k)]; }
};

// trilinear value with the step kernel's operation order (tri_lds_at / tri_global)
// and its gradient in the fractional coordinates
template <class Acc>
__device__ __forceinline__ void tri_vg(const Acc &a, int q, int i, int j, int k, float fx, float fy,
                                       float fz, float &val, float gr[3]) {
    const float v0 = a.F(q, i, j, k), v1 = a.F(q, i + 1, j, k);
    const float v2 = a.F(q, i, j + 1, k), v3 = a.F(q, i + 1, j + 1, k);
    const float v4 = a.F(q, i, j, k + 1), v5 = a.F(q, i + 1, j, k + 1);
    const float v6 = a.F(q, i, j + 1, k + 1), v7 = a.F(q, i + 1, j + 1, k + 1);
    const float c00 = lerpf(v0, v1, fx), c10 = lerpf(v2, v3, fx);
    const float c01 = lerpf(v4, v5, fx), c11 = lerpf(v6, v7, fx);
    const float c0 = lerpf(c00, c10, fy), c1 = lerpf(c01, c11, fy);
    val = lerpf(c0, c1, fz);
    gr[2] = c1 - c0;
    gr[1] = lerpf(c10 - c00, c11 - c01, fz);
    gr[0] = lerpf(lerpf(v1 - v0, v3 - v2, fy), lerpf(v5 - v4, v7 - v6, fy), fz);
}

// corner and fractions of component q (E0..2, Bbar0..2) on its staggered
// sub-grid for a particle at offset o in cell l (any coordinates): E_a is
// half-staggered along a, Bbar_a along the two other axes
__device__ __forceinline__ void stagger(int q, const int l[3], const float o[3], int c[3],
                                        float f[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const bool half = q < 3 ? (a == q) : (a != q - 3);
        if (half) {
            half_axis(o[a], l[a], c[a], f[a]);
        } else {
            c[a] = l[a];
            f[a] = o[a];
        }
    }
}

// adjoint of one straight segment inside cell `cell`, given per axis its
// midpoint W relative to that cell and its displacement D: adds d/ds and d/de
// (cell units) of sum_edges lam . J_segment, with D = e - s, W = (s + e)/2 - cell.
template <class Acc>
__device__ __forceinline__ void segment_vjp(const Acc &a, const int cell[3], const float W[3],
                                            const float D[3], const float ampc[3],
                                            const float ampc_lo[3], float ls[3], float le[3]) {
    // per component c, from its four edge adjoints lam_q (q = o1 + 2 o2, o1
    // along b1, o2 along b2) with weights w(0) = 1 - W, w(1) = W:
    //   d/dD_c:   sum_q lam_q w1 w2 + D_b1 D_b2 / 12 sum_q s_q lam_q
    //   d/dW_b1:  D_c sum_q lam_q (2 o1 - 1) w2,  d/dW_b2 likewise
    //   d/dD_b1:  D_c D_b2 / 12 sum_q s_q lam_q,  d/dD_b2 likewise
    // with s_q = +1 where o1 = o2, else -1
    float lD[3] = {0.f, 0.f, 0.f}, lW[3] = {0.f, 0.f, 0.f};
    const float d12[3] = {D[0] * (1.f / 12.f), D[1] * (1.f / 12.f), D[2] * (1.f / 12.f)};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int b1 = (c + 1) % 3, b2 = (c + 2) % 3;
        float lam[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int p[3] = {cell[0], cell[1], cell[2]};
            p[b1] += q & 1;
            p[b2] += q >> 1;
            const float Lc = a.L(c, p[0], p[1], p[2]);
            lam[q] = fmaf(Lc, ampc_lo[c], Lc * ampc[c]);
        }
        const float u1 = W[b1], u2 = W[b2];
        const float e10 = lam[1] - lam[0], e32 = lam[3] - lam[2];
        const float e20 = lam[2] - lam[0], e31 = lam[3] - lam[1];
        const float a0 = fmaf(u1, e10, lam[0]), a1 = fmaf(u1, e32, lam[2]);
        const float bil = fmaf(u2, a1 - a0, a0);
        const float cross = e32 - e10;  // lam0 - lam1 - lam2 + lam3
        lD[c] += fmaf(D[b1] * d12[b2], cross, bil);
        lW[b1] += D[c] * fmaf(u2, e32 - e10, e10);
        lW[b2] += D[c] * fmaf(u1, e31 - e20, e20);
        const float kc = D[c] * cross;
        lD[b1] = fmaf(kc, d12[b2], lD[b1]);
        lD[b2] = fmaf(kc, d12[b1], lD[b2]);
    }
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        ls[b] += -lD[b] + 0.5f * lW[b];
        le[b] += lD[b] + 0.5f * lW[b];
    }
}

struct AdjArgs {
    GridP g;
    TileInfo ti;
    const float *E[3];
    const float *Bb[3];
    const float *lJ[3];  // adjoint of E^{n+1}; lam_J = -dt * lam_E'
    float *lEg[3];       // accumulated adjoint of E^n through the gather
    float *lBb[3];       // accumulated adjoint of Bbar
    float dtd[3], dtd_lo[3];  // dt / d_a and dt as FP32 pairs (split_f32)
    float inv_d[3];
    float dt, dt_lo;
    uint32_t *fb_mask;   // bit p: slot p of this species is outside its tile window
    unsigned *fb_count;  // marked particles
    float *l6[6];        // per slot: lam_Ep, lam_Bp from pass 1 (scratch)
    int *tile_exp;       // per tile: exponent bound of its lam_Ep, lam_Bp
};

struct AdjSpecies {
    const uint32_t *cell;
    const float *pos[3];
    const float *u[3];
    const float *w;            // per-particle weight or nullptr
    float *lx[3];
    float *lu[3];
    const int32_t *tile_off;   // the state's tile offsets
    float r, r_lo;             // q dt / (2 m) as an FP32 pair
    float qc[3], qc_lo[3];     // q w d_a / (dt dV) as FP32 pairs (w = 1 when per-particle)
};

// One particle's adjoint up to the gather scatter: returns lam_Ep, lam_Bp in
// l6 and updates lam_x, lam_u (lx, lu in/out).  Cell coordinates l are the
// accessor's (window-local or global).
template <class Acc>
__device__ __forceinline__ void particle_vjp(const Acc &acc, const AdjArgs &A, const AdjSpecies &S,
                                             const int l[3], const float o[3], const float u[3],
                                             float wq, float lx[3], float lu[3], float l6[6]) {
    // ---- forward re-computation: gather (value and d/d offset) ----
    float F6[6], G6[6][3];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        int c[3];
        float f[3];
        stagger(q, l, o, c, f);
        tri_vg(acc, q, c[0], c[1], c[2], f[0], f[1], f[2], F6[q], G6[q]);
    }
    // ---- Boris with the step kernel's operations, keeping intermediates ----
    const float r = S.r, r_lo = S.r_lo;
    float um[3], t[3], s[3], up[3], un[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) um[a] = fmaf(r_lo, F6[a], fmaf(r, F6[a], u[a]));
    const float igm = rsq_nr(fmaf(um[0], um[0], fmaf(um[1], um[1], fmaf(um[2], um[2], 1.f))));
    const float rig = r * igm;
#pragma unroll
    for (int a = 0; a < 3; ++a) t[a] = rig * F6[3 + a];
    const float den = fmaf(t[0], t[0], fmaf(t[1], t[1], fmaf(t[2], t[2], 1.f)));
    const float iden = rcp_nr(den);
    const float sf = 2.f * iden;
#pragma unroll
    for (int a = 0; a < 3; ++a) s[a] = sf * t[a];
    up[0] = um[0] + (um[1] * t[2] - um[2] * t[1]);
    up[1] = um[1] + (um[2] * t[0] - um[0] * t[2]);
    up[2] = um[2] + (um[0] * t[1] - um[1] * t[0]);
    un[0] = fmaf(r_lo, F6[0], fmaf(r, F6[0], um[0] + (up[1] * s[2] - up[2] * s[1])));
    un[1] = fmaf(r_lo, F6[1], fmaf(r, F6[1], um[1] + (up[2] * s[0] - up[0] * s[2])));
    un[2] = fmaf(r_lo, F6[2], fmaf(r, F6[2], um[2] + (up[0] * s[1] - up[1] * s[0])));
    const float ign = rsq_nr(fmaf(un[0], un[0], fmaf(un[1], un[1], fmaf(un[2], un[2], 1.f))));
    float dx[3], e[3];
    int dc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float no;
        dx[a] = move_cells(un[a] * ign, A.dtd[a], A.dtd_lo[a]);
        move_axis_sel(o[a], dx[a], e[a], dc[a], no);
    }
    // ---- deposit adjoint: lam_J = -dt lam_E' on the touched edges ----
    // Always as two ZigZag segments: a move inside one cell has its relay at
    // the mid-point on every axis, and the line integral over the two halves
    // equals the step kernel's single straight segment, so one code path
    // serves every lane of a wave.
    // q w d_c / (dt dV) per particle as an FP32 pair: hi = the rounded
    // product, lo = its rounding error (FMA) plus the low part of the constant
    float ampc[3], ampc_lo[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        ampc[c] = S.qc[c] * wq;
        ampc_lo[c] = fmaf(S.qc_lo[c], wq, fmaf(S.qc[c], wq, -ampc[c]));
    }
    float l1[3], l2[3];
    {
        float WA[3], DA[3], WB[3], DB[3];
        float lsA[3] = {0.f, 0.f, 0.f}, leA[3] = {0.f, 0.f, 0.f};
        float lsB[3] = {0.f, 0.f, 0.f}, leB[3] = {0.f, 0.f, 0.f};
        zigzag_split(o, dx, e, dc, WA, DA, WB, DB);
        const int lb[3] = {l[0] + dc[0], l[1] + dc[1], l[2] + dc[2]};
        segment_vjp(acc, l, WA, DA, ampc, ampc_lo, lsA, leA);
        segment_vjp(acc, lb, WB, DB, ampc, ampc_lo, lsB, leB);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            // relay point: the mid-point (derivative 1/2 in both ends) or a face
            const float lr = dc[a] == 0 ? 0.5f * (leA[a] + lsB[a]) : 0.f;
            l1[a] = lsA[a] + lr;
            l2[a] = leB[a] + lr;
        }
    }
    // ---- position chain: x' = x + dt v', end point e = o + dt v'/d ----
    float lxn[3], lv[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        // lam_J = -dt lam_E'; dt as its FP32 pair
        const float m1 = -fmaf(A.dt_lo, l1[a], A.dt * l1[a]);
        const float m2 = -fmaf(A.dt_lo, l2[a], A.dt * l2[a]);
        lxn[a] = lx[a] + (m1 + m2) * A.inv_d[a];
        const float xv = lx[a] + m2 * A.inv_d[a];
        lv[a] = fmaf(A.dt_lo, xv, A.dt * xv);
    }
    const float uv = un[0] * lv[0] + un[1] * lv[1] + un[2] * lv[2];
    const float ign3 = ign * ign * ign;
    float lupl[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) lupl[a] = lu[a] + lv[a] * ign - un[a] * uv * ign3;
    // ---- Boris adjoint ----
    float lE[3], lB[3], lum[3], lup[3], ls[3], lt[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lE[a] = fmaf(r_lo, lupl[a], r * lupl[a]);
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
        lE[a] = fmaf(r_lo, lum[a], fmaf(r, lum[a], lE[a]));
    }
    // ---- gather adjoint: derivative in x (the scatter is the caller's) ----
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        l6[a] = lE[a];
        l6[3 + a] = lB[a];
    }
    float dxi[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < 6; ++q)
#pragma unroll
        for (int a = 0; a < 3; ++a) dxi[a] += l6[q] * G6[q][a];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lx[a] = lxn[a] + dxi[a] * A.inv_d[a];
        lu[a] = lum[a];
    }
}

// v times the 8 trilinear weights of fractions f (corner o: bit 0 x, 1 y, 2 z)
__device__ __forceinline__ void tri_weights(const float f[3], float v, float w[8]) {
    const float z0 = v * (1.f - f[2]), z1 = v * f[2];
    const float y00 = z0 * (1.f - f[1]), y10 = z0 * f[1], y01 = z1 * (1.f - f[1]), y11 = z1 * f[1];
    w[0] = y00 * (1.f - f[0]);
    w[1] = y00 * f[0];
    w[2] = y10 * (1.f - f[0]);
    w[3] = y10 * f[0];
    w[4] = y01 * (1.f - f[0]);
    w[5] = y01 * f[0];
    w[6] = y11 * (1.f - f[0]);
    w[7] = y11 * f[0];
}

// gather-as-scatter of one particle straight into global memory (float atomics)
__device__ void scatter_global(const GlobAcc &G, float *const lEg[3], float *const lBb[3],
                               const int l[3], const float o[3], const float l6[6]) {
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        if (l6[q] == 0.f) continue;
        int c[3];
        float f[3], w[8];
        stagger(q, l, o, c, f);
        tri_weights(f, l6[q], w);
        float *dst = q < 3 ? lEg[q] : lBb[q - 3];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            atomicAdd(dst + G.idx(c[0] + (k & 1), c[1] + ((k >> 1) & 1), c[2] + (k >> 2)), w[k]);
    }
}

// window-row tables of a tile: global x index, y*ext0, z*ext0*ext1 (periodic)
template <class TL>
__device__ __forceinline__ void window_rows(const GridP &g, const int wo[3],
                                            int sG[3][TL::ROWS]) {
    constexpr int ROWS = TL::ROWS;
    const int tid = threadIdx.x;
    if (tid < 3 * ROWS) {
        const int a = tid / ROWS, r = tid % ROWS;
        const int wl = a == 0 ? TL::JWX : (a == 1 ? TL::JWY : TL::JWZ);
        if (r < wl) {
            const int mul = a == 0 ? 1 : (a == 1 ? g.ext[0] : g.ext[0] * g.ext[1]);
            sG[a][r] = pwrap(wo[a] + r, g.n[a]) * mul;
        }
    }
}

template <class TL>
__device__ __forceinline__ int tile_of_block(const TileInfo &ti, int wo[3]) {
    constexpr int TX = TL::TX, TY = TL::TY, TZ = TL::TZ;
    const int nb8 = gridDim.x >> 3;
    const int tile = (blockIdx.x & 7) * nb8 + (blockIdx.x >> 3);  // XCD-contiguous tiles
    const int tx = tile % ti.nt[0];
    const int tyz = tile / ti.nt[0];
    const int ty = tyz % ti.nt[1], tz = tyz / ti.nt[1];
    wo[0] = tx * TX - MARGIN - 1;
    wo[1] = ty * TY - MARGIN - 1;
    wo[2] = tz * TZ - MARGIN - 1;
    return tile;
}

// Pass 1, one workgroup per tile: every particle's adjoint up to the gather
// scatter (lam_x, lam_u updated in place; lam_Ep, lam_Bp to the per-slot
// arrays A.l6, zero for particles handled elsewhere) and the tile's exponent:
// all its |lam_Ep|, |lam_Bp| < 2^tile_exp.
// three waves per SIMD measure faster than two without spills
template <class TL>
__global__ __launch_bounds__(ADJ_THREADS, 3) void k_adj_particles(AdjArgs A, AdjSpecies S) {
    constexpr int FWX = TL::FWX, FWY = TL::FWY, FW3 = TL::FW3;
    constexpr int JWX = TL::JWX, JWY = TL::JWY, JW3 = TL::JW3;
    __shared__ float sF[6 * FW3];
    __shared__ float sL[3 * JW3];
    __shared__ int sG[3][TL::ROWS];
    __shared__ int sE;
    __shared__ unsigned sNfb;

    const GridP &g = A.g;
    int wo[3];
    const int tile = tile_of_block<TL>(A.ti, wo);
    if (tile >= A.ti.ntiles) return;
    const int beg = S.tile_off[tile], end = S.tile_off[tile + 1];
    if (beg >= end) return;
    const int tid = threadIdx.x;
    window_rows<TL>(g, wo, sG);
    if (tid == 0) {
        sE = NO_EXP;
        sNfb = 0u;
    }
    __syncthreads();
    // a thread owns the same window points of every component: the global
    // offset of a point is worked out once, and all loads of a window are
    // issued before any is waited on
    {
        constexpr int NR = (FW3 + ADJ_THREADS - 1) / ADJ_THREADS;
        int off[NR];
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const int r = min(tid + q * ADJ_THREADS, FW3 - 1);
            const int lz = r / (FWX * FWY);
            const int r2 = r - lz * (FWX * FWY);
            const int ly = r2 / FWX, lx = r2 - ly * FWX;
            off[q] = sG[0][lx] + sG[1][ly] + sG[2][lz];
        }
        float tmp[6][NR];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const float *src = c < 3 ? A.E[c] : A.Bb[c - 3];
#pragma unroll
            for (int q = 0; q < NR; ++q) tmp[c][q] = src[off[q]];
        }
#pragma unroll
        for (int c = 0; c < 6; ++c)
#pragma unroll
            for (int q = 0; q < NR; ++q)
                if (tid + q * ADJ_THREADS < FW3) sF[c * FW3 + tid + q * ADJ_THREADS] = tmp[c][q];
    }
    {
        constexpr int NR = (JW3 + ADJ_THREADS - 1) / ADJ_THREADS;
        int off[NR];
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const int r = min(tid + q * ADJ_THREADS, JW3 - 1);
            const int lz = r / (JWX * JWY);
            const int r2 = r - lz * (JWX * JWY);
            const int ly = r2 / JWX, lx = r2 - ly * JWX;
            off[q] = sG[0][lx] + sG[1][ly] + sG[2][lz];
        }
        float tmp[3][NR];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int q = 0; q < NR; ++q) tmp[c][q] = A.lJ[c][off[q]];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int q = 0; q < NR; ++q)
                if (tid + q * ADJ_THREADS < JW3) sL[c * JW3 + tid + q * ADJ_THREADS] = tmp[c][q];
    }
    __syncthreads();

    const LdsAcc<TL> lacc{sF, sL};
    const GlobAcc gacc{g.n[0], g.n[1], g.n[2], g.ext[0], g.ext[1],
                       {A.E[0], A.E[1], A.E[2]}, {A.Bb[0], A.Bb[1], A.Bb[2]},
                       {A.lJ[0], A.lJ[1], A.lJ[2]}};
    constexpr int LHI_X = TL::LHI_X, LHI_Y = TL::LHI_Y, LHI_Z = TL::LHI_Z;
    int emax = NO_EXP;
    unsigned nfb = 0u;
    for (int base = (beg & ~(APPT - 1)) + tid * APPT; base < end; base += ADJ_THREADS * APPT) {
        const vuA c4 = *(const vuA *)(S.cell + base);
        const vfA ox4 = *(const vfA *)(S.pos[0] + base), oy4 = *(const vfA *)(S.pos[1] + base),
                  oz4 = *(const vfA *)(S.pos[2] + base);
        const vfA ux4 = *(const vfA *)(S.u[0] + base), uy4 = *(const vfA *)(S.u[1] + base),
                  uz4 = *(const vfA *)(S.u[2] + base);
        vfA w4 = (vfA)(1.f);
        if (S.w) w4 = *(const vfA *)(S.w + base);
        vfA lx4[3], lu4[3], l64[6];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lx4[a] = *(const vfA *)(S.lx[a] + base);
            lu4[a] = *(const vfA *)(S.lu[a] + base);
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) l64[q] = (vfA)(0.f);
#pragma unroll
        for (int k = 0; k < APPT; ++k) {
            const int p = base + k;
            const uint32_t c = c4[k];
            if (p < beg || p >= end || c == DEAD) continue;
            const float o[3] = {ox4[k], oy4[k], oz4[k]};
            const float u[3] = {ux4[k], uy4[k], uz4[k]};
            float lx[3] = {lx4[0][k], lx4[1][k], lx4[2][k]};
            float lu[3] = {lu4[0][k], lu4[1][k], lu4[2][k]};
            float l6[6];
            const int gl[3] = {cell_i(c), cell_j(c), cell_k(c)};
            const int wl[3] = {local_axis(g, 0, gl[0], wo[0]), local_axis(g, 1, gl[1], wo[1]),
                               local_axis(g, 2, gl[2], wo[2])};
            const bool inwin = wl[0] >= 1 && wl[0] <= LHI_X && wl[1] >= 1 && wl[1] <= LHI_Y &&
                               wl[2] >= 1 && wl[2] <= LHI_Z;
            if (inwin) {
                particle_vjp(lacc, A, S, wl, o, u, w4[k], lx, lu, l6);
                float m = 0.f;
#pragma unroll
                for (int q = 0; q < 6; ++q) m = fmaxf(m, fabsf(l6[q]));
                if (m > 0.f && m <= 3.0e38f) {
                    int ex;
                    frexpf(m, &ex);  // m < 2^ex
                    emax = max(emax, ex);
#pragma unroll
                    for (int q = 0; q < 6; ++q) l64[q][k] = l6[q];
                } else if (m != 0.f) {
                    // not finite: let it reach the result through global memory
                    scatter_global(gacc, A.lEg, A.lBb, gl, o, l6);
                }
            } else {
                // drifted more than MARGIN cells out of its tile since the sort:
                // marked for k_adj_fallback (its adjoints stay as loaded here);
                // an atomic whose result is not waited for; the count is
                // summed per workgroup
                atomicOr(A.fb_mask + (p >> 5), 1u << (p & 31));
                ++nfb;
                continue;
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                lx4[a][k] = lx[a];
                lu4[a][k] = lu[a];
            }
        }
        if (base >= beg && base + APPT <= end) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                *(vfA *)(S.lx[a] + base) = lx4[a];
                *(vfA *)(S.lu[a] + base) = lu4[a];
            }
#pragma unroll
            for (int q = 0; q < 6; ++q) *(vfA *)(A.l6[q] + base) = l64[q];
        } else {
#pragma unroll
            for (int k = 0; k < APPT; ++k) {
                const int p = base + k;
                if (p < beg || p >= end) continue;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    S.lx[a][p] = lx4[a][k];
                    S.lu[a][p] = lu4[a][k];
                }
#pragma unroll
                for (int q = 0; q < 6; ++q) A.l6[q][p] = l64[q][k];
            }
        }
    }
    if (emax != NO_EXP) atomicMax(&sE, emax);
    if (nfb) atomicAdd(&sNfb, nfb);
    __syncthreads();
    if (tid == 0) {
        A.tile_exp[tile] = sE;
        if (sNfb) atomicAdd(A.fb_count, sNfb);
    }
}

// Pass 2, one workgroup per tile: the gather scatter of pass 1's lam_Ep,
// lam_Bp onto the six Yee sub-grids, accumulated in an int64 LDS window in
// units of 2^(tile_exp - 31): every contribution is below 2^31 there and is
// rounded to an int32 (error <= 2^-32 of the tile's largest |lam|); one
// entry takes at most one contribution per particle, so the sum cannot
// overflow.  A lane takes SPPT consecutive particles and the lanes of a wave
// are SPPT x 8 = 32 particles apart, in different cells.
template <class TL>
__global__ __launch_bounds__(SCAT_THREADS) void k_adj_scatter(AdjArgs A, AdjSpecies S) {
    constexpr int FWX = TL::FWX, FWY = TL::FWY, FW3 = TL::FW3;
    // LDS layout of the window: row, plane and component strides (words)
    constexpr int RX = FWX, PS = FWX * FWY, CS = FW3;
    __shared__ unsigned long long sA[6 * CS];
    __shared__ int sG[3][TL::ROWS];

    const GridP &g = A.g;
    int wo[3];
    const int tile = tile_of_block<TL>(A.ti, wo);
    if (tile >= A.ti.ntiles) return;
    const int beg = S.tile_off[tile], end = S.tile_off[tile + 1];
    if (beg >= end) return;
    const int et = A.tile_exp[tile];
    if (et == NO_EXP) return;
    const int ee = max(et, -96);  // keeps the scale a finite float
    const int tid = threadIdx.x;
    window_rows<TL>(g, wo, sG);
    for (int e = tid; e < 6 * CS; e += SCAT_THREADS) sA[e] = 0ull;
    __syncthreads();
    constexpr int LHI_X = TL::LHI_X, LHI_Y = TL::LHI_Y, LHI_Z = TL::LHI_Z;
    const float scale = ldexpf(1.f, EB - ee);  // at most 2^127
    const int q0 = (tid & 63) * (SPPT * (SCAT_THREADS / 64)) + (tid >> 6) * SPPT;
    for (int base = (beg & ~(SPPT - 1)) + q0; base < end; base += SCAT_THREADS * SPPT) {
        const vuS c4 = *(const vuS *)(S.cell + base);
        const vfS ox4 = *(const vfS *)(S.pos[0] + base), oy4 = *(const vfS *)(S.pos[1] + base),
                  oz4 = *(const vfS *)(S.pos[2] + base);
        vfS l64[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) l64[q] = *(const vfS *)(A.l6[q] + base);
#pragma unroll
        for (int k = 0; k < SPPT; ++k) {
            const int p = base + k;
            const uint32_t c = c4[k];
            if (p < beg || p >= end || c == DEAD) continue;
            const int wl[3] = {local_axis(g, 0, cell_i(c), wo[0]), local_axis(g, 1, cell_j(c), wo[1]),
                               local_axis(g, 2, cell_k(c), wo[2])};
            if (!(wl[0] >= 1 && wl[0] <= LHI_X && wl[1] >= 1 && wl[1] <= LHI_Y && wl[2] >= 1 &&
                  wl[2] <= LHI_Z))
                continue;  // handled by k_adj_fallback
            const float o[3] = {ox4[k], oy4[k], oz4[k]};
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                const float v = l64[q][k];
                if (v == 0.f) continue;
                int cq[3];
                float f[3], w[8];
                stagger(q, wl, o, cq, f);
                tri_weights(f, v * scale, w);  // exact power-of-two scaling
                unsigned long long *dst = sA + q * CS + cq[0] + RX * cq[1] + PS * cq[2];
#pragma unroll
                for (int oo = 0; oo < 8; ++oo)
                    atomicAdd(dst + (oo & 1) + RX * ((oo >> 1) & 1) + PS * (oo >> 2),
                              (unsigned long long)(long long)__float2int_rn(w[oo]));
            }
        }
    }
    __syncthreads();
    // add the window to the global gather adjoints (non-zero entries only)
    const double inv = ldexp(1.0, ee - EB);
    for (int r = tid; r < FW3; r += SCAT_THREADS) {
        const int lz = r / (FWX * FWY);
        const int r2 = r - lz * (FWX * FWY);
        const int ly = r2 / FWX, lx = r2 - ly * FWX;
        const int o = sG[0][lx] + sG[1][ly] + sG[2][lz];
#pragma unroll
        for (int comp = 0; comp < 6; ++comp) {
            const long long fx = (long long)sA[comp * CS + lx + RX * ly + PS * lz];
            if (fx == 0) continue;
            float *dst = comp < 3 ? A.lEg[comp] : A.lBb[comp - 3];
            atomicAdd(dst + o, (float)((double)fx * inv));
        }
    }
}

// Marked out-of-window particles, entirely through global memory: the set
// bits of the species' mask words, each word cleared once read (nothing to
// scan when none was marked).
__global__ __launch_bounds__(256) void k_adj_fallback(AdjArgs A, AdjSpecies S, long long words) {
    const unsigned n = *(volatile unsigned *)A.fb_count;
    const GlobAcc gacc{A.g.n[0], A.g.n[1], A.g.n[2], A.g.ext[0], A.g.ext[1],
                       {A.E[0], A.E[1], A.E[2]}, {A.Bb[0], A.Bb[1], A.Bb[2]},
                       {A.lJ[0], A.lJ[1], A.lJ[2]}};
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; n != 0 && t < words;
         t += (long long)gridDim.x * blockDim.x) {
      uint32_t bits = A.fb_mask[t];
      if (!bits) continue;
      A.fb_mask[t] = 0u;
      while (bits) {
        const int p = (int)(t * 32) + __builtin_ctz(bits);
        bits &= bits - 1u;
        const uint32_t c = S.cell[p];
        const int gl[3] = {cell_i(c), cell_j(c), cell_k(c)};
        const float o[3] = {S.pos[0][p], S.pos[1][p], S.pos[2][p]};
        const float u[3] = {S.u[0][p], S.u[1][p], S.u[2][p]};
        const float wq = S.w ? S.w[p] : 1.f;
        float lx[3] = {S.lx[0][p], S.lx[1][p], S.lx[2][p]};
        float lu[3] = {S.lu[0][p], S.lu[1][p], S.lu[2][p]};
        float l6[6];
        particle_vjp(gacc, A, S, gl, o, u, wq, lx, lu, l6);
        scatter_global(gacc, A.lEg, A.lBb, gl, o, l6);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            S.lx[a][p] = lx[a];
            S.lu[a][p] = lu[a];
        }
      }
    }
}

// periodic neighbour offsets
__device__ inline long long nb(const GridP &g, int i, int j, int k, int a, int dir) {
    int p[3] = {i, j, k};
    p[a] += dir;
    return pwrap(p[0], g.n[0]) +
           (long long)g.ext[0] * (pwrap(p[1], g.n[1]) + (long long)g.ext[1] * pwrap(p[2], g.n[2]));
}

__global__ void k_adj_bprime(GridP g, const float *lEx, const float *lEy, const float *lEz,
                             float *lBx, float *lBy, float *lBz, const float *lbx,
                             const float *lby, const float *lbz, float *tx, float *ty, float *tz) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y * blockDim.y + threadIdx.y,
              k = blockIdx.z;
    if (i >= g.n[0] || j >= g.n[1]) return;
    const long long p = i + (long long)g.ext[0] * (j + (long long)g.ext[1] * k);
    const float *lE[3] = {lEx, lEy, lEz};
    float *lB[3] = {lBx, lBy, lBz};
    const float *lb[3] = {lbx, lby, lbz};
    float *tB[3] = {tx, ty, tz};
    const float dt = (float)g.dt, dt_lo = (float)(g.dt - (double)dt);  // an FP32 pair
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
        const float curl = (lE[a2][nb(g, i, j, k, a1, 1)] - lE[a2][p]) * (float)g.inv_d[a1] -
                           (lE[a1][nb(g, i, j, k, a2, 1)] - lE[a1][p]) * (float)g.inv_d[a2];
        const float t = lB[c][p] + dt * curl + dt_lo * curl + 0.5f * lb[c][p];
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
    const long long p = i + (long long)g.ext[0] * (j + (long long)g.ext[1] * k);
    float *lE[3] = {lEx, lEy, lEz};
    const float *ge[3] = {gx, gy, gz};
    const float *tB[3] = {tx, ty, tz};
    const float dt = (float)g.dt, dt_lo = (float)(g.dt - (double)dt);  // an FP32 pair
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
        const float curl = (tB[a2][p] - tB[a2][nb(g, i, j, k, a1, -1)]) * (float)g.inv_d[a1] -
                           (tB[a1][p] - tB[a1][nb(g, i, j, k, a2, -1)]) * (float)g.inv_d[a2];
        lE[c][p] = lE[c][p] + ge[c][p] - dt * curl - dt_lo * curl;
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

// Six arrays of n floats cleared in one launch: 16-byte stores when every
// array is 16-byte aligned (vec), single floats otherwise
__global__ void k_zero6(Lam6 z, long long n, int vec) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long t0 = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (!vec) {
        for (long long i = t0; i < n; i += stride)
#pragma unroll
            for (int a = 0; a < 6; ++a) z.p[a][i] = 0.f;
        return;
    }
    const long long n4 = n >> 2;
    for (long long i = t0; i < n4; i += stride)
#pragma unroll
        for (int a = 0; a < 6; ++a) ((float4 *)z.p[a])[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (t0 < n - 4 * n4)
#pragma unroll
        for (int a = 0; a < 6; ++a) z.p[a][4 * n4 + t0] = 0.f;
}

}  // namespace

void launch_step_vjp(const GridP &g, const TileInfo &ti, float *const E[3], float *const Bbar[3],
                     float *const lE[3], float *const lJdep[3], float *const lB[3],
                     float *const lEg[3],
                     float *const lBb[3], float *const tB[3], const SpeciesP *sp,
                     const int32_t *const *tile_off, float *const (*lx)[3],
                     float *const (*lu)[3], int nsp, uint32_t *fb_mask, unsigned *fb_count,
                     float *const (*l6)[6], int *tile_exp, hipStream_t s) {
    {
        Lam6 z;
        int vec = 1;
        for (int a = 0; a < 3; ++a) {
            z.p[a] = lEg[a];
            z.p[3 + a] = lBb[a];
        }
        for (int a = 0; a < 6; ++a) vec &= ((uintptr_t)z.p[a] & 15u) == 0 ? 1 : 0;
        hipLaunchKernelGGL(k_zero6, dim3(2048), dim3(256), 0, s, z, g.V, vec);
    }
    AdjArgs A;
    A.g = g;
    A.ti = ti;
    for (int a = 0; a < 3; ++a) {
        A.E[a] = E[a];
        A.Bb[a] = Bbar[a];
        A.lJ[a] = lJdep[a];
        A.lEg[a] = lEg[a];
        A.lBb[a] = lBb[a];
        split_f32(g.dt / g.d[a], A.dtd[a], A.dtd_lo[a]);
        A.inv_d[a] = (float)(1.0 / g.d[a]);
    }
    split_f32(g.dt, A.dt, A.dt_lo);
    A.fb_mask = fb_mask;
    A.fb_count = fb_count;
    A.tile_exp = tile_exp;
    const double dV = g.d[0] * g.d[1] * g.d[2];
    // one workgroup per tile; a multiple of 8 for the XCD-contiguous tile map
    const unsigned nblocks = (unsigned)(8 * ((ti.ntiles + 7) / 8));
    for (int i = 0; i < nsp; ++i) {
        if (sp[i].capacity <= 0) continue;
        AdjSpecies S;
        S.cell = sp[i].cell;
        for (int a = 0; a < 3; ++a) {
            S.pos[a] = (const float *)sp[i].pos[a];
            S.u[a] = (const float *)sp[i].u[a];
            S.lx[a] = lx[i][a];
            S.lu[a] = lu[i][a];
        }
        S.w = (sp[i].per_particle_w && sp[i].w) ? (const float *)sp[i].w : nullptr;
        S.tile_off = tile_off[i];
        split_f32(sp[i].q * g.dt / (2.0 * sp[i].m), S.r, S.r_lo);
        const double w = sp[i].per_particle_w ? 1.0 : sp[i].w_species;
        for (int a = 0; a < 3; ++a) split_f32(sp[i].q * w * g.d[a] / (g.dt * dV), S.qc[a], S.qc_lo[a]);
        for (int q = 0; q < 6; ++q) A.l6[q] = l6[i][q];
        launch_fill_i32((int32_t *)fb_count, 1, 0, s);
        if (ti.slab)
            hipLaunchKernelGGL(k_adj_particles<TileSlab>, dim3(nblocks), dim3(ADJ_THREADS), 0, s,
                               A, S);
        else
            hipLaunchKernelGGL(k_adj_particles<TileCube>, dim3(nblocks), dim3(ADJ_THREADS), 0, s,
                               A, S);
        hipLaunchKernelGGL(k_adj_fallback, dim3(1024), dim3(256), 0, s, A, S,
                           (long long)((sp[i].capacity + 31) / 32));
        if (ti.slab)
            hipLaunchKernelGGL(k_adj_scatter<TileSlab>, dim3(nblocks), dim3(SCAT_THREADS), 0, s,
                               A, S);
        else
            hipLaunchKernelGGL(k_adj_scatter<TileCube>, dim3(nblocks), dim3(SCAT_THREADS), 0, s,
                               A, S);
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
