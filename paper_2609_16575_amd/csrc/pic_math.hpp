// pic_math.hpp -- per-particle arithmetic of the FP32 path shared by the
// fused step kernel and its adjoint, so that the adjoint re-computes each
// particle's step with exactly the forward kernel's operations and branch
// decisions: staggered CIC gather (Sec. 2.5), relativistic Boris push
// (Sec. 2.4), move with offset canonicalization, ZigZag segments and their
// exact straight-segment edge weights (Sec. 2.5), and the LDS window indexing.
#pragma once

#include "internal.hpp"

namespace empic {

typedef float vf4 __attribute__((ext_vector_type(4)));
typedef uint32_t vu4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float rcpf(float x) { return __builtin_amdgcn_rcpf(x); }
// 1/sqrt(x) in one hardware approximation (one transcendental instead of a
// square root and a reciprocal)
__device__ __forceinline__ float rsqf(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float lerpf(float a, float b, float t) { return fmaf(t, b - a, a); }
// 1/x and 1/sqrt(x) to about half an ulp: the hardware approximation and one
// Newton step (the approximations alone can err by an ulp in the same
// direction over a range of arguments, a systematic error of the velocity
// that would accumulate over many steps)
__device__ __forceinline__ float rcp_nr(float x) {
    const float y = rcpf(x);
    return fmaf(y, fmaf(-x, y, 1.f), y);
}
__device__ __forceinline__ float rsq_nr(float x) {
    const float y = rsqf(x);
    return fmaf(0.5f * y, fmaf(-x * y, y, 1.f), y);
}

// global index of cell-axis coordinate x on axis a: periodic wrap (any x),
// -1 outside an absorbing axis' array
__device__ __forceinline__ int gaxis(const GridP &g, int a, int x) {
    if (g.bc[a] == EMPIC_BC_PERIODIC) {
        int m = x % g.n[a];
        return m < 0 ? m + g.n[a] : m;
    }
    return (x < 0 || x >= g.ext[a]) ? -1 : x;
}

__device__ inline float tri_global(const GridP &g, const float *F, int i0, int j0, int k0, float fx,
                            float fy, float fz) {
    float v[8];
#pragma unroll
    for (int o = 0; o < 8; ++o) {
        const int gx = gaxis(g, 0, i0 + (o & 1)), gy = gaxis(g, 1, j0 + ((o >> 1) & 1)),
                  gz = gaxis(g, 2, k0 + (o >> 2));
        v[o] = (gx < 0 || gy < 0 || gz < 0)
                   ? 0.f
                   : F[gx + (long long)g.ext[0] * (gy + (long long)g.ext[1] * gz)];
    }
    const float c00 = lerpf(v[0], v[1], fx), c10 = lerpf(v[2], v[3], fx);
    const float c01 = lerpf(v[4], v[5], fx), c11 = lerpf(v[6], v[7], fx);
    return lerpf(lerpf(c00, c10, fy), lerpf(c01, c11, fy), fz);
}

// ---------------------------------------------------------------------------
// Second-order shapes (the shape-function equation of Sec. 2.4 with l = 1):
// weighting by the quadratic B-spline b_2 on the nearest index m of a
// sub-grid and its two neighbours.  For a point at m + d, |d| <= 1/2:
//   b_2(d + 1) = (1/2 - d)^2 / 2, b_2(d) = 3/4 - d^2, b_2(d - 1) = (1/2 + d)^2 / 2
// (weights of m - 1, m, m + 1).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void b2_w(float d, float w[3]) {
    const float a = 0.5f - d, b = 0.5f + d;
    w[0] = 0.5f * a * a;
    w[1] = fmaf(-d, d, 0.75f);
    w[2] = 0.5f * b * b;
}

// Stencil of an in-cell offset o on one axis, relative to the particle's
// cell: node (integer) sub-grids m = (o >= 1/2), d = o - m; half-integer
// sub-grids (index i at i + 1/2) m = 0, d = o - 1/2.
__device__ __forceinline__ void b2_node(float o, int &m, float &d) {
    m = o >= 0.5f ? 1 : 0;
    d = o - (float)m;
}

// 27-point b_2 interpolation from global memory (m: nearest index per axis;
// points outside an absorbing axis' array contribute zero)
__device__ inline float tri2_global(const GridP &g, const float *F, int m0, int m1, int m2,
                                    const float wx[3], const float wy[3], const float wz[3]) {
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int gz = gaxis(g, 2, m2 - 1 + k);
        if (gz < 0) continue;
        float sy = 0.f;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int gy = gaxis(g, 1, m1 - 1 + j);
            if (gy < 0) continue;
            float sx = 0.f;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int gx = gaxis(g, 0, m0 - 1 + i);
                if (gx < 0) continue;
                sx = fmaf(wx[i], F[gx + (long long)g.ext[0] * (gy + (long long)g.ext[1] * gz)], sx);
            }
            sy = fmaf(wy[j], sx, sy);
        }
        s = fmaf(wz[k], sy, s);
    }
    return s;
}

// E and Bbar at a particle with b_2 weights, each component from its own
// Yee sub-grid (Ex half-integer along x, Bx half-integer along y and z, ...)
__device__ inline void gather2_global(const GridP &g, const float *const E[3],
                                      const float *const Bb[3], int ci, int cj, int ck, float ox,
                                      float oy, float oz, float Ep[3], float Bp[3]) {
    const int c[3] = {ci, cj, ck};
    const float o[3] = {ox, oy, oz};
    int mn[3], mh[3];
    float wn[3][3], wh[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int m;
        float d;
        b2_node(o[a], m, d);
        mn[a] = c[a] + m;
        b2_w(d, wn[a]);
        mh[a] = c[a];
        b2_w(o[a] - 0.5f, wh[a]);
    }
    Ep[0] = tri2_global(g, E[0], mh[0], mn[1], mn[2], wh[0], wn[1], wn[2]);
    Ep[1] = tri2_global(g, E[1], mn[0], mh[1], mn[2], wn[0], wh[1], wn[2]);
    Ep[2] = tri2_global(g, E[2], mn[0], mn[1], mh[2], wn[0], wn[1], wh[2]);
    Bp[0] = tri2_global(g, Bb[0], mn[0], mh[1], mh[2], wn[0], wh[1], wh[2]);
    Bp[1] = tri2_global(g, Bb[1], mh[0], mn[1], mh[2], wh[0], wn[1], wh[2]);
    Bp[2] = tri2_global(g, Bb[2], mh[0], mh[1], mn[2], wh[0], wh[1], wn[2]);
}

// Esirkepov's decomposition of one part of a move that stays in the b_2
// cell m (relative to the particle's cell) on every axis, from sA to sB
// (offsets relative to the particle's cell).  With S0 = b_2 weights at sA,
// dS = (weights at sB) - S0 on the nodes m - 1 .. m + 1 of each axis,
//   W_c = dS_c (S0_b S0_e + dS_b S0_e / 2 + S0_b dS_e / 2 + dS_b dS_e / 3),
// and J_c on the edge between nodes l and l + 1 along c is -(sum of W_c up
// to l) times the charge factor (the third running sum is zero).
// sink.origin(x, y, z) receives the part's first node m - 1 per axis
// (relative to the particle's cell), then sink(c, x, y, z, v) the value v for
// the edge or node index origin + (x, y, z), with x, y, z known at compile
// time once unrolled; v still lacks the charge factor of component c.
template <class Sink>
__device__ __forceinline__ void ez2_part(const float sA[3], const float sB[3], const int m[3],
                                         float wq, Sink &sink) {
    sink.origin(m[0] - 1, m[1] - 1, m[2] - 1);
    float S0[3][3], dS[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float w1[3];
        b2_w(sA[a] - (float)m[a], S0[a]);
        b2_w(sB[a] - (float)m[a], w1);
#pragma unroll
        for (int i = 0; i < 3; ++i) dS[a][i] = w1[i] - S0[a][i];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int b = c == 2 ? 0 : c + 1, e = c == 0 ? 2 : c - 1;
        const int bb = b < e ? b : e, ee = b < e ? e : b;  // T[ib][ie] over (b, e)
        const float r0 = -wq * dS[c][0], r1 = -wq * (dS[c][0] + dS[c][1]);
#pragma unroll
        for (int ib = 0; ib < 3; ++ib)
#pragma unroll
            for (int ie = 0; ie < 3; ++ie) {
                const float T = fmaf(dS[bb][ib], fmaf(0.5f, S0[ee][ie], dS[ee][ie] * (1.f / 3.f)),
                                     S0[bb][ib] * fmaf(0.5f, dS[ee][ie], S0[ee][ie]));
                int idx[3];
                idx[bb] = ib;
                idx[ee] = ie;
                idx[c] = 0;
                sink(c, idx[0], idx[1], idx[2], r0 * T);
                idx[c] = 1;
                sink(c, idx[0], idx[1], idx[2], r1 * T);
            }
    }
}

// The EZ current of a move from offset o by dx (cell units, relative to the
// particle's cell): one Esirkepov part inside one b_2 cell, else two parts
// split at the ZigZag relay point (the crossed half-integer plane on a
// crossing axis, the mid-point on the others).
template <class Sink>
__device__ __forceinline__ void ez2_move(const float o[3], const float dx[3], float wq,
                                         Sink &sink) {
    float s1[3];
    int m0[3], m1[3];
    bool cross = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        s1[a] = o[a] + dx[a];
        m0[a] = o[a] >= 0.5f ? 1 : 0;
        m1[a] = (int)floorf(s1[a] + 0.5f);
        cross = cross || m0[a] != m1[a];
    }
    if (!cross) {
        ez2_part(o, s1, m0, wq, sink);
        return;
    }
    float r[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
        r[a] = m0[a] != m1[a] ? (float)max(m0[a], m1[a]) - 0.5f : 0.5f * (o[a] + s1[a]);
    ez2_part(o, r, m0, wq, sink);
    ez2_part(r, s1, m1, wq, sink);
}

__device__ __forceinline__ void half_axis(float o, int l, int &h, float &fh) {
    if (o < 0.5f) {
        h = l - 1;
        fh = o + 0.5f;
    } else {
        h = l;
        fh = o - 0.5f;
    }
}

__device__ inline void gather_global(const GridP &g, const float *const E[3], const float *const Bb[3],
                              int ci, int cj, int ck, float ox, float oy, float oz, float Ep[3],
                              float Bp[3]) {
    int hx, hy, hz;
    float fx, fy, fz;
    half_axis(ox, ci, hx, fx);
    half_axis(oy, cj, hy, fy);
    half_axis(oz, ck, hz, fz);
    Ep[0] = tri_global(g, E[0], hx, cj, ck, fx, oy, oz);
    Ep[1] = tri_global(g, E[1], ci, hy, ck, ox, fy, oz);
    Ep[2] = tri_global(g, E[2], ci, cj, hz, ox, oy, fz);
    Bp[0] = tri_global(g, Bb[0], ci, hy, hz, ox, fy, fz);
    Bp[1] = tri_global(g, Bb[1], hx, cj, hz, fx, oy, fz);
    Bp[2] = tri_global(g, Bb[2], hx, hy, ck, fx, fy, oz);
}

// relativistic Boris push in FP32 (standard t/s rotation); returns 1/gamma of u+.
// r = q dt / (2 m) as the FP32 pair (r, r_lo): the electric half kicks add
// both parts (no systematic error from the rounding of r); the rotation uses r.
__device__ __forceinline__ float boris_f32(float &ux, float &uy, float &uz, const float E[3],
                                           const float B[3], float r, float r_lo, float &gam) {
    const float umx = fmaf(r_lo, E[0], fmaf(r, E[0], ux));
    const float umy = fmaf(r_lo, E[1], fmaf(r, E[1], uy));
    const float umz = fmaf(r_lo, E[2], fmaf(r, E[2], uz));
    const float ig = rsq_nr(fmaf(umx, umx, fmaf(umy, umy, fmaf(umz, umz, 1.f))));  // 1/gamma-
    const float rig = r * ig;
    const float tx = rig * B[0], ty = rig * B[1], tz = rig * B[2];
    const float sf = 2.f * rcp_nr(fmaf(tx, tx, fmaf(ty, ty, fmaf(tz, tz, 1.f))));
    const float sx = sf * tx, sy = sf * ty, sz = sf * tz;
    const float upx = umx + (umy * tz - umz * ty);
    const float upy = umy + (umz * tx - umx * tz);
    const float upz = umz + (umx * ty - umy * tx);
    const float plx = umx + (upy * sz - upz * sy);
    const float ply = umy + (upz * sx - upx * sz);
    const float plz = umz + (upx * sy - upy * sx);
    ux = fmaf(r_lo, E[0], fmaf(r, E[0], plx));
    uy = fmaf(r_lo, E[1], fmaf(r, E[1], ply));
    uz = fmaf(r_lo, E[2], fmaf(r, E[2], plz));
    const float g2 = fmaf(ux, ux, fmaf(uy, uy, fmaf(uz, uz, 1.f)));
    const float igp = rsq_nr(g2);
    gam = g2 * igp;
    return igp;
}

// Line integral of the bilinear CIC edge weights along a straight segment
// inside one cell, given per axis the segment midpoint W (relative to that
// cell) and its displacement D (cell units):
// out[0..3] J_x edges (oy,oz) = (0,0),(1,0),(0,1),(1,1); out[4..7] J_y edges
// (oz,ox); out[8..11] J_z edges (ox,oy).
// Component c is amp_c D_c [w_b1 w_b2 +- D_b1 D_b2 / 12] with (w(0), w(1)) =
// (1 - W, W); it is evaluated as four FMAs on amp_c D_c (1 - W_b1), amp_c D_c
// W_b1 and the cross term amp_c D_0 D_1 D_2 / 12, whose triple product all
// three components share (30 operations per segment).
__device__ __forceinline__ void segment_weights(const float W[3], const float D[3],
                                                const float amp_c[3], float out[12]) {
    const float p3 = D[0] * D[1] * (D[2] * (1.f / 12.f));
    const float om[3] = {1.f - W[0], 1.f - W[1], 1.f - W[2]};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int b1 = (c + 1) % 3, b2 = (c + 2) % 3;
        const float a = amp_c[c] * D[c];
        const float a0 = a * om[b1], a1 = a * W[b1];
        const float cr = amp_c[c] * p3;
        out[4 * c + 0] = fmaf(a0, om[b2], cr);
        out[4 * c + 1] = fmaf(a1, om[b2], -cr);
        out[4 * c + 2] = fmaf(a0, W[b2], -cr);
        out[4 * c + 3] = fmaf(a1, W[b2], cr);
    }
}

// Midpoints and displacements of the ZigZag segments of a move from offset o
// by dxi (end e = o + dxi as rounded, cell step dc per axis).  The
// displacement is taken from dxi itself wherever the segment does not end on
// a cell face, so that a small move keeps its full FP32 precision instead of
// the difference of two rounded offsets.
//   no crossing: one segment, W = o + dxi/2, D = dxi
//   crossing:    relay xr = 1 (dc = +1), 0 (dc = -1), mid-point (dc = 0);
//                segment A in the particle's cell, B in the cell + dc
__device__ __forceinline__ void zigzag_split(const float o[3], const float dxi[3],
                                             const float e[3], const int dc[3], float WA[3],
                                             float DA[3], float WB[3], float DB[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (dc[a] == 0) {
            DA[a] = DB[a] = 0.5f * dxi[a];
            WA[a] = fmaf(0.25f, dxi[a], o[a]);
            WB[a] = fmaf(0.75f, dxi[a], o[a]);
        } else {
            const float xr = dc[a] > 0 ? 1.f : 0.f;
            DA[a] = xr - o[a];
            WA[a] = 0.5f * (o[a] + xr);
            DB[a] = e[a] - xr;
            WB[a] = 0.5f * (xr + e[a]) - (float)dc[a];
        }
    }
}

// Per-axis move of a particle: new end point e (relative to its cell), cell
// step dc in {-1,0,1} and canonical new offset in [0,1).  When e + 1 rounds
// to 1 the particle is put at offset 0 of its own cell and e is set to 0,
// so that deposit and stored state agree.
__device__ __forceinline__ void move_axis(float o, float dxi, float &e, int &dc, float &no) {
    e = o + dxi;
    dc = 0;
    if (e >= 1.f) {
        dc = 1;
        no = e - 1.f;
    } else if (e < 0.f) {
        const float t = e + 1.f;
        if (t >= 1.f) {
            e = 0.f;
            no = 0.f;
        } else {
            dc = -1;
            no = t;
        }
    } else {
        no = e;
    }
}

__device__ __forceinline__ bool new_cell(const GridP &g, int a, int c, int dc, int &out) {
    int x = c + dc;
    if (g.bc[a] == EMPIC_BC_PERIODIC) {
        x = x < 0 ? x + g.n[a] : (x >= g.n[a] ? x - g.n[a] : x);
    } else if (x < 0 || x >= g.n[a]) {
        return false;
    }
    out = x;
    return true;
}

// ---- LDS window versions ----
// trilinear value from the LDS field window at byte address pb (the corner
// of lowest index)
template <class TL>
__device__ __forceinline__ float tri_lds_at(const char *pb, float fx, float fy, float fz) {
    constexpr int FWX = TL::FWX, FWY = TL::FWY;
    const float *p = (const float *)pb;
    const float c00 = lerpf(p[0], p[1], fx);
    const float c10 = lerpf(p[FWX], p[FWX + 1], fx);
    const float c01 = lerpf(p[FWX * FWY], p[FWX * FWY + 1], fx);
    const float c11 = lerpf(p[FWX * FWY + FWX], p[FWX * FWY + FWX + 1], fx);
    return lerpf(lerpf(c00, c10, fy), lerpf(c01, c11, fy), fz);
}

// J window offsets of the 12 edges of a cell, in segment_weights order
template <class TL>
__device__ __forceinline__ int edge_off(int q) {
    constexpr int JWX = TL::JWX, JWY = TL::JWY, JW3 = TL::JW3;
    // J_x (oy,oz); J_y (oz,ox); J_z (ox,oy)
    const int c = q >> 2, b = q & 3, o1 = b & 1, o2 = b >> 1;
    if (c == 0) return JW3 * 0 + o1 * JWX + o2 * JWX * JWY;
    if (c == 1) return JW3 * 1 + o1 * JWX * JWY + o2;
    return JW3 * 2 + o1 + o2 * JWX;
}

// Displacement in cells of a particle with velocity v along an axis with
// dt / d = (dtd, dtd_lo) (an FP32 pair, see split_f32)
__device__ __forceinline__ float move_cells(float v, float dtd, float dtd_lo) {
    return fmaf(v, dtd_lo, v * dtd);
}

// Float -> int64 fixed point, round to nearest: the sum with 1.5 * 2^52 puts
// the integer part of x * scale in the low mantissa bits (valid for
// |x * scale| < 2^51, which the choice of the scale guarantees).
__device__ __forceinline__ long long to_fixed(float x, double scale) {
    const double t = fma((double)x, scale, 6755399441055744.0);
    return __double_as_longlong(t) - 0x4338000000000000LL;
}

__device__ __forceinline__ int local_axis(const GridP &g, int a, int c, int wo) {
    if (g.bc[a] == EMPIC_BC_PERIODIC) {
        int m = c - wo - 1;
        m = m < 0 ? m + g.n[a] : (m >= g.n[a] ? m - g.n[a] : m);
        return m + 1;
    }
    return c - wo;
}

// Branch-free move of one axis (see move_axis).
__device__ __forceinline__ void move_axis_sel(float o, float dx, float &e, int &dc, float &no) {
    e = o + dx;
    const bool up = e >= 1.f;
    const bool dn = e < 0.f;
    const float t = e + 1.f;
    const bool rc = dn && t >= 1.f;  // e + 1 rounds to 1: stay at offset 0 of this cell
    dc = up ? 1 : ((dn && !rc) ? -1 : 0);
    no = up ? (e - 1.f) : (dn ? (rc ? 0.f : t) : e);
    e = rc ? 0.f : e;
}

}  // namespace empic
