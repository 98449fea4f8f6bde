// push_f32.hip -- FP32 cell-relative particle path for gfx950.
//
// Storage: per particle a packed cell index (i | j<<11 | k<<22), an FP32
// in-cell offset in [0,1) per axis and FP32 u = gamma v; 28 bytes (+4 for a
// per-particle weight).  Offsets relative to the cell keep the rounding of a
// position at 2^-24 of a cell wherever the particle is in the grid.
//
// k_push_fused: one workgroup (512 threads) per 8x8x4 tile of cells (16x2x8
// on grids at most three cells thick along y; particles counting-sorted by
// tile, then cell).  The workgroup
//   1. stages E^n and the centred B^n of the tile plus a halo into LDS
//      (12 x 12 x 8 cells x 6 components; a thread owns the same window
//      points of every component and issues all its loads before waiting),
//   2. zeroes an LDS current window (13 x 13 x 9 edges x 3),
//   3. streams its particles: each thread owns PPT = 4 consecutive particles,
//      one 16-byte access per array (one particle per thread in a tile with
//      at most 1024 of a species; species 0's are then loaded together with
//      the window), and for each does the staggered CIC gather from LDS (Sec.
//      2.5), the relativistic Boris push (Sec. 2.4), the move and the ZigZag
//      deposit (Sec. 2.5): 12 int64 LDS atomics per straight segment (24 for
//      a particle crossing a cell face),
//   4. adds the non-zero LDS current to global J with float atomics.
// Particles that drifted more than MARGIN cells out of their tile since the
// last sort are handled entirely through global memory (rare, counted).
// Particles are read from one buffer set and written to another (the same
// one for a step in place; a saved state and the next one when the states
// between checkpoints of a differentiable run are re-computed).
//
// Algorithmic bytes per particle: 28 read + 28 written.
#include <hip/hip_ext.h>

#include "internal.hpp"
#include "pic_math.hpp"

namespace empic {

namespace {

struct FusedArgs {
    GridP g;
    TileInfo ti;
    const float *E[3];
    const float *Bb[3];
    unsigned long long *Jf[3];  // the step's current in units of 1/jscale (int64 sums)
    const DevSpecies *tbl;  // species parameters (device memory)
    int nsp;
    unsigned cur_mask;      // bit s: buffer set species s is read from
    unsigned wr_mask;       // bit s: buffer set species s is written to (the same for a step in place)
    float dtd[3], dtd_lo[3];  // dt / d_a as FP32 pairs (split_f32)
    double jscale, jinv;    // fixed-point scale of the current (LDS window and Jf) and its inverse
    uint32_t *fault;
    unsigned long long *fallback;  // cumulative count of out-of-window particles
    uint32_t *fb_mask;             // bit p of species s's words: slot p is out of its window
    long long mask_words;          // words per species in fb_mask
    int *fb_tiles;                 // tiles with marked particles this step
    unsigned *fb_count;            // [0] particles marked this step, [1] unused, [2]
                                   // entries in fb_tiles (cleared by k_faraday)
    unsigned long long *publish;   // host-visible copy of *fallback (k_push_fallback), or null
};

// global atomic deposit of one segment's 12 values at cell (ci,cj,ck), in
// the fixed point of the tile windows (mult[c]: the scale times the charge
// factor of component c)
__device__ void deposit_global(const GridP &g, unsigned long long *const Jf[3], int ci, int cj,
                               int ck, const float v[12], const double mult[3]) {
    const int cell[3] = {ci, cj, ck};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int b1 = (c + 1) % 3, b2 = (c + 2) % 3;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int p[3] = {cell[0], cell[1], cell[2]};
            p[b1] += q & 1;
            p[b2] += q >> 1;
            const int gx = gaxis(g, 0, p[0]), gy = gaxis(g, 1, p[1]), gz = gaxis(g, 2, p[2]);
            if (gx < 0 || gy < 0 || gz < 0) continue;
            const int gc = c == 0 ? gx : (c == 1 ? gy : gz);
            if (g.bc[c] != EMPIC_BC_PERIODIC && gc >= g.n[c]) continue;  // padding
            atomicAdd(Jf[c] + gx + (long long)g.ext[0] * (gy + (long long)g.ext[1] * gz),
                      (unsigned long long)to_fixed(v[4 * c + q], mult[c]));
        }
    }
}

// Order-2 current of a particle into the global fixed-point sums
struct GlobalSink2 {
    const GridP &g;
    unsigned long long *const *Jf;
    int cell[3];
    const double *mult;
    int o[3] = {0, 0, 0};
    __device__ void origin(int x, int y, int z) {
        o[0] = cell[0] + x;
        o[1] = cell[1] + y;
        o[2] = cell[2] + z;
    }
    __device__ void operator()(int c, int x, int y, int z, float v) const {
        const int gx = gaxis(g, 0, o[0] + x), gy = gaxis(g, 1, o[1] + y),
                  gz = gaxis(g, 2, o[2] + z);
        if (gx < 0 || gy < 0 || gz < 0 || v == 0.f) return;
        atomicAdd(Jf[c] + gx + (long long)g.ext[0] * (gy + (long long)g.ext[1] * gz),
                  (unsigned long long)to_fixed(v, mult[c]));
    }
};

// Whole particle through global memory (drifted out of the LDS window).
template <int ORDER>
__device__ void particle_global(const FusedArgs &A, const DevSpecies &D, uint32_t &c, float &ox,
                                             float &oy, float &oz, float &ux, float &uy,
                                             float &uz, float wq, uint32_t &fbits) {
    const GridP &g = A.g;
    const int ci = cell_i(c), cj = cell_j(c), ck = cell_k(c);
    float Ep[3], Bp[3];
    if constexpr (ORDER == 2) gather2_global(g, A.E, A.Bb, ci, cj, ck, ox, oy, oz, Ep, Bp);
    else gather_global(g, A.E, A.Bb, ci, cj, ck, ox, oy, oz, Ep, Bp);
    float gam;
    const float ig = boris_f32(ux, uy, uz, Ep, Bp, D.r, D.r_lo, gam);
    if (!isfinite(gam)) fbits |= EMPIC_FAULT_NONFINITE;
    const float o[3] = {ox, oy, oz};
    const float uu[3] = {ux, uy, uz};
    float e[3], no[3], dx[3];
    int dc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        dx[a] = move_cells(uu[a] * ig, A.dtd[a], A.dtd_lo[a]);
        if (!(fabsf(dx[a]) < 1.f)) fbits |= EMPIC_FAULT_FAST;
        move_axis(o[a], dx[a], e[a], dc[a], no[a]);
    }
    // as in the tile kernel: weights with the particle's weight in FP32, the
    // charge factor in FP64 in the conversion to fixed point
    const float amp[3] = {wq, wq, wq};
    const double mult[3] = {A.jscale * D.qcd[0], A.jscale * D.qcd[1], A.jscale * D.qcd[2]};
    float v[12];
    if constexpr (ORDER == 2) {
        GlobalSink2 sink{g, A.Jf, {ci, cj, ck}, mult};
        ez2_move(o, dx, wq, sink);
    } else if ((dc[0] | dc[1] | dc[2]) == 0) {
        const float W[3] = {fmaf(0.5f, dx[0], o[0]), fmaf(0.5f, dx[1], o[1]),
                            fmaf(0.5f, dx[2], o[2])};
        segment_weights(W, dx, amp, v);  // one straight segment in this cell
        deposit_global(g, A.Jf, ci, cj, ck, v, mult);
    } else {
        float WA[3], DA[3], WB[3], DB[3];
        zigzag_split(o, dx, e, dc, WA, DA, WB, DB);
        segment_weights(WA, DA, amp, v);
        deposit_global(g, A.Jf, ci, cj, ck, v, mult);
        segment_weights(WB, DB, amp, v);
        deposit_global(g, A.Jf, ci + dc[0], cj + dc[1], ck + dc[2], v, mult);
    }
    int ni, nj, nk;
    const int ok = (int)new_cell(g, 0, ci, dc[0], ni) & (int)new_cell(g, 1, cj, dc[1], nj) &
                   (int)new_cell(g, 2, ck, dc[2], nk);
    c = ok ? pack_cell(ni, nj, nk) : DEAD;
    ox = no[0];
    oy = no[1];
    oz = no[2];
}

// The LDS current window accumulates int64 fixed point: integer LDS atomics
// are an order of magnitude faster than float ones on this LDS, and the tile's
// sums become exact and independent of the order of the adds.  The segment's
// edge weights are formed in FP32 with the particle's weight wq alone; the
// charge factor q w d_c / (dt dV) enters in FP64 with the window's scale,
// mult[c], in the conversion to fixed point.
template <class TL>
__device__ __forceinline__ void lds_add_segment(unsigned long long *sJ, int base, const float W[3],
                                                const float D[3], float wq, const double mult[3]) {
    const float amp[3] = {wq, wq, wq};
    float v[12];
    segment_weights(W, D, amp, v);
#pragma unroll
    for (int q = 0; q < 12; ++q)
        atomicAdd(sJ + base + edge_off<TL>(q), (unsigned long long)to_fixed(v[q], mult[q >> 2]));
}

typedef float __attribute__((address_space(1))) gfloat;
typedef uint32_t __attribute__((address_space(1))) guint;

// P consecutive particles of one thread as loaded (one access of P elements
// per array; weight 1 without per-particle weights)
template <int P>
struct Batch {
    typedef float VF __attribute__((ext_vector_type(P)));
    typedef uint32_t VU __attribute__((ext_vector_type(P)));
    VU c;
    VF ox, oy, oz, ux, uy, uz, w;
};

template <int P>
__device__ __forceinline__ int batch_base0(int beg) {
    return P == 1 ? beg : (beg & ~(P - 1));
}

template <int P>
__device__ __forceinline__ void load_batch(const SpeciesP &S, int base, Batch<P> &b) {
    typedef typename Batch<P>::VF VF;
    typedef typename Batch<P>::VU VU;
    b.c = __builtin_nontemporal_load((const VU *)((const guint *)S.cell + base));
    b.ox = __builtin_nontemporal_load((const VF *)((const gfloat *)S.pos[0] + base));
    b.oy = __builtin_nontemporal_load((const VF *)((const gfloat *)S.pos[1] + base));
    b.oz = __builtin_nontemporal_load((const VF *)((const gfloat *)S.pos[2] + base));
    b.ux = __builtin_nontemporal_load((const VF *)((const gfloat *)S.u[0] + base));
    b.uy = __builtin_nontemporal_load((const VF *)((const gfloat *)S.u[1] + base));
    b.uz = __builtin_nontemporal_load((const VF *)((const gfloat *)S.u[2] + base));
#pragma unroll
    for (int k = 0; k < P; ++k) b.w[k] = 1.f;
    if (S.per_particle_w) b.w = __builtin_nontemporal_load((const VF *)((const gfloat *)S.w + base));
}

// Mid-point and displacement of the second ZigZag segment of a move from
// offset o by dx with cell step dc, relative to the cell + dc: from the relay
// point (the face crossed, or the mid-point of the move on an axis without a
// crossing) to the end o + dx (Sec. 2.5)
__device__ __forceinline__ void second_segment(const float o[3], const float dx[3],
                                               const int dc[3], float WB[3], float DB[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float e = o[a] + dx[a];  // the end point as the move computed it
        const float xr = dc[a] > 0 ? 1.f : 0.f;
        DB[a] = dc[a] != 0 ? e - xr : 0.5f * dx[a];
        WB[a] = dc[a] != 0 ? fmaf(0.5f, xr + e, -(float)dc[a]) : fmaf(0.75f, dx[a], o[a]);
    }
}

// Marks particle (s, p) for k_push_fallback when `outside`: a bit in the
// out-of-window mask, set by an atomic whose result is not waited for (a
// list slot claimed with a returning atomic made every wave with such a
// particle wait for the round trip).  True when marked.
__device__ __forceinline__ bool list_fallback(const FusedArgs &A, bool outside, int s, int p,
                                              unsigned &nfb) {
    if (!outside) return false;
    ++nfb;
    atomicOr(A.fb_mask + (long long)s * A.mask_words + (p >> 5), 1u << (p & 31));
    return true;
}

// Queue of second ZigZag segments (TL::QCAP entries of 32 bytes): per entry
// the particle's offset o and move dx (cell units), a code word (the
// current-window index of its cell in bits 0-10, the cell step + 1 per axis
// in bits 11-16, the species from bit 17) and the weight.
struct SegQueue {
    float4 *q;       // 2 float4 per entry
    unsigned *n;     // entries claimed (may exceed the capacity)
};

// Per-tile constants of the particle loop.
struct TileCtx {
    int wo[3];          // global cell of window point 0 per axis
    uint32_t wo_pack;   // the same, packed (interior tiles only)
};

// One species of one tile: P consecutive particles per thread (one access
// of P elements per array), gather from the LDS field window, Boris (Sec.
// 2.4), move, ZigZag deposit (Sec. 2.5) into the LDS current window; the
// new state goes to the write set.  With use_pre, `pre` holds this thread's
// first batch (the caller issued its loads early).
//
// INTERIOR: the tile's current window lies inside the grid on every axis,
// so that window-relative and new cell indices need no periodic wrap and no
// removal test: both are sums on the packed cell index.
//
// The deposit of a particle that crosses a cell face is split as usual
// (relay point per axis); its first segment is deposited with every other
// particle's move, and its move goes to the workgroup's queue, whose second
// segments are deposited once the tile's particles are done, so that the
// rare crossings do not make every lane of a wave wait for a second
// segment.  A full queue makes the particle deposit its second segment at
// once.
template <class TL, int P, bool INTERIOR>
__device__ __forceinline__ void push_species(const FusedArgs &A, const DevSpecies &D,
                                             const SpeciesP &S, const SpeciesP &Wr, int beg,
                                             int end, const TileCtx &T, const float *sF,
                                             unsigned long long *sJ, const SegQueue &Q, int s,
                                             uint32_t &fbits, unsigned &nfb, const Batch<P> &pre,
                                             bool use_pre) {
    typedef float VF __attribute__((ext_vector_type(P)));
    typedef uint32_t VU __attribute__((ext_vector_type(P)));
    constexpr int FW3 = TL::FW3, FWX = TL::FWX, FWY = TL::FWY, JWX = TL::JWX, JWY = TL::JWY;
    constexpr int LHI_X = TL::LHI_X, LHI_Y = TL::LHI_Y, LHI_Z = TL::LHI_Z;
    const GridP &g = A.g;
    const float r = D.r, r_lo = D.r_lo;
    const double mult[3] = {A.jscale * D.qcd[0], A.jscale * D.qcd[1], A.jscale * D.qcd[2]};
    guint *CQ = (guint *)Wr.cell;
    gfloat *OXQ = (gfloat *)Wr.pos[0], *OYQ = (gfloat *)Wr.pos[1], *OZQ = (gfloat *)Wr.pos[2];
    gfloat *UXQ = (gfloat *)Wr.u[0], *UYQ = (gfloat *)Wr.u[1], *UZQ = (gfloat *)Wr.u[2];
    // per-component window bases, opaque to the compiler so that it keeps one
    // register base per component and puts the eight corner offsets of a
    // gather into the ds_read2 offset fields
    const char *sFc[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        uint32_t o = c * FW3 * 4;
        asm volatile("" : "+s"(o));
        sFc[c] = (const char *)sF + o;
    }
    const int lane = (int)(threadIdx.x & 63);
    const int base0 = batch_base0<P>(beg) + (int)threadIdx.x * P;
    // one (non-temporal) access of P consecutive particles per array; with
    // one particle per thread the batch of the next pass is loaded at the
    // end of this one (the first may come from the caller)
    Batch<P> b;
    if constexpr (P == 1) {
        if (use_pre) b = pre;
        else if (base0 < end) load_batch<P>(S, base0, b);
    }
    for (int base = base0; base < end; base += PUSH_THREADS * P) {
        if constexpr (P != 1) load_batch<P>(S, base, b);
        // a pushed particle's new state replaces its loaded one in the batch
        // registers; one not pushed here keeps its record
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const int p = base + k;
            const uint32_t c = b.c[k];
            if (!(p >= beg && p < end && c != DEAD)) continue;
            // window-relative cell
            int lx, ly, lz;
            if constexpr (INTERIOR) {
                const uint32_t cl = c - T.wo_pack;  // exact for every particle inside the window
                lx = (int)(cl & 0x7FFu);
                ly = (int)((cl >> 11) & 0x7FFu);
                lz = (int)(cl >> 22);
            } else {
                lx = local_axis(g, 0, cell_i(c), T.wo[0]);
                ly = local_axis(g, 1, cell_j(c), T.wo[1]);
                lz = local_axis(g, 2, cell_k(c), T.wo[2]);
            }
            // drifted out of the tile window since the last sort: listed for
            // k_push_fallback
            const bool outside = !((unsigned)(lx - 1) < (unsigned)LHI_X &&
                                   (unsigned)(ly - 1) < (unsigned)LHI_Y &&
                                   (unsigned)(lz - 1) < (unsigned)LHI_Z);
            if (list_fallback(A, outside, s, p, nfb)) continue;
            const float ox = b.ox[k], oy = b.oy[k], oz = b.oz[k];
            // a NaN offset is caught below as a non-finite momentum
            if (!(fminf(fminf(ox, oy), oz) >= 0.f && fmaxf(fmaxf(ox, oy), oz) < 1.f))
                fbits |= EMPIC_FAULT_OFFSET;
            int hx, hy, hz;
            float fx, fy, fz;
            half_axis(ox, lx, hx, fx);
            half_axis(oy, ly, hy, fy);
            half_axis(oz, lz, hz, fz);
            // byte offsets of the node (l) and half (h) positions per axis
            const uint32_t xl = (uint32_t)lx * 4u, xh = (uint32_t)hx * 4u;
            const uint32_t yl = __umul24((uint32_t)ly, FWX * 4), yh = __umul24((uint32_t)hy, FWX * 4);
            const uint32_t zl = __umul24((uint32_t)lz, FWX * FWY * 4),
                           zh = __umul24((uint32_t)hz, FWX * FWY * 4);
            float Ep[3], Bp[3];
            Ep[0] = tri_lds_at<TL>(sFc[0] + (xh + yl + zl), fx, oy, oz);
            Ep[1] = tri_lds_at<TL>(sFc[1] + (xl + yh + zl), ox, fy, oz);
            Ep[2] = tri_lds_at<TL>(sFc[2] + (xl + yl + zh), ox, oy, fz);
            Bp[0] = tri_lds_at<TL>(sFc[3] + (xl + yh + zh), ox, fy, fz);
            Bp[1] = tri_lds_at<TL>(sFc[4] + (xh + yl + zh), fx, oy, fz);
            Bp[2] = tri_lds_at<TL>(sFc[5] + (xh + yh + zl), fx, fy, oz);
            float ux = b.ux[k], uy = b.uy[k], uz = b.uz[k], gam;
            const float ig = boris_f32(ux, uy, uz, Ep, Bp, r, r_lo, gam);
            if (!isfinite(gam)) fbits |= EMPIC_FAULT_NONFINITE;
            const float o[3] = {ox, oy, oz};
            const float dx[3] = {move_cells(ux * ig, A.dtd[0], A.dtd_lo[0]),
                                 move_cells(uy * ig, A.dtd[1], A.dtd_lo[1]),
                                 move_cells(uz * ig, A.dtd[2], A.dtd_lo[2])};
            if (!(fmaxf(fmaxf(fabsf(dx[0]), fabsf(dx[1])), fabsf(dx[2])) < 1.f))
                fbits |= EMPIC_FAULT_FAST;
            float e[3], no[3];
            int dc[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) move_axis_sel(o[a], dx[a], e[a], dc[a], no[a]);
            const float wq = b.w[k];

            const int jb = lx + JWX * (ly + JWY * lz);
            const bool cross = (dc[0] | dc[1] | dc[2]) != 0;
            // first segment: the whole move inside the cell, or from the start
            // to the relay point (Sec. 2.5, ZigZag)
            const float half = cross ? 0.5f : 1.f;
            float WA[3], DA[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const float xr = dc[a] > 0 ? 1.f : 0.f;
                DA[a] = dc[a] != 0 ? xr - o[a] : half * dx[a];
                WA[a] = fmaf(0.5f, DA[a], o[a]);
            }
            lds_add_segment<TL>(sJ, jb, WA, DA, wq, mult);
            // second segment of the crossing particles: from the relay point
            // to the end, in the cell + dc; queued as the move itself (the
            // segment is worked out when the queue is deposited)
            const unsigned long long m = __ballot(cross);
            if (m) {
                bool now = cross;
                if constexpr (TL::QCAP > 0) {
                    unsigned qb = 0;
                    if (lane == __builtin_ctzll(__ballot(1)))
                        qb = atomicAdd(Q.n, (unsigned)__popcll(m));
                    const unsigned slot =
                        __builtin_amdgcn_readfirstlane(qb) +
                        __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                    if (cross && slot < (unsigned)TL::QCAP) {
                        const uint32_t code = (uint32_t)jb | ((uint32_t)(dc[0] + 1) << 11) |
                                              ((uint32_t)(dc[1] + 1) << 13) |
                                              ((uint32_t)(dc[2] + 1) << 15) | ((uint32_t)s << 17);
                        Q.q[2 * slot] = make_float4(o[0], o[1], o[2], __uint_as_float(code));
                        Q.q[2 * slot + 1] = make_float4(dx[0], dx[1], dx[2], wq);
                        now = false;
                    }
                }
                if (now) {
                    float WB[3], DB[3];
                    second_segment(o, dx, dc, WB, DB);
                    lds_add_segment<TL>(sJ, jb + dc[0] + JWX * (dc[1] + JWY * dc[2]), WB, DB, wq,
                                        mult);
                }
            }
            if constexpr (INTERIOR) {
                // inside the grid on every axis: a step of the packed index
                b.c[k] = c + (uint32_t)(dc[0] + (dc[1] << 11) + (dc[2] << 22));
            } else {
                int ni, nj, nk;
                const int in = (int)new_cell(g, 0, cell_i(c), dc[0], ni) &
                               (int)new_cell(g, 1, cell_j(c), dc[1], nj) &
                               (int)new_cell(g, 2, cell_k(c), dc[2], nk);
                b.c[k] = in ? pack_cell(ni, nj, nk) : DEAD;
            }
            b.ox[k] = no[0];
            b.oy[k] = no[1];
            b.oz[k] = no[2];
            b.ux[k] = ux;
            b.uy[k] = uy;
            b.uz[k] = uz;
        }
        if (base >= beg && base + P <= end) {
            __builtin_nontemporal_store(b.c, (VU *)(CQ + base));
            __builtin_nontemporal_store(b.ox, (VF *)(OXQ + base));
            __builtin_nontemporal_store(b.oy, (VF *)(OYQ + base));
            __builtin_nontemporal_store(b.oz, (VF *)(OZQ + base));
            __builtin_nontemporal_store(b.ux, (VF *)(UXQ + base));
            __builtin_nontemporal_store(b.uy, (VF *)(UYQ + base));
            __builtin_nontemporal_store(b.uz, (VF *)(UZQ + base));
        } else {
            // every slot of this tile, removed ones too (a step into another
            // buffer set carries the whole record)
#pragma unroll
            for (int k = 0; k < P; ++k) {
                const int p = base + k;
                if (p < beg || p >= end) continue;
                CQ[p] = b.c[k];
                OXQ[p] = b.ox[k];
                OYQ[p] = b.oy[k];
                OZQ[p] = b.oz[k];
                UXQ[p] = b.ux[k];
                UYQ[p] = b.uy[k];
                UZQ[p] = b.uz[k];
            }
        }
        if constexpr (P == 1)
            if (base + PUSH_THREADS * P < end) load_batch<P>(S, base + PUSH_THREADS * P, b);
    }
}

// 27-point b_2 interpolation from the LDS field window of one component;
// (x, y, z): window index of the stencil's first point (nearest index - 1)
template <class TL>
__device__ __forceinline__ float tri2_lds(const float *F, int x, int y, int z, const float wx[3],
                                          const float wy[3], const float wz[3]) {
    constexpr int FWX = TL::FWX, FWY = TL::FWY;
    const float *p = F + x + FWX * (y + FWY * z);
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        float sy = 0.f;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const float *row = p + FWX * (j + FWY * k);
            sy = fmaf(wy[j], fmaf(wx[2], row[2], fmaf(wx[1], row[1], wx[0] * row[0])), sy);
        }
        s = fmaf(wz[k], sy, s);
    }
    return s;
}

// Order-2 current of a particle into the LDS window (fixed point): one base
// address per part, the constant offsets of its 54 entries folded into the
// LDS instructions
template <class TL>
struct LdsSink2 {
    unsigned long long *sJ;
    int jb;  // window index of the particle's cell
    const double *mult;
    unsigned long long *b = nullptr;
    __device__ __forceinline__ void origin(int x, int y, int z) {
        b = sJ + jb + x + TL::JWX * (y + TL::JWY * z);
    }
    __device__ __forceinline__ void operator()(int c, int x, int y, int z, float v) const {
        atomicAdd(b + c * TL::JW3 + x + TL::JWX * (y + TL::JWY * z),
                  (unsigned long long)to_fixed(v, mult[c]));
    }
};

// One species of one tile with second-order shapes: the b_2 gather from the
// LDS field window, Boris, move, and the EZ current into the LDS window.
// Particles up to MARGIN cells outside their tile, as at first order: the
// field window (one point longer per axis, TileCube2) holds every gather
// stencil; a particle whose move takes its current stencil past the current
// window is left as loaded and marked for k_push_fallback, which pushes it
// through global memory (a second, inlined global deposit here made the
// kernel spill registers).
template <class TL, int P>
__device__ __forceinline__ void push_species2(const FusedArgs &A, const DevSpecies &D,
                                              const SpeciesP &S, const SpeciesP &Wr, int beg,
                                              int end, const TileCtx &T, const float *sF,
                                              unsigned long long *sJ, int s, uint32_t &fbits,
                                              unsigned &nfb) {
    typedef float VF __attribute__((ext_vector_type(P)));
    typedef uint32_t VU __attribute__((ext_vector_type(P)));
    constexpr int FW3 = TL::FW3, JWX = TL::JWX, JWY = TL::JWY;
    const GridP &g = A.g;
    const float r = D.r, r_lo = D.r_lo;
    const double mult[3] = {A.jscale * D.qcd[0], A.jscale * D.qcd[1], A.jscale * D.qcd[2]};
    guint *CQ = (guint *)Wr.cell;
    gfloat *OXQ = (gfloat *)Wr.pos[0], *OYQ = (gfloat *)Wr.pos[1], *OZQ = (gfloat *)Wr.pos[2];
    gfloat *UXQ = (gfloat *)Wr.u[0], *UYQ = (gfloat *)Wr.u[1], *UZQ = (gfloat *)Wr.u[2];
    const int base0 = batch_base0<P>(beg) + (int)threadIdx.x * P;
    Batch<P> b;
    for (int base = base0; base < end; base += PUSH_THREADS * P) {
        load_batch<P>(S, base, b);
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const int p = base + k;
            const uint32_t c = b.c[k];
            if (!(p >= beg && p < end && c != DEAD)) continue;
            const int lx = local_axis(g, 0, cell_i(c), T.wo[0]);
            const int ly = local_axis(g, 1, cell_j(c), T.wo[1]);
            const int lz = local_axis(g, 2, cell_k(c), T.wo[2]);
            const bool outside = !((unsigned)(lx - 1) < (unsigned)TL::LHI_X &&
                                   (unsigned)(ly - 1) < (unsigned)TL::LHI_Y &&
                                   (unsigned)(lz - 1) < (unsigned)TL::LHI_Z);
            if (list_fallback(A, outside, s, p, nfb)) continue;
            const float o[3] = {b.ox[k], b.oy[k], b.oz[k]};
            if (!(fminf(fminf(o[0], o[1]), o[2]) >= 0.f && fmaxf(fmaxf(o[0], o[1]), o[2]) < 1.f))
                fbits |= EMPIC_FAULT_OFFSET;
            const int l[3] = {lx, ly, lz};
            int xn[3], xh[3];  // window index of each stencil's first point
            float wn[3][3], wh[3][3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                int m;
                float d;
                b2_node(o[a], m, d);
                xn[a] = l[a] + m - 1;
                b2_w(d, wn[a]);
                xh[a] = l[a] - 1;
                b2_w(o[a] - 0.5f, wh[a]);
            }
            float Ep[3], Bp[3];
            Ep[0] = tri2_lds<TL>(sF + 0 * FW3, xh[0], xn[1], xn[2], wh[0], wn[1], wn[2]);
            Ep[1] = tri2_lds<TL>(sF + 1 * FW3, xn[0], xh[1], xn[2], wn[0], wh[1], wn[2]);
            Ep[2] = tri2_lds<TL>(sF + 2 * FW3, xn[0], xn[1], xh[2], wn[0], wn[1], wh[2]);
            Bp[0] = tri2_lds<TL>(sF + 3 * FW3, xn[0], xh[1], xh[2], wn[0], wh[1], wh[2]);
            Bp[1] = tri2_lds<TL>(sF + 4 * FW3, xh[0], xn[1], xh[2], wh[0], wn[1], wh[2]);
            Bp[2] = tri2_lds<TL>(sF + 5 * FW3, xh[0], xh[1], xn[2], wh[0], wh[1], wn[2]);
            float ux = b.ux[k], uy = b.uy[k], uz = b.uz[k], gam;
            const float ig = boris_f32(ux, uy, uz, Ep, Bp, r, r_lo, gam);
            if (!isfinite(gam)) fbits |= EMPIC_FAULT_NONFINITE;
            const float dx[3] = {move_cells(ux * ig, A.dtd[0], A.dtd_lo[0]),
                                 move_cells(uy * ig, A.dtd[1], A.dtd_lo[1]),
                                 move_cells(uz * ig, A.dtd[2], A.dtd_lo[2])};
            if (!(fmaxf(fmaxf(fabsf(dx[0]), fabsf(dx[1])), fabsf(dx[2])) < 1.f))
                fbits |= EMPIC_FAULT_FAST;
            // the window indices the current's stencils span (first node
            // m - 1 of the lower cell to m + 1 of the upper, per axis)
            const int JW[3] = {JWX, JWY, TL::JWZ};
            bool fits = true;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int m0 = o[a] >= 0.5f ? 1 : 0;
                const int m1 = (int)floorf(o[a] + dx[a] + 0.5f);
                fits = fits && l[a] + min(m0, m1) - 1 >= 0 && l[a] + max(m0, m1) + 1 < JW[a];
            }
            // a particle whose current leaves the window is pushed again by
            // k_push_fallback from its loaded state (kept here)
            if (list_fallback(A, !fits, s, p, nfb)) continue;
            {
                LdsSink2<TL> sink{sJ, lx + JWX * (ly + JWY * lz), mult};
                ez2_move(o, dx, b.w[k], sink);
            }
            float e[3], no[3];
            int dc[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) move_axis_sel(o[a], dx[a], e[a], dc[a], no[a]);
            int ni, nj, nk;
            const int in = (int)new_cell(g, 0, cell_i(c), dc[0], ni) &
                           (int)new_cell(g, 1, cell_j(c), dc[1], nj) &
                           (int)new_cell(g, 2, cell_k(c), dc[2], nk);
            b.c[k] = in ? pack_cell(ni, nj, nk) : DEAD;
            b.ox[k] = no[0];
            b.oy[k] = no[1];
            b.oz[k] = no[2];
            b.ux[k] = ux;
            b.uy[k] = uy;
            b.uz[k] = uz;
        }
        if (base >= beg && base + P <= end) {
            __builtin_nontemporal_store(b.c, (VU *)(CQ + base));
            __builtin_nontemporal_store(b.ox, (VF *)(OXQ + base));
            __builtin_nontemporal_store(b.oy, (VF *)(OYQ + base));
            __builtin_nontemporal_store(b.oz, (VF *)(OZQ + base));
            __builtin_nontemporal_store(b.ux, (VF *)(UXQ + base));
            __builtin_nontemporal_store(b.uy, (VF *)(UYQ + base));
            __builtin_nontemporal_store(b.uz, (VF *)(UZQ + base));
        } else {
#pragma unroll
            for (int k = 0; k < P; ++k) {
                const int p = base + k;
                if (p < beg || p >= end) continue;
                CQ[p] = b.c[k];
                OXQ[p] = b.ox[k];
                OYQ[p] = b.oy[k];
                OZQ[p] = b.oz[k];
                UXQ[p] = b.ux[k];
                UYQ[p] = b.uy[k];
                UZQ[p] = b.uz[k];
            }
        }
    }
}

template <class TL>
__device__ __forceinline__ void push_tile2(const FusedArgs &A, const TileCtx &T, int tile,
                                           const float *sF, unsigned long long *sJ,
                                           uint32_t &fbits, unsigned &nfb) {
    for (int s = 0; s < A.nsp; ++s) {
        const DevSpecies &D = A.tbl[s];
        const SpeciesP &S = D.p[(A.cur_mask >> s) & 1u];
        const SpeciesP &Wr = D.p[(A.wr_mask >> s) & 1u];
        const int beg = S.tile_off[tile], end = S.tile_off[tile + 1];
        if (beg >= end) continue;
        // two particles per thread in dense tiles: four made the 27-point
        // gathers and the EZ deposit spill registers
        if (end - beg <= 2 * PUSH_THREADS)
            push_species2<TL, 1>(A, D, S, Wr, beg, end, T, sF, sJ, s, fbits, nfb);
        else
            push_species2<TL, 2>(A, D, S, Wr, beg, end, T, sF, sJ, s, fbits, nfb);
    }
}

// Every species of one tile (sparse ones one particle per thread, so that all
// the workgroup's waves work; dense ones four per thread).
template <class TL, bool INTERIOR>
__device__ __forceinline__ void push_tile(const FusedArgs &A, const TileCtx &T, int tile,
                                          bool sparse0, int beg0, int end0, const Batch<1> &pre1,
                                          const float *sF, unsigned long long *sJ,
                                          const SegQueue &Q, uint32_t &fbits, unsigned &nfb) {
    if (sparse0)
        push_species<TL, 1, INTERIOR>(A, A.tbl[0], A.tbl[0].p[A.cur_mask & 1u],
                                      A.tbl[0].p[A.wr_mask & 1u], beg0, end0, T, sF, sJ, Q, 0,
                                      fbits, nfb, pre1, true);
    for (int s = sparse0 ? 1 : 0; s < A.nsp; ++s) {
        const DevSpecies &D = A.tbl[s];
        const SpeciesP &S = D.p[(A.cur_mask >> s) & 1u];
        const SpeciesP &Wr = D.p[(A.wr_mask >> s) & 1u];
        const int beg = S.tile_off[tile], end = S.tile_off[tile + 1];
        if (beg >= end) continue;
        if (end - beg <= 2 * PUSH_THREADS)
            push_species<TL, 1, INTERIOR>(A, D, S, Wr, beg, end, T, sF, sJ, Q, s, fbits, nfb,
                                          pre1, false);
        else
            push_species<TL, PPT, INTERIOR>(A, D, S, Wr, beg, end, T, sF, sJ, Q, s, fbits, nfb,
                                            Batch<PPT>(), false);
    }
}

template <class TL, int ORDER>
__global__ __launch_bounds__(PUSH_THREADS, 4) void k_push_fused(FusedArgs A) {
    constexpr int TX = TL::TX, TY = TL::TY, TZ = TL::TZ;
    constexpr int FWX = TL::FWX, FWY = TL::FWY, FWZ = TL::FWZ, FW3 = TL::FW3;
    constexpr int JWX = TL::JWX, JWY = TL::JWY, JWZ = TL::JWZ, JW3 = TL::JW3;
    constexpr int ROWS = TL::ROWS;
    constexpr int QN = TL::QCAP > 0 ? 2 * TL::QCAP : 1;
    __shared__ float sF[6 * FW3];
    __shared__ __align__(16) unsigned long long sJ[3 * JW3 + 1];
    __shared__ float4 sQ[QN];
    __shared__ unsigned sQn;
    __shared__ unsigned sNfb;  // particles of this tile marked for k_push_fallback
    __shared__ uint32_t sFbits;  // fault bits raised in this tile
    __shared__ int sG[3][ROWS];
    __shared__ int sPad[3][ROWS];

    const GridP &g = A.g;
    const int nb8 = gridDim.x >> 3;
    const int tile = (blockIdx.x & 7) * nb8 + (blockIdx.x >> 3);  // XCD-contiguous tiles
    if (tile >= A.ti.ntiles) return;
    int total = 0;
    for (int s = 0; s < A.nsp; ++s)
        total += A.tbl[s].p[0].tile_off[tile + 1] - A.tbl[s].p[0].tile_off[tile];
    if (total == 0) return;

    // a sparse tile of species 0 (one particle per thread) loads its particles
    // together with the field window: one memory latency for both
    const SpeciesP &S0 = A.tbl[0].p[A.cur_mask & 1u];
    const int beg0 = S0.tile_off[tile], end0 = S0.tile_off[tile + 1];
    const bool sparse0 = ORDER == 1 && end0 > beg0 && end0 - beg0 <= 2 * PUSH_THREADS;
    Batch<1> pre1;
    if (sparse0 && beg0 + (int)threadIdx.x < end0) load_batch<1>(S0, beg0 + (int)threadIdx.x, pre1);

    const int tx = tile % A.ti.nt[0];
    const int tyz = tile / A.ti.nt[0];
    const int ty = tyz % A.ti.nt[1], tz = tyz / A.ti.nt[1];
    TileCtx T;
    T.wo[0] = tx * TX - MARGIN - 1;
    T.wo[1] = ty * TY - MARGIN - 1;
    T.wo[2] = tz * TZ - MARGIN - 1;
    const int JW[3] = {JWX, JWY, JWZ};
    bool interior = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) interior = interior && T.wo[a] >= 0 && T.wo[a] + JW[a] <= g.n[a];
    T.wo_pack = interior ? pack_cell(T.wo[0], T.wo[1], T.wo[2]) : 0u;
    const int tid = threadIdx.x;

    // global index tables of the window rows: x index, y*ext0, z*ext0*ext1
    if (tid == 0) {
        sQn = 0u;
        sNfb = 0u;
        sFbits = 0u;
    }
    if (tid < 3 * ROWS) {
        const int a = tid / ROWS, l = tid % ROWS;
        const int wl = a == 0 ? JWX : (a == 1 ? JWY : JWZ);
        if (l < wl) {
            const int woa = a == 0 ? T.wo[0] : (a == 1 ? T.wo[1] : T.wo[2]);
            const int gi = gaxis(g, a, woa + l);
            const int mul = a == 0 ? 1 : (a == 1 ? g.ext[0] : g.ext[0] * g.ext[1]);
            sG[a][l] = gi < 0 ? -1 : gi * mul;
            sPad[a][l] = (gi >= 0 && g.bc[a] != EMPIC_BC_PERIODIC && gi >= g.n[a]) ? 1 : 0;
        }
    }
    __syncthreads();
    {
        // a thread owns one (x, y) column of the window at every ZG-th z and
        // the same points of all six components: their global offsets are
        // worked out once, and every load is issued before any is waited on
        constexpr int NCOL = FWX * FWY, ZG = PUSH_THREADS / NCOL, NZ = (FWZ + ZG - 1) / ZG;
        const int col = tid % NCOL, zg = tid / NCOL;
        if (zg < ZG) {
            const int ly = col / FWX, lx = col - ly * FWX;
            const int gxy = (sG[0][lx] >= 0 && sG[1][ly] >= 0) ? sG[0][lx] + sG[1][ly] : -1;
            int off[NZ];
#pragma unroll
            for (int q = 0; q < NZ; ++q) {
                const int lz = zg + q * ZG;
                off[q] = (lz < FWZ && gxy >= 0 && sG[2][lz] >= 0) ? gxy + sG[2][lz] : -1;
            }
            float tmp[6][NZ];
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                const float *src = c < 3 ? A.E[c] : A.Bb[c - 3];
#pragma unroll
                for (int q = 0; q < NZ; ++q) tmp[c][q] = off[q] >= 0 ? src[off[q]] : 0.f;
            }
#pragma unroll
            for (int c = 0; c < 6; ++c)
#pragma unroll
                for (int q = 0; q < NZ; ++q) {
                    const int lz = zg + q * ZG;
                    if (lz < FWZ) sF[c * FW3 + col + lz * NCOL] = tmp[c][q];
                }
        }
    }
    {
        // 16-byte stores (the window has an even number of words with its pad)
        uint4 *z4 = (uint4 *)sJ;
        for (int e = tid; e < (3 * JW3 + 1) / 2; e += PUSH_THREADS) z4[e] = make_uint4(0u, 0u, 0u, 0u);
    }
    __syncthreads();

    uint32_t fbits = 0;
    unsigned nfb = 0;
    const SegQueue Q = {sQ, &sQn};
    if constexpr (ORDER == 2)
        push_tile2<TL>(A, T, tile, sF, sJ, fbits, nfb);
    else if (interior)
        push_tile<TL, true>(A, T, tile, sparse0, beg0, end0, pre1, sF, sJ, Q, fbits, nfb);
    else
        push_tile<TL, false>(A, T, tile, sparse0, beg0, end0, pre1, sF, sJ, Q, fbits, nfb);
    // counts and fault bits gathered per workgroup in LDS: a global atomic per
    // thread on these single words serialised the whole step once many
    // particles were out of their windows
    if (fbits) atomicOr(&sFbits, fbits);
    if (nfb) atomicAdd(&sNfb, nfb);
    __syncthreads();
    if constexpr (TL::QCAP > 0 && ORDER == 1) {
        // the queued second segments
        static_assert(TL::JW3 <= 2048, "window index in the 11 bits of a queue entry's code");
        const int nq = (int)min(sQn, (unsigned)TL::QCAP);
        for (int q = tid; q < nq; q += PUSH_THREADS) {
            const float4 a = sQ[2 * q], bq = sQ[2 * q + 1];
            const uint32_t code = __float_as_uint(a.w);
            const int dc[3] = {(int)((code >> 11) & 3u) - 1, (int)((code >> 13) & 3u) - 1,
                               (int)((code >> 15) & 3u) - 1};
            const double *qcd = A.tbl[code >> 17].qcd;
            const double mult[3] = {A.jscale * qcd[0], A.jscale * qcd[1], A.jscale * qcd[2]};
            const float o[3] = {a.x, a.y, a.z}, dx[3] = {bq.x, bq.y, bq.z};
            float WB[3], DB[3];
            second_segment(o, dx, dc, WB, DB);
            lds_add_segment<TL>(sJ, (int)(code & 0x7FFu) + dc[0] + JWX * (dc[1] + JWY * dc[2]),
                                WB, DB, bq.w, mult);
        }
        __syncthreads();
    }
    // add the tile's current to the global fixed-point sums (non-zero entries
    // only: integer adds, so the sums do not depend on their order); a thread
    // owns one (x, y) column of the window at every ZG-th z, the same points
    // of the three components
    {
        constexpr int NCOL = JWX * JWY, ZG = PUSH_THREADS / NCOL, NZ = (JWZ + ZG - 1) / ZG;
        const int col = tid % NCOL, zg = tid / NCOL;
        if (zg < ZG) {
            const int ly = col / JWX, lx = col - ly * JWX;
            const int gx = sG[0][lx], gy = sG[1][ly];
            const bool skip0 = sPad[0][lx] != 0, skip1 = sPad[1][ly] != 0;
            if (gx >= 0 && gy >= 0) {
#pragma unroll
                for (int q = 0; q < NZ; ++q) {
                    const int lz = zg + q * ZG;
                    if (lz >= JWZ) break;
                    const int gz = sG[2][lz];
                    if (gz < 0) continue;
                    const int r = col + lz * NCOL;
                    const bool skip[3] = {skip0, skip1, sPad[2][lz] != 0};
#pragma unroll
                    for (int comp = 0; comp < 3; ++comp) {
                        const long long fx = (long long)sJ[comp * JW3 + r];
                        if (fx == 0 || skip[comp]) continue;
                        atomicAdd(A.Jf[comp] + gx + gy + gz, (unsigned long long)fx);
                    }
                }
            }
        }
    }
    // a tile with marked particles lists itself for k_push_fallback (last, so
    // that no wave waits for this returning atomic before its own work)
    if (tid == 0) {
        if (sFbits | sNfb) atomicOr(A.fault, sFbits | (sNfb ? EMPIC_FAULT_FALLBACK : 0u));
        if (sNfb) {
            atomicAdd(A.fallback, (unsigned long long)sNfb);
            atomicAdd(A.fb_count, sNfb);
            A.fb_tiles[atomicAdd(A.fb_count + 2, 1u)] = tile;
        }
    }
}

// Out-of-window particles of this step, whole particle through global memory
// (gather from E and Bbar, global atomic deposit).  A thread takes one mask
// word of a listed tile's slot range (flat over the listed tiles, so that
// all of them are scanned at once rather than one after another per
// workgroup), keeps the bits inside the range (a word can straddle two
// tiles), clears them and pushes their particles.  The counts and the tile
// list are cleared by the next step's Faraday kernel (a ticket for the last
// workgroup, a returning atomic of every workgroup on one word, cost more
// than the pass itself in most steps).
constexpr int FB_WPT = 160;  // words per item stride: the 129 of a 4096-particle tile
template <int ORDER>
__global__ __launch_bounds__(256) void k_push_fallback(FusedArgs A) {
    if (A.publish && blockIdx.x == 0 && threadIdx.x == 0) {
        // every tile workgroup of this step has finished: the count is final
        *(volatile unsigned long long *)A.publish = *(volatile unsigned long long *)A.fallback;
        __threadfence_system();
    }
    const unsigned ntl = *(volatile unsigned *)(A.fb_count + 2);
    uint32_t fbits = 0;
    // items (listed tile, word j < FB_WPT); a tile with more words takes
    // them FB_WPT apart
    const long long items = (long long)ntl * FB_WPT;
    for (long long it = blockIdx.x * (long long)blockDim.x + threadIdx.x; it < items;
         it += (long long)gridDim.x * blockDim.x)
    for (int s = 0; s < A.nsp; ++s) {
        const int j = (int)(it % FB_WPT);
        const int tile = A.fb_tiles[it / FB_WPT];
        const DevSpecies &D = A.tbl[s];
        const SpeciesP &S = D.p[(A.cur_mask >> s) & 1u];
        const SpeciesP &Wr = D.p[(A.wr_mask >> s) & 1u];
        const int beg = S.tile_off[tile], end = S.tile_off[tile + 1];
        if (beg >= end) continue;
        const int w0 = beg >> 5, w1 = (end - 1) >> 5;
        for (int w = w0 + j; w <= w1; w += FB_WPT) {
        const int lo = w == w0 ? (beg & 31) : 0, hi = w == w1 ? ((end - 1) & 31) : 31;
        const uint32_t range = (0xffffffffu >> (31 - hi)) & (0xffffffffu << lo);
        uint32_t *mw = A.fb_mask + (long long)s * A.mask_words + w;
        uint32_t bits = *mw & range;
        if (!bits) continue;
        atomicAnd(mw, ~bits);
        const int p0 = w * 32;
        while (bits) {
            const int p = p0 + __builtin_ctz(bits);
            bits &= bits - 1u;
            uint32_t c = S.cell[p];
            float ox = ((float *)S.pos[0])[p], oy = ((float *)S.pos[1])[p],
                  oz = ((float *)S.pos[2])[p];
            float ux = ((float *)S.u[0])[p], uy = ((float *)S.u[1])[p], uz = ((float *)S.u[2])[p];
            const float wq = (S.per_particle_w && S.w) ? ((const float *)S.w)[p] : 1.f;
            particle_global<ORDER>(A, D, c, ox, oy, oz, ux, uy, uz, wq, fbits);
            Wr.cell[p] = c;
            ((float *)Wr.pos[0])[p] = ox;
            ((float *)Wr.pos[1])[p] = oy;
            ((float *)Wr.pos[2])[p] = oz;
            ((float *)Wr.u[0])[p] = ux;
            ((float *)Wr.u[1])[p] = uy;
            ((float *)Wr.u[2])[p] = uz;
        }
        }
    }
    if (fbits) atomicOr(A.fault, fbits);
}

// ---------------------------------------------------------------------------
// Diagnostics and conversions (one thread per particle slot)
// ---------------------------------------------------------------------------
__global__ void k_dry_push_f32(GridP g, const float *Ex, const float *Ey, const float *Ez,
                               const float *Bx, const float *By, const float *Bz, SpeciesP sp,
                               float r, float r_lo, double *partial, uint32_t *fault) {
    __shared__ double sm[16];
    const float *E[3] = {Ex, Ey, Ez};
    const float *Bb[3] = {Bx, By, Bz};
    const long long count = *sp.count;
    const float *WP = (sp.per_particle_w && sp.w) ? (const float *)sp.w : nullptr;
    double ks = 0.0;
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < count;
         p += (long long)gridDim.x * blockDim.x) {
        const uint32_t c = sp.cell[p];
        if (c == DEAD) continue;
        const float ox = ((const float *)sp.pos[0])[p], oy = ((const float *)sp.pos[1])[p],
                    oz = ((const float *)sp.pos[2])[p];
        float ux = ((const float *)sp.u[0])[p], uy = ((const float *)sp.u[1])[p],
              uz = ((const float *)sp.u[2])[p];
        float Ep[3], Bp[3];
        if (g.shape_order == 2)
            gather2_global(g, E, Bb, cell_i(c), cell_j(c), cell_k(c), ox, oy, oz, Ep, Bp);
        else
            gather_global(g, E, Bb, cell_i(c), cell_j(c), cell_k(c), ox, oy, oz, Ep, Bp);
        float gam;
        boris_f32(ux, uy, uz, Ep, Bp, r, r_lo, gam);
        if (!isfinite(gam)) atomicOr(fault, (uint32_t)EMPIC_FAULT_NONFINITE);
        const double uu = (double)ux * ux + (double)uy * uy + (double)uz * uz;
        const double wp = WP ? (double)WP[p] : sp.w_species;
        ks += wp * sp.m * uu / (sqrt(1.0 + uu) + 1.0);
    }
    const double t = block_reduce<false>(ks, sm);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ void k_kinetic_f32(SpeciesP sp, double *partial) {
    __shared__ double sm[16];
    const long long count = *sp.count;
    const float *WP = (sp.per_particle_w && sp.w) ? (const float *)sp.w : nullptr;
    double ks = 0.0;
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < count;
         p += (long long)gridDim.x * blockDim.x) {
        if (sp.cell[p] == DEAD) continue;
        const double ux = ((const float *)sp.u[0])[p], uy = ((const float *)sp.u[1])[p],
                     uz = ((const float *)sp.u[2])[p];
        const double uu = ux * ux + uy * uy + uz * uz;
        const double wp = WP ? (double)WP[p] : sp.w_species;
        ks += wp * sp.m * uu / (sqrt(1.0 + uu) + 1.0);
    }
    const double t = block_reduce<false>(ks, sm);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// b_2 charge density at nodes (second-order shapes), FP64 global atomics
__global__ void k_rho2_f32(GridP g, SpeciesP sp, double *rho) {
    const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (p >= *sp.count) return;
    const uint32_t c = sp.cell[p];
    if (c == DEAD) return;
    const float *WP = (sp.per_particle_w && sp.w) ? (const float *)sp.w : nullptr;
    const double dV = g.d[0] * g.d[1] * g.d[2];
    const double qsp = sp.q * (WP ? (double)WP[p] : sp.w_species);
    const int ci[3] = {cell_i(c), cell_j(c), cell_k(c)};
    int m[3];
    double w[3][3];
    for (int a = 0; a < 3; ++a) {
        const double o = ((const float *)sp.pos[a])[p];
        m[a] = ci[a] + (o >= 0.5 ? 1 : 0);
        const double d = o - (o >= 0.5 ? 1.0 : 0.0);
        w[a][0] = 0.5 * (0.5 - d) * (0.5 - d);
        w[a][1] = 0.75 - d * d;
        w[a][2] = 0.5 * (0.5 + d) * (0.5 + d);
    }
    for (int k = 0; k < 3; ++k) {
        const int gz = gaxis(g, 2, m[2] - 1 + k);
        if (gz < 0) continue;
        for (int j = 0; j < 3; ++j) {
            const int gy = gaxis(g, 1, m[1] - 1 + j);
            if (gy < 0) continue;
            for (int i = 0; i < 3; ++i) {
                const int gx = gaxis(g, 0, m[0] - 1 + i);
                if (gx < 0) continue;
                atomicAdd(rho + gx + (long long)g.ext[0] * (gy + (long long)g.ext[1] * gz),
                          qsp / dV * w[0][i] * w[1][j] * w[2][k]);
            }
        }
    }
}

__global__ void k_rho_f32(GridP g, SpeciesP sp, double *rho) {
    const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (p >= *sp.count) return;
    const uint32_t c = sp.cell[p];
    if (c == DEAD) return;
    const float *WP = (sp.per_particle_w && sp.w) ? (const float *)sp.w : nullptr;
    const double dV = g.d[0] * g.d[1] * g.d[2];
    const double qsp = sp.q * (WP ? (double)WP[p] : sp.w_species);
    const int ci[3] = {cell_i(c), cell_j(c), cell_k(c)};
    const double f[3] = {((const float *)sp.pos[0])[p], ((const float *)sp.pos[1])[p],
                         ((const float *)sp.pos[2])[p]};
    for (int o = 0; o < 8; ++o) {
        const int ox = o & 1, oy = (o >> 1) & 1, oz = o >> 2;
        const int gx = gaxis(g, 0, ci[0] + ox), gy = gaxis(g, 1, ci[1] + oy),
                  gz = gaxis(g, 2, ci[2] + oz);
        if (gx < 0 || gy < 0 || gz < 0) continue;
        const double wt = (ox ? f[0] : 1.0 - f[0]) * (oy ? f[1] : 1.0 - f[1]) *
                          (oz ? f[2] : 1.0 - f[2]);
        atomicAdd(rho + gx + (long long)g.ext[0] * (gy + (long long)g.ext[1] * gz), qsp / dV * wt);
    }
}

// CIC rho of particles still grouped by the tiles of the last sort: one
// workgroup per tile accumulates its particles in an LDS window of nodes as
// int64 fixed point (scale: one contribution <= 2^48), then adds the window
// to the global FP64 array, one atomic per touched node instead of eight per
// particle.  Particles that drifted out of the window add their eight
// contributions directly.
template <class TL>
__global__ __launch_bounds__(256) void k_rho_tiles(GridP g, TileInfo ti, SpeciesP sp,
                                                   double scale, double *rho) {
    constexpr int TX = TL::TX, TY = TL::TY, TZ = TL::TZ;
    constexpr int FWX = TL::FWX, FWY = TL::FWY, FWZ = TL::FWZ, FW3 = TL::FW3, ROWS = TL::ROWS;
    constexpr int LHI_X = TL::LHI_X, LHI_Y = TL::LHI_Y, LHI_Z = TL::LHI_Z;
    __shared__ unsigned long long acc[FW3];
    __shared__ int sG[3][ROWS];
    const int nb8 = gridDim.x >> 3;
    const int tile = (blockIdx.x & 7) * nb8 + (blockIdx.x >> 3);  // XCD-contiguous tiles
    if (tile >= ti.ntiles) return;
    const int beg = sp.tile_off[tile], end = sp.tile_off[tile + 1];
    if (beg >= end) return;
    const int tx = tile % ti.nt[0];
    const int tyz = tile / ti.nt[0];
    const int ty = tyz % ti.nt[1], tz = tyz / ti.nt[1];
    const int wo[3] = {tx * TX - MARGIN - 1, ty * TY - MARGIN - 1, tz * TZ - MARGIN - 1};
    const int tid = threadIdx.x;
    if (tid < 3 * ROWS) {
        const int a = tid / ROWS, l = tid % ROWS;
        const int wl = a == 0 ? FWX : (a == 1 ? FWY : FWZ);
        if (l < wl) {
            const int gi = gaxis(g, a, wo[a] + l);
            const int mul = a == 0 ? 1 : (a == 1 ? g.ext[0] : g.ext[0] * g.ext[1]);
            sG[a][l] = gi < 0 ? -1 : gi * mul;
        }
    }
    for (int e = tid; e < FW3; e += 256) acc[e] = 0ull;
    __syncthreads();
    const float *WP = (sp.per_particle_w && sp.w) ? (const float *)sp.w : nullptr;
    const double dV = g.d[0] * g.d[1] * g.d[2];
    for (int p = beg + tid; p < end; p += 256) {
        const uint32_t c = sp.cell[p];
        if (c == DEAD) continue;
        const double amp = sp.q * (WP ? (double)WP[p] : sp.w_species) / dV;
        const int ci[3] = {cell_i(c), cell_j(c), cell_k(c)};
        const double f[3] = {((const float *)sp.pos[0])[p], ((const float *)sp.pos[1])[p],
                             ((const float *)sp.pos[2])[p]};
        const int lx = local_axis(g, 0, ci[0], wo[0]), ly = local_axis(g, 1, ci[1], wo[1]),
                  lz = local_axis(g, 2, ci[2], wo[2]);
        const bool inwin =
            lx >= 1 && lx <= LHI_X && ly >= 1 && ly <= LHI_Y && lz >= 1 && lz <= LHI_Z;
        for (int o = 0; o < 8; ++o) {
            const int ox = o & 1, oy = (o >> 1) & 1, oz = o >> 2;
            const double wt = (ox ? f[0] : 1.0 - f[0]) * (oy ? f[1] : 1.0 - f[1]) *
                              (oz ? f[2] : 1.0 - f[2]);
            if (inwin) {
                const long long v = __double2ll_rn(amp * wt * scale);
                atomicAdd(acc + (lx + ox) + FWX * ((ly + oy) + FWY * (lz + oz)),
                          (unsigned long long)v);
            } else {
                const int gx = gaxis(g, 0, ci[0] + ox), gy = gaxis(g, 1, ci[1] + oy),
                          gz = gaxis(g, 2, ci[2] + oz);
                if (gx < 0 || gy < 0 || gz < 0) continue;
                atomicAdd(rho + gx + (long long)g.ext[0] * (gy + (long long)g.ext[1] * gz), amp * wt);
            }
        }
    }
    __syncthreads();
    const double inv = 1.0 / scale;
    for (int e = tid; e < FW3; e += 256) {
        const long long v = (long long)acc[e];
        if (v == 0) continue;
        const int lz = e / (FWX * FWY);
        const int r = e - lz * (FWX * FWY);
        const int ly = r / FWX, lx = r - ly * FWX;
        const int gx = sG[0][lx], gy = sG[1][ly], gz = sG[2][lz];
        if (gx < 0 || gy < 0 || gz < 0) continue;
        atomicAdd(rho + gx + gy + gz, (double)v * inv);
    }
}

// FP64 global positions -> packed cell + FP32 offset (on the device)
__global__ void k_load_f32(GridP g, SpeciesP sp, long long count, const double *pos,
                           const double *u, const double *w, const int32_t *ids, uint32_t *fault) {
    const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (p == 0) *sp.count = (int32_t)count;
    if (p >= count) return;
    int ci[3];
    float off[3];
    bool ok = true;
    for (int a = 0; a < 3; ++a) {
        const double xi = pos[3 * p + a] / g.d[a];
        const double fl = floor(xi);
        int i = (int)fl;
        float o = (float)(xi - fl);
        if (o >= 1.f) {
            o = 0.f;
            i += 1;
            if (g.bc[a] == EMPIC_BC_PERIODIC && i == g.n[a]) i = 0;
        }
        if (!(xi >= 0.0) || i < 0 || i >= g.n[a]) ok = false;
        ci[a] = i;
        off[a] = o;
    }
    if (!ok) atomicOr(fault, (uint32_t)EMPIC_FAULT_CELL);
    sp.cell[p] = ok ? pack_cell(ci[0], ci[1], ci[2]) : DEAD;
    for (int a = 0; a < 3; ++a) {
        ((float *)sp.pos[a])[p] = off[a];
        ((float *)sp.u[a])[p] = (float)u[3 * p + a];
    }
    sp.id[p] = ids ? ids[p] : (int32_t)p;
    if (sp.w && w) ((float *)sp.w)[p] = (float)w[p];
}

__global__ void k_store_f32(GridP g, SpeciesP sp, double *pos, double *u, int32_t *ids) {
    const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (p >= *sp.count) return;
    const uint32_t c = sp.cell[p];
    const int ci[3] = {cell_i(c), cell_j(c), cell_k(c)};
    for (int a = 0; a < 3; ++a) {
        pos[3 * p + a] = c == DEAD ? __builtin_nan("")
                                   : ((double)ci[a] + (double)((const float *)sp.pos[a])[p]) * g.d[a];
        u[3 * p + a] = (double)((const float *)sp.u[a])[p];
    }
    if (ids) ids[p] = c == DEAD ? -1 : sp.id[p];
}

// ---------------------------------------------------------------------------
// Counting sort by (tile, cell): rank within key from the histogram atomics,
// exclusive scan of the key counts, scatter into the other buffer set.
// ---------------------------------------------------------------------------
// Every lane of a wave takes part (no early exit before the shuffles):
// consecutive lanes with the same key (particles still in cell order, as
// generated or as left by a previous sort) take their ranks from one atomic
// of their run's first lane.
__global__ void k_sort_count(TileInfo ti, GridP g, SpeciesP sp, int32_t *counts, int32_t *rank,
                             uint32_t *fault) {
    const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const bool in = p < *sp.count;
    long long key = -1;
    if (in) {
        const uint32_t c = sp.cell[p];
        const int i = cell_i(c), j = cell_j(c), k = cell_k(c);
        if (c != DEAD) {
            if (i >= g.n[0] || j >= g.n[1] || k >= g.n[2])
                atomicOr(fault, (uint32_t)EMPIC_FAULT_CELL);
            else
                key = sort_key(ti, i, j, k);
        }
        if (key < 0) rank[p] = -1;
    }
    const int lane = (int)(threadIdx.x & 63);
    const long long prev = __shfl_up(key, 1u, 64);
    const bool head = key >= 0 && (lane == 0 || prev != key);
    const unsigned long long heads = __ballot(head);
    const unsigned long long stops = heads | ~__ballot(key >= 0);  // lanes that end a run
    int base = 0;
    if (head) {
        const unsigned long long above = lane == 63 ? 0ull : stops & (~0ull << (lane + 1));
        const int e = above ? __builtin_ctzll(above) : 64;
        base = atomicAdd(counts + key, e - lane);
    }
    // the first lane of this lane's run: the highest head at or below it
    const unsigned long long upto = heads & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull));
    const int h = upto ? 63 - __builtin_clzll(upto) : lane;
    base = __shfl(base, h, 64);
    if (key >= 0) rank[p] = base + (lane - h);
}

// Counting pass when the particles are still grouped by the tiles of the
// previous sort (the usual case): one workgroup per old tile ranks the
// particles that stayed in the tile with LDS atomics, then reserves each
// key's range with one global atomic; particles that moved to another tile
// take a global atomic directly.  rank: >= 0 final, -1 removed, <= -2 local
// rank (-2 - r) awaiting its key's base.
constexpr int SORT_T = 512;
constexpr int SCAT_NS = 9;                    // particles per thread of a tile held in registers
constexpr int SCAT_CAP = SORT_T * SCAT_NS;    // 4608: the largest tile handled that way
__global__ __launch_bounds__(SORT_T) void k_sort_count_tiles(TileInfo ti, GridP g, SpeciesP sp,
                                                             int32_t *counts, int32_t *rank,
                                                             uint32_t *fault) {
    __shared__ int hist[TC];
    __shared__ int basek[TC];
    const int t = blockIdx.x;
    const int beg = sp.tile_off[t], end = sp.tile_off[t + 1];
    if (beg >= end) return;
    for (int l = threadIdx.x; l < TC; l += SORT_T) hist[l] = 0;
    __syncthreads();
    const long long t0 = (long long)t * TC;
    if (end - beg <= SORT_T * SCAT_NS) {
        // the tile's particles fit SCAT_NS per thread: cells loaded at once,
        // local ranks kept in registers for the final pass
        int kl[SCAT_NS], lr[SCAT_NS];  // key within the tile (-1: none), local rank
#pragma unroll
        for (int k = 0; k < SCAT_NS; ++k) {
            const int p = beg + (int)threadIdx.x + k * SORT_T;
            kl[k] = -1;
            lr[k] = 0;
            if (p >= end) continue;
            const uint32_t c = sp.cell[p];
            const int i = cell_i(c), j = cell_j(c), kk = cell_k(c);
            if (c == DEAD || i >= g.n[0] || j >= g.n[1] || kk >= g.n[2]) {
                if (c != DEAD) atomicOr(fault, (uint32_t)EMPIC_FAULT_CELL);
                rank[p] = -1;
                continue;
            }
            const long long key = sort_key(ti, i, j, kk);
            if (key >= t0 && key < t0 + TC) {
                kl[k] = (int)(key - t0);
                lr[k] = atomicAdd(hist + kl[k], 1);
            } else {
                rank[p] = atomicAdd(counts + key, 1);
            }
        }
        __syncthreads();
        for (int l = threadIdx.x; l < TC; l += SORT_T)
            basek[l] = hist[l] ? atomicAdd(counts + t0 + l, hist[l]) : 0;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < SCAT_NS; ++k)
            if (kl[k] >= 0) rank[beg + (int)threadIdx.x + k * SORT_T] = basek[kl[k]] + lr[k];
        return;
    }
    for (int p = beg + threadIdx.x; p < end; p += SORT_T) {
        const uint32_t c = sp.cell[p];
        if (c == DEAD) {
            rank[p] = -1;
            continue;
        }
        const int i = cell_i(c), j = cell_j(c), k = cell_k(c);
        if (i >= g.n[0] || j >= g.n[1] || k >= g.n[2]) {
            atomicOr(fault, (uint32_t)EMPIC_FAULT_CELL);
            rank[p] = -1;
            continue;
        }
        const long long key = sort_key(ti, i, j, k);
        if (key >= t0 && key < t0 + TC)
            rank[p] = -2 - atomicAdd(hist + (key - t0), 1);
        else
            rank[p] = atomicAdd(counts + key, 1);
    }
    __syncthreads();
    for (int l = threadIdx.x; l < TC; l += SORT_T)
        basek[l] = hist[l] ? atomicAdd(counts + t0 + l, hist[l]) : 0;
    __syncthreads();
    for (int p = beg + threadIdx.x; p < end; p += SORT_T) {
        const int r = rank[p];
        if (r > -2) continue;
        const uint32_t c = sp.cell[p];
        const long long key = sort_key(ti, cell_i(c), cell_j(c), cell_k(c));
        rank[p] = basek[key - t0] + (-2 - r);
    }
}

constexpr int SCAN_T = 256, SCAN_PER = 4, SCAN_B = SCAN_T * SCAN_PER;

__device__ inline int block_exclusive_scan(int v, int *sm, int &total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) sm[wid] = x;
    __syncthreads();
    int off = 0;
    total = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
        if (w < wid) off += sm[w];
        total += sm[w];
    }
    __syncthreads();
    return off + x - v;
}

__global__ void k_scan_reduce(const int32_t *counts, long long NK, int32_t *bsum) {
    __shared__ int sm[16];
    const long long base = (long long)blockIdx.x * SCAN_B;
    int s = 0;
    for (int q = 0; q < SCAN_PER; ++q) {
        const long long i = base + threadIdx.x * SCAN_PER + q;
        if (i < NK) s += counts[i];
    }
    int total;
    block_exclusive_scan(s, sm, total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ void k_scan_blocks(int32_t *bsum, int nb, int32_t *counts, long long NK) {
    __shared__ int sm[16];
    int carry = 0;
    for (int base = 0; base < nb; base += SCAN_T) {
        const int i = base + threadIdx.x;
        const int v = i < nb ? bsum[i] : 0;
        int total;
        const int ex = block_exclusive_scan(v, sm, total);
        if (i < nb) bsum[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) counts[NK] = carry;  // total number of live particles
}

__global__ void k_scan_down(int32_t *counts, long long NK, const int32_t *bsum) {
    __shared__ int sm[16];
    const long long base = (long long)blockIdx.x * SCAN_B + threadIdx.x * SCAN_PER;
    int v[SCAN_PER], s = 0;
    for (int q = 0; q < SCAN_PER; ++q) {
        v[q] = base + q < NK ? counts[base + q] : 0;
        s += v[q];
    }
    int total;
    int ex = block_exclusive_scan(s, sm, total) + bsum[blockIdx.x];
    for (int q = 0; q < SCAN_PER; ++q) {
        if (base + q < NK) counts[base + q] = ex;
        ex += v[q];
    }
}

__global__ void k_sort_scatter(TileInfo ti, SpeciesP cur, SpeciesP alt, const int32_t *offs,
                               const int32_t *rank, int32_t *perm) {
    const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (p >= *cur.count) return;
    const int rk = rank[p];
    if (rk < 0) return;
    const uint32_t c = cur.cell[p];
    const long long dst = offs[sort_key(ti, cell_i(c), cell_j(c), cell_k(c))] + rk;
    alt.cell[dst] = c;
    for (int a = 0; a < 3; ++a) {
        ((float *)alt.pos[a])[dst] = ((const float *)cur.pos[a])[p];
        ((float *)alt.u[a])[dst] = ((const float *)cur.u[a])[p];
    }
    alt.id[dst] = cur.id[p];
    if (cur.w && alt.w) ((float *)alt.w)[dst] = ((const float *)cur.w)[p];
    if (perm) perm[dst] = (int32_t)p;
}

// Scatter pass after k_sort_count_tiles: one workgroup per old tile.  The
// particles that stay in their tile (most of them between sorts) reach
// their new slots through LDS, so that both the reads of the old range and
// the writes of the new range are coalesced: each thread loads every array
// of its old slots at once, then one array at a time goes to LDS in the old
// order and out in the new order.  Particles that moved to another tile are
// written straight to their slots (the slots of the new range that they
// fill are skipped by their new tile's workgroup), and so is every particle
// of a tile whose old or new range exceeds the LDS staging.
__global__ __launch_bounds__(SORT_T) void k_sort_scatter_tiles(TileInfo ti, SpeciesP cur,
                                                               SpeciesP alt, const int32_t *offs,
                                                               const int32_t *rank,
                                                               int32_t *perm) {
    __shared__ uint32_t buf[SCAT_CAP];
    __shared__ int src_of[SCAT_CAP];  // new slot -> old slot of a stayer, -1: filled elsewhere
    const int t = blockIdx.x, tid = threadIdx.x;
    const int beg = cur.tile_off[t], end = cur.tile_off[t + 1];
    const int n_old = end - beg;
    if (n_old <= 0) return;
    const long long t0 = (long long)t * TC;
    const int nb = offs[t0], n_new = offs[t0 + TC] - nb;
    const bool has_w = cur.w && alt.w;
    const uint32_t *S[9] = {cur.cell, (const uint32_t *)cur.pos[0], (const uint32_t *)cur.pos[1],
                            (const uint32_t *)cur.pos[2], (const uint32_t *)cur.u[0],
                            (const uint32_t *)cur.u[1], (const uint32_t *)cur.u[2],
                            (const uint32_t *)cur.id, (const uint32_t *)cur.w};
    uint32_t *D[9] = {alt.cell, (uint32_t *)alt.pos[0], (uint32_t *)alt.pos[1],
                      (uint32_t *)alt.pos[2], (uint32_t *)alt.u[0], (uint32_t *)alt.u[1],
                      (uint32_t *)alt.u[2], (uint32_t *)alt.id, (uint32_t *)alt.w};
    if (n_old > SCAT_CAP || n_new > SCAT_CAP) {
        for (int p = beg + tid; p < end; p += SORT_T) {
            const int rk = rank[p];
            if (rk < 0) continue;
            const uint32_t c = cur.cell[p];
            const long long d = offs[sort_key(ti, cell_i(c), cell_j(c), cell_k(c))] + rk;
#pragma unroll
            for (int a = 0; a < 9; ++a)
                if (a < 8 || has_w) D[a][d] = S[a][p];
            if (perm) perm[d] = p;
        }
        return;
    }
    for (int j = tid; j < n_new; j += SORT_T) src_of[j] = -1;
    uint32_t v[9][SCAT_NS];
    int rk[SCAT_NS];
#pragma unroll
    for (int k = 0; k < SCAT_NS; ++k) {
        const int i = tid + k * SORT_T;
        rk[k] = -1;
        if (i < n_old) {
            rk[k] = rank[beg + i];
#pragma unroll
            for (int a = 0; a < 9; ++a)
                if (a < 8 || has_w) v[a][k] = S[a][beg + i];
        }
    }
    __syncthreads();  // src_of cleared
#pragma unroll
    for (int k = 0; k < SCAT_NS; ++k) {
        const int i = tid + k * SORT_T;
        if (i >= n_old || rk[k] < 0) continue;
        const uint32_t c = v[0][k];
        const long long d = offs[sort_key(ti, cell_i(c), cell_j(c), cell_k(c))] + rk[k];
        if (d >= nb && d < (long long)nb + n_new) {
            src_of[d - nb] = i;
        } else {
#pragma unroll
            for (int a = 0; a < 9; ++a)
                if (a < 8 || has_w) D[a][d] = v[a][k];
            if (perm) perm[d] = beg + i;
        }
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        if (a < 8 || has_w) {  // uniform across the workgroup
#pragma unroll
            for (int k = 0; k < SCAT_NS; ++k) {
                const int i = tid + k * SORT_T;
                if (i < n_old) buf[i] = v[a][k];
            }
            __syncthreads();
            for (int j = tid; j < n_new; j += SORT_T) {
                const int o = src_of[j];
                if (o >= 0) D[a][nb + j] = buf[o];
            }
            __syncthreads();
        }
    }
    if (perm)
        for (int j = tid; j < n_new; j += SORT_T) {
            const int o = src_of[j];
            if (o >= 0) perm[nb + j] = beg + o;
        }
}

__global__ void k_tile_offsets(const int32_t *offs, long long NK, int ntiles, int32_t *tile_off,
                               int32_t *count) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t > ntiles) return;
    tile_off[t] = t == ntiles ? offs[NK] : offs[(long long)t * TC];
    if (t == ntiles) *count = offs[NK];
}

__global__ void k_fill_i32(int32_t *p, long long n, int32_t v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

inline unsigned nblk(long long n, int t) { return (unsigned)((n + t - 1) / t); }

__global__ void k_write_species(DevSpecies *dst, DevSpecies v) { *dst = v; }

// moving window: the cell index of every particle moves `cells` back along
// ax (offsets are relative to the cell and do not change); below 0: removed
__global__ void k_window_particles(SpeciesP sp, int ax, int cells) {
    const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (p >= *sp.count) return;
    const uint32_t c = sp.cell[p];
    if (c == DEAD) return;
    int v[3] = {cell_i(c), cell_j(c), cell_k(c)};
    v[ax] -= cells;
    sp.cell[p] = v[ax] < 0 ? DEAD : pack_cell(v[0], v[1], v[2]);
}

// reserve m slots after the current count (one thread)
__global__ void k_inject_reserve(int32_t *count, long long cap, long long m, int32_t *reserve,
                                 uint32_t *fault) {
    const long long base = *count;
    if (base + m <= cap) {
        *count = (int32_t)(base + m);
        *reserve = (int32_t)base;
    } else {
        *reserve = -1;
        atomicOr(fault, (uint32_t)EMPIC_FAULT_CAPACITY);
    }
}

// cold particles on a quiet lattice in cells [lo, lo + nc): per axis
// (m + 1/2)/per offsets; x fastest, then y, then z over the lattice points
__global__ void k_inject(SpeciesP sp, int lo0, int lo1, int lo2, int nx, int ny, int nz, int px,
                         int py, int pz, float w, int next_id, const int32_t *reserve) {
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long NX = (long long)nx * px, NY = (long long)ny * py, NZ = (long long)nz * pz;
    const int32_t base = *reserve;
    if (base < 0 || t >= NX * NY * NZ) return;
    const int ix = (int)(t % NX), iy = (int)((t / NX) % NY), iz = (int)(t / (NX * NY));
    const long long p = base + t;
    sp.cell[p] = pack_cell(lo0 + ix / px, lo1 + iy / py, lo2 + iz / pz);
    ((float *)sp.pos[0])[p] = ((float)(ix % px) + 0.5f) / (float)px;
    ((float *)sp.pos[1])[p] = ((float)(iy % py) + 0.5f) / (float)py;
    ((float *)sp.pos[2])[p] = ((float)(iz % pz) + 0.5f) / (float)pz;
    for (int a = 0; a < 3; ++a) ((float *)sp.u[a])[p] = 0.f;
    sp.id[p] = next_id + (int32_t)t;
    if (sp.per_particle_w && sp.w) ((float *)sp.w)[p] = w;
}

}  // namespace

void launch_fill_i32(int32_t *p, long long n, int32_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_i32, dim3(1024), dim3(256), 0, s, p, n, v);
}

void launch_window_particles(const SpeciesP &sp, int ax, int cells, hipStream_t s) {
    if (sp.capacity <= 0) return;
    hipLaunchKernelGGL(k_window_particles, dim3(nblk(sp.capacity, 256)), dim3(256), 0, s, sp, ax,
                       cells);
}

void launch_inject(const SpeciesP &sp, const int lo[3], const int nc[3], const int per[3],
                   float w, int next_id, int32_t *reserve, uint32_t *fault, hipStream_t s) {
    const long long m = (long long)nc[0] * per[0] * nc[1] * per[1] * nc[2] * per[2];
    if (m <= 0) return;
    hipLaunchKernelGGL(k_inject_reserve, dim3(1), dim3(1), 0, s, sp.count, sp.capacity, m, reserve,
                       fault);
    hipLaunchKernelGGL(k_inject, dim3(nblk(m, 256)), dim3(256), 0, s, sp, lo[0], lo[1], lo[2],
                       nc[0], nc[1], nc[2], per[0], per[1], per[2], w, next_id, reserve);
}

void fill_species_consts(DevSpecies &D, const GridP &g, double q, double m, double w) {
    split_f32(q * g.dt / (2.0 * m), D.r, D.r_lo);
    const double dV = g.d[0] * g.d[1] * g.d[2];
    for (int a = 0; a < 3; ++a) {
        D.qcd[a] = q * w * g.d[a] / (g.dt * dV);
        D.qc[a] = (float)D.qcd[a];
    }
}

void launch_write_species(DevSpecies *dst, const DevSpecies &v, hipStream_t s) {
    hipLaunchKernelGGL(k_write_species, dim3(1), dim3(1), 0, s, dst, v);
}

namespace {
template <class TL, int ORDER>
void launch_fused(const FusedArgs &A, int nb, hipStream_t s, hipEvent_t ev_start,
                  hipEvent_t ev_stop) {
    if (ev_start)  // timestamps taken by the dispatch itself
        hipExtLaunchKernelGGL((k_push_fused<TL, ORDER>), dim3(nb), dim3(PUSH_THREADS), 0, s,
                              ev_start, ev_stop, 0, A);
    else
        hipLaunchKernelGGL((k_push_fused<TL, ORDER>), dim3(nb), dim3(PUSH_THREADS), 0, s, A);
}
}  // namespace

void launch_push_fused(const GridP &g, const TileInfo &ti, float *const E[3],
                       float *const Bbar[3], unsigned long long *const Jf[3],
                       const DevSpecies *tbl, int nsp,
                       unsigned cur_mask, unsigned wr_mask, uint32_t *fault, unsigned long long *fallback,
                       uint32_t *fb_mask, long long mask_words, int *fb_tiles,
                       unsigned *fb_count, double jscale,
                       bool fallback_pass, hipStream_t s, hipEvent_t ev_start,
                       hipEvent_t ev_stop, unsigned long long *publish) {
    FusedArgs A;
    A.g = g;
    A.ti = ti;
    for (int a = 0; a < 3; ++a) {
        A.E[a] = E[a];
        A.Bb[a] = Bbar[a];
        A.Jf[a] = Jf[a];
        split_f32(g.dt / g.d[a], A.dtd[a], A.dtd_lo[a]);
    }
    A.tbl = tbl;
    A.nsp = nsp;
    A.cur_mask = cur_mask;
    A.wr_mask = wr_mask;
    A.jscale = jscale;
    A.jinv = 1.0 / jscale;
    A.fault = fault;
    A.fallback = fallback;
    A.fb_mask = fb_mask;
    A.mask_words = mask_words;
    A.fb_tiles = fb_tiles;
    A.fb_count = fb_count;
    A.publish = publish;
    const int nb = 8 * ((ti.ntiles + 7) / 8);
    if (fallback_pass)
        // a grid that fills the chip: after many steps without a sort the
        // list can hold most tiles
        hipLaunchKernelGGL(g.shape_order == 2 ? k_push_fallback<2> : k_push_fallback<1>,
                           dim3(2048), dim3(256), 0, s, A);
    else if (ti.slab)
        launch_fused<TileSlab, 1>(A, nb, s, ev_start, ev_stop);  // order 2 is refused on slab grids
    else if (g.shape_order == 2)
        launch_fused<TileCube2, 2>(A, nb, s, ev_start, ev_stop);
    else
        launch_fused<TileCube, 1>(A, nb, s, ev_start, ev_stop);
}

void launch_dry_push_f32(const GridP &g, float *const E[3], float *const Bbar[3],
                         const SpeciesP &sp, double *partial_slot, uint32_t *fault,
                         hipStream_t s) {
    float r, r_lo;
    split_f32(sp.q * g.dt / (2.0 * sp.m), r, r_lo);
    hipLaunchKernelGGL(k_dry_push_f32, dim3(RED_BLOCKS), dim3(256), 0, s, g, E[0], E[1], E[2],
                       Bbar[0], Bbar[1], Bbar[2], sp, r, r_lo, partial_slot, fault);
}

void launch_kinetic_f32(const SpeciesP &sp, double *partial_slot, hipStream_t s) {
    hipLaunchKernelGGL(k_kinetic_f32, dim3(RED_BLOCKS), dim3(256), 0, s, sp, partial_slot);
}

void launch_rho_f32(const GridP &g, const TileInfo &ti, bool tiles_valid, double scale,
                    const SpeciesP &sp, double *rho, hipStream_t s) {
    if (sp.capacity <= 0) return;
    if (g.shape_order == 2) {
        hipLaunchKernelGGL(k_rho2_f32, dim3(nblk(sp.capacity, 256)), dim3(256), 0, s, g, sp, rho);
        return;
    }
    const unsigned nb = 8 * ((ti.ntiles + 7) / 8);
    if (tiles_valid && ti.slab)
        hipLaunchKernelGGL(k_rho_tiles<TileSlab>, dim3(nb), dim3(256), 0, s, g, ti, sp, scale, rho);
    else if (tiles_valid)
        hipLaunchKernelGGL(k_rho_tiles<TileCube>, dim3(nb), dim3(256), 0, s, g, ti, sp, scale, rho);
    else
        hipLaunchKernelGGL(k_rho_f32, dim3(nblk(sp.capacity, 256)), dim3(256), 0, s, g, sp, rho);
}

void launch_load_f32(const GridP &g, const SpeciesP &sp, long long count, const double *pos,
                     const double *u, const double *w, const int32_t *ids, uint32_t *fault,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_load_f32, dim3(nblk(count > 0 ? count : 1, 256)), dim3(256), 0, s, g, sp,
                       count, pos, u, w, ids, fault);
}

void launch_store_f32(const GridP &g, const SpeciesP &sp, double *pos, double *u, int32_t *ids,
                      hipStream_t s) {
    if (sp.capacity <= 0) return;
    hipLaunchKernelGGL(k_store_f32, dim3(nblk(sp.capacity, 256)), dim3(256), 0, s, g, sp, pos, u,
                       ids);
}

void launch_sort(const GridP &g, const TileInfo &ti, const SpeciesP &cur, const SpeciesP &alt,
                 int32_t *counts, int32_t *scan_blocks, int32_t *rank, int32_t *tile_off,
                 uint32_t *fault, bool tiles_valid, int32_t *perm, hipStream_t s) {
    const long long NK = ti.NK;
    launch_fill_i32(counts, NK + 1, 0, s);
    if (perm && cur.capacity > 0) launch_fill_i32(perm, cur.capacity, -1, s);
    if (cur.capacity > 0) {
        if (tiles_valid)
            hipLaunchKernelGGL(k_sort_count_tiles, dim3(ti.ntiles), dim3(SORT_T), 0, s, ti, g, cur,
                               counts, rank, fault);
        else
            hipLaunchKernelGGL(k_sort_count, dim3(nblk(cur.capacity, 256)), dim3(256), 0, s, ti,
                               g, cur, counts, rank, fault);
    }
    const int nb = (int)((NK + SCAN_B - 1) / SCAN_B);
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(SCAN_T), 0, s, counts, NK, scan_blocks);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(SCAN_T), 0, s, scan_blocks, nb, counts, NK);
    hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(SCAN_T), 0, s, counts, NK, scan_blocks);
    if (cur.capacity > 0) {
        if (tiles_valid)
            hipLaunchKernelGGL(k_sort_scatter_tiles, dim3(ti.ntiles), dim3(SORT_T), 0, s, ti, cur,
                               alt, counts, rank, perm);
        else
            hipLaunchKernelGGL(k_sort_scatter, dim3(nblk(cur.capacity, 256)), dim3(256), 0, s,
                               ti, cur, alt, counts, rank, perm);
    }
    hipLaunchKernelGGL(k_tile_offsets, dim3(nblk(ti.ntiles + 1, 256)), dim3(256), 0, s, counts,
                       NK, ti.ntiles, tile_off, cur.count);
}

}  // namespace empic
