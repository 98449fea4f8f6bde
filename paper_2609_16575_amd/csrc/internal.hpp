// internal.hpp -- device-side types and helpers shared by the libempic
// translation units (kernels + runtime).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "empic.h"

namespace empic {

// ---------------------------------------------------------------------------
// Grid parameters passed by value to every kernel.
// ---------------------------------------------------------------------------
struct GridP {
    int n[3];     // cells per axis
    int ext[3];   // stored entries per axis (n + 1 on an absorbing axis)
    int bc[3];    // EMPIC_BC_*
    double d[3];  // cell sizes
    double inv_d[3];
    double dt;
    long long V;  // ext0 * ext1 * ext2
    int shape_order = 1;  // 1: CIC weighting (the paper's); 2: b_2 weighting, EZ current
};

// Drift margin: particles up to MARGIN cells outside their tile (moved since
// the last sort) are still served from the tile's LDS windows.
constexpr int MARGIN = 1;
constexpr int PUSH_THREADS = 512;
constexpr int PPT = 4;  // consecutive particles per thread (one 16-byte access per array)
constexpr int TC = 256;  // cells per tile (every shape)

// Tile of cells owned by one workgroup of the fused FP32 particle kernel, and
// its LDS windows: the field window covers the gather stencil (cells -1..+1
// around a particle cell), the current window one cell more (the second
// ZigZag segment) and the far edges.
//
// QCAP: entries of the LDS queue of second ZigZag segments (particles that
// cross a cell face deposit their first segment at once and queue the
// second, which the workgroup deposits after the tile's particles); 0: no
// queue, the second segment is deposited at once.
// FE: extra field-window points past the upper end of each axis (the
// second-order stencil of a node sub-grid reaches one point further).
template <int X, int Y, int Z, int Q, int FE = 0>
struct TileT {
    static constexpr int TX = X, TY = Y, TZ = Z, QCAP = Q;
    static constexpr int FWX = X + 2 * MARGIN + 2 + FE, FWY = Y + 2 * MARGIN + 2 + FE,
                         FWZ = Z + 2 * MARGIN + 2 + FE;
    static constexpr int JWX = X + 2 * MARGIN + 3, JWY = Y + 2 * MARGIN + 3, JWZ = Z + 2 * MARGIN + 3;
    static constexpr int FW3 = FWX * FWY * FWZ, JW3 = JWX * JWY * JWZ;
    static constexpr int LHI_X = X + 2 * MARGIN, LHI_Y = Y + 2 * MARGIN, LHI_Z = Z + 2 * MARGIN;
    static constexpr int ROWS = 24;  // rows of the window index tables
    static_assert(X * Y * Z == TC, "every tile shape holds TC cells");
    static_assert(JWX <= ROWS && JWY <= ROWS && JWZ <= ROWS, "window index tables");
    static_assert((X & (X - 1)) == 0 && (Y & (Y - 1)) == 0 && (Z & (Z - 1)) == 0,
                  "power-of-two tile sides (sort keys use shifts)");
};
// Three-dimensional grids: 8 x 8 x 4, field window 27.6 KB + int64 current
// window 36.5 KB + a 16 KB crossing queue, two workgroups per CU (158.4 of
// the 160 KB of LDS).
using TileCube = TileT<8, 8, 4, 512>;
// Grids at most three cells thick along y (the two-dimensional runs):
// 16 x 2 x 8 keeps 256 cells per tile where the cube would hold 8 x 2 x 4;
// 34.6 KB + 45.9 KB, still two workgroups in a CU's 160 KB of LDS, which
// leaves no room for a crossing queue.
using TileSlab = TileT<16, 2, 8, 0>;
// Second-order shapes (three-dimensional grids): the 8 x 8 x 4 tile with a
// 13 x 13 x 9 field window (36.5 KB) and the same current window, no queue:
// 73 KB, two workgroups per CU.
using TileCube2 = TileT<8, 8, 4, 0, 1>;

// A constant c of the FP32 path as the pair (hi, lo) of FP32 numbers with
// hi = c rounded and lo = c - hi rounded.  Products c x are formed as
// fma(lo, x, hi x) (or added in two FMAs), so that the rounding of c itself
// leaves no systematic relative error of up to 2^-24 in every step: such an
// error would shift the frequencies of the discrete system (for instance the
// plasma frequency through q dt / m, q w / (dt dV), dt / d and dt) and its
// phase would grow with the number of steps.
__host__ inline void split_f32(double c, float &hi, float &lo) {
    hi = (float)c;
    lo = (float)(c - (double)hi);
}

// Packed cell index of the FP32 path: i | j << 11 | k << 22; all ones = removed.
constexpr uint32_t DEAD = 0xFFFFFFFFu;
__host__ __device__ inline uint32_t pack_cell(int i, int j, int k) {
    return (uint32_t)i | ((uint32_t)j << 11) | ((uint32_t)k << 22);
}
__host__ __device__ inline int cell_i(uint32_t c) { return (int)(c & 0x7FFu); }
__host__ __device__ inline int cell_j(uint32_t c) { return (int)((c >> 11) & 0x7FFu); }
__host__ __device__ inline int cell_k(uint32_t c) { return (int)(c >> 22); }

struct TileInfo {
    int nt[3];      // tiles per axis
    int lg[3];      // log2 of the tile sides
    int ntiles;
    int slab;       // 1: TileSlab, 0: TileCube
    long long NK;   // ntiles * TC sort keys
};

__host__ __device__ inline long long sort_key(const TileInfo &t, int i, int j, int k) {
    const int tx = i >> t.lg[0], ty = j >> t.lg[1], tz = k >> t.lg[2];
    const int lx = i - (tx << t.lg[0]), ly = j - (ty << t.lg[1]), lz = k - (tz << t.lg[2]);
    const long long tile = tx + (long long)t.nt[0] * (ty + (long long)t.nt[1] * tz);
    return tile * TC + (lx + ((ly + (lz << t.lg[1])) << t.lg[0]));
}

// Per-species launch parameters of the particle kernels.
struct SpeciesP {
    uint32_t *cell;
    void *pos[3];
    void *u[3];
    int32_t *id;
    void *w;          // per-particle weight or nullptr
    const int32_t *tile_off;  // FP32: ntiles + 1 particle offsets after the last sort
    int32_t *count;   // device slot count
    long long capacity;
    double q, m, w_species;
    int per_particle_w;
};

// Device-side table of a species' parameters for both buffer sets, written
// once when the species is registered; the fused kernel picks the current set
// with a bit of `cur_mask` (kernel arguments are never indexed dynamically).
struct DevSpecies {
    SpeciesP p[2];
    float r, r_lo;  // q dt / (2 m) as an FP32 pair (split_f32)
    float qc[3];    // q w d_a / (dt dV)  (w = 1 when per-particle), rounded
    double qcd[3];  // the same in FP64: the current window's fixed-point multipliers
};
void fill_species_consts(DevSpecies &D, const GridP &g, double q, double m, double w);
void launch_write_species(DevSpecies *dst, const DevSpecies &v, hipStream_t s);

constexpr int NQ = 16;       // reduction slots
constexpr int RED_BLOCKS = 1024;  // grid-stride particle reductions
enum Slot {
    Q_EE = 0, Q_BB = 1, Q_KM = 2, Q_KP = 6, Q_GMAX = 10, Q_G2 = 11, Q_CMAX = 12, Q_RMAX = 13,
    Q_DOT = 14
};

__host__ __device__ inline bool slot_is_max(int q) {
    return q == Q_GMAX || q == Q_CMAX || q == Q_RMAX;
}

// periodic wrap (an index at most one period away)
__device__ inline int wrap1(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// wave64 + block reductions in double
__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}
__device__ inline double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    return v;
}
template <bool IS_MAX>
__device__ inline double block_reduce(double v, double *smem /* >= 16 */) {
    v = IS_MAX ? wave_max(v) : wave_sum(v);
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int nthr = blockDim.x * blockDim.y * blockDim.z;
    const int lane = tid & 63, wid = tid >> 6;
    __syncthreads();
    if (lane == 0) smem[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (tid == 0) {
        const int nw = (nthr + 63) >> 6;
        r = smem[0];
        for (int i = 1; i < nw; ++i) r = IS_MAX ? fmax(r, smem[i]) : r + smem[i];
    }
    return r;  // valid in thread 0 of the block
}

// Reduction partials: NQ slots of PSTRIDE per-block values each.
constexpr int PSTRIDE = 16384;
dim3 reduction_grid(const GridP &g);

// ---------------------------------------------------------------------------
// Launchers (defined in the kernel translation units).
// ---------------------------------------------------------------------------
// Faraday + centring of B; zeroes J (FP64 path) or the fixed-point Jf (FP32
// path) when given
template <typename T>
void launch_faraday(const GridP &g, T *const E[3], T *const B[3], T *const Bbar[3],
                    T *const J[3], unsigned long long *const Jf[3], bool write_B, hipStream_t s,
                    unsigned *fb_reset = nullptr);
// Ampere-Maxwell; with Jf, J is first set to Jf * jinv (FP32 path)
template <typename T>
void launch_ampere(const GridP &g, T *const E[3], T *const B[3], T *const J[3],
                   const long long *const Jf[3], double jinv, hipStream_t s);
void launch_j_from_fixed(const GridP &g, float *const J[3], const long long *const Jf[3],
                         double jinv, hipStream_t s);
// dst[a][i] = src[a][i], six arrays of n floats, one launch
void launch_copy6(const float *const src[6], float *const dst[6], long long n, hipStream_t s);
template <typename T>
void launch_mur_save(const GridP &g, T *const E[3], T *planes, long long plane_stride,
                     hipStream_t s);
template <typename T>
void launch_mur_apply(const GridP &g, T *const E[3], const T *planes, long long plane_stride,
                      hipStream_t s);
template <typename T>
void launch_laser(const GridP &g, T *const E[3], const empic_laser_desc &L, double t_half,
                  hipStream_t s);
template <typename T>
void launch_pec(const GridP &g, T *const E[3], hipStream_t s);
// moving window: fields `cells` planes back along ax (tmp: three arrays)
template <typename T>
void launch_window_shift(const GridP &g, T *const F[3], T *const tmp[3], int ax, int cells,
                         bool isB, hipStream_t s);
// moving window: particle cells `cells` back along ax, removed below 0; cold
// lattice injection into the cells [lo, lo + nc) after the slot count
// (capacity exceeded: EMPIC_FAULT_CAPACITY, nothing injected)
void launch_window_particles(const SpeciesP &sp, int ax, int cells, hipStream_t s);
void launch_inject(const SpeciesP &sp, const int lo[3], const int nc[3], const int per[3],
                   float w, int next_id, int32_t *reserve, uint32_t *fault, hipStream_t s);
// current filter: `passes` binomial passes per axis, then the compensator;
// tmp: three more arrays of the grid's size
template <typename T>
void launch_filter(const GridP &g, T *const F[3], T *const tmp[3], int passes, int compensate,
                   hipStream_t s);
template <typename T>
void launch_port(const GridP &g, T *const E[3], const empic_port_desc &P, double t, hipStream_t s);
template <typename T>
void launch_field_energy(const GridP &g, T *const E[3], T *const B[3], double *partials,
                         hipStream_t s);

// FP32 cell-relative path; the current goes to Jf as int64 multiples of
// 1/jscale.  fallback_pass = false launches the fused tile
// kernel, true the follow-up pass over particles that left their tile window;
// that pass also writes the cumulative out-of-window count to `publish`
// (device-accessible pinned host memory) when it is not null.
void launch_push_fused(const GridP &g, const TileInfo &ti, float *const E[3],
                       float *const Bbar[3], unsigned long long *const Jf[3],
                       const DevSpecies *tbl, int nsp,
                       unsigned cur_mask, unsigned wr_mask, uint32_t *fault, unsigned long long *fallback,
                       uint32_t *fb_mask, long long mask_words, int *fb_tiles,
                       unsigned *fb_count, double jscale,
                       bool fallback_pass, hipStream_t s, hipEvent_t ev_start = nullptr,
                       hipEvent_t ev_stop = nullptr, unsigned long long *publish = nullptr);
void launch_dry_push_f32(const GridP &g, float *const E[3], float *const Bbar[3],
                         const SpeciesP &sp, double *partial_slot, uint32_t *fault,
                         hipStream_t s);
void launch_kinetic_f32(const SpeciesP &sp, double *partial_slot, hipStream_t s);
// CIC rho of an FP32 species added to rho (FP64 nodes); tile-grouped
// particles (tiles_valid) are accumulated per tile in fixed point at `scale`
// (a power of two with one particle's contribution below 2^48).
void launch_rho_f32(const GridP &g, const TileInfo &ti, bool tiles_valid, double scale,
                    const SpeciesP &sp, double *rho, hipStream_t s);
void launch_load_f32(const GridP &g, const SpeciesP &sp, long long count, const double *pos,
                     const double *u, const double *w, const int32_t *ids, uint32_t *fault,
                     hipStream_t s);
void launch_store_f32(const GridP &g, const SpeciesP &sp, double *pos, double *u, int32_t *ids,
                      hipStream_t s);
// Counting sort by (tile, cell) of `cur` into `alt`.  tiles_valid: `cur` is
// still grouped by the tile offsets of its previous sort (faster counting).
void launch_sort(const GridP &g, const TileInfo &ti, const SpeciesP &cur, const SpeciesP &alt,
                 int32_t *counts, int32_t *scan_blocks, int32_t *rank, int32_t *tile_off,
                 uint32_t *fault, bool tiles_valid, int32_t *perm, hipStream_t s);

// FP64 plain path
void launch_push_f64(const GridP &g, double *const E[3], double *const Bbar[3],
                     double *const J[3], const SpeciesP &sp, long long count, uint32_t *fault,
                     hipStream_t s);
void launch_dry_push_f64(const GridP &g, double *const E[3], double *const Bbar[3],
                         const SpeciesP &sp, long long count, double *partial_slot,
                         uint32_t *fault, hipStream_t s);
void launch_kinetic_f64(const SpeciesP &sp, long long count, double *partial_slot,
                        hipStream_t s);
void launch_rho_f64(const GridP &g, const SpeciesP &sp, long long count, double *rho,
                    hipStream_t s);
void launch_load_f64(const GridP &g, const SpeciesP &sp, long long count, const double *pos,
                     const double *u, const double *w, const int32_t *ids, uint32_t *fault,
                     hipStream_t s);
void launch_store_f64(const SpeciesP &sp, long long count, double *pos, double *u, int32_t *ids,
                      hipStream_t s);

// adjoint of one FP32 step (periodic)
// lJdep: the adjoint the deposit sees, lE' itself or the filtered lE' when a
// (symmetric) current filter acts between deposit and Ampere
void launch_step_vjp(const GridP &g, const TileInfo &ti, float *const E[3], float *const Bbar[3],
                     float *const lE[3], float *const lJdep[3], float *const lB[3],
                     float *const lEg[3],
                     float *const lBb[3], float *const tB[3], const SpeciesP *sp,
                     const int32_t *const *tile_off, float *const (*lx)[3],
                     float *const (*lu)[3], int nsp, uint32_t *fb_mask, unsigned *fb_count,
                     float *const (*l6)[6], int *tile_exp, hipStream_t s);
// adjoint of a recorded sort: lam[perm[j]] = lam_post[j] (scratch: 6 x cap floats)
void launch_sort_vjp(const int32_t *perm, long long cap, float *const lx[3], float *const lu[3],
                     float *const scratch[6], hipStream_t s);

// diagnostics
void launch_zero_f64(double *p, long long n, hipStream_t s);
template <typename T>
void launch_gauss(const GridP &g, T *const E[3], const double *rho, double rho_bg,
                  double *partials, hipStream_t s);
template <typename T>
void launch_continuity(const GridP &g, T *const J[3], const double *rho_now,
                       const double *rho_prev, double *partials, hipStream_t s);
void launch_final_reduce(const double *partials, double *result, hipStream_t s);
void launch_fill_i32(int32_t *p, long long n, int32_t v, hipStream_t s);
// largest |x| of n doubles into *out (one workgroup; set-up path only)
// FP64 sum of a[i] * b[i] into *result (fixed order: RED_BLOCKS partials)
void launch_dot_f64(const float *a, const float *b, long long n, double *partials,
                    double *result, hipStream_t s);
void launch_absmax_f64(const double *x, long long n, double *out, hipStream_t s);

}  // namespace empic
