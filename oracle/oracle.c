/*
 * oracle.c -- plain, slow, single-threaded FP64 CPU reference of one explicit
 * electromagnetic particle-in-cell step (KEMPIC-3D, arXiv 2609.16575).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; it shares no header, helper, table or kernel with the
 * HIP path.  Only the tests, the smoke check and the CPU baseline leg of the
 * benchmark load it (through oracle/oracle.py).
 *
 * Everything is written as loops over the definitions, in the order the paper
 * gives them (Sec. 2.2, Fig. "PIC algorithm"): Faraday -> temporal centring of
 * B -> staggered CIC gather -> relativistic Boris push -> ZigZag current
 * deposit -> Ampere-Maxwell -> boundaries.  Units: c = eps0 = mu0 = 1, which
 * is what the bare "- dt J" term of the Ampere-Maxwell update implies.
 *
 * Grid layout (shared convention, not shared code): arrays are [k][j][i],
 * x fastest, with `ext[a] = n[a] + (absorbing ? 1 : 0)` entries per axis.
 * Component locations in cell units:
 *   Ex(i+1/2, j, k)  Ey(i, j+1/2, k)  Ez(i, j, k+1/2)     J like E
 *   Bx(i, j+1/2, k+1/2)  By(i+1/2, j, k+1/2)  Bz(i+1/2, j+1/2, k)
 *   rho at nodes (i, j, k).
 *
 * Readings of points the paper leaves open are marked READING below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PERIODIC 0
#define ORC_ABSORBING 1
#define ORC_PEC 2

typedef struct {
    int32_t n[3];  /* cells per axis */
    int32_t bc[3]; /* ORC_PERIODIC, ORC_ABSORBING or ORC_PEC, per axis */
    double d[3];   /* cell size */
    double dt;     /* time step */
} orc_grid;

typedef struct {
    double a0;      /* peak field amplitude (normalised vector potential) */
    double w0;      /* 1/e field waist */
    double tau;     /* intensity FWHM duration */
    double t0;      /* time of the envelope peak */
    double omega0;  /* carrier frequency */
    double yc, zc;  /* transverse centre of the spot */
    int32_t i_s;    /* x node index of the current sheet */
    int32_t slab;   /* 1: spot Gaussian in z only, uniform along y (2D slab runs) */
} orc_laser;

typedef struct {
    int32_t axis;      /* normal of the port plane */
    int32_t plane;     /* node index of the plane along axis */
    int32_t comp;      /* driven E component (transverse to axis) */
    int32_t prof_axis; /* transverse axis of the half-sine profile */
    double e0;         /* amplitude */
    double omega;      /* angular frequency */
    double tau;        /* time constant of the envelope 1 - exp(-t/tau) */
} orc_port;

/* ------------------------------------------------------------------------ */
/* indexing helpers                                                          */
/* ------------------------------------------------------------------------ */

/* walled (absorbing or PEC) axes store n+1 node planes */
static int64_t ext_of(const orc_grid *g, int a) {
    return (int64_t)g->n[a] + (g->bc[a] != ORC_PERIODIC ? 1 : 0);
}

static int64_t vol_of(const orc_grid *g) {
    return ext_of(g, 0) * ext_of(g, 1) * ext_of(g, 2);
}

/* Linear index of (i,j,k); periodic axes wrap, walled axes return -1 when
 * the point lies outside the stored array. */
static int64_t at(const orc_grid *g, int64_t i, int64_t j, int64_t k) {
    int64_t p[3] = {i, j, k};
    for (int a = 0; a < 3; ++a) {
        int64_t e = ext_of(g, a);
        if (g->bc[a] == ORC_PERIODIC) {
            int64_t n = g->n[a];
            p[a] = ((p[a] % n) + n) % n;
        } else if (p[a] < 0 || p[a] >= e) {
            return -1;
        }
    }
    return p[0] + ext_of(g, 0) * (p[1] + ext_of(g, 1) * p[2]);
}

/* Stagger of E_c and B_c along axis a: 1 = half-integer position, 0 = node. */
static int stag_E(int c, int a) { return a == c ? 1 : 0; }
static int stag_B(int c, int a) { return a == c ? 0 : 1; }

/* Number of stored values of a component along axis a: periodic axes hold n,
 * walled axes hold n+1 node values or n half-cell values. */
static int64_t count_along(const orc_grid *g, int a, int half) {
    if (g->bc[a] == ORC_PERIODIC) return g->n[a];
    return half ? g->n[a] : (int64_t)g->n[a] + 1;
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.3, Yee FDTD.  Faraday: the B_x equation of the paper, the other two  */
/* components by cyclic permutation of (x, y, z).                             */
/* B^{n+1/2} = B^{n-1/2} - dt curl E^n, forward differences.                  */
/* Also writes the time-centred field of Sec. 2.5 (Eq. "B centred"):          */
/* Bbar^n = (B^{n-1/2} + B^{n+1/2}) / 2.                                      */
/* READING: the paper's "half step" wording and the full-step equation agree  */
/* in exact arithmetic once B is centred by averaging; the full step plus     */
/* average is taken.                                                          */
/* ------------------------------------------------------------------------ */
void orc_faraday(const orc_grid *g, const double *E, double *B, double *Bbar) {
    const int64_t V = vol_of(g);
    for (int c = 0; c < 3; ++c) {
        const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
        int64_t cnt[3];
        for (int a = 0; a < 3; ++a) cnt[a] = count_along(g, a, stag_B(c, a));
        for (int64_t k = 0; k < cnt[2]; ++k)
            for (int64_t j = 0; j < cnt[1]; ++j)
                for (int64_t i = 0; i < cnt[0]; ++i) {
                    int64_t p[3] = {i, j, k};
                    int64_t q1[3] = {i, j, k}, q2[3] = {i, j, k};
                    q1[a1] += 1; /* +1 along a1 */
                    q2[a2] += 1; /* +1 along a2 */
                    const int64_t ip = at(g, p[0], p[1], p[2]);
                    const int64_t i1 = at(g, q1[0], q1[1], q1[2]);
                    const int64_t i2 = at(g, q2[0], q2[1], q2[2]);
                    /* (curl E)_c = d_{a1} E_{a2} - d_{a2} E_{a1} */
                    const double curl = (E[a2 * V + i1] - E[a2 * V + ip]) / g->d[a1] -
                                        (E[a1 * V + i2] - E[a1 * V + ip]) / g->d[a2];
                    const double old = B[c * V + ip];
                    const double nw = old - g->dt * curl;
                    B[c * V + ip] = nw;
                    if (Bbar) Bbar[c * V + ip] = 0.5 * (old + nw);
                }
    }
}

/* Is the E_c value at (i,j,k) on a face of a walled axis where it is a      */
/* tangential component (its update then belongs to the boundary condition)? */
static int e_on_wall_face(const orc_grid *g, int c, const int64_t p[3]) {
    for (int a = 0; a < 3; ++a) {
        if (a == c || g->bc[a] == ORC_PERIODIC) continue;
        if (p[a] == 0 || p[a] == g->n[a]) return 1;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.3, Ampere-Maxwell: the E_x equation of the paper and its cyclic      */
/* permutations.  E^{n+1} = E^n + dt curl B^{n+1/2} - dt J^{n+1/2}, backward   */
/* differences.  Tangential E on walled faces is left to orc_mur / orc_pec.   */
/* ------------------------------------------------------------------------ */
void orc_ampere(const orc_grid *g, double *E, const double *B, const double *J) {
    const int64_t V = vol_of(g);
    for (int c = 0; c < 3; ++c) {
        const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
        int64_t cnt[3];
        for (int a = 0; a < 3; ++a) cnt[a] = count_along(g, a, stag_E(c, a));
        for (int64_t k = 0; k < cnt[2]; ++k)
            for (int64_t j = 0; j < cnt[1]; ++j)
                for (int64_t i = 0; i < cnt[0]; ++i) {
                    int64_t p[3] = {i, j, k};
                    if (e_on_wall_face(g, c, p)) continue;
                    int64_t q1[3] = {i, j, k}, q2[3] = {i, j, k};
                    q1[a1] -= 1;
                    q2[a2] -= 1;
                    const int64_t ip = at(g, p[0], p[1], p[2]);
                    const int64_t i1 = at(g, q1[0], q1[1], q1[2]);
                    const int64_t i2 = at(g, q2[0], q2[1], q2[2]);
                    /* (curl B)_c = d_{a1} B_{a2} - d_{a2} B_{a1} */
                    const double curl = (B[a2 * V + ip] - B[a2 * V + i1]) / g->d[a1] -
                                        (B[a1 * V + ip] - B[a1 * V + i2]) / g->d[a2];
                    E[c * V + ip] += g->dt * curl - g->dt * (J ? J[c * V + ip] : 0.0);
                }
    }
}

/* ------------------------------------------------------------------------ */
/* Boundaries (Sec. 2.2 lists a boundary module; its kind is not given).      */
/* READING: first-order Mur absorbing condition (Mur 1981) on tangential E at */
/* every face of an absorbing axis, c = 1:                                    */
/*   E_0^{n+1} = E_1^n + (dt - d)/(dt + d) (E_1^{n+1} - E_0^n)                */
/* and the mirror formula at the far face.  Axes are processed x, then y,     */
/* then z; an edge value shared by two faces ends with the later axis.        */
/* E_old is a copy of E^n taken before orc_ampere.                            */
/* ------------------------------------------------------------------------ */
void orc_mur(const orc_grid *g, double *E, const double *E_old) {
    const int64_t V = vol_of(g);
    for (int a = 0; a < 3; ++a) {
        if (g->bc[a] != ORC_ABSORBING) continue;
        const double coef = (g->dt - g->d[a]) / (g->dt + g->d[a]);
        const int64_t n = g->n[a];
        for (int c = 0; c < 3; ++c) {
            if (c == a) continue;
            int64_t cnt[3];
            for (int b = 0; b < 3; ++b) cnt[b] = count_along(g, b, stag_E(c, b));
            cnt[a] = 1; /* iterate the face plane only */
            for (int64_t k = 0; k < cnt[2]; ++k)
                for (int64_t j = 0; j < cnt[1]; ++j)
                    for (int64_t i = 0; i < cnt[0]; ++i) {
                        for (int side = 0; side < 2; ++side) {
                            int64_t p0[3] = {i, j, k}, p1[3] = {i, j, k};
                            p0[a] = side ? n : 0;
                            p1[a] = side ? n - 1 : 1;
                            const int64_t b0 = at(g, p0[0], p0[1], p0[2]);
                            const int64_t b1 = at(g, p1[0], p1[1], p1[2]);
                            E[c * V + b0] = E_old[c * V + b1] +
                                            coef * (E[c * V + b1] - E_old[c * V + b0]);
                        }
                    }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Moving window (a module of Sec. 2.2; used by the wakefield run of Sec. 4; */
/* its algorithm is not given).  READING: the window advances `cells` cells  */
/* along the walled axis `axis` at once: every E and B value moves `cells`   */
/* planes toward index 0, planes leaving at index 0 are dropped and the new  */
/* planes at the far end start at zero.  (Particles are shifted, removed and  */
/* injected by the caller.)                                                   */
/* ------------------------------------------------------------------------ */
void orc_window_shift(const orc_grid *g, double *E, double *B, int32_t axis, int32_t cells) {
    const int64_t V = vol_of(g);
    double *F[2] = {E, B};
    for (int f = 0; f < 2; ++f)
        for (int c = 0; c < 3; ++c) {
            int64_t cnt[3];
            for (int b = 0; b < 3; ++b)
                cnt[b] = count_along(g, b, f == 0 ? stag_E(c, b) : stag_B(c, b));
            const int64_t L = cnt[axis];
            for (int64_t k = 0; k < cnt[2]; ++k)
                for (int64_t j = 0; j < cnt[1]; ++j)
                    for (int64_t i = 0; i < cnt[0]; ++i) {
                        int64_t p[3] = {i, j, k};
                        const int64_t m = p[axis];
                        const int64_t dst = at(g, p[0], p[1], p[2]);
                        double v = 0.0;
                        if (m + cells < L) {
                            p[axis] = m + cells;
                            v = F[f][c * V + at(g, p[0], p[1], p[2])];
                        }
                        F[f][c * V + dst] = v;
                    }
        }
}

/* ------------------------------------------------------------------------ */
/* Current filtering (the "compensated smoothing" module of Sec. 2.2/2.5;     */
/* its stencil is not given).  READING: along each axis in turn (x, y, z) and */
/* for each J component on its own sub-grid, `passes` applications of the    */
/* binomial stencil (1/4, 1/2, 1/4), then, if `compensate`, one of the        */
/* compensator (-1/4, 3/2, -1/4).  A mode exp(i k) is multiplied by           */
/* cos^(2 passes)(k/2), times 1 + sin^2(k/2) with the compensator.  Periodic  */
/* axes wrap; on a walled axis values beyond the stored ones count as zero.   */
/* Applied to J after the deposit, before Ampere.                             */
/* ------------------------------------------------------------------------ */
static void filter_line(double *v, double *tmp, int64_t L, int periodic, double a, double b) {
    for (int64_t i = 0; i < L; ++i) {
        double lo = 0.0, hi = 0.0;
        if (i > 0) lo = v[i - 1];
        else if (periodic) lo = v[L - 1];
        if (i < L - 1) hi = v[i + 1];
        else if (periodic) hi = v[0];
        tmp[i] = a * lo + b * v[i] + a * hi;
    }
    memcpy(v, tmp, (size_t)L * sizeof(double));
}

void orc_filter_J(const orc_grid *g, double *J, int32_t passes, int32_t compensate) {
    const int64_t V = vol_of(g);
    for (int ax = 0; ax < 3; ++ax)
        for (int c = 0; c < 3; ++c) {
            int64_t cnt[3];
            for (int b = 0; b < 3; ++b) cnt[b] = count_along(g, b, stag_E(c, b));
            const int64_t L = cnt[ax];
            double *line = (double *)malloc((size_t)L * sizeof(double));
            double *tmp = (double *)malloc((size_t)L * sizeof(double));
            int64_t lc[3] = {cnt[0], cnt[1], cnt[2]};
            lc[ax] = 1;
            for (int64_t k = 0; k < lc[2]; ++k)
                for (int64_t j = 0; j < lc[1]; ++j)
                    for (int64_t i = 0; i < lc[0]; ++i) {
                        int64_t p[3] = {i, j, k};
                        for (int64_t m = 0; m < L; ++m) {
                            p[ax] = m;
                            line[m] = J[c * V + at(g, p[0], p[1], p[2])];
                        }
                        const int per = g->bc[ax] == ORC_PERIODIC;
                        for (int32_t q = 0; q < passes; ++q) filter_line(line, tmp, L, per, 0.25, 0.5);
                        if (compensate) filter_line(line, tmp, L, per, -0.25, 1.5);
                        for (int64_t m = 0; m < L; ++m) {
                            p[ax] = m;
                            J[c * V + at(g, p[0], p[1], p[2])] = line[m];
                        }
                    }
            free(line);
            free(tmp);
        }
}

/* ------------------------------------------------------------------------ */
/* Perfectly conducting walls (the waveguide walls of Sec. 3.2).  READING:    */
/* tangential E is zero on the node planes 0 and n of a PEC axis; Ampere      */
/* leaves those values alone and this sets them to zero after every step.     */
/* Normal B on the walls then keeps its initial value (zero) by Faraday.      */
/* Particles leaving through a PEC face are removed, as at an absorbing one.  */
/* ------------------------------------------------------------------------ */
void orc_pec(const orc_grid *g, double *E) {
    const int64_t V = vol_of(g);
    for (int a = 0; a < 3; ++a) {
        if (g->bc[a] != ORC_PEC) continue;
        for (int c = 0; c < 3; ++c) {
            if (c == a) continue;
            int64_t cnt[3];
            for (int b = 0; b < 3; ++b) cnt[b] = count_along(g, b, stag_E(c, b));
            cnt[a] = 1;
            for (int64_t k = 0; k < cnt[2]; ++k)
                for (int64_t j = 0; j < cnt[1]; ++j)
                    for (int64_t i = 0; i < cnt[0]; ++i)
                        for (int side = 0; side < 2; ++side) {
                            int64_t p[3] = {i, j, k};
                            p[a] = side ? g->n[a] : 0;
                            E[c * V + at(g, p[0], p[1], p[2])] = 0.0;
                        }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Port excitation of the waveguide benchmark (Sec. 3.2): a monochromatic     */
/* field prescribed on the input plane, switched on with the envelope        */
/* g(t) = 1 - exp(-t/tau).  READING: a hard source on the node plane `plane`  */
/* of axis `axis`: E_comp = e0 sin(pi s / L) g(t) sin(omega t) with s the    */
/* component's position along prof_axis and L that axis' length (the TE10   */
/* profile), at t = t^{n+1}, written after the other boundary updates.       */
/* ------------------------------------------------------------------------ */
void orc_port_apply(const orc_grid *g, double *E, const orc_port *P, double t) {
    const int64_t V = vol_of(g);
    const int c = P->comp, a = P->axis, pa = P->prof_axis;
    const double L = g->n[pa] * g->d[pa];
    const double amp = P->e0 * (1.0 - exp(-t / P->tau)) * sin(P->omega * t);
    int64_t cnt[3];
    for (int b = 0; b < 3; ++b) cnt[b] = count_along(g, b, stag_E(c, b));
    cnt[a] = 1;
    for (int64_t k = 0; k < cnt[2]; ++k)
        for (int64_t j = 0; j < cnt[1]; ++j)
            for (int64_t i = 0; i < cnt[0]; ++i) {
                int64_t p[3] = {i, j, k};
                p[a] = P->plane;
                const double spos = ((double)p[pa] + 0.5 * stag_E(c, pa)) * g->d[pa];
                const int64_t ip = at(g, p[0], p[1], p[2]);
                /* sin(pi s/L) evaluated from the nearer wall: exactly 0 on both */
                const double sw = spos < L - spos ? spos : L - spos;
                if (ip >= 0) E[c * V + ip] = amp * sin(acos(-1.0) * sw / L);
            }
}

/* READING (laser injection, configuration with a0 = 2): a soft current sheet */
/* J_y on the x-node plane i_s radiating the incident field                   */
/*   E_inc = a0 exp(-r^2/w0^2) exp(-2 ln2 (t-t0)^2/tau^2) sin(omega0 (t-t0))   */
/* in both directions (K = -2 E_inc, J = K/dx); the backward half is absorbed */
/* by the x = 0 face.  Applied to E after Ampere as -dt * J_sheet at         */
/* t = t^{n+1/2}.                                                              */
double orc_laser_field(const orc_laser *L, double t, double y, double z) {
    const double ry2 = L->slab ? 0.0 : (y - L->yc) * (y - L->yc);
    const double r2 = ry2 + (z - L->zc) * (z - L->zc);
    const double tt = t - L->t0;
    return L->a0 * exp(-r2 / (L->w0 * L->w0)) *
           exp(-2.0 * log(2.0) * tt * tt / (L->tau * L->tau)) * sin(L->omega0 * tt);
}

void orc_laser_apply(const orc_grid *g, double *E, const orc_laser *L, double t_half) {
    const int64_t V = vol_of(g);
    int64_t cnt[3];
    for (int b = 0; b < 3; ++b) cnt[b] = count_along(g, b, stag_E(1, b));
    for (int64_t k = 0; k < cnt[2]; ++k)
        for (int64_t j = 0; j < cnt[1]; ++j) {
            int64_t p[3] = {L->i_s, j, k};
            if (e_on_wall_face(g, 1, p)) continue;
            const double y = ((double)j + 0.5) * g->d[1];
            const double z = (double)k * g->d[2];
            const double Jy = -2.0 * orc_laser_field(L, t_half, y, z) / g->d[0];
            const int64_t ip = at(g, p[0], p[1], p[2]);
            if (ip >= 0) E[V + ip] -= g->dt * Jy;
        }
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.5: staggered CIC (trilinear) gather.  Each component is            */
/* interpolated from its own Yee sub-grid: per axis t = xi - s (s = 0 or 1/2), */
/* i0 = floor(t), weight of i0+1 is t - i0.  Points outside an absorbing      */
/* axis' array contribute zero.                                               */
/* ------------------------------------------------------------------------ */
static double gather_one(const orc_grid *g, const double *F, const int stag[3],
                         const double xi[3]) {
    int64_t i0[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        const double t = xi[a] - 0.5 * stag[a];
        const double fl = floor(t);
        i0[a] = (int64_t)fl;
        f[a] = t - fl;
    }
    double s = 0.0;
    for (int oz = 0; oz < 2; ++oz)
        for (int oy = 0; oy < 2; ++oy)
            for (int ox = 0; ox < 2; ++ox) {
                const int64_t ip = at(g, i0[0] + ox, i0[1] + oy, i0[2] + oz);
                if (ip < 0) continue;
                const double w = (ox ? f[0] : 1.0 - f[0]) * (oy ? f[1] : 1.0 - f[1]) *
                                 (oz ? f[2] : 1.0 - f[2]);
                s += w * F[ip];
            }
    return s;
}

void orc_gather(const orc_grid *g, const double *E, const double *Bbar, const double pos[3],
                double Ep[3], double Bp[3]) {
    const int64_t V = vol_of(g);
    double xi[3];
    for (int a = 0; a < 3; ++a) xi[a] = pos[a] / g->d[a];
    for (int c = 0; c < 3; ++c) {
        int se[3], sb[3];
        for (int a = 0; a < 3; ++a) {
            se[a] = stag_E(c, a);
            sb[a] = stag_B(c, a);
        }
        Ep[c] = gather_one(g, E + c * V, se, xi);
        Bp[c] = gather_one(g, Bbar + c * V, sb, xi);
    }
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.4: relativistic Boris push (Boris 1970).  u = gamma v (c = 1),      */
/* r = q dt / (2 m).  Half electric kick, magnetic rotation, half kick.       */
/* READING: the rotation is described in words only; the standard t/s form   */
/* is used: t = r B / gamma^-, s = 2 t / (1 + t.t).                           */
/* ------------------------------------------------------------------------ */
void orc_boris(double u[3], const double Ep[3], const double Bp[3], double r) {
    double um[3], t[3], s[3], up[3], upl[3];
    for (int a = 0; a < 3; ++a) um[a] = u[a] + r * Ep[a];
    const double gm = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
    for (int a = 0; a < 3; ++a) t[a] = r * Bp[a] / gm;
    const double tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    for (int a = 0; a < 3; ++a) s[a] = 2.0 * t[a] / (1.0 + tt);
    /* u' = u- + u- x t */
    up[0] = um[0] + (um[1] * t[2] - um[2] * t[1]);
    up[1] = um[1] + (um[2] * t[0] - um[0] * t[2]);
    up[2] = um[2] + (um[0] * t[1] - um[1] * t[0]);
    /* u+ = u- + u' x s */
    upl[0] = um[0] + (up[1] * s[2] - up[2] * s[1]);
    upl[1] = um[1] + (up[2] * s[0] - up[0] * s[2]);
    upl[2] = um[2] + (up[0] * s[1] - up[1] * s[0]);
    for (int a = 0; a < 3; ++a) u[a] = upl[a] + r * Ep[a];
}

/* Single particle in prescribed uniform fields (Sec. 3.1 benchmarks): nsteps */
/* Boris pushes and position updates x += dt u/gamma.  traj (nullable) gets   */
/* the position after each step, 3 per step.                                  */
void orc_particle_uniform(double r, const double E[3], const double B[3], double dt,
                          int64_t nsteps, double x[3], double u[3], double *traj) {
    for (int64_t s = 0; s < nsteps; ++s) {
        orc_boris(u, E, B, r);
        const double gm = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        for (int a = 0; a < 3; ++a) x[a] += dt * u[a] / gm;
        if (traj)
            for (int a = 0; a < 3; ++a) traj[3 * s + a] = x[a];
    }
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.5: ZigZag charge-conserving current deposit (Umeda et al. 2003).   */
/* Per axis, in cell units: i1 = floor(xi1), i2 = floor(xi2), relay point     */
/*   xr = min(min(i1,i2)+1, max(max(i1,i2), (xi1+xi2)/2)).                    */
/* The move is split into segment A (xi1 -> xr) inside cell i1 and segment B  */
/* (xr -> xi2) inside cell i2.  Each straight segment inside one cell          */
/* deposits on the 12 edges of that cell.                                     */
/* READING: the paper does not print the 3D weights.  The line integral of    */
/* the bilinear CIC weights along the straight segment is used:               */
/*   J_a(edge o_b, o_c) += q dx_a/(dt dV) * d_a * [w_b(o_b) w_c(o_c)          */
/*                                     + sgn dxi_b dxi_c / 12]                 */
/* with w(0) = 1 - W, w(1) = W, W the segment midpoint relative to the cell,  */
/* sgn = +1 when o_b == o_c else -1.  midpoint_only = 1 drops the /12 term    */
/* (the literal midpoint-product weights of the 2D derivation).               */
/* ------------------------------------------------------------------------ */
static void add_edge(const orc_grid *g, double *J, int c, int64_t i, int64_t j, int64_t k,
                     double v) {
    const int64_t ip = at(g, i, j, k);
    if (ip < 0) return; /* walled axis: edge outside the array */
    int64_t p[3] = {i, j, k};
    /* a walled axis' half-cell components stop at index n-1 */
    for (int a = 0; a < 3; ++a)
        if (g->bc[a] != ORC_PERIODIC && stag_E(c, a) && p[a] >= g->n[a]) return;
    J[c * vol_of(g) + ip] += v;
}

static void deposit_segment(const orc_grid *g, double *J, const int64_t cell[3],
                            const double s[3], const double e[3], double qsp,
                            int midpoint_only) {
    const double dV = g->d[0] * g->d[1] * g->d[2];
    double dxi[3], W[3];
    for (int a = 0; a < 3; ++a) {
        dxi[a] = e[a] - s[a];
        W[a] = 0.5 * (s[a] + e[a]) - (double)cell[a];
    }
    for (int c = 0; c < 3; ++c) {
        const int b1 = (c + 1) % 3, b2 = (c + 2) % 3;
        const double amp = qsp * dxi[c] * g->d[c] / (g->dt * dV);
        const double cross = midpoint_only ? 0.0 : dxi[b1] * dxi[b2] / 12.0;
        for (int o2 = 0; o2 < 2; ++o2)
            for (int o1 = 0; o1 < 2; ++o1) {
                const double w1 = o1 ? W[b1] : 1.0 - W[b1];
                const double w2 = o2 ? W[b2] : 1.0 - W[b2];
                const double sg = (o1 == o2) ? 1.0 : -1.0;
                int64_t p[3] = {cell[0], cell[1], cell[2]};
                p[b1] += o1;
                p[b2] += o2;
                add_edge(g, J, c, p[0], p[1], p[2], amp * (w1 * w2 + sg * cross));
            }
    }
}

void orc_zigzag(const orc_grid *g, double *J, const double xi1[3], const double xi2[3],
                double qsp, int midpoint_only) {
    int64_t c1[3], c2[3];
    double xr[3];
    for (int a = 0; a < 3; ++a) {
        const int64_t i1 = (int64_t)floor(xi1[a]);
        const int64_t i2 = (int64_t)floor(xi2[a]);
        const double lo = (double)((i1 < i2 ? i1 : i2) + 1);
        const double hi = (double)(i1 > i2 ? i1 : i2);
        const double mid = 0.5 * (xi1[a] + xi2[a]);
        xr[a] = fmin(lo, fmax(hi, mid));
        c1[a] = i1;
        c2[a] = i2;
    }
    deposit_segment(g, J, c1, xi1, xr, qsp, midpoint_only);
    deposit_segment(g, J, c2, xr, xi2, qsp, midpoint_only);
}

/* ------------------------------------------------------------------------ */
/* One species through gather -> Boris -> move -> ZigZag (Sec. 2.2 order).   */
/* pos: 3*np global positions x^n (in [0, L)), u: 3*np momenta u^{n-1/2}     */
/* (gamma v); both rewritten to x^{n+1}, u^{n+1/2}.  alive (nullable) marks   */
/* particles removed by an absorbing face.  wpp (nullable) per-particle       */
/* macro weight, else w.  q_sp = q w, m_sp = m w (Sec. 2.1).  dry = 1 only    */
/* gathers and pushes a copy of u to accumulate the kinetic energy of         */
/* u^{n+1/2} (nothing is written).  kin (nullable) += sum w m (gamma - 1) of  */
/* the pushed momenta.                                                        */
/* ------------------------------------------------------------------------ */
void orc_push_deposit(const orc_grid *g, const double *E, const double *Bbar, double *J,
                      int64_t np, double *pos, double *u, int8_t *alive, const double *wpp,
                      double q, double m, double w, int midpoint_only, int dry, double *kin) {
    const double r = q * g->dt / (2.0 * m);
    double L[3];
    for (int a = 0; a < 3; ++a) L[a] = g->n[a] * g->d[a];
    double ksum = 0.0;
    for (int64_t p = 0; p < np; ++p) {
        if (alive && !alive[p]) continue;
        const double wp = wpp ? wpp[p] : w;
        double Ep[3], Bp[3], un[3];
        orc_gather(g, E, Bbar, pos + 3 * p, Ep, Bp);
        for (int a = 0; a < 3; ++a) un[a] = u[3 * p + a];
        orc_boris(un, Ep, Bp, r);
        const double uu = un[0] * un[0] + un[1] * un[1] + un[2] * un[2];
        const double gm = sqrt(1.0 + uu);
        ksum += wp * m * uu / (gm + 1.0); /* gamma - 1 = u.u / (gamma + 1) */
        if (dry) continue;
        double xi1[3], xi2[3];
        for (int a = 0; a < 3; ++a) {
            xi1[a] = pos[3 * p + a] / g->d[a];
            xi2[a] = xi1[a] + g->dt * un[a] / (gm * g->d[a]);
        }
        if (J) orc_zigzag(g, J, xi1, xi2, q * wp, midpoint_only);
        for (int a = 0; a < 3; ++a) {
            u[3 * p + a] = un[a];
            double x = pos[3 * p + a] + g->dt * un[a] / gm;
            if (g->bc[a] == ORC_PERIODIC) {
                if (x >= L[a]) x -= L[a];
                if (x < 0.0) {
                    x += L[a];
                    if (x >= L[a]) x = 0.0;
                }
            } else if (x < 0.0 || x >= L[a]) {
                if (alive) alive[p] = 0;
            }
            pos[3 * p + a] = x;
        }
    }
    if (kin) *kin += ksum;
}

/* ------------------------------------------------------------------------ */
/* Second-order shapes (the shape-function equation of Sec. 2.4 with l = 1; */
/* the paper runs l = 0 and names higher orders as an extension, Sec. 5).   */
/* A super-particle with the triangular cloud b_1 weighs the grid with      */
/* b_2 = b_1 * b_0, the quadratic B-spline:                                 */
/*   b_2(t) = 3/4 - t^2 for |t| <= 1/2, (3/2 - |t|)^2 / 2 for |t| <= 3/2.   */
/* A point at t (sub-grid index units) touches the nearest index            */
/* m = floor(t + 1/2) and its two neighbours.                               */
/* ------------------------------------------------------------------------ */
static double b2(double t) {
    const double a = fabs(t);
    if (a <= 0.5) return 0.75 - a * a;
    if (a < 1.5) return 0.5 * (1.5 - a) * (1.5 - a);
    return 0.0;
}

/* one component from its Yee sub-grid (stag as for gather_one) */
static double gather2_one(const orc_grid *g, const double *F, const int stag[3],
                          const double xi[3]) {
    double t[3];
    int64_t m[3];
    for (int a = 0; a < 3; ++a) {
        t[a] = xi[a] - 0.5 * stag[a];
        m[a] = (int64_t)floor(t[a] + 0.5);
    }
    double s = 0.0;
    for (int64_t k = m[2] - 1; k <= m[2] + 1; ++k)
        for (int64_t j = m[1] - 1; j <= m[1] + 1; ++j)
            for (int64_t i = m[0] - 1; i <= m[0] + 1; ++i) {
                const int64_t ip = at(g, i, j, k);
                if (ip < 0) continue;
                s += b2(t[0] - (double)i) * b2(t[1] - (double)j) * b2(t[2] - (double)k) * F[ip];
            }
    return s;
}

void orc_gather2(const orc_grid *g, const double *E, const double *Bbar, const double pos[3],
                 double Ep[3], double Bp[3]) {
    const int64_t V = vol_of(g);
    double xi[3];
    for (int a = 0; a < 3; ++a) xi[a] = pos[a] / g->d[a];
    for (int c = 0; c < 3; ++c) {
        int se[3], sb[3];
        for (int a = 0; a < 3; ++a) {
            se[a] = stag_E(c, a);
            sb[a] = stag_B(c, a);
        }
        Ep[c] = gather2_one(g, E + c * V, se, xi);
        Bp[c] = gather2_one(g, Bbar + c * V, sb, xi);
    }
}

/* Esirkepov's decomposition (Esirkepov 2001) of one move xi0 -> xi1 (cell  */
/* units, |xi1 - xi0| < 1 per axis) with the b_2 weights S on the nodes     */
/* lo .. lo+3 that cover both positions:                                    */
/*   W_c = dS_c (S0_b S0_e + dS_b S0_e / 2 + S0_b dS_e / 2 + dS_b dS_e / 3) */
/* ((b, e) the other two axes, dS = S1 - S0), and discrete continuity fixes  */
/* J_c on the edge between nodes l and l+1 along c as the running sum        */
/* -q d_c / (dt dV) sum_{l' <= l} W_c(l').                                  */
static void esirkepov2(const orc_grid *g, double *J, const double xi0[3], const double xi1[3],
                       double qsp) {
    const double dV = g->d[0] * g->d[1] * g->d[2];
    int64_t lo[3];
    double S0[3][4], dS[3][4];
    for (int a = 0; a < 3; ++a) {
        const int64_t m0 = (int64_t)floor(xi0[a] + 0.5), m1 = (int64_t)floor(xi1[a] + 0.5);
        lo[a] = (m0 < m1 ? m0 : m1) - 1;
        for (int l = 0; l < 4; ++l) {
            S0[a][l] = b2(xi0[a] - (double)(lo[a] + l));
            dS[a][l] = b2(xi1[a] - (double)(lo[a] + l)) - S0[a][l];
        }
    }
    for (int c = 0; c < 3; ++c) {
        const int b = (c + 1) % 3, e = (c + 2) % 3;
        const double scale = -qsp * g->d[c] / (g->dt * dV);
        for (int lb = 0; lb < 4; ++lb)
            for (int le = 0; le < 4; ++le) {
                const double T = S0[b][lb] * S0[e][le] + 0.5 * dS[b][lb] * S0[e][le] +
                                 0.5 * S0[b][lb] * dS[e][le] + dS[b][lb] * dS[e][le] / 3.0;
                double run = 0.0;
                for (int l = 0; l < 4; ++l) {
                    run += dS[c][l] * T;
                    int64_t p[3];
                    p[c] = lo[c] + l;
                    p[b] = lo[b] + lb;
                    p[e] = lo[e] + le;
                    if (run != 0.0) add_edge(g, J, c, p[0], p[1], p[2], scale * run);
                }
            }
    }
}

/* EZ at second order (Steiniger et al., the hybrid the paper names in      */
/* Sec. 2.5): a move that crosses a cell of the b_2 stencil (the planes      */
/* between half-integers, i.e. the cells of the ZigZag rule shifted by 1/2)  */
/* is split at the ZigZag relay point, so that each part stays in one such   */
/* cell, and each part gets Esirkepov's decomposition.  READING: a move      */
/* inside one cell is one part (ZigZag's mid-point split is the same thing   */
/* at first order, where the weights are linear in the position; at second   */
/* order it would add a loop current).                                       */
void orc_ez2(const orc_grid *g, double *J, const double xi1[3], const double xi2[3],
             double qsp) {
    int cross = 0;
    for (int a = 0; a < 3; ++a) cross |= floor(xi1[a] + 0.5) != floor(xi2[a] + 0.5);
    if (!cross) {
        esirkepov2(g, J, xi1, xi2, qsp);
        return;
    }
    double xr[3];
    for (int a = 0; a < 3; ++a) {
        /* the cell of the b_2 stencil: m = floor(xi + 1/2), planes m +- 1/2 */
        const double m1 = floor(xi1[a] + 0.5), m2 = floor(xi2[a] + 0.5);
        const double lo = fmin(m1, m2) + 0.5, hi = fmax(m1, m2) - 0.5;
        xr[a] = fmin(lo, fmax(hi, 0.5 * (xi1[a] + xi2[a])));
    }
    esirkepov2(g, J, xi1, xr, qsp);
    esirkepov2(g, J, xr, xi2, qsp);
}

/* orc_push_deposit with second-order shapes: b_2 gather, Boris, move, EZ.  */
void orc_push_deposit2(const orc_grid *g, const double *E, const double *Bbar, double *J,
                       int64_t np, double *pos, double *u, int8_t *alive, const double *wpp,
                       double q, double m, double w, int dry, double *kin) {
    const double r = q * g->dt / (2.0 * m);
    double L[3];
    for (int a = 0; a < 3; ++a) L[a] = g->n[a] * g->d[a];
    double ksum = 0.0;
    for (int64_t p = 0; p < np; ++p) {
        if (alive && !alive[p]) continue;
        const double wp = wpp ? wpp[p] : w;
        double Ep[3], Bp[3], un[3];
        orc_gather2(g, E, Bbar, pos + 3 * p, Ep, Bp);
        for (int a = 0; a < 3; ++a) un[a] = u[3 * p + a];
        orc_boris(un, Ep, Bp, r);
        const double uu = un[0] * un[0] + un[1] * un[1] + un[2] * un[2];
        const double gm = sqrt(1.0 + uu);
        ksum += wp * m * uu / (gm + 1.0);
        if (dry) continue;
        double xi1[3], xi2[3];
        for (int a = 0; a < 3; ++a) {
            xi1[a] = pos[3 * p + a] / g->d[a];
            xi2[a] = xi1[a] + g->dt * un[a] / (gm * g->d[a]);
        }
        if (J) orc_ez2(g, J, xi1, xi2, q * wp);
        for (int a = 0; a < 3; ++a) {
            u[3 * p + a] = un[a];
            double x = pos[3 * p + a] + g->dt * un[a] / gm;
            if (g->bc[a] == ORC_PERIODIC) {
                if (x >= L[a]) x -= L[a];
                if (x < 0.0) {
                    x += L[a];
                    if (x >= L[a]) x = 0.0;
                }
            } else if (x < 0.0 || x >= L[a]) {
                if (alive) alive[p] = 0;
            }
            pos[3 * p + a] = x;
        }
    }
    if (kin) *kin += ksum;
}

/* b_2 charge density at nodes, rho += (q_sp / dV) prod_a b_2(xi_a - i_a).  */
void orc_rho2(const orc_grid *g, int64_t np, const double *pos, const int8_t *alive,
              const double *wpp, double q, double w, double *rho) {
    const double dV = g->d[0] * g->d[1] * g->d[2];
    for (int64_t p = 0; p < np; ++p) {
        if (alive && !alive[p]) continue;
        const double qsp = q * (wpp ? wpp[p] : w);
        double t[3];
        int64_t m[3];
        for (int a = 0; a < 3; ++a) {
            t[a] = pos[3 * p + a] / g->d[a];
            m[a] = (int64_t)floor(t[a] + 0.5);
        }
        for (int64_t k = m[2] - 1; k <= m[2] + 1; ++k)
            for (int64_t j = m[1] - 1; j <= m[1] + 1; ++j)
                for (int64_t i = m[0] - 1; i <= m[0] + 1; ++i) {
                    const int64_t ip = at(g, i, j, k);
                    if (ip < 0) continue;
                    rho[ip] += qsp / dV * b2(t[0] - (double)i) * b2(t[1] - (double)j) *
                               b2(t[2] - (double)k);
                }
    }
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.5: CIC charge density at nodes, rho += (q_sp / dV) prod_a w_a.     */
/* ------------------------------------------------------------------------ */
void orc_rho(const orc_grid *g, int64_t np, const double *pos, const int8_t *alive,
             const double *wpp, double q, double w, double *rho) {
    const double dV = g->d[0] * g->d[1] * g->d[2];
    for (int64_t p = 0; p < np; ++p) {
        if (alive && !alive[p]) continue;
        const double qsp = q * (wpp ? wpp[p] : w);
        int64_t i0[3];
        double f[3];
        for (int a = 0; a < 3; ++a) {
            const double t = pos[3 * p + a] / g->d[a];
            const double fl = floor(t);
            i0[a] = (int64_t)fl;
            f[a] = t - fl;
        }
        for (int oz = 0; oz < 2; ++oz)
            for (int oy = 0; oy < 2; ++oy)
                for (int ox = 0; ox < 2; ++ox) {
                    const int64_t ip = at(g, i0[0] + ox, i0[1] + oy, i0[2] + oz);
                    if (ip < 0) continue;
                    const double wt = (ox ? f[0] : 1.0 - f[0]) * (oy ? f[1] : 1.0 - f[1]) *
                                      (oz ? f[2] : 1.0 - f[2]);
                    rho[ip] += qsp / dV * wt;
                }
    }
}

/* Discrete divergence at nodes with backward differences (the operator for  */
/* which Yee + a charge-conserving deposit keep Gauss's law, Sec. 2.3):      */
/*   div F(i,j,k) = sum_a (F_a(p) - F_a(p - e_a)) / d_a.                      */
void orc_div_nodes(const orc_grid *g, const double *F, double *out) {
    const int64_t V = vol_of(g);
    int64_t cnt[3];
    for (int a = 0; a < 3; ++a) cnt[a] = count_along(g, a, 0);
    for (int64_t k = 0; k < cnt[2]; ++k)
        for (int64_t j = 0; j < cnt[1]; ++j)
            for (int64_t i = 0; i < cnt[0]; ++i) {
                const int64_t ip = at(g, i, j, k);
                double s = 0.0;
                for (int a = 0; a < 3; ++a) {
                    int64_t q[3] = {i, j, k};
                    q[a] -= 1;
                    const int64_t iq = at(g, q[0], q[1], q[2]);
                    /* an absorbing axis' padding entry (index n of a half-cell
                     * component) is never written and stays zero */
                    const double fp = F[a * V + ip];
                    const double fm = iq < 0 ? 0.0 : F[a * V + iq];
                    s += (fp - fm) / g->d[a];
                }
                out[ip] = s;
            }
}

/* Field energies (Sec. 3.3, energy conservation).  READING: the paper does  */
/* not state time levels.  U_E^n = dV/2 sum |E^n|^2 and                      */
/* U_B^n = dV/2 sum B^{n-1/2} . B^{n+1/2}, with B^{n+1/2} formed from the     */
/* state as B^{n-1/2} - dt curl E^n; their sum is the quadratic form that the */
/* vacuum Yee leapfrog keeps exactly.                                         */
double orc_energy_E(const orc_grid *g, const double *E) {
    const int64_t V = vol_of(g);
    const double dV = g->d[0] * g->d[1] * g->d[2];
    double s = 0.0;
    for (int64_t i = 0; i < 3 * V; ++i) s += E[i] * E[i];
    return 0.5 * dV * s;
}

double orc_energy_B(const orc_grid *g, const double *E, const double *B) {
    const int64_t V = vol_of(g);
    const double dV = g->d[0] * g->d[1] * g->d[2];
    double *Bn = (double *)malloc(sizeof(double) * 3 * V);
    memcpy(Bn, B, sizeof(double) * 3 * V);
    orc_faraday(g, E, Bn, NULL);
    double s = 0.0;
    for (int64_t i = 0; i < 3 * V; ++i) s += B[i] * Bn[i];
    free(Bn);
    return 0.5 * dV * s;
}

/* Sum of w m (gamma - 1) over the momenta as stored. */
double orc_kinetic(int64_t np, const double *u, const int8_t *alive, const double *wpp,
                   double m, double w) {
    double s = 0.0;
    for (int64_t p = 0; p < np; ++p) {
        if (alive && !alive[p]) continue;
        const double uu = u[3 * p] * u[3 * p] + u[3 * p + 1] * u[3 * p + 1] +
                          u[3 * p + 2] * u[3 * p + 2];
        s += (wpp ? wpp[p] : w) * m * uu / (sqrt(1.0 + uu) + 1.0);
    }
    return s;
}

/* ======================================================================== */
/* Adjoint of one step (vector-Jacobian product), periodic grids.             */
/* Not in the paper: the differentiable variant of the cycle.  The step is    */
/*   B' = B - dt Cf E,  Bbar = (B + B')/2,  E_p = G_E(x) E,  B_p = G_B(x) Bbar, */
/*   u' = Boris(u, E_p, B_p),  x' = x + dt u'/gamma',  J = Z(x, x'),          */
/*   E' = E + dt Cb B' - dt J                                                 */
/* with Cf / Cb the forward / backward difference curls (Cf^T = Cb on a       */
/* periodic grid).  Given the adjoints of (E', B', x', u') it returns those   */
/* of (E, B, x, u), differentiating inside the current piece of every         */
/* piecewise map (relay-point branch and interpolation corners frozen).       */
/* ======================================================================== */

/* adjoint of the Boris push: forward from (u, E, B), reverse with lu' */
static void boris_vjp(const double u[3], const double Ep[3], const double Bp[3], double r,
                      const double lup[3], double lu[3], double lE[3], double lB[3]) {
    double um[3], t[3], s[3], up[3];
    for (int a = 0; a < 3; ++a) um[a] = u[a] + r * Ep[a];
    const double gm = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
    for (int a = 0; a < 3; ++a) t[a] = r * Bp[a] / gm;
    const double tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    for (int a = 0; a < 3; ++a) s[a] = 2.0 * t[a] / (1.0 + tt);
    up[0] = um[0] + (um[1] * t[2] - um[2] * t[1]);
    up[1] = um[1] + (um[2] * t[0] - um[0] * t[2]);
    up[2] = um[2] + (um[0] * t[1] - um[1] * t[0]);
    /* u' = upl + r E */
    double lupl[3], lum[3], lupv[3], ls[3], lt[3];
    for (int a = 0; a < 3; ++a) {
        lupl[a] = lup[a];
        lE[a] = r * lup[a];
    }
    /* upl = um + up x s: d/d up -> s x l ; d/d s -> l x up */
    for (int a = 0; a < 3; ++a) lum[a] = lupl[a];
    lupv[0] = s[1] * lupl[2] - s[2] * lupl[1];
    lupv[1] = s[2] * lupl[0] - s[0] * lupl[2];
    lupv[2] = s[0] * lupl[1] - s[1] * lupl[0];
    ls[0] = lupl[1] * up[2] - lupl[2] * up[1];
    ls[1] = lupl[2] * up[0] - lupl[0] * up[2];
    ls[2] = lupl[0] * up[1] - lupl[1] * up[0];
    /* up = um + um x t: d/d um -> l + t x l ; d/d t -> l x um */
    lum[0] += lupv[0] + (t[1] * lupv[2] - t[2] * lupv[1]);
    lum[1] += lupv[1] + (t[2] * lupv[0] - t[0] * lupv[2]);
    lum[2] += lupv[2] + (t[0] * lupv[1] - t[1] * lupv[0]);
    lt[0] = lupv[1] * um[2] - lupv[2] * um[1];
    lt[1] = lupv[2] * um[0] - lupv[0] * um[2];
    lt[2] = lupv[0] * um[1] - lupv[1] * um[0];
    /* s = 2 t / (1 + t.t) */
    const double den = 1.0 + tt;
    const double tls = t[0] * ls[0] + t[1] * ls[1] + t[2] * ls[2];
    for (int a = 0; a < 3; ++a) lt[a] += 2.0 * ls[a] / den - 4.0 * t[a] * tls / (den * den);
    /* t = r B / gm */
    double tlt = 0.0;
    for (int a = 0; a < 3; ++a) {
        lB[a] = r * lt[a] / gm;
        tlt += t[a] * lt[a];
    }
    const double lgm = -tlt / gm;
    /* gm = sqrt(1 + um.um) */
    for (int a = 0; a < 3; ++a) lum[a] += lgm * um[a] / gm;
    /* um = u + r E */
    for (int a = 0; a < 3; ++a) {
        lu[a] = lum[a];
        lE[a] += r * lum[a];
    }
}

/* gather adjoint for one component: scatter l * weights into lF and return */
/* the derivative of the interpolated value along xi (cell units) times l  */
static void gather_one_vjp(const orc_grid *g, const double *F, double *lF, const int stag[3],
                           const double xi[3], double l, double dxi[3]) {
    int64_t i0[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        const double t = xi[a] - 0.5 * stag[a];
        const double fl = floor(t);
        i0[a] = (int64_t)fl;
        f[a] = t - fl;
    }
    for (int oz = 0; oz < 2; ++oz)
        for (int oy = 0; oy < 2; ++oy)
            for (int ox = 0; ox < 2; ++ox) {
                const int64_t ip = at(g, i0[0] + ox, i0[1] + oy, i0[2] + oz);
                const double wx = ox ? f[0] : 1.0 - f[0], wy = oy ? f[1] : 1.0 - f[1],
                             wz = oz ? f[2] : 1.0 - f[2];
                lF[ip] += l * wx * wy * wz;
                const double v = l * F[ip];
                dxi[0] += v * (ox ? 1.0 : -1.0) * wy * wz;
                dxi[1] += v * wx * (oy ? 1.0 : -1.0) * wz;
                dxi[2] += v * wx * wy * (oz ? 1.0 : -1.0);
            }
}

/* adjoint of deposit_segment: d/d s and d/d e of sum_edges lJ . J_seg */
static void deposit_segment_vjp(const orc_grid *g, const double *lJ, const int64_t cell[3],
                                const double s[3], const double e[3], double qsp, double ls[3],
                                double le[3]) {
    const double dV = g->d[0] * g->d[1] * g->d[2];
    const int64_t V = vol_of(g);
    double dxi[3], W[3], lD[3] = {0, 0, 0}, lW[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a) {
        dxi[a] = e[a] - s[a];
        W[a] = 0.5 * (s[a] + e[a]) - (double)cell[a];
    }
    for (int c = 0; c < 3; ++c) {
        const int b1 = (c + 1) % 3, b2 = (c + 2) % 3;
        const double ampc = qsp * g->d[c] / (g->dt * dV); /* J = ampc * dxi_c * weight */
        for (int o2 = 0; o2 < 2; ++o2)
            for (int o1 = 0; o1 < 2; ++o1) {
                int64_t p[3] = {cell[0], cell[1], cell[2]};
                p[b1] += o1;
                p[b2] += o2;
                const double lam = lJ[c * V + at(g, p[0], p[1], p[2])];
                const double w1 = o1 ? W[b1] : 1.0 - W[b1];
                const double w2 = o2 ? W[b2] : 1.0 - W[b2];
                const double sg = (o1 == o2) ? 1.0 : -1.0;
                const double weight = w1 * w2 + sg * dxi[b1] * dxi[b2] / 12.0;
                lD[c] += lam * ampc * weight;
                const double k = lam * ampc * dxi[c];
                lW[b1] += k * (o1 ? 1.0 : -1.0) * w2;
                lW[b2] += k * w1 * (o2 ? 1.0 : -1.0);
                lD[b1] += k * sg * dxi[b2] / 12.0;
                lD[b2] += k * sg * dxi[b1] / 12.0;
            }
    }
    for (int a = 0; a < 3; ++a) {
        ls[a] += -lD[a] + 0.5 * lW[a];
        le[a] += lD[a] + 0.5 * lW[a];
    }
}

static void zigzag_vjp(const orc_grid *g, const double *lJ, const double xi1[3],
                       const double xi2[3], double qsp, double l1[3], double l2[3]) {
    int64_t c1[3], c2[3];
    double xr[3], dr1[3], dr2[3];
    for (int a = 0; a < 3; ++a) {
        const int64_t i1 = (int64_t)floor(xi1[a]);
        const int64_t i2 = (int64_t)floor(xi2[a]);
        const double lo = (double)((i1 < i2 ? i1 : i2) + 1);
        const double hi = (double)(i1 > i2 ? i1 : i2);
        const double mid = 0.5 * (xi1[a] + xi2[a]);
        xr[a] = fmin(lo, fmax(hi, mid));
        /* relay point: mid-point (both derivatives 1/2) unless clamped to a face */
        const int is_mid = (mid >= hi) && (mid <= lo);
        dr1[a] = is_mid ? 0.5 : 0.0;
        dr2[a] = is_mid ? 0.5 : 0.0;
        c1[a] = i1;
        c2[a] = i2;
    }
    double lsA[3] = {0, 0, 0}, leA[3] = {0, 0, 0}, lsB[3] = {0, 0, 0}, leB[3] = {0, 0, 0};
    deposit_segment_vjp(g, lJ, c1, xi1, xr, qsp, lsA, leA);
    deposit_segment_vjp(g, lJ, c2, xr, xi2, qsp, lsB, leB);
    for (int a = 0; a < 3; ++a) {
        const double lr = leA[a] + lsB[a];
        l1[a] += lsA[a] + lr * dr1[a];
        l2[a] += leB[a] + lr * dr2[a];
    }
}

/* Cf^T = Cb: out += scale * curl_b(F) (F B-located, out E-located) and
 * out += scale * curl_f(F) (F E-located, out B-located), periodic.          */
static void curl_b_add(const orc_grid *g, const double *F, double *out, double scale) {
    const int64_t V = vol_of(g);
    double *Z = (double *)calloc(3 * V, sizeof(double));
    orc_ampere(g, Z, F, NULL); /* Z = dt curl_b(F) */
    for (int64_t i = 0; i < 3 * V; ++i) out[i] += scale * Z[i] / g->dt;
    free(Z);
}
static void curl_f_add(const orc_grid *g, const double *F, double *out, double scale) {
    const int64_t V = vol_of(g);
    double *Z = (double *)calloc(3 * V, sizeof(double));
    orc_faraday(g, F, Z, NULL); /* Z = -dt curl_f(F) */
    for (int64_t i = 0; i < 3 * V; ++i) out[i] -= scale * Z[i] / g->dt;
    free(Z);
}

/* One species' particle adjoint.  pos/u: state at n (x^n, u^{n-1/2});
 * lx/lu in: adjoints of x^{n+1}, u^{n+1/2}; out: of x^n, u^{n-1/2}.
 * lJ = -dt * (adjoint of E^{n+1}); accumulates into lE (adjoint of E^n
 * through the gather) and lBbar.                                            */
void orc_particles_vjp(const orc_grid *g, const double *E, const double *Bbar, const double *lJ,
                       int64_t np, const double *pos, const double *u, const double *wpp,
                       double q, double m, double w, double *lx, double *lu, double *lE,
                       double *lBbar) {
    const int64_t V = vol_of(g);
    const double r = q * g->dt / (2.0 * m);
    for (int64_t p = 0; p < np; ++p) {
        const double wp = wpp ? wpp[p] : w;
        double xi1[3], Ep[3], Bp[3], un[3];
        for (int a = 0; a < 3; ++a) xi1[a] = pos[3 * p + a] / g->d[a];
        orc_gather(g, E, Bbar, pos + 3 * p, Ep, Bp);
        for (int a = 0; a < 3; ++a) un[a] = u[3 * p + a];
        orc_boris(un, Ep, Bp, r);
        const double uu = un[0] * un[0] + un[1] * un[1] + un[2] * un[2];
        const double gm = sqrt(1.0 + uu);
        double xi2[3];
        for (int a = 0; a < 3; ++a) xi2[a] = xi1[a] + g->dt * un[a] / (gm * g->d[a]);
        /* deposit adjoint */
        double l1[3] = {0, 0, 0}, l2[3] = {0, 0, 0};
        zigzag_vjp(g, lJ, xi1, xi2, q * wp, l1, l2);
        /* x' = x + dt v'; xi2 = x/d + dt v'/d; xi1 = x/d */
        double lxn[3], lv[3];
        for (int a = 0; a < 3; ++a) {
            lxn[a] = lx[3 * p + a] + l1[a] / g->d[a] + l2[a] / g->d[a];
            lv[a] = g->dt * (lx[3 * p + a] + l2[a] / g->d[a]);
        }
        /* v' = u'/gamma': d/du' = I/g - u' u'^T / g^3 */
        const double uv = un[0] * lv[0] + un[1] * lv[1] + un[2] * lv[2];
        double lup[3];
        for (int a = 0; a < 3; ++a)
            lup[a] = lu[3 * p + a] + lv[a] / gm - un[a] * uv / (gm * gm * gm);
        double lu0[3], lEp[3], lBp[3];
        boris_vjp(u + 3 * p, Ep, Bp, r, lup, lu0, lEp, lBp);
        /* gather adjoint */
        double dxi[3] = {0, 0, 0};
        for (int c = 0; c < 3; ++c) {
            int se[3], sb[3];
            for (int a = 0; a < 3; ++a) {
                se[a] = stag_E(c, a);
                sb[a] = stag_B(c, a);
            }
            gather_one_vjp(g, E + c * V, lE + c * V, se, xi1, lEp[c], dxi);
            gather_one_vjp(g, Bbar + c * V, lBbar + c * V, sb, xi1, lBp[c], dxi);
        }
        for (int a = 0; a < 3; ++a) {
            lx[3 * p + a] = lxn[a] + dxi[a] / g->d[a];
            lu[3 * p + a] = lu0[a];
        }
    }
}

/* Field part of the step adjoint.  lE, lB in: adjoints of E^{n+1}, B^{n+1/2};
 * lE_gather, lBbar: accumulated by orc_particles_vjp.  Out (in place):
 * adjoints of E^n, B^{n-1/2}.                                               */
void orc_fields_vjp(const orc_grid *g, double *lE, double *lB, const double *lE_gather,
                    const double *lBbar) {
    const int64_t V = vol_of(g);
    double *lBt = (double *)malloc(sizeof(double) * 3 * V);
    /* lB' = lB + dt Cb^T lE' + lBbar/2 = lB + dt Cf(lE') + lBbar/2 */
    for (int64_t i = 0; i < 3 * V; ++i) lBt[i] = lB[i] + 0.5 * lBbar[i];
    curl_f_add(g, lE, lBt, g->dt);
    /* lB = lB' + lBbar/2 ; lE = lE' + lE_gather - dt Cf^T lB' = ... - dt Cb(lB') */
    for (int64_t i = 0; i < 3 * V; ++i) {
        lB[i] = lBt[i] + 0.5 * lBbar[i];
        lE[i] += lE_gather[i];
    }
    curl_b_add(g, lBt, lE, -g->dt);
    free(lBt);
}
