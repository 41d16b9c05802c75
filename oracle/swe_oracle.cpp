/*
 * swe_oracle.cpp -- serial FP64 reference of one explicit 2D predictor-corrector
 * MacCormack time step of the shallow-water mass and momentum equations, and
 * of the derivatives of a gauge-misfit loss through a sequence of such steps.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct checker
 * for the GPU library.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no source with the GPU path:
 * no headers, no helpers, no constant tables.
 *
 * What the paper fixes (Seitz et al., "A GPU Implementation for
 * Two-Dimensional Shallow Water Modeling", 2013):
 *   - the method: a 2D predictor-corrector MacCormack scheme solving for the
 *     water elevation and the two velocity components every time step (§1);
 *   - explicitness: a step depends only on the previous step's values (§1);
 *   - the step is split into 16 dependent sub-steps, each needing neighbour
 *     values produced by the sub-step before it, while inside a sub-step every
 *     cell is independent, so any cell order gives the same result (§1, §6.1);
 *   - a variable time step computed after each step from the new data (§3.1);
 *   - the scheme cannot handle dry cells (§6.2).
 * The paper defers the equations themselves to Ransom's thesis, which is not
 * available, so the discrete scheme below is our reading of the standard
 * MacCormack form for open-channel flow.  Every expression is written with its
 * evaluation order fixed so that an independent implementation doing the same
 * correctly rounded operations (+ - * / sqrt) reproduces it bit for bit.  The
 * one cube root (friction, S14) is not left to a math library, whose cbrt is
 * only faithful to about an ulp and differs between libraries; it is the
 * fixed sequence cbrt3 below, whose operations are all exact or correctly
 * rounded.
 *
 * PDEs (conservative, surface-gradient pressure form), unknowns eta (water
 * surface elevation) and q = (qx, qy) (unit discharges), h = eta - z:
 *   d(eta)/dt + d(qx)/dx + d(qy)/dy = 0
 *   d(qx)/dt + d(qx u)/dx + d(qy u)/dy + g h d(eta)/dx = -m qx |u| h^(-4/3)
 *   d(qy)/dt + d(qx v)/dx + d(qy v)/dy + g h d(eta)/dy = -m qy |u| h^(-4/3)
 *   u = qx/h, v = qy/h, m = g n^2 (n: Manning coefficient field).
 *
 * One step (U^n = (eta, qx, qy), t^n, dt = dt^n, sigma = +1 for even n and -1
 * for odd n) is the sixteen sweeps S1..S16 below, in order.  Arrays are
 * cell-centred, row-major with x fastest, padded with a one-cell ghost ring
 * (index i in [-1, nx], j in [-1, ny]); the four ghost corners are never read.
 *   S1  BC(U^n, t^n): ghost ring of U^n.  eta_g = eta of the adjacent cell for
 *       every kind.  WALL: normal discharge mirrored, tangential copied.  OPEN:
 *       both copied.  INFLOW: normal discharge = q_in(t) pointing into the
 *       domain, tangential 0.  An INFLOW edge acts as WALL outside its face
 *       band [lo, hi).  z of a ghost = z of the adjacent cell.
 *   S2  PRIM(U^n): h = eta - z; wet <=> h > h_dry; r = wet ? 1/h : 0;
 *       u = qx*r; v = qy*r.  Over every padded cell.  With the thin-film
 *       reading (h_film > 0) r = wet ? min(1/h, 1/h_film) : 0: in films
 *       thinner than h_film the velocities are q/h_film and S3 measures the
 *       curvature against h_film.  (In such films 1/h, and its depth
 *       derivative 1/h^2 through the velocities and the switch, is what makes
 *       the discrete adjoint of a flood over dry land grow without bound.)
 *   S3  SWITCH: nu_x = 0.25*(|(eta_E - eta_C) - (eta_C - eta_W)| * r_C), nu_y
 *       likewise with N/S.  Interior cells.
 *   S4  DISS: face coefficient eps = (wet_L && wet_R) ?
 *       min(kappa*max(nu_L, nu_R), eps_max) : 0 on interior faces, 0 on
 *       boundary faces; for each of eta, qx, qy:
 *       D = (eps_E*(U_E - U_C) - eps_W*(U_C - U_W))
 *         + (eps_N*(U_N - U_C) - eps_S*(U_C - U_S)).
 *   S5  XFLUX(U^n, sigma), every x-face between cells L = i and R = i+1:
 *       WALL face: all four terms 0.  Otherwise donor d = sigma > 0 ? R : L
 *       (INFLOW face: d = the ghost cell); fm = wet_d ? qx_d : 0 (INFLOW face:
 *       fm = qx_d unconditionally); Fm = fm, Fx = fm*u_d, Fy = fm*v_d.
 *       Pressure Px = (g*(0.5*(h+_L + h+_R)))*(eta_R - eta_L) on interior
 *       faces (h+ = max(h, 0)), 0 on boundary faces and on dry-bank faces
 *       (one side not wet and its z above the other side's eta).
 *   S6  YFLUX(U^n, sigma): S5 with x and y exchanged (Gm = fm from qy,
 *       Gx = fm*u_d, Gy = fm*v_d, Py from eta_N - eta_S).
 *   S7  PRED: rx = dt/dx, ry = dt/dy, P_x = sigma > 0 ? Px_E : Px_W (same in y)
 *       eta* = (eta - rx*(Fm_E - Fm_W)) - ry*(Gm_N - Gm_S)
 *       qx*  = (qx - rx*((Fx_E - Fx_W) + P_x)) - ry*(Gx_N - Gx_S)
 *       qy*  = (qy - rx*(Fy_E - Fy_W)) - ry*((Gy_N - Gy_S) + P_y)
 *   S8  BC(U*, t^n + dt): S1 applied to U*.
 *   S9  PRIM(U*).
 *   S10 XFLUX(U*, -sigma).   S11 YFLUX(U*, -sigma).
 *   S12 CORR: with the S10/S11 faces and -sigma for the pressure side, the S7
 *       expressions applied to U* give a; U^c = 0.5*(U^n + a).
 *   S13 ADD-DISS: U^d = U^c + D.
 *   S14 FRIC (point-implicit Manning), wet cells of U^d only:
 *       r = 1/h; s = sqrt(qx*qx + qy*qy)*r; k = r*cbrt3(r) (= h^(-4/3));
 *       phi = 1 + ((dt*m)*s)*k; psi = 1/phi; qx = qx*psi; qy = qy*psi.
 *   S15 DRY-FIX: h = eta - z; if h < 0: defect += (0 - h), eta = z.  Then if
 *       eta - z is not > h_dry: qx = qy = 0.  A non-finite value raises the
 *       NaN flag.
 *   S16 CFL: over wet cells of U^{n+1}: r = 1/h, u = qx*r, v = qy*r,
 *       c = sqrt(g*h), lam = (|u| + c)*(1/dx) + (|v| + c)*(1/dy); lam_max is
 *       the maximum.  dt^{n+1} = dt_fixed if dt_fixed > 0, else
 *       min(cfl/lam_max, dt_max) if lam_max > 0, else dt_max.
 *       t^{n+1} = t^n + dt^n.  dt^0 is S16 applied to U^0.
 * cbrt3(x), x > 0 normal: the exponent-thirding first guess (integer
 * arithmetic on the high 32 bits w of the IEEE-754 pattern of x: the guess
 * has high word w/3 + 0x2A9F7893 and low word 0, as in Kahan's cube-root
 * note) followed by two steps of Halley's method for
 * y^3 = x: t = (y*y)*y, y = y*((t + (x + x))/((t + t) + x)).  The guess is
 * within 3.3% and each Halley step triples the digits, leaving a relative
 * error below 7e-15.
 * q_in(t) is the piecewise-linear hydrograph (t_k, q_k), held constant before
 * its first and after its last point:
 *   q_in = q_k + ((t - t_k)/(t_{k+1} - t_k))*(q_{k+1} - q_k).
 *
 * Derivatives.  The step is written once, generic over its number type S, and
 * instantiated three times:
 *   S = double  the oracle step itself (every operation as listed above);
 *   S = Dual    value and one directional derivative carried together
 *               (forward mode): the tangent of the loss along (dn, dz);
 *   S = Rev     value and a node on a tape of the operations of one step
 *               (reverse mode): replaying the tape backwards from the
 *               adjoint of U^{n+1} gives the adjoint of U^n and the
 *               step's contributions to dJ/dn and dJ/dz.
 * Branches (wet/dry tests, bank rule, max/min, clipping) are taken on the
 * values, so the three instantiations follow the same path and their values
 * are bit for bit those of the double step.  The derivative is that of the
 * operations executed: a selected branch passes its derivative, a constant
 * (a ghost's inflow, zeroed discharge, the cube root's first guess) has none,
 * max/min pass the argument they return (the second on a tie), |x| has
 * derivative sign(x) (0 at 0) and sqrt has derivative 0 at 0.  dt^n is not
 * differentiated: the loss is a function of (n, z) with the sequence of time
 * steps of a forward run held fixed.
 * Loss: J = sum over observation steps s = k*obs_every (k = 1, 2, ...,
 * s <= nsteps) and gauges g (flattened cell index j*nx + i) of
 * (h_g^s - hobs[k-1][g])^2, h^s = eta^s - z the depth after step s.
 */
#define _POSIX_C_SOURCE 199309L
#include <math.h>
#include <time.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <vector>
#if defined(_OPENMP)
#include <omp.h>
#endif

enum { BC_WALL = 0, BC_OPEN = 1, BC_INFLOW = 2, FACE_INTERIOR = 3 };
enum { EDGE_W = 0, EDGE_E = 1, EDGE_S = 2, EDGE_N = 3 };
enum { ORC_FLAG_NAN = 1u, ORC_FLAG_CLIPPED = 2u, ORC_FLAG_BADDT = 4u };

/* Number of padded arrays one traced step exposes, and scalar slots. */
#define ORC_NTRACE 47
#define ORC_NSCALAR 16

extern "C" {

typedef struct orc_cfg {
    int32_t nx, ny;
    int32_t bc[4];      /* W, E, S, N: BC_WALL, BC_OPEN or BC_INFLOW */
    int32_t in_lo[4];   /* INFLOW face band [lo, hi) along each edge */
    int32_t in_hi[4];
    int32_t hydro_len;  /* number of hydrograph points (0: q_in = 0) */
    int32_t pad_;
    double dx, dy, g, cfl, h_dry, kappa, eps_max, dt_max, dt_fixed;
    const double *hydro_t, *hydro_q;
    double h_film;      /* > 0: thin-film depth of S2/S9's reciprocal (reading); 0: off */
} orc_cfg;

typedef struct orc_stats {
    int64_t steps;      /* steps taken by the call */
    int64_t bad_step;   /* global index of the step that raised a flag, -1 none */
    uint32_t flags;
    uint32_t pad_;
    double t, dt;       /* time and next time step after the call */
    double dt_min, dt_max;  /* extremes of the time steps used */
    double volume;      /* sum of h dx dy over the final state */
    double defect;      /* clipped volume added during the call */
    double lambda_max;  /* lam_max of the final state */
    double loop_seconds;    /* wall time of the step loop alone (no setup) */
} orc_stats;

}  /* extern "C" */

namespace {

/* ------------------------------------------------------- number types */

/* Forward mode: value and one directional derivative. */
struct Dual {
    double v, d;
    Dual() : v(0.0), d(0.0) {}
    Dual(double x) : v(x), d(0.0) {}
    Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
    double q = a.v / b.v;
    return Dual(q, (a.d - q * b.d) / b.v);
}

/* Reverse mode: value and the index of its node on the tape of the current
 * step (-1 for a constant).  A node records up to two operands and the
 * partial derivatives of the result with respect to them. */
struct Node {
    int32_t a, b;
    double da, db;
};
std::vector<Node> g_tape;

struct Rev {
    double v;
    int32_t id;
    Rev() : v(0.0), id(-1) {}
    Rev(double x) : v(x), id(-1) {}
    Rev(double x, int32_t i) : v(x), id(i) {}
};
inline Rev rnode(double v, int32_t a, double da, int32_t b, double db) {
    if (a < 0 && b < 0) return Rev(v);
    g_tape.push_back(Node{a, b, da, db});
    return Rev(v, (int32_t)g_tape.size() - 1);
}
inline Rev rleaf(double v) {
    g_tape.push_back(Node{-1, -1, 0.0, 0.0});
    return Rev(v, (int32_t)g_tape.size() - 1);
}
inline Rev operator+(Rev a, Rev b) { return rnode(a.v + b.v, a.id, 1.0, b.id, 1.0); }
inline Rev operator-(Rev a, Rev b) { return rnode(a.v - b.v, a.id, 1.0, b.id, -1.0); }
inline Rev operator-(Rev a) { return rnode(-a.v, a.id, -1.0, -1, 0.0); }
inline Rev operator*(Rev a, Rev b) { return rnode(a.v * b.v, a.id, b.v, b.id, a.v); }
inline Rev operator/(Rev a, Rev b) {
    double q = a.v / b.v;
    return rnode(q, a.id, 1.0 / b.v, b.id, -q / b.v);
}

/* Single precision: value rounded to IEEE-754 binary32 after every
 * operation (constants are rounded when they enter an operation).  The step
 * instantiated with it is a rounding reference for FP32 state: how far plain
 * float arithmetic, correctly rounded, drifts from the double step on a given
 * workload (orc_run_f32). */
struct F32 {
    float v;
    F32() : v(0.0f) {}
    F32(double x) : v((float)x) {}
};
inline F32 mkf(float x) {
    F32 r;
    r.v = x;
    return r;
}
inline F32 operator+(F32 a, F32 b) { return mkf(a.v + b.v); }
inline F32 operator-(F32 a, F32 b) { return mkf(a.v - b.v); }
inline F32 operator-(F32 a) { return mkf(-a.v); }
inline F32 operator*(F32 a, F32 b) { return mkf(a.v * b.v); }
inline F32 operator/(F32 a, F32 b) { return mkf(a.v / b.v); }

inline double val(double x) { return x; }
inline double val(Dual x) { return x.v; }
inline double val(Rev x) { return x.v; }
inline double val(F32 x) { return (double)x.v; }

inline double sfabs(double x) { return fabs(x); }
inline Dual sfabs(Dual x) { return Dual(fabs(x.v), x.v > 0.0 ? x.d : (x.v < 0.0 ? -x.d : 0.0)); }
inline Rev sfabs(Rev x) {
    return rnode(fabs(x.v), x.id, x.v > 0.0 ? 1.0 : (x.v < 0.0 ? -1.0 : 0.0), -1, 0.0);
}
inline F32 sfabs(F32 x) { return mkf(fabsf(x.v)); }
inline F32 ssqrt(F32 x) { return mkf(sqrtf(x.v)); }
inline double ssqrt(double x) { return sqrt(x); }
inline Dual ssqrt(Dual x) {
    double s = sqrt(x.v);
    return Dual(s, x.v > 0.0 ? x.d * (0.5 / s) : 0.0);
}
inline Rev ssqrt(Rev x) {
    double s = sqrt(x.v);
    return rnode(s, x.id, x.v > 0.0 ? 0.5 / s : 0.0, -1, 0.0);
}

/* ---------------------------------------------------------------- helpers */

/* Built with -fopenmp (the benchmark's all-core CPU figure only), the cell
 * sweeps of the double step run their rows on all host threads.  Every cell
 * of a sweep is computed from the previous sweep's arrays alone (§1: any
 * cell order gives the same result), so the state is bit for bit that of the
 * serial build; the sums (clipped volume, volume, lam_max) stay serial.  The
 * other number types run serially (the reverse tape is one global list). */
#if defined(_OPENMP)
#define SWEEP_PARALLEL _Pragma("omp parallel for schedule(static) if (sweep_parallel<S>::on)")
#else
#define SWEEP_PARALLEL
#endif
template <typename S> struct sweep_parallel { static const bool on = false; };
template <> struct sweep_parallel<double> { static const bool on = true; };

typedef struct {
    int nx, ny, P;      /* P = nx + 2: padded row length */
} Grid;

inline size_t at(const Grid* G, int i, int j) {
    return (size_t)(j + 1) * (size_t)G->P + (size_t)(i + 1);
}

int face_kind(const orc_cfg* c, int edge, int k) {
    int kind = c->bc[edge];
    if (kind == BC_INFLOW && !(k >= c->in_lo[edge] && k < c->in_hi[edge])) return BC_WALL;
    return kind;
}

double q_inflow(const orc_cfg* c, double t) {
    int L = c->hydro_len;
    if (L <= 0) return 0.0;
    if (t <= c->hydro_t[0]) return c->hydro_q[0];
    if (t >= c->hydro_t[L - 1]) return c->hydro_q[L - 1];
    int k = 0;
    while (k + 1 < L && !(t < c->hydro_t[k + 1])) ++k;
    double w = (t - c->hydro_t[k]) / (c->hydro_t[k + 1] - c->hydro_t[k]);
    return c->hydro_q[k] + w * (c->hydro_q[k + 1] - c->hydro_q[k]);
}

template <typename S> inline S pos(S h) { return val(h) > 0.0 ? h : S(0.0); }
template <typename S> inline S dmax(S a, S b) { return val(a) > val(b) ? a : b; }
template <typename S> inline S dmin(S a, S b) { return val(a) < val(b) ? a : b; }

/* Cube root of x > 0 (normal): exponent-thirding guess, two Halley steps. */
template <typename S> S cbrt3(S x) {
    double xv = val(x);
    uint64_t b;
    memcpy(&b, &xv, sizeof b);
    uint32_t w = (uint32_t)(b >> 32);
    b = (uint64_t)(w / 3u + 0x2A9F7893u) << 32;
    double y0;
    memcpy(&y0, &b, sizeof y0);
    S y = S(y0);
    for (int k = 0; k < 2; ++k) {
        S t = (y * y) * y;
        y = y * ((t + (x + x)) / ((t + t) + x));
    }
    return y;
}

/* Work arrays of one step, in trace order; each is a padded (ny+2) x (nx+2)
 * array.  Face arrays store the face between cells i and i+1 (x) or j and j+1
 * (y) in the slot of cell i (resp. j), so faces -1/2 sit in the ghost slot. */
template <typename S> struct Work {
    S *Un[3];           /* S1   */
    S *h, *r, *u, *v;   /* S2   */
    S *nux, *nuy;       /* S3   */
    S *D[3];            /* S4   */
    S *F[4];            /* S5: Fm, Fx, Fy, Px */
    S *G[4];            /* S6: Gm, Gx, Gy, Py */
    S *Us[3];           /* S7 interior + S8 ghosts */
    S *hs, *rs, *us, *vs;   /* S9 */
    S *Fs[4];           /* S10  */
    S *Gs[4];           /* S11  */
    S *Uc[3];           /* S12  */
    S *Ud[3];           /* S13  */
    S *Uf[3];           /* S14  */
    S *Unew[3];         /* S15  */
    S *zp, *mp;         /* padded bed and m = g n^2 */
    std::vector<S> store;

    /* Carve the ORC_NTRACE arrays and zp, mp out of `block` (or of own
     * storage when block is null). */
    void init(const Grid* grid, S* block) {
        size_t N = (size_t)grid->P * (size_t)(grid->ny + 2);
        if (!block) {
            store.assign((size_t)(ORC_NTRACE + 2) * N, S(0.0));
            block = store.data();
        } else {
            for (size_t k = 0; k < (size_t)ORC_NTRACE * N; ++k) block[k] = S(0.0);
        }
        S* p[ORC_NTRACE];
        for (int k = 0; k < ORC_NTRACE; ++k) p[k] = block + (size_t)k * N;
        int k = 0;
        for (int a = 0; a < 3; ++a) Un[a] = p[k++];
        h = p[k++]; r = p[k++]; u = p[k++]; v = p[k++];
        nux = p[k++]; nuy = p[k++];
        for (int a = 0; a < 3; ++a) D[a] = p[k++];
        for (int a = 0; a < 4; ++a) F[a] = p[k++];
        for (int a = 0; a < 4; ++a) G[a] = p[k++];
        for (int a = 0; a < 3; ++a) Us[a] = p[k++];
        hs = p[k++]; rs = p[k++]; us = p[k++]; vs = p[k++];
        for (int a = 0; a < 4; ++a) Fs[a] = p[k++];
        for (int a = 0; a < 4; ++a) Gs[a] = p[k++];
        for (int a = 0; a < 3; ++a) Uc[a] = p[k++];
        for (int a = 0; a < 3; ++a) Ud[a] = p[k++];
        for (int a = 0; a < 3; ++a) Uf[a] = p[k++];
        for (int a = 0; a < 3; ++a) Unew[a] = p[k++];
        zp = mp = nullptr;
        if (!store.empty()) {
            zp = store.data() + (size_t)ORC_NTRACE * N;
            mp = zp + N;
        }
    }
};

/* Padded copies of the static fields: z and m = g n^2, ghosts = adjacent. */
template <typename S>
void static_fields(const orc_cfg* c, const Grid* G, const S* z, const S* nman, S* zp, S* mp) {
    int nx = G->nx, ny = G->ny;
    for (int j = -1; j <= ny; ++j)
        for (int i = -1; i <= nx; ++i) {
            int ii = i < 0 ? 0 : (i >= nx ? nx - 1 : i);
            int jj = j < 0 ? 0 : (j >= ny ? ny - 1 : j);
            int corner = (i < 0 || i >= nx) && (j < 0 || j >= ny);
            size_t s = (size_t)jj * (size_t)nx + (size_t)ii;
            S nn = nman[s];
            zp[at(G, i, j)] = corner ? S(0.0) : z[s];
            mp[at(G, i, j)] = corner ? S(0.0) : c->g * (nn * nn);
        }
}

/* ------------------------------------------------------------- sub-steps */

/* S1 / S8: ghost ring of (eta, qx, qy) for the boundary kinds at time t. */
template <typename S>
void fill_ghosts(const orc_cfg* c, const Grid* G, double qin, S* eta, S* qx, S* qy) {
    int nx = G->nx, ny = G->ny;
    for (int j = 0; j < ny; ++j) {
        for (int side = 0; side < 2; ++side) {
            int edge = side == 0 ? EDGE_W : EDGE_E;
            size_t g = side == 0 ? at(G, -1, j) : at(G, nx, j);
            size_t a = side == 0 ? at(G, 0, j) : at(G, nx - 1, j);
            int kind = face_kind(c, edge, j);
            eta[g] = eta[a];
            if (kind == BC_OPEN) {
                qx[g] = qx[a];
                qy[g] = qy[a];
            } else if (kind == BC_INFLOW) {
                qx[g] = S(side == 0 ? qin : -qin);
                qy[g] = S(0.0);
            } else {
                qx[g] = -qx[a];
                qy[g] = qy[a];
            }
        }
    }
    for (int i = 0; i < nx; ++i) {
        for (int side = 0; side < 2; ++side) {
            int edge = side == 0 ? EDGE_S : EDGE_N;
            size_t g = side == 0 ? at(G, i, -1) : at(G, i, ny);
            size_t a = side == 0 ? at(G, i, 0) : at(G, i, ny - 1);
            int kind = face_kind(c, edge, i);
            eta[g] = eta[a];
            if (kind == BC_OPEN) {
                qx[g] = qx[a];
                qy[g] = qy[a];
            } else if (kind == BC_INFLOW) {
                qy[g] = S(side == 0 ? qin : -qin);
                qx[g] = S(0.0);
            } else {
                qy[g] = -qy[a];
                qx[g] = qx[a];
            }
        }
    }
}

/* S2 / S9: primitive variables over every padded cell. */
template <typename S>
void prim(const orc_cfg* c, const Grid* G, S* const U[3], const S* zp, S* h, S* r, S* u, S* v) {
    size_t N = (size_t)G->P * (size_t)(G->ny + 2);
    SWEEP_PARALLEL
    for (size_t s = 0; s < N; ++s) {
        S hh = U[0][s] - zp[s];
        S rr = val(hh) > c->h_dry ? S(1.0) / hh : S(0.0);
        if (c->h_film > 0.0) rr = dmin(rr, S(1.0 / c->h_film));   /* thin-film reading */
        h[s] = hh;
        r[s] = rr;
        u[s] = U[1][s] * rr;
        v[s] = U[2][s] * rr;
    }
}

/* S3: dissipation switch from the curvature of the water surface. */
template <typename S>
void switch_nu(const Grid* G, const S* eta, const S* r, S* nux, S* nuy) {
    SWEEP_PARALLEL
    for (int j = 0; j < G->ny; ++j)
        for (int i = 0; i < G->nx; ++i) {
            size_t C = at(G, i, j);
            S ax = eta[at(G, i + 1, j)] - eta[C];
            S bx = eta[C] - eta[at(G, i - 1, j)];
            S ay = eta[at(G, i, j + 1)] - eta[C];
            S by = eta[C] - eta[at(G, i, j - 1)];
            nux[C] = S(0.25) * (sfabs(ax - bx) * r[C]);
            nuy[C] = S(0.25) * (sfabs(ay - by) * r[C]);
        }
}

/* Face coefficient of S4 between cells a and b (interior faces only). */
template <typename S>
S eps_face(const orc_cfg* c, const S* h, const S* nu, size_t a, size_t b) {
    if (!(val(h[a]) > c->h_dry && val(h[b]) > c->h_dry)) return S(0.0);
    return dmin(S(c->kappa) * dmax(nu[a], nu[b]), S(c->eps_max));
}

/* S4: switched second-difference dissipation of U^n. */
template <typename S>
void dissipation(const orc_cfg* c, const Grid* G, S* const U[3], const S* h, const S* nux,
                 const S* nuy, S* D[3]) {
    int nx = G->nx, ny = G->ny;
    SWEEP_PARALLEL
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t C = at(G, i, j), E = at(G, i + 1, j), W = at(G, i - 1, j);
            size_t N = at(G, i, j + 1), Sd = at(G, i, j - 1);
            S eE = i + 1 < nx ? eps_face(c, h, nux, C, E) : S(0.0);
            S eW = i > 0 ? eps_face(c, h, nux, W, C) : S(0.0);
            S eN = j + 1 < ny ? eps_face(c, h, nuy, C, N) : S(0.0);
            S eS = j > 0 ? eps_face(c, h, nuy, Sd, C) : S(0.0);
            for (int a = 0; a < 3; ++a) {
                const S* q = U[a];
                S dxq = eE * (q[E] - q[C]) - eW * (q[C] - q[W]);
                S dyq = eN * (q[N] - q[C]) - eS * (q[C] - q[Sd]);
                D[a][C] = dxq + dyq;
            }
        }
}

/* One face of S5/S6/S10/S11.  L and R are the cells on the low and high side
 * of the face, ghost_is_R says which of them is the ghost of a boundary face,
 * kind is the face kind, qn is the discharge normal to the face, and the
 * outputs are (mass, x-momentum, y-momentum, pressure). */
template <typename S>
void face_flux(const orc_cfg* c, int sigma, int kind, size_t L, size_t R, int ghost_is_R,
               const S* eta, const S* qn, const S* h, const S* u, const S* v, const S* zp,
               S out[4]) {
    if (kind == BC_WALL) {
        out[0] = out[1] = out[2] = out[3] = S(0.0);
        return;
    }
    size_t d;
    S fm;
    if (kind == BC_INFLOW) {
        d = ghost_is_R ? R : L;
        fm = qn[d];
    } else {
        d = sigma > 0 ? R : L;
        fm = val(h[d]) > c->h_dry ? qn[d] : S(0.0);
    }
    out[0] = fm;
    out[1] = fm * u[d];
    out[2] = fm * v[d];
    if (kind != FACE_INTERIOR) {
        out[3] = S(0.0);
        return;
    }
    int wetL = val(h[L]) > c->h_dry, wetR = val(h[R]) > c->h_dry;
    int bank = (!wetL && val(zp[L]) > val(eta[R])) || (!wetR && val(zp[R]) > val(eta[L]));
    out[3] = bank ? S(0.0)
                  : (S(c->g) * (S(0.5) * (pos(h[L]) + pos(h[R])))) * (eta[R] - eta[L]);
}

/* S5 / S10: fluxes through every x-face (i = -1 .. nx-1). */
template <typename S>
void xflux(const orc_cfg* c, const Grid* G, int sigma, S* const U[3], const S* h, const S* u,
           const S* v, const S* zp, S* F[4]) {
    int nx = G->nx, ny = G->ny;
    SWEEP_PARALLEL
    for (int j = 0; j < ny; ++j)
        for (int i = -1; i < nx; ++i) {
            int kind = i == -1 ? face_kind(c, EDGE_W, j)
                               : (i == nx - 1 ? face_kind(c, EDGE_E, j) : FACE_INTERIOR);
            S o[4];
            face_flux(c, sigma, kind, at(G, i, j), at(G, i + 1, j), i == nx - 1, U[0], U[1], h,
                      u, v, zp, o);
            size_t s = at(G, i, j);
            for (int a = 0; a < 4; ++a) F[a][s] = o[a];
        }
}

/* S6 / S11: fluxes through every y-face (j = -1 .. ny-1). */
template <typename S>
void yflux(const orc_cfg* c, const Grid* G, int sigma, S* const U[3], const S* h, const S* u,
           const S* v, const S* zp, S* Gf[4]) {
    int nx = G->nx, ny = G->ny;
    SWEEP_PARALLEL
    for (int j = -1; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            int kind = j == -1 ? face_kind(c, EDGE_S, i)
                               : (j == ny - 1 ? face_kind(c, EDGE_N, i) : FACE_INTERIOR);
            S o[4];
            face_flux(c, sigma, kind, at(G, i, j), at(G, i, j + 1), j == ny - 1, U[0], U[2], h,
                      u, v, zp, o);
            size_t s = at(G, i, j);
            for (int a = 0; a < 4; ++a) Gf[a][s] = o[a];
        }
}

/* S7 (base = U^n, out = U*) and the inner part of S12 (base = U*): the flux
 * divergence update base - L_sigma with the pressure on the sigma-side face. */
template <typename S>
void flux_update(const Grid* G, int sigma, double rx, double ry, S* const base[3],
                 S* const F[4], S* const Gf[4], S* out[3]) {
    S RX(rx), RY(ry);
    SWEEP_PARALLEL
    for (int j = 0; j < G->ny; ++j)
        for (int i = 0; i < G->nx; ++i) {
            size_t C = at(G, i, j), W = at(G, i - 1, j), Sd = at(G, i, j - 1);
            S px = sigma > 0 ? F[3][C] : F[3][W];
            S py = sigma > 0 ? Gf[3][C] : Gf[3][Sd];
            out[0][C] = (base[0][C] - RX * (F[0][C] - F[0][W])) - RY * (Gf[0][C] - Gf[0][Sd]);
            out[1][C] = (base[1][C] - RX * ((F[1][C] - F[1][W]) + px)) - RY * (Gf[1][C] - Gf[1][Sd]);
            out[2][C] = (base[2][C] - RX * (F[2][C] - F[2][W])) - RY * ((Gf[2][C] - Gf[2][Sd]) + py);
        }
}

/* S12: U^c = 0.5*(U^n + (U* - L_{-sigma}(U*))). */
template <typename S>
void corrector(const Grid* G, int sigma, double rx, double ry, S* const Un[3], S* const Us[3],
               S* const Fs[4], S* const Gs[4], S* Uc[3]) {
    flux_update(G, -sigma, rx, ry, Us, Fs, Gs, Uc);
    SWEEP_PARALLEL
    for (int j = 0; j < G->ny; ++j)
        for (int i = 0; i < G->nx; ++i) {
            size_t C = at(G, i, j);
            for (int a = 0; a < 3; ++a) Uc[a][C] = S(0.5) * (Un[a][C] + Uc[a][C]);
        }
}

/* S13 */
template <typename S>
void add_diss(const Grid* G, S* const Uc[3], S* const D[3], S* Ud[3]) {
    SWEEP_PARALLEL
    for (int j = 0; j < G->ny; ++j)
        for (int i = 0; i < G->nx; ++i) {
            size_t C = at(G, i, j);
            for (int a = 0; a < 3; ++a) Ud[a][C] = Uc[a][C] + D[a][C];
        }
}

/* S14: point-implicit Manning friction on wet cells. */
template <typename S>
void friction(const orc_cfg* c, const Grid* G, double dt, S* const Ud[3], const S* zp,
              const S* mp, S* Uf[3]) {
    SWEEP_PARALLEL
    for (int j = 0; j < G->ny; ++j)
        for (int i = 0; i < G->nx; ++i) {
            size_t C = at(G, i, j);
            S eta = Ud[0][C], qx = Ud[1][C], qy = Ud[2][C];
            S h = eta - zp[C];
            if (val(h) > c->h_dry) {
                S r = S(1.0) / h;
                S s = ssqrt(qx * qx + qy * qy) * r;
                S k = r * cbrt3(r);
                S phi = S(1.0) + ((S(dt) * mp[C]) * s) * k;
                S psi = S(1.0) / phi;
                qx = qx * psi;
                qy = qy * psi;
            }
            Uf[0][C] = eta;
            Uf[1][C] = qx;
            Uf[2][C] = qy;
        }
}

/* S15: clip negative depth (volume recorded), zero the discharge of dry
 * cells, raise the NaN flag on non-finite values.  Returns sum of (0 - h). */
template <typename S>
double dry_fix(const orc_cfg* c, const Grid* G, S* const Uf[3], const S* zp, S* Un1[3],
               uint32_t* flags) {
    double defect = 0.0;
    for (int j = 0; j < G->ny; ++j)
        for (int i = 0; i < G->nx; ++i) {
            size_t C = at(G, i, j);
            S eta = Uf[0][C], qx = Uf[1][C], qy = Uf[2][C];
            double h = val(eta) - val(zp[C]);
            if (h < 0.0) {
                defect += 0.0 - h;
                eta = zp[C];
                *flags |= ORC_FLAG_CLIPPED;
            }
            if (!(val(eta) - val(zp[C]) > c->h_dry)) {
                qx = S(0.0);
                qy = S(0.0);
            }
            if (!isfinite(val(eta)) || !isfinite(val(qx)) || !isfinite(val(qy)))
                *flags |= ORC_FLAG_NAN;
            Un1[0][C] = eta;
            Un1[1][C] = qx;
            Un1[2][C] = qy;
        }
    return defect;
}

/* S16 on an unpadded state (pitch nx): lam_max and the volume sum of h. */
void cfl_scan(const orc_cfg* c, int nx, int ny, const double* eta, const double* qx,
              const double* qy, const double* z, double* lam_max, double* hsum) {
    double idx = 1.0 / c->dx, idy = 1.0 / c->dy;
    double lmax = 0.0, vs = 0.0;
    size_t N = (size_t)nx * (size_t)ny;
    for (size_t s = 0; s < N; ++s) {
        double h = eta[s] - z[s];
        vs += h;
        if (h > c->h_dry) {
            double r = 1.0 / h;
            double u = qx[s] * r, v = qy[s] * r;
            double cc = sqrt(c->g * h);
            double lam = (fabs(u) + cc) * idx + (fabs(v) + cc) * idy;
            if (!(lam <= lmax)) lmax = lam;  /* a NaN lam propagates */
        }
    }
    *lam_max = lmax;
    *hsum = vs;
}

/* S16 in the arithmetic of S (the binary32 run): lam_max and the volume sum
 * of h, both returned in double. */
template <typename S>
void cfl_scan_s(const orc_cfg* c, int nx, int ny, const S* eta, const S* qx, const S* qy,
                const S* z, double* lam_max, double* hsum) {
    S idx = S(1.0 / c->dx), idy = S(1.0 / c->dy), g = S(c->g);
    double lmax = 0.0, vs = 0.0;
    size_t N = (size_t)nx * (size_t)ny;
    for (size_t s = 0; s < N; ++s) {
        S h = eta[s] - z[s];
        vs += val(h);
        if (val(h) > c->h_dry) {
            S r = S(1.0) / h;
            S u = qx[s] * r, v = qy[s] * r;
            S cc = ssqrt(g * h);
            double lam = val((sfabs(u) + cc) * idx + (sfabs(v) + cc) * idy);
            if (!(lam <= lmax)) lmax = lam;
        }
    }
    *lam_max = lmax;
    *hsum = vs;
}

double next_dt(const orc_cfg* c, double lam_max) {
    if (c->dt_fixed > 0.0) return c->dt_fixed;
    if (lam_max > 0.0) return dmin(c->cfl / lam_max, c->dt_max);
    return c->dt_max;
}

/* ------------------------------------------------------------ one step */

typedef struct {
    double qin_n, qin_n1, rx, ry, defect;
    uint32_t flags;
} StepOut;

/* S1..S15 of step n (t = t^n, dt = dt^n) on the unpadded state (pitch nx),
 * advanced in place; zp and mp are the padded static fields. */
template <typename S>
void step_body(const orc_cfg* c, const Grid* G, Work<S>* w, S* eta, S* qx, S* qy, double t,
               int64_t n, double dt, StepOut* o) {
    int nx = G->nx, ny = G->ny;
    int sigma = (n & 1) ? -1 : 1;
    double rx = dt / c->dx, ry = dt / c->dy;
    double qin0 = q_inflow(c, t);
    double qin1 = q_inflow(c, t + dt);
    /* S1: copy U^n into the padded arrays and build its ghost ring. */
    SWEEP_PARALLEL
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t s = (size_t)j * (size_t)nx + (size_t)i;
            w->Un[0][at(G, i, j)] = eta[s];
            w->Un[1][at(G, i, j)] = qx[s];
            w->Un[2][at(G, i, j)] = qy[s];
        }
    fill_ghosts(c, G, qin0, w->Un[0], w->Un[1], w->Un[2]);
    prim(c, G, w->Un, w->zp, w->h, w->r, w->u, w->v);                       /* S2 */
    switch_nu(G, w->Un[0], w->r, w->nux, w->nuy);                           /* S3 */
    dissipation(c, G, w->Un, w->h, w->nux, w->nuy, w->D);                   /* S4 */
    xflux(c, G, sigma, w->Un, w->h, w->u, w->v, w->zp, w->F);               /* S5 */
    yflux(c, G, sigma, w->Un, w->h, w->u, w->v, w->zp, w->G);               /* S6 */
    flux_update(G, sigma, rx, ry, w->Un, w->F, w->G, w->Us);                /* S7 */
    fill_ghosts(c, G, qin1, w->Us[0], w->Us[1], w->Us[2]);                  /* S8 */
    prim(c, G, w->Us, w->zp, w->hs, w->rs, w->us, w->vs);                   /* S9 */
    xflux(c, G, -sigma, w->Us, w->hs, w->us, w->vs, w->zp, w->Fs);          /* S10 */
    yflux(c, G, -sigma, w->Us, w->hs, w->us, w->vs, w->zp, w->Gs);          /* S11 */
    corrector(G, sigma, rx, ry, w->Un, w->Us, w->Fs, w->Gs, w->Uc);         /* S12 */
    add_diss(G, w->Uc, w->D, w->Ud);                                        /* S13 */
    friction(c, G, dt, w->Ud, w->zp, w->mp, w->Uf);                         /* S14 */
    uint32_t flags = 0;
    double defect = dry_fix(c, G, w->Uf, w->zp, w->Unew, &flags);           /* S15 */
    SWEEP_PARALLEL
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t s = (size_t)j * (size_t)nx + (size_t)i;
            eta[s] = w->Unew[0][at(G, i, j)];
            qx[s] = w->Unew[1][at(G, i, j)];
            qy[s] = w->Unew[2][at(G, i, j)];
        }
    o->qin_n = qin0;
    o->qin_n1 = qin1;
    o->rx = rx;
    o->ry = ry;
    o->defect = defect;
    o->flags = flags;
}

typedef struct {
    double qin_n, qin_n1, rx, ry, defect, lam_max, dt_next, volume, t_next;
    uint32_t flags;
} StepInfo;

/* The oracle step: S1..S15, then S16 on the new state. */
void one_step(const orc_cfg* c, const Grid* G, Work<double>* w, const double* z, double* eta,
              double* qx, double* qy, double t, int64_t n, double dt, StepInfo* o) {
    StepOut so;
    step_body(c, G, w, eta, qx, qy, t, n, dt, &so);
    uint32_t flags = so.flags;
    double lam, hsum;
    cfl_scan(c, G->nx, G->ny, eta, qx, qy, z, &lam, &hsum);
    double dtn = next_dt(c, lam);
    if (!isfinite(lam)) flags |= ORC_FLAG_NAN;
    if (!(dtn > 0.0) || !isfinite(dtn)) flags |= ORC_FLAG_BADDT;
    o->qin_n = so.qin_n;
    o->qin_n1 = so.qin_n1;
    o->rx = so.rx;
    o->ry = so.ry;
    o->defect = so.defect;
    o->lam_max = lam;
    o->dt_next = dtn;
    o->volume = hsum * (c->dx * c->dy);
    o->t_next = t + dt;
    o->flags = flags;
}

int check_cfg(const orc_cfg* c) {
    if (c->nx < 1 || c->ny < 1) return -1;
    if (!(c->dx > 0.0) || !(c->dy > 0.0)) return -1;
    if (c->hydro_len > 0 && (!c->hydro_t || !c->hydro_q)) return -1;
    for (int k = 0; k < 4; ++k)
        if (c->bc[k] < BC_WALL || c->bc[k] > BC_INFLOW) return -1;
    return 0;
}

/* ------------------------------------------------------------ the loss */

struct LossSpec {
    int64_t nsteps;
    const double* dts;      /* dt^n of the steps, held fixed */
    int32_t ngauge;
    const int64_t* gauges;  /* flattened cell indices j*nx + i */
    int32_t obs_every;
    const double* hobs;     /* [nobs][ngauge] */
};

int check_loss(const orc_cfg* c, const LossSpec* L) {
    if (L->nsteps < 0 || !L->dts || L->ngauge < 0 || L->obs_every < 1) return -1;
    if (L->ngauge > 0 && (!L->gauges || !L->hobs)) return -1;
    int64_t N = (int64_t)c->nx * c->ny;
    for (int32_t g = 0; g < L->ngauge; ++g)
        if (L->gauges[g] < 0 || L->gauges[g] >= N) return -1;
    return 0;
}

/* Misfit of the observation after step s (s a multiple of obs_every). */
template <typename S>
S misfit(const LossSpec* L, int64_t s, const S* eta, const S* z) {
    S J = S(0.0);
    const double* ho = L->hobs + (size_t)(s / L->obs_every - 1) * (size_t)L->ngauge;
    for (int32_t g = 0; g < L->ngauge; ++g) {
        int64_t k = L->gauges[g];
        S d = (eta[k] - z[k]) - S(ho[g]);
        J = J + d * d;
    }
    return J;
}

/* Forward pass over the loss's steps with number type S; returns J. */
template <typename S>
S loss_forward(const orc_cfg* c, const LossSpec* L, S* eta, S* qx, S* qy, const S* z,
               const S* nman, double t0, int64_t step0) {
    Grid G = {c->nx, c->ny, c->nx + 2};
    Work<S> w;
    w.init(&G, nullptr);
    static_fields(c, &G, z, nman, w.zp, w.mp);
    S J = S(0.0);
    double t = t0;
    for (int64_t k = 0; k < L->nsteps; ++k) {
        StepOut so;
        step_body(c, &G, &w, eta, qx, qy, t, step0 + k, L->dts[k], &so);
        t = t + L->dts[k];
        if ((k + 1) % L->obs_every == 0) J = J + misfit(L, k + 1, eta, z);
    }
    return J;
}

}  // namespace

/* ------------------------------------------------------------ public API */

extern "C" {

int orc_ntrace(void) { return ORC_NTRACE; }

/* Threads the cell sweeps run on (1 unless built with -fopenmp). */
int orc_threads(void) {
#if defined(_OPENMP)
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* The friction step's cube root, exposed so that it can be pinned. */
double orc_cbrt3(double x) { return cbrt3(x); }
int orc_nscalar(void) { return ORC_NSCALAR; }

/* dt^0 of a state (S16) and its volume.  Returns dt; lam_max and volume are
 * written through the pointers when they are not NULL. */
double orc_initial_dt(const orc_cfg* c, const double* eta, const double* qx, const double* qy,
                      const double* z, double* lam_max, double* volume) {
    double lam, hsum;
    cfl_scan(c, c->nx, c->ny, eta, qx, qy, z, &lam, &hsum);
    if (lam_max) *lam_max = lam;
    if (volume) *volume = hsum * (c->dx * c->dy);
    return next_dt(c, lam);
}

/* Advance the state in place by up to nsteps steps, stopping early once
 * t >= t_end or when a step raises the NaN or bad-dt flag.  *t, *step and *dt
 * hold t^n, n and dt^n on entry (a *dt <= 0 means: compute dt^0 from the
 * state) and the values after the last step on return.  When dts is not NULL
 * it receives the dt^n of every step taken.  Returns 0 on success, 1 when a
 * step raised a fatal flag, -1 on bad arguments. */
int orc_run_record(const orc_cfg* c, double* eta, double* qx, double* qy, const double* z,
                   const double* nman, double* t, int64_t* step, double* dt, int64_t nsteps,
                   double t_end, orc_stats* st, double* dts) {
    if (check_cfg(c) || !eta || !qx || !qy || !z || !nman || !t || !step || !dt) return -1;
    Grid G = {c->nx, c->ny, c->nx + 2};
    Work<double> w;
    w.init(&G, nullptr);
    static_fields(c, &G, z, nman, w.zp, w.mp);
    if (!(*dt > 0.0)) *dt = orc_initial_dt(c, eta, qx, qy, z, NULL, NULL);
    orc_stats S;
    memset(&S, 0, sizeof S);
    S.bad_step = -1;
    S.dt_min = INFINITY;
    S.dt_max = 0.0;
    double lam = 0.0, vol;
    orc_initial_dt(c, eta, qx, qy, z, &lam, &vol);
    S.volume = vol;
    S.lambda_max = lam;
    int rc = 0;
    struct timespec ts0, ts1;
    clock_gettime(CLOCK_MONOTONIC, &ts0);
    for (int64_t k = 0; k < nsteps; ++k) {
        if (!(*t < t_end)) break;
        StepInfo o;
        one_step(c, &G, &w, z, eta, qx, qy, *t, *step, *dt, &o);
        if (dts) dts[k] = *dt;
        S.dt_min = dmin(S.dt_min, *dt);
        S.dt_max = dmax(S.dt_max, *dt);
        S.defect += o.defect * (c->dx * c->dy);
        S.flags |= o.flags;
        S.volume = o.volume;
        S.lambda_max = o.lam_max;
        S.steps += 1;
        *t = o.t_next;
        *dt = o.dt_next;
        *step += 1;
        if (o.flags & (ORC_FLAG_NAN | ORC_FLAG_BADDT)) {
            S.bad_step = *step - 1;
            rc = 1;
            break;
        }
    }
    clock_gettime(CLOCK_MONOTONIC, &ts1);
    S.loop_seconds = (double)(ts1.tv_sec - ts0.tv_sec) + 1e-9 * (double)(ts1.tv_nsec - ts0.tv_nsec);
    S.t = *t;
    S.dt = *dt;
    if (st) *st = S;
    return rc;
}

int orc_run(const orc_cfg* c, double* eta, double* qx, double* qy, const double* z,
            const double* nman, double* t, int64_t* step, double* dt, int64_t nsteps,
            double t_end, orc_stats* st) {
    return orc_run_record(c, eta, qx, qy, z, nman, t, step, dt, nsteps, t_end, st, NULL);
}

/* orc_run in binary32: the same sixteen sub-steps with every operation
 * rounded to float (inputs, which should already be float values, are
 * rounded on entry; g, h_dry, kappa and eps_max are rounded to float, as a
 * float implementation holds them).  t, dt and the volume stay double, and
 * dt^{n+1} is formed in double from the float lam_max.  A rounding
 * reference for FP32 state, not a parity target: a float implementation
 * that rounds differently (approximate reciprocals, another cube root)
 * drifts from the double step by an amount of the same order.  Returns as
 * orc_run. */
int orc_run_f32(const orc_cfg* c0, double* eta, double* qx, double* qy, const double* z,
                const double* nman, double* t, int64_t* step, double* dt, int64_t nsteps,
                double t_end, orc_stats* st) {
    if (check_cfg(c0) || !eta || !qx || !qy || !z || !nman || !t || !step || !dt) return -1;
    orc_cfg cf = *c0;
    cf.g = (double)(float)c0->g;
    cf.h_dry = (double)(float)c0->h_dry;
    cf.kappa = (double)(float)c0->kappa;
    cf.eps_max = (double)(float)c0->eps_max;
    const orc_cfg* c = &cf;
    Grid G = {c->nx, c->ny, c->nx + 2};
    const size_t N = (size_t)c->nx * (size_t)c->ny;
    std::vector<F32> e(N), a(N), b(N), zf(N), nf(N);
    for (size_t s = 0; s < N; ++s) {
        e[s] = F32(eta[s]);
        a[s] = F32(qx[s]);
        b[s] = F32(qy[s]);
        zf[s] = F32(z[s]);
        nf[s] = F32(nman[s]);
    }
    Work<F32> w;
    w.init(&G, nullptr);
    static_fields(c, &G, zf.data(), nf.data(), w.zp, w.mp);
    orc_stats S;
    memset(&S, 0, sizeof S);
    S.bad_step = -1;
    S.dt_min = INFINITY;
    S.dt_max = 0.0;
    double lam = 0.0, hs = 0.0;
    cfl_scan_s(c, c->nx, c->ny, e.data(), a.data(), b.data(), zf.data(), &lam, &hs);
    if (!(*dt > 0.0)) *dt = next_dt(c, lam);
    S.volume = hs * (c->dx * c->dy);
    S.lambda_max = lam;
    int rc = 0;
    for (int64_t k = 0; k < nsteps; ++k) {
        if (!(*t < t_end)) break;
        StepOut so;
        step_body(c, &G, &w, e.data(), a.data(), b.data(), *t, *step, *dt, &so);
        cfl_scan_s(c, c->nx, c->ny, e.data(), a.data(), b.data(), zf.data(), &lam, &hs);
        double dtn = next_dt(c, lam);
        uint32_t flags = so.flags;
        if (!isfinite(lam)) flags |= ORC_FLAG_NAN;
        if (!(dtn > 0.0) || !isfinite(dtn)) flags |= ORC_FLAG_BADDT;
        S.dt_min = dmin(S.dt_min, *dt);
        S.dt_max = dmax(S.dt_max, *dt);
        S.defect += so.defect * (c->dx * c->dy);
        S.flags |= flags;
        S.volume = hs * (c->dx * c->dy);
        S.lambda_max = lam;
        S.steps += 1;
        *t = *t + *dt;
        *dt = dtn;
        *step += 1;
        if (flags & (ORC_FLAG_NAN | ORC_FLAG_BADDT)) {
            S.bad_step = *step - 1;
            rc = 1;
            break;
        }
    }
    for (size_t s = 0; s < N; ++s) {
        eta[s] = val(e[s]);
        qx[s] = val(a[s]);
        qy[s] = val(b[s]);
    }
    S.t = *t;
    S.dt = *dt;
    if (st) *st = S;
    return rc;
}

/* One step with every intermediate exposed.  `arrays` receives ORC_NTRACE
 * padded (ny+2) x (nx+2) arrays in the order S1 (eta, qx, qy), S2 (h, r, u, v),
 * S3 (nu_x, nu_y), S4 (D_eta, D_qx, D_qy), S5 (Fm, Fx, Fy, Px), S6 (Gm, Gx,
 * Gy, Py), S7+S8 (eta*, qx*, qy*), S9 (h*, r*, u*, v*), S10 (4), S11 (4),
 * S12 (3), S13 (3), S14 (3), S15 (3).  `scalars` receives ORC_NSCALAR
 * values: q_in(t^n), q_in(t^n + dt), rx, ry, sum of clipped depth, lam_max,
 * dt^{n+1}, volume, flags, sigma, t^{n+1}; the rest 0.  The state is advanced
 * in place.  Returns 0, or -1 on bad arguments. */
int orc_trace(const orc_cfg* c, double* eta, double* qx, double* qy, const double* z,
              const double* nman, double t, int64_t step, double dt, double* arrays,
              double* scalars) {
    if (check_cfg(c) || !arrays || !scalars) return -1;
    Grid G = {c->nx, c->ny, c->nx + 2};
    Work<double> w;
    w.init(&G, arrays);
    size_t N = (size_t)G.P * (size_t)(G.ny + 2);
    std::vector<double> zm(2 * N, 0.0);
    w.zp = zm.data();
    w.mp = zm.data() + N;
    static_fields(c, &G, z, nman, w.zp, w.mp);
    StepInfo o;
    one_step(c, &G, &w, z, eta, qx, qy, t, step, dt, &o);
    for (int k = 0; k < ORC_NSCALAR; ++k) scalars[k] = 0.0;
    scalars[0] = o.qin_n;
    scalars[1] = o.qin_n1;
    scalars[2] = o.rx;
    scalars[3] = o.ry;
    scalars[4] = o.defect;
    scalars[5] = o.lam_max;
    scalars[6] = o.dt_next;
    scalars[7] = o.volume;
    scalars[8] = (double)o.flags;
    scalars[9] = (step & 1) ? -1.0 : 1.0;
    scalars[10] = o.t_next;
    return 0;
}

/* The gauge-misfit loss J of nsteps steps from (eta0, qx0, qy0) at t0, step0
 * with the time steps dts[0..nsteps) held fixed (see the loss definition at
 * the top).  With dn and dz both NULL, *J only; otherwise also the
 * directional derivative *dJ of J along the perturbation (dn, dz) of the
 * Manning and bed fields (a NULL direction is zero), by forward mode.
 * Returns 0, or -1 on bad arguments. */
int orc_loss_tangent(const orc_cfg* c, const double* eta0, const double* qx0, const double* qy0,
                     const double* z, const double* nman, double t0, int64_t step0,
                     int64_t nsteps, const double* dts, int32_t ngauge, const int64_t* gauges,
                     int32_t obs_every, const double* hobs, const double* dn, const double* dz,
                     double* J, double* dJ) {
    LossSpec L = {nsteps, dts, ngauge, gauges, obs_every, hobs};
    if (check_cfg(c) || check_loss(c, &L) || !eta0 || !qx0 || !qy0 || !z || !nman || !J)
        return -1;
    size_t N = (size_t)c->nx * (size_t)c->ny;
    if (!dn && !dz) {
        std::vector<double> e(eta0, eta0 + N), a(qx0, qx0 + N), b(qy0, qy0 + N);
        *J = loss_forward<double>(c, &L, e.data(), a.data(), b.data(), z, nman, t0, step0);
        if (dJ) *dJ = 0.0;
        return 0;
    }
    std::vector<Dual> e(N), a(N), b(N), zd(N), nd(N);
    for (size_t s = 0; s < N; ++s) {
        e[s] = Dual(eta0[s]);
        a[s] = Dual(qx0[s]);
        b[s] = Dual(qy0[s]);
        zd[s] = Dual(z[s], dz ? dz[s] : 0.0);
        nd[s] = Dual(nman[s], dn ? dn[s] : 0.0);
    }
    Dual r = loss_forward<Dual>(c, &L, e.data(), a.data(), b.data(), zd.data(), nd.data(), t0,
                                step0);
    *J = r.v;
    if (dJ) *dJ = r.d;
    return 0;
}

/* The gradient of the same loss with respect to the Manning field (gn) and
 * the bed (gz), both nx*ny, by reverse mode: the states U^0 .. U^{nsteps-1}
 * are kept from a forward pass, then each step is taped and replayed
 * backwards from the last to the first.  *J receives the loss.  Returns 0,
 * or -1 on bad arguments. */
int orc_loss_gradient(const orc_cfg* c, const double* eta0, const double* qx0, const double* qy0,
                      const double* z, const double* nman, double t0, int64_t step0,
                      int64_t nsteps, const double* dts, int32_t ngauge, const int64_t* gauges,
                      int32_t obs_every, const double* hobs, double* J, double* gn, double* gz) {
    LossSpec L = {nsteps, dts, ngauge, gauges, obs_every, hobs};
    if (check_cfg(c) || check_loss(c, &L) || !eta0 || !qx0 || !qy0 || !z || !nman || !J || !gn ||
        !gz)
        return -1;
    const size_t N = (size_t)c->nx * (size_t)c->ny;
    Grid G = {c->nx, c->ny, c->nx + 2};
    /* forward: states before every step, the loss, the times */
    std::vector<double> states((size_t)nsteps * 3 * N);
    std::vector<double> times((size_t)nsteps);
    {
        Work<double> w;
        w.init(&G, nullptr);
        static_fields(c, &G, z, nman, w.zp, w.mp);
        std::vector<double> e(eta0, eta0 + N), a(qx0, qx0 + N), b(qy0, qy0 + N);
        double Jv = 0.0, t = t0;
        for (int64_t k = 0; k < nsteps; ++k) {
            double* sk = states.data() + (size_t)k * 3 * N;
            memcpy(sk, e.data(), N * sizeof(double));
            memcpy(sk + N, a.data(), N * sizeof(double));
            memcpy(sk + 2 * N, b.data(), N * sizeof(double));
            times[(size_t)k] = t;
            StepOut so;
            step_body(c, &G, &w, e.data(), a.data(), b.data(), t, step0 + k, dts[k], &so);
            t = t + dts[k];
            if ((k + 1) % obs_every == 0) Jv = Jv + misfit(&L, k + 1, e.data(), z);
        }
        *J = Jv;
    }
    for (size_t s = 0; s < N; ++s) gn[s] = gz[s] = 0.0;
    /* adjoint of U^{k+1}: starts at zero after the last step */
    std::vector<double> lam(3 * N, 0.0);
    std::vector<double> adj;
    for (int64_t k = nsteps - 1; k >= 0; --k) {
        g_tape.clear();
        const double* sk = states.data() + (size_t)k * 3 * N;
        std::vector<Rev> e(N), a(N), b(N), zr(N), nr(N);
        for (size_t s = 0; s < N; ++s) e[s] = rleaf(sk[s]);
        for (size_t s = 0; s < N; ++s) a[s] = rleaf(sk[N + s]);
        for (size_t s = 0; s < N; ++s) b[s] = rleaf(sk[2 * N + s]);
        for (size_t s = 0; s < N; ++s) zr[s] = rleaf(z[s]);
        for (size_t s = 0; s < N; ++s) nr[s] = rleaf(nman[s]);
        std::vector<int32_t> in_e(N), in_a(N), in_b(N), in_z(N), in_n(N);
        for (size_t s = 0; s < N; ++s) {
            in_e[s] = e[s].id; in_a[s] = a[s].id; in_b[s] = b[s].id;
            in_z[s] = zr[s].id; in_n[s] = nr[s].id;
        }
        Work<Rev> w;
        w.init(&G, nullptr);
        static_fields(c, &G, zr.data(), nr.data(), w.zp, w.mp);
        StepOut so;
        step_body(c, &G, &w, e.data(), a.data(), b.data(), times[(size_t)k], step0 + k, dts[k], &so);
        adj.assign(g_tape.size(), 0.0);
        /* seed: the adjoint of U^{k+1}, plus the observation after step k+1 */
        for (size_t s = 0; s < N; ++s) {
            if (e[s].id >= 0) adj[(size_t)e[s].id] += lam[s];
            if (a[s].id >= 0) adj[(size_t)a[s].id] += lam[N + s];
            if (b[s].id >= 0) adj[(size_t)b[s].id] += lam[2 * N + s];
        }
        if ((k + 1) % obs_every == 0) {
            const double* ho = hobs + (size_t)((k + 1) / obs_every - 1) * (size_t)ngauge;
            for (int32_t g = 0; g < ngauge; ++g) {
                size_t s = (size_t)gauges[g];
                double d = (e[s].v - z[s]) - ho[g];
                double two_d = d + d;
                if (e[s].id >= 0) adj[(size_t)e[s].id] += two_d;
                gz[s] += 0.0 - two_d;
            }
        }
        for (size_t m = g_tape.size(); m-- > 0;) {
            double am = adj[m];
            if (am == 0.0) continue;
            const Node& nd = g_tape[m];
            if (nd.a >= 0) adj[(size_t)nd.a] += nd.da * am;
            if (nd.b >= 0) adj[(size_t)nd.b] += nd.db * am;
        }
        for (size_t s = 0; s < N; ++s) {
            lam[s] = adj[(size_t)in_e[s]];
            lam[N + s] = adj[(size_t)in_a[s]];
            lam[2 * N + s] = adj[(size_t)in_b[s]];
            gz[s] += adj[(size_t)in_z[s]];
            gn[s] += adj[(size_t)in_n[s]];
        }
    }
    g_tape.clear();
    g_tape.shrink_to_fit();
    return 0;
}

}  /* extern "C" */
