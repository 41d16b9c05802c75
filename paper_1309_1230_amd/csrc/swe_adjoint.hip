// swe_adjoint.hip -- discrete adjoint of one time step (FP64).
//
// Reverse mode through S15 .. S1 of one step.  The step's forward data are
// U^n, U* (after S7) and U^d (after S13, before friction), pitched like the
// state, which the tracing fused step writes; everything else the reverse
// sweep needs (the ghost rings of S1 and S8, the primitives of S2 and S9, the
// switches of S3, the friction of S14 and the dry fix of S15) is recomputed
// here from them with the forward step's own expressions, so each value is
// bit for bit the one the forward step used.  The adjoint lam^{n+1} of
// U^{n+1} (plus the gauge misfit terms of the loss when step n+1 is
// observed) becomes lam^n, the adjoint of U^n, and the step's contributions
// to dJ/dn and dJ/dz are added to the accumulators.  dt^n is held fixed (not
// differentiated).
//
// Every kernel gathers: a thread owns one cell (or one padded cell) and
// recomputes what it needs from the faces and neighbours that reach it, so
// there are no atomics and the result does not depend on thread order.
// Derivative conventions (the same as the CPU reference's): branches are
// taken as in the forward step; max/min pass the derivative to the argument
// they return (the second on a tie); |x| has derivative sign(x) (0 at 0);
// sqrt has derivative 0 at 0; the cube root's first guess is a constant and
// its two Halley steps are differentiated as executed.  A derivative that
// divides by a forward quantity whose reciprocal the step already forms
// (1/h, 1/phi) multiplies by that reciprocal instead: the same derivative,
// rounded differently, one FP64 division less.
#include <algorithm>

#include "swe_common.hpp"
#include "swe_internal.hpp"

namespace swe {

namespace {

constexpr int kBX = 128, kBY = 2;   // 2D blocks of the adjoint sweeps (measured best of 32..256 x 1..16)

// The adjoint's own arrays are padded with a one-cell ring: element (i, j),
// i in [-1, nx], j in [-1, ny], at (j+1)*(nx+2) + (i+1).
struct Pad {
    int nx, ny, P2;
    long long N;
    __device__ __forceinline__ long long at(int i, int j) const {
        return (long long)(j + 1) * P2 + (i + 1);
    }
    __device__ __forceinline__ bool interior(int i, int j) const {
        return i >= 0 && i < nx && j >= 0 && j < ny;
    }
};

__device__ __forceinline__ Pad pad_of(const Params& P) {
    Pad d;
    d.nx = P.nx;
    d.ny = P.ny;
    d.P2 = P.nx + 2;
    d.N = (long long)(P.nx + 2) * (long long)(P.ny + 2);
    return d;
}

__device__ __forceinline__ double* wk(const AdjointArgs& a, const Pad& d, int k) {
    return a.work + (long long)k * d.N;
}

// Adjoint work arrays (padded): corrector inner adjoint a-bar (3), U^d-bar
// (= D-bar, 3), U*-bar (3), U^n-bar (3), nu-bar (2), zp-bar, lambda (3),
// dJ/dn and dJ/dz accumulators.
enum { W_AB = 0, W_AD = 3, W_AUS = 6, W_AUN = 9, W_ANX = 12, W_ANY = 13, W_AZP = 14,
       W_LAM = 15, W_GN = 18, W_GZ = 19 };

__device__ __forceinline__ long long pitched(const Params& P, int i, int j) {
    return (long long)j * P.pitch + i;
}

// eta of U^n or U* at padded cell (i, j): a ghost copies the adjacent cell.
__device__ __forceinline__ double eta_at(const Params& P, const double* E, int i, int j) {
    return E[pitched(P, min(max(i, 0), P.nx - 1), min(max(j, 0), P.ny - 1))];
}

// A state (U^n with q_in(t^n), or U* with q_in(t^n + dt)) at padded cell
// (i, j), not a corner: the interior value or the ghost ring rule (S1, S8),
// with its primitives (S2, S9).
struct Cell { double e, qx, qy, h, r, u, v; };

// The ghost rule (S1, S8) and the primitives (S2, S9) of padded cell (i, j)
// from the state at its clamped interior position (e, qx, qy) and its bed.
// kW, kE: kinds of the west and east boundary faces of row j.  (Every edge
// index here is a constant: a per-thread index into the parameter block would
// make the compiler read it through vector memory.)
// XEDGE = false: the caller knows that i is an interior column; YEDGE =
// false: that j is an interior row.
template <bool XEDGE = true, bool YEDGE = true>
__device__ __forceinline__ Cell make_cell(const Params& P, double e, double qx, double qy,
                                          double qin, int i, int j, double zpv, int kW, int kE) {
    Cell c;
    c.e = e;
    c.qx = qx;
    c.qy = qy;
    if (XEDGE && (i < 0 || i >= P.nx))
        ghost(i < 0 ? kW : kE, true, i < 0 ? qin : -qin, c.e, c.qx, c.qy, c.e, c.qx, c.qy);
    else if (YEDGE && (j < 0 || j >= P.ny))
        ghost(j < 0 ? face_kind(P, EDGE_S, i) : face_kind(P, EDGE_N, i), false,
              j < 0 ? qin : -qin, c.e, c.qx, c.qy, c.e, c.qx, c.qy);
    c.h = c.e - zpv;
    c.r = recip_prim(c.h, P.h_dry, P.rcap);
    c.u = c.qx * c.r;
    c.v = c.qy * c.r;
    return c;
}

// A cell from carried values (the same products as make_cell).
__device__ __forceinline__ Cell carried_cell(double e, double qx, double qy, double h, double r) {
    Cell c;
    c.e = e;
    c.qx = qx;
    c.qy = qy;
    c.h = h;
    c.r = r;
    c.u = qx * r;
    c.v = qy * r;
    return c;
}

__device__ __forceinline__ Cell cell_at(const AdjointArgs& a, const Pad& d,
                                        const double* const* U, double qin, int i, int j) {
    const Params& P = a.P;
    const long long s = pitched(P, min(max(i, 0), P.nx - 1), min(max(j, 0), P.ny - 1));
    return make_cell(P, U[0][s], U[1][s], U[2][s], qin, i, j, a.zp[d.at(i, j)],
                     face_kind(P, EDGE_W, j), face_kind(P, EDGE_E, j));
}

// S3: switch of U^n at interior cell (i, j) along x (xdir) or y.
__device__ __forceinline__ double nu_at(const AdjointArgs& a, int i, int j, bool xdir, double eC,
                                        double rC) {
    const double* E = a.un[0];
    const double eM = xdir ? eta_at(a.P, E, i - 1, j) : eta_at(a.P, E, i, j - 1);
    const double eP = xdir ? eta_at(a.P, E, i + 1, j) : eta_at(a.P, E, i, j + 1);
    return curv_switch(eM, eC, eP, rC);
}

// The friction cube root y = cbrt3(x) with its Halley steps kept: the same
// operations as tcbrt, so y[2] is tcbrt(x) bit for bit.
struct CbrtTape { double y[3], q[2], den[2]; };

__device__ __forceinline__ CbrtTape cbrt3_tape(double x) {
    CbrtTape c;
    const unsigned w = (unsigned)__double2hiint(x);
    c.y[0] = __hiloint2double((int)(w / 3u + 0x2A9F7893u), 0);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double tt = (c.y[k] * c.y[k]) * c.y[k];
        const double num = tt + (x + x);
        c.den[k] = (tt + tt) + x;
        c.q[k] = num / c.den[k];
        c.y[k + 1] = c.y[k] * c.q[k];
    }
    return c;
}

// Reverse of the cube root: x-bar given y-bar and the tape of x.
__device__ __forceinline__ double cbrt3_adjoint(const CbrtTape& c, double ybar) {
    double xbar = 0.0;
#pragma unroll
    for (int k = 1; k >= 0; --k) {
        const double qbar = ybar * c.y[k];
        ybar = ybar * c.q[k];
        const double numbar = qbar / c.den[k];
        const double denbar = -(numbar * c.q[k]);   // -(qbar q)/den
        // den = (t + t) + x, num = t + (x + x)
        xbar += denbar;
        double tbar = denbar + denbar + numbar;
        xbar += numbar + numbar;
        // t = (y*y)*y
        const double yy = c.y[k] * c.y[k];
        const double yybar = tbar * c.y[k];
        ybar += tbar * yy;
        ybar += yybar * c.y[k] + yybar * c.y[k];
    }
    return xbar;
}

// Fold the adjoint of a ghost cell into its interior neighbour C (the ghost
// ring copies eta, and copies, mirrors or replaces the discharges).
__device__ __forceinline__ void fold_ghost(double* A, const Pad& d, long long C, long long g,
                                           int kind, bool normal_is_x) {
    A[C] += A[g];
    if (kind == BC_OPEN) {
        A[d.N + C] += A[d.N + g];
        A[2 * d.N + C] += A[2 * d.N + g];
    } else if (kind == BC_WALL) {
        if (normal_is_x) {
            A[d.N + C] -= A[d.N + g];
            A[2 * d.N + C] += A[2 * d.N + g];
        } else {
            A[d.N + C] += A[d.N + g];
            A[2 * d.N + C] -= A[2 * d.N + g];
        }
    }
    // an inflow ghost's discharges are imposed: no adjoint flows back
}

__device__ __forceinline__ void fold_ring(const AdjointArgs& a, double* A, const Pad& d, int i,
                                          int j) {
    const long long C = d.at(i, j);
    if (i == 0) fold_ghost(A, d, C, d.at(-1, j), face_kind(a.P, EDGE_W, j), true);
    if (i == d.nx - 1) fold_ghost(A, d, C, d.at(d.nx, j), face_kind(a.P, EDGE_E, j), true);
    if (j == 0) fold_ghost(A, d, C, d.at(i, -1), face_kind(a.P, EDGE_S, i), false);
    if (j == d.ny - 1) fold_ghost(A, d, C, d.at(i, d.ny), face_kind(a.P, EDGE_N, i), false);
}

// The same fold into a copy: a[0..2] start as A at cell (i, j) and receive
// its ghost cells' contributions in the order of fold_ring.
__device__ __forceinline__ void fold_ghost_into(const double* A, const Pad& d, long long g,
                                                int kind, bool normal_is_x, double* a) {
    a[0] += A[g];
    if (kind == BC_OPEN) {
        a[1] += A[d.N + g];
        a[2] += A[2 * d.N + g];
    } else if (kind == BC_WALL) {
        if (normal_is_x) {
            a[1] -= A[d.N + g];
            a[2] += A[2 * d.N + g];
        } else {
            a[1] += A[d.N + g];
            a[2] -= A[2 * d.N + g];
        }
    }
}

// fold_ghost_into with the ghost's adjoint given as values.
__device__ __forceinline__ void fold_value(double g0, double g1, double g2, int kind,
                                           bool normal_is_x, double* a) {
    a[0] += g0;
    if (kind == BC_OPEN) {
        a[1] += g1;
        a[2] += g2;
    } else if (kind == BC_WALL) {
        if (normal_is_x) {
            a[1] -= g1;
            a[2] += g2;
        } else {
            a[1] += g1;
            a[2] -= g2;
        }
    }
}

__device__ __forceinline__ void fold_ring_into(const AdjointArgs& a, const double* A, const Pad& d,
                                               int i, int j, double* v) {
    if (i == 0) fold_ghost_into(A, d, d.at(-1, j), face_kind(a.P, EDGE_W, j), true, v);
    if (i == d.nx - 1) fold_ghost_into(A, d, d.at(d.nx, j), face_kind(a.P, EDGE_E, j), true, v);
    if (j == 0) fold_ghost_into(A, d, d.at(i, -1), face_kind(a.P, EDGE_S, i), false, v);
    if (j == d.ny - 1) fold_ghost_into(A, d, d.at(i, d.ny), face_kind(a.P, EDGE_N, i), false, v);
}

// S15 and S14 reversed at one interior cell: U^d = (ed, qx, qy), the bed zp,
// m = g n^2 (mp) and n, and the adjoint (le, lx, ly) of U^{n+1}.  Returns the
// adjoint of U^d, the bed's share and, for a wet cell, the dJ/dn term.
struct FaOut { double e, x, y, azp, gn; bool wet; };

__device__ __forceinline__ FaOut fa_point(double ed, double qx, double qy, double zp, double mp,
                                          double n, double le, double lx, double ly, double dt,
                                          double hdry, double g) {
    const double ef = ed;
    const bool clip = ef - zp < 0.0;
    const double en = clip ? zp : ef;
    // S15 dry fix (S14 leaves eta as U^d's)
    const bool dry = !(en - zp > hdry);
    double azp = clip ? le : 0.0;
    const double efb = clip ? 0.0 : le;
    const double qxfb = dry ? 0.0 : lx, qyfb = dry ? 0.0 : ly;
    // S14 friction
    const double h = ed - zp;
    double edb = efb, qxdb = qxfb, qydb = qyfb;
    FaOut o;
    o.wet = h > hdry;
    o.gn = 0.0;
    if (o.wet) {
        const double r = 1.0 / h;
        const double x2 = qx * qx + qy * qy;
        const double w = sqrt(x2);
        const double s = w * r;
        const CbrtTape ct = cbrt3_tape(r);
        const double c3 = ct.y[2];   // tcbrt(r)
        const double k = r * c3;
        const double dtm = dt * mp;
        const double A = dtm * s;
        const double B = A * k;
        const double phi = 1.0 + B;
        const double psi = 1.0 / phi;
        const double psib = qxfb * qx + qyfb * qy;
        qxdb = qxfb * psi;
        qydb = qyfb * psi;
        const double phib = -(psib * psi) * psi;   // psi = 1/phi
        const double Ab = phib * k, kb = phib * A;
        const double dtmb = Ab * s, sb = Ab * dtm;
        const double mb = dtmb * dt;
        double rb = kb * c3 + sb * w;
        rb += cbrt3_adjoint(ct, kb * r);
        const double wb = sb * r;
        if (x2 > 0.0) {
            const double x2b = wb * (0.5 / w);
            qxdb += x2b * qx + x2b * qx;
            qydb += x2b * qy + x2b * qy;
        }
        const double hb = -(rb * r) * r;   // r = 1/h
        edb += hb;
        azp -= hb;
        // m = g n^2 at this cell
        const double mg = mb * g;
        o.gn = mg * n + mg * n;
    }
    o.e = edb;
    o.x = qxdb;
    o.y = qydb;
    o.azp = azp;
    return o;
}

// S1 of the step reversed before this one (its ghost ring of U^n folded into
// lambda, the bed's padded adjoint into dJ/dz), the loss terms of this step
// when it is observed (lambda_eta += 2 d, dJ/dz -= 2 d at each gauge,
// d = (eta^{n+1} - z) - h_obs, eta^{n+1} being the dry fix of eta^d since
// friction leaves eta unchanged), then S15, S14, S13 and the U^n share of
// S12, per interior cell.  gmap: gauge index of each cell (j*nx + i), or -1;
// hobs: this step's observations, or NULL.
__global__ void k_adj_fa(AdjointArgs a, const int* gmap, const double* hobs) {
    const Pad d = pad_of(a.P);
    const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y;
    if (i >= d.nx || j >= d.ny) return;
    const long long C = d.at(i, j), o = pitched(a.P, i, j);
    const double hdry = a.P.h_dry, zp = a.zp[C];
    // previous step's S1: lambda = AUN with the ghost ring folded in
    const double* AUN = wk(a, d, W_AUN);
    double lam[3] = {AUN[C], AUN[d.N + C], AUN[2 * d.N + C]};
    fold_ring_into(a, AUN, d, i, j, lam);
    double* AZP = wk(a, d, W_AZP);
    double gzs = AZP[C];
    const long long gs[4] = {i == 0 ? d.at(-1, j) : -1, i == d.nx - 1 ? d.at(d.nx, j) : -1,
                             j == 0 ? d.at(i, -1) : -1, j == d.ny - 1 ? d.at(i, d.ny) : -1};
    for (int k = 0; k < 4; ++k)
        if (gs[k] >= 0) {
            gzs += AZP[gs[k]];
            AZP[gs[k]] = 0.0;
        }
    double gz = wk(a, d, W_GZ)[C] + gzs;
    // this step's loss terms
    const double ed = a.ud[0][o], qx = a.ud[1][o], qy = a.ud[2][o];
    const double ef = ed;
    const bool clip = ef - zp < 0.0;
    const double en = clip ? zp : ef;
    if (hobs) {
        const int g = gmap[(long long)j * d.nx + i];
        if (g >= 0) {
            const double dd = (en - zp) - hobs[g];
            lam[0] += dd + dd;
            gz += 0.0 - (dd + dd);
        }
    }
    wk(a, d, W_GZ)[C] = gz;
    const FaOut f = fa_point(ed, qx, qy, zp, a.mp[C], a.nman[o], lam[0], lam[1], lam[2], a.dt,
                             hdry, a.P.g);
    if (f.wet) wk(a, d, W_GN)[C] += f.gn;
    const double edb = f.e, qxdb = f.x, qydb = f.y, azp = f.azp;
    // S13: U^d = U^c + D; S12: U^c = 0.5*(U^n + a)
    double* AD = wk(a, d, W_AD);
    double* AB = wk(a, d, W_AB);
    AD[C] = edb; AD[d.N + C] = qxdb; AD[2 * d.N + C] = qydb;
    AB[C] = 0.5 * edb; AB[d.N + C] = 0.5 * qxdb; AB[2 * d.N + C] = 0.5 * qydb;
    AZP[C] = azp;
}

// Adjoint of the flux-divergence update out = base - L_dir (S7 / inner S12)
// seen from one face: the face's (Fm, Fx, Fy, P) adjoints, given the
// adjoint A of `out` on the two cells of the face (zero off the interior).
struct FaceBar { double m, x, y, p; };

// The adjoint 3-vector A (padded, three arrays d.N apart) at cell (i, j):
// zero off the interior; with `fold`, an edge cell also receives its ghost
// cells' contributions (the S8 fold of U*-bar, applied where it is read).
__device__ __forceinline__ void vec_at(const AdjointArgs& a, const double* A, const Pad& d, int i,
                                       int j, bool fold, double* v) {
    if (!d.interior(i, j)) {
        v[0] = v[1] = v[2] = 0.0;
        return;
    }
    const long long C = d.at(i, j);
    v[0] = A[C];
    v[1] = A[d.N + C];
    v[2] = A[2 * d.N + C];
    if (fold) fold_ring_into(a, A, d, i, j, v);
}

__device__ __forceinline__ FaceBar face_bar_v(double aL0, double aL1, double aL2, double aR0,
                                              double aR1, double aR2, double coef, int dir,
                                              bool xface) {
    FaceBar f;
    f.m = coef * aR0 - coef * aL0;
    f.x = coef * aR1 - coef * aL1;
    f.y = coef * aR2 - coef * aL2;
    // the pressure sits in the x-momentum update (x faces) or the
    // y-momentum update (y faces) of the cell on the dir side
    const double aPL = xface ? aL1 : aL2, aPR = xface ? aR1 : aR2;
    f.p = dir > 0 ? -(coef * aPL) : -(coef * aPR);
    return f;
}

__device__ __forceinline__ FaceBar face_bar(const AdjointArgs& a, const double* A, bool fold,
                                            const Pad& d, int iL, int jL, int iR, int jR,
                                            double coef, int dir, bool xface) {
    double vL[3], vR[3];
    vec_at(a, A, d, iL, jL, fold, vL);
    vec_at(a, A, d, iR, jR, fold, vR);
    return face_bar_v(vL[0], vL[1], vL[2], vR[0], vR[1], vR[2], coef, dir, xface);
}

// Contributions of one face's flux adjoint to the adjoints of the cell
// `me` (L or R of the face): eta-bar, qx-bar, qy-bar, u-bar, v-bar, h-bar.
struct CellBar { double e, qx, qy, u, v, h; };

__device__ __forceinline__ void face_flux_adjoint(const FaceBar& fb, int kind, int dir,
                                                  bool ghost_is_R, bool me_is_L, bool xface,
                                                  const Cell& L, const Cell& R, double zL,
                                                  double zR, double hdry, double hg,
                                                  CellBar& cb) {
    if (kind == BC_WALL) return;
    bool dnR, pass;
    if (kind == BC_INFLOW) {
        dnR = ghost_is_R;
        pass = true;
    } else {
        dnR = dir > 0;
        pass = (dnR ? R.h : L.h) > hdry;
    }
    if (dnR != me_is_L) {   // the donor cell is `me`
        const Cell& D = dnR ? R : L;
        const double fm = pass ? (xface ? D.qx : D.qy) : 0.0;
        const double fmb = (fb.m + fb.x * D.u) + fb.y * D.v;
        cb.u += fb.x * fm;
        cb.v += fb.y * fm;
        if (pass) {
            if (xface)
                cb.qx += fmb;
            else
                cb.qy += fmb;
        }
    }
    if (kind >= 0) return;   // boundary faces carry no pressure
    const bool wetL = L.h > hdry, wetR = R.h > hdry;
    const bool bank = (!wetL && zL > R.e) || (!wetR && zR > L.e);
    if (bank) return;
    const double A = hg * (hpos(L.h) + hpos(R.h));
    const double del = R.e - L.e;
    const double Ab = fb.p * del, delb = fb.p * A;
    const double Sb = Ab * hg;
    if (me_is_L) {
        cb.e -= delb;
        cb.h += L.h > 0.0 ? Sb : 0.0;
    } else {
        cb.e += delb;
        cb.h += R.h > 0.0 ? Sb : 0.0;
    }
}

__device__ __forceinline__ int xface_kind(const Params& P, int fi, int j) {
    return fi == -1 ? face_kind(P, EDGE_W, j) : (fi == P.nx - 1 ? face_kind(P, EDGE_E, j) : -1);
}
__device__ __forceinline__ int yface_kind(const Params& P, int i, int fj) {
    return fj == -1 ? face_kind(P, EDGE_S, i) : (fj == P.ny - 1 ? face_kind(P, EDGE_N, i) : -1);
}

// Sum over the (up to) four faces of padded cell (i, j) of the flux
// adjoints, for the fluxes of state U (with inflow qin) whose cell `me` is,
// donor direction dir, whose update's adjoint is A (three arrays).
__device__ CellBar gather_faces(const AdjointArgs& a, const Pad& d, int i, int j, const Cell& me,
                                const double* const* U, double qin, int dir, const double* A,
                                bool fold, double rx, double ry) {
    CellBar cb = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const double hdry = a.P.h_dry, hg = 0.5 * a.P.g;
    const double zme = a.zp[d.at(i, j)];
    if (j >= 0 && j < d.ny) {    // x faces: rows 0 .. ny-1, slots -1 .. nx-1
        for (int side = 0; side < 2; ++side) {
            const int fi = side == 0 ? i : i - 1;    // me is L of face fi when side == 0
            if (fi < -1 || fi > d.nx - 1) continue;
            const int kind = xface_kind(a.P, fi, j);
            const FaceBar fb = face_bar(a, A, fold, d, fi, j, fi + 1, j, rx, dir, true);
            const int io = side == 0 ? i + 1 : i - 1;
            const Cell other = cell_at(a, d, U, qin, io, j);
            const double zo = a.zp[d.at(io, j)];
            if (side == 0)
                face_flux_adjoint(fb, kind, dir, fi == d.nx - 1, true, true, me, other, zme, zo,
                                  hdry, hg, cb);
            else
                face_flux_adjoint(fb, kind, dir, fi == d.nx - 1, false, true, other, me, zo, zme,
                                  hdry, hg, cb);
        }
    }
    if (i >= 0 && i < d.nx) {    // y faces: columns 0 .. nx-1, slots -1 .. ny-1
        for (int side = 0; side < 2; ++side) {
            const int fj = side == 0 ? j : j - 1;
            if (fj < -1 || fj > d.ny - 1) continue;
            const int kind = yface_kind(a.P, i, fj);
            const FaceBar fb = face_bar(a, A, fold, d, i, fj, i, fj + 1, ry, dir, false);
            const int jo = side == 0 ? j + 1 : j - 1;
            const Cell other = cell_at(a, d, U, qin, i, jo);
            const double zo = a.zp[d.at(i, jo)];
            if (side == 0)
                face_flux_adjoint(fb, kind, dir, fj == d.ny - 1, true, false, me, other, zme, zo,
                                  hdry, hg, cb);
            else
                face_flux_adjoint(fb, kind, dir, fj == d.ny - 1, false, false, other, me, zo, zme,
                                  hdry, hg, cb);
        }
    }
    return cb;
}

__device__ __forceinline__ bool padded_cell(const Pad& d, int pi, int pj, int& i, int& j) {
    if (pi >= d.nx + 2 || pj >= d.ny + 2) return false;
    i = pi - 1;
    j = pj - 1;
    const bool gx = i < 0 || i >= d.nx, gy = j < 0 || j >= d.ny;
    return !(gx && gy);   // corners are never read
}

// S12 (flux part), S11, S10, S9: the adjoint of U* on every padded cell.
__global__ void k_adj_c(AdjointArgs a) {
    const Pad d = pad_of(a.P);
    int i, j;
    if (!padded_cell(d, blockIdx.x * kBX + threadIdx.x, blockIdx.y * kBY + threadIdx.y, i, j))
        return;
    const long long C = d.at(i, j);
    const double qin1 = a.qin1;
    const double* AB = wk(a, d, W_AB);
    const Cell me = cell_at(a, d, a.us, qin1, i, j);
    const CellBar cb = gather_faces(a, d, i, j, me, a.us, qin1, -a.sigma, AB, false, a.rx, a.ry);
    const bool in = d.interior(i, j);
    double eb = cb.e + (in ? AB[C] : 0.0);
    double qxb = cb.qx + (in ? AB[d.N + C] : 0.0);
    double qyb = cb.qy + (in ? AB[2 * d.N + C] : 0.0);
    // S9: h = eta - zp, r = wet ? 1/h : 0, u = qx r, v = qy r
    const double h = me.h, r = me.r;
    qxb += cb.u * r;
    qyb += cb.v * r;
    const double rb = cb.u * me.qx + cb.v * me.qy;
    // r = min(1/h, rcap): its depth derivative vanishes where the cap was taken
    const double hb = cb.h + (h > a.P.h_dry && r < a.P.rcap ? -(rb * r) * r : 0.0);
    eb += hb;
    double* AUS = wk(a, d, W_AUS);
    AUS[C] = eb;
    AUS[d.N + C] = qxb;
    AUS[2 * d.N + C] = qyb;
    wk(a, d, W_AZP)[C] -= hb;
}

// Face coefficient of S4 between cells L and R and the derivative of it
// with respect to nu: which of the two it follows (0: L, 1: R, -1: none).
__device__ __forceinline__ double eps_and_arg(double hL, double hR, double nuL, double nuR,
                                              double hdry, double kap, double emax, int& arg) {
    arg = -1;
    if (!(hL > hdry && hR > hdry)) return 0.0;
    const bool takeL = nuL > nuR;
    const double t = kap * (takeL ? nuL : nuR);
    if (t < emax) {
        arg = takeL ? 0 : 1;
        return t;
    }
    return emax;
}

// S4: dissipation adjoint on interior cells: nu-bar, and the U^n adjoint's
// first terms (the corrector's U^n share and the differences of S4).
__global__ void k_adj_e1(AdjointArgs a) {
    const Pad d = pad_of(a.P);
    const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y;
    if (i >= d.nx || j >= d.ny) return;
    const long long C = d.at(i, j);
    const double hdry = a.P.h_dry, kap = a.P.kappa, emax = a.P.eps_max;
    const double qin0 = a.qin0;
    const double* AD = wk(a, d, W_AD);
    const double* AB = wk(a, d, W_AB);
    const Cell me = cell_at(a, d, a.un, qin0, i, j);
    const double nuMe[2] = {nu_at(a, i, j, true, me.e, me.r), nu_at(a, i, j, false, me.e, me.r)};
    double un[3] = {AB[C], AB[d.N + C], AB[2 * d.N + C]};
    double nub[2] = {0.0, 0.0};
    for (int f = 0; f < 4; ++f) {
        const bool xf = f < 2;
        const int ni = xf ? (f == 0 ? i + 1 : i - 1) : i;
        const int nj = xf ? j : (f == 2 ? j + 1 : j - 1);
        if (ni < 0 || ni >= d.nx || nj < 0 || nj >= d.ny) continue;   // boundary face: eps = 0
        const long long nb = d.at(ni, nj);
        const Cell on = cell_at(a, d, a.un, qin0, ni, nj);
        const double nuOn = nu_at(a, ni, nj, xf, on.e, on.r);
        const bool meL = f == 0 || f == 2;
        const long long L = meL ? C : nb, R = meL ? nb : C;
        const Cell& cL = meL ? me : on;
        const Cell& cR = meL ? on : me;
        const double nuL = meL ? nuMe[xf ? 0 : 1] : nuOn, nuR = meL ? nuOn : nuMe[xf ? 0 : 1];
        int arg;
        const double eps = eps_and_arg(cL.h, cR.h, nuL, nuR, hdry, kap, emax, arg);
        const double qL[3] = {cL.e, cL.qx, cL.qy}, qR[3] = {cR.e, cR.qx, cR.qy};
        double epsb = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double* ad = AD + (long long)k * d.N;
            epsb += (ad[L] - ad[R]) * (qR[k] - qL[k]);
            un[k] += eps * (ad[nb] - ad[C]);
        }
        if (arg == (meL ? 0 : 1)) nub[xf ? 0 : 1] += epsb * kap;
    }
    double* AUN = wk(a, d, W_AUN);
    AUN[C] = un[0];
    AUN[d.N + C] = un[1];
    AUN[2 * d.N + C] = un[2];
    wk(a, d, W_ANX)[C] = nub[0];
    wk(a, d, W_ANY)[C] = nub[1];
}

// d-bar of the curvature switch at interior cell X (x or y direction), and
// its |d| for the r-bar term.
__device__ __forceinline__ double switch_dbar(double eXm, double eX, double eXp, double rX,
                                              double nubX, double& absd_t) {
    const double dd = (eXp - eX) - (eX - eXm);
    const double t = 0.25 * nubX;
    absd_t = t * __builtin_fabs(dd);
    const double absb = t * rX;
    return dd > 0.0 ? absb : (dd < 0.0 ? -absb : 0.0);
}

// S7, S6, S5, S3, S2: the rest of the U^n adjoint on every padded cell.
__global__ void k_adj_e2(AdjointArgs a) {
    const Pad d = pad_of(a.P);
    int i, j;
    if (!padded_cell(d, blockIdx.x * kBX + threadIdx.x, blockIdx.y * kBY + threadIdx.y, i, j))
        return;
    const long long C = d.at(i, j);
    const bool in = d.interior(i, j);
    const double qin0 = a.qin0;
    const double* AUS = wk(a, d, W_AUS);
    const Cell me = cell_at(a, d, a.un, qin0, i, j);
    const CellBar cb = gather_faces(a, d, i, j, me, a.un, qin0, a.sigma, AUS, true, a.rx, a.ry);
    double* AUN = wk(a, d, W_AUN);
    double eb = cb.e, qxb = cb.qx, qyb = cb.qy;
    if (in) {
        double us[3];
        vec_at(a, AUS, d, i, j, true, us);
        eb += AUN[C] + us[0];
        qxb += AUN[d.N + C] + us[1];
        qyb += AUN[2 * d.N + C] + us[2];
    }
    // S3: nu = 0.25*(|d| r) at interior cells X; d reaches X-1, X, X+1
    const double* E = a.un[0];
    double rb = cb.u * me.qx + cb.v * me.qy;
    for (int dirn = 0; dirn < 2; ++dirn) {
        const double* NUB = wk(a, d, dirn == 0 ? W_ANX : W_ANY);
        for (int o = -1; o <= 1; ++o) {
            const int xi = dirn == 0 ? i + o : i, xj = dirn == 0 ? j : j + o;
            if (!d.interior(xi, xj)) continue;
            const double eX = E[pitched(a.P, xi, xj)];
            const double eXm = dirn == 0 ? eta_at(a.P, E, xi - 1, xj) : eta_at(a.P, E, xi, xj - 1);
            const double eXp = dirn == 0 ? eta_at(a.P, E, xi + 1, xj) : eta_at(a.P, E, xi, xj + 1);
            const double rX = recip_prim(eX - a.zp[d.at(xi, xj)], a.P.h_dry, a.P.rcap);
            double absd_t;
            const double db = switch_dbar(eXm, eX, eXp, rX, NUB[d.at(xi, xj)], absd_t);
            if (o == 0) {
                eb += -db - db;
                rb += absd_t;
            } else {
                eb += db;
            }
        }
    }
    // S2: h = eta - zp, r = wet ? 1/h : 0, u = qx r, v = qy r
    const double h = me.h, r = me.r;
    qxb += cb.u * r;
    qyb += cb.v * r;
    // r = min(1/h, rcap): its depth derivative vanishes where the cap was taken
    const double hb = cb.h + (h > a.P.h_dry && r < a.P.rcap ? -(rb * r) * r : 0.0);
    eb += hb;
    AUN[C] = eb;
    AUN[d.N + C] = qxb;
    AUN[2 * d.N + C] = qyb;
    wk(a, d, W_AZP)[C] -= hb;
}

// S1: fold the ghost ring of U^n into lambda^n; the bed's padded adjoint
// (edge ghosts copy the adjacent cell's z) into dJ/dz.
__global__ void k_adj_f(AdjointArgs a) {
    const Pad d = pad_of(a.P);
    const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y;
    if (i >= d.nx || j >= d.ny) return;
    const long long C = d.at(i, j);
    double* AUN = wk(a, d, a.lam_slot);
    fold_ring(a, AUN, d, i, j);
    double* LAM = wk(a, d, W_LAM);
    LAM[C] = AUN[C];
    LAM[d.N + C] = AUN[d.N + C];
    LAM[2 * d.N + C] = AUN[2 * d.N + C];
    double* AZP = wk(a, d, a.azp_slot);
    double gz = AZP[C];
    AZP[C] = 0.0;
    const long long gs[4] = {i == 0 ? d.at(-1, j) : -1, i == d.nx - 1 ? d.at(d.nx, j) : -1,
                             j == 0 ? d.at(i, -1) : -1, j == d.ny - 1 ? d.at(i, d.ny) : -1};
    for (int k = 0; k < 4; ++k)
        if (gs[k] >= 0) {
            gz += AZP[gs[k]];
            AZP[gs[k]] = 0.0;
        }
    wk(a, d, W_GZ)[C] += gz;
}

// Gauge misfits of the forward pass: m[g] = ((eta - z) - h_obs)^2 at the
// gauge cells of a pitched state.
template <typename T>
__global__ void k_misfit(Params P, const T* eta, const T* z, const long long* cells, int ngauge,
                         const double* hobs, double* out) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ngauge) return;
    const long long c = cells[g];
    const long long o = (c / P.nx) * P.pitch + (c % P.nx);
    const double dd = ((double)eta[o] - (double)z[o]) - hobs[g];
    out[g] = dd * dd;
}

// gmap[c] = -1 for every cell, then gmap[cells[g]] = g (gauge cells are
// distinct).
__global__ void k_gauge_clear(int* gmap, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride)
        gmap[k] = -1;
}
__global__ void k_gauge_set(const long long* cells, int ngauge, int* gmap) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < ngauge) gmap[cells[g]] = g;
}

__global__ void k_promote(const float* src, double* dst, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride)
        dst[k] = (double)src[k];
}

// Copy the interior of a padded accumulator to a pitched field.
__global__ void k_unpad(Params P, const double* src, double* dst) {
    const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y;
    if (i >= P.nx || j >= P.ny) return;
    dst[(long long)j * P.pitch + i] = src[(long long)(j + 1) * (P.nx + 2) + (i + 1)];
}

// ------------------------------------------------------------ reverse march
//
// The four gather kernels above as one pass.  A 64-lane wave owns a strip of
// padded columns and marches up a chunk of rows, ingesting one row of U^n,
// U*, U^d, the bed and lambda per iteration; earlier rows stay in the lane's
// registers and x neighbours come from the adjacent lanes by DPP shifts.  The
// phases trail the ingested row R:
//   row R    : S15, S14, S13 and the U^n share of S12 (kernel A's work);
//   row R-1  : the flux part of S12, S11, S10, S9 (the U* adjoint, kernel C);
//   row R-2  : the S8 fold of the U* adjoint, S4 (kernel E1) and the switch
//              derivatives of S3;
//   row R-3  : S7, S6, S5, S3 and S2 (kernel E2): lambda^n and the bed's share.
// Each phase reaches one cell further than the one before it, so of the 64
// lanes the middle 58 are output columns.  The expressions, and the order in
// which each cell sums its terms, are those of the gather kernels, so the
// results agree bit for bit.  The adjoint of U^{n+1} is read from one slot of
// a pair and lambda^n written to the other; dJ/dn and dJ/dz are updated in
// place by the cell's owner only.

constexpr int kMarchOutW = kWave - 6;   // output columns per strip

// Padded cell (i, j) that is not a corner.
__device__ __forceinline__ bool padded_ok(const Pad& d, int i, int j) {
    if (i < -1 || i > d.nx || j < -1 || j > d.ny) return false;
    return !((i < 0 || i >= d.nx) && (j < 0 || j >= d.ny));
}

// One neighbour of a cell for the face sums: its cell, bed and adjoint
// vector (zero off the interior).
struct Nbr { Cell c; double z, a0, a1, a2; };

// The terms an x face passes to the cell east of it (the only fields an x
// face changes).
struct XDelta { double e, qx, u, v, h; };

// face_flux_adjoint of an x face for both of its cells at once: the west
// cell's terms are added to cb, the east cell's are returned in d (started
// at zero), with the expressions of face_flux_adjoint for me_is_L true and
// false.
__device__ __forceinline__ void xface_both(const FaceBar& fb, int kind, int dir, bool ghost_is_R,
                                           const Cell& L, const Cell& R, double zL, double zR,
                                           double hdry, double hg, CellBar& cb, XDelta& d) {
    if (kind == BC_WALL) return;
    bool dnR, pass;
    if (kind == BC_INFLOW) {
        dnR = ghost_is_R;
        pass = true;
    } else {
        dnR = dir > 0;
        pass = (dnR ? R.h : L.h) > hdry;
    }
    const Cell& D = dnR ? R : L;
    const double fm = pass ? D.qx : 0.0;
    const double fmb = (fb.m + fb.x * D.u) + fb.y * D.v;
    if (dnR) {
        d.u += fb.x * fm;
        d.v += fb.y * fm;
        if (pass) d.qx += fmb;
    } else {
        cb.u += fb.x * fm;
        cb.v += fb.y * fm;
        if (pass) cb.qx += fmb;
    }
    if (kind >= 0) return;   // boundary faces carry no pressure
    const bool wetL = L.h > hdry, wetR = R.h > hdry;
    const bool bank = (!wetL && zL > R.e) || (!wetR && zR > L.e);
    if (bank) return;
    const double A = hg * (hpos(L.h) + hpos(R.h));
    const double del = R.e - L.e;
    const double Ab = fb.p * del, delb = fb.p * A;
    const double Sb = Ab * hg;
    cb.e -= delb;
    cb.h += L.h > 0.0 ? Sb : 0.0;
    d.e += delb;
    d.h += R.h > 0.0 ? Sb : 0.0;
}

// The x faces of padded cell (i, j) in gather_faces' order: face i (this
// cell west of it, computed here) then face i-1 (computed by the west lane,
// its east terms shifted in).  Every lane of the wave must call it (a DPP
// shift).  EDGE = false: column i and its x neighbours are interior.
template <bool EDGE, bool BND>
__device__ __forceinline__ void x_faces(const Params& P, int i, int j, const Cell& me, double zme,
                                        double am0, double am1, double am2, const Nbr& E, int dir,
                                        double rx, double hdry, double hg, CellBar& cb) {
    if (BND && !(j >= 0 && j < P.ny)) return;   // uniform: rows -1 and ny have no x faces
    XDelta d = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (!EDGE || (i >= -1 && i <= P.nx - 1)) {
        const FaceBar fb = face_bar_v(am0, am1, am2, E.a0, E.a1, E.a2, rx, dir, true);
        xface_both(fb, EDGE ? xface_kind(P, i, j) : -1, dir, EDGE && i == P.nx - 1, me, E.c, zme,
                   E.z, hdry, hg, cb, d);
    }
    const double we = from_west(d.e), wqx = from_west(d.qx), wu = from_west(d.u),
                 wv = from_west(d.v), wh = from_west(d.h);
    if (!EDGE || (i - 1 >= -1 && i - 1 <= P.nx - 1)) {
        cb.u += wu;
        cb.v += wv;
        cb.qx += wqx;
        cb.e += we;
        cb.h += wh;
    }
}

// The y faces of padded cell (i, j), after its x faces, in gather_faces'
// order and with its face rules.  BND = false: rows j-1 .. j+1 are interior,
// so both y faces are interior faces.
template <bool EDGE, bool BND>
__device__ __forceinline__ void y_faces(const Params& P, int i, int j, const Cell& me, double zme,
                                        double am0, double am1, double am2, const Nbr& N,
                                        const Nbr& S, int dir, double ry, double hdry, double hg,
                                        CellBar& cb) {
    if (!EDGE || (i >= 0 && i < P.nx)) {
        if (!BND || (j >= -1 && j <= P.ny - 1)) {
            const FaceBar fb = face_bar_v(am0, am1, am2, N.a0, N.a1, N.a2, ry, dir, false);
            face_flux_adjoint(fb, BND ? yface_kind(P, i, j) : -1, dir, BND && j == P.ny - 1, true,
                              false, me, N.c, zme, N.z, hdry, hg, cb);
        }
        if (!BND || (j - 1 >= -1 && j - 1 <= P.ny - 1)) {
            const FaceBar fb = face_bar_v(S.a0, S.a1, S.a2, am0, am1, am2, ry, dir, false);
            face_flux_adjoint(fb, BND ? yface_kind(P, i, j - 1) : -1, dir,
                              BND && j - 1 == P.ny - 1, false, false, S.c, me, S.z, zme, hdry,
                              hg, cb);
        }
    }
}

// The neighbour in the lane to the east (lane + 1) or in this lane (another
// row).  Depths are formed as e - z from the carried values,
// the expression the cell was built with.
__device__ __forceinline__ Nbr nbr_east(double e, double qx, double qy, double r, double z,
                                        double a0, double a1, double a2) {
    Nbr n;
    const double ee = from_east(e), ze = from_east(z);
    n.c = carried_cell(ee, from_east(qx), from_east(qy), ee - ze, from_east(r));
    n.z = ze;
    n.a0 = from_east(a0);
    n.a1 = from_east(a1);
    n.a2 = from_east(a2);
    return n;
}
__device__ __forceinline__ Nbr nbr_here(double e, double qx, double qy, double r, double z,
                                        double a0, double a1, double a2) {
    Nbr n;
    n.c = carried_cell(e, qx, qy, e - z, r);
    n.z = z;
    n.a0 = a0;
    n.a1 = a1;
    n.a2 = a2;
    return n;
}

// Inputs of one row at the lane's column (clamped into the arrays).
struct MarchRow {
    double ue, ux, uy, se, sx, sy, z, de, dx, dy, m, n, l0, l1, l2, azi, gz, gn;
    int gm;
};

// EDGE: the strip holds the west or the east edge column (its lanes may be
// ghost or outside columns); otherwise every lane is an interior column and
// the column tests are compiled out.
template <bool HOBS, bool EDGE, int PART = 0, bool FLAGS = false>
struct AdjMarch {
    const AdjointArgs& a;
    const int* gmap;
    const double* hobs;
    Pad d;
    const double* LIN;
    const double* AZI;
    double* LOUT;
    double* AZO;
    double* GZ;
    double* GN;
    int i, ii, ic, j0, j1;
    bool colOut;
    double hdry, hg, kap, emax, rcap;
    // outputs of the previous iteration, stored at the start of the next one
    // (ahead of its prefetch, so that waiting for the prefetch never waits
    // for stores): dJ/dz and dJ/dn of row R-1, lambda^n and the bed's share
    // of row R-4
    double o_gz = 0.0, o_gn = 0.0, o_l0 = 0.0, o_l1 = 0.0, o_l2 = 0.0, o_az = 0.0;
    bool o_fa = false, o_wet = false, o_e2 = false;

    // carried rows; index k holds row R - k (ue..zz, ad, azp), R-1-k (aus),
    // R-2-k (fs, un, db, at).  S12's inner adjoint is 0.5 times the U^d
    // adjoint (the product kernel A forms), depths are e - z.
    double ue[5], ux[5], uy[5], ur[5], zz[5];   // U^n cells
    double se[3], sx[3], sy[3], sr[3];          // U* cells
    double ade[4], adx[4], ady[4];              // U^d adjoint (D-bar)
    double azp[4];                              // bed's share
    double ause[3], ausx[3], ausy[3];           // U* adjoint
    double fse[3], fsx[3], fsy[3];              // U* adjoint, S8 fold applied
    double une[2], unx[2], uny[2];              // U^n adjoint, S12 and S4 terms
    double dbx[2], atx[2], aty[2], dby[3];      // switch derivatives of S3
    MarchRow pf;
    // PART 1 and 2 (two waves of one workgroup): the rows wave 1 forms and
    // wave 2 reads, in an LDS ring of 8 rows per field: D-bar of row r
    // (fields 0..2), the bed's share of row r-1 after S12's flux part, the
    // U* adjoint of row r-1 (fields 4..6), all filed under r.
    double* ring = nullptr;
    int lane = 0;
    __device__ __forceinline__ double& rg(int f, int r) const {
        return ring[(f * 8 + (r & 7)) * kWave + lane];
    }
    // FLAGS: the waves hand rows over through two progress counters in LDS
    // (prog[0]: the last row the first wave filed, prog[1]: the last row whose
    // ring slots the second wave has read) instead of a barrier per step, so
    // the first wave may run up to five rows ahead.  Every wait is bounded;
    // a wave whose wait runs out stops waiting (the tile's values are then
    // not to be trusted) and raises *stall.
    int* prog = nullptr;
    int* stall = nullptr;
    int spin_cap = 0;
    bool stalled = false;
    __device__ __forceinline__ void wait_row(int who, int need) {
        if (stalled) return;
        for (int n = 0;; ++n) {
            const int v = __builtin_amdgcn_readfirstlane(__hip_atomic_load(
                prog + who, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP));
            if (v >= need) return;
            if (n >= spin_cap) {
                stalled = true;
                if (lane == 0) __hip_atomic_store(stall, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    __device__ __forceinline__ void post_row(int who, int r) {
        __hip_atomic_store(prog + who, r, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    }

    __device__ AdjMarch(const AdjointArgs& a_, const int* g, const double* h)
        : a(a_), gmap(g), hobs(h) {}

    // Loads at a 32-bit byte offset from a uniform base (every array here is
    // below 4 GiB), so that no per-lane 64-bit address is formed.
    template <typename V>
    __device__ __forceinline__ static V at_off(const V* base, unsigned off) {
        return *(const V*)((const char*)base + off);
    }

    __device__ __forceinline__ void prefetch(int R) {
        const int jj = min(max(R, 0), d.ny - 1);
        const unsigned o = (unsigned)(jj * (int)a.P.pitch + ii) * 8u;
        const unsigned C = (unsigned)((min(max(R, -1), d.ny) + 1) * d.P2 + ic + 1) * 8u;
        const unsigned NB = (unsigned)d.N * 8u;
        if (PART != 1) {
            pf.ue = at_off(a.un[0], o); pf.ux = at_off(a.un[1], o); pf.uy = at_off(a.un[2], o);
        }
        pf.z = at_off(a.zp, C);
        if (PART == 2) return;
        pf.se = at_off(a.us[0], o); pf.sx = at_off(a.us[1], o); pf.sy = at_off(a.us[2], o);
        pf.de = at_off(a.ud[0], o); pf.dx = at_off(a.ud[1], o); pf.dy = at_off(a.ud[2], o);
        pf.m = at_off(a.mp, C);
        pf.n = at_off(a.nman, o);
        pf.l0 = at_off(LIN, C); pf.l1 = at_off(LIN, C + NB); pf.l2 = at_off(LIN, C + 2 * NB);
        pf.azi = at_off(AZI, C);
        pf.gz = at_off(GZ, C);
        pf.gn = at_off(GN, C);
        pf.gm = HOBS ? at_off(gmap, (unsigned)(jj * d.nx + ii) * 4u) : -1;
    }

    template <int K>
    __device__ __forceinline__ static void shift(double* x) {
#pragma unroll
        for (int k = K - 1; k > 0; --k) x[k] = x[k - 1];
    }

    // BND = false: every row an iteration touches is interior (1 .. ny-2),
    // so the row tests are compiled out as well
    __device__ __forceinline__ bool col_in(int x) const { return !EDGE || (x >= 0 && x < d.nx); }
    template <bool BND>
    __device__ __forceinline__ bool in(int x, int y) const {
        return col_in(x) && (!BND || (y >= 0 && y < d.ny));
    }
    template <bool BND>
    __device__ __forceinline__ bool pad_ok(int y) const {
        if (!BND) return !EDGE || (i >= -1 && i <= d.nx);
        return EDGE ? padded_ok(d, i, y) : (y >= -1 && y <= d.ny);
    }

    __device__ __forceinline__ void store_previous(int R) {
        if (PART != 2 && o_fa) {
            const long long C = d.at(i, R - 1);
            GZ[C] = o_gz;
            if (o_wet) GN[C] = o_gn;
        }
        if (PART != 1 && o_e2) {
            const long long C = d.at(i, R - 4);
            LOUT[C] = o_l0;
            LOUT[d.N + C] = o_l1;
            LOUT[2 * d.N + C] = o_l2;
            AZO[C] = o_az;
        }
    }

    // Iteration R forms row R of kernel A's work, row R-1 of C, row R-2 of
    // the fold and E1 and row R-3 of E2.
    template <bool BND>
    __device__ __forceinline__ void iter(int R) {
        const MarchRow q = pf;
        store_previous(R);
        prefetch(R + 1);
        int kW = BC_WALL, kE = BC_WALL;
        if (EDGE) {
            kW = face_kind(a.P, EDGE_W, R);
            kE = face_kind(a.P, EDGE_E, R);
        }
        shift<5>(ue); shift<5>(ux); shift<5>(uy); shift<5>(ur); shift<5>(zz);
        shift<3>(se); shift<3>(sx); shift<3>(sy); shift<3>(sr);
        shift<4>(ade); shift<4>(adx); shift<4>(ady); shift<4>(azp);
        shift<3>(ause); shift<3>(ausx); shift<3>(ausy);
        shift<3>(fse); shift<3>(fsx); shift<3>(fsy);
        shift<2>(une); shift<2>(unx); shift<2>(uny);
        shift<2>(dbx); shift<2>(atx); shift<2>(aty); shift<3>(dby);

        // ---- ingest row R: U^n and U* cells (ghost rule, primitives), bed
        zz[0] = q.z;
        if (PART != 1) {
            const Cell c = make_cell<EDGE, BND>(a.P, q.ue, q.ux, q.uy, a.qin0, i, R, q.z, kW, kE);
            ue[0] = c.e; ux[0] = c.qx; uy[0] = c.qy; ur[0] = c.r;
        }
        if (PART != 2) {
            const Cell c = make_cell<EDGE, BND>(a.P, q.se, q.sx, q.sy, a.qin1, i, R, q.z, kW, kE);
            se[0] = c.e; sx[0] = c.qx; sy[0] = c.qy; sr[0] = c.r;
        }

        // ---- row R: S15, S14, S13, S12's U^n share (with the step reversed
        // before this one's S1 fold and this step's gauge terms)
        if (PART != 2) {
            // the west and east ghosts of lambda and of the bed's share are
            // the neighbouring lanes' values of this row
            double lw0 = 0.0, lw1 = 0.0, lw2 = 0.0, le0 = 0.0, le1 = 0.0, le2 = 0.0;
            double zw = 0.0, ze = 0.0;
            if (EDGE) {
                lw0 = from_west(q.l0); lw1 = from_west(q.l1); lw2 = from_west(q.l2);
                le0 = from_east(q.l0); le1 = from_east(q.l1); le2 = from_east(q.l2);
                zw = from_west(q.azi); ze = from_east(q.azi);
            }
            double o0 = 0.0, o1 = 0.0, o2 = 0.0, oz = 0.0;
            o_fa = false;
            o_wet = false;
            if (in<BND>(i, R)) {
                double lam[3] = {q.l0, q.l1, q.l2};
                if (EDGE && i == 0) fold_value(lw0, lw1, lw2, kW, true, lam);
                if (EDGE && i == d.nx - 1) fold_value(le0, le1, le2, kE, true, lam);
                if (BND && R == 0) {
                    const long long g = d.at(i, -1);
                    fold_value(LIN[g], LIN[d.N + g], LIN[2 * d.N + g], face_kind(a.P, EDGE_S, i),
                               false, lam);
                }
                if (BND && R == d.ny - 1) {
                    const long long g = d.at(i, d.ny);
                    fold_value(LIN[g], LIN[d.N + g], LIN[2 * d.N + g], face_kind(a.P, EDGE_N, i),
                               false, lam);
                }
                const bool own = colOut && R >= j0 && R < j1;
                double gz = 0.0;
                if (own) {
                    double gzs = q.azi;
                    if (EDGE && i == 0) gzs += zw;
                    if (EDGE && i == d.nx - 1) gzs += ze;
                    if (BND && R == 0) gzs += AZI[d.at(i, -1)];
                    if (BND && R == d.ny - 1) gzs += AZI[d.at(i, d.ny)];
                    gz = q.gz + gzs;
                }
                if (HOBS && q.gm >= 0) {
                    const double ef = q.de;
                    const bool clip = ef - q.z < 0.0;
                    const double en = clip ? q.z : ef;
                    const double dd = (en - q.z) - hobs[q.gm];
                    lam[0] += dd + dd;
                    gz += 0.0 - (dd + dd);
                }
                const FaOut f = fa_point(q.de, q.dx, q.dy, q.z, q.m, q.n, lam[0], lam[1], lam[2],
                                         a.dt, hdry, a.P.g);
                o_fa = own;
                o_wet = own && f.wet;
                o_gz = gz;
                o_gn = q.gn + f.gn;
                o0 = f.e; o1 = f.x; o2 = f.y; oz = f.azp;
            }
            ade[0] = o0; adx[0] = o1; ady[0] = o2;
            azp[0] = oz;
        }

        // ---- row R-1: flux part of S12, S11, S10, S9 (the U* adjoint)
        if (PART != 2) {
            const int j = R - 1;
            const double b0 = 0.5 * ade[1], b1 = 0.5 * adx[1], b2 = 0.5 * ady[1];
            const Nbr E = nbr_east(se[1], sx[1], sy[1], sr[1], zz[1], b0, b1, b2);
            const Cell me = carried_cell(se[1], sx[1], sy[1], se[1] - zz[1], sr[1]);
            CellBar cb = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            x_faces<EDGE, BND>(a.P, i, j, me, zz[1], b0, b1, b2, E, -a.sigma, a.rx, hdry, hg, cb);
            double eb = 0.0, qxb = 0.0, qyb = 0.0;
            if (pad_ok<BND>(j)) {
                const Nbr N = nbr_here(se[0], sx[0], sy[0], sr[0], zz[0], 0.5 * ade[0],
                                       0.5 * adx[0], 0.5 * ady[0]);
                const Nbr S = nbr_here(se[2], sx[2], sy[2], sr[2], zz[2], 0.5 * ade[2],
                                       0.5 * adx[2], 0.5 * ady[2]);
                y_faces<EDGE, BND>(a.P, i, j, me, zz[1], b0, b1, b2, N, S, -a.sigma, a.ry, hdry, hg,
                              cb);
                const bool inC = in<BND>(i, j);
                eb = cb.e + (inC ? b0 : 0.0);
                qxb = cb.qx + (inC ? b1 : 0.0);
                qyb = cb.qy + (inC ? b2 : 0.0);
                const double h = me.h, r = me.r;
                qxb += cb.u * r;
                qyb += cb.v * r;
                const double rb = cb.u * me.qx + cb.v * me.qy;
                // r = min(1/h, rcap): no depth derivative where the cap was taken
                const double hb = cb.h + (h > hdry && r < rcap ? -(rb * r) * r : 0.0);
                eb += hb;
                azp[1] -= hb;
            }
            ause[0] = eb; ausx[0] = qxb; ausy[0] = qyb;
        }

        if (PART == 1) {
            // file this iteration's rows for the second wave (with FLAGS, once
            // it has read the slots' previous rows, R-8, last read in its
            // iteration R-5)
            if (FLAGS) wait_row(1, R - 5);
            rg(0, R) = ade[0]; rg(1, R) = adx[0]; rg(2, R) = ady[0];
            rg(3, R) = azp[1];
            rg(4, R) = ause[0]; rg(5, R) = ausx[0]; rg(6, R) = ausy[0];
            if (FLAGS) post_row(0, R);
        }
        if (PART == 2) {
            // the first wave's rows: D-bar of rows R-1..R-3, the bed's share of
            // row R-3, the U* adjoint of rows R-1..R-3
            if (FLAGS) wait_row(0, R);
#pragma unroll
            for (int k = 1; k < 4; ++k) {
                ade[k] = rg(0, R - k); adx[k] = rg(1, R - k); ady[k] = rg(2, R - k);
            }
            azp[3] = rg(3, R - 2);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                ause[k] = rg(4, R - k); ausx[k] = rg(5, R - k); ausy[k] = rg(6, R - k);
            }
            if (FLAGS) post_row(1, R);
        }

        // ---- row R-2: the S8 fold of the U* adjoint
        if (PART != 1) {
            const int j = R - 2;
            double we = 0.0, wx = 0.0, wy = 0.0, ee = 0.0, ex = 0.0, ey = 0.0;
            if (EDGE) {
                we = from_west(ause[1]); wx = from_west(ausx[1]); wy = from_west(ausy[1]);
                ee = from_east(ause[1]); ex = from_east(ausx[1]); ey = from_east(ausy[1]);
            }
            double v[3] = {0.0, 0.0, 0.0};
            if (in<BND>(i, j)) {
                v[0] = ause[1]; v[1] = ausx[1]; v[2] = ausy[1];
                if (EDGE && i == 0) fold_value(we, wx, wy, face_kind(a.P, EDGE_W, j), true, v);
                if (EDGE && i == d.nx - 1)
                    fold_value(ee, ex, ey, face_kind(a.P, EDGE_E, j), true, v);
                if (BND && j == 0)
                    fold_value(ause[2], ausx[2], ausy[2], face_kind(a.P, EDGE_S, i), false, v);
                if (BND && j == d.ny - 1)
                    fold_value(ause[0], ausx[0], ausy[0], face_kind(a.P, EDGE_N, i), false, v);
            }
            fse[0] = v[0]; fsx[0] = v[1]; fsy[0] = v[2];
        }

        // ---- row R-2: S4 (nu-bar and the U^n adjoint's first terms), then
        // the switch derivatives of S3
        if (PART != 1) {
            const int j = R - 2;
            const Cell me = carried_cell(ue[2], ux[2], uy[2], ue[2] - zz[2], ur[2]);
            const double eW = from_west(ue[2]), eE = from_east(ue[2]);
            const double zW = from_west(zz[2]), zE = from_east(zz[2]);
            const double nux = curv_switch(eW, me.e, eE, me.r);
            const double nuy = curv_switch(ue[3], me.e, ue[1], me.r);
            const double nuE = from_east(nux), nuW = from_west(nux);
            const Cell cE = carried_cell(eE, from_east(ux[2]), from_east(uy[2]), eE - zE, 0.0);
            const Cell cW = carried_cell(eW, from_west(ux[2]), from_west(uy[2]), eW - zW, 0.0);
            const double dE[3] = {from_east(ade[2]), from_east(adx[2]), from_east(ady[2])};
            const double dW[3] = {from_west(ade[2]), from_west(adx[2]), from_west(ady[2])};
            double un[3] = {0.0, 0.0, 0.0};
            double dbxv = 0.0, atxv = 0.0, dbyv = 0.0, atyv = 0.0;
            if (in<BND>(i, j)) {
                const double dC[3] = {ade[2], adx[2], ady[2]};
                const double dN[3] = {ade[1], adx[1], ady[1]};
                const double dS[3] = {ade[3], adx[3], ady[3]};
                const Cell cN = carried_cell(ue[1], ux[1], uy[1], ue[1] - zz[1], ur[1]);
                const Cell cS = carried_cell(ue[3], ux[3], uy[3], ue[3] - zz[3], ur[3]);
                const double nuN = curv_switch(ue[2], ue[1], ue[0], ur[1]);
                const double nuS = curv_switch(ue[4], ue[3], ue[2], ur[3]);
                un[0] = 0.5 * ade[2]; un[1] = 0.5 * adx[2]; un[2] = 0.5 * ady[2];
                double nub[2] = {0.0, 0.0};
#pragma unroll
                for (int f = 0; f < 4; ++f) {
                    const bool xf = f < 2;
                    const int ni = xf ? (f == 0 ? i + 1 : i - 1) : i;
                    const int nj = xf ? j : (f == 2 ? j + 1 : j - 1);
                    if (!in<BND>(ni, nj)) continue;   // boundary face: eps = 0
                    const Cell& on = f == 0 ? cE : (f == 1 ? cW : (f == 2 ? cN : cS));
                    const double nuOn = f == 0 ? nuE : (f == 1 ? nuW : (f == 2 ? nuN : nuS));
                    const double* dn = f == 0 ? dE : (f == 1 ? dW : (f == 2 ? dN : dS));
                    const double nuMe = xf ? nux : nuy;
                    const bool meL = f == 0 || f == 2;
                    const Cell& cL = meL ? me : on;
                    const Cell& cR = meL ? on : me;
                    const double nuL = meL ? nuMe : nuOn, nuR = meL ? nuOn : nuMe;
                    int arg;
                    const double eps = eps_and_arg(cL.h, cR.h, nuL, nuR, hdry, kap, emax, arg);
                    const double qL[3] = {cL.e, cL.qx, cL.qy}, qR[3] = {cR.e, cR.qx, cR.qy};
                    double epsb = 0.0;
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const double adL = meL ? dC[k] : dn[k], adR = meL ? dn[k] : dC[k];
                        epsb += (adL - adR) * (qR[k] - qL[k]);
                        un[k] += eps * (dn[k] - dC[k]);
                    }
                    if (arg == (meL ? 0 : 1)) nub[xf ? 0 : 1] += epsb * kap;
                }
                dbxv = switch_dbar(eW, me.e, eE, me.r, nub[0], atxv);
                dbyv = switch_dbar(ue[3], me.e, ue[1], me.r, nub[1], atyv);
            }
            une[0] = un[0]; unx[0] = un[1]; uny[0] = un[2];
            dbx[0] = dbxv; atx[0] = atxv; dby[0] = dbyv; aty[0] = atyv;
        }

        // ---- row R-3: S7, S6, S5, S3, S2: lambda^n and the bed's share
        if (PART != 1) {
            const int j = R - 3;
            const Nbr E = nbr_east(ue[3], ux[3], uy[3], ur[3], zz[3], fse[1], fsx[1], fsy[1]);
            const double dbW = from_west(dbx[1]), dbE = from_east(dbx[1]);
            const Cell me = carried_cell(ue[3], ux[3], uy[3], ue[3] - zz[3], ur[3]);
            CellBar cb = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            x_faces<EDGE, BND>(a.P, i, j, me, zz[3], fse[1], fsx[1], fsy[1], E, a.sigma, a.rx, hdry, hg,
                          cb);
            o_e2 = colOut && j >= j0 && j < j1 && pad_ok<BND>(j);
            if (o_e2) {
                const Nbr N = nbr_here(ue[2], ux[2], uy[2], ur[2], zz[2], fse[0], fsx[0], fsy[0]);
                const Nbr S = nbr_here(ue[4], ux[4], uy[4], ur[4], zz[4], fse[2], fsx[2], fsy[2]);
                y_faces<EDGE, BND>(a.P, i, j, me, zz[3], fse[1], fsx[1], fsy[1], N, S, a.sigma, a.ry,
                              hdry, hg, cb);
                const bool inC = in<BND>(i, j);
                double eb = cb.e, qxb = cb.qx, qyb = cb.qy;
                if (inC) {
                    eb += une[1] + fse[1];
                    qxb += unx[1] + fsx[1];
                    qyb += uny[1] + fsy[1];
                }
                double rb = cb.u * me.qx + cb.v * me.qy;
                if (in<BND>(i - 1, j)) eb += dbW;
                if (inC) {
                    eb += -dbx[1] - dbx[1];
                    rb += atx[1];
                }
                if (in<BND>(i + 1, j)) eb += dbE;
                if (in<BND>(i, j - 1)) eb += dby[2];
                if (inC) {
                    eb += -dby[1] - dby[1];
                    rb += aty[1];
                }
                if (in<BND>(i, j + 1)) eb += dby[0];
                const double h = me.h, r = me.r;
                qxb += cb.u * r;
                qyb += cb.v * r;
                // r = min(1/h, rcap): no depth derivative where the cap was taken
                const double hb = cb.h + (h > hdry && r < rcap ? -(rb * r) * r : 0.0);
                eb += hb;
                o_l0 = eb;
                o_l1 = qxb;
                o_l2 = qyb;
                o_az = azp[3] - hb;
            }
        }
    }

    // Dry tile.  Where U^n, U* and U^d are dry (0 <= h <= h_dry for U^d, h <=
    // h_dry for the others) on every cell within two cells of the tile's
    // output cells, and the tile is away from the domain edges, the reversed
    // step reduces to: lambda_eta passes through (with this step's gauge
    // term), lambda_q and the bed's share vanish, and dJ/dz takes the bed
    // share of the step reversed before (no donor flux, no dissipation, no
    // friction and no clipping act there, and every pressure term is
    // multiplied by a zero momentum adjoint).  The values equal the full
    // march's; only the sign of a zero can differ.  The test reads three
    // depths per cell and stops at the first batch of rows with a wet cell.
    // Both loops work in batches of kBatch rows, all loads of a batch issued
    // before its test or its stores, so that they do not wait on memory row
    // after row.
    static constexpr int kBatch = 8;

    __device__ __forceinline__ bool dry_tile(int lane) const {
        const double* E0 = a.un[0];
        const double* E1 = a.us[0];
        const double* E2 = a.ud[0];
        const bool edgeLane = lane < 1 || lane > kWave - 2;
        for (int j = j0 - 2; j <= j1 + 1; j += kBatch) {
            bool wet = false;
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int jj = j + u;
                if (jj <= j1 + 1) {
                    const long long o = pitched(a.P, ii, jj);
                    const double z = a.zp[d.at(ic, jj)];
                    const double hn = E0[o] - z, hs = E1[o] - z, hd = E2[o] - z;
                    wet = wet ||
                          !(edgeLane || (hn <= hdry && hs <= hdry && hd <= hdry && hd >= 0.0));
                }
            }
            if (__ballot(wet) != 0ull) return false;
        }
        return true;
    }

    __device__ __forceinline__ void dry_rows() {
        if (!colOut) return;
        for (int j = j0; j < j1; j += kBatch) {
            double l0[kBatch], gz[kBatch];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                if (j + u < j1) {
                    const long long C = d.at(i, j + u);
                    l0[u] = LIN[C];
                    gz[u] = GZ[C] + AZI[C];
                }
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                if (j + u >= j1) continue;
                const int jj = j + u;
                const long long C = d.at(i, jj);
                if (HOBS) {
                    const int g = gmap[(long long)jj * d.nx + i];
                    if (g >= 0) {
                        const double ef = a.ud[0][pitched(a.P, i, jj)], z = a.zp[C];
                        const bool clip = ef - z < 0.0;
                        const double en = clip ? z : ef;
                        const double dd = (en - z) - hobs[g];
                        l0[u] += dd + dd;
                        gz[u] += 0.0 - (dd + dd);
                    }
                }
                LOUT[C] = l0[u];
                LOUT[d.N + C] = 0.0;
                LOUT[2 * d.N + C] = 0.0;
                AZO[C] = 0.0;
                GZ[C] = gz[u];
            }
        }
    }

    __device__ __forceinline__ void run(int lane_, int strip, int chunk, int H, int lout,
                                        int zout) {
        lane = lane_;
        d = pad_of(a.P);
        LIN = wk(a, d, a.lam_slot);
        AZI = wk(a, d, a.azp_slot);
        LOUT = wk(a, d, lout);
        AZO = wk(a, d, zout);
        GZ = wk(a, d, W_GZ);
        GN = wk(a, d, W_GN);
        hdry = a.P.h_dry;
        rcap = a.P.rcap;
        hg = 0.5 * a.P.g;
        kap = a.P.kappa;
        emax = a.P.eps_max;
        const int pc = strip * kMarchOutW - 3 + lane;   // padded column of the lane
        i = pc - 1;
        ii = min(max(i, 0), a.P.nx - 1);
        ic = min(max(i, -1), a.P.nx);
        colOut = lane >= 3 && lane < 3 + kMarchOutW && pc <= a.P.nx + 1;
        const int py0 = chunk * H, py1 = min(py0 + H, a.P.ny + 2);
        j0 = py0 - 1;
        j1 = py1 - 1;
        // a tile of an interior strip at least five rows from the south and
        // north edges may be a dry tile
        if (!EDGE && j0 - 5 >= 0 && j1 + 4 <= d.ny - 1 && dry_tile(lane)) {
            if (PART != 2) dry_rows();
            return;
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) ue[k] = ux[k] = uy[k] = ur[k] = zz[k] = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            se[k] = sx[k] = sy[k] = sr[k] = 0.0;
            ause[k] = ausx[k] = ausy[k] = 0.0;
            fse[k] = fsx[k] = fsy[k] = 0.0;
            dby[k] = 0.0;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) ade[k] = adx[k] = ady[k] = azp[k] = 0.0;
#pragma unroll
        for (int k = 0; k < 2; ++k) une[k] = unx[k] = uny[k] = dbx[k] = atx[k] = aty[k] = 0.0;
        // iterations j0-3 .. j0+2 fill the pipeline; from j0+3 on, iteration
        // R forms lambda^n of row R-3 (stored by the next iteration).  (Leaving
        // the unneeded phases out of the filling iterations was measured
        // slower: the extra code raises the main loop's register pressure.)
        if (PART == 0) {
            prefetch(j0 - 3);
            // rows that reach the domain's first or last two rows take the
            // general iteration, the others the interior one
            int R = j0 - 3;
            for (; R <= j1 + 2 && R < 5; ++R) iter<true>(R);
            for (; R <= j1 + 2 && R <= d.ny - 3; ++R) iter<false>(R);
            for (; R <= j1 + 2; ++R) iter<true>(R);
            store_previous(j1 + 3);
            return;
        }
        // Two waves: the first forms rows R and R-1 of iteration R, the
        // second rows R-2 and R-3 of the same iteration after it, from the
        // rows the first filed in the ring (zero before any is filed, as the
        // carried rows are).  FLAGS: the progress counters order the two;
        // otherwise one workgroup barrier per step, the second wave one step
        // behind.
        if (PART == 1) {
            for (int k = 0; k < 7 * 8; ++k) ring[k * kWave + lane] = 0.0;
            if (FLAGS && lane == 0) prog[0] = prog[1] = j0 - 4;
        }
        __syncthreads();
        prefetch(j0 - 3);
        if (FLAGS) {
            for (int R = j0 - 3; R <= j1 + 2; ++R) {
                if (R >= 5 && R <= d.ny - 3)
                    iter<false>(R);
                else
                    iter<true>(R);
            }
            store_previous(j1 + 3);
            return;
        }
        for (int t = j0 - 3; t <= j1 + 3; ++t) {
            const int R = PART == 1 ? t : t - 1;
            if (PART == 1 ? R <= j1 + 2 : R >= j0 - 3) {
                if (R >= 5 && R <= d.ny - 3)
                    iter<false>(R);
                else
                    iter<true>(R);
            }
            __syncthreads();
        }
        store_previous(j1 + 3);
    }
};

// Strips holding an edge column: strip 0 and strips from `se` on (a lane of
// strip s sits in column 58 s - 4 + lane).
__host__ __device__ inline int march_first_east_strip(int nx) {
    const int v = nx - (kWave - 4);
    return v <= 0 ? 0 : (v + kMarchOutW - 1) / kMarchOutW;
}

// Tiles: strip 0 in chunks of He rows, the interior strips in chunks of H,
// the east edge strips in chunks of He (an edge strip's iteration costs more,
// so its chunks are shorter and its waves end with the others).
struct MarchTiles {
    int H, He, gy, gye, strips, se;
    __host__ __device__ int count() const {
        return se <= 1 ? strips * gye : gye + (se - 1) * gy + (strips - se) * gye;
    }
};

template <bool HOBS>
__global__ void __launch_bounds__(kWave, 1)
k_adj_march(AdjointArgs a, const int* gmap, const double* hobs, MarchTiles T, int lout, int zout) {
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    int strip, chunk, H;
    if (T.se <= 1) {
        strip = t / T.gye; chunk = t % T.gye; H = T.He;
    } else if (t < T.gye) {
        strip = 0; chunk = t; H = T.He;
    } else if (t < T.gye + (T.se - 1) * T.gy) {
        strip = 1 + (t - T.gye) / T.gy; chunk = (t - T.gye) % T.gy; H = T.H;
    } else {
        const int u = t - T.gye - (T.se - 1) * T.gy;
        strip = T.se + u / T.gye; chunk = u % T.gye; H = T.He;
    }
    const int lane = threadIdx.x;
    if (strip == 0 || strip >= T.se) {
        AdjMarch<HOBS, true> M(a, gmap, hobs);
        M.run(lane, strip, chunk, H, lout, zout);
    } else {
        AdjMarch<HOBS, false> M(a, gmap, hobs);
        M.run(lane, strip, chunk, H, lout, zout);
    }
}

// The march as a two-wave pipeline (one workgroup of two waves per tile):
// wave 0 forms rows R and R-1 of each iteration (S15..S9: D-bar, the U*
// adjoint, dJ/dn and dJ/dz), wave 1 rows R-2 and R-3 (the S8 fold, S4, S3 and
// S7..S2: lambda^n and the bed's share), behind it, from the rows wave 0
// files in LDS (FLAGS: ordered by two LDS progress counters, wave 0 up to five
// rows ahead; otherwise in step at a barrier, one step behind).  Each wave
// carries about half the rows, so two fit per SIMD (256 registers) where the
// one-wave march holds one; the sums and their order are the one-wave march's,
// so the results are the same bits.  The hardware places the two waves of a
// workgroup on two SIMDs of the compute unit.
template <bool HOBS, bool FLAGS>
__global__ void __launch_bounds__(2 * kWave, 2)
k_adj_march2(AdjointArgs a, const int* gmap, const double* hobs, MarchTiles T, int lout,
             int zout, int* stall, int spin_cap) {
    __shared__ double ring[7 * 8 * kWave];
    __shared__ int prog[2];
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    int strip, chunk, H;
    if (T.se <= 1) {
        strip = t / T.gye; chunk = t % T.gye; H = T.He;
    } else if (t < T.gye) {
        strip = 0; chunk = t; H = T.He;
    } else if (t < T.gye + (T.se - 1) * T.gy) {
        strip = 1 + (t - T.gye) / T.gy; chunk = (t - T.gye) % T.gy; H = T.H;
    } else {
        const int u = t - T.gye - (T.se - 1) * T.gy;
        strip = T.se + u / T.gye; chunk = u % T.gye; H = T.He;
    }
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const bool edge = strip == 0 || strip >= T.se;
    if (edge && wave == 0) {
        AdjMarch<HOBS, true, 1, FLAGS> M(a, gmap, hobs);
        M.ring = ring;
        M.prog = prog;
        M.stall = stall;
        M.spin_cap = spin_cap;
        M.run(lane, strip, chunk, H, lout, zout);
    } else if (edge) {
        AdjMarch<HOBS, true, 2, FLAGS> M(a, gmap, hobs);
        M.ring = ring;
        M.prog = prog;
        M.stall = stall;
        M.spin_cap = spin_cap;
        M.run(lane, strip, chunk, H, lout, zout);
    } else if (wave == 0) {
        AdjMarch<HOBS, false, 1, FLAGS> M(a, gmap, hobs);
        M.ring = ring;
        M.prog = prog;
        M.stall = stall;
        M.spin_cap = spin_cap;
        M.run(lane, strip, chunk, H, lout, zout);
    } else {
        AdjMarch<HOBS, false, 2, FLAGS> M(a, gmap, hobs);
        M.ring = ring;
        M.prog = prog;
        M.stall = stall;
        M.spin_cap = spin_cap;
        M.run(lane, strip, chunk, H, lout, zout);
    }
}

inline dim3 grid2(int w, int h) { return dim3((w + kBX - 1) / kBX, (h + kBY - 1) / kBY); }

}  // namespace

int adjoint_work_arrays() { return 20; }

hipError_t launch_adjoint_step(const AdjointArgs& a, const int* gmap, const double* hobs,
                               hipStream_t s) {
    const int nx = a.P.nx, ny = a.P.ny;
    const dim3 b2(kBX, kBY);
    hipLaunchKernelGGL(k_adj_fa, grid2(nx, ny), b2, 0, s, a, gmap, hobs);
    hipLaunchKernelGGL(k_adj_c, grid2(nx + 2, ny + 2), b2, 0, s, a);
    hipLaunchKernelGGL(k_adj_e1, grid2(nx, ny), b2, 0, s, a);
    hipLaunchKernelGGL(k_adj_e2, grid2(nx + 2, ny + 2), b2, 0, s, a);
    return hipGetLastError();
}

namespace {

// Edge strips' rows cost about 1.75 interior rows (the best of 1.3 .. 2.3 on 1024 x 1024);
// every chunk also pays 6 rows of pipeline fill.
MarchTiles march_tiles(const Params& P, int H) {
    MarchTiles T;
    T.H = H;
    T.He = std::max(4, (int)std::lround((H + 6) / 1.75) - 6);
    T.strips = (P.nx + 2 + kMarchOutW - 1) / kMarchOutW;
    T.se = std::min(march_first_east_strip(P.nx), T.strips);
    T.gy = (P.ny + 2 + T.H - 1) / T.H;
    T.gye = (P.ny + 2 + T.He - 1) / T.He;
    return T;
}

}  // namespace

bool adjoint_march_fits(const Params& P) {
    // the march addresses its arrays by 32-bit byte offsets: three padded
    // fields from one base, and one pitched field
    const double pad = (double)(P.nx + 2) * (double)(P.ny + 2) * 8.0;
    const double pit = (double)P.ny * (double)P.pitch * 8.0;
    return 3.0 * pad < 4294967296.0 && pit < 4294967296.0;
}

int adjoint_march_rows(const Params& P, int ncu, int per_cu) {
    // the smallest chunk height (8 .. 256) whose tiles fit per_cu per compute
    // unit in one round.  Four: one wave per SIMD for the one-wave march, two
    // (one two-wave workgroup per SIMD pair of waves) for the two-wave march.
    // Three, when a recompute runs beside the march: two SIMDs then hold one
    // march wave of 208 registers and have room for one of the tracing step
    const long long slots = (long long)std::max(per_cu, 1) * std::max(ncu, 1);
    int H = 8;
    while (H < 256 && march_tiles(P, H).count() > slots) ++H;
    return H;
}

hipError_t launch_adjoint_march(const AdjointArgs& a, const int* gmap, const double* hobs, int H,
                                hipStream_t s, MarchMode mode, int* stall, int spin_cap) {
    if (H < 1) return hipErrorInvalidValue;
    if (mode == MarchMode::flags && !stall) return hipErrorInvalidValue;
    const MarchTiles T = march_tiles(a.P, H);
    const int lout = a.lam_slot == kAdjLamSlot[0] ? kAdjLamSlot[1] : kAdjLamSlot[0];
    const int zout = a.azp_slot == kAdjZpSlot[0] ? kAdjZpSlot[1] : kAdjZpSlot[0];
    const dim3 g(T.count()), b2(2 * kWave);
    switch (mode) {
    case MarchMode::flags:
        if (hobs)
            hipLaunchKernelGGL((k_adj_march2<true, true>), g, b2, 0, s, a, gmap, hobs, T, lout, zout, stall, spin_cap);
        else
            hipLaunchKernelGGL((k_adj_march2<false, true>), g, b2, 0, s, a, gmap, hobs, T, lout, zout, stall, spin_cap);
        break;
    case MarchMode::barrier:
        if (hobs)
            hipLaunchKernelGGL((k_adj_march2<true, false>), g, b2, 0, s, a, gmap, hobs, T, lout, zout, stall, spin_cap);
        else
            hipLaunchKernelGGL((k_adj_march2<false, false>), g, b2, 0, s, a, gmap, hobs, T, lout, zout, stall, spin_cap);
        break;
    case MarchMode::one_wave:
        if (hobs)
            hipLaunchKernelGGL(k_adj_march<true>, g, dim3(kWave), 0, s, a, gmap, hobs, T, lout, zout);
        else
            hipLaunchKernelGGL(k_adj_march<false>, g, dim3(kWave), 0, s, a, gmap, hobs, T, lout, zout);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_adjoint_finish(const AdjointArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_f, grid2(a.P.nx, a.P.ny), dim3(kBX, kBY), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_gauge_map(const Params& P, const long long* cells, int ngauge, int* gmap,
                            hipStream_t s) {
    const size_t n = (size_t)P.nx * (size_t)P.ny;
    size_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_gauge_clear, dim3((unsigned)blocks), dim3(256), 0, s, gmap, n);
    if (ngauge > 0)
        hipLaunchKernelGGL(k_gauge_set, dim3((ngauge + 255) / 256), dim3(256), 0, s, cells,
                           ngauge, gmap);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_misfit(const Params& P, const T* eta, const T* z, const long long* cells,
                         int ngauge, const double* hobs, double* out, hipStream_t s) {
    if (ngauge <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_misfit<T>, dim3((ngauge + 255) / 256), dim3(256), 0, s, P, eta, z, cells,
                       ngauge, hobs, out);
    return hipGetLastError();
}
template hipError_t launch_misfit<float>(const Params&, const float*, const float*,
                                         const long long*, int, const double*, double*,
                                         hipStream_t);
template hipError_t launch_misfit<double>(const Params&, const double*, const double*,
                                          const long long*, int, const double*, double*,
                                          hipStream_t);

hipError_t launch_promote(const float* src, double* dst, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_promote, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_unpad(const Params& P, const double* src, double* dst, hipStream_t s) {
    hipLaunchKernelGGL(k_unpad, grid2(P.nx, P.ny), dim3(kBX, kBY), 0, s, P, src, dst);
    return hipGetLastError();
}

}  // namespace swe
