// swe_adjoint.hip -- discrete adjoint of one time step (FP64).
//
// Reverse mode through S15 .. S1 of one step, given the forward
// intermediates of that step as the unfused path records them (the 47
// padded arrays of the parity ladder, plus the padded bed zp and m = g n^2).
// The adjoint lam^{n+1} of U^{n+1} (plus the gauge misfit terms of the loss
// when step n+1 is observed) becomes lam^n, the adjoint of U^n, and the
// step's contributions to dJ/dn and dJ/dz are added to the accumulators.
// dt^n is held fixed (not differentiated).
//
// Every kernel gathers: a thread owns one cell (or one padded cell) and
// recomputes what it needs from the faces and neighbours that reach it, so
// there are no atomics and the result does not depend on thread order.
// Derivative conventions (the same as the CPU reference's): branches are
// taken as in the forward step; max/min pass the derivative to the argument
// they return (the second on a tie); |x| has derivative sign(x) (0 at 0);
// sqrt has derivative 0 at 0; the cube root's first guess is a constant and
// its two Halley steps are differentiated as executed.
#include "swe_common.hpp"
#include "swe_internal.hpp"

namespace swe {

namespace {

constexpr int kBX = 64, kBY = 4;

enum {
    T_UN = 0, T_H = 3, T_R = 4, T_U = 5, T_V = 6, T_NUX = 7, T_NUY = 8, T_D = 9, T_F = 12,
    T_G = 16, T_US = 20, T_HS = 23, T_RS = 24, T_USU = 25, T_USV = 26, T_FS = 27, T_GS = 31,
    T_UC = 35, T_UD = 38, T_UF = 41, T_UNEW = 44
};

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

__device__ __forceinline__ const double* tr(const AdjointArgs& a, const Pad& d, int k) {
    return a.trace + (long long)k * d.N;
}
__device__ __forceinline__ double* wk(const AdjointArgs& a, const Pad& d, int k) {
    return a.work + (long long)k * d.N;
}

// Adjoint work arrays (padded): corrector inner adjoint a-bar (3), U^d-bar
// (= D-bar, 3), U*-bar (3), U^n-bar (3), nu-bar (2), zp-bar, lambda (3),
// dJ/dn and dJ/dz accumulators.
enum { W_AB = 0, W_AD = 3, W_AUS = 6, W_AUN = 9, W_ANX = 12, W_ANY = 13, W_AZP = 14,
       W_LAM = 15, W_GN = 18, W_GZ = 19 };

// Reverse of the friction cube root y = cbrt3(x): returns x-bar given y-bar.
__device__ double cbrt3_adjoint(double x, double ybar) {
    const unsigned w = (unsigned)__double2hiint(x);
    double y[3];
    y[0] = __hiloint2double((int)(w / 3u + 0x2A9F7893u), 0);
    double tt[2], num[2], den[2], q[2];
    for (int k = 0; k < 2; ++k) {
        tt[k] = (y[k] * y[k]) * y[k];
        num[k] = tt[k] + (x + x);
        den[k] = (tt[k] + tt[k]) + x;
        q[k] = num[k] / den[k];
        y[k + 1] = y[k] * q[k];
    }
    double xbar = 0.0;
    for (int k = 1; k >= 0; --k) {
        const double qbar = ybar * y[k];
        ybar = ybar * q[k];
        const double numbar = qbar / den[k];
        const double denbar = -(qbar * q[k]) / den[k];
        // den = (t + t) + x, num = t + (x + x)
        xbar += denbar;
        double tbar = denbar + denbar + numbar;
        xbar += numbar + numbar;
        // t = (y*y)*y
        const double yy = y[k] * y[k];
        const double yybar = tbar * y[k];
        ybar += tbar * yy;
        ybar += yybar * y[k] + yybar * y[k];
    }
    return xbar;
}

// Loss terms of an observed step: lambda_eta += 2 d and dJ/dz -= 2 d at
// each gauge, d = (eta^{n+1} - z) - h_obs.  Gauge cells are distinct.
__global__ void k_adj_seed(AdjointArgs a, const long long* cells, int ngauge, const double* hobs) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ngauge) return;
    const Pad d = pad_of(a.P);
    const long long c = cells[g];
    const int i = (int)(c % a.P.nx), j = (int)(c / a.P.nx);
    const long long C = d.at(i, j);
    const double dd = (tr(a, d, T_UNEW)[C] - a.zp[C]) - hobs[g];
    wk(a, d, W_LAM)[C] += dd + dd;
    wk(a, d, W_GZ)[C] += 0.0 - (dd + dd);
}

// S15, S14, S13 and the U^n share of S12, per interior cell.
__global__ void k_adj_a(AdjointArgs a) {
    const Pad d = pad_of(a.P);
    const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y;
    if (i >= d.nx || j >= d.ny) return;
    const long long C = d.at(i, j);
    const double hdry = a.P.h_dry, zp = a.zp[C];
    const double* LAM = wk(a, d, W_LAM);
    const double le = LAM[C], lx = LAM[d.N + C], ly = LAM[2 * d.N + C];
    // S15 dry fix
    const double ef = tr(a, d, T_UF)[C];
    const bool clip = ef - zp < 0.0;
    const double en = clip ? zp : ef;
    const bool dry = !(en - zp > hdry);
    double azp = clip ? le : 0.0;
    const double efb = clip ? 0.0 : le;
    const double qxfb = dry ? 0.0 : lx, qyfb = dry ? 0.0 : ly;
    // S14 friction
    const double ed = tr(a, d, T_UD)[C], qx = tr(a, d, T_UD + 1)[C], qy = tr(a, d, T_UD + 2)[C];
    const double h = ed - zp;
    double edb = efb, qxdb = qxfb, qydb = qyfb;
    if (h > hdry) {
        const double r = 1.0 / h;
        const double x2 = qx * qx + qy * qy;
        const double w = sqrt(x2);
        const double s = w * r;
        const double c3 = tcbrt(r);
        const double k = r * c3;
        const double dtm = a.dt * a.mp[C];
        const double A = dtm * s;
        const double B = A * k;
        const double phi = 1.0 + B;
        const double psi = 1.0 / phi;
        const double psib = qxfb * qx + qyfb * qy;
        qxdb = qxfb * psi;
        qydb = qyfb * psi;
        const double phib = -(psib * psi) / phi;
        const double Ab = phib * k, kb = phib * A;
        const double dtmb = Ab * s, sb = Ab * dtm;
        const double mb = dtmb * a.dt;
        double rb = kb * c3 + sb * w;
        rb += cbrt3_adjoint(r, kb * r);
        const double wb = sb * r;
        if (x2 > 0.0) {
            const double x2b = wb * (0.5 / w);
            qxdb += x2b * qx + x2b * qx;
            qydb += x2b * qy + x2b * qy;
        }
        const double hb = -(rb * r) / h;
        edb += hb;
        azp -= hb;
        // m = g n^2 at this cell
        const double n = a.nman[(long long)j * a.P.pitch + i];
        const double mg = mb * a.P.g;
        wk(a, d, W_GN)[C] += mg * n + mg * n;
    }
    // S13: U^d = U^c + D; S12: U^c = 0.5*(U^n + a)
    double* AD = wk(a, d, W_AD);
    double* AB = wk(a, d, W_AB);
    AD[C] = edb; AD[d.N + C] = qxdb; AD[2 * d.N + C] = qydb;
    AB[C] = 0.5 * edb; AB[d.N + C] = 0.5 * qxdb; AB[2 * d.N + C] = 0.5 * qydb;
    wk(a, d, W_AZP)[C] = azp;
}

// Adjoint of the flux-divergence update out = base - L_dir (S7 / inner S12)
// seen from one face: the face's (Fm, Fx, Fy, P) adjoints, given the
// adjoint A of `out` on the two cells of the face (zero off the interior).
struct FaceBar { double m, x, y, p; };

__device__ __forceinline__ FaceBar face_bar(const double* A0, const double* A1, const double* A2,
                                            const Pad& d, int iL, int jL, int iR, int jR,
                                            double coef, int dir, bool xface) {
    const bool inL = d.interior(iL, jL), inR = d.interior(iR, jR);
    const long long L = d.at(iL, jL), R = d.at(iR, jR);
    FaceBar f;
    const double aL0 = inL ? A0[L] : 0.0, aR0 = inR ? A0[R] : 0.0;
    const double aL1 = inL ? A1[L] : 0.0, aR1 = inR ? A1[R] : 0.0;
    const double aL2 = inL ? A2[L] : 0.0, aR2 = inR ? A2[R] : 0.0;
    f.m = coef * aR0 - coef * aL0;
    f.x = coef * aR1 - coef * aL1;
    f.y = coef * aR2 - coef * aL2;
    // the pressure sits in the x-momentum update (x faces) or the
    // y-momentum update (y faces) of the cell on the dir side
    const double aPL = xface ? aL1 : aL2, aPR = xface ? aR1 : aR2;
    f.p = dir > 0 ? -(coef * aPL) : -(coef * aPR);
    return f;
}

// Contributions of one face's flux adjoint to the adjoints of the cell
// `me` (one of L, R): eta-bar, qx-bar, qy-bar, u-bar, v-bar, h-bar.
struct CellBar { double e, qx, qy, u, v, h; };

__device__ __forceinline__ void face_flux_adjoint(const FaceBar& fb, int kind, int dir,
                                                  bool ghost_is_R, long long L, long long R,
                                                  bool me_is_L, bool xface, const double* E,
                                                  const double* QN, const double* H,
                                                  const double* U, const double* V,
                                                  const double* Z, double hdry, double hg,
                                                  CellBar& cb) {
    if (kind == BC_WALL) return;
    long long dn;
    bool pass;
    if (kind == BC_INFLOW) {
        dn = ghost_is_R ? R : L;
        pass = true;
    } else {
        dn = dir > 0 ? R : L;
        pass = H[dn] > hdry;
    }
    const long long me = me_is_L ? L : R;
    if (dn == me) {
        const double fm = pass ? QN[dn] : 0.0;
        const double fmb = (fb.m + fb.x * U[dn]) + fb.y * V[dn];
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
    const bool wetL = H[L] > hdry, wetR = H[R] > hdry;
    const bool bank = (!wetL && Z[L] > E[R]) || (!wetR && Z[R] > E[L]);
    if (bank) return;
    const double hL = H[L], hR = H[R];
    const double A = hg * (hpos(hL) + hpos(hR));
    const double del = E[R] - E[L];
    const double Ab = fb.p * del, delb = fb.p * A;
    const double Sb = Ab * hg;
    if (me_is_L) {
        cb.e -= delb;
        cb.h += hL > 0.0 ? Sb : 0.0;
    } else {
        cb.e += delb;
        cb.h += hR > 0.0 ? Sb : 0.0;
    }
}

__device__ __forceinline__ int xface_kind(const Params& P, int fi, int j) {
    return fi == -1 ? face_kind(P, EDGE_W, j) : (fi == P.nx - 1 ? face_kind(P, EDGE_E, j) : -1);
}
__device__ __forceinline__ int yface_kind(const Params& P, int i, int fj) {
    return fj == -1 ? face_kind(P, EDGE_S, i) : (fj == P.ny - 1 ? face_kind(P, EDGE_N, i) : -1);
}

// Sum over the (up to) four faces of padded cell (i, j) of the flux
// adjoints, for the fluxes of the state at trace slots (src, prim) with
// donor direction dir, whose update's adjoint is A (three arrays).
__device__ CellBar gather_faces(const AdjointArgs& a, const Pad& d, int i, int j, int src,
                                int prim, int dir, const double* A0, const double* A1,
                                const double* A2, double rx, double ry) {
    CellBar cb = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const double hdry = a.P.h_dry, hg = 0.5 * a.P.g;
    const double* E = tr(a, d, src);
    const double* QX = tr(a, d, src + 1);
    const double* QY = tr(a, d, src + 2);
    const double* H = tr(a, d, prim);
    const double* U = tr(a, d, prim + 2);
    const double* V = tr(a, d, prim + 3);
    if (j >= 0 && j < d.ny) {    // x faces: rows 0 .. ny-1, slots -1 .. nx-1
        for (int side = 0; side < 2; ++side) {
            const int fi = side == 0 ? i : i - 1;    // me is L of face fi when side == 0
            if (fi < -1 || fi > d.nx - 1) continue;
            const int kind = xface_kind(a.P, fi, j);
            const FaceBar fb = face_bar(A0, A1, A2, d, fi, j, fi + 1, j, rx, dir, true);
            face_flux_adjoint(fb, kind, dir, fi == d.nx - 1, d.at(fi, j), d.at(fi + 1, j),
                              side == 0, true, E, QX, H, U, V, a.zp, hdry, hg, cb);
        }
    }
    if (i >= 0 && i < d.nx) {    // y faces: columns 0 .. nx-1, slots -1 .. ny-1
        for (int side = 0; side < 2; ++side) {
            const int fj = side == 0 ? j : j - 1;
            if (fj < -1 || fj > d.ny - 1) continue;
            const int kind = yface_kind(a.P, i, fj);
            const FaceBar fb = face_bar(A0, A1, A2, d, i, fj, i, fj + 1, ry, dir, false);
            face_flux_adjoint(fb, kind, dir, fj == d.ny - 1, d.at(i, fj), d.at(i, fj + 1),
                              side == 0, false, E, QY, H, U, V, a.zp, hdry, hg, cb);
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
    const double* AB = wk(a, d, W_AB);
    const CellBar cb = gather_faces(a, d, i, j, T_US, T_HS, -a.sigma, AB, AB + d.N, AB + 2 * d.N,
                                    a.rx, a.ry);
    const bool in = d.interior(i, j);
    double eb = cb.e + (in ? AB[C] : 0.0);
    double qxb = cb.qx + (in ? AB[d.N + C] : 0.0);
    double qyb = cb.qy + (in ? AB[2 * d.N + C] : 0.0);
    // S9: h = eta - zp, r = wet ? 1/h : 0, u = qx r, v = qy r
    const double h = tr(a, d, T_HS)[C], r = tr(a, d, T_RS)[C];
    const double qx = tr(a, d, T_US + 1)[C], qy = tr(a, d, T_US + 2)[C];
    qxb += cb.u * r;
    qyb += cb.v * r;
    const double rb = cb.u * qx + cb.v * qy;
    const double hb = cb.h + (h > a.P.h_dry ? -(rb * r) / h : 0.0);
    eb += hb;
    double* AUS = wk(a, d, W_AUS);
    AUS[C] = eb;
    AUS[d.N + C] = qxb;
    AUS[2 * d.N + C] = qyb;
    wk(a, d, W_AZP)[C] -= hb;
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

// S8: the ghost ring of U* folded into the edge cells.
__global__ void k_adj_d(AdjointArgs a) {
    const Pad d = pad_of(a.P);
    const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y;
    if (i >= d.nx || j >= d.ny) return;
    if (i > 0 && i < d.nx - 1 && j > 0 && j < d.ny - 1) return;
    fold_ring(a, wk(a, d, W_AUS), d, i, j);
}

// Face coefficient of S4 between cells L and R and the derivative of it
// with respect to nu: which of the two it follows (0: L, 1: R, -1: none).
__device__ __forceinline__ double eps_and_arg(const double* H, const double* NU, long long L,
                                              long long R, double hdry, double kap, double emax,
                                              int& arg) {
    arg = -1;
    if (!(H[L] > hdry && H[R] > hdry)) return 0.0;
    const bool takeL = NU[L] > NU[R];
    const double t = kap * (takeL ? NU[L] : NU[R]);
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
    const double* H = tr(a, d, T_H);
    const double* Q = tr(a, d, T_UN);
    const double* AD = wk(a, d, W_AD);
    const double* AB = wk(a, d, W_AB);
    double un[3] = {AB[C], AB[d.N + C], AB[2 * d.N + C]};
    double nub[2] = {0.0, 0.0};
    for (int f = 0; f < 4; ++f) {
        const bool xf = f < 2;
        const int ni = xf ? (f == 0 ? i + 1 : i - 1) : i;
        const int nj = xf ? j : (f == 2 ? j + 1 : j - 1);
        if (ni < 0 || ni >= d.nx || nj < 0 || nj >= d.ny) continue;   // boundary face: eps = 0
        const long long nb = d.at(ni, nj);
        const bool meL = f == 0 || f == 2;
        const long long L = meL ? C : nb, R = meL ? nb : C;
        const double* NU = tr(a, d, xf ? T_NUX : T_NUY);
        int arg;
        const double eps = eps_and_arg(H, NU, L, R, hdry, kap, emax, arg);
        double epsb = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double* q = Q + (long long)k * d.N;
            const double* ad = AD + (long long)k * d.N;
            epsb += (ad[L] - ad[R]) * (q[R] - q[L]);
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
__device__ __forceinline__ double switch_dbar(const double* E, const double* R, const double* NUB,
                                              long long Xm, long long X, long long Xp,
                                              double& absd_t) {
    const double dd = (E[Xp] - E[X]) - (E[X] - E[Xm]);
    const double t = 0.25 * NUB[X];
    absd_t = t * __builtin_fabs(dd);
    const double absb = t * R[X];
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
    const double* AUS = wk(a, d, W_AUS);
    const CellBar cb = gather_faces(a, d, i, j, T_UN, T_H, a.sigma, AUS, AUS + d.N,
                                    AUS + 2 * d.N, a.rx, a.ry);
    double* AUN = wk(a, d, W_AUN);
    double eb = cb.e, qxb = cb.qx, qyb = cb.qy;
    if (in) {
        eb += AUN[C] + AUS[C];
        qxb += AUN[d.N + C] + AUS[d.N + C];
        qyb += AUN[2 * d.N + C] + AUS[2 * d.N + C];
    }
    // S3: nu = 0.25*(|d| r) at interior cells X; d reaches X-1, X, X+1
    const double* E = tr(a, d, T_UN);
    const double* R = tr(a, d, T_R);
    double rb = cb.u * tr(a, d, T_UN + 1)[C] + cb.v * tr(a, d, T_UN + 2)[C];
    for (int dirn = 0; dirn < 2; ++dirn) {
        const double* NUB = wk(a, d, dirn == 0 ? W_ANX : W_ANY);
        for (int o = -1; o <= 1; ++o) {
            const int xi = dirn == 0 ? i + o : i, xj = dirn == 0 ? j : j + o;
            if (!d.interior(xi, xj)) continue;
            const long long X = d.at(xi, xj);
            const long long Xm = dirn == 0 ? d.at(xi - 1, xj) : d.at(xi, xj - 1);
            const long long Xp = dirn == 0 ? d.at(xi + 1, xj) : d.at(xi, xj + 1);
            double absd_t;
            const double db = switch_dbar(E, R, NUB, Xm, X, Xp, absd_t);
            if (o == 0) {
                eb += -db - db;
                rb += absd_t;
            } else {
                eb += db;
            }
        }
    }
    // S2: h = eta - zp, r = wet ? 1/h : 0, u = qx r, v = qy r
    const double h = tr(a, d, T_H)[C], r = R[C];
    qxb += cb.u * r;
    qyb += cb.v * r;
    const double hb = cb.h + (h > a.P.h_dry ? -(rb * r) / h : 0.0);
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
    double* AUN = wk(a, d, W_AUN);
    fold_ring(a, AUN, d, i, j);
    double* LAM = wk(a, d, W_LAM);
    LAM[C] = AUN[C];
    LAM[d.N + C] = AUN[d.N + C];
    LAM[2 * d.N + C] = AUN[2 * d.N + C];
    double* AZP = wk(a, d, W_AZP);
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

inline dim3 grid2(int w, int h) { return dim3((w + kBX - 1) / kBX, (h + kBY - 1) / kBY); }

}  // namespace

int adjoint_work_arrays() { return 20; }

hipError_t launch_adjoint_step(const AdjointArgs& a, const long long* cells, int ngauge,
                               const double* hobs, hipStream_t s) {
    const int nx = a.P.nx, ny = a.P.ny;
    const dim3 b2(kBX, kBY);
    if (ngauge > 0 && hobs)
        hipLaunchKernelGGL(k_adj_seed, dim3((ngauge + 255) / 256), dim3(256), 0, s, a, cells,
                           ngauge, hobs);
    hipLaunchKernelGGL(k_adj_a, grid2(nx, ny), b2, 0, s, a);
    hipLaunchKernelGGL(k_adj_c, grid2(nx + 2, ny + 2), b2, 0, s, a);
    hipLaunchKernelGGL(k_adj_d, grid2(nx, ny), b2, 0, s, a);
    hipLaunchKernelGGL(k_adj_e1, grid2(nx, ny), b2, 0, s, a);
    hipLaunchKernelGGL(k_adj_e2, grid2(nx + 2, ny + 2), b2, 0, s, a);
    hipLaunchKernelGGL(k_adj_f, grid2(nx, ny), b2, 0, s, a);
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
