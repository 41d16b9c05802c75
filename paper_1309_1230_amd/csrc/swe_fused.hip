// swe_fused.hip -- one kernel per time step: all sixteen sub-steps of the
// MacCormack step fused on a register-resident tile.
//
// Design for gfx950.  The paper's shared-memory version staged 16x16 tiles
// plus a halo in shared memory and still launched one kernel per sub-step
// (§3.2); here a whole step is one launch.  A workgroup is one 64-lane wave
// that owns a strip of 64 consecutive columns (60 output columns plus a halo
// of two on each side: the dissipation switch reaches two cells, the
// MacCormack pair one) and marches up the rows of a chunk of `H` output rows.
// Each iteration ingests one row of U^n (eta, qx, qy, z); the y neighbours of
// every sub-step are earlier rows held in the lane's own registers, and the x
// neighbours are exchanged between adjacent lanes of the wave, so no LDS
// barrier is ever needed.  The output row trails the ingested row by two:
//   row R     : S2 PRIM, S3 switch in x, S4 dissipation in x, S5 x fluxes
//   row R-1   : S3 switch in y, S6 y face R-1/2 -> S7 predictor U*, S9 PRIM*,
//               S10 x fluxes of U*
//   row R-2   : S4 dissipation in y, S11 y face of U*, S12 corrector, S13,
//               S14 friction, S15 dry fix, S16 CFL/volume partials, store.
// HBM traffic per cell update is the algorithmic minimum plus halo re-reads:
// read eta, qx, qy, z, m and write eta, qx, qy (8 words).  Boundary faces are
// evaluated from the face rules directly (no ghost ring in memory): ghost
// columns/rows read the adjacent cell, and wall, open and inflow faces take
// their fluxes from the rules.  dt lives on the device: the block that
// finishes last (ticket counter) reduces the per-block partials in a fixed
// order and writes dt^{n+1}.
#include "swe_common.hpp"
#include "swe_internal.hpp"

namespace swe {

constexpr int kOutW = kWave - 4;   // output columns per strip

__device__ __forceinline__ float sh_dn(float x) { return __shfl_down(x, 1, kWave); }
__device__ __forceinline__ double sh_dn(double x) { return __shfl_down(x, 1, kWave); }
__device__ __forceinline__ float sh_up(float x) { return __shfl_up(x, 1, kWave); }
__device__ __forceinline__ double sh_up(double x) { return __shfl_up(x, 1, kWave); }

// Workgroup id -> tile id so that each XCD (workgroups are dealt round-robin
// over the 8 XCDs) receives one contiguous run of tiles: vertically adjacent
// chunks of a strip, and neighbouring strips, then share an L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int per = nb / 8, rem = nb % 8;
    const int xcd = b % 8, loc = b / 8;
    return xcd < rem ? xcd * (per + 1) + loc : rem * (per + 1) + (xcd - rem) * per + loc;
}

template <typename T>
struct XDiv { T m, x, y; };     // x part of the flux divergence (pressure included)
template <typename T>
struct YFace { T m, x, y, p; }; // fluxes through one y face

template <typename T, int SIG>
__global__ void __launch_bounds__(kWave)
k_fused_step(FusedArgs<T> A) {
    Ctl* ctl = A.ctl;
    if (step_is_noop(ctl, A.t_end)) return;
    const Params& P = A.P;
    const T rx = T(ctl->rx), ry = T(ctl->ry), dt = T(ctl->dt);
    const T qin0 = T(ctl->qin0), qin1 = T(ctl->qin1);
    const T hdry = T(P.h_dry), g = T(P.g), kap = T(P.kappa), emax = T(P.eps_max);
    const T idx = T(P.idx), idy = T(P.idy);
    const int nx = P.nx, ny = P.ny;
    const long long pitch = P.pitch;

    const int lane = threadIdx.x;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int strip = tile / A.gy, chunk = tile - strip * A.gy;
    const int x0 = strip * kOutW, y0 = chunk * A.H;
    const int yEnd = min(y0 + A.H, ny);
    const int i = x0 - 2 + lane;
    const int ic = min(max(i, 0), nx - 1);
    const bool colOut = lane >= 2 && lane < 2 + kOutW && i < nx;
    const bool faceE_interior = i >= 0 && i <= nx - 2;   // face i+1/2 is interior
    const int kS = face_kind(P, EDGE_S, ic), kN = face_kind(P, EDGE_N, ic);

    const T* __restrict__ eta = A.eta;
    const T* __restrict__ qx = A.qx;
    const T* __restrict__ qy = A.qy;
    const T* __restrict__ zb = A.z;
    const T* __restrict__ mm = A.m;

    // Kind of the W and E faces of row j (only used by the lanes at i == 0 and
    // i == nx-1).
    auto kindW = [&](int j) { return face_kind(P, EDGE_W, min(max(j, 0), ny - 1)); };
    auto kindE = [&](int j) { return face_kind(P, EDGE_E, min(max(j, 0), ny - 1)); };

    // x part of the flux divergence of one row (S5 / S10 and the x pressure
    // of S7 / S12), donor direction dir, inflow discharge qin.
    auto xdiv = [&](int dir, T e, T q_n, T h, T r, T u, T v, T z, T qin, int kW, int kE) {
        const T fm = h > hdry ? q_n : T(0);
        const T fx = fm * u, fy = fm * v;
        T FmE, FxE, FyE, FmW, FxW, FyW, Ps;
        if (dir > 0) {
            FmE = sh_dn(fm); FxE = sh_dn(fx); FyE = sh_dn(fy);
            FmW = fm; FxW = fx; FyW = fy;
            const T eR = sh_dn(e), hR = sh_dn(h), zR = sh_dn(z);
            Ps = face_pressure(e, h, z, eR, hR, zR, hdry, g);
        } else {
            FmE = fm; FxE = fx; FyE = fy;
            FmW = sh_up(fm); FxW = sh_up(fx); FyW = sh_up(fy);
            const T eL = sh_up(e), hL = sh_up(h), zL = sh_up(z);
            Ps = face_pressure(eL, hL, zL, e, h, z, hdry, g);
        }
        if (i == nx - 1) {
            boundary_flux(kE, true, fm, fx, fy, -qin, r, FmE, FxE, FyE);
            if (dir > 0) Ps = T(0);
        }
        if (i == 0) {
            boundary_flux(kW, true, fm, fx, fy, qin, r, FmW, FxW, FyW);
            if (dir < 0) Ps = T(0);
        }
        XDiv<T> d;
        d.m = FmE - FmW;
        d.x = (FxE - FxW) + Ps;
        d.y = FyE - FyW;
        return d;
    };

    // Fluxes through the y face j+1/2 between a lower cell S (row j) and an
    // upper cell N (row j+1), donor direction dir (S6 / S11).
    auto yface = [&](int j, int dir, T eS, T qS, T hS, T rS, T uS, T vS, T zS, T eN, T qN, T hN,
                     T rN, T uN, T vN, T zN, T qin) {
        YFace<T> f;
        if (j == -1 || j == ny - 1) {
            // boundary face: the adjacent interior cell is N for the south
            // face and S for the north face
            const bool south = j == -1;
            const T qa = south ? qN : qS, ha = south ? hN : hS, ra = south ? rN : rS;
            const T ua = south ? uN : uS, va = south ? vN : vS;
            const T fm = ha > hdry ? qa : T(0);
            boundary_flux(south ? kS : kN, false, fm, fm * ua, fm * va, south ? qin : -qin, ra,
                          f.m, f.x, f.y);
            f.p = T(0);
        } else {
            const T qd = dir > 0 ? qN : qS, hd = dir > 0 ? hN : hS;
            const T ud = dir > 0 ? uN : uS, vd = dir > 0 ? vN : vS;
            const T fm = hd > hdry ? qd : T(0);
            f.m = fm;
            f.x = fm * ud;
            f.y = fm * vd;
            f.p = face_pressure(eS, hS, zS, eN, hN, zN, hdry, g);
        }
        return f;
    };

    // ---- carried state (rows relative to the ingested row R)
    T e1 = 0, a1 = 0, b1 = 0, z1 = 0, h1 = 0, r1 = 0, u1 = 0, v1 = 0;  // U^n row R-1
    T e2 = 0, a2 = 0, b2 = 0, z2 = 0, h2 = 0;                           // U^n row R-2
    T nuy2 = 0;                      // nu_y(R-2)
    T dx1m = 0, dx1a = 0, dx1b = 0;  // x dissipation of row R-1
    T dx2m = 0, dx2a = 0, dx2b = 0;  // x dissipation of row R-2
    T phm = 0, pha = 0, phb = 0;     // y dissipation flux through face (R-3)+1/2
    XDiv<T> A1 = {0, 0, 0};          // predictor x part of row R-1
    YFace<T> G1 = {0, 0, 0, 0};      // predictor y face (R-2)+1/2
    T se2 = 0, sa2 = 0, sb2 = 0, sh2 = 0, sr2 = 0, su2 = 0, sv2 = 0;  // U* row R-2
    XDiv<T> B2 = {0, 0, 0};          // corrector x part of row R-2
    YFace<T> H1 = {0, 0, 0, 0};      // corrector y face (R-3)+1/2

    double vol = 0.0, def = 0.0;
    T lmax = T(0);
    unsigned flags = 0u;

    // software prefetch of the first ingested row
    auto rowoff = [&](int R) {
        return (long long)min(max(R, 0), ny - 1) * pitch + ic;
    };
    long long off = rowoff(y0 - 2);
    T ne = eta[off], na = qx[off], nb = qy[off], nz = zb[off];
    T nm = T(0);

    for (int R = y0 - 2; R <= yEnd + 1; ++R) {
        const T e0 = ne, a0 = na, b0 = nb, z0 = nz;
        const T m2 = nm;                    // m of row R-2
        {
            const long long o = rowoff(R + 1);
            ne = eta[o]; na = qx[o]; nb = qy[o]; nz = zb[o];
            nm = mm[rowoff(R - 1)];
        }
        // ---- S2 on row R
        const T h0 = e0 - z0;
        const T r0 = recip_depth(h0, hdry);
        const T u0 = a0 * r0, v0 = b0 * r0;

        // ---- S3/S4 in x on row R
        const T eE = sh_dn(e0), eW = sh_up(e0);
        const T nux0 = curv_switch(eW, e0, eE, r0);
        const T nuxE = sh_dn(nux0), hE = sh_dn(h0);
        const T aE = sh_dn(a0), bE = sh_dn(b0);
        const T epsE = faceE_interior ? face_eps(h0, hE, nux0, nuxE, hdry, kap, emax) : T(0);
        const T fxm = epsE * (eE - e0), fxa = epsE * (aE - a0), fxb = epsE * (bE - b0);
        const T dx0m = fxm - sh_up(fxm), dx0a = fxa - sh_up(fxa), dx0b = fxb - sh_up(fxb);

        // ---- S5 (+ x pressure of S7) on row R
        const XDiv<T> A0 = xdiv(SIG, e0, a0, h0, r0, u0, v0, z0, qin0, kindW(R), kindE(R));

        // ---- S3 in y at row R-1, S4 in y through face (R-2)+1/2
        const T nuy1 = curv_switch(e2, e1, e0, r1);
        const int jf = R - 2;   // face between rows R-2 and R-1
        const T epsN = (jf >= 0 && jf <= ny - 2) ? face_eps(h2, h1, nuy2, nuy1, hdry, kap, emax)
                                                 : T(0);
        const T pnm = epsN * (e1 - e2), pna = epsN * (a1 - a2), pnb = epsN * (b1 - b2);
        const T Dm = dx2m + (pnm - phm), Da = dx2a + (pna - pha), Db = dx2b + (pnb - phb);

        // ---- S6 through face (R-1)+1/2, S7 predictor of row R-1
        const YFace<T> G0 = yface(R - 1, SIG, e1, b1, h1, r1, u1, v1, z1, e0, b0, h0, r0, u0, v0,
                                  z0, qin0);
        const T pys = SIG > 0 ? G0.p : G1.p;
        const T se1 = (e1 - rx * A1.m) - ry * (G0.m - G1.m);
        const T sa1 = (a1 - rx * A1.x) - ry * (G0.x - G1.x);
        const T sb1 = (b1 - rx * A1.y) - ry * ((G0.y - G1.y) + pys);

        // ---- S9 on U*(R-1), S10 on U*(R-1)
        const T sh1 = se1 - z1;
        const T sr1 = recip_depth(sh1, hdry);
        const T su1 = sa1 * sr1, sv1 = sb1 * sr1;
        const XDiv<T> B1 = xdiv(-SIG, se1, sa1, sh1, sr1, su1, sv1, z1, qin1, kindW(R - 1),
                                kindE(R - 1));

        // ---- S11 through face (R-2)+1/2, S12 corrector of row R-2
        const YFace<T> H0 = yface(R - 2, -SIG, se2, sb2, sh2, sr2, su2, sv2, z2, se1, sb1, sh1,
                                  sr1, su1, sv1, z1, qin1);
        const T pcs = -SIG > 0 ? H0.p : H1.p;
        const T ce = T(0.5) * (e2 + ((se2 - rx * B2.m) - ry * (H0.m - H1.m)));
        const T ca = T(0.5) * (a2 + ((sa2 - rx * B2.x) - ry * (H0.x - H1.x)));
        const T cb = T(0.5) * (b2 + ((sb2 - rx * B2.y) - ry * ((H0.y - H1.y) + pcs)));

        // ---- S13 .. S16 on row R-2
        const int jo = R - 2;
        if (jo >= y0 && jo < yEnd && colOut) {
            T e = ce + Dm, a = ca + Da, b = cb + Db;
            T h = e - z2;
            T r = T(0);
            if (h > hdry) {
                r = T(1) / h;
                manning(dt, m2, r, a, b);
            }
            if (h < T(0)) {
                def = def + (0.0 - (double)h);
                e = z2;
                flags |= FLAG_CLIPPED;
            }
            h = e - z2;
            if (!(h > hdry)) {
                a = T(0);
                b = T(0);
            } else {
                lmax = lam_acc(lmax, cfl_lambda(h, r, a, b, g, idx, idy));
            }
            if (!tfinite(e) || !tfinite(a) || !tfinite(b)) flags |= FLAG_NAN;
            vol = vol + (double)h;
            const long long so = (long long)jo * pitch + i;
            A.eta1[so] = e;
            A.qx1[so] = a;
            A.qy1[so] = b;
        }

        // ---- rotate the carried rows
        e2 = e1; a2 = a1; b2 = b1; z2 = z1; h2 = h1;
        e1 = e0; a1 = a0; b1 = b0; z1 = z0; h1 = h0; r1 = r0; u1 = u0; v1 = v0;
        nuy2 = nuy1;
        dx2m = dx1m; dx2a = dx1a; dx2b = dx1b;
        dx1m = dx0m; dx1a = dx0a; dx1b = dx0b;
        phm = pnm; pha = pna; phb = pnb;
        A1 = A0;
        G1 = G0;
        se2 = se1; sa2 = sa1; sb2 = sb1; sh2 = sh1; sr2 = sr1; su2 = su1; sv2 = sv1;
        B2 = B1;
        H1 = H0;
    }

    // ---- block partials, then the last block finalises the step
    vol = wave_sum(vol);
    def = wave_sum(def);
    const unsigned long long lb = wave_max_u64(lam_to_bits(lmax));
    flags = wave_or(flags);
    publish_partial(ctl, A.part_def, A.part_vol, tile, lb, flags, def, vol);
    __threadfence();
    unsigned ticket = 0;
    if (lane == 0) ticket = atomicAdd(&ctl->ticket, 1u);
    ticket = __shfl(ticket, 0, kWave);
    if (ticket == gridDim.x - 1) {
        __threadfence();
        finalize_wave(ctl, P, A.part_def, A.part_vol, gridDim.x, sizeof(T) == 4, 1);
    }
}

template <typename T>
hipError_t launch_fused(const FusedArgs<T>& a, int sigma, hipStream_t s) {
    const int gx = (a.P.nx + kOutW - 1) / kOutW;
    const int nblk = gx * a.gy;
    if (sigma > 0)
        hipLaunchKernelGGL((k_fused_step<T, 1>), dim3(nblk), dim3(kWave), 0, s, a);
    else
        hipLaunchKernelGGL((k_fused_step<T, -1>), dim3(nblk), dim3(kWave), 0, s, a);
    return hipGetLastError();
}

int fused_blocks(int nx, int ny, int H) {
    const int gx = (nx + kOutW - 1) / kOutW;
    const int gy = (ny + H - 1) / H;
    return gx * gy;
}

template hipError_t launch_fused<float>(const FusedArgs<float>&, int, hipStream_t);
template hipError_t launch_fused<double>(const FusedArgs<double>&, int, hipStream_t);

}  // namespace swe
