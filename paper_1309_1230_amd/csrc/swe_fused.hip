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
// neighbours come from the adjacent lanes through DPP wavefront shifts (one
// VALU move per 32 bits, no LDS traffic and no barrier).  The output row
// trails the ingested row R by two:
//   row R     : S2 PRIM, S3 switch in x, S4 dissipation in x, S5 x fluxes
//   row R-1   : S3 switch in y, S6 y face R-1/2 -> S7 predictor U*, S9 PRIM*,
//               S10 x fluxes of U*
//   row R-2   : S4 dissipation in y, S11 y face of U*, S12 corrector, S13,
//               S14 friction, S15 dry fix, S16 CFL/volume partials, store.
// HBM traffic per cell update is the algorithmic minimum plus halo re-reads:
// read eta, qx, qy, z, m and write eta, qx, qy (8 words).  Boundary faces are
// evaluated from the face rules directly (no ghost ring in memory): ghost
// columns/rows read the adjacent cell, and wall, open and inflow faces take
// their fluxes from the rules; only strips that touch the west or east edge
// execute that code.  dt lives on the device: per-workgroup records are
// reduced through a two-level ticket (groups of 64 tiles, then the groups)
// in a fixed order, and the last workgroup writes dt^{n+1}; no device-wide
// fence is taken, since on gfx950 such a fence writes back and invalidates
// the whole L2 of the XCD.
#include "swe_common.hpp"
#include "swe_internal.hpp"

namespace swe {

constexpr int kOutW = kWave - 4;   // output columns per strip

__device__ __forceinline__ bool is_neg_zero(float x) { return __float_as_uint(x) == 0x80000000u; }
__device__ __forceinline__ bool is_neg_zero(double x) {
    return (unsigned long long)__double_as_longlong(x) == 0x8000000000000000ull;
}

// Dry-tile skip.  A cell whose neighbourhood of radius two is dry, finite,
// without discharge and away from the domain edge maps to itself under the
// step: every donor flux is zero (dry donor), the dissipation coefficient of
// every face vanishes (dry sides), so U* has the cell's eta and the corrector
// returns 0.5*(eta + eta) = eta; a pressure term can make the momentum of U*
// non-zero but the dry-cell rule of S15 clears it again.  The dissipation sum
// is a signed zero, which leaves eta unchanged unless eta is -0 itself, so a
// cell with eta = -0 does not count as dry here.  Tile flag words, one per
// tile and step parity:
constexpr unsigned kDryStill = 1u;    // after the step every output cell is dry
                                      // (h <= h_dry), finite and not eta = -0
constexpr unsigned kDrySkipped = 2u;  // the step skipped the tile

template <typename T>
struct XDiv { T m, x, y; };     // x part of the flux divergence (pressure included)
template <typename T>
struct YFace { T m, x, y, p; }; // fluxes through one y face

// Per-wave constants of one step.
template <typename T>
struct Consts {
    T rx, ry, dt, qin0, qin1, hdry, hg, g, kap, emax, idx, idy, rcap;
};

// Override the fluxes of the west (i == 0) or east (i == nx-1) boundary face
// with the face rules; (fm, fx, fy) are the adjacent cell's donor fluxes.
template <typename T>
__device__ __forceinline__ void x_boundary(bool at, int kind, T fm, T fx, T fy, T qs, T r, T& Fm,
                                           T& Fx, T& Fy) {
    T bm, bx, by;
    boundary_flux(kind, true, fm, fx, fy, qs, r, bm, bx, by);
    Fm = at ? bm : Fm;
    Fx = at ? bx : Fx;
    Fy = at ? by : Fy;
}

// x part of the flux divergence of one row (S5 / S10 and the x pressure of
// S7 / S12), donor direction DIR.  eN/hN/zN are the neighbour on the DIR
// side (east for DIR > 0, west otherwise), already shifted in.
template <typename T, int DIR>
__device__ __forceinline__ XDiv<T> x_divergence(const Consts<T>& c, T e, T q, T h, T r, T u, T v,
                                                T z, T eN, T hN, T zN, T qin, bool edge, bool atW,
                                                bool atE, int kW, int kE) {
    const T fm = h > c.hdry ? q : T(0);
    const T fx = fm * u, fy = fm * v;
    T FmE, FxE, FyE, FmW, FxW, FyW, Ps;
    if (DIR > 0) {
        FmE = from_east(fm); FxE = from_east(fx); FyE = from_east(fy);
        FmW = fm; FxW = fx; FyW = fy;
        Ps = face_pressure(e, h, z, eN, hN, zN, c.hdry, c.hg);
    } else {
        FmE = fm; FxE = fx; FyE = fy;
        FmW = from_west(fm); FxW = from_west(fx); FyW = from_west(fy);
        Ps = face_pressure(eN, hN, zN, e, h, z, c.hdry, c.hg);
    }
    if (edge) {   // uniform: this strip contains the west or the east edge
        x_boundary(atE, kE, fm, fx, fy, -qin, r, FmE, FxE, FyE);
        x_boundary(atW, kW, fm, fx, fy, qin, r, FmW, FxW, FyW);
        Ps = ((DIR > 0 && atE) || (DIR < 0 && atW)) ? T(0) : Ps;
    }
    XDiv<T> d;
    d.m = FmE - FmW;
    d.x = (FxE - FxW) + Ps;
    d.y = FyE - FyW;
    return d;
}

// Fluxes through the y face j+1/2 between a lower cell S (row j) and an upper
// cell N (row j+1), donor direction DIR (S6 / S11).  `bnd` is uniform: the
// face is the south (j == -1) or north (j == ny-1) boundary face.
template <typename T, int DIR>
__device__ __forceinline__ YFace<T> y_face(const Consts<T>& c, bool bnd, bool south, int kS,
                                           int kN, T eS, T qS, T hS, T rS, T uS, T vS, T zS, T eN,
                                           T qN, T hN, T rN, T uN, T vN, T zN, T qin) {
    YFace<T> f;
    if (!bnd) {
        const T qd = DIR > 0 ? qN : qS, hd = DIR > 0 ? hN : hS;
        const T ud = DIR > 0 ? uN : uS, vd = DIR > 0 ? vN : vS;
        const T fm = hd > c.hdry ? qd : T(0);
        f.m = fm;
        f.x = fm * ud;
        f.y = fm * vd;
        f.p = face_pressure(eS, hS, zS, eN, hN, zN, c.hdry, c.hg);
    } else {
        // the adjacent interior cell is N for the south face, S for the north
        const T qa = south ? qN : qS, ha = south ? hN : hS, ra = south ? rN : rS;
        const T ua = south ? uN : uS, va = south ? vN : vS;
        const T fm = ha > c.hdry ? qa : T(0);
        boundary_flux(south ? kS : kN, false, fm, fm * ua, fm * va, south ? qin : -qin, ra, f.m,
                      f.x, f.y);
        f.p = T(0);
    }
    return f;
}

// State of one wave's march up its chunk: per-lane constants, the rows and
// faces carried from one iteration to the next, the prefetched row and the
// running partial sums.  Rows are named relative to the ingested row R.
// The two-wave form of the march: values per row of its LDS ring, and rows
// of the ring: 3 in FP64 (23 KB a tile, 6 tiles per compute unit); 6 in the
// dense FP32 step (20 KB: 8 tiles, so 4 waves per SIMD where registers would
// allow 5, and the first wave may run 5 rows ahead: 156 against 160 us at
// 4096^2), 3 with the dry-tile skip (its short tiles run 88 against 82 us
// with 6).
constexpr int kSplitFields = 13;
template <typename T, bool DRY>
constexpr int split_slots() { return sizeof(T) == 4 && !DRY ? 6 : 3; }

template <typename T, int SIG, bool DRY, bool TRACE = false, int PART = 0>
struct March {
    Consts<T> c;
    const Params* P;
    const T* __restrict__ eta;
    const T* __restrict__ qx;
    const T* __restrict__ qy;
    const T* __restrict__ zb;
    const T* __restrict__ mm;
    T* __restrict__ eta1;
    T* __restrict__ qx1;
    T* __restrict__ qy1;
    // TRACE: U* (S7) and U^d (S13, before friction) of the output cells
    T* tus[3];
    T* tud[3];
    long long pitch;
    int nx, ny, i, ic, y0, yEnd, kS, kN;
    bool colOut, faceE_interior, atW, atE;

    // Depths are not carried: h = eta - z is recomputed from the carried
    // eta and z (the same operands, so the same bits) to save registers.
    T e1 = 0, a1 = 0, b1 = 0, z1 = 0, r1 = 0;   // U^n row R-1
    T e2 = 0, a2 = 0, b2 = 0, z2 = 0, r2 = 0;   // U^n row R-2
    T nuy2 = 0;                      // nu_y(R-2)
    T phm = 0, pha = 0, phb = 0;     // y dissipation flux through face (R-3)+1/2
    XDiv<T> A1 = {0, 0, 0};          // predictor x part of row R-1
    YFace<T> G1 = {0, 0, 0, 0};      // predictor y face (R-2)+1/2
    T se2 = 0, sa2 = 0, sb2 = 0, sr2 = 0;  // U* row R-2
    XDiv<T> B2 = {0, 0, 0};          // corrector x part of row R-2
    YFace<T> H1 = {0, 0, 0, 0};      // corrector y face (R-3)+1/2
    // Prefetched rows, double-buffered: the iteration that consumes slot S
    // loads the next row into slot 1-S, so a loaded register is read by the
    // next iteration directly and no copy (which would have to wait for the
    // load) sits on the loop's back edge.
    T pe[2] = {0, 0}, pa[2] = {0, 0}, pb[2] = {0, 0}, pz[2] = {0, 0}, pm[2] = {0, 0};

    double vol = 0.0, def = 0.0;
    T lmax = T(0);
    unsigned flags = 0u;
    bool dirty = false;   // an output cell is wet, not finite, or has eta = -0 (DRY only)

    // PART 1 and 2 (two waves of one workgroup): the first wave runs the
    // predictor half of each iteration (S2..S7), the second the corrector
    // half (S9..S16 and the stores) from the values the first files in an
    // LDS ring of split_slots<T, DRY>() rows (kSplitFields values per lane and row).
    // Two progress counters order them (prog[0]: the last row the first wave
    // filed, prog[1]: the last row the second has taken), so the first may
    // run split_slots<T, DRY>() - 1 rows ahead.  Every wait is bounded; a wave whose
    // wait runs out stops waiting and the step raises FLAG_STALL.
    T* ring = nullptr;
    int* prog = nullptr;
    int* note = nullptr;   // the first wave's stall, for the second wave's record
    int lane = 0;
    int spin_cap = 0;
    bool stalled = false;
    __device__ __forceinline__ T& rg(int f, int R) const {
        constexpr int NS = split_slots<T, DRY>();
        return ring[(f * NS + (R + NS) % NS) * kWave + lane];
    }
    __device__ __forceinline__ void wait_row(int who, int need) {
        if (stalled) return;
        for (int n = 0;; ++n) {
            const int v = __builtin_amdgcn_readfirstlane(__hip_atomic_load(
                prog + who, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP));
            if (v >= need) return;
            if (n >= spin_cap) {
                stalled = true;
                // noted before any later row is posted, so the second wave's
                // acquire of that row sees it
                if (PART == 1 && lane == 0)
                    __hip_atomic_store(note, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                return;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    __device__ __forceinline__ void post_row(int who, int R) {
        __hip_atomic_store(prog + who, R, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    }

    __device__ __forceinline__ long long rowoff(int R) const {
        return (long long)min(max(R, 0), ny - 1) * pitch + ic;
    }

    template <int S>
    __device__ __forceinline__ void prefetch(int R) {
        const long long o = rowoff(R);
        pe[S] = eta[o]; pa[S] = qx[o]; pb[S] = qy[o]; pz[S] = zb[o];
    }

    // One iteration of the march, ingesting row R from prefetch slot SLOT.
    // EDGE: the strip holds the west or east edge; BND: a y face of this
    // iteration may be a boundary face (otherwise 2 <= R <= ny-2), and then
    // `out` says whether row R-2 is an output row of the chunk (always so
    // when !BND).
    template <bool EDGE, bool BND, int SLOT>
    __device__ __forceinline__ void iter(int R, bool out) {
        // the predictor half's values the corrector half reads: U* of row
        // R-1, the bed of rows R-1 and R-2, U^n, 1/h and m of row R-2 and the
        // y dissipation flux through face (R-2)+1/2
        T se1, sa1, sb1, z1x, z2x, e2x, a2x, b2x, r2x, m2x, pnm, pna, pnb;
        if constexpr (PART != 2) {
            const T e0 = pe[SLOT], a0 = pa[SLOT], b0 = pb[SLOT], z0 = pz[SLOT];
            const T m2 = pm[SLOT];              // m of row R-2
            prefetch<1 - SLOT>(R + 1);
            pm[1 - SLOT] = mm[rowoff(R - 1)];
            int kW0 = BC_WALL, kE0 = BC_WALL;
            if (EDGE) {
                const int Rc = min(max(R, 0), ny - 1);
                kW0 = face_kind(*P, EDGE_W, Rc); kE0 = face_kind(*P, EDGE_E, Rc);
            }

            // ---- S2 on row R
            const T h0 = e0 - z0;
            const T r0 = recip_prim(h0, c.hdry, c.rcap);
            const T u0 = a0 * r0, v0 = b0 * r0;

            // ---- S5 (+ x pressure of S7) on row R (S3/S4 in x on this row
            // follow in the corrector half, two iterations later)
            const T eE = from_east(e0), eW = from_west(e0);
            const T hE = from_east(h0);
            XDiv<T> A0;
            if (SIG > 0)
                A0 = x_divergence<T, 1>(c, e0, a0, h0, r0, u0, v0, z0, eE, hE, from_east(z0), c.qin0,
                                        EDGE, atW, atE, kW0, kE0);
            else
                A0 = x_divergence<T, -1>(c, e0, a0, h0, r0, u0, v0, z0, eW, from_west(h0),
                                         from_west(z0), c.qin0, EDGE, atW, atE, kW0, kE0);

            // ---- S3 in y at row R-1, S4 in y through face (R-2)+1/2
            const T nuy1 = curv_switch(e2, e1, e0, r1);
            const bool fInt = !BND || (R - 2 >= 0 && R - 2 <= ny - 2);
            const T h1 = e1 - z1, h2 = e2 - z2;
            const T epsN = fInt ? face_eps(h2, h1, nuy2, nuy1, c.hdry, c.kap, c.emax) : T(0);
            pnm = epsN * (e1 - e2); pna = epsN * (a1 - a2); pnb = epsN * (b1 - b2);

            // ---- S6 through face (R-1)+1/2, S7 predictor of row R-1
            const bool bndG = BND && ((R - 1 == -1) || (R - 1 == ny - 1));
            const YFace<T> G0 = y_face<T, SIG>(c, bndG, R - 1 == -1, kS, kN, e1, b1, h1, r1,
                                               a1 * r1, b1 * r1, z1, e0, b0, h0, r0, u0, v0, z0,
                                               c.qin0);
            const T pys = SIG > 0 ? G0.p : G1.p;
            se1 = (e1 - c.rx * A1.m) - c.ry * (G0.m - G1.m);
            sa1 = (a1 - c.rx * A1.x) - c.ry * (G0.x - G1.x);
            sb1 = (b1 - c.rx * A1.y) - c.ry * ((G0.y - G1.y) + pys);
            z1x = z1; z2x = z2; e2x = e2; a2x = a2; b2x = b2; r2x = r2; m2x = m2;

            // ---- rotate the predictor half's carried rows
            e2 = e1; a2 = a1; b2 = b1; z2 = z1; r2 = r1;
            e1 = e0; a1 = a0; b1 = b0; z1 = z0; r1 = r0;
            nuy2 = nuy1;
            A1 = A0;
            G1 = G0;
        }
        if constexpr (PART == 1) {
            // file row R once the second wave has taken the slot's last row
            wait_row(1, R - split_slots<T, DRY>());
            rg(0, R) = se1; rg(1, R) = sa1; rg(2, R) = sb1; rg(3, R) = z1x; rg(4, R) = z2x;
            rg(5, R) = e2x; rg(6, R) = a2x; rg(7, R) = b2x; rg(8, R) = r2x; rg(9, R) = m2x;
            rg(10, R) = pnm; rg(11, R) = pna; rg(12, R) = pnb;
            post_row(0, R);
            return;
        }
        if constexpr (PART == 2) {
            wait_row(0, R);
            se1 = rg(0, R); sa1 = rg(1, R); sb1 = rg(2, R); z1x = rg(3, R); z2x = rg(4, R);
            e2x = rg(5, R); a2x = rg(6, R); b2x = rg(7, R); r2x = rg(8, R); m2x = rg(9, R);
            pnm = rg(10, R); pna = rg(11, R); pnb = rg(12, R);
            post_row(1, R);
        }
        int kW1 = BC_WALL, kE1 = BC_WALL;
        if (EDGE) {
            const int R1c = min(max(R - 1, 0), ny - 1);
            kW1 = face_kind(*P, EDGE_W, R1c); kE1 = face_kind(*P, EDGE_E, R1c);
        }

        // ---- S9 on U*(R-1), S10 on U*(R-1)
        const T sh1 = se1 - z1x;
        const T sr1 = recip_prim(sh1, c.hdry, c.rcap);
        const T su1 = sa1 * sr1, sv1 = sb1 * sr1;
        if (TRACE && colOut && R - 1 >= y0 && R - 1 < yEnd) {
            const long long so = (long long)(R - 1) * pitch + i;
            tus[0][so] = se1;
            tus[1][so] = sa1;
            tus[2][so] = sb1;
        }
        XDiv<T> B1;
        if (SIG > 0)   // corrector donor direction -1: neighbour on the west
            B1 = x_divergence<T, -1>(c, se1, sa1, sh1, sr1, su1, sv1, z1x, from_west(se1),
                                     from_west(sh1), from_west(z1x), c.qin1, EDGE, atW, atE, kW1,
                                     kE1);
        else
            B1 = x_divergence<T, 1>(c, se1, sa1, sh1, sr1, su1, sv1, z1x, from_east(se1),
                                    from_east(sh1), from_east(z1x), c.qin1, EDGE, atW, atE, kW1,
                                    kE1);

        // ---- S11 through face (R-2)+1/2
        const bool bndH = BND && ((R - 2 == -1) || (R - 2 == ny - 1));
        const T sh2 = se2 - z2x;
        const YFace<T> H0 = y_face<T, -SIG>(c, bndH, R - 2 == -1, kS, kN, se2, sb2, sh2, sr2,
                                            sa2 * sr2, sb2 * sr2, z2x, se1, sb1, sh1, sr1, su1, sv1,
                                            z1x, c.qin1);

        if (!BND || out) {
            // ---- S3/S4 in x on row R-2 (every lane active: the shifts read
            // the neighbouring lanes)
            const T eE2 = from_east(e2x), eW2 = from_west(e2x);
            const T h2x = e2x - z2x;
            const T hE2 = from_east(h2x);
            const T nux2 = curv_switch(eW2, e2x, eE2, r2x);
            const T nuxE2 = from_east(nux2);
            const T epsE = faceE_interior ? face_eps(h2x, hE2, nux2, nuxE2, c.hdry, c.kap, c.emax)
                                          : T(0);
            const T fdm = epsE * (eE2 - e2x);
            const T fda = epsE * (from_east(a2x) - a2x);
            const T fdb = epsE * (from_east(b2x) - b2x);
            const T dxm = fdm - from_west(fdm), dxa = fda - from_west(fda),
                    dxb = fdb - from_west(fdb);

            // ---- S4 total, S12 corrector, S13 .. S16 on row R-2
            const T Dm = dxm + (pnm - phm), Da = dxa + (pna - pha), Db = dxb + (pnb - phb);
            const T pcs = -SIG > 0 ? H0.p : H1.p;
            const T ce = T(0.5) * (e2x + ((se2 - c.rx * B2.m) - c.ry * (H0.m - H1.m)));
            const T ca = T(0.5) * (a2x + ((sa2 - c.rx * B2.x) - c.ry * (H0.x - H1.x)));
            const T cb = T(0.5) * (b2x + ((sb2 - c.rx * B2.y) - c.ry * ((H0.y - H1.y) + pcs)));
            T e = ce + Dm, a = ca + Da, b = cb + Db;
            if (TRACE && colOut) {
                const long long so = (long long)(R - 2) * pitch + i;
                tud[0][so] = e;
                tud[1][so] = a;
                tud[2][so] = b;
            }
            T h = e - z2x;
            T lam = T(0);
            if (h > c.hdry) {
                const T r = trcp(h);
                manning(c.dt, m2x, r, a, b);
                // wet stays wet through S15 (h is unchanged), so S16 uses r
                lam = cfl_lambda(h, r, a, b, c.g, c.idx, c.idy);
            } else {
                if (h < T(0)) {
                    def = def + (colOut ? 0.0 - (double)h : 0.0);
                    e = z2x;
                    flags |= colOut ? FLAG_CLIPPED : 0u;
                    h = e - z2x;
                }
                a = T(0);
                b = T(0);
            }
            if (colOut) {
                lmax = lam_acc(lmax, lam);
                if (!tfinite(e) || !tfinite(a) || !tfinite(b)) flags |= FLAG_NAN;
                vol = vol + (double)h;
                if (DRY) dirty = dirty || !(h <= c.hdry) || !tfinite(e) || is_neg_zero(e);
                const long long so = (long long)(R - 2) * pitch + i;
                eta1[so] = e;
                qx1[so] = a;
                qy1[so] = b;
            }
        }

        // ---- rotate the corrector half's carried rows
        phm = pnm; pha = pna; phb = pnb;
        se2 = se1; sa2 = sa1; sb2 = sb1; sr2 = sr1;
        B2 = B1;
        H1 = H0;
    }

    template <bool EDGE>
    __device__ __forceinline__ void run() {
        if constexpr (PART != 2) prefetch<0>(y0 - 2);
        // rows y0-2 .. y0+1 only fill the pipeline: no output row yet; the
        // iteration at row R reads slot (R - y0) mod 2
        for (int R = y0 - 2; R < y0 + 2; R += 2) {
            iter<EDGE, true, 0>(R, false);
            iter<EDGE, true, 1>(R + 1, false);
        }
        int R = y0 + 2;
        const int lim = min(yEnd + 1, ny - 2);   // rows whose faces are all interior
        for (; R + 1 <= lim; R += 2) {
            iter<EDGE, false, 0>(R, true);
            iter<EDGE, false, 1>(R + 1, true);
        }
        for (; R <= yEnd + 1; R += 2) {
            iter<EDGE, true, 0>(R, true);
            if (R + 1 <= yEnd + 1) iter<EDGE, true, 1>(R + 1, true);
        }
    }
};

// Agent-scope relaxed loads and stores: coherent across the XCDs (their L2
// caches are not), with no cache-wide write-back or invalidation, unlike a
// device-scope fence.
__device__ __forceinline__ void st_agent(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(unsigned long long* p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(unsigned* p, unsigned v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_agent(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_agent(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Wait until every memory access this wave issued has completed (s_waitcnt
// vmcnt(0)): the record stores are then at the coherence point, before the
// ticket increment that announces them.
__device__ __forceinline__ void wait_stores() { __builtin_amdgcn_s_waitcnt(0x0F70); }

__device__ __forceinline__ void put_record(TilePart* r, double def, double vol,
                                           unsigned long long lam, unsigned long long fs) {
    st_agent(&r->def, def);
    st_agent(&r->vol, vol);
    st_agent(&r->lam, lam);
    st_agent(&r->fs, fs);
}

// End of a workgroup's share of a step: a two-level ticket.  The last
// workgroup to finish in each group of kGroup consecutive tiles reduces the
// group's records (one coalesced read, fixed order) into a group record; the
// last group to finish reduces the group records and finalises the step.
// The order of every sum is fixed by the tile numbering, never by the order
// in which workgroups finish, so results are reproducible; and no address
// takes more than kGroup (or number-of-groups) atomics per step.  The
// records travel through agent-scope accesses and the stores are complete
// before each ticket increment, so no device-wide fence is needed (the
// output fields are read only by the next launch).
template <typename T>
__device__ __forceinline__ void finish_step(const FusedArgs<T>& A, int tile, int nblk,
                                            bool lam_is_f32) {
    const int lane = threadIdx.x % kWave;
    const int g = tile / kGroup;
    const int gsize = min(kGroup, nblk - g * kGroup);
    wait_stores();
    unsigned t = 0;
    if (lane == 0) t = atomicAdd(&A.gticket[g], 1u);
    t = __shfl(t, 0, kWave);
    if (t != (unsigned)gsize - 1) return;
    double def = 0.0, vol = 0.0;
    unsigned long long lam = 0ull, fs = 0ull;
    if (lane < gsize) {
        const TilePart* r = A.tpart + g * kGroup + lane;
        def = ld_agent(&r->def);
        vol = ld_agent(&r->vol);
        lam = ld_agent(&r->lam);
        fs = ld_agent(&r->fs);
    }
    const double gdef = wave_sum(def);
    const double gvol = wave_sum(vol);
    const unsigned long long glam = wave_max_u64(lam);
    const unsigned gflags = wave_or((unsigned)fs);
    unsigned gskip = (unsigned)(fs >> 32);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) gskip += __shfl_xor(gskip, off, kWave);
    const int ngroups = (nblk + kGroup - 1) / kGroup;
    if (lane == 0) {
        put_record(A.gpart + g, gdef, gvol, glam,
                   (unsigned long long)gflags | ((unsigned long long)gskip << 32));
        st_agent(&A.gticket[g], 0u);   // every member has counted: ready for the next step
    }
    wait_stores();
    Ctl* ctl = A.ctl;
    unsigned t2 = 0;
    if (lane == 0) t2 = atomicAdd(&ctl->ticket, 1u);
    t2 = __shfl(t2, 0, kWave);
    if (t2 != (unsigned)ngroups - 1) return;
    double sd = 0.0, sv = 0.0;
    unsigned long long lm = 0ull, sk = 0ull;
    unsigned fl = 0u;
    for (int k = lane; k < ngroups; k += kWave) {
        const TilePart* q = A.gpart + k;
        sd = sd + ld_agent(&q->def);
        sv = sv + ld_agent(&q->vol);
        const unsigned long long ql = ld_agent(&q->lam), qf = ld_agent(&q->fs);
        lm = ql > lm ? ql : lm;
        fl |= (unsigned)qf;
        sk += qf >> 32;
    }
    sd = wave_sum(sd);
    sv = wave_sum(sv);
    lm = wave_max_u64(lm);
    fl = wave_or(fl);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) sk += __shfl_xor(sk, off, kWave);
    if (lane == 0) {
        if (A.log_dt) {
            *A.log_dt = ctl->dt;
            *A.log_t = ctl->t;
        }
        ctl->skipped = ctl->skipped + sk;
        finalize_scalars(ctl, A.P, sd, sv, lam_from_bits(lm, lam_is_f32), fl, 1);
    }
}

// One workgroup's share of a fused step: tile `blk` of the nblk tiles of the
// grid described by A (in the single-grid launch blk = blockIdx.x and nblk =
// gridDim.x; in an ensemble launch, the workgroup's tile within its
// scenario).  The last of the nblk workgroups to finish finalises the step.
// DRY: the dry-tile skip is compiled in and used when A.dry is not NULL.  A
// tile skips the step when it and its eight neighbour tiles were flagged
// kDryStill by the previous step and no cell within two of its output cells
// is a boundary cell or beyond; it then writes the record a computed step
// would (zero defect, no wave speed, no flags; the volume in the record is
// still its unchanged volume) and refreshes the output buffer only if the
// previous step computed it (after a skip both buffers already hold the
// tile's state).
// Strip of the pos-th strip position of a tile run: strips in pairs of
// neighbours, the pairs enumerated by residue class mod 8.  Each XCD's
// contiguous run of tiles then covers strip pairs spread over the whole
// domain (wet and dry strips balance across the XCDs), and the two strips of
// a pair share the row lines they overlap in one L2.
__device__ __forceinline__ int paired_strip(int pos, int gx) {
    const int npair = (gx + 1) / 2;
    int base = 0;
    for (int r = 0; r < 8 && r < npair; ++r) {
        // strips of the pairs r, r+8, r+16, ... (the last pair may be single)
        const int last = npair - 1;
        const int n_pairs = (last - r) / 8 + 1;
        const bool short_last = (gx & 1) && ((last - r) % 8 == 0);
        const int n_r = 2 * n_pairs - (short_last ? 1 : 0);
        if (pos < base + n_r) {
            const int q = pos - base;
            return 2 * (r + 8 * (q / 2)) + (q & 1);
        }
        base += n_r;
    }
    return pos;
}

// PART 0: one wave does the whole tile.  PART 1 and 2: the two waves of a
// workgroup share it (the predictor and the corrector half of every
// iteration, rows passed through `ring`); the second wave keeps the record.
template <typename T, int SIG, bool DRY, bool TRACE, int PART>
__device__ __forceinline__ void fused_tile(const FusedArgs<T>& A, int blk, int nblk, T* ring,
                                           int* prog, int* note) {
    Ctl* ctl = A.ctl;
    if (step_is_noop(ctl, A.t_end)) return;
    const Params& P = A.P;
    March<T, SIG, DRY, TRACE, PART> M;
    if (TRACE)
        for (int f = 0; f < 3; ++f) {
            M.tus[f] = A.tus[f];
            M.tud[f] = A.tud[f];
        }
    M.c.rx = T(ctl->rx); M.c.ry = T(ctl->ry); M.c.dt = T(ctl->dt);
    M.c.qin0 = T(ctl->qin0); M.c.qin1 = T(ctl->qin1);
    M.c.hdry = T(P.h_dry); M.c.g = T(P.g); M.c.hg = T(0.5 * P.g);
    M.c.kap = T(P.kappa); M.c.emax = T(P.eps_max);
    M.c.idx = T(P.idx); M.c.idy = T(P.idy);
    M.c.rcap = T(P.rcap);
    M.P = &A.P;
    M.eta = A.eta; M.qx = A.qx; M.qy = A.qy; M.zb = A.z; M.mm = A.m;
    M.eta1 = A.eta1; M.qx1 = A.qx1; M.qy1 = A.qy1;
    M.nx = P.nx;
    M.ny = P.ny;
    M.pitch = P.pitch;

    const int lane = threadIdx.x % kWave;
    const int tile = xcd_tile(blk, nblk);
    const int pos = tile / A.gy, chunk = tile - pos * A.gy;
    const int gx = (P.nx + kOutW - 1) / kOutW;
    const int strip = paired_strip(pos, gx);
    const int x0 = strip * kOutW;
    M.y0 = chunk * A.H;
    M.yEnd = min(M.y0 + A.H, P.ny);
    M.i = x0 - 2 + lane;
    M.ic = min(max(M.i, 0), P.nx - 1);
    M.colOut = lane >= 2 && lane < 2 + kOutW && M.i < P.nx;
    M.faceE_interior = M.i >= 0 && M.i <= P.nx - 2;   // face i+1/2 is interior
    M.atW = M.i == 0;
    M.atE = M.i == P.nx - 1;
    M.kS = face_kind(P, EDGE_S, M.ic);
    M.kN = face_kind(P, EDGE_N, M.ic);
    const bool edge = x0 - 2 <= 0 || x0 + kWave - 2 >= P.nx;  // uniform

    bool skip = false;
    unsigned* dcur = nullptr;
    int gi = 0;
    if (DRY && A.dry) {
        const int ntile = gx * A.gy;
        gi = strip * A.gy + chunk;
        const int par = (int)(ctl->step & 1);
        const unsigned* dprev = A.dry + par * ntile;
        dcur = A.dry + (1 - par) * ntile;
        // output columns x0 .. x0+59 and rows y0 .. yEnd-1 at least two
        // cells from every edge, and the radius-two halo inside the eight
        // neighbour tiles (H >= 2)
        const bool inner = !edge && strip >= 1 && strip + 1 < gx && chunk >= 1 &&
                           chunk + 1 < A.gy && A.H >= 2 && M.y0 >= 2 && M.yEnd + 2 <= P.ny;
        if (inner) {
            unsigned f = kDryStill;
            if (lane < 9) f = dprev[(strip + lane % 3 - 1) * A.gy + (chunk + lane / 3 - 1)];
            skip = __ballot(!(f & kDryStill)) == 0ull;
        }
        if (skip && PART != 1) {
            if (!(dprev[gi] & kDrySkipped) && M.colOut) {
                for (int r = M.y0; r < M.yEnd; ++r) {
                    const long long o = (long long)r * P.pitch + M.i;
                    A.eta1[o] = A.eta[o];
                    A.qx1[o] = T(0);
                    A.qy1[o] = T(0);
                }
            }
            if (lane == 0) {
                dcur[gi] = kDryStill | kDrySkipped;
                // the volume of the record is the tile's unchanged volume
                TilePart* rec = A.tpart + tile;
                st_agent(&rec->def, 0.0);
                st_agent(&rec->lam, 0ull);
                st_agent(&rec->fs, (unsigned long long)((M.yEnd - M.y0) * kOutW) << 32);
            }
        }
    }

    if (skip) {
        if (PART != 1) finish_step(A, tile, nblk, sizeof(T) == 4);
        return;
    }
    if (PART != 0) {
        M.ring = ring;
        M.prog = prog;
        M.note = note;
        M.lane = lane;
        M.spin_cap = A.spin_cap;
        if (PART == 1 && lane == 0) {
            prog[0] = prog[1] = M.y0 - 3;   // no row filed or taken yet
            *note = 0;
        }
        __syncthreads();
    }
    {
        if (edge)
            M.template run<true>();
        else
            M.template run<false>();
        // a stall of the first wave reaches the record through the second
        if (PART == 1) return;
        if (PART == 2 && (M.stalled || __hip_atomic_load(note, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_WORKGROUP)))
            M.flags |= FLAG_STALL;
        // ---- the workgroup's record (lane 0's reduction order is the fixed one)
        const double vol = wave_sum(M.vol);
        const double def = wave_sum(M.def);
        const unsigned long long lb = wave_max_u64(lam_to_bits(M.lmax));
        const unsigned flags = wave_or(M.flags);
        if (lane == 0) put_record(A.tpart + tile, def, vol, lb, flags);
        if (DRY && dcur) {
            const bool still = __ballot(M.dirty) == 0ull;
            if (lane == 0) dcur[gi] = still ? kDryStill : 0u;
        }
    }
    finish_step(A, tile, nblk, sizeof(T) == 4);
}

template <typename T, int SIG, bool DRY, bool TRACE = false>
__device__ __forceinline__ void fused_step(const FusedArgs<T>& A, int blk, int nblk) {
    fused_tile<T, SIG, DRY, TRACE, 0>(A, blk, nblk, nullptr, nullptr, nullptr);
}

// The two-wave workgroup of a tile: wave 0 the predictor half, wave 1 the
// corrector half.
template <typename T, int SIG, bool DRY, bool TRACE = false>
__device__ __forceinline__ void fused_step_split(const FusedArgs<T>& A, int blk, int nblk) {
    __shared__ T ring[kSplitFields * split_slots<T, DRY>() * kWave];
    __shared__ int prog[2];
    __shared__ int note;
    if (threadIdx.x < kWave)
        fused_tile<T, SIG, DRY, TRACE, 1>(A, blk, nblk, ring, prog, &note);
    else
        fused_tile<T, SIG, DRY, TRACE, 2>(A, blk, nblk, ring, prog, &note);
}

// The two precisions get their own entry points so that each can be given
// the register budget of its best occupancy: FP64 holds about twice the live
// state and runs at 2 waves per SIMD (216 VGPRs), FP32 at 4 (128 VGPRs).
template <int SIG, bool DRY>
__global__ void __launch_bounds__(kWave, 2) k_fused_step_f64(FusedArgs<double> A) {
    fused_step<double, SIG, DRY>(A, blockIdx.x, gridDim.x);
}
template <int SIG, bool DRY>
__global__ void __launch_bounds__(kWave, 3) k_fused_step_f32(FusedArgs<float> A) {
    fused_step<float, SIG, DRY>(A, blockIdx.x, gridDim.x);
}
// The same steps with one more resident wave per SIMD than the register
// budget above allows (FP64 3, FP32 5; the state the march carries then
// partly spills to scratch): the occupancy variant that a launch asks for
// with `more_waves` (a measurement of what occupancy buys; the results are
// the same bits, only the register allocation differs).
template <int SIG>
__global__ void __launch_bounds__(kWave, 3) k_fused_step_f64_w3(FusedArgs<double> A) {
    fused_step<double, SIG, false>(A, blockIdx.x, gridDim.x);
}
template <int SIG>
__global__ void __launch_bounds__(kWave, 5) k_fused_step_f32_w5(FusedArgs<float> A) {
    fused_step<float, SIG, false>(A, blockIdx.x, gridDim.x);
}
// The FP64 step that also writes U* and U^d (the forward data of the adjoint).
template <int SIG>
__global__ void __launch_bounds__(kWave, 2) k_fused_trace_f64(FusedArgs<double> A) {
    fused_step<double, SIG, false, true>(A, blockIdx.x, gridDim.x);
}
// The same steps with two waves per tile, each running half of every
// iteration: half the carried rows per wave, so more waves fit per SIMD (FP64
// 3 at 141 registers; FP32 88 registers, 4 waves as its ring sets) than one
// wave per tile allows (2 and 4).
// (FP64 at 4 waves per SIMD, 128 registers with 48-56 bytes spilled, took 394
// against 283 us.)
constexpr int kSplitWavesF64 = 3, kSplitWavesF32 = 5;
template <int SIG, bool DRY>
__global__ void __launch_bounds__(2 * kWave, kSplitWavesF64) k_fused_split_f64(FusedArgs<double> A) {
    fused_step_split<double, SIG, DRY>(A, blockIdx.x, gridDim.x);
}
template <int SIG, bool DRY>
__global__ void __launch_bounds__(2 * kWave, kSplitWavesF32) k_fused_split_f32(FusedArgs<float> A) {
    fused_step_split<float, SIG, DRY>(A, blockIdx.x, gridDim.x);
}

// Ensemble launch: the workgroups of every scenario in one grid.  Scenario s
// owns workgroups first[s] .. first[s+1]-1 (first[count] = total); its
// arguments are args[s].  A workgroup finds its scenario by binary search.
template <typename T>
__device__ __forceinline__ void ensemble_locate(const int* first, int count, int& s, int& blk,
                                                int& nblk) {
    const int b = blockIdx.x;
    int lo = 0, hi = count;   // first[lo] <= b < first[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (first[mid] <= b) lo = mid; else hi = mid;
    }
    s = lo;
    blk = b - first[lo];
    nblk = first[lo + 1] - first[lo];
}

template <int SIG, bool DRY>
__global__ void __launch_bounds__(kWave, 2)
k_ensemble_step_f64(const FusedArgs<double>* args, const int* first, int count) {
    int sc, blk, nblk;
    ensemble_locate<double>(first, count, sc, blk, nblk);
    fused_step<double, SIG, DRY>(args[sc], blk, nblk);
}
// FP32 at four waves per SIMD (128 registers; the single-grid FP32 step fits
// four without a bound): 90 G against 79 G cell-updates/s at three for the
// 256-scenario flood ensemble.
template <int SIG, bool DRY>
__global__ void __launch_bounds__(kWave, 4)
k_ensemble_step_f32(const FusedArgs<float>* args, const int* first, int count) {
    int sc, blk, nblk;
    ensemble_locate<float>(first, count, sc, blk, nblk);
    fused_step<float, SIG, DRY>(args[sc], blk, nblk);
}

// The same with two waves per tile (the split step), FP32 only: the FP64
// form, with the ensemble's scenario lookup on top, spills 120-170 bytes per
// lane at three waves per SIMD, so FP64 ensembles keep one wave per tile.
template <int SIG, bool DRY>
__global__ void __launch_bounds__(2 * kWave, kSplitWavesF32)
k_ensemble_split_f32(const FusedArgs<float>* args, const int* first, int count) {
    int sc, blk, nblk;
    ensemble_locate<float>(first, count, sc, blk, nblk);
    fused_step_split<float, SIG, DRY>(args[sc], blk, nblk);
}

template <typename T, int SIG, bool DRY, bool SPLIT>
constexpr auto ensemble_kernel() {
    if constexpr (SPLIT && sizeof(T) == 4) {
        return &k_ensemble_split_f32<SIG, DRY>;
    } else if constexpr (sizeof(T) == 8) {
        return &k_ensemble_step_f64<SIG, DRY>;
    } else {
        return &k_ensemble_step_f32<SIG, DRY>;
    }
}

template <typename T, bool SPLIT>
static hipError_t launch_ensemble_k(const FusedArgs<T>* args, const int* first, int count,
                                    int total, int sigma, bool dry, hipStream_t s) {
    const auto k = sigma > 0 ? (dry ? ensemble_kernel<T, 1, true, SPLIT>() : ensemble_kernel<T, 1, false, SPLIT>())
                             : (dry ? ensemble_kernel<T, -1, true, SPLIT>() : ensemble_kernel<T, -1, false, SPLIT>());
    hipLaunchKernelGGL(k, dim3(total), dim3(SPLIT && sizeof(T) == 4 ? 2 * kWave : kWave), 0, s, args,
                       first, count);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ensemble(const FusedArgs<T>* args, const int* first, int count, int total,
                           int sigma, bool dry, hipStream_t s, bool split) {
    if (total <= 0) return hipSuccess;
    return split && sizeof(T) == 4
               ? launch_ensemble_k<T, true>(args, first, count, total, sigma, dry, s)
               : launch_ensemble_k<T, false>(args, first, count, total, sigma, dry, s);
}

template <typename T, int SIG, bool DRY>
constexpr auto fused_kernel() {
    if constexpr (sizeof(T) == 8)
        return &k_fused_step_f64<SIG, DRY>;
    else
        return &k_fused_step_f32<SIG, DRY>;
}
template <typename T, int SIG>
constexpr auto fused_kernel_more() {
    if constexpr (sizeof(T) == 8)
        return &k_fused_step_f64_w3<SIG>;
    else
        return &k_fused_step_f32_w5<SIG>;
}
template <typename T, int SIG, bool DRY>
constexpr auto fused_kernel_split() {
    if constexpr (sizeof(T) == 8)
        return &k_fused_split_f64<SIG, DRY>;
    else
        return &k_fused_split_f32<SIG, DRY>;
}

template <typename T>
hipError_t launch_fused(const FusedArgs<T>& a, int sigma, hipStream_t s, bool more_waves,
                        bool split) {
    const int gx = (a.P.nx + kOutW - 1) / kOutW;
    const int nblk = gx * a.gy;
    const bool dry = a.dry != nullptr;
    if (split && !more_waves) {
        const auto k = sigma > 0 ? (dry ? fused_kernel_split<T, 1, true>() : fused_kernel_split<T, 1, false>())
                                 : (dry ? fused_kernel_split<T, -1, true>() : fused_kernel_split<T, -1, false>());
        hipLaunchKernelGGL(k, dim3(nblk), dim3(2 * kWave), 0, s, a);
        return hipGetLastError();
    }
    auto k = sigma > 0 ? (dry ? fused_kernel<T, 1, true>() : fused_kernel<T, 1, false>())
                       : (dry ? fused_kernel<T, -1, true>() : fused_kernel<T, -1, false>());
    if (more_waves && !dry) k = sigma > 0 ? fused_kernel_more<T, 1>() : fused_kernel_more<T, -1>();
    hipLaunchKernelGGL(k, dim3(nblk), dim3(kWave), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fused_trace(const FusedArgs<double>& a, int sigma, hipStream_t s) {
    const int gx = (a.P.nx + kOutW - 1) / kOutW;
    const int nblk = gx * a.gy;
    if (sigma > 0)
        hipLaunchKernelGGL(k_fused_trace_f64<1>, dim3(nblk), dim3(kWave), 0, s, a);
    else
        hipLaunchKernelGGL(k_fused_trace_f64<-1>, dim3(nblk), dim3(kWave), 0, s, a);
    return hipGetLastError();
}

int fused_blocks(int nx, int ny, int H) {
    const int gx = (nx + kOutW - 1) / kOutW;
    const int gy = (ny + H - 1) / H;
    return gx * gy;
}

int fused_strips(int nx) { return (nx + kOutW - 1) / kOutW; }

int fused_auto_rows(int nx, int ny, long long slots, bool dry_skip) {
    const int gx = fused_strips(nx);
    if (slots <= 0) return dry_skip ? 32 : 128;
    long long gy = slots / gx;
    if (gy < 1) gy = 1;
    int H = (int)((ny + gy - 1) / gy);
    if (H < 6) H = 6;
    if (dry_skip && H > 32) H = 32;
    return H;
}

size_t fused_part_bytes(int ntiles) {
    const size_t ng = (size_t)(ntiles + kGroup - 1) / kGroup;
    return ((size_t)ntiles + ng) * sizeof(TilePart) + ng * sizeof(unsigned);
}

template <typename T>
void fused_part_layout(FusedArgs<T>& a, void* buf, int ntiles) {
    const size_t ng = (size_t)(ntiles + kGroup - 1) / kGroup;
    a.tpart = (TilePart*)buf;
    a.gpart = a.tpart + ntiles;
    a.gticket = (unsigned*)(a.gpart + ng);
}

template <typename T>
int fused_waves_per_cu(bool more_waves) {
    int nb = 0;
    const void* k = more_waves ? (const void*)fused_kernel_more<T, 1>()
                               : (const void*)fused_kernel<T, 1, false>();
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kWave, 0) != hipSuccess) return 0;
    return nb;
}

template <typename T>
int fused_split_tiles_per_cu() {
    int nb = 0;
    const void* k = (const void*)fused_kernel_split<T, 1, false>();
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, 2 * kWave, 0) != hipSuccess) return 0;
    return nb;
}

// Access-pattern probe of the step: the tiles, tile order, strip map and row
// march of the one-wave step, k_fused_step (64-lane strips of 60 output
// columns, chunks of H rows, the row ahead prefetched into two register
// slots, the output row two behind the ingested one; the split step reads and
// writes the same rows in the same order, from its first and its second wave),
// the same five loads and three stores per row, and a handful of operations
// in place of the sixteen sub-steps.  Every loaded value reaches a store, so
// none of the traffic is optimised away.
template <typename T>
__global__ void __launch_bounds__(kWave) k_probe_march(ProbeMarchArgs A) {
    const T* __restrict__ f0 = (const T*)A.in[0];
    const T* __restrict__ f1 = (const T*)A.in[1];
    const T* __restrict__ f2 = (const T*)A.in[2];
    const T* __restrict__ f3 = (const T*)A.in[3];
    const T* __restrict__ f4 = (const T*)A.in[4];
    T* __restrict__ o0 = (T*)A.out[0];
    T* __restrict__ o1 = (T*)A.out[1];
    T* __restrict__ o2 = (T*)A.out[2];
    const int lane = threadIdx.x;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int pos = tile / A.gy, chunk = tile - pos * A.gy;
    const int gx = (A.nx + kOutW - 1) / kOutW;
    const int i = paired_strip(pos, gx) * kOutW - 2 + lane;
    const int ic = min(max(i, 0), A.nx - 1);
    const bool colOut = lane >= 2 && lane < 2 + kOutW && i < A.nx;
    const int y0 = chunk * A.H, yEnd = min(y0 + A.H, A.ny);
    auto off = [&](int R) { return (long long)min(max(R, 0), A.ny - 1) * A.pitch + ic; };
    T pe[2], pa[2], pb[2], pz[2], pm[2] = {T(0), T(0)};
    T e1 = 0, a1 = 0, b1 = 0, z1 = 0, e2 = 0, a2 = 0, b2 = 0, z2 = 0;
    {
        const long long o = off(y0 - 2);
        pe[0] = f0[o]; pa[0] = f1[o]; pb[0] = f2[o]; pz[0] = f3[o];
    }
    auto iter = [&](int R, int S) {
        const T e0 = pe[S], a0 = pa[S], b0 = pb[S], z0 = pz[S], m2 = pm[S];
        const long long o = off(R + 1);
        pe[1 - S] = f0[o]; pa[1 - S] = f1[o]; pb[1 - S] = f2[o]; pz[1 - S] = f3[o];
        pm[1 - S] = f4[off(R - 1)];
        // the shifts run with every lane active (a disabled source lane reads 0)
        const T e1E = from_east(e1), a1W = from_west(a1);
        if (R - 2 >= y0 && R - 2 < yEnd && colOut) {
            const long long so = (long long)(R - 2) * A.pitch + i;
            o0[so] = e2 + e1E * m2;
            o1[so] = a2 + z2 * a1W + e0;
            o2[so] = b2 + b1 * z1 + a0 * b0 + z0;
        }
        e2 = e1; a2 = a1; b2 = b1; z2 = z1;
        e1 = e0; a1 = a0; b1 = b0; z1 = z0;
    };
    for (int R = y0 - 2; R <= yEnd + 1; R += 2) {
        iter(R, 0);
        iter(R + 1, 1);
    }
}

int probe_march_rows(int elem_bytes, int nx, int ny, int cus) {
    const int per_cu = elem_bytes == 4 ? fused_waves_per_cu<float>(false) : fused_waves_per_cu<double>(false);
    return fused_auto_rows(nx, ny, (long long)cus * per_cu, false);
}

hipError_t launch_probe_march(const ProbeMarchArgs& a, int elem_bytes, hipStream_t s) {
    const int gx = (a.nx + kOutW - 1) / kOutW;
    const int nblk = gx * a.gy;
    if (elem_bytes == 4)
        hipLaunchKernelGGL(k_probe_march<float>, dim3(nblk), dim3(kWave), 0, s, a);
    else
        hipLaunchKernelGGL(k_probe_march<double>, dim3(nblk), dim3(kWave), 0, s, a);
    return hipGetLastError();
}

template hipError_t launch_ensemble<float>(const FusedArgs<float>*, const int*, int, int, int,
                                           bool, hipStream_t, bool);
template hipError_t launch_ensemble<double>(const FusedArgs<double>*, const int*, int, int, int,
                                            bool, hipStream_t, bool);
template hipError_t launch_fused<float>(const FusedArgs<float>&, int, hipStream_t, bool, bool);
template hipError_t launch_fused<double>(const FusedArgs<double>&, int, hipStream_t, bool, bool);
template void fused_part_layout<float>(FusedArgs<float>&, void*, int);
template void fused_part_layout<double>(FusedArgs<double>&, void*, int);
template int fused_waves_per_cu<float>(bool);
template int fused_waves_per_cu<double>(bool);
template int fused_split_tiles_per_cu<float>();
template int fused_split_tiles_per_cu<double>();

}  // namespace swe
