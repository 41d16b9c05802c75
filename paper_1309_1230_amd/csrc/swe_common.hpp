// swe_common.hpp -- device-side definitions shared by the fused and the
// unfused kernels of libswe: the control block that keeps t, dt and the
// diagnostics resident on the GPU, the problem parameters, the per-face and
// per-cell formulas of the scheme, wave reductions and the finalisation of a
// time step (the new dt is computed on the device; the paper copied the state
// to the host every step for this, §3.1, which is what this layout removes).
//
// The discrete scheme (our reading; the paper, §1, fixes the predictor-
// corrector MacCormack method, explicitness and the sixteen cell-independent
// sub-steps per step, and defers the equations to a thesis that is not
// available).  Unknowns eta, qx, qy; h = eta - z; wet <=> h > h_dry.
//   S1  ghost ring of U^n (eta copied; WALL mirrors the normal discharge,
//       OPEN copies, INFLOW imposes q_in(t^n) inward with zero tangential).
//   S2  h = eta - z, r = wet ? 1/h : 0, u = qx*r, v = qy*r; thin-film reading:
//       r = wet ? min(1/h, 1/h_film) : 0.
//   S3  nu_x = 0.25*(|(eta_E - eta_C) - (eta_C - eta_W)| * r_C), nu_y alike.
//   S4  eps_f = (wet_L && wet_R) ? min(kappa*max(nu_L, nu_R), eps_max) : 0 on
//       interior faces, 0 on boundary faces;
//       D = (eps_E*(U_E-U_C) - eps_W*(U_C-U_W)) + (eps_N*(U_N-U_C) - eps_S*(U_C-U_S)).
//   S5/S6  face fluxes with the donor on the sigma side (sigma = +1 on even
//       steps): fm = wet_d ? q_d : 0, (fm, fm*u_d, fm*v_d); pressure
//       P = (g*(0.5*(h+_L + h+_R)))*(eta_R - eta_L) on interior faces that are
//       not dry banks.  WALL faces carry nothing; OPEN faces carry the flux of
//       the adjacent cell; INFLOW faces carry q_in inward with momentum
//       q_in*(q_in*r_adj).
//   S7  U* = U^n - dt/dx*(dF + P_x on the sigma face) - dt/dy*(dG + P_y).
//   S8..S11  the same on U* with -sigma and q_in(t^n + dt).
//   S12 U^c = 0.5*(U^n + (U* - L_{-sigma}(U*))).   S13 U^d = U^c + D.
//   S14 point-implicit Manning: q /= 1 + dt*m*|q|/h*h^(-4/3) (m = g n^2),
//       h^(-4/3) = r*cbrt(r) with the reproducible cube root tcbrt.
//   S15 negative depth clipped (volume recorded), dry cells lose discharge.
//   S16 lam = (|u|+c)/dx + (|v|+c)/dy over wet cells (c = sqrt(g h)),
//       dt^{n+1} = min(cfl/max lam, dt_max) (or dt_fixed).
// Every expression keeps one fixed evaluation order and the code is built
// without floating-point contraction, so FP64 results are reproducible bit
// for bit by any implementation of the same order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swe {

constexpr int kWave = 64;
constexpr int BC_WALL = 0, BC_OPEN = 1, BC_INFLOW = 2;
constexpr int EDGE_W = 0, EDGE_E = 1, EDGE_S = 2, EDGE_N = 3;
constexpr unsigned FLAG_NAN = 1u, FLAG_CLIPPED = 2u, FLAG_BADDT = 4u, FLAG_STALL = 8u;
constexpr unsigned FLAG_FATAL = FLAG_NAN | FLAG_BADDT | FLAG_STALL;
constexpr int kMaxHydro = 4096;
// Polls (each about 100 cycles) after which a wave of the split fused step
// stops waiting for its partner: some 40 ms, far beyond any row's time.
constexpr int kSplitSpinCap = 1 << 20;

// Device-resident scalars of one handle.  Written only by the finalisation of
// a step (one wave, after every block of the step has finished its sweep) and
// read by every block at the start of the next step.
struct Ctl {
    double t;            // t^n
    double dt;           // dt^n: the step the next launch takes
    double rx, ry;       // dt/dx, dt/dy
    double qin0, qin1;   // q_in(t^n), q_in(t^n + dt^n)
    double defect;       // clipped volume since create
    double volume;       // sum h dx dy of the current state
    double lam_max;      // lam_max of the current state
    double dt_min, dt_max_used;  // over the current host call
    double last_defect_depth;    // sum of clipped depth of the last step
    long long step;      // n
    long long bad_step;  // first step that raised a fatal flag, or -1
    long long call_steps;
    unsigned flags;      // OR of all flags
    unsigned step_flags; // flags raised by the step in flight
    unsigned last_step_flags;
    unsigned ticket;     // blocks of the step in flight that have finished
    unsigned long long lam_bits;  // running max of lam (IEEE bits, lam >= 0)
    unsigned long long skipped;   // cell updates the dry-tile skip left out, this call
};

struct Params {
    int nx, ny;
    long long pitch;
    int bc[4], lo[4], hi[4];
    int hydro_len;
    double dx, dy, g, cfl, h_dry, kappa, eps_max, dt_max, dt_fixed;
    double idx, idy;     // 1/dx, 1/dy
    double rcap;         // S3's cap on the reciprocal depth: 1/h_film, or +inf
    const double* hydro_t;   // device copies
    const double* hydro_q;
};

// Kind of the boundary face number k along an edge (INFLOW outside its band
// is a wall).
__host__ __device__ inline int face_kind(const Params& P, int edge, int k) {
    int kind = P.bc[edge];
    if (kind == BC_INFLOW && !(k >= P.lo[edge] && k < P.hi[edge])) return BC_WALL;
    return kind;
}

// Piecewise-linear hydrograph of L points (times ht, discharges hq),
// constant outside its points.  Host and device evaluate the same IEEE
// expression, so both give the same bits.
__host__ __device__ inline double q_inflow_at(const double* ht, const double* hq, int L,
                                              double t) {
    if (L <= 0) return 0.0;
    if (t <= ht[0]) return hq[0];
    if (t >= ht[L - 1]) return hq[L - 1];
    int k = 0;
    while (k + 1 < L && !(t < ht[k + 1])) ++k;
    double w = (t - ht[k]) / (ht[k + 1] - ht[k]);
    return hq[k] + w * (hq[k + 1] - hq[k]);
}
__device__ inline double q_inflow(const Params& P, double t) {
    return q_inflow_at(P.hydro_t, P.hydro_q, P.hydro_len, t);
}

__device__ inline double next_dt(const Params& P, double lam) {
    if (P.dt_fixed > 0.0) return P.dt_fixed;
    if (lam > 0.0) {
        double d = P.cfl / lam;
        return d < P.dt_max ? d : P.dt_max;
    }
    return P.dt_max;
}

// ------------------------------------------------------------ wave layout

// DPP wavefront shifts: lane l receives the value of lane l+1 (from_east) or
// l-1 (from_west).  The end lanes (63, resp. 0) receive 0; they are halo
// lanes whose shifted values feed no output column.
__device__ __forceinline__ int dpp_from_east(int v) {
    return __builtin_amdgcn_mov_dpp(v, 0x130, 0xF, 0xF, true);   // wave_shl:1
}
__device__ __forceinline__ int dpp_from_west(int v) {
    return __builtin_amdgcn_mov_dpp(v, 0x138, 0xF, 0xF, true);   // wave_shr:1
}
__device__ __forceinline__ float from_east(float x) {
    return __int_as_float(dpp_from_east(__float_as_int(x)));
}
__device__ __forceinline__ float from_west(float x) {
    return __int_as_float(dpp_from_west(__float_as_int(x)));
}
__device__ __forceinline__ double from_east(double x) {
    return __hiloint2double(dpp_from_east(__double2hiint(x)), dpp_from_east(__double2loint(x)));
}
__device__ __forceinline__ double from_west(double x) {
    return __hiloint2double(dpp_from_west(__double2hiint(x)), dpp_from_west(__double2loint(x)));
}

// Workgroup id -> tile id so that each XCD (workgroups are dealt round-robin
// over the 8 XCDs) receives one contiguous run of tiles: vertically adjacent
// chunks of a strip, and neighbouring strips, then share an L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int per = nb / 8, rem = nb % 8;
    const int xcd = b % 8, loc = b / 8;
    return xcd < rem ? xcd * (per + 1) + loc : rem * (per + 1) + (xcd - rem) * per + loc;
}

// ------------------------------------------------------------ cell formulas

__device__ __forceinline__ float tfabs(float x) { return __builtin_fabsf(x); }
__device__ __forceinline__ double tfabs(double x) { return __builtin_fabs(x); }
// Reciprocal and square root.  FP64: correctly rounded, so the FP64 path is
// reproducible bit for bit by any IEEE implementation of the same expression
// order.  FP32: the single hardware instructions (1 ulp); the FP32 state is
// held to a tolerance against the FP64 oracle, not to bit equality.
__device__ __forceinline__ double trcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float trcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float tsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double tsqrt(double x) { return __builtin_sqrt(x); }
// Cube root of x > 0 used by the friction step: the exponent-thirding guess
// (integer arithmetic on the IEEE-754 bits: high word w/3 + 0x2A9F7893, low
// word 0 in FP64; bits/3 + 0x2A5137A0 in FP32; Kahan's cube-root note) refined by
// two Halley steps y <- y*((t + 2x)/(2t + x)), t = y^3.  Every operation is
// exact or correctly rounded, so the FP64 result is reproducible bit for bit
// on any IEEE machine (a math library's cbrt is only faithful to about an ulp
// and differs between libraries).  Relative error < 7e-15 (FP64).  The FP32
// version divides through the hardware reciprocal: a few ulp.
__device__ __forceinline__ double tcbrt(double x) {
    const unsigned w = (unsigned)__double2hiint(x);
    double y = __hiloint2double((int)(w / 3u + 0x2A9F7893u), 0);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double t = (y * y) * y;
        y = y * ((t + (x + x)) / ((t + t) + x));
    }
    return y;
}
__device__ __forceinline__ float tcbrt(float x) {
    unsigned b = __float_as_uint(x);
    b = b / 3u + 0x2A5137A0u;
    float y = __uint_as_float(b);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const float t = (y * y) * y;
        y = y * ((t + (x + x)) * trcp((t + t) + x));
    }
    return y;
}
__device__ __forceinline__ bool tfinite(float x) { return __builtin_isfinite(x); }
__device__ __forceinline__ bool tfinite(double x) { return __builtin_isfinite(x); }

template <typename T> __device__ __forceinline__ T hpos(T h) { return h > T(0) ? h : T(0); }
template <typename T> __device__ __forceinline__ T tmax(T a, T b) { return a > b ? a : b; }
template <typename T> __device__ __forceinline__ T tmin(T a, T b) { return a < b ? a : b; }

// Reciprocal depth of a wet cell, 0 for a dry one (friction, CFL).
template <typename T> __device__ __forceinline__ T recip_depth(T h, T hdry) {
    return h > hdry ? trcp(h) : T(0);
}

// S2 / S9: the reciprocal depth of the primitive variables, min(1/h, rcap)
// for a wet cell (the thin-film reading: velocities and switch of films
// thinner than 1/rcap use that depth instead; rcap = +inf when the reading is
// off, and the selection then returns 1/h itself), 0 for a dry one.
template <typename T> __device__ __forceinline__ T recip_prim(T h, T hdry, T rcap) {
    if (!(h > hdry)) return T(0);
    const T r = trcp(h);
    return r < rcap ? r : rcap;
}

// S3: curvature switch of the water surface at a cell.
template <typename T> __device__ __forceinline__ T curv_switch(T eW, T eC, T eE, T rC) {
    return T(0.25) * (tfabs((eE - eC) - (eC - eW)) * rC);
}

// S4: dissipation coefficient of an interior face.
template <typename T>
__device__ __forceinline__ T face_eps(T hL, T hR, T nuL, T nuR, T hdry, T kappa, T emax) {
    return (hL > hdry && hR > hdry) ? tmin(kappa * tmax(nuL, nuR), emax) : T(0);
}

// S5/S6: pressure of an interior face between cells L (low) and R (high),
// (g*(0.5*(h+_L + h+_R)))*(eta_R - eta_L).  hg = 0.5*g: halving is exact, so
// hg*S rounds the same real number as g*(0.5*S) and the two forms agree bit
// for bit (no underflow is possible at these magnitudes).
template <typename T>
__device__ __forceinline__ T face_pressure(T eL, T hL, T zL, T eR, T hR, T zR, T hdry, T hg) {
    bool bank = (!(hL > hdry) && zL > eR) || (!(hR > hdry) && zR > eL);
    return bank ? T(0) : (hg * (hpos(hL) + hpos(hR))) * (eR - eL);
}

// Flux a boundary face carries when the adjacent interior cell has the
// donor fluxes (fm, fa, fb) (fa: momentum along the face normal... see
// normal_is_x) and reciprocal depth r.  qs is the signed inflow discharge
// (positive along +x or +y).  For x faces the normal momentum is the second
// component, for y faces the third.
template <typename T>
__device__ __forceinline__ void boundary_flux(int kind, bool normal_is_x, T fm, T f1, T f2, T qs,
                                              T r, T& Fm, T& F1, T& F2) {
    if (kind == BC_WALL) {
        Fm = T(0); F1 = T(0); F2 = T(0);
    } else if (kind == BC_OPEN) {
        Fm = fm; F1 = f1; F2 = f2;
    } else {
        Fm = qs;
        if (normal_is_x) {
            F1 = qs * (qs * r);
            F2 = qs * (T(0) * r);
        } else {
            F1 = qs * (T(0) * r);
            F2 = qs * (qs * r);
        }
    }
}

// S1 / S8: ghost value of a W/E (normal = qx) or S/N (normal = qy) edge
// cell (e, qx, qy: the adjacent interior cell; inward: the signed inflow).
template <typename T>
__device__ __forceinline__ void ghost(int kind, bool normal_is_x, T inward, T e, T qx, T qy,
                                      T& ge, T& gqx, T& gqy) {
    ge = e;
    if (kind == BC_OPEN) {
        gqx = qx;
        gqy = qy;
    } else if (kind == BC_INFLOW) {
        gqx = normal_is_x ? inward : T(0);
        gqy = normal_is_x ? T(0) : inward;
    } else {
        gqx = normal_is_x ? -qx : qx;
        gqy = normal_is_x ? qy : -qy;
    }
}

// S14: point-implicit Manning friction of a wet cell with reciprocal depth r.
template <typename T>
__device__ __forceinline__ void manning(T dt, T m, T r, T& qx, T& qy) {
    T s = tsqrt(qx * qx + qy * qy) * r;
    T k = r * tcbrt(r);
    T phi = T(1) + ((dt * m) * s) * k;
    T psi = trcp(phi);
    qx = qx * psi;
    qy = qy * psi;
}

// S16: characteristic speed sum of a wet cell.
template <typename T>
__device__ __forceinline__ T cfl_lambda(T h, T r, T qx, T qy, T g, T idx, T idy) {
    T u = qx * r, v = qy * r;
    T c = tsqrt(g * h);
    return (tfabs(u) + c) * idx + (tfabs(v) + c) * idy;
}

// Running max of lam that lets a NaN through.
template <typename T> __device__ __forceinline__ T lam_acc(T acc, T lam) {
    return !(lam <= acc) ? lam : acc;
}

__device__ __forceinline__ unsigned long long lam_to_bits(float x) {
    return (unsigned long long)__float_as_uint(x);
}
__device__ __forceinline__ unsigned long long lam_to_bits(double x) {
    return (unsigned long long)__double_as_longlong(x);
}

// ------------------------------------------------------------- reductions

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = v + __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        unsigned long long o = __shfl_xor(v, off, kWave);
        v = o > v ? o : v;
    }
    return v;
}

__device__ __forceinline__ unsigned wave_or(unsigned v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v |= __shfl_xor(v, off, kWave);
    return v;
}

// Finalise a step (mode 1) or the initial scan (mode 0) from its reduced
// partials: defect and volume sums sd, sv (depth units), lam_max, and the
// flags the step raised.  Computes dt^{n+1} and the inflow values of the
// next step, advances t and the step counter, and clears the accumulators
// for the next launch.  One lane.
__device__ inline void finalize_scalars(Ctl* ctl, const Params& P, double sd, double sv,
                                        double lam, unsigned sf, int mode) {
    double dtn = next_dt(P, lam);
    if (!__builtin_isfinite(lam)) sf |= FLAG_NAN;
    if (!(dtn > 0.0) || !__builtin_isfinite(dtn)) sf |= FLAG_BADDT;
    const double area = P.dx * P.dy;
    if (mode == 1) {
        double dt_used = ctl->dt;
        ctl->defect = ctl->defect + sd * area;
        ctl->last_defect_depth = sd;
        ctl->t = ctl->t + dt_used;
        ctl->dt_min = dt_used < ctl->dt_min ? dt_used : ctl->dt_min;
        ctl->dt_max_used = dt_used > ctl->dt_max_used ? dt_used : ctl->dt_max_used;
        if ((sf & FLAG_FATAL) && ctl->bad_step < 0) ctl->bad_step = ctl->step;
        ctl->step = ctl->step + 1;
        ctl->call_steps = ctl->call_steps + 1;
    }
    ctl->flags |= sf;
    ctl->last_step_flags = sf;
    ctl->volume = sv * area;
    ctl->lam_max = lam;
    ctl->dt = dtn;
    ctl->rx = dtn / P.dx;
    ctl->ry = dtn / P.dy;
    ctl->qin0 = q_inflow(P, ctl->t);
    ctl->qin1 = q_inflow(P, ctl->t + dtn);
    ctl->lam_bits = 0ull;
    ctl->step_flags = 0u;
    ctl->ticket = 0u;
}

__device__ __forceinline__ double lam_from_bits(unsigned long long bits, bool lam_is_f32) {
    return lam_is_f32 ? (double)__uint_as_float((unsigned)bits) : __longlong_as_double((long long)bits);
}

// Finalisation after a kernel boundary (unfused path, initial scan): one wave
// sums the nparts partials in a fixed order; lam_max and the flags come from
// the control block's accumulators.
__device__ inline void finalize_wave(Ctl* ctl, const Params& P, const double* part_def,
                                     const double* part_vol, int nparts, bool lam_is_f32,
                                     int mode) {
    const int lane = threadIdx.x;
    double sd = 0.0, sv = 0.0;
    for (int k = lane; k < nparts; k += kWave) {
        sd = sd + part_def[k];
        sv = sv + part_vol[k];
    }
    sd = wave_sum(sd);
    sv = wave_sum(sv);
    if (lane == 0) {
        unsigned long long bits = __hip_atomic_load(&ctl->lam_bits, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        unsigned sf = __hip_atomic_load(&ctl->step_flags, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
        finalize_scalars(ctl, P, sd, sv, lam_from_bits(bits, lam_is_f32), sf, mode);
    }
}

// Partial results of one workgroup of the fused step (and, reduced, of a
// group of kGroup workgroups): defect and volume sums, max lam (IEEE bits of
// the kernel's precision, lam >= 0), flags, and the cell updates the
// dry-tile skip left out.  32 bytes, so a wave reads 64 of them in one
// coalesced sweep.  Records are written and read with agent-scope atomic
// accesses, which are coherent across the XCDs' separate L2 caches without
// a whole-cache write-back or invalidation.
struct TilePart {
    double def, vol;
    unsigned long long lam;
    unsigned long long fs;   // flags | skipped << 32
};
constexpr int kGroup = kWave;

// Whether the launch for the current step should do nothing: the run already
// reached t_end, or an earlier step raised a fatal flag.
__device__ __forceinline__ bool step_is_noop(const Ctl* ctl, double t_end) {
    return !(ctl->t < t_end) || (ctl->flags & FLAG_FATAL);
}

}  // namespace swe
