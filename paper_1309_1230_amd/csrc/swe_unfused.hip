// swe_unfused.hip -- one kernel per sub-step (S1..S16), every intermediate
// in device memory, plus the small utility kernels of the library.
//
// This path mirrors the paper's own structure, where kernel boundaries are
// the only synchronisation inside a time step (§3.1), and is kept for two
// jobs: it is the parity ladder (each sub-step's output can be compared with
// the CPU reference array by array) and the "one launch per sub-step"
// comparison point for the fused kernel.  Intermediates live in padded
// (nx+2) x (ny+2) arrays with a one-cell ghost ring, in the order the trace
// interface exposes them; faces between cells k and k+1 are stored in the slot
// of cell k.
#include <algorithm>

#include "swe_common.hpp"
#include "swe_internal.hpp"

namespace swe {

namespace {

constexpr int kBX = 64, kBY = 4;     // 2D blocks of the sweeps
constexpr int kRB = 16;              // rows per block of the reducing sweeps

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
};

__device__ __forceinline__ Pad pad_of(const Params& P) {
    Pad d;
    d.nx = P.nx;
    d.ny = P.ny;
    d.P2 = P.nx + 2;
    d.N = (long long)(P.nx + 2) * (long long)(P.ny + 2);
    return d;
}

template <typename T>
__device__ __forceinline__ T* arr(T* trace, const Pad& d, int k) {
    return trace + (long long)k * d.N;
}

// S1: copy U^n into the padded arrays and build its ghost ring.
template <typename T>
__global__ void k_s1(UnfusedArgs<T> a) {
    if (step_is_noop(a.ctl, a.t_end)) return;
    const Pad d = pad_of(a.P);
    const int pi = blockIdx.x * kBX + threadIdx.x, pj = blockIdx.y * kBY + threadIdx.y;
    if (pi >= d.nx + 2 || pj >= d.ny + 2) return;
    const int i = pi - 1, j = pj - 1;
    const bool gx = i < 0 || i >= d.nx, gy = j < 0 || j >= d.ny;
    if (gx && gy) return;  // corners are never read
    const int ii = min(max(i, 0), d.nx - 1), jj = min(max(j, 0), d.ny - 1);
    const long long src = (long long)jj * a.P.pitch + ii;
    T e = a.eta[src], qx = a.qx[src], qy = a.qy[src];
    const T qin = T(a.ctl->qin0);
    if (gx) {
        const int edge = i < 0 ? EDGE_W : EDGE_E;
        ghost(face_kind(a.P, edge, j), true, i < 0 ? qin : -qin, e, qx, qy, e, qx, qy);
    } else if (gy) {
        const int edge = j < 0 ? EDGE_S : EDGE_N;
        ghost(face_kind(a.P, edge, i), false, j < 0 ? qin : -qin, e, qx, qy, e, qx, qy);
    }
    const long long s = d.at(i, j);
    arr(a.trace, d, T_UN + 0)[s] = e;
    arr(a.trace, d, T_UN + 1)[s] = qx;
    arr(a.trace, d, T_UN + 2)[s] = qy;
}

// S8: ghost ring of U* (interior written by S7).
template <typename T>
__global__ void k_s8(UnfusedArgs<T> a) {
    if (step_is_noop(a.ctl, a.t_end)) return;
    const Pad d = pad_of(a.P);
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const T qin = T(a.ctl->qin1);
    T* E = arr(a.trace, d, T_US + 0);
    T* QX = arr(a.trace, d, T_US + 1);
    T* QY = arr(a.trace, d, T_US + 2);
    if (k < d.ny) {
        const int j = k;
        for (int side = 0; side < 2; ++side) {
            const int ig = side ? d.nx : -1, ia = side ? d.nx - 1 : 0;
            const long long s = d.at(ia, j), g = d.at(ig, j);
            ghost(face_kind(a.P, side ? EDGE_E : EDGE_W, j), true, side ? -qin : qin, E[s], QX[s],
                  QY[s], E[g], QX[g], QY[g]);
        }
    }
    if (k < d.nx) {
        const int i = k;
        for (int side = 0; side < 2; ++side) {
            const int jg = side ? d.ny : -1, ja = side ? d.ny - 1 : 0;
            const long long s = d.at(i, ja), g = d.at(i, jg);
            ghost(face_kind(a.P, side ? EDGE_N : EDGE_S, i), false, side ? -qin : qin, E[s], QX[s],
                  QY[s], E[g], QX[g], QY[g]);
        }
    }
}

// S2 / S9: primitive variables over every padded cell.
template <typename T>
__global__ void k_prim(UnfusedArgs<T> a, int src, int dst_h) {
    if (step_is_noop(a.ctl, a.t_end)) return;
    const Pad d = pad_of(a.P);
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= d.N) return;
    const T hdry = T(a.P.h_dry);
    const T h = arr(a.trace, d, src)[s] - a.zp[s];
    const T r = recip_prim(h, hdry, T(a.P.rcap));
    arr(a.trace, d, dst_h + 0)[s] = h;
    arr(a.trace, d, dst_h + 1)[s] = r;
    arr(a.trace, d, dst_h + 2)[s] = arr(a.trace, d, src + 1)[s] * r;
    arr(a.trace, d, dst_h + 3)[s] = arr(a.trace, d, src + 2)[s] * r;
}

// S3: curvature switch.
template <typename T>
__global__ void k_s3(UnfusedArgs<T> a) {
    if (step_is_noop(a.ctl, a.t_end)) return;
    const Pad d = pad_of(a.P);
    const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y;
    if (i >= d.nx || j >= d.ny) return;
    const T* E = arr(a.trace, d, T_UN);
    const T* R = arr(a.trace, d, T_R);
    const long long C = d.at(i, j);
    arr(a.trace, d, T_NUX)[C] = curv_switch(E[d.at(i - 1, j)], E[C], E[d.at(i + 1, j)], R[C]);
    arr(a.trace, d, T_NUY)[C] = curv_switch(E[d.at(i, j - 1)], E[C], E[d.at(i, j + 1)], R[C]);
}

// S4: switched dissipation of U^n.
template <typename T>
__global__ void k_s4(UnfusedArgs<T> a) {
    if (step_is_noop(a.ctl, a.t_end)) return;
    const Pad d = pad_of(a.P);
    const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y;
    if (i >= d.nx || j >= d.ny) return;
    const T hdry = T(a.P.h_dry), kap = T(a.P.kappa), emax = T(a.P.eps_max);
    const T* H = arr(a.trace, d, T_H);
    const T* NX = arr(a.trace, d, T_NUX);
    const T* NY = arr(a.trace, d, T_NUY);
    const long long C = d.at(i, j), E = d.at(i + 1, j), W = d.at(i - 1, j);
    const long long N = d.at(i, j + 1), S = d.at(i, j - 1);
    const T eE = i + 1 < d.nx ? face_eps(H[C], H[E], NX[C], NX[E], hdry, kap, emax) : T(0);
    const T eW = i > 0 ? face_eps(H[W], H[C], NX[W], NX[C], hdry, kap, emax) : T(0);
    const T eN = j + 1 < d.ny ? face_eps(H[C], H[N], NY[C], NY[N], hdry, kap, emax) : T(0);
    const T eS = j > 0 ? face_eps(H[S], H[C], NY[S], NY[C], hdry, kap, emax) : T(0);
    for (int v = 0; v < 3; ++v) {
        const T* q = arr(a.trace, d, T_UN + v);
        const T dxq = eE * (q[E] - q[C]) - eW * (q[C] - q[W]);
        const T dyq = eN * (q[N] - q[C]) - eS * (q[C] - q[S]);
        arr(a.trace, d, T_D + v)[C] = dxq + dyq;
    }
}

// One face between L and R (x or y), kind is FACE_* with interior = -1.
template <typename T>
__device__ __forceinline__ void face(int kind, int dir, bool ghost_is_R, long long L, long long R,
                                     const T* E, const T* QN, const T* H, const T* U, const T* V,
                                     const T* Z, T hdry, T hg, T out[4]) {
    if (kind == BC_WALL) {
        out[0] = out[1] = out[2] = out[3] = T(0);
        return;
    }
    long long dn;
    T fm;
    if (kind == BC_INFLOW) {
        dn = ghost_is_R ? R : L;
        fm = QN[dn];
    } else {
        dn = dir > 0 ? R : L;
        fm = H[dn] > hdry ? QN[dn] : T(0);
    }
    out[0] = fm;
    out[1] = fm * U[dn];
    out[2] = fm * V[dn];
    out[3] = kind < 0 ? face_pressure(E[L], H[L], Z[L], E[R], H[R], Z[R], hdry, hg) : T(0);
}

// S5 / S10: x faces i = -1 .. nx-1 of rows 0 .. ny-1.
template <typename T>
__global__ void k_xflux(UnfusedArgs<T> a, int dir, int src, int prim, int dst) {
    if (step_is_noop(a.ctl, a.t_end)) return;
    const Pad d = pad_of(a.P);
    const int i = (int)(blockIdx.x * kBX + threadIdx.x) - 1, j = blockIdx.y * kBY + threadIdx.y;
    if (i >= d.nx || j >= d.ny) return;
    const int kind = i == -1 ? face_kind(a.P, EDGE_W, j)
                             : (i == d.nx - 1 ? face_kind(a.P, EDGE_E, j) : -1);
    T o[4];
    face(kind, dir, i == d.nx - 1, d.at(i, j), d.at(i + 1, j), arr(a.trace, d, src),
         arr(a.trace, d, src + 1), arr(a.trace, d, prim), arr(a.trace, d, prim + 2),
         arr(a.trace, d, prim + 3), a.zp, T(a.P.h_dry), T(0.5 * a.P.g), o);
    const long long s = d.at(i, j);
    for (int v = 0; v < 4; ++v) arr(a.trace, d, dst + v)[s] = o[v];
}

// S6 / S11: y faces j = -1 .. ny-1 of columns 0 .. nx-1.
template <typename T>
__global__ void k_yflux(UnfusedArgs<T> a, int dir, int src, int prim, int dst) {
    if (step_is_noop(a.ctl, a.t_end)) return;
    const Pad d = pad_of(a.P);
    const int i = blockIdx.x * kBX + threadIdx.x, j = (int)(blockIdx.y * kBY + threadIdx.y) - 1;
    if (i >= d.nx || j >= d.ny) return;
    const int kind = j == -1 ? face_kind(a.P, EDGE_S, i)
                             : (j == d.ny - 1 ? face_kind(a.P, EDGE_N, i) : -1);
    T o[4];
    face(kind, dir, j == d.ny - 1, d.at(i, j), d.at(i, j + 1), arr(a.trace, d, src),
         arr(a.trace, d, src + 2), arr(a.trace, d, prim), arr(a.trace, d, prim + 2),
         arr(a.trace, d, prim + 3), a.zp, T(a.P.h_dry), T(0.5 * a.P.g), o);
    const long long s = d.at(i, j);
    for (int v = 0; v < 4; ++v) arr(a.trace, d, dst + v)[s] = o[v];
}

// S7 (corr = false: out = base - L) and S12 (corr = true: out = 0.5*(U^n +
// (base - L))), with the pressure on the dir side.
template <typename T>
__global__ void k_update(UnfusedArgs<T> a, int dir, int base, int F, int G, int dst, bool corr) {
    if (step_is_noop(a.ctl, a.t_end)) return;
    const Pad d = pad_of(a.P);
    const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y;
    if (i >= d.nx || j >= d.ny) return;
    const T rx = T(a.ctl->rx), ry = T(a.ctl->ry);
    const long long C = d.at(i, j), W = d.at(i - 1, j), S = d.at(i, j - 1);
    const T* Fm = arr(a.trace, d, F);
    const T* Fx = arr(a.trace, d, F + 1);
    const T* Fy = arr(a.trace, d, F + 2);
    const T* Px = arr(a.trace, d, F + 3);
    const T* Gm = arr(a.trace, d, G);
    const T* Gx = arr(a.trace, d, G + 1);
    const T* Gy = arr(a.trace, d, G + 2);
    const T* Py = arr(a.trace, d, G + 3);
    const T px = dir > 0 ? Px[C] : Px[W];
    const T py = dir > 0 ? Py[C] : Py[S];
    T o0 = (arr(a.trace, d, base)[C] - rx * (Fm[C] - Fm[W])) - ry * (Gm[C] - Gm[S]);
    T o1 = (arr(a.trace, d, base + 1)[C] - rx * ((Fx[C] - Fx[W]) + px)) - ry * (Gx[C] - Gx[S]);
    T o2 = (arr(a.trace, d, base + 2)[C] - rx * (Fy[C] - Fy[W])) - ry * ((Gy[C] - Gy[S]) + py);
    if (corr) {
        o0 = T(0.5) * (arr(a.trace, d, T_UN)[C] + o0);
        o1 = T(0.5) * (arr(a.trace, d, T_UN + 1)[C] + o1);
        o2 = T(0.5) * (arr(a.trace, d, T_UN + 2)[C] + o2);
    }
    arr(a.trace, d, dst)[C] = o0;
    arr(a.trace, d, dst + 1)[C] = o1;
    arr(a.trace, d, dst + 2)[C] = o2;
}

// S13 + S14: U^d = U^c + D, then point-implicit friction of wet cells.
template <typename T>
__global__ void k_s13(UnfusedArgs<T> a) {
    if (step_is_noop(a.ctl, a.t_end)) return;
    const Pad d = pad_of(a.P);
    const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y;
    if (i >= d.nx || j >= d.ny) return;
    const long long C = d.at(i, j);
    for (int v = 0; v < 3; ++v)
        arr(a.trace, d, T_UD + v)[C] = arr(a.trace, d, T_UC + v)[C] + arr(a.trace, d, T_D + v)[C];
}

template <typename T>
__global__ void k_s14(UnfusedArgs<T> a) {
    if (step_is_noop(a.ctl, a.t_end)) return;
    const Pad d = pad_of(a.P);
    const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y;
    if (i >= d.nx || j >= d.ny) return;
    const long long C = d.at(i, j);
    const T e = arr(a.trace, d, T_UD)[C];
    T qx = arr(a.trace, d, T_UD + 1)[C], qy = arr(a.trace, d, T_UD + 2)[C];
    const T h = e - a.zp[C];
    if (h > T(a.P.h_dry)) manning(T(a.ctl->dt), a.mp[C], trcp(h), qx, qy);
    arr(a.trace, d, T_UF)[C] = e;
    arr(a.trace, d, T_UF + 1)[C] = qx;
    arr(a.trace, d, T_UF + 2)[C] = qy;
}

// S15: dry fix; writes U^{n+1} padded (trace) and pitched (state), and one
// clipped-depth partial per block.
template <typename T>
__global__ void k_s15(UnfusedArgs<T> a) {
    if (step_is_noop(a.ctl, a.t_end)) return;
    const Pad d = pad_of(a.P);
    const int i = blockIdx.x * kWave + threadIdx.x;
    const int j0 = blockIdx.y * kRB;
    const T hdry = T(a.P.h_dry);
    double def = 0.0;
    unsigned flags = 0u;
    if (i < d.nx) {
        for (int j = j0; j < min(j0 + kRB, d.ny); ++j) {
            const long long C = d.at(i, j);
            T e = arr(a.trace, d, T_UF)[C], qx = arr(a.trace, d, T_UF + 1)[C],
              qy = arr(a.trace, d, T_UF + 2)[C];
            const T z = a.zp[C];
            const T h = e - z;
            if (h < T(0)) {
                def = def + (0.0 - (double)h);
                e = z;
                flags |= FLAG_CLIPPED;
            }
            if (!(e - z > hdry)) {
                qx = T(0);
                qy = T(0);
            }
            if (!tfinite(e) || !tfinite(qx) || !tfinite(qy)) flags |= FLAG_NAN;
            arr(a.trace, d, T_UNEW)[C] = e;
            arr(a.trace, d, T_UNEW + 1)[C] = qx;
            arr(a.trace, d, T_UNEW + 2)[C] = qy;
            const long long o = (long long)j * a.P.pitch + i;
            a.eta1[o] = e;
            a.qx1[o] = qx;
            a.qy1[o] = qy;
        }
    }
    def = wave_sum(def);
    flags = wave_or(flags);
    if (threadIdx.x == 0) {
        a.part_def[blockIdx.y * gridDim.x + blockIdx.x] = def;
        if (flags) atomicOr(&a.ctl->step_flags, flags);
    }
}

// S16 sweep: lam_max (atomic max of the IEEE bits) and one volume partial per
// block; mode 0 also clears the clipped-depth partials (initial scan).
template <typename T>
__global__ void k_scan(Params P, Ctl* ctl, double t_end, const T* eta, const T* qx, const T* qy,
                       const T* z, double* part_def, double* part_vol, int mode) {
    if (mode == 1 && step_is_noop(ctl, t_end)) return;
    const int i = blockIdx.x * kWave + threadIdx.x;
    const int j0 = blockIdx.y * kRB;
    const T hdry = T(P.h_dry), g = T(P.g), idx = T(P.idx), idy = T(P.idy);
    double vol = 0.0;
    T lmax = T(0);
    if (i < P.nx) {
        for (int j = j0; j < min(j0 + kRB, P.ny); ++j) {
            const long long o = (long long)j * P.pitch + i;
            const T h = eta[o] - z[o];
            vol = vol + (double)h;
            if (h > hdry) lmax = lam_acc(lmax, cfl_lambda(h, trcp(h), qx[o], qy[o], g, idx, idy));
        }
    }
    vol = wave_sum(vol);
    const unsigned long long lb = wave_max_u64(lam_to_bits(lmax));
    if (threadIdx.x == 0) {
        const int blk = blockIdx.y * gridDim.x + blockIdx.x;
        part_vol[blk] = vol;
        if (mode == 0) part_def[blk] = 0.0;
        if (lb) atomicMax(&ctl->lam_bits, lb);
    }
}

template <typename T>
__global__ void k_finalize(Params P, Ctl* ctl, double t_end, const double* part_def,
                           const double* part_vol, int nparts, int mode) {
    if (mode == 1 && step_is_noop(ctl, t_end)) return;
    finalize_wave(ctl, P, part_def, part_vol, nparts, sizeof(T) == 4, mode);
}

__global__ void k_begin_call(Ctl* ctl, unsigned* dry, int ndry) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->dt_min = __builtin_inf();
        ctl->dt_max_used = 0.0;
        ctl->call_steps = 0;
        ctl->skipped = 0ull;
    }
    if (dry)
        for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < ndry; k += gridDim.x * blockDim.x)
            dry[k] = 0u;
}

// Control block of a replayed step n with a known dt^n: the values the
// finalisation of step n-1 would have left (dt/dx and dt/dy as dt / dx, dt /
// dy; the inflow at t^n and t^n + dt^n), flags and accumulators cleared.
__global__ void k_replay_ctl(Params P, Ctl* ctl, double t, long long step, double dt) {
    if (threadIdx.x == 0) {
        ctl->t = t;
        ctl->dt = dt;
        ctl->rx = dt / P.dx;
        ctl->ry = dt / P.dy;
        ctl->qin0 = q_inflow(P, t);
        ctl->qin1 = q_inflow(P, t + dt);
        ctl->step = step;
        ctl->flags = 0u;
        ctl->step_flags = 0u;
        ctl->ticket = 0u;
        ctl->lam_bits = 0ull;
        ctl->bad_step = -1;
    }
}

// The next step takes the prescribed dt instead of the one the previous
// finalisation chose: dt, dt/dx, dt/dy and q_in(t^n + dt) as that
// finalisation would have set them for this dt.
__global__ void k_set_dt(Params P, Ctl* ctl, double dt) {
    if (threadIdx.x == 0) {
        ctl->dt = dt;
        ctl->rx = dt / P.dx;
        ctl->ry = dt / P.dy;
        ctl->qin1 = q_inflow(P, ctl->t + dt);
    }
}

__global__ void k_init_ctl(Ctl* ctl, double t, long long step, unsigned flags, double defect) {
    if (threadIdx.x == 0) {
        ctl->t = t;
        ctl->dt = 0.0;
        ctl->rx = ctl->ry = 0.0;
        ctl->qin0 = ctl->qin1 = 0.0;
        ctl->defect = defect;
        ctl->volume = 0.0;
        ctl->lam_max = 0.0;
        ctl->dt_min = __builtin_inf();
        ctl->dt_max_used = 0.0;
        ctl->last_defect_depth = 0.0;
        ctl->step = step;
        ctl->bad_step = -1;
        ctl->call_steps = 0;
        ctl->flags = flags;
        ctl->step_flags = 0u;
        ctl->last_step_flags = 0u;
        ctl->ticket = 0u;
        ctl->lam_bits = 0ull;
        ctl->skipped = 0ull;
    }
}

template <typename T>
__global__ void k_pad_static(Params P, const T* z, const T* m, T* zp, T* mp) {
    const int pi = blockIdx.x * kBX + threadIdx.x, pj = blockIdx.y * kBY + threadIdx.y;
    if (pi >= P.nx + 2 || pj >= P.ny + 2) return;
    const int i = pi - 1, j = pj - 1;
    const bool corner = (i < 0 || i >= P.nx) && (j < 0 || j >= P.ny);
    const int ii = min(max(i, 0), P.nx - 1), jj = min(max(j, 0), P.ny - 1);
    const long long o = (long long)jj * P.pitch + ii;
    const long long s = (long long)pj * (P.nx + 2) + pi;
    zp[s] = corner ? T(0) : z[o];
    mp[s] = corner ? T(0) : m[o];
}

template <typename T>
__global__ void k_manning_m(Params P, const T* n, T* m) {
    const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y;
    if (i >= P.nx || j >= P.ny) return;
    const long long o = (long long)j * P.pitch + i;
    const T nn = n[o];
    m[o] = T(P.g) * (nn * nn);
}

__global__ void k_copy16(uint4* __restrict__ dst, const uint4* __restrict__ src, size_t n) {
    size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; k < n; k += stride) dst[k] = src[k];
}

inline dim3 grid2(int w, int h) { return dim3((w + kBX - 1) / kBX, (h + kBY - 1) / kBY); }

}  // namespace

template <typename T>
hipError_t launch_unfused_step(const UnfusedArgs<T>& a, int sigma, hipStream_t s, bool s16) {
    const int nx = a.P.nx, ny = a.P.ny;
    const dim3 b2(kBX, kBY);
    const long long N = (long long)(nx + 2) * (ny + 2);
    const int b1 = 256;
    const dim3 gN((unsigned)((N + b1 - 1) / b1));
    hipLaunchKernelGGL(k_s1<T>, grid2(nx + 2, ny + 2), b2, 0, s, a);                 // S1
    hipLaunchKernelGGL(k_prim<T>, gN, dim3(b1), 0, s, a, (int)T_UN, (int)T_H);        // S2
    hipLaunchKernelGGL(k_s3<T>, grid2(nx, ny), b2, 0, s, a);                          // S3
    hipLaunchKernelGGL(k_s4<T>, grid2(nx, ny), b2, 0, s, a);                          // S4
    hipLaunchKernelGGL(k_xflux<T>, grid2(nx + 1, ny), b2, 0, s, a, sigma, (int)T_UN, (int)T_H,
                       (int)T_F);                                                     // S5
    hipLaunchKernelGGL(k_yflux<T>, grid2(nx, ny + 1), b2, 0, s, a, sigma, (int)T_UN, (int)T_H,
                       (int)T_G);                                                     // S6
    hipLaunchKernelGGL(k_update<T>, grid2(nx, ny), b2, 0, s, a, sigma, (int)T_UN, (int)T_F,
                       (int)T_G, (int)T_US, false);                                   // S7
    hipLaunchKernelGGL(k_s8<T>, dim3((max(nx, ny) + 255) / 256), dim3(256), 0, s, a); // S8
    hipLaunchKernelGGL(k_prim<T>, gN, dim3(b1), 0, s, a, (int)T_US, (int)T_HS);       // S9
    hipLaunchKernelGGL(k_xflux<T>, grid2(nx + 1, ny), b2, 0, s, a, -sigma, (int)T_US, (int)T_HS,
                       (int)T_FS);                                                    // S10
    hipLaunchKernelGGL(k_yflux<T>, grid2(nx, ny + 1), b2, 0, s, a, -sigma, (int)T_US, (int)T_HS,
                       (int)T_GS);                                                    // S11
    hipLaunchKernelGGL(k_update<T>, grid2(nx, ny), b2, 0, s, a, -sigma, (int)T_US, (int)T_FS,
                       (int)T_GS, (int)T_UC, true);                                   // S12
    hipLaunchKernelGGL(k_s13<T>, grid2(nx, ny), b2, 0, s, a);                         // S13
    hipLaunchKernelGGL(k_s14<T>, grid2(nx, ny), b2, 0, s, a);                         // S14
    const dim3 gr((nx + kWave - 1) / kWave, (ny + kRB - 1) / kRB);
    hipLaunchKernelGGL(k_s15<T>, gr, dim3(kWave), 0, s, a);                           // S15
    if (!s16) return hipGetLastError();
    hipLaunchKernelGGL(k_scan<T>, gr, dim3(kWave), 0, s, a.P, a.ctl, a.t_end,
                       (const T*)a.eta1, (const T*)a.qx1, (const T*)a.qy1, a.z, a.part_def,
                       a.part_vol, 1);                                                // S16
    hipLaunchKernelGGL(k_finalize<T>, dim3(1), dim3(kWave), 0, s, a.P, a.ctl, a.t_end,
                       (const double*)a.part_def, (const double*)a.part_vol,
                       (int)(gr.x * gr.y), 1);
    return hipGetLastError();
}

int unfused_partials(int nx, int ny) {
    return ((nx + kWave - 1) / kWave) * ((ny + kRB - 1) / kRB);
}
int scan_partials(int nx, int ny) { return unfused_partials(nx, ny); }

template <typename T>
hipError_t launch_scan(const Params& P, Ctl* ctl, double t_end, const T* eta, const T* qx,
                       const T* qy, const T* z, double* part_def, double* part_vol, int mode,
                       hipStream_t s) {
    const dim3 gr((P.nx + kWave - 1) / kWave, (P.ny + kRB - 1) / kRB);
    hipLaunchKernelGGL(k_scan<T>, gr, dim3(kWave), 0, s, P, ctl, t_end, eta, qx, qy, z, part_def,
                       part_vol, mode);
    hipLaunchKernelGGL(k_finalize<T>, dim3(1), dim3(kWave), 0, s, P, ctl, t_end,
                       (const double*)part_def, (const double*)part_vol, (int)(gr.x * gr.y),
                       mode);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pad_static(const Params& P, const T* z, const T* m, T* zp, T* mp,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_pad_static<T>, grid2(P.nx + 2, P.ny + 2), dim3(kBX, kBY), 0, s, P, z, m,
                       zp, mp);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_manning_m(const Params& P, const T* n, T* m, hipStream_t s) {
    hipLaunchKernelGGL(k_manning_m<T>, grid2(P.nx, P.ny), dim3(kBX, kBY), 0, s, P, n, m);
    return hipGetLastError();
}

hipError_t launch_begin_call(Ctl* ctl, hipStream_t s, unsigned* dry, int ndry) {
    const int blocks = dry ? std::min(256, std::max(1, (ndry + 255) / 256)) : 1;
    hipLaunchKernelGGL(k_begin_call, dim3(blocks), dim3(256), 0, s, ctl, dry, dry ? ndry : 0);
    return hipGetLastError();
}

hipError_t launch_replay_ctl(const Params& P, Ctl* ctl, double t, long long step, double dt,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_replay_ctl, dim3(1), dim3(kWave), 0, s, P, ctl, t, step, dt);
    return hipGetLastError();
}

hipError_t launch_set_dt(const Params& P, Ctl* ctl, double dt, hipStream_t s) {
    hipLaunchKernelGGL(k_set_dt, dim3(1), dim3(kWave), 0, s, P, ctl, dt);
    return hipGetLastError();
}

hipError_t launch_init_ctl(Ctl* ctl, double t, long long step, unsigned flags, double defect,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_init_ctl, dim3(1), dim3(kWave), 0, s, ctl, t, step, flags, defect);
    return hipGetLastError();
}

// The access pattern of the fused step as a plain stream: five arrays read
// and three written, 16 bytes per lane per array, grid-stride.  The bytes are
// moved as integers (out0 = in0 ^ in3, out1 = in1 ^ in4, out2 = in2), so the
// same kernel serves either precision.  NT: loads and stores carry the
// non-temporal hint.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <bool NT>
__global__ void __launch_bounds__(256) k_stream8(const u32x4* a0, const u32x4* a1, const u32x4* a2,
                                                 const u32x4* a3, const u32x4* a4, u32x4* b0,
                                                 u32x4* b1, u32x4* b2, size_t n16) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n16; k += stride) {
        if (NT) {
            const u32x4 x0 = __builtin_nontemporal_load(a0 + k), x1 = __builtin_nontemporal_load(a1 + k),
                        x2 = __builtin_nontemporal_load(a2 + k), x3 = __builtin_nontemporal_load(a3 + k),
                        x4 = __builtin_nontemporal_load(a4 + k);
            __builtin_nontemporal_store(x0 ^ x3, b0 + k);
            __builtin_nontemporal_store(x1 ^ x4, b1 + k);
            __builtin_nontemporal_store(x2, b2 + k);
        } else {
            const u32x4 x0 = a0[k], x1 = a1[k], x2 = a2[k], x3 = a3[k], x4 = a4[k];
            b0[k] = x0 ^ x3;
            b1[k] = x1 ^ x4;
            b2[k] = x2;
        }
    }
}

hipError_t launch_stream8(const void* const* in, void* const* out, size_t n16, bool nt,
                          hipStream_t s) {
    if (n16 == 0) return hipSuccess;
    int cus = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    const unsigned blocks = (unsigned)(8 * std::max(cus, 1));
    const auto k = nt ? k_stream8<true> : k_stream8<false>;
    hipLaunchKernelGGL(k, dim3(blocks), dim3(256), 0, s, (const u32x4*)in[0], (const u32x4*)in[1],
                       (const u32x4*)in[2], (const u32x4*)in[3], (const u32x4*)in[4],
                       (u32x4*)out[0], (u32x4*)out[1], (u32x4*)out[2], n16);
    return hipGetLastError();
}

hipError_t launch_copy16(void* dst, const void* src, size_t n16, hipStream_t s) {
    if (n16 == 0) return hipSuccess;
    size_t blocks = (n16 + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, s, (uint4*)dst,
                       (const uint4*)src, n16);
    return hipGetLastError();
}

#define SWE_INST(T)                                                                            \
    template hipError_t launch_unfused_step<T>(const UnfusedArgs<T>&, int, hipStream_t, bool);        \
    template hipError_t launch_scan<T>(const Params&, Ctl*, double, const T*, const T*,         \
                                       const T*, const T*, double*, double*, int, hipStream_t); \
    template hipError_t launch_pad_static<T>(const Params&, const T*, const T*, T*, T*,         \
                                             hipStream_t);                                      \
    template hipError_t launch_manning_m<T>(const Params&, const T*, T*, hipStream_t);
SWE_INST(float)
SWE_INST(double)
#undef SWE_INST

}  // namespace swe
