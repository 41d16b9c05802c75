// swe_internal.hpp -- launch interfaces between the C ABI layer and the
// kernels of libswe (not part of the public interface).
#pragma once

#include <hip/hip_runtime.h>
#include "swe_common.hpp"

namespace swe {

// Arguments of the fused step kernel.
template <typename T>
struct FusedArgs {
    Params P;
    Ctl* ctl;
    double t_end;
    const T* eta;
    const T* qx;
    const T* qy;
    const T* z;
    const T* m;
    T* eta1;
    T* qx1;
    T* qy1;
    TilePart* tpart;    // one record per tile (tile index)
    TilePart* gpart;    // one record per group of kGroup tiles
    unsigned* gticket;  // per group: members finished this step (0 between steps)
    int gy;             // chunks along y
    int H;              // output rows per chunk
    // Dry-tile skip: NULL (off), or two flag words per tile (one set per step
    // parity, tile index strip * gy + chunk), cleared at the start of every
    // host call.
    unsigned* dry = nullptr;
    // when not NULL, the step's finalisation stores dt^n and t^n (the step's
    // own time step and start time) here
    double* log_dt = nullptr;
    double* log_t = nullptr;
    // launch_fused_trace only: U* and U^d of every cell (pitched, 3 fields each)
    T* tus[3] = {nullptr, nullptr, nullptr};
    T* tud[3] = {nullptr, nullptr, nullptr};
    // the split step (two waves per tile): polls after which a wave stops
    // waiting for the other and the step raises FLAG_STALL
    int spin_cap = kSplitSpinCap;
};

// more_waves: the occupancy variant (one more resident wave per SIMD, some
// of the carried state in scratch; not with the dry-tile skip).
// split: two waves per tile, one running the predictor half (S2..S7) and one
// the corrector half (S9..S16) of every row, rows handed over through LDS
// (not with more_waves); the same state bits as one wave per tile.
template <typename T>
hipError_t launch_fused(const FusedArgs<T>& a, int sigma, hipStream_t s, bool more_waves = false,
                        bool split = false);
// The FP64 fused step that also writes U* (after S7) and U^d (after S13,
// before friction) of every cell to a.tus and a.tud (one wave per tile).
hipError_t launch_fused_trace(const FusedArgs<double>& a, int sigma, hipStream_t s);
// One fused step of every scenario of an ensemble in one launch: scenario s
// owns workgroups first[s] .. first[s+1]-1 of `total` (args, first: device).
// dry: some scenario has the dry-tile skip on (its args carry the flags).
// split: two waves per tile (FP32 only; FP64 keeps one wave per tile; a
// measured variant, not the default).
template <typename T>
hipError_t launch_ensemble(const FusedArgs<T>* args, const int* first, int count, int total,
                           int sigma, bool dry, hipStream_t s, bool split = false);
int fused_blocks(int nx, int ny, int H);
// Bytes of the fused path's partial-result buffer for up to `ntiles` tiles
// (tile records, group records, group tickets; zero it before first use).
size_t fused_part_bytes(int ntiles);
// Carve that buffer into the three arrays of FusedArgs.
template <typename T>
void fused_part_layout(FusedArgs<T>& a, void* buf, int ntiles);
int fused_strips(int nx);
// Resident fused workgroups (one wave each) per compute unit, or 0.
template <typename T>
int fused_waves_per_cu(bool more_waves = false);
// Resident two-wave workgroups (tiles) of the split step per compute unit, or 0.
template <typename T>
int fused_split_tiles_per_cu();
// Automatic tile height of the fused step for `slots` resident waves: as
// many chunks per strip as fit one round of waves, at least 6 rows; with
// the dry-tile skip at most 32.
int fused_auto_rows(int nx, int ny, long long slots, bool dry_skip);

// Access-pattern probe of the fused step (k_probe_march): in[0..4] read,
// out[0..2] written, nx x ny elements at `pitch`, chunks of H rows (gy per
// strip).
struct ProbeMarchArgs {
    const void* in[5];
    void* out[3];
    int nx, ny, H, gy;
    long long pitch;
};
hipError_t launch_probe_march(const ProbeMarchArgs& a, int elem_bytes, hipStream_t s);
// The tile height k_fused_step picks by itself on a device of `cus` compute
// units for an nx x ny grid of elem_bytes-byte elements.
int probe_march_rows(int elem_bytes, int nx, int ny, int cus);

// Arguments of the unfused path: the trace block holds the 47 padded arrays
// in trace order; zp/mp are the padded static fields.
template <typename T>
struct UnfusedArgs {
    Params P;
    Ctl* ctl;
    double t_end;
    const T* eta;       // U^n (pitched)
    const T* qx;
    const T* qy;
    const T* z;         // pitched
    T* eta1;            // U^{n+1} (pitched)
    T* qx1;
    T* qy1;
    T* trace;           // 47 * (nx+2) * (ny+2)
    const T* zp;        // padded
    const T* mp;
    double* part_def;
    double* part_vol;
};

constexpr int kTraceArrays = 47;

template <typename T>
// s16 = false leaves out S16 (the CFL scan and the dt finalisation): a replay
// of a step whose dt is already known.
hipError_t launch_unfused_step(const UnfusedArgs<T>& a, int sigma, hipStream_t s, bool s16 = true);
int unfused_partials(int nx, int ny);

// Pad the static fields z and m (= g n^2, already computed) into (nx+2) x
// (ny+2) arrays whose ghost ring copies the adjacent cell.
template <typename T>
hipError_t launch_pad_static(const Params& P, const T* z, const T* m, T* zp, T* mp, hipStream_t s);

// m = g n^2 on the pitched layout.
template <typename T>
hipError_t launch_manning_m(const Params& P, const T* n, T* m, hipStream_t s);

// Initial scan: lam_max and volume of the state, then dt^0 (mode 0) -- also
// the S16 sweep of the unfused path (mode 1).
template <typename T>
hipError_t launch_scan(const Params& P, Ctl* ctl, double t_end, const T* eta, const T* qx,
                       const T* qy, const T* z, double* part_def, double* part_vol, int mode,
                       hipStream_t s);
int scan_partials(int nx, int ny);

// Reset the per-call statistics (dt_min, dt_max_used, call_steps, skipped
// cells) and, when `dry` is not NULL, clear its `ndry` flag words.
hipError_t launch_begin_call(Ctl* ctl, hipStream_t s, unsigned* dry = nullptr, int ndry = 0);
// Control block of a replayed step n whose dt^n is known: t, n, dt, dt/dx,
// dt/dy and the inflow values set as the finalisation of step n-1 sets them.
hipError_t launch_replay_ctl(const Params& P, Ctl* ctl, double t, long long step, double dt,
                             hipStream_t s);
// Bandwidth probe with the fused step's access pattern: 5 arrays of n16
// 16-byte vectors read, 3 written (nt: non-temporal hints).
hipError_t launch_stream8(const void* const* in, void* const* out, size_t n16, bool nt,
                          hipStream_t s);
// The next step takes dt (its dt/dx, dt/dy and q_in(t^n + dt) follow).
hipError_t launch_set_dt(const Params& P, Ctl* ctl, double dt, hipStream_t s);
// Set the control block from host values (t, step, flags, defect) and clear
// the accumulators.
hipError_t launch_init_ctl(Ctl* ctl, double t, long long step, unsigned flags, double defect,
                           hipStream_t s);

// Arguments of the adjoint of one step (FP64): the step's forward data U^n,
// U* and U^d (pitched, as launch_fused_trace writes them), the step's inflow
// values, the padded static fields, and the
// adjoint work arrays (adjoint_work_arrays() padded arrays; lambda in slots
// 15..17 on entry and exit, dJ/dn and dJ/dz accumulators in 18, 19).
struct AdjointArgs {
    Params P;
    double qin0, qin1;       // q_in(t^n) and q_in(t^n + dt) of the step
    const double* un[3];
    const double* us[3];
    const double* ud[3];
    const double* zp;        // padded bed and m = g n^2 (ghosts copy the edge cell)
    const double* mp;
    const double* nman;      // Manning field (pitched)
    double* work;
    double dt, rx, ry;
    int sigma;
    // work-array slots holding the adjoint of U^{n+1} (lambda, before the
    // fold of its ghost ring) and the bed's padded adjoint of the step
    // reversed before this one; the reverse march writes the other slot of
    // each pair (kAdjLamSlot, kAdjZpSlot), the gather kernels keep the first
    int lam_slot = 9, azp_slot = 14;
};

int adjoint_work_arrays();
constexpr int kAdjLambda = 15, kAdjGradN = 18, kAdjGradZ = 19;
constexpr int kAdjLamSlot[2] = {9, 0}, kAdjZpSlot[2] = {14, 12};
// Adjoint of one step.  It first completes the step reversed before it (the
// ghost ring of its U^n adjoint; nothing on the first), then adds this
// step's gauge terms when hobs is not NULL (gmap from launch_gauge_map).
hipError_t launch_adjoint_step(const AdjointArgs& a, const int* gmap, const double* hobs,
                               hipStream_t s);
// The same step as one fused reverse march (one wave per strip of columns,
// chunks of H rows): reads lambda and the bed adjoint from a.lam_slot and
// a.azp_slot, writes them to the other slot of each pair.  The result is bit
// for bit the one launch_adjoint_step gives.  one_wave: one wave per tile;
// barrier: a workgroup of two waves per tile, each forming half of the phases,
// one step apart, in step at a workgroup barrier; flags: the same two waves
// handing rows over through LDS progress counters, the first up to five rows
// ahead.  stall (flags: required, else unused) is a device int the kernel sets
// to 1 if a wave's wait for the other ran out after spin_cap polls (the values
// are then wrong); the caller clears it.
enum class MarchMode { one_wave, barrier, flags };
// Polls (each about 100 cycles) after which a wave of the flag-synchronised
// march stops waiting for the other: some 40 ms, far beyond any row's time.
constexpr int kMarchSpinCap = 1 << 20;
hipError_t launch_adjoint_march(const AdjointArgs& a, const int* gmap, const double* hobs, int H,
                                hipStream_t s, MarchMode mode, int* stall,
                                int spin_cap = kMarchSpinCap);
// Chunk height of the reverse march for a grid on a device with ncu compute
// units.
int adjoint_march_rows(const Params& P, int ncu, int per_cu = 4);
// Whether the reverse march can address the grid's arrays (below about
// 13000 x 13000 cells); launch_adjoint_step serves the others.
bool adjoint_march_fits(const Params& P);
// Completes the last step reversed (lambda and dJ/dz of its ghost ring).
hipError_t launch_adjoint_finish(const AdjointArgs& a, hipStream_t s);
// gmap[j*nx + i] = gauge index of cell (i, j), or -1 (nx*ny ints).
hipError_t launch_gauge_map(const Params& P, const long long* cells, int ngauge, int* gmap,
                            hipStream_t s);
// out[g] = ((eta - z)(cell g) - hobs[g])^2 on a pitched state, in FP64 (an FP32
// state is promoted before the difference).
template <typename T>
hipError_t launch_misfit(const Params& P, const T* eta, const T* z, const long long* cells,
                         int ngauge, const double* hobs, double* out, hipStream_t s);
// dst[k] = (double)src[k], k < n.
hipError_t launch_promote(const float* src, double* dst, size_t n, hipStream_t s);
// Interior of a padded array into a pitched one.
hipError_t launch_unpad(const Params& P, const double* src, double* dst, hipStream_t s);

// Copy `n16` 16-byte words.
hipError_t launch_copy16(void* dst, const void* src, size_t n16, hipStream_t s);

}  // namespace swe
