// Internal declarations shared by the kernels (rm_kernels.hip) and the C-ABI host
// code (rm_api.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "rm_geometry.h"

namespace rmk {

// Output tile of the one-step kernels: TX columns (one wave64 wide) by TY rows,
// computed by a workgroup of WG = 256 threads (4 waves, each thread owns one
// column and TY/4 rows).
constexpr int TX = 64;
constexpr int WG = 256;
constexpr int TY = 32;

// One entry of a plan's tile table.  inst < 0 marks padding (the table length is
// a multiple of 8 so that the XCD-aware block remap is a bijection).
struct Tile {
  int32_t inst, x0, y0, pad;
};

// Per-instance layout: packed offset, size, and the [tile_begin, tile_end) range
// of its tiles in the full tile table.
struct Inst {
  int64_t off;
  int32_t n;
  int32_t tile_begin;
  int32_t tile_end;
  int32_t pad;
};

// Table-1 schemes (values equal rm_method).
enum { M_RICH = 0, M_NAG = 1, M_MOM = 2, M_NAGEX = 3 };
constexpr bool uses_momentum(int method) { return method != M_RICH; }
constexpr bool uses_lookahead(int method) { return method == M_NAG || method == M_NAGEX; }

// Device-side view of a plan.
struct PlanDev {
  const Tile* tiles;    // full tile table (padded)
  int32_t ntiles;       // padded length
  const Inst* inst;     // [B]
  int32_t B;
  const float* coef32;  // [B][8]: slots 0..4 stencil, slot 5 = 1 / centre (Jacobi)
  const double* coef64; // [B][8], same layout
  const float* mu;      // [B][2]  (log10 eps, theta) or (0, kappa)
  const float* gersh;   // [B]
  int32_t jacobi;       // 1: weighted-Jacobi preconditioning, omega scaled by 1 / centre
};

// Per-step factors of a Table-1 scheme for instance b, weight index i: the weight
// (times 1/D under Jacobi preconditioning), the momentum factor and the look-ahead
// factor (NAG: the momentum factor; NAGex: the second half of alpha, [2][B][m]).
template <typename T, int METHOD>
__device__ __forceinline__ void step_factors(const PlanDev& p, const float* omega, const float* alpha, int m,
                                             int b, int i, T& w, T& a, T& at) {
  w = (T)omega[b * m + i];
  if (p.jacobi) w = w * (sizeof(T) == 4 ? (T)p.coef32[b * 8 + 5] : (T)p.coef64[b * 8 + 5]);
  a = uses_momentum(METHOD) ? (T)alpha[b * m + i] : T(0);
  at = METHOD == M_NAG ? a : (METHOD == M_NAGEX ? (T)alpha[(p.B + b) * m + i] : T(0));
}

// ---- launchers (all asynchronous on `st`) ---------------------------------
// y = A x                                      (dtype float or double)
template <typename T>
void launch_apply(const PlanDev& p, const Tile* tiles, int ntiles, const T* x, T* y, hipStream_t st);
// r = b - A x (r may be null) with per-tile partial sums of ||r||^2 and ||b||^2
template <typename T>
void launch_residual(const PlanDev& p, const Tile* tiles, int ntiles, const T* b, const T* x, T* r,
                     double* partial2, const int* active, hipStream_t st);
// one fused inner step of a Table-1 scheme (method M_RICH, M_NAG, M_MOM or M_NAGEX)
template <typename T>
void launch_step(int method, const PlanDev& p, const Tile* tiles, int ntiles, const float* omega,
                 const float* alpha, int m, int i, const T* f, const T* u, const T* v, T* u_out,
                 T* v_out, const int* active, hipStream_t st);
// per-instance fixed-order sums of per-tile partials over the instance's tiles t:
// out0[b*stride] = sum_t partial2[2t], out1[b*stride] = sum_t partial2[2t+1],
// ratio[b] = out0 / out1 as float (any output may be null).  The tiles of instance b are
// [ranges[2b], ranges[2b+1]) when ranges is given, else its range in the plan's tile table.
void launch_reduce_partials(const PlanDev& p, const double* partial2, double* out0, double* out1,
                            int stride, float* ratio, hipStream_t st, const int* ranges = nullptr);
// FP64 refinement: r = b - A x, r32 = fl32(r), d = v = 0, partials of ||r||^2, ||b||^2
void launch_refine_residual(const PlanDev& p, const double* b, const double* x, float* r32,
                            float* d, float* v, double* partial2, const int* round_mask,
                            hipStream_t st);
// x += d for instances with round_mask[b] != 0; d is d0 or d1 depending on the parity of
// (start[b] + outer_count[b]) * flips (the solve swaps its two buffers `flips` times per
// outer iteration, and the instance's round began at outer iteration start[b] of the solve;
// start may be null: 0)
void launch_refine_update(const PlanDev& p, double* x, const float* d0, const float* d1, const int* start,
                          const int* outer_count, int flips, const int* round_mask, hipStream_t st);
// Per-instance refinement state of the refined solve (device arrays of length B; history
// [max_rounds + 1][B]).
struct RoundState {
  int *pending, *active, *status, *round, *strikes, *start, *tot, *count, *since, *gains;
  double *prev_rho, *relres, *history, *target2, *rhs2, *best2;
};
struct RoundParams {
  double tol, tol_inner;
  int max_rounds, start;
};
// The decision at the end of each waiting instance's round (k_round_decide): from the
// refinement residual's partials (one-step tile table), record rho, finish the instance or
// start its next inner solve at outer iteration rp.start.
void launch_round_decide(const PlanDev& p, const double* partial2, const RoundParams& rp, RoundState rs,
                         hipStream_t st);
// Inner-solve bookkeeping after one outer iteration, two launches: res2[b] = the sum of the
// instance's residual partials (one wave per instance, the order of
// launch_reduce_partials), then for active
// instances the outer count, divergence / target / cap / stagnation tests and the new
// active flag, and *n_active = the number still active.  The partial slots of instance b
// are [r[2b], r[2b+1]) with r = tranges when bit cls[b] of tailmask is set (its class ran
// its tail configuration), else ranges; with ranges null, its range in the plan's tile
// table.  With host_word (pinned host memory, may be null) the count is also published
// there as one 64-bit word, (seq << 32) | count, so a host thread that reads the word
// knows which launch wrote it; host_cnt (pinned, may be null) receives the active
// instances of each of the ncls classes as words of the same form (cls may be null when
// ncls <= 1).  With pending given, an instance whose inner solve ends sets pending[b] and
// counts as not done (so do instances already waiting); host_word[1] then receives the
// count of waiting instances, and the counts above include them.
// With hist given, an active instance also stores res2 at hist[k * B + b], k = tot[b] + (its
// outer count in this round) - 1, when k < hist_len.
void launch_outer_flags(const PlanDev& p, const double* partial2, const int* ranges, const int* tranges,
                        const int* cls, unsigned long long tailmask, int ncls, double* res2, const double* rhs2,
                        const double* target2, double* best2, int* since, int* gains, int stall_min, int stall_max,
                        int cap, int* active, int* outer_count, int* status, int* pending, int* n_active,
                        unsigned long long* host_word, unsigned long long* host_cnt, unsigned seq,
                        const int* tot, double* hist, int hist_len, hipStream_t st);
void launch_fill_i32(int* p, int value, int64_t count, hipStream_t st);
void launch_fill_f32(float* p, float value, int64_t count, hipStream_t st);
void launch_fill_f64(double* p, double value, int64_t count, hipStream_t st);
// adjoint: terminal values of the squared-relative-residual loss
void launch_adj_terminal(const PlanDev& p, const float* b, const float* rK, const double* r2b2,
                         const float* g_loss, float* ub, float* fb, float* loss, hipStream_t st);
// adjoint: one reverse step (see rm_solve_adjoint); partial4 gets per tile
// <g, r_s>, <g, v>, <ut_bar, v> (4 doubles per slot)
void launch_adj_step(int method, const PlanDev& p, const float* omega, const float* alpha, int m,
                     int i, const float* f, const float* u, const float* v, const float* ub,
                     const float* vb, float* ub_out, float* vb_out, float* fb, double* partial4,
                     hipStream_t st);
// After the reverse steps of one checkpoint segment (steps s = s_first .. s_first + E - 1,
// whose tile partials sit at partial4 + t * 4 * nslot for t = s - s_first): for t from
// E - 1 down to 0 and i = s mod m, sum each component over the instance's tiles and add
// acc_w[b*m + i] += (Jacobi ? 1/D : 1) * <g, r>, the momentum gradient to acc_a
// (NAG: <g, v> + <ut_bar, v>; MOM, NAGex: <g, v>) and, for NAGex, <ut_bar, v> to
// acc_a[(B + b)*m + i].
void launch_adj_accumulate(int method, const PlanDev& p, const double* partial4, int nslot, int E, int s_first,
                           int m, double* acc_w, double* acc_a, hipStream_t st, const int* ranges = nullptr);
void launch_f64_to_f32(const double* src, float* dst, int64_t count, hipStream_t st);
// meta network
void launch_meta_forward(const PlanDev& p, int m, const float* params, float* omega, float* alpha,
                         hipStream_t st);
void launch_meta_backward(const PlanDev& p, int m, const float* params, const float* d_omega,
                          const float* d_alpha, float* per_inst, float* d_params, hipStream_t st);

// ---- temporal-blocked steps (rm_block.hip) ---------------------------------
// Variants, windows and tile tables: rm_geometry.h.
// T fused steps (s0 .. s0 + T - 1) over a table of extended tiles.  Tiles must
// overlap by at least T points at interior edges (T + 1 when partial2 is given,
// which then receives ||f - A u||^2 of the final u over each tile's owned part).
// Returns false for an unsupported (variant, cw).
// With `states` given, the owned state after every step but the last is also stored:
// u at states + t * state_stride, v at states + t * state_stride + state_stride / 2
// (t = 0 .. T - 2), offsets as in the packed vectors.
bool launch_block(int variant, int T, int cw, int method, const PlanDev& p, const BTile* tiles, int ntiles,
                  const float* omega, const float* alpha, int m, int s0, const float* f, const float* u,
                  const float* v, float* u_out, float* v_out, const int* active, double* partial2,
                  hipStream_t st, float* states = nullptr, int64_t state_stride = 0);

// ---- row-streaming temporal-blocked steps (rm_stream.hip) ----------------------
// One workgroup of 64 ceil(n / 64) threads per window of whole rows: tiles carry
// x0 = 0, ox0 = 0, ox1 = n and the window [y0, min(n, y0 + wlen)) with owned rows
// [oy0, oy1); windows overlap by at least T rows at cuts (T + 1 with partial2).
// Same step semantics, partial2 and states layout as launch_block.  Returns false
// when n or T is outside what is built.  The reverse steps (launch_adj_stream) are
// built for n <= kAdjStreamMaxN.
bool launch_stream(int T, int wlen, int n, int method, const PlanDev& p, const BTile* tiles, int ntiles,
                   const float* omega, const float* alpha, int m, int s0, const float* f, const float* u,
                   const float* v, float* u_out, float* v_out, const int* active, double* partial2,
                   hipStream_t st, float* states = nullptr, int64_t state_stride = 0);

// T (1..kStreamMaxT) forward steps of every size class in one launch of kMixedThreads-
// thread workgroups over a group table (rmgeo::make_groups) whose tiles are the
// classes' row-pipeline tables; the groups of a class with bit c set in leave_out do
// nothing (c < 64).  Results, residual partials and slots as with launch_stream.
bool launch_stream_mixed(int T, int method, const PlanDev& p, const BTile* tiles, const MGroup* groups, int ngroups,
                         unsigned long long leave_out, const float* omega, const float* alpha, int m, int s0,
                         const float* f, const float* u, const float* v, float* u_out, float* v_out,
                         const int* active, double* partial2, hipStream_t st);

// Up to kAdjMaxT reverse steps per launch over a row-streaming tile table (windows
// overlapping by at least T + 1 rows).  Level l = 1..T reverses the forward step whose
// state (before the step) is u[l - 1], v[l - 1] and whose weight index is i[l - 1]
// (consecutive levels go back in time); ub, vb are the adjoints after the latest step
// and ub_out, vb_out receive them before the earliest one; fb (may be null) gets
// w g added per step in place; part[l - 1] + 4 slot receives the window's
// <g, r>, <g, v>, <utb, v>, 0 for level l (as launch_adj_step's partial4).
struct AdjLevels {
  const float* u[kAdjMaxT];
  const float* v[kAdjMaxT];
  double* part[kAdjMaxT];
  int i[kAdjMaxT];
};
bool launch_adj_stream(int T, int wlen, int n, int method, const PlanDev& p, const BTile* tiles, int ntiles,
                       const float* omega, const float* alpha, int m, const AdjLevels& lev, const float* f,
                       const float* ub, const float* vb, float* ub_out, float* vb_out, float* fb, hipStream_t st);

// ---- SSOR-preconditioned steps (rm_ssor.hip) ----------------------------------
// One inner step of a Table-1 scheme with the four-colour SSOR preconditioner of
// relaxation factor `relax` (0 < relax < 2), over the plan's one-step tile table.
template <typename T>
void launch_ssor_step(int method, const PlanDev& p, const Tile* tiles, int ntiles, const float* omega,
                      const float* alpha, int m, int i, double relax, const T* f, const T* u, const T* v, T* u_out,
                      T* v_out, const int* active, hipStream_t st);
// Reverse of one SSOR-preconditioned step; partial4 as for launch_adj_step, slot 0
// holding <g, B^{-1} r>.
void launch_adj_ssor_step(int method, const PlanDev& p, const float* omega, const float* alpha, int m, int i,
                          double relax, const float* f, const float* u, const float* v, const float* ub,
                          const float* vb, float* ub_out, float* vb_out, float* fb, double* partial4,
                          hipStream_t st);

// ---- batched flexible GMRES (rm_krylov.hip) -----------------------------------
// partial[i * nslot + slot] = per-tile dot of w with V + i * stride, i < nvec (active
// instances only).
void launch_mdot(const PlanDev& p, const double* V, int64_t stride, int nvec, const double* w, const int* active,
                 double* partial, int nslot, hipStream_t st);
// out[b * ldo + col0 + i] = (or +=) the instance's sum of those partials, in tile order.
void launch_mreduce(const PlanDev& p, const double* partial, int nvec, int nslot, const int* active, double* out,
                    int ldo, int col0, bool accumulate, hipStream_t st);
// w -= sum_i h[b * ldh + col0 + i] (V + i * stride).
void launch_maxpy(const PlanDev& p, const double* V, int64_t stride, int nvec, const double* h, int ldh, int col0,
                  double* w, const int* active, hipStream_t st);
// dst = src / sqrt(nrm2[b * ldn]) (0 for a zero norm).
void launch_scale(const PlanDev& p, const double* src, const double* nrm2, int ldn, double* dst, const int* active,
                  hipStream_t st);
void launch_f32_to_f64(const float* s, double* d, int64_t count, hipStream_t st);
// dst = fl32(src) for active instances, 0 for the others.
void launch_to_f32_masked(const PlanDev& p, const double* src, float* dst, const int* active, hipStream_t st);
// Per-instance cycle start, Givens step, back substitution and x += Z y; H is
// [B][restart columns][restart + 1], g [B][restart + 1], cs, sn, y [B][restart].
void launch_fgm_start(int B, const double* r2b2, double tol, int max_iter, const int* iters, int* running,
                      int* active, int* status, double* relres, double* g, int ldg, int* jdone, hipStream_t st);
void launch_fgm_givens(int B, int j, int restart, double* H, const double* hn2, double* cs, double* sn, double* g,
                       const double* r2b2, double tol, int max_iter, int* iters, int* jdone, int* active, double* est,
                       hipStream_t st);
void launch_fgm_backsolve(int B, int restart, const double* H, const double* g, const int* jdone, double* y,
                          hipStream_t st);
void launch_fgm_xupdate(const PlanDev& p, const float* Z, int64_t stride, const double* y, int restart,
                        const int* jdone, double* x, hipStream_t st);

// ---- two-grid correction (rm_twogrid.hip) -------------------------------------
// Largest FFT length n + 1 of the coarse sine transform.
constexpr int kTgMaxFFT = 1024;

// Per-instance coarse layout: packed offset of the nc x nc coarse field, nc,
// log2(n + 1) and the orthonormal DST scale 1 / sqrt(n + 1).
struct TgInst {
  int64_t coff;
  int32_t nc, lg;
  float scale;
  int32_t pad;
};

struct TgDev {
  const TgInst* inst;  // [B]
  const float2* tw;    // [kTgMaxFFT / 2]: exp(-2 pi i k / kTgMaxFFT)
};

// mode 0: rc = scale * R (f - A u), the residual in FP64;  mode 1: rc = scale * R u.  tiles: 64 x 8 coarse
// points each (x0, y0 coarse), table length a multiple of 8.
void launch_tg_restrict(int mode, const PlanDev& p, const TgDev& g, const Tile* tiles, int ntiles, const float* f,
                        const float* u, float* rc, float scale, hipStream_t st);
// Sine-transform passes over groups of 8 coarse rows (y0 = first row); mmax is the
// largest n + 1 among the instances of the launch (sizes the LDS):
// pass 0: in[J][I] -> out[p][J];  pass 2: in[p][J] -> out[J][I];
// pass 1: in[p][J] -> [p][q]; shat_out given: store it and stop; else
//         dsym[q][p] += coef * shat[p][q] (if dsym), coef *= symbol[q][p] (if symbol),
//         and transform back -> out[p][J] (out may equal in).
void launch_tg_dst(int pass, const TgDev& g, const Tile* groups, int ngroups, int mmax, const float* in, float* out,
                   const float* symbol, const float* shat, float* shat_out, float* dsym, hipStream_t st);
// uo = ui + P ec (uo may equal ui), over the plan's fine tile table.
void launch_tg_prolong(const PlanDev& p, const TgDev& g, const float* ec, const float* ui, float* uo,
                       hipStream_t st);
// ub_out = ub - A R^T ybar (R^T = P / 4, stencil summed in FP64) and fb += R^T ybar
// (fb may be null); ub_out must not alias ub.
void launch_tg_adj_correct(const PlanDev& p, const TgDev& g, const float* ybar, const float* ub, float* ub_out,
                           float* fb, hipStream_t st);

// ---- symbol network of the two-grid cycle (rm_symbolnet.hip) --------------------
int symbolnet_param_count();
// symbol = base * exp(net(features)) over 16 x 16 mode tiles (tiles[k].pad = k); a1, a2:
// [16][Pc] activations kept for the backward pass.
void launch_symbolnet_forward(const PlanDev& p, const TgDev& g, const Tile* tiles, int ntiles, int64_t Pc,
                              const float* params, float* a1, float* a2, float* symbol, hipStream_t st);
// d_params = gradient of sum(d_symbol * symbol) (a1, a2, symbol from the forward pass with
// the same params; gz [Pc], g1, g2 [16][Pc], part [ntiles][2320] and gsum
// [ceil(ntiles / 64)][2320] doubles are scratch).
void launch_symbolnet_backward(const PlanDev& p, const TgDev& g, const Tile* tiles, int ntiles, int64_t Pc,
                               const float* params, const float* a1, const float* a2, const float* symbol,
                               const float* d_symbol, float* gz, float* g1, float* g2, float* part, double* gsum,
                               float* d_params, hipStream_t st);

}  // namespace rmk
