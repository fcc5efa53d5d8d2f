// Launchers of the device kernels (kernels.hip).  All pointers are device
// pointers; complex FP64 vectors are double2 arrays of length n per vector.
#pragma once
#include <hip/hip_runtime.h>
#include <array>
#include <cstdint>
#include <utility>
#include <vector>

namespace klst {
namespace dev {

// Launch choices chosen by the autotuner, kept in a process-wide table keyed by
// (Ny, Nxi, nvec, precision 0 = FP64 / 1 = FP32); 0 = the built-in heuristic.
//   apply_rt: FP64 matrix-core operator row tiles per workgroup (1, 2, 3, 6), or
//             FP32 operator rows per thread (4, 8, 16);
//   apply_nw: FP64 operator wavefronts per workgroup (1, or 4 with an LDS copy of D_x);
//   msplit:   column parts per node of the moment sums (1..8; read from the
//             nvec = 1 entry for every batch size);
//   gemv:     wavefronts per workgroup of the block GEMVs (4, 8, 16; nvec = 1 entry).
// Tile and wave choices leave every result bit-identical; msplit and gemv change
// the order of summation, so a table must be fixed before the solves it serves.
struct Tuning {
  int apply_rt = 0, apply_nw = 0, msplit = 0, gemv = 0;
};
void tune_set(int Ny, int Nxi, int nvec, int prec, const Tuning& t);
bool tune_get(int Ny, int Nxi, int nvec, int prec, Tuning* t);
void tune_erase(int Ny, int Nxi, int nvec, int prec);
void tune_clear();
std::vector<std::pair<std::array<int, 4>, Tuning>> tune_all();
int moment_splits(int Ny, int nvec, int Nxi, int prec);

// Moment partial sums: mom must hold Ny * r * nvec * 9 entries (up to 8 column
// parts; the many-vector operator writes the totals over the parts after them).
void launch_moments(hipStream_t st, const double2* x, int64_t n, int nvec, int Ny, int Nxi, int r,
                    const double* M, double2* mom, const int* skip);
void launch_apply(hipStream_t st, const double2* x, double2* y, int64_t n, int nvec, int Ny, int Nxi,
                  int r, double tre, double tim, double beta, const double* Dx, const double* xix,
                  const double* xiy, const double* nu, const double* U, double2* mom,
                  const int* skip);
void launch_csr_build(hipStream_t st, int64_t* rowptr, int32_t* col, double2* val, int Ny, int Nxi,
                      int r, double beta, const double* Dx, const double* xix, const double* xiy,
                      const double* nu, const double* U, const double* M, int npos, int nneg);
void launch_csr_spmv(hipStream_t st, const int64_t* rowptr, const int32_t* col, const double2* val,
                     const double2* x, double2* y, int64_t n, int Ny, int Nxi, const double* xix,
                     double tre, double tim, const int* skip);
void launch_ilu_apply(hipStream_t st, const double2* x, double2* y, int Ny, int Nxi, int nl,
                      int nblocks, const double2* Fc, const double2* C, const int* skip);
// y = (A - sigma B)^{-1} x in the structured form: line inverses Pinv [nslots][Ny x Ny]
// (column-major; slot s is P^{-1} of node slot_node[s] and, conjugated, of node
// slot_mate[s] when >= 0), capacitance inverse Sinv [(r Ny)^2] (row-major,
// q = j r + a), moment functionals M, coupling columns U, xi_x for the inflow
// rows; mom (one vector of moment partials) and d (r Ny) are scratch.  x and y
// must not overlap.
void launch_structured_inverse(hipStream_t st, const double2* x, double2* y, int Ny, int Nxi, int r,
                               const double2* Pinv, const int* slot_node, const int* slot_mate, int nslots,
                               const double2* Sinv, const double* M, const double* U, const double* xix,
                               double2* mom, double2* d, const int* skip);
void launch_structured_inverse(hipStream_t st, const float2* x, float2* y, int Ny, int Nxi, int r,
                               const float2* Pinv, const int* slot_node, const int* slot_mate, int nslots,
                               const float2* Sinv, const float* M, const float* U, const float* xix,
                               float2* mom, float2* d, const int* skip);
// Device set-up of the structured inverse at shift sigma = (sre, sim): the line
// blocks of the nslots stored slots built and inverted into Pinv [nslots][Ny x
// Ny] (column-major), the capacitance S = I - M P^{-1} Ut assembled from
// kCapParts partial sums (part: kCapParts (r Ny)^2 entries of scratch, reused
// for the inversion's second buffer and pivot list) and inverted into Sinv
// [(r Ny)^2] (row-major) by one Gauss-Jordan pivot step per launch.  slot_of / conj_of [Nxi]: node k's
// slot and whether it is the slot's mirrored node.  Dx row-major.
// status [1 + nslots]: status[0] = 1 for a singular capacitance, status[1 + s]
// = 1 for a singular line block of slot s.  Needs 2 (r Ny) x 16 + (r Ny) x 4
// bytes of LDS (r Ny <= 2048).
constexpr int kCapParts = 4;
void launch_structured_setup(hipStream_t st, double2* Pinv, double2* Sinv, double2* part, int Ny, int Nxi, int r,
                             const int* slot_node, int nslots, const int* slot_of, const int* conj_of,
                             const double* Dx, const double* xix, const double* xiy, const double* nu,
                             const double* U, const double* M, double beta, double sre, double sim,
                             int* status);
// y = P^{-1} x: one pass of the structured inverse's line inverses alone (no
// moment coupling), as above.
void launch_line_inverse(hipStream_t st, const double2* x, double2* y, int Ny, int Nxi, int r,
                         const double2* Pinv, const int* slot_node, const int* slot_mate, int nslots,
                         const double* U, const double* xix);
void launch_blockinv_apply(hipStream_t st, const double2* x, double2* y, int Ny, int Nxi, int nl,
                           int nblocks, const double2* Kinv, const int64_t* koff, const int* skip);
void launch_subm(hipStream_t st, const double2* s0, int m0, const double2* s1, int m1,
                 const double2* c, double2* x, double2* dst, int64_t n, double sign, const int* skip);
void launch_combine(hipStream_t st, const double2* S, int m, int64_t n, const double2* coef, int ldc,
                    int k, double2* out, const int* count);
// x (or dst) = x / sqrt(nrm2); dst32, when given, also receives the result in FP32
void launch_scale_rsqrt(hipStream_t st, double2* x, double2* dst, int64_t n, const double2* nrm2,
                        const int* skip, float2* dst32 = nullptr);
void launch_axpby(hipStream_t st, const double2* x, double2* y, int64_t n, double are, double aim,
                  int accum);
// *skip_out = done || ||x||^2 after a Gram-Schmidt pass (norm partials of the
// pass's k_subm_fused over n) >= eta2 x ||x||^2 before it (row m of the with_norm
// dot partials): the DGKS test for a second pass.
void launch_reorth_test(hipStream_t st, const double2* partial, int m, int nch, int64_t n,
                        const double2* norm_part, double eta2, const int* done, int* skip_out);
// First cycle (first != 0): *beta = ||r0||; later restart cycles keep it.
void launch_gmres_init(hipStream_t st, const double2* nrm2, double2* g, int* done, int* steps,
                       double* beta, int first);
void launch_gmres_solve(hipStream_t st, const double2* H, int ldh, const double2* g, const int* steps,
                        double2* yk);
void launch_mask_bc(hipStream_t st, const double2* x, double2* y, int64_t n, int Ny, int Nxi,
                    const double* xix);
void launch_set_int(hipStream_t st, int* p, int v);
// Macroscopic perturbations of nvec vectors x: macros [nvec][Ny][5] complex (rho,
// u, v, E, T hats), umag [nvec][Ny] = |U_hat| / max_j |U_hat|; mom is scratch of
// Ny * r * nvec * 8 entries, base [Ny][rho, u, E, T].  nvec <= 65535.
void launch_perturbation_macros(hipStream_t st, const double2* x, int64_t n, int nvec, int Ny, int Nxi, int r,
                                const double* M, double2* mom, const double* base, double2* macros,
                                double* umag);
// One RK4 stage (1..4) of the BE-BGK relaxation over all nodes; state q
// [(2 j + f) Nxi + k]; kprev (nullptr at stage 1) and a form the stage state;
// kout, acc and (stage 4) qout as documented at the kernel; resid optional
// [Ny * bgk_parts(Nxi)] (per-workgroup max |kout|).
int bgk_parts(int Nxi);
void launch_bgk_stage(hipStream_t st, const double* q, const double* kprev, double a, double* kout, double* acc,
                      double* qout, double dt6, int stage, int Ny, int Nxi, int Dv, const double* xix,
                      const double* xiy, const double* w, const double* inv_dx, double nu_inf, double s_visc,
                      double* resid);
// Non-equilibrium level of the base g per node (gc == nullptr: an EQ base, zeros).
void launch_noneq_level(hipStream_t st, const double* gc, const double* base, const double* xix,
                        const double* xiy, const double* w, int Ny, int Nxi, int Dv, double* eneq);

// ---- FP32 overloads (mixed-precision inner solve); coefficients stay FP64 ----
void launch_moments(hipStream_t st, const float2* x, int64_t n, int nvec, int Ny, int Nxi, int r,
                    const float* M, float2* mom, const int* skip);
void launch_apply(hipStream_t st, const float2* x, float2* y, int64_t n, int nvec, int Ny, int Nxi,
                  int r, double tre, double tim, double beta, const float* Dx, const float* xix,
                  const float* xiy, const float* nu, const float* U, float2* mom,
                  const int* skip);
void launch_blockinv_apply(hipStream_t st, const float2* x, float2* y, int Ny, int Nxi, int nl,
                           int nblocks, const float2* Kinv, const int64_t* koff, const int* skip);
void launch_subm(hipStream_t st, const float2* s0, int m0, const float2* s1, int m1,
                 const double2* c, float2* x, float2* dst, int64_t n, double sign, const int* skip);
void launch_combine(hipStream_t st, const float2* S, int m, int64_t n, const double2* coef, int ldc,
                    int k, float2* out, const int* count);
// FP32-stored vectors combined into FP64 outputs
void launch_combine(hipStream_t st, const float2* S, int m, int64_t n, const double2* coef, int ldc,
                    int k, double2* out, const int* count);
void launch_scale_rsqrt(hipStream_t st, float2* x, float2* dst, int64_t n, const double2* nrm2,
                        const int* skip);
void launch_axpby(hipStream_t st, const float2* x, float2* y, int64_t n, double are, double aim,
                  int accum);
// out_v = R conj(x_v) for nvec vectors of length n: entry (j, f, k) is the
// conjugate of entry (j, f, mk[k]) (mk: the xi_y reflection of the nodes).
void launch_mirror_conj(hipStream_t st, const double2* x, double2* out, int64_t n, int nvec, int Nxi,
                        const int* mk);
// precision conversion of n complex entries: y32 = x64; y64 = x32 (+ y64 if accum)
void launch_narrow(hipStream_t st, const double2* x, float2* y, int64_t n);
void launch_widen(hipStream_t st, const float2* x, double2* y, int64_t n, int accum);

// ---- two-phase reductions (partials + consumer-side fixed-order reduction) ----
// Returns the number of chunks (columns of the partial table) for the consumer.
int launch_dot_partial(hipStream_t st, const double2* s0, int m0, const double2* s1, int m1,
                       const double2* x, int64_t n, double2* partial, int with_norm, const int* skip);
int launch_dot_partial(hipStream_t st, const float2* s0, int m0, const float2* s1, int m1,
                       const float2* x, int64_t n, double2* partial, int with_norm, const int* skip);
// FP32-stored vectors against an FP64 x, FP64 arithmetic
int launch_dot_partial(hipStream_t st, const float2* s0, int m0, const float2* s1, int m1,
                       const double2* x, int64_t n, double2* partial, int with_norm, const int* skip);
void launch_dot_reduce(hipStream_t st, const double2* partial, int m, int nch, double2* out, int mode,
                       const double2* Hinv, double2* out2, const int* skip);
void launch_subm_fused(hipStream_t st, const double2* s0, int m0, const double2* s1, int m1,
                       const double2* partial, int nch, const double2* Hinv, double2* coef_set,
                       double2* coef_add, double2* x, int64_t n, double2* norm_part, const int* skip);
void launch_subm_fused(hipStream_t st, const float2* s0, int m0, const float2* s1, int m1,
                       const double2* partial, int nch, const double2* Hinv, double2* coef_set,
                       double2* coef_add, float2* x, int64_t n, double2* norm_part, const int* skip);
// FP32-stored vectors subtracted from an FP64 x, FP64 arithmetic
void launch_subm_fused(hipStream_t st, const float2* s0, int m0, const float2* s1, int m1,
                       const double2* partial, int nch, const double2* Hinv, double2* coef_set,
                       double2* coef_add, double2* x, int64_t n, double2* norm_part, const int* skip);
void launch_scale_norm(hipStream_t st, double2* x, double2* dst, int64_t n, const double2* norm_part,
                       double2* nrm2_out, double2* H, int ldh, int j, double* cs, double2* sn, double2* g,
                       int* done, int* steps, const double* beta, double rtol);
void launch_scale_norm(hipStream_t st, float2* x, float2* dst, int64_t n, const double2* norm_part,
                       double2* nrm2_out, double2* H, int ldh, int j, double* cs, double2* sn, double2* g,
                       int* done, int* steps, const double* beta, double rtol);
// FP64 x normalised in place, its FP32 copy written to dst32
void launch_scale_norm(hipStream_t st, double2* x, float2* dst32, int64_t n, const double2* norm_part,
                       double2* nrm2_out, double2* H, int ldh, int j, double* cs, double2* sn, double2* g,
                       int* done, int* steps, const double* beta, double rtol);

}  // namespace dev
}  // namespace klst
