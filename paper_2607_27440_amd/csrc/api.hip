// C ABI of the kLST library (include/klst.h): context, assembly, operator and
// preconditioner entry points, and the Jacobi-Davidson driver.
//
// The Jacobi-Davidson driver keeps every n-vector in HBM.  The host sees only small projected
// matrices (R, M_B, the partial Schur form), scalars and flags: one host
// synchronisation per expansion and one per residual check.  The GMRES solve of
// the correction equation runs entirely on the device (Hessenberg, Givens
// rotations and early-exit flag in device memory).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <unordered_map>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "host.hpp"
#include "kernels.hpp"
#include "klst.h"

using klst::cd;

struct klst_ctx {
  klst_options opt{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  bool assembled = false;
  klst::Problem prob;
  // device tables
  double *d_Dx = nullptr, *d_DxT = nullptr, *d_xix = nullptr, *d_xiy = nullptr, *d_nu = nullptr,
         *d_U = nullptr, *d_M = nullptr;
  double2* d_mom = nullptr;
  int mom_cap = 0;   // vectors
  int mom32_cap = 0; // vectors the FP32 moment partials hold
  // post-processing: weights, base macros [Ny][rho, u, E, T], NONEQ base g
  double *d_w = nullptr, *d_base = nullptr, *d_gc = nullptr;
  // explicit CSR
  int64_t* d_rowptr = nullptr;
  int32_t* d_col = nullptr;
  double2* d_val = nullptr;
  // preconditioner
  klst::ILU0 ilu;
  double2 *d_F = nullptr, *d_C = nullptr, *d_Kinv = nullptr;
  int64_t* d_koff = nullptr;
  int pc_kernel_built = -1;
  bool pc_ready = false;
  cd pc_sigma = 0.0;
  int pc_lines = 0;
  // FP32 copies for the mixed-precision inner solve
  float *d_Dx32 = nullptr, *d_DxT32 = nullptr, *d_xix32 = nullptr, *d_xiy32 = nullptr, *d_nu32 = nullptr,
        *d_U32 = nullptr, *d_M32 = nullptr;
  float2* d_mom32 = nullptr;
  float2* d_Kinv32 = nullptr;
  // structured exact inverse (pc_kernel 2): line inverses, capacitance inverse, d scratch
  double2 *d_Pinv = nullptr, *d_Sinv = nullptr, *d_capd = nullptr;
  int* d_slots = nullptr;   // [2][nslots]: node, mirrored node (-1: none) per stored line inverse
  int nslots = 0;
  float2 *d_Pinv32 = nullptr, *d_Sinv32 = nullptr, *d_capd32 = nullptr;
  // reductions
  double2* d_partial = nullptr;
  double2* d_npart = nullptr;     // per-workgroup norm partials (<= 2^16 workgroups)
  klst_stats stats{};
  std::vector<double> history;   // per outer iteration: outer, nconv, rel residual, Re/Im theta, shift flag
  const volatile int* cancel = nullptr;   // set by the server: stop the current solve
};

// Moment partial sums of klst_apply_many_noalloc: a file-scope device array, one
// copy per GPU, held until the process ends.  Host code reaches it only through
// the per-device address that klst_create resolves with hipGetSymbolAddress.
constexpr size_t kScratchEntries = (size_t)1 << 19;   // double2 entries (8 MiB)
static __device__ __align__(256) double2 scratch[kScratchEntries];

namespace {

#define HIPCHK(expr)                                                            \
  do {                                                                          \
    hipError_t e_ = (expr);                                                     \
    if (e_ != hipSuccess) {                                                     \
      ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);             \
      return KLST_EDEVICE;                                                      \
    }                                                                           \
  } while (0)

std::mutex g_scratch_mu;
std::vector<double2*> g_scratch_ptr;   // device address of `scratch`, per device ordinal

// Resolve `scratch` on the current device (ordinal dev) once; called by
// klst_create with that device current.
bool resolve_scratch(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (g_scratch_ptr[dev]) return true;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return false;
  }
  g_scratch_ptr[dev] = (double2*)ptr;
  return true;
}

double2* scratch_on(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return (dev >= 0 && dev < (int)g_scratch_ptr.size()) ? g_scratch_ptr[dev] : nullptr;
}

klst_status fail(klst_ctx* ctx, klst_status s, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return s;
}

// Device memory is stream-ordered (hipMallocAsync / hipFreeAsync on the
// context's stream), so a context freeing its buffers never synchronises the
// device under other contexts working concurrently (served mode).
template <class T>
void dfree(klst_ctx* ctx, T*& p) {
  if (p) (void)hipFreeAsync((void*)p, ctx->stream);
  p = nullptr;
}

klst_status dalloc(klst_ctx* ctx, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  const hipError_t e = hipMallocAsync(p, bytes, ctx->stream);
  if (e != hipSuccess) {
    *p = nullptr;
    ctx->err = "hipMalloc(" + std::to_string(bytes) + " bytes) failed: " + hipGetErrorString(e);
    (void)hipGetLastError();
    return KLST_ENOMEM;
  }
  return KLST_OK;
}

#define ALLOC(ptr, bytes)                                                        \
  do {                                                                           \
    klst_status s_ = dalloc(ctx, (void**)&(ptr), (bytes));                       \
    if (s_ != KLST_OK) return s_;                                                \
  } while (0)

void free_problem(klst_ctx* ctx) {
  dfree(ctx, ctx->d_Dx); dfree(ctx, ctx->d_DxT); dfree(ctx, ctx->d_xix); dfree(ctx, ctx->d_xiy); dfree(ctx, ctx->d_nu); dfree(ctx, ctx->d_U);
  dfree(ctx, ctx->d_M); dfree(ctx, ctx->d_mom); dfree(ctx, ctx->d_rowptr); dfree(ctx, ctx->d_col); dfree(ctx, ctx->d_val);
  dfree(ctx, ctx->d_F); dfree(ctx, ctx->d_C); dfree(ctx, ctx->d_Kinv); dfree(ctx, ctx->d_koff);
  dfree(ctx, ctx->d_Dx32); dfree(ctx, ctx->d_DxT32); dfree(ctx, ctx->d_xix32); dfree(ctx, ctx->d_xiy32); dfree(ctx, ctx->d_nu32); dfree(ctx, ctx->d_U32);
  dfree(ctx, ctx->d_M32); dfree(ctx, ctx->d_mom32); dfree(ctx, ctx->d_Kinv32);
  dfree(ctx, ctx->d_Pinv); dfree(ctx, ctx->d_Sinv); dfree(ctx, ctx->d_capd); dfree(ctx, ctx->d_slots);
  dfree(ctx, ctx->d_Pinv32); dfree(ctx, ctx->d_Sinv32); dfree(ctx, ctx->d_capd32);
  dfree(ctx, ctx->d_w); dfree(ctx, ctx->d_base); dfree(ctx, ctx->d_gc);
  ctx->mom_cap = 0;
  ctx->mom32_cap = 0;
  ctx->pc_ready = false;
  ctx->assembled = false;
}

klst_status ensure_mom(klst_ctx* ctx, int nvec) {
  if (ctx->mom_cap >= nvec) return KLST_OK;
  dfree(ctx, ctx->d_mom);
  ALLOC(ctx->d_mom, sizeof(double2) * (size_t)ctx->prob.Ny * ctx->prob.r * nvec * 9);
  ctx->mom_cap = nvec;
  return KLST_OK;
}

// FP32 moment partials for nvec vectors (up to 8 column parts each) and their
// totals (the streaming kernel's input).
klst_status ensure_mom32(klst_ctx* ctx, int nvec) {
  if (ctx->mom32_cap >= nvec) return KLST_OK;
  dfree(ctx, ctx->d_mom32);
  ctx->mom32_cap = 0;
  ALLOC(ctx->d_mom32, sizeof(float2) * (size_t)ctx->prob.Ny * ctx->prob.r * nvec * 9);
  ctx->mom32_cap = nvec;
  return KLST_OK;
}

klst_status ensure_csr(klst_ctx* ctx) {
  if (ctx->d_val) return KLST_OK;
  const klst::Problem& p = ctx->prob;
  const int64_t n = p.n(), nnz = p.nnz();
  if (nnz >= (int64_t)1 << 62) return fail(ctx, KLST_EINVAL, "matrix too large");
  ALLOC(ctx->d_rowptr, sizeof(int64_t) * (n + 1));
  ALLOC(ctx->d_col, sizeof(int32_t) * nnz);
  const klst_status s = dalloc(ctx, (void**)&ctx->d_val, sizeof(double2) * nnz);
  if (s != KLST_OK) {
    dfree(ctx, ctx->d_rowptr); dfree(ctx, ctx->d_col);
    return s;
  }
  int npos = 0, nneg = 0;
  for (int k = 0; k < p.Nxi; ++k) { npos += p.xi_x[k] > 0; nneg += p.xi_x[k] < 0; }
  klst::dev::launch_csr_build(ctx->stream, ctx->d_rowptr, ctx->d_col, ctx->d_val, p.Ny, p.Nxi, p.r,
                              p.beta, ctx->d_Dx, ctx->d_xix, ctx->d_xiy, ctx->d_nu, ctx->d_U,
                              ctx->d_M, npos, nneg);
  HIPCHK(hipGetLastError());
  return KLST_OK;
}

// y = (A - tau B) x on the device (nvec vectors).
klst_status op_apply(klst_ctx* ctx, cd tau, const double2* x, double2* y, int nvec, int mode,
                     const int* skip) {
  const klst::Problem& p = ctx->prob;
  if (mode == 1) {
    klst_status s = ensure_csr(ctx);
    if (s != KLST_OK) return s;
    for (int v = 0; v < nvec; ++v)
      klst::dev::launch_csr_spmv(ctx->stream, ctx->d_rowptr, ctx->d_col, ctx->d_val, x + v * p.n(),
                                 y + v * p.n(), p.n(), p.Ny, p.Nxi, ctx->d_xix, tau.real(),
                                 tau.imag(), skip);
  } else {
    klst_status s = ensure_mom(ctx, nvec);
    if (s != KLST_OK) return s;
    klst::dev::launch_moments(ctx->stream, x, p.n(), nvec, p.Ny, p.Nxi, p.r, ctx->d_M, ctx->d_mom,
                              skip);
    klst::dev::launch_apply(ctx->stream, x, y, p.n(), nvec, p.Ny, p.Nxi, p.r, tau.real(), tau.imag(),
                            p.beta, ctx->d_DxT, ctx->d_xix, ctx->d_xiy, ctx->d_nu, ctx->d_U,
                            ctx->d_mom, skip);
  }
  HIPCHK(hipGetLastError());
  ctx->stats.op_applies += nvec;
  return KLST_OK;
}

// pk_override >= 0 selects the preconditioner kind instead of opt.pc_kernel.
klst_status pc_setup(klst_ctx* ctx, cd sigma, int pk_override = -1) {
  const klst::Problem& p = ctx->prob;
  const int lines = std::max(1, ctx->opt.lines_per_block);
  const int pk = pk_override >= 0 ? pk_override : ctx->opt.pc_kernel;
  if (ctx->pc_ready && ctx->pc_sigma == sigma && ctx->pc_lines == lines && ctx->pc_kernel_built == pk)
    return KLST_OK;
  ctx->pc_ready = false;
  const unsigned hw = std::thread::hardware_concurrency();
  const int nth = (int)std::max(1u, std::min(hw, 16u));
  // dynamic LDS of the apply kernels stays within 64 KiB per workgroup: the block
  // GEMV stages nl Ny inputs plus up to 16 x 64 partial sums, the line inverse 2 Ny
  // inputs plus 2 x 16 x 64, the capacitance GEMV its r Ny right-hand side
  const size_t lds_max = 64 * 1024;
  if (pk == 2 && (16 * (4 * (size_t)p.Ny + 2048) > lds_max || 16 * (size_t)p.r * p.Ny > lds_max))
    return fail(ctx, KLST_EINVAL, "Ny too large for the structured inverse (Ny <= 512)");
  if (pk == 0 && 16 * (size_t)lines * p.Ny > lds_max)
    return fail(ctx, KLST_EINVAL, "lines_per_block * Ny too large for the level-set sweeps (<= 4096)");
  if (pk == 1 && 16 * ((size_t)lines * p.Ny + 1024) > lds_max)
    return fail(ctx, KLST_EINVAL, "lines_per_block * Ny too large for the stored block inverse (<= 3072)");
  if (pk == 2) {
    klst_status s;
    if ((s = ensure_mom(ctx, 1)) != KLST_OK) return s;
    const int Rd = p.r * p.Ny;
    std::vector<int> slot_node, slot_mate, slot_of, conj_of;
    klst::structured_slots(p, sigma, slot_node, slot_mate, slot_of, conj_of);
    const int nslots = (int)slot_node.size();
    dfree(ctx, ctx->d_Pinv); dfree(ctx, ctx->d_Pinv32);
    dfree(ctx, ctx->d_Sinv); dfree(ctx, ctx->d_Sinv32);
    dfree(ctx, ctx->d_slots);
    ctx->nslots = nslots;
    ALLOC(ctx->d_Pinv, sizeof(double2) * (size_t)nslots * p.Ny * p.Ny);
    ALLOC(ctx->d_Sinv, sizeof(double2) * (size_t)Rd * Rd);
    {
      std::vector<int> sl(slot_node);
      sl.insert(sl.end(), slot_mate.begin(), slot_mate.end());
      ALLOC(ctx->d_slots, sizeof(int) * sl.size());
      HIPCHK(hipMemcpyAsync(ctx->d_slots, sl.data(), sizeof(int) * sl.size(), hipMemcpyHostToDevice, ctx->stream));
      HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    if ((size_t)Rd * (2 * sizeof(double2) + sizeof(int)) <= 64 * 1024) {
      // set-up on the device: line blocks inverted in place, capacitance assembled
      // and inverted there; the host reads back only the singularity flags
      int *d_aux = nullptr;
      double2* d_part = nullptr;
      ALLOC(d_aux, sizeof(int) * (2 * (size_t)p.Nxi + 1 + nslots));
      const klst_status sp = dalloc(ctx, (void**)&d_part, sizeof(double2) * klst::dev::kCapParts * (size_t)Rd * Rd);
      if (sp != KLST_OK) { dfree(ctx, d_aux); return sp; }
      std::vector<int> aux(slot_of);
      aux.insert(aux.end(), conj_of.begin(), conj_of.end());
      int* d_status = d_aux + 2 * p.Nxi;
      HIPCHK(hipMemcpyAsync(d_aux, aux.data(), sizeof(int) * aux.size(), hipMemcpyHostToDevice, ctx->stream));
      klst::dev::launch_structured_setup(ctx->stream, ctx->d_Pinv, ctx->d_Sinv, d_part, p.Ny, p.Nxi, p.r,
                                         ctx->d_slots, nslots, d_aux, d_aux + p.Nxi, ctx->d_Dx, ctx->d_xix,
                                         ctx->d_xiy, ctx->d_nu, ctx->d_U, ctx->d_M, p.beta, sigma.real(),
                                         sigma.imag(), d_status);
      HIPCHK(hipGetLastError());
      std::vector<int> status(1 + nslots);
      HIPCHK(hipMemcpyAsync(status.data(), d_status, sizeof(int) * status.size(), hipMemcpyDeviceToHost,
                            ctx->stream));
      HIPCHK(hipStreamSynchronize(ctx->stream));
      dfree(ctx, d_part);
      dfree(ctx, d_aux);
      for (int sl = 0; sl < nslots; ++sl)
        if (status[1 + sl]) return fail(ctx, KLST_ENOCONV, "singular velocity-line block at node " +
                                                             std::to_string(slot_node[sl]));
      if (status[0]) return fail(ctx, KLST_ENOCONV, "singular moment capacitance matrix");
    } else {
      // (r Ny)^2 too large for the one-workgroup capacitance inversion: host set-up
      klst::StructuredInverse si;
      const std::string e = klst::build_structured_inverse(p, sigma, si, nth);
      if (!e.empty()) return fail(ctx, KLST_ENOCONV, e);
      HIPCHK(hipMemcpyAsync(ctx->d_Pinv, si.Pinv.data(), sizeof(double2) * si.Pinv.size(), hipMemcpyHostToDevice,
                            ctx->stream));
      HIPCHK(hipMemcpyAsync(ctx->d_Sinv, si.Sinv.data(), sizeof(double2) * si.Sinv.size(), hipMemcpyHostToDevice,
                            ctx->stream));
      HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    if (ctx->opt.precision == 1) {
      const size_t np = (size_t)nslots * p.Ny * p.Ny;
      ALLOC(ctx->d_Pinv32, sizeof(float2) * np);
      ALLOC(ctx->d_Sinv32, sizeof(float2) * (size_t)Rd * Rd);
      klst::dev::launch_narrow(ctx->stream, ctx->d_Pinv, ctx->d_Pinv32, (int64_t)np);
      klst::dev::launch_narrow(ctx->stream, ctx->d_Sinv, ctx->d_Sinv32, (int64_t)Rd * Rd);
      HIPCHK(hipGetLastError());
    }
    dfree(ctx, ctx->d_capd);
    dfree(ctx, ctx->d_capd32);
    ALLOC(ctx->d_capd, sizeof(double2) * (size_t)Rd);
    if (ctx->opt.precision == 1) ALLOC(ctx->d_capd32, sizeof(float2) * (size_t)Rd);
    ctx->ilu = klst::ILU0{};
    ctx->pc_ready = true;
    ctx->pc_sigma = sigma;
    ctx->pc_lines = lines;
    ctx->pc_kernel_built = pk;
    ctx->stats.pivots_floored = 0;
    return KLST_OK;
  }
  klst::build_ilu0(p, sigma, lines, ctx->ilu, nth);
  dfree(ctx, ctx->d_Kinv);
  dfree(ctx, ctx->d_koff);
  if (pk == 1) {
    std::vector<cd> Kinv;
    std::vector<int64_t> koff;
    klst::build_block_inverse(ctx->ilu, Kinv, koff, nth);
    ALLOC(ctx->d_Kinv, sizeof(double2) * Kinv.size());
    ALLOC(ctx->d_koff, sizeof(int64_t) * koff.size());
    HIPCHK(hipMemcpyAsync(ctx->d_Kinv, Kinv.data(), sizeof(double2) * Kinv.size(), hipMemcpyHostToDevice,
                          ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->d_koff, koff.data(), sizeof(int64_t) * koff.size(), hipMemcpyHostToDevice,
                          ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    dfree(ctx, ctx->d_Kinv32);
    if (ctx->opt.precision == 1) {
      std::vector<float2> K32(Kinv.size());
      for (size_t i = 0; i < Kinv.size(); ++i)
        K32[i] = make_float2((float)Kinv[i].real(), (float)Kinv[i].imag());
      ALLOC(ctx->d_Kinv32, sizeof(float2) * K32.size());
      HIPCHK(hipMemcpyAsync(ctx->d_Kinv32, K32.data(), sizeof(float2) * K32.size(), hipMemcpyHostToDevice,
                            ctx->stream));
      HIPCHK(hipStreamSynchronize(ctx->stream));
    }
  }
  // F column-major per line for the device sweeps
  const int Ny = p.Ny;
  std::vector<cd> Fc(ctx->ilu.F.size());
  for (int l = 0; l < ctx->ilu.nlines; ++l) {
    const cd* Fr = &ctx->ilu.F[(size_t)l * Ny * Ny];
    cd* Fo = &Fc[(size_t)l * Ny * Ny];
    for (int j = 0; j < Ny; ++j)
      for (int m = 0; m < Ny; ++m) Fo[(size_t)m * Ny + j] = Fr[(size_t)j * Ny + m];
    // the device sweeps multiply by the reciprocal pivot
    for (int j = 0; j < Ny; ++j) Fo[(size_t)j * Ny + j] = 1.0 / Fr[(size_t)j * Ny + j];
  }
  dfree(ctx, ctx->d_F);
  dfree(ctx, ctx->d_C);
  ALLOC(ctx->d_F, sizeof(double2) * Fc.size());
  ALLOC(ctx->d_C, sizeof(double2) * std::max<size_t>(1, ctx->ilu.C.size()));
  HIPCHK(hipMemcpyAsync(ctx->d_F, Fc.data(), sizeof(double2) * Fc.size(), hipMemcpyHostToDevice,
                        ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->d_C, ctx->ilu.C.data(), sizeof(double2) * ctx->ilu.C.size(),
                        hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  ctx->pc_ready = true;
  ctx->pc_sigma = sigma;
  ctx->pc_lines = lines;
  ctx->pc_kernel_built = pk;
  ctx->stats.pivots_floored = ctx->ilu.floored;
  return KLST_OK;
}

klst_status pc_apply(klst_ctx* ctx, const double2* x, double2* y, const int* skip) {
  const klst::Problem& p = ctx->prob;
  if (ctx->pc_kernel_built == 2)
    klst::dev::launch_structured_inverse(ctx->stream, x, y, p.Ny, p.Nxi, p.r, ctx->d_Pinv, ctx->d_slots,
                                         ctx->d_slots + ctx->nslots, ctx->nslots, ctx->d_Sinv, ctx->d_M,
                                         ctx->d_U, ctx->d_xix, ctx->d_mom, ctx->d_capd, skip);
  else if (ctx->pc_kernel_built == 1)
    klst::dev::launch_blockinv_apply(ctx->stream, x, y, p.Ny, p.Nxi, ctx->ilu.nl, ctx->ilu.nblocks,
                                     ctx->d_Kinv, ctx->d_koff, skip);
  else
    klst::dev::launch_ilu_apply(ctx->stream, x, y, p.Ny, p.Nxi, ctx->ilu.nl, ctx->ilu.nblocks, ctx->d_F,
                                ctx->d_C, skip);
  HIPCHK(hipGetLastError());
  ctx->stats.pc_applies += 1;
  return KLST_OK;
}

// Precision-generic operator / preconditioner for the GMRES correction solve.
klst_status op_v(klst_ctx* ctx, cd tau, const double2* x, double2* y, const int* skip) {
  return op_apply(ctx, tau, x, y, 1, ctx->opt.op_mode, skip);
}
klst_status op_v(klst_ctx* ctx, cd tau, const float2* x, float2* y, const int* skip) {
  const klst::Problem& p = ctx->prob;
  klst::dev::launch_moments(ctx->stream, x, p.n(), 1, p.Ny, p.Nxi, p.r, ctx->d_M32, ctx->d_mom32, skip);
  klst::dev::launch_apply(ctx->stream, x, y, p.n(), 1, p.Ny, p.Nxi, p.r, tau.real(), tau.imag(), p.beta,
                          ctx->d_DxT32, ctx->d_xix32, ctx->d_xiy32, ctx->d_nu32, ctx->d_U32, ctx->d_mom32,
                          skip);
  HIPCHK(hipGetLastError());
  ctx->stats.op_applies += 1;
  return KLST_OK;
}
klst_status pc_v(klst_ctx* ctx, const double2* x, double2* y, const int* skip) {
  return pc_apply(ctx, x, y, skip);
}
klst_status pc_v(klst_ctx* ctx, const float2* x, float2* y, const int* skip) {
  const klst::Problem& p = ctx->prob;
  if (ctx->pc_kernel_built == 2)
    klst::dev::launch_structured_inverse(ctx->stream, x, y, p.Ny, p.Nxi, p.r, ctx->d_Pinv32, ctx->d_slots,
                                         ctx->d_slots + ctx->nslots, ctx->nslots, ctx->d_Sinv32,
                                         ctx->d_M32, ctx->d_U32, ctx->d_xix32, ctx->d_mom32, ctx->d_capd32, skip);
  else
    klst::dev::launch_blockinv_apply(ctx->stream, x, y, p.Ny, p.Nxi, ctx->ilu.nl, ctx->ilu.nblocks,
                                     ctx->d_Kinv32, ctx->d_koff, skip);
  HIPCHK(hipGetLastError());
  ctx->stats.pc_applies += 1;
  return KLST_OK;
}

// FP32 copies of the operator tables (mixed precision).
klst_status upload_fp32_tables(klst_ctx* ctx) {
  const klst::Problem& q = ctx->prob;
  auto up = [&](float*& d, const std::vector<double>& h) -> klst_status {
    std::vector<float> f(h.begin(), h.end());
    ALLOC(d, sizeof(float) * std::max<size_t>(1, f.size()));
    HIPCHK(hipMemcpyAsync(d, f.data(), sizeof(float) * f.size(), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return KLST_OK;
  };
  klst_status s;
  if ((s = up(ctx->d_Dx32, q.Dx)) != KLST_OK) return s;
  {
    std::vector<double> DxT(q.Dx.size());
    for (int j = 0; j < q.Ny; ++j)
      for (int m = 0; m < q.Ny; ++m) DxT[(size_t)m * q.Ny + j] = q.Dx[(size_t)j * q.Ny + m];
    if ((s = up(ctx->d_DxT32, DxT)) != KLST_OK) return s;
  }
  if ((s = up(ctx->d_xix32, q.xi_x)) != KLST_OK) return s;
  if ((s = up(ctx->d_xiy32, q.xi_y)) != KLST_OK) return s;
  if ((s = up(ctx->d_nu32, q.nu)) != KLST_OK) return s;
  if ((s = up(ctx->d_U32, q.U)) != KLST_OK) return s;
  if ((s = up(ctx->d_M32, q.M)) != KLST_OK) return s;
  ALLOC(ctx->d_mom32, sizeof(float2) * (size_t)q.Ny * q.r * 8);
  ctx->mom32_cap = 1;
  return KLST_OK;
}

// ---- SplitMix64 start vector (Steele, Lea & Flood 2014) ----
uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

void start_vector(const klst::Problem& p, uint64_t seed, uint64_t stream, std::vector<cd>& out) {
  const int64_t n = p.n();
  out.resize(n);
  const uint64_t key = seed * 0x100000001B3ULL + stream;
  const double scale = 1.0 / 9007199254740992.0;   // 2^-53
  for (int64_t i = 0; i < n; ++i) {
    const double a = 2.0 * (double)(splitmix64(key + 2 * (uint64_t)i) >> 11) * scale - 1.0;
    const double b = 2.0 * (double)(splitmix64(key + 2 * (uint64_t)i + 1) >> 11) * scale - 1.0;
    const int64_t nc = 2LL * p.Nxi;
    const int j = (int)(i / nc);
    const int k = (int)(i % nc) % p.Nxi;
    out[i] = p.is_bc(j, k) ? cd(0.0) : cd(a, b);
  }
}

}  // namespace

// =================================================================== ABI ===

extern "C" {

void klst_default_options(klst_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->device = 0;
  o->stream = nullptr;
  o->precision = 0;
  o->op_mode = 0;
  o->lines_per_block = 1;
  o->m_max = 30;
  o->m_min = 6;
  o->gmres_m = 20;
  o->max_it = 10000;
  o->tol = 1e-10;
  o->inner_rtol = 1e-6;
  o->fix = 0.01;
  o->seed = 0;
  o->pc_kernel = 2;
  o->inner_max_it = 0;
  o->reorth = 0;
  o->method = 0;
  o->krylov32 = 0;
}

const char* klst_strerror(klst_status s) {
  switch (s) {
    case KLST_OK: return "ok";
    case KLST_EINVAL: return "invalid argument";
    case KLST_ENOMEM: return "out of memory";
    case KLST_EDEVICE: return "device error";
    case KLST_ENOCONV: return "not converged";
    case KLST_EBUSY: return "busy";
    case KLST_ECANCELLED: return "cancelled";
    case KLST_ESTATE: return "call out of order";
  }
  return "unknown status";
}

const char* klst_last_error(const klst_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

klst_status klst_create(klst_ctx** out, const klst_options* opt) {
  if (!out) return KLST_EINVAL;
  *out = nullptr;
  klst_options o;
  if (opt) o = *opt; else klst_default_options(&o);
  if (o.m_min < 1 || o.m_max < o.m_min + 2 || o.gmres_m < 1 || o.gmres_m > 256 || o.max_it < 1 ||
      !(o.tol > 0) || !(o.inner_rtol > 0) || o.lines_per_block < 1 || o.lines_per_block > 16 ||
      (o.precision != 0 && o.precision != 1) || (o.op_mode != 0 && o.op_mode != 1) || o.m_max > 248 ||
      o.pc_kernel < 0 || o.pc_kernel > 2 || (o.precision == 1 && o.pc_kernel == 0) ||
      o.inner_max_it < 0 || o.inner_max_it > 100000 || (o.reorth != 0 && o.reorth != 1) ||
      (o.method != 0 && o.method != 1) || (o.krylov32 != 0 && o.krylov32 != 1))
    return KLST_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || o.device < 0 || o.device >= ndev) {
    (void)hipGetLastError();
    return KLST_EDEVICE;
  }
  klst_ctx* ctx = new klst_ctx();
  ctx->opt = o;
  if (hipSetDevice(o.device) != hipSuccess) { delete ctx; return KLST_EDEVICE; }
  if (!resolve_scratch(o.device)) { delete ctx; return KLST_EDEVICE; }
  // NULL selects the device's default (null) stream, so work is ordered with
  // anything else the caller issues there (torch's default stream included).
  ctx->stream = (hipStream_t)o.stream;
  ctx->own_stream = false;
  if (dalloc(ctx, (void**)&ctx->d_partial, sizeof(double2) * 512 * 256) != KLST_OK ||
      dalloc(ctx, (void**)&ctx->d_npart, sizeof(double2) * 65536) != KLST_OK) {
    klst_destroy(ctx);
    return KLST_ENOMEM;
  }
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) {
    klst_destroy(ctx);
    return KLST_EDEVICE;
  }
  *out = ctx;
  return KLST_OK;
}

void klst_destroy(klst_ctx* ctx) {
  if (!ctx) return;
  hipSetDevice(ctx->opt.device);
  if (ctx->stream) hipStreamSynchronize(ctx->stream);
  free_problem(ctx);
  dfree(ctx, ctx->d_partial);
  dfree(ctx, ctx->d_npart);
  if (ctx->stream) hipStreamSynchronize(ctx->stream);
  if (ctx->own_stream && ctx->stream) hipStreamDestroy(ctx->stream);
  delete ctx;
}

klst_status klst_host_tables(const klst_grid* grid, const klst_vel* vel, const klst_base* base,
                             double beta, double* Dx, double* nu, double* U, double* M, uint8_t* bc) {
  klst::Problem p;
  const std::string e = klst::build_problem(grid, vel, base, beta, p);
  if (!e.empty()) return KLST_EINVAL;
  if (Dx) std::memcpy(Dx, p.Dx.data(), sizeof(double) * p.Dx.size());
  if (nu) std::memcpy(nu, p.nu.data(), sizeof(double) * p.nu.size());
  if (U) std::memcpy(U, p.U.data(), sizeof(double) * p.U.size());
  if (M) std::memcpy(M, p.M.data(), sizeof(double) * p.M.size());
  if (bc) std::memcpy(bc, p.bc.data(), p.bc.size());
  return KLST_OK;
}

klst_status klst_host_select_output(int k, const double* lam, const double* G, const double* nrm2,
                                    const double sigma[2], int nev, double* out_lam, int* out_src,
                                    int* out_mirrored, int* nout) {
  if (k < 0 || nev < 0 || !sigma || !nout || (k > 0 && !lam) || (G && !nrm2)) return KLST_EINVAL;
  std::vector<cd> l(k), g(G ? (size_t)k * k : 0);
  for (int i = 0; i < k; ++i) l[i] = cd(lam[2 * i], lam[2 * i + 1]);
  for (size_t i = 0; i < g.size(); ++i) g[i] = cd(G[2 * i], G[2 * i + 1]);
  const auto sel = klst::select_output(l, G ? g.data() : nullptr, nrm2, cd(sigma[0], sigma[1]), nev);
  *nout = (int)sel.size();
  for (size_t o = 0; o < sel.size(); ++o) {
    if (out_lam) { out_lam[2 * o] = sel[o].lam.real(); out_lam[2 * o + 1] = sel[o].lam.imag(); }
    if (out_src) out_src[o] = sel[o].src;
    if (out_mirrored) out_mirrored[o] = sel[o].mirrored ? 1 : 0;
  }
  return KLST_OK;
}

klst_status klst_gp_shock(double mach, double gamma, double Pr, double s_visc, double delta, int nz,
                          const double* z, double* rho, double* u, double* T, double* thickness) {
  if (nz < 0 || (nz > 0 && (!z || !rho || !u || !T))) return KLST_EINVAL;
  for (int i = 0; i < nz; ++i)
    if (!std::isfinite(z[i])) return KLST_EINVAL;
  return klst::gp_shock(mach, gamma, Pr, s_visc, delta, nz, z, rho, u, T, thickness).empty() ? KLST_OK
                                                                                               : KLST_EINVAL;
}

klst_status klst_host_sorted_schur(int m, const double* G, double* U, double* T) {
  if (m < 1 || !G || !U || !T) return KLST_EINVAL;
  std::vector<cd> g(m * m), u(m * m), t(m * m);
  for (int i = 0; i < m * m; ++i) g[i] = cd(G[2 * i], G[2 * i + 1]);
  if (!klst::sorted_schur(m, g.data(), u.data(), t.data())) return KLST_ENOCONV;
  for (int i = 0; i < m * m; ++i) {
    U[2 * i] = u[i].real(); U[2 * i + 1] = u[i].imag();
    T[2 * i] = t[i].real(); T[2 * i + 1] = t[i].imag();
  }
  return KLST_OK;
}

klst_status klst_assemble(klst_ctx* ctx, const klst_grid* grid, const klst_vel* vel,
                          const klst_base* base, double beta) {
  if (!ctx) return KLST_EINVAL;
  HIPCHK(hipSetDevice(ctx->opt.device));
  klst::Problem p;
  const std::string e = klst::build_problem(grid, vel, base, beta, p);
  if (!e.empty()) return fail(ctx, KLST_EINVAL, e);
  HIPCHK(hipStreamSynchronize(ctx->stream));
  free_problem(ctx);
  ctx->prob = std::move(p);
  const klst::Problem& q = ctx->prob;
  ALLOC(ctx->d_Dx, sizeof(double) * q.Dx.size());
  ALLOC(ctx->d_DxT, sizeof(double) * q.Dx.size());
  std::vector<double> DxT(q.Dx.size());
  for (int j = 0; j < q.Ny; ++j)
    for (int m = 0; m < q.Ny; ++m) DxT[(size_t)m * q.Ny + j] = q.Dx[(size_t)j * q.Ny + m];
  HIPCHK(hipMemcpyAsync(ctx->d_DxT, DxT.data(), sizeof(double) * DxT.size(), hipMemcpyHostToDevice, ctx->stream));
  ALLOC(ctx->d_xix, sizeof(double) * q.Nxi);
  ALLOC(ctx->d_xiy, sizeof(double) * q.Nxi);
  ALLOC(ctx->d_nu, sizeof(double) * q.Ny);
  ALLOC(ctx->d_U, sizeof(double) * q.U.size());
  ALLOC(ctx->d_M, sizeof(double) * q.M.size());
  HIPCHK(hipMemcpyAsync(ctx->d_Dx, q.Dx.data(), sizeof(double) * q.Dx.size(), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->d_xix, q.xi_x.data(), sizeof(double) * q.Nxi, hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->d_xiy, q.xi_y.data(), sizeof(double) * q.Nxi, hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->d_nu, q.nu.data(), sizeof(double) * q.Ny, hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->d_U, q.U.data(), sizeof(double) * q.U.size(), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->d_M, q.M.data(), sizeof(double) * q.M.size(), hipMemcpyHostToDevice, ctx->stream));
  {
    std::vector<double> base((size_t)q.Ny * 4);
    for (int j = 0; j < q.Ny; ++j) {
      base[(size_t)j * 4 + 0] = q.rho[j]; base[(size_t)j * 4 + 1] = q.u[j];
      base[(size_t)j * 4 + 2] = q.E[j]; base[(size_t)j * 4 + 3] = q.T[j];
    }
    ALLOC(ctx->d_w, sizeof(double) * q.Nxi);
    ALLOC(ctx->d_base, sizeof(double) * base.size());
    HIPCHK(hipMemcpyAsync(ctx->d_w, q.w.data(), sizeof(double) * q.Nxi, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->d_base, base.data(), sizeof(double) * base.size(), hipMemcpyHostToDevice,
                          ctx->stream));
    if (!q.gc.empty()) {
      ALLOC(ctx->d_gc, sizeof(double) * q.gc.size());
      HIPCHK(hipMemcpyAsync(ctx->d_gc, q.gc.data(), sizeof(double) * q.gc.size(), hipMemcpyHostToDevice,
                            ctx->stream));
    }
    // the host base state is not read again while the tables above are alive
    HIPCHK(hipStreamSynchronize(ctx->stream));
  }
  klst_status s = ensure_mom(ctx, 1);
  if (s != KLST_OK) return s;
  if (ctx->opt.precision == 1 && (s = upload_fp32_tables(ctx)) != KLST_OK) return s;
  if (ctx->opt.op_mode == 1) {
    s = ensure_csr(ctx);
    if (s != KLST_OK) return s;
  }
  HIPCHK(hipStreamSynchronize(ctx->stream));
  ctx->assembled = true;
  return KLST_OK;
}

klst_status klst_dims(const klst_ctx* ctx, int64_t* n, int64_t* nnz, int* n_bc) {
  if (!ctx) return KLST_EINVAL;
  if (!ctx->assembled) return KLST_ESTATE;
  if (n) *n = ctx->prob.n();
  if (nnz) *nnz = ctx->prob.nnz();
  if (n_bc) *n_bc = ctx->prob.n_bc;
  return KLST_OK;
}

klst_status klst_apply(klst_ctx* ctx, const double tau[2], const void* x, void* y) {
  if (!ctx || !tau || !x || !y) return KLST_EINVAL;
  if (!ctx->assembled) return fail(ctx, KLST_ESTATE, "klst_apply before klst_assemble");
  HIPCHK(hipSetDevice(ctx->opt.device));
  return op_apply(ctx, cd(tau[0], tau[1]), (const double2*)x, (double2*)y, 1, ctx->opt.op_mode, nullptr);
}

klst_status klst_apply_f32(klst_ctx* ctx, const double tau[2], const void* x, void* y) {
  if (!ctx || !tau || !x || !y) return KLST_EINVAL;
  if (!ctx->assembled) return fail(ctx, KLST_ESTATE, "klst_apply_f32 before klst_assemble");
  if (ctx->opt.precision != 1 || !ctx->d_DxT32)
    return fail(ctx, KLST_ESTATE, "klst_apply_f32 needs a mixed-precision context (precision = 1)");
  HIPCHK(hipSetDevice(ctx->opt.device));
  return op_v(ctx, cd(tau[0], tau[1]), (const float2*)x, (float2*)y, nullptr);
}

klst_status klst_apply_many_f32(klst_ctx* ctx, const double tau[2], int nvec, const void* x, void* y) {
  if (!ctx || !tau || !x || !y || nvec < 1 || nvec > 65535) return KLST_EINVAL;
  if (!ctx->assembled) return fail(ctx, KLST_ESTATE, "klst_apply_many_f32 before klst_assemble");
  if (ctx->opt.precision != 1 || !ctx->d_DxT32)
    return fail(ctx, KLST_ESTATE, "klst_apply_many_f32 needs a mixed-precision context (precision = 1)");
  HIPCHK(hipSetDevice(ctx->opt.device));
  klst_status s = ensure_mom32(ctx, nvec);
  if (s != KLST_OK) return s;
  const klst::Problem& p = ctx->prob;
  klst::dev::launch_moments(ctx->stream, (const float2*)x, p.n(), nvec, p.Ny, p.Nxi, p.r, ctx->d_M32, ctx->d_mom32,
                            nullptr);
  klst::dev::launch_apply(ctx->stream, (const float2*)x, (float2*)y, p.n(), nvec, p.Ny, p.Nxi, p.r, tau[0], tau[1],
                          p.beta, ctx->d_DxT32, ctx->d_xix32, ctx->d_xiy32, ctx->d_nu32, ctx->d_U32, ctx->d_mom32,
                          nullptr);
  HIPCHK(hipGetLastError());
  ctx->stats.op_applies += nvec;
  return KLST_OK;
}

klst_status klst_apply_many(klst_ctx* ctx, const double tau[2], int nvec, const void* x, void* y) {
  if (!ctx || !tau || !x || !y || nvec < 1 || nvec > 65535) return KLST_EINVAL;
  if (!ctx->assembled) return fail(ctx, KLST_ESTATE, "klst_apply_many before klst_assemble");
  HIPCHK(hipSetDevice(ctx->opt.device));
  return op_apply(ctx, cd(tau[0], tau[1]), (const double2*)x, (double2*)y, nvec, 0, nullptr);
}

klst_status klst_apply_many_noalloc(klst_ctx* ctx, const double tau[2], int nvec, const void* x, void* y) {
  if (!ctx || !tau || !x || !y || nvec < 1 || nvec > 65535) return KLST_EINVAL;
  if (!ctx->assembled) return fail(ctx, KLST_ESTATE, "klst_apply_many_noalloc before klst_assemble");
  const klst::Problem& p = ctx->prob;
  // moment partials (up to 8 column parts) and their totals: nvec x Ny x r x 9 entries
  if ((size_t)nvec * p.Ny * p.r * 9 > kScratchEntries)
    return fail(ctx, KLST_EINVAL, "klst_apply_many_noalloc: nvec * Ny * r * 9 = " +
                                      std::to_string((size_t)nvec * p.Ny * p.r * 9) + " exceeds the " +
                                      std::to_string(kScratchEntries) + "-entry scratch");
  HIPCHK(hipSetDevice(ctx->opt.device));
  double2* mom = scratch_on(ctx->opt.device);
  if (!mom) return fail(ctx, KLST_EDEVICE, "scratch address not resolved for this device");
  const cd t(tau[0], tau[1]);
  klst::dev::launch_moments(ctx->stream, (const double2*)x, p.n(), nvec, p.Ny, p.Nxi, p.r, ctx->d_M, mom, nullptr);
  klst::dev::launch_apply(ctx->stream, (const double2*)x, (double2*)y, p.n(), nvec, p.Ny, p.Nxi, p.r, t.real(),
                          t.imag(), p.beta, ctx->d_DxT, ctx->d_xix, ctx->d_xiy, ctx->d_nu, ctx->d_U, mom, nullptr);
  HIPCHK(hipGetLastError());
  ctx->stats.op_applies += nvec;
  return KLST_OK;
}

klst_status klst_apply_csr(klst_ctx* ctx, const double tau[2], const void* x, void* y) {
  if (!ctx || !tau || !x || !y) return KLST_EINVAL;
  if (!ctx->assembled) return fail(ctx, KLST_ESTATE, "klst_apply_csr before klst_assemble");
  HIPCHK(hipSetDevice(ctx->opt.device));
  return op_apply(ctx, cd(tau[0], tau[1]), (const double2*)x, (double2*)y, 1, 1, nullptr);
}

klst_status klst_precond_setup(klst_ctx* ctx, const double sigma[2]) {
  if (!ctx || !sigma) return KLST_EINVAL;
  if (!ctx->assembled) return fail(ctx, KLST_ESTATE, "klst_precond_setup before klst_assemble");
  HIPCHK(hipSetDevice(ctx->opt.device));
  return pc_setup(ctx, cd(sigma[0], sigma[1]));
}

klst_status klst_precond_apply(klst_ctx* ctx, const void* x, void* y) {
  if (!ctx || !x || !y) return KLST_EINVAL;
  if (!ctx->pc_ready) return fail(ctx, KLST_ESTATE, "klst_precond_apply before klst_precond_setup");
  HIPCHK(hipSetDevice(ctx->opt.device));
  return pc_apply(ctx, (const double2*)x, (double2*)y, nullptr);
}

klst_status klst_precond_apply_lines(klst_ctx* ctx, const void* x, void* y) {
  if (!ctx || !x || !y || x == y) return KLST_EINVAL;
  if (!ctx->pc_ready || ctx->pc_kernel_built != 2)
    return fail(ctx, KLST_ESTATE, "klst_precond_apply_lines needs the structured inverse (pc_kernel 2) set up");
  HIPCHK(hipSetDevice(ctx->opt.device));
  const klst::Problem& p = ctx->prob;
  klst::dev::launch_line_inverse(ctx->stream, (const double2*)x, (double2*)y, p.Ny, p.Nxi, p.r, ctx->d_Pinv,
                                 ctx->d_slots, ctx->d_slots + ctx->nslots, ctx->nslots, ctx->d_U, ctx->d_xix);
  HIPCHK(hipGetLastError());
  return KLST_OK;
}

klst_status klst_precond_export(klst_ctx* ctx, double* Pinv, double* Sinv, int* slot_node, int* nslots) {
  if (!ctx || !nslots) return KLST_EINVAL;
  if (!ctx->pc_ready || ctx->pc_kernel_built != 2)
    return fail(ctx, KLST_ESTATE, "klst_precond_export needs the structured inverse (pc_kernel 2) set up");
  HIPCHK(hipSetDevice(ctx->opt.device));
  const klst::Problem& p = ctx->prob;
  const size_t Rd = (size_t)p.r * p.Ny;
  *nslots = ctx->nslots;
  if (Pinv)
    HIPCHK(hipMemcpyAsync(Pinv, ctx->d_Pinv, sizeof(double2) * (size_t)ctx->nslots * p.Ny * p.Ny,
                          hipMemcpyDeviceToHost, ctx->stream));
  if (Sinv) HIPCHK(hipMemcpyAsync(Sinv, ctx->d_Sinv, sizeof(double2) * Rd * Rd, hipMemcpyDeviceToHost, ctx->stream));
  if (slot_node)
    HIPCHK(hipMemcpyAsync(slot_node, ctx->d_slots, sizeof(int) * ctx->nslots, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return KLST_OK;
}

klst_status klst_host_structured_inverse(const klst_grid* grid, const klst_vel* vel, const klst_base* base,
                                         double beta, const double sigma[2], double* Pinv, double* Sinv,
                                         int* slot_node, int* nslots) {
  if (!sigma || !nslots) return KLST_EINVAL;
  klst::Problem p;
  if (!klst::build_problem(grid, vel, base, beta, p).empty()) return KLST_EINVAL;
  klst::StructuredInverse si;
  const unsigned hw = std::thread::hardware_concurrency();
  if (!klst::build_structured_inverse(p, cd(sigma[0], sigma[1]), si, (int)std::max(1u, std::min(hw, 16u))).empty())
    return KLST_ENOCONV;
  *nslots = (int)si.slot_node.size();
  if (Pinv) std::memcpy(Pinv, si.Pinv.data(), sizeof(cd) * si.Pinv.size());
  if (Sinv) std::memcpy(Sinv, si.Sinv.data(), sizeof(cd) * si.Sinv.size());
  if (slot_node) std::memcpy(slot_node, si.slot_node.data(), sizeof(int) * si.slot_node.size());
  return KLST_OK;
}

klst_status klst_export_csr(klst_ctx* ctx, void* rowptr, void* col, void* val, int on_device) {
  if (!ctx || !rowptr || !col || !val) return KLST_EINVAL;
  if (!ctx->assembled) return fail(ctx, KLST_ESTATE, "klst_export_csr before klst_assemble");
  HIPCHK(hipSetDevice(ctx->opt.device));
  klst_status s = ensure_csr(ctx);
  if (s != KLST_OK) return s;
  const int64_t n = ctx->prob.n(), nnz = ctx->prob.nnz();
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  HIPCHK(hipMemcpyAsync(rowptr, ctx->d_rowptr, sizeof(int64_t) * (n + 1), kind, ctx->stream));
  HIPCHK(hipMemcpyAsync(col, ctx->d_col, sizeof(int32_t) * nnz, kind, ctx->stream));
  HIPCHK(hipMemcpyAsync(val, ctx->d_val, sizeof(double2) * nnz, kind, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return KLST_OK;
}

klst_status klst_autotune(klst_ctx* ctx, int nvec, int precision, int reps, klst_tune_entry* out) {
  using klst::dev::Tuning;
  if (!ctx || nvec < 1 || nvec > 4096 || (precision != 0 && precision != 1) || reps < 1) return KLST_EINVAL;
  if (!ctx->assembled) return fail(ctx, KLST_ESTATE, "klst_autotune before klst_assemble");
  if (precision == 1 && (ctx->opt.precision != 1 || nvec != 1))
    return fail(ctx, KLST_EINVAL, "FP32 tuning needs a mixed-precision context and nvec = 1");
  HIPCHK(hipSetDevice(ctx->opt.device));
  const klst::Problem& p = ctx->prob;
  const int64_t n = p.n();
  const int Ny = p.Ny, Nxi = p.Nxi, nc = 2 * Nxi;
  hipStream_t st = ctx->stream;
  const bool with_pc = (nvec == 1) && ctx->pc_ready && (ctx->pc_kernel_built == 1 || ctx->pc_kernel_built == 2);
  void *x = nullptr, *y = nullptr, *z = nullptr;
  const size_t esz = precision ? sizeof(float2) : sizeof(double2);
  klst_status s;
  if ((s = dalloc(ctx, &x, esz * n * nvec)) != KLST_OK) return s;
  if ((s = dalloc(ctx, &y, esz * n * nvec)) != KLST_OK) { dfree(ctx, x); return s; }
  if ((s = dalloc(ctx, &z, esz * n)) != KLST_OK) { dfree(ctx, x); dfree(ctx, y); return s; }
  HIPCHK(hipMemsetAsync(x, 0, esz * n * nvec, st));
  if ((s = ensure_mom(ctx, nvec)) != KLST_OK) return s;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  // average time of one operator (+ preconditioner) application, microseconds
  auto time_it = [&](bool op, bool pc) -> double {
    auto once = [&]() {
      if (op) {
        if (precision) (void)op_v(ctx, 0.1, (const float2*)x, (float2*)y, nullptr);
        else (void)op_apply(ctx, 0.1, (const double2*)x, (double2*)y, nvec, 0, nullptr);
      }
      if (pc) {
        if (precision) (void)pc_v(ctx, (const float2*)x, (float2*)z, nullptr);
        else (void)pc_apply(ctx, (const double2*)x, (double2*)z, nullptr);
      }
    };
    for (int w = 0; w < 2; ++w) once();
    (void)hipEventRecord(e0, st);
    for (int i = 0; i < reps; ++i) once();
    (void)hipEventRecord(e1, st);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    return 1e3 * ms / reps;
  };
  const int key_nv = nvec;
  klst::dev::tune_erase(Ny, Nxi, key_nv, precision);
  Tuning base;
  const bool had_shape = (nvec > 1) && klst::dev::tune_get(Ny, Nxi, 1, precision, &base);
  (void)had_shape;
  const double t_default = time_it(true, with_pc);
  Tuning best;
  double tbest = 1e300;
  // operator tiling (result-invariant)
  std::vector<std::pair<int, int>> tiles;
  if (precision) {
    tiles = {{4, 0}, {8, 0}, {16, 0}};                 // the scalar FP32 kernel, rows per thread
    for (int rt : {1, 2, 3, 6})
      if ((rt - 1) * 16 < Ny)
        for (int nw : {1, 4}) tiles.push_back({rt, nw});   // the FP32 matrix-core kernel
  } else {
    for (int rt : {1, 2, 3, 6})
      if ((rt - 1) * 16 < Ny)
        for (int nw : {1, 4}) tiles.push_back({rt, nw});
    if (nvec >= 8) tiles.push_back({0, 8});   // the streaming many-vector kernel
  }
  for (auto [rt, nw] : tiles) {
    Tuning t;
    t.apply_rt = rt;
    t.apply_nw = nw;
    klst::dev::tune_set(Ny, Nxi, key_nv, precision, t);
    const double tt = time_it(true, false);
    if (tt < tbest) { tbest = tt; best = t; }
  }
  if (nvec == 1) {
    // column splits of the moment sums (operator and preconditioner share them)
    double tb2 = 1e300;
    for (int ms : {1, 2, 3, 4, 5, 6, 8}) {
      if (ms > 1 && nc / ms < 64) continue;
      Tuning t = best;
      t.msplit = ms;
      klst::dev::tune_set(Ny, Nxi, 1, precision, t);
      const double tt = time_it(true, with_pc);
      if (tt < tb2) { tb2 = tt; best.msplit = ms; }
    }
    if (with_pc) {
      double tb3 = 1e300;
      for (int g : {4, 8, 16}) {
        Tuning t = best;
        t.gemv = g;
        klst::dev::tune_set(Ny, Nxi, 1, precision, t);
        const double tt = time_it(false, true);
        if (tt < tb3) { tb3 = tt; best.gemv = g; }
      }
    }
  }
  klst::dev::tune_set(Ny, Nxi, key_nv, precision, best);
  const double t_tuned = time_it(true, with_pc);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIPCHK(hipStreamSynchronize(st));
  dfree(ctx, x);
  dfree(ctx, y);
  dfree(ctx, z);
  if (out) {
    out->Ny = Ny; out->Nxi = Nxi; out->nvec = nvec; out->precision = precision;
    out->apply_tile = best.apply_rt; out->apply_waves = best.apply_nw;
    out->moment_splits = best.msplit; out->gemv_waves = best.gemv;
    out->us_default = t_default; out->us_tuned = t_tuned;
  }
  return KLST_OK;
}

klst_status klst_tune_save(const char* path) {
  if (!path) return KLST_EINVAL;
  FILE* f = std::fopen(path, "w");
  if (!f) return KLST_EINVAL;
  std::fprintf(f, "# klst launch table: Ny Nxi nvec precision apply_tile apply_waves moment_splits gemv_waves\n");
  for (const auto& [k, t] : klst::dev::tune_all())
    std::fprintf(f, "%d %d %d %d %d %d %d %d\n", k[0], k[1], k[2], k[3], t.apply_rt, t.apply_nw, t.msplit, t.gemv);
  std::fclose(f);
  return KLST_OK;
}

klst_status klst_tune_load(const char* path) {
  if (!path) return KLST_EINVAL;
  FILE* f = std::fopen(path, "r");
  if (!f) return KLST_EINVAL;
  char line[512];
  klst_status st = KLST_OK;
  while (std::fgets(line, sizeof line, f)) {
    if (line[0] == '#' || line[0] == '\n') continue;
    int v[8];
    if (std::sscanf(line, "%d %d %d %d %d %d %d %d", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5], &v[6], &v[7]) != 8 ||
        v[0] < 3 || v[1] < 1 || v[2] < 1 || (v[3] != 0 && v[3] != 1)) {
      st = KLST_EINVAL;
      break;
    }
    klst::dev::Tuning t;
    t.apply_rt = v[4]; t.apply_nw = v[5]; t.msplit = v[6]; t.gemv = v[7];
    klst::dev::tune_set(v[0], v[1], v[2], v[3], t);
  }
  std::fclose(f);
  return st;
}

void klst_tune_clear(void) { klst::dev::tune_clear(); }

klst_status klst_get_stats(const klst_ctx* ctx, klst_stats* out) {
  if (!ctx || !out) return KLST_EINVAL;
  *out = ctx->stats;
  return KLST_OK;
}

klst_status klst_get_history(const klst_ctx* ctx, double* rec, int cap, int* count) {
  if (!ctx || !count || cap < 0 || (cap > 0 && !rec)) return KLST_EINVAL;
  const int total = (int)(ctx->history.size() / KLST_HISTORY_FIELDS);
  *count = total;
  const int nrec = std::min(cap, total);
  std::copy(ctx->history.begin(), ctx->history.begin() + (size_t)nrec * KLST_HISTORY_FIELDS, rec);
  return KLST_OK;
}

klst_status klst_perturbation_macros(klst_ctx* ctx, const void* X, int nvec, void* macros, double* umag) {
  if (!ctx || !X || !macros || !umag || nvec < 1 || nvec > 65535) return KLST_EINVAL;
  if (!ctx->assembled) return fail(ctx, KLST_ESTATE, "klst_perturbation_macros before klst_assemble");
  HIPCHK(hipSetDevice(ctx->opt.device));
  const klst::Problem& p = ctx->prob;
  klst_status s = ensure_mom(ctx, nvec);
  if (s != KLST_OK) return s;
  klst::dev::launch_perturbation_macros(ctx->stream, (const double2*)X, p.n(), nvec, p.Ny, p.Nxi, p.r, ctx->d_M,
                                        ctx->d_mom, ctx->d_base, (double2*)macros, umag);
  HIPCHK(hipGetLastError());
  return KLST_OK;
}

klst_status klst_bgk_relax(klst_ctx* ctx, const klst_grid* grid, const klst_vel* vel, double nu_inf,
                           double s_visc, double* g, double* h, double dt, int max_steps, double tol,
                           int check_every, int* steps_done, double* resid) {
  if (!ctx || !grid || !vel || !g || !h || !vel->xi_x || !vel->xi_y || !vel->w) return KLST_EINVAL;
  const int Ny = grid->Ny, Nxi = vel->Nxi, Dv = vel->Dv;
  if (Ny < 3 || Nxi < 1 || (Dv != 1 && Dv != 2) || !(dt > 0) || !std::isfinite(dt) || max_steps < 0 ||
      check_every < 1 || !(nu_inf >= 0) || !std::isfinite(nu_inf) || !std::isfinite(s_visc) ||
      !(grid->L > 0) || !(grid->s_inf > 0) || !std::isfinite(grid->L) || !std::isfinite(grid->s_inf))
    return fail(ctx, KLST_EINVAL, "klst_bgk_relax: bad sizes, time step or grid");
  for (int k = 0; k < Nxi; ++k)
    if (!(vel->w[k] > 0) || !std::isfinite(vel->xi_x[k]) || !std::isfinite(vel->xi_y[k]))
      return fail(ctx, KLST_EINVAL, "klst_bgk_relax: bad velocity table");
  const size_t cells = (size_t)Ny * Nxi;
  for (size_t e = 0; e < cells; ++e)
    if (!std::isfinite(g[e]) || !std::isfinite(h[e])) return fail(ctx, KLST_EINVAL, "klst_bgk_relax: non-finite state");
  HIPCHK(hipSetDevice(ctx->opt.device));
  hipStream_t st = ctx->stream;
  // cell widths (x_{j-1} - x_{j+1}) / 2 of the mapped nodes; the end nodes are held
  std::vector<double> x(Ny), inv_dx(Ny, 0.0);
  klst::mapped_nodes(Ny, grid->L, grid->s_inf, x.data());
  for (int j = 1; j < Ny - 1; ++j) inv_dx[j] = 2.0 / (x[j - 1] - x[j + 1]);
  std::vector<double> hq(2 * cells);
  for (int j = 0; j < Ny; ++j)
    for (int k = 0; k < Nxi; ++k) {
      hq[((size_t)2 * j) * Nxi + k] = g[(size_t)j * Nxi + k];
      hq[((size_t)2 * j + 1) * Nxi + k] = h[(size_t)j * Nxi + k];
    }
  struct Buffers {
    klst_ctx* c;
    double *q0 = nullptr, *q1 = nullptr, *ka = nullptr, *kb = nullptr, *acc = nullptr, *tab = nullptr,
           *res = nullptr;
    ~Buffers() {
      if (q0) (void)hipStreamSynchronize(c->stream);
      dfree(c, q0); dfree(c, q1); dfree(c, ka); dfree(c, kb); dfree(c, acc); dfree(c, tab); dfree(c, res);
    }
  } b{ctx};
  const size_t nb = sizeof(double) * 2 * cells;
  if (dalloc(ctx, (void**)&b.q0, nb) != KLST_OK || dalloc(ctx, (void**)&b.q1, nb) != KLST_OK ||
      dalloc(ctx, (void**)&b.ka, nb) != KLST_OK || dalloc(ctx, (void**)&b.kb, nb) != KLST_OK ||
      dalloc(ctx, (void**)&b.acc, nb) != KLST_OK ||
      dalloc(ctx, (void**)&b.tab, sizeof(double) * (3 * (size_t)Nxi + Ny)) != KLST_OK ||
      dalloc(ctx, (void**)&b.res, sizeof(double) * Ny * klst::dev::bgk_parts(Nxi)) != KLST_OK)
    return KLST_ENOMEM;
  double *d_xix = b.tab, *d_xiy = b.tab + Nxi, *d_w = b.tab + 2 * Nxi, *d_idx = b.tab + 3 * Nxi;
  HIPCHK(hipMemcpyAsync(b.q0, hq.data(), nb, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(d_xix, vel->xi_x, sizeof(double) * Nxi, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(d_xiy, vel->xi_y, sizeof(double) * Nxi, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(d_w, vel->w, sizeof(double) * Nxi, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(d_idx, inv_dx.data(), sizeof(double) * Ny, hipMemcpyHostToDevice, st));
  std::vector<double> hres((size_t)Ny * klst::dev::bgk_parts(Nxi));
  auto max_resid = [&](double& r) -> klst_status {
    HIPCHK(hipMemcpyAsync(hres.data(), b.res, sizeof(double) * hres.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    r = 0.0;
    for (double v : hres) r = (v > r || !std::isfinite(v)) ? v : r;   // keeps a NaN or inf
    return KLST_OK;
  };
  using klst::dev::launch_bgk_stage;
  double* q = b.q0;
  double* qn = b.q1;
  const double dt6 = dt / 6.0;
  int step = 0;
  for (; step < max_steps; ++step) {
    const bool check = tol > 0 && step % check_every == 0;
    launch_bgk_stage(st, q, nullptr, 0.0, b.ka, b.acc, nullptr, dt6, 1, Ny, Nxi, Dv, d_xix, d_xiy, d_w, d_idx,
                     nu_inf, s_visc, check ? b.res : nullptr);
    if (check) {
      double r = 0.0;
      const klst_status sr = max_resid(r);
      if (sr != KLST_OK) return sr;
      if (!std::isfinite(r)) return fail(ctx, KLST_ENOCONV, "klst_bgk_relax: non-finite state");
      if (r <= tol) break;
    }
    launch_bgk_stage(st, q, b.ka, 0.5 * dt, b.kb, b.acc, nullptr, dt6, 2, Ny, Nxi, Dv, d_xix, d_xiy, d_w, d_idx,
                     nu_inf, s_visc, nullptr);
    launch_bgk_stage(st, q, b.kb, 0.5 * dt, b.ka, b.acc, nullptr, dt6, 3, Ny, Nxi, Dv, d_xix, d_xiy, d_w, d_idx,
                     nu_inf, s_visc, nullptr);
    launch_bgk_stage(st, q, b.ka, dt, b.kb, b.acc, qn, dt6, 4, Ny, Nxi, Dv, d_xix, d_xiy, d_w, d_idx, nu_inf,
                     s_visc, nullptr);
    std::swap(q, qn);
  }
  HIPCHK(hipGetLastError());
  // residual of the final state
  launch_bgk_stage(st, q, nullptr, 0.0, b.ka, b.acc, nullptr, dt6, 1, Ny, Nxi, Dv, d_xix, d_xiy, d_w, d_idx,
                   nu_inf, s_visc, b.res);
  double rfin = 0.0;
  const klst_status sr = max_resid(rfin);
  if (sr != KLST_OK) return sr;
  HIPCHK(hipMemcpyAsync(hq.data(), q, nb, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int j = 0; j < Ny; ++j)
    for (int k = 0; k < Nxi; ++k) {
      g[(size_t)j * Nxi + k] = hq[((size_t)2 * j) * Nxi + k];
      h[(size_t)j * Nxi + k] = hq[((size_t)2 * j + 1) * Nxi + k];
    }
  if (steps_done) *steps_done = step;
  if (resid) *resid = rfin;
  return std::isfinite(rfin) ? KLST_OK : fail(ctx, KLST_ENOCONV, "klst_bgk_relax: non-finite state");
}

klst_status klst_noneq_level(klst_ctx* ctx, double* eneq) {
  if (!ctx || !eneq) return KLST_EINVAL;
  if (!ctx->assembled) return fail(ctx, KLST_ESTATE, "klst_noneq_level before klst_assemble");
  HIPCHK(hipSetDevice(ctx->opt.device));
  const klst::Problem& p = ctx->prob;
  klst::dev::launch_noneq_level(ctx->stream, ctx->d_gc, ctx->d_base, ctx->d_xix, ctx->d_xiy, ctx->d_w, p.Ny,
                                p.Nxi, p.Dv, eneq);
  HIPCHK(hipGetLastError());
  return KLST_OK;
}

}  // extern "C"

// ================================================================ solver ===

namespace {

struct Workspace {
  klst_ctx* ctx;
  int64_t n;
  std::vector<void*> ptrs;
  ~Workspace() {
    for (void* p : ptrs) (void)hipFreeAsync(p, ctx->stream);
  }
  double2* vec(int count) {
    void* p = nullptr;
    if (dalloc(ctx, &p, sizeof(double2) * (size_t)count * n) != KLST_OK) return nullptr;
    ptrs.push_back(p);
    return (double2*)p;
  }
  float2* vec32(int count) {
    void* p = nullptr;
    if (dalloc(ctx, &p, sizeof(float2) * (size_t)count * n) != KLST_OK) return nullptr;
    ptrs.push_back(p);
    return (float2*)p;
  }
  template <class T>
  T* small(size_t count) {
    void* p = nullptr;
    if (dalloc(ctx, &p, sizeof(T) * count) != KLST_OK) return nullptr;
    ptrs.push_back(p);
    return (T*)p;
  }
};

// Upper-triangular solve R X = B (m x m, row-major), in place on B (m x ncols).
void trsm_upper(int m, const std::vector<cd>& R, std::vector<cd>& B, int ncols) {
  for (int c = 0; c < ncols; ++c)
    for (int i = m - 1; i >= 0; --i) {
      cd s = B[(size_t)i * ncols + c];
      for (int q = i + 1; q < m; ++q) s -= R[(size_t)i * m + q] * B[(size_t)q * ncols + c];
      B[(size_t)i * ncols + c] = s / R[(size_t)i * m + i];
    }
}

}  // namespace

extern "C" klst_status klst_solve_shift_invert(klst_ctx* ctx, const double sigma_in[2], int nev,
                                               double* lambda, void* X, int X_on_device, double* resid,
                                               int* nconv_out);

extern "C" klst_status klst_solve(klst_ctx* ctx, const double sigma_in[2], int nev, double* lambda,
                                  void* X, int X_on_device, double* resid, int* nconv_out) {
  using namespace klst::dev;
  if (ctx && ctx->opt.method == 1)
    return klst_solve_shift_invert(ctx, sigma_in, nev, lambda, X, X_on_device, resid, nconv_out);
  if (!ctx || !sigma_in || !lambda) return KLST_EINVAL;
  if (!ctx->assembled) return fail(ctx, KLST_ESTATE, "klst_solve before klst_assemble");
  HIPCHK(hipSetDevice(ctx->opt.device));
  const auto t_start = std::chrono::steady_clock::now();
  const klst::Problem& p = ctx->prob;
  const klst_options& o = ctx->opt;
  const int64_t n = p.n();
  if (nev < 1 || nev > n - p.n_bc || nev > 100 || nev + std::max(o.m_max, o.m_min + 2) > 250)
    return fail(ctx, KLST_EINVAL, "nev out of range (1 <= nev <= min(100, n - n_bc, 250 - m_max))");
  const int m_max = std::max(o.m_max, o.m_min + 2);
  const int m_min = o.m_min;
  const int gm = o.gmres_m;
  // correction-equation budget: inner_max_it, or for 0 one GMRES cycle in FP64
  // and three FP64-refined FP32 cycles in mixed precision (one FP32 cycle alone
  // can stall an ill-conditioned pair near relative residual 1e-7)
  const int imax = o.inner_max_it > 0 ? o.inner_max_it : (o.precision == 1 ? 3 * o.gmres_m : o.gmres_m);
  const cd sigma(sigma_in[0], sigma_in[1]);
  hipStream_t st = ctx->stream;
  ctx->stats = klst_stats{};
  ctx->history.clear();

  klst_status s = pc_setup(ctx, sigma);
  if (s != KLST_OK) return s;
  ctx->stats.pivots_floored = ctx->ilu.floored;
  const double t_setup = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();

  Workspace ws{ctx, n, {}};
  double2* V = ws.vec(m_max + 1);
  double2* W = ws.vec(m_max + 1);
  // up to kcap pairs are locked: after nev, JD goes on until a newly locked
  // eigenvalue is not nearer than the nev-th nearest locked one (it has moved past
  // the nev nearest, so none of them was skipped), then returns the nev nearest
  const int kcap = std::min({2 * nev, 100, 250 - m_max});
  double2* Qb = ws.vec(kcap + 1);
  double2* Zb = ws.vec(kcap + 1);
  double2* Yb = ws.vec(kcap + 1);
  double2* Gb = ws.vec(gm + 1);
  double2* Tmp = ws.vec(m_max);
  double2* tv = ws.vec(1);
  double2* uv = ws.vec(1);
  double2* zv = ws.vec(1);
  double2* rv = ws.vec(1);
  double2* av = ws.vec(1);
  double2* bv = ws.vec(1);
  const bool mixed = (o.precision == 1);
  double2* rho64 = mixed ? ws.vec(1) : nullptr;
  // FP32 mirrors for the mixed-precision inner solve: Krylov basis, [Q u], [K^-1 Z, K^-1 z]
  float2 *Gb32 = nullptr, *Q32 = nullptr, *Y32 = nullptr, *a32 = nullptr, *b32 = nullptr,
         *d32 = nullptr;
  if (mixed) {
    Gb32 = ws.vec32(gm + 1);
    Q32 = ws.vec32(kcap + 1);
    Y32 = ws.vec32(kcap + 1);
    a32 = ws.vec32(1);
    b32 = ws.vec32(1);
    d32 = ws.vec32(1);
    if (!Gb32 || !Q32 || !Y32 || !a32 || !b32 || !d32 || !rho64) return KLST_ENOMEM;
  }
  // FP64 solve with the inner GMRES Krylov basis stored in FP32: the basis and
  // one FP64 work vector holding the current basis vector
  const bool kb32 = !mixed && o.krylov32 == 1;
  float2* Gk32 = kb32 ? ws.vec32(gm + 1) : nullptr;
  double2* wk = kb32 ? ws.vec(1) : nullptr;
  if (kb32 && (!Gk32 || !wk)) return KLST_ENOMEM;
  std::vector<cd> HQY32;   // Q32^H Y32 of the locked vectors (mixed precision)
  // Small device results gathered for one host transfer.  Every column count below
  // is at most kcap + m_max <= 250 (expansion) or kcap + 1 <= 101 (locking), so
  // each region of the expansion layout holds 256 entries and each region of the
  // locking layout 128; regions of one layout never overlap.
  const int SM = 1024;
  enum { X_MB = 4, X_VW = 260, X_CW = 516 };                       // expansion
  enum { L_SA = 0, L_SB = 128, L_QY = 256, L_YQ = 384, L_QY32 = 512, L_YQ32 = 640 };   // locking
  double2* d_c = ws.small<double2>(SM);        // coefficients of Gram-Schmidt passes
  double2* d_c2 = ws.small<double2>(SM);
  double2* d_cw = ws.small<double2>(SM);
  double2* d_small = ws.small<double2>(SM);    // host-bound results
  // basis rotations (m_max x m_max at most), extraction pairs (2 m_max), output
  // vectors (kcap x nev)
  double2* d_coef = ws.small<double2>((size_t)std::max({m_max * m_max, 2 * m_max, kcap * nev}));
  double2* d_Hinv = ws.small<double2>((size_t)(kcap + 1) * (kcap + 1));
  double2* d_H = ws.small<double2>((size_t)(gm + 1) * gm);
  double* d_cs = ws.small<double>(gm);
  double2* d_sn = ws.small<double2>(gm);
  double2* d_g = ws.small<double2>(gm + 1);
  double2* d_yk = ws.small<double2>(gm + 1);
  int* d_done = ws.small<int>(4);
  int* d_steps = ws.small<int>(4);
  int* d_reorth = ws.small<int>(4);   // skip flag of the second Gram-Schmidt pass
  double* d_beta = ws.small<double>(2);
  if (!V || !W || !Qb || !Zb || !Yb || !Gb || !Tmp || !tv || !uv || !zv || !rv || !av || !bv || !d_c || !d_cw ||
      !d_c2 || !d_small || !d_coef || !d_Hinv || !d_H || !d_cs || !d_sn || !d_g || !d_yk || !d_done ||
      !d_steps || !d_beta || !d_reorth)
    return KLST_ENOMEM;
  double2* partial = ctx->d_partial;
  std::vector<double2> hsmall(SM);

  double2* npart = ctx->d_npart;
  if (n > 256LL * 65536) return fail(ctx, KLST_EINVAL, "problem too large for the norm partial table");
  // small results of S^H x (mode as launch_dot_reduce) written to `out` on the device
  auto dot = [&](const double2* s0, int m0, const double2* s1, int m1, const double2* x, double2* out,
                 int mode, const double2* Hinv = nullptr, double2* out2 = nullptr,
                 const int* skip = nullptr) {
    if (m0 + m1 + (mode == 3 ? 1 : 0) == 0) return;
    const int nch = launch_dot_partial(st, s0, m0, s1, m1, x, n, partial, mode == 3 ? 1 : 0, skip);
    launch_dot_reduce(st, partial, m0 + m1, nch, out, mode, Hinv, out2, skip);
  };
  auto sub = [&](const double2* s0, int m0, const double2* s1, int m1, const double2* c, double2* x,
                 const int* skip = nullptr) { launch_subm(st, s0, m0, s1, m1, c, x, nullptr, n, 1.0, skip); };
  double t_host = 0.0, t_wait = 0.0;
  auto since = [](std::chrono::steady_clock::time_point a) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - a).count();
  };
  auto fetch = [&](int count) -> klst_status {
    const auto t0 = std::chrono::steady_clock::now();
    HIPCHK(hipMemcpyAsync(hsmall.data(), d_small, sizeof(double2) * count, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    t_wait += since(t0);
    return KLST_OK;
  };
  auto upload = [&](double2* dst, const std::vector<cd>& src) -> klst_status {
    HIPCHK(hipMemcpyAsync(dst, src.data(), sizeof(double2) * src.size(), hipMemcpyHostToDevice, st));
    return KLST_OK;
  };
  // CGS2 of x against (s0: m0, s1: m1); coefficients summed into c (device), norm^2 into nrm.
  auto dot32 = [&](const float2* s0, int m0, const float2* s1, int m1, const float2* x, double2* out,
                   int mode, const double2* Hinv = nullptr) {
    if (m0 + m1 + (mode == 3 ? 1 : 0) == 0) return;
    const int nch = launch_dot_partial(st, s0, m0, s1, m1, x, n, partial, mode == 3 ? 1 : 0, nullptr);
    launch_dot_reduce(st, partial, m0 + m1, nch, out, mode, Hinv, nullptr, nullptr);
  };
  // CGS2 of x against (s0: m0, s1: m1): coefficients summed into c (device),
  // ||x||^2 into nrm, x / ||x|| into dst
  auto cgs2 = [&](const double2* s0, int m0, const double2* s1, int m1, double2* x, double2* c,
                  double2* nrm, double2* dst) {
    if (m0 + m1 > 0) {
      int nch = launch_dot_partial(st, s0, m0, s1, m1, x, n, partial, 0, nullptr);
      launch_subm_fused(st, s0, m0, s1, m1, partial, nch, nullptr, c, nullptr, x, n, nullptr, nullptr);
      nch = launch_dot_partial(st, s0, m0, s1, m1, x, n, partial, 0, nullptr);
      launch_subm_fused(st, s0, m0, s1, m1, partial, nch, nullptr, nullptr, c, x, n, npart, nullptr);
    } else {
      launch_subm_fused(st, s0, 0, s1, 0, partial, 1, nullptr, nullptr, nullptr, x, n, npart, nullptr);
    }
    launch_scale_norm(st, x, dst, n, npart, nrm, nullptr, 0, 0, nullptr, nullptr, nullptr, nullptr, nullptr,
                      nullptr, 0.0);
  };

  // host mirrors of projected quantities
  std::vector<cd> R, MB, SA, SB, HQY;   // R, MB: m x m; SA, SB, HQY: k x k (row-major)
  int m = 0, k = 0;
  std::vector<cd> h_t;
  start_vector(p, o.seed, 0, h_t);
  if ((s = upload(tv, h_t)) != KLST_OK) return s;
  launch_set_int(st, d_steps, 0);

  int outer = 0, inner = 0, restarts = 0;
  // A pair locks once its deflated Schur-vector residual is below tol / 2: the
  // returned eigenvectors are combinations of the Schur vectors, and their own
  // residuals, checked against tol at the end, run a little above the Schur
  // vectors' ones.
  const double tol_lock = 0.5 * o.tol;
  std::vector<cd> U, T, UL, SR, G, coef;
  cd theta = 0.0;
  bool need_fresh = false;

  auto resize_sq = [](std::vector<cd>& A, int oldm, int newm) {
    std::vector<cd> B((size_t)newm * newm, cd(0.0));
    for (int i = 0; i < std::min(oldm, newm); ++i)
      for (int j = 0; j < std::min(oldm, newm); ++j) B[(size_t)i * newm + j] = A[(size_t)i * oldm + j];
    A.swap(B);
  };
  // sorted Schur of G = R^{-1} MB and QR of R U
  auto extract = [&]() -> bool {
    const auto t0 = std::chrono::steady_clock::now();
    struct Acc { double& t; std::chrono::steady_clock::time_point a; ~Acc() {
      t += std::chrono::duration<double>(std::chrono::steady_clock::now() - a).count(); } } acc{t_host, t0};
    G = MB;
    trsm_upper(m, R, G, m);
    U.assign((size_t)m * m, 0.0);
    T.assign((size_t)m * m, 0.0);
    // the extraction uses the first Schur vector, a restart the first m_min
    if (!klst::sorted_schur(m, G.data(), U.data(), T.data(), std::max(1, m_min))) return false;
    std::vector<cd> RU((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i)
      for (int q = i; q < m; ++q) {
        const cd rv_ = R[(size_t)i * m + q];
        for (int j = 0; j < m; ++j) RU[(size_t)i * m + j] += rv_ * U[(size_t)q * m + j];
      }
    UL.assign((size_t)m * m, 0.0);
    SR.assign((size_t)m * m, 0.0);
    klst::qr_square(m, RU.data(), UL.data(), SR.data());
    return true;
  };
  // The dominant Petrov pair only (largest |mu| of R^{-1} M_B, its unit eigenvector
  // as U[:,0], R U[:,0] / ||R U[:,0]|| as UL[:,0]): what an iteration that does
  // not lock or restart needs, at a fraction of the full sorted Schur form's cost.
  auto extract_first = [&]() -> bool {
    const auto t0 = std::chrono::steady_clock::now();
    struct Acc { double& t; std::chrono::steady_clock::time_point a; ~Acc() {
      t += std::chrono::duration<double>(std::chrono::steady_clock::now() - a).count(); } } acc{t_host, t0};
    G = MB;
    trsm_upper(m, R, G, m);
    cd mu;
    std::vector<cd> x(m), ru(m, 0.0);
    if (!klst::dominant_eig(m, G.data(), mu, x.data())) return false;
    U.assign((size_t)m * m, 0.0);
    T.assign((size_t)m * m, 0.0);
    UL.assign((size_t)m * m, 0.0);
    T[0] = mu;
    double nr = 0.0;
    for (int i = 0; i < m; ++i) {
      U[(size_t)i * m] = x[i];
      for (int q = i; q < m; ++q) ru[i] += R[(size_t)i * m + q] * x[q];
      nr += std::norm(ru[i]);
    }
    nr = std::sqrt(nr);
    if (!(nr > 0)) return false;
    for (int i = 0; i < m; ++i) UL[(size_t)i * m] = ru[i] / nr;
    return true;
  };
  // rotate basis B (m vectors) by columns [c0, c0+cnt) of Mx (m x m) in place
  auto rotate = [&](double2* Bv, const std::vector<cd>& Mx, int c0, int cnt) -> klst_status {
    coef.assign((size_t)m * cnt, 0.0);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < cnt; ++j) coef[(size_t)i * cnt + j] = Mx[(size_t)i * m + c0 + j];
    klst_status s2 = upload(d_coef, coef);
    if (s2 != KLST_OK) return s2;
    launch_combine(st, Bv, m, n, d_coef, cnt, cnt, Tmp, nullptr);
    HIPCHK(hipMemcpyAsync(Bv, Tmp, sizeof(double2) * n * cnt, hipMemcpyDeviceToDevice, st));
    return KLST_OK;
  };
  // new projected matrices after keeping Schur columns [c0, c0+cnt)
  auto project = [&](int c0, int cnt) {
    // MB' = UL^H MB U, R' = SR
    std::vector<cd> MU((size_t)m * m, 0.0), MBn((size_t)cnt * cnt, 0.0), Rn((size_t)cnt * cnt, 0.0);
    for (int i = 0; i < m; ++i)
      for (int q = 0; q < m; ++q) {
        const cd a = MB[(size_t)i * m + q];
        for (int j = c0; j < c0 + cnt; ++j) MU[(size_t)i * m + j] += a * U[(size_t)q * m + j];
      }
    for (int i = c0; i < c0 + cnt; ++i)
      for (int j = c0; j < c0 + cnt; ++j) {
        cd acc = 0.0;
        for (int q = 0; q < m; ++q) acc += std::conj(UL[(size_t)q * m + i]) * MU[(size_t)q * m + j];
        MBn[(size_t)(i - c0) * cnt + (j - c0)] = acc;
        Rn[(size_t)(i - c0) * cnt + (j - c0)] = SR[(size_t)i * m + j];
      }
    MB.swap(MBn);
    R.swap(Rn);
  };

  // is the last locked eigenvalue not nearer than the nev-th nearest of those
  // locked (beyond it, or tied with it as a conjugate partner is for a real target)?
  // After nev locks, each further lock is a guard: the set is complete once
  // guard_run consecutive guards were not nearer than the nev-th nearest locked
  // eigenvalue (beyond it, or tied as a conjugate partner is for a real target).
  const int guard_run = std::max(1, nev / 25);
  int guard_streak = 0;
  // A guard may never reach the locking tolerance: next to a nearly defective
  // eigenvalue pair the residual a Petrov pair can attain is about sqrt(u) of
  // the operator scale.  A guard that stays below kSettleRes and not nearer than
  // the nev-th nearest locked eigenvalue for kSettleIts consecutive outer
  // iterations (with no lock in between), with a margin of sqrt(residual) for
  // the error of its Petrov value, also completes the set.
  constexpr double kSettleRes = 1e-6;
  constexpr int kSettleIts = 50;
  int settle_count = 0, settle_k = -1;
  auto passed_nearest = [&]() {
    std::vector<double> d(k);
    for (int i = 0; i < k; ++i) d[i] = std::abs(SA[(size_t)i * k + i] / SB[(size_t)i * k + i] - sigma);
    const double last = d[k - 1];
    std::nth_element(d.begin(), d.begin() + (nev - 1), d.end());
    guard_streak = (last >= d[nev - 1] * (1.0 - 1e-12)) ? guard_streak + 1 : 0;
    return guard_streak >= guard_run;
  };
  klst_status status = KLST_OK;
  bool complete = false;
  while (!complete) {
    if (outer >= o.max_it) { status = KLST_ENOCONV; break; }
    if (ctx->cancel && *ctx->cancel) { status = KLST_ECANCELLED; break; }
    ++outer;
    // ---- restart
    if (m >= m_max) {
      if (!extract()) return fail(ctx, KLST_ENOCONV, "projected Schur form did not converge");
      if ((s = rotate(V, U, 0, m_min)) != KLST_OK) return s;
      if ((s = rotate(W, UL, 0, m_min)) != KLST_OK) return s;
      project(0, m_min);
      m = m_min;
      ++restarts;
    }
    // ---- expansion: v = orth(t | Q, V); w = orth((A - sigma B) v | Z, W)
    double2* vnew = V + (size_t)m * n;
    double2* wnew = W + (size_t)m * n;
    cgs2(Qb, k, V, m, tv, d_c, d_small + 0, vnew);
    if ((s = op_apply(ctx, sigma, vnew, av, 1, o.op_mode, nullptr)) != KLST_OK) return s;
    cgs2(Zb, k, W, m, av, d_cw, d_small + 1, wnew);
    // small results gathered for one transfer: [0] |v|^2, [1] |w|^2, [3] GMRES steps,
    // [X_MB..] M_B column W^H v_new (m + 1), [X_VW..] V^H w_new (m), [X_CW..] Z,W
    // coefficients (k + m)
    dot(W, m + 1, nullptr, 0, vnew, d_small + X_MB, 0);
    if (m > 0) dot(V, m, nullptr, 0, wnew, d_small + X_VW, 0);
    HIPCHK(hipMemcpyAsync(d_small + 3, d_steps, sizeof(int), hipMemcpyDeviceToDevice, st));
    if (k + m > 0)
      HIPCHK(hipMemcpyAsync(d_small + X_CW, d_cw, sizeof(double2) * (k + m), hipMemcpyDeviceToDevice, st));
    if ((s = fetch(X_CW + k + m)) != KLST_OK) return s;
    {
      const double v2 = hsmall[0].x, w2 = hsmall[1].x;
      if (!(v2 > 0) || !std::isfinite(v2) || !(w2 > 0) || !std::isfinite(w2))
        return fail(ctx, KLST_ENOCONV, "search space breakdown (zero or non-finite expansion vector)");
      int st_prev;
      std::memcpy(&st_prev, &hsmall[3], sizeof(int));
      if (outer > 1 && !need_fresh) inner += st_prev;
      need_fresh = false;
      resize_sq(R, m, m + 1);
      resize_sq(MB, m, m + 1);
      // R column: Gram-Schmidt coefficients against W (after the k Z-coefficients)
      for (int i = 0; i < m; ++i)
        R[(size_t)i * (m + 1) + m] = cd(hsmall[X_CW + k + i].x, hsmall[X_CW + k + i].y);
      R[(size_t)m * (m + 1) + m] = std::sqrt(w2);
      for (int i = 0; i <= m; ++i) MB[(size_t)i * (m + 1) + m] = cd(hsmall[X_MB + i].x, hsmall[X_MB + i].y);
      for (int i = 0; i < m; ++i)
        MB[(size_t)m * (m + 1) + i] = std::conj(cd(hsmall[X_VW + i].x, hsmall[X_VW + i].y));
      ++m;
    }
    // ---- extraction, locking while pairs converge
    double rel = 0.0;
    bool have_pair = false;
    while (true) {
      // the dominant pair first; a converged pair is locked with the full sorted
      // Schur form, whose first pair is the same one up to phase (with a tie in
      // |mu| it may be the other, so its residual is checked again)
      if (!extract_first()) return fail(ctx, KLST_ENOCONV, "projected eigenproblem did not converge");
      bool full = false;
      for (;;) {
        theta = sigma + 1.0 / T[0];
        // u = V U[:,0], z = W UL[:,0]
        coef.assign(2 * (size_t)m, 0.0);
        for (int i = 0; i < m; ++i) { coef[i] = U[(size_t)i * m]; coef[m + i] = UL[(size_t)i * m]; }
        if ((s = upload(d_coef, coef)) != KLST_OK) return s;
        launch_combine(st, V, m, n, d_coef, 1, 1, uv, nullptr);
        launch_combine(st, W, m, n, d_coef + m, 1, 1, zv, nullptr);
        if ((s = op_apply(ctx, theta, uv, rv, 1, o.op_mode, nullptr)) != KLST_OK) return s;
        if (k > 0) {
          dot(Zb, k, nullptr, 0, rv, d_c, 0);
          sub(Zb, k, nullptr, 0, d_c, rv);
        }
        dot(nullptr, 0, nullptr, 0, rv, d_small, 3);
        if ((s = fetch(1)) != KLST_OK) return s;
        const double rn = std::sqrt(hsmall[0].x);
        const double scale = std::abs(theta) >= 1e-6 ? std::abs(theta) : 1.0;
        rel = rn / scale;
        if (!std::isfinite(rel)) return fail(ctx, KLST_ENOCONV, "non-finite residual");
        if (rel > tol_lock || full) break;
        if (!extract()) return fail(ctx, KLST_ENOCONV, "projected Schur form did not converge");
        full = true;
      }
      if (rel > tol_lock) { have_pair = true; break; }
      // ---- lock (u, z): Q, Z, Y = K^{-1} z, partial Schur columns, Q^H Y
      HIPCHK(hipMemcpyAsync(Qb + (size_t)k * n, uv, sizeof(double2) * n, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(Zb + (size_t)k * n, zv, sizeof(double2) * n, hipMemcpyDeviceToDevice, st));
      if ((s = pc_apply(ctx, zv, Yb + (size_t)k * n, nullptr)) != KLST_OK) return s;
      if ((s = op_apply(ctx, 0.0, uv, av, 1, o.op_mode, nullptr)) != KLST_OK) return s;
      launch_mask_bc(st, uv, bv, n, p.Ny, p.Nxi, ctx->d_xix);
      dot(Zb, k + 1, nullptr, 0, av, d_small + L_SA, 0);                   // S_A column
      dot(Zb, k + 1, nullptr, 0, bv, d_small + L_SB, 0);                   // S_B column
      dot(Qb, k + 1, nullptr, 0, Yb + (size_t)k * n, d_small + L_QY, 0);   // Q^H y_new
      dot(Yb, k, nullptr, 0, Qb + (size_t)k * n, d_small + L_YQ, 0);       // Y^H q_new
      if (mixed) {   // FP32 mirrors of the new locked pair for the inner solve
        launch_narrow(st, uv, Q32 + (size_t)k * n, n);
        launch_narrow(st, zv, a32, n);
        if ((s = pc_v(ctx, a32, Y32 + (size_t)k * n, nullptr)) != KLST_OK) return s;
        dot32(Q32, k + 1, nullptr, 0, Y32 + (size_t)k * n, d_small + L_QY32, 0);
        if (k > 0)
          dot32(Y32, k, nullptr, 0, Q32 + (size_t)k * n, d_small + L_YQ32, 0);
      }
      if ((s = fetch(mixed ? L_YQ32 + k : L_YQ + k)) != KLST_OK) return s;
      if (mixed) {
        resize_sq(HQY32, k, k + 1);
        for (int i = 0; i <= k; ++i)
          HQY32[(size_t)i * (k + 1) + k] = cd(hsmall[L_QY32 + i].x, hsmall[L_QY32 + i].y);
        for (int i = 0; i < k; ++i)
          HQY32[(size_t)k * (k + 1) + i] = std::conj(cd(hsmall[L_YQ32 + i].x, hsmall[L_YQ32 + i].y));
      }
      resize_sq(SA, k, k + 1);
      resize_sq(SB, k, k + 1);
      resize_sq(HQY, k, k + 1);
      for (int i = 0; i <= k; ++i) {
        SA[(size_t)i * (k + 1) + k] = cd(hsmall[L_SA + i].x, hsmall[L_SA + i].y);
        SB[(size_t)i * (k + 1) + k] = cd(hsmall[L_SB + i].x, hsmall[L_SB + i].y);
        HQY[(size_t)i * (k + 1) + k] = cd(hsmall[L_QY + i].x, hsmall[L_QY + i].y);
      }
      for (int i = 0; i < k; ++i)
        HQY[(size_t)k * (k + 1) + i] = std::conj(cd(hsmall[L_YQ + i].x, hsmall[L_YQ + i].y));
      ++k;
      // deflate the search and test spaces
      if (m > 1) {
        if ((s = rotate(V, U, 1, m - 1)) != KLST_OK) return s;
        if ((s = rotate(W, UL, 1, m - 1)) != KLST_OK) return s;
      }
      project(1, m - 1);
      --m;
      if (k >= kcap || (k > nev && passed_nearest()) || (k >= nev && m == 0)) { complete = true; break; }
      if (m == 0) break;
    }
    if (complete) break;
    if (!have_pair) {
      // search space emptied by deflation: start again from a fresh vector
      start_vector(p, o.seed, (uint64_t)outer, h_t);
      if ((s = upload(tv, h_t)) != KLST_OK) return s;
      need_fresh = true;
      launch_set_int(st, d_steps, 0);
      continue;
    }
    if (k >= nev) {
      std::vector<double> d(k);
      for (int i = 0; i < k; ++i) d[i] = std::abs(SA[(size_t)i * k + i] / SB[(size_t)i * k + i] - sigma);
      std::nth_element(d.begin(), d.begin() + (nev - 1), d.end());
      // theta itself may be off by about sqrt(rel) (relative) from its eigenvalue
      const double scale = std::abs(theta) >= 1e-6 ? std::abs(theta) : 1.0;
      const bool beyond = std::abs(theta - sigma) - std::sqrt(rel) * scale >= d[nev - 1] * (1.0 - 1e-12);
      if (rel <= kSettleRes && beyond) {
        settle_count = (settle_k == k) ? settle_count + 1 : 1;
        settle_k = k;
      } else {
        settle_count = 0;
      }
      if (settle_count >= kSettleIts) { complete = true; break; }
    }
    // ---- correction equation
    // (I - Zt Zt^H)(A - shift B)(I - Qt Qt^H) t = -r, t _|_ Qt, Qt = [Q u], Zt = [Z z],
    // left-preconditioned with K and the oblique projection I - Yt Ht^{-1} Qt^H,
    // Yt = K^{-1} Zt, Ht = Qt^H Yt (Fokkema-Sleijpen-van der Vorst 1998).
    const cd shift = (rel <= o.fix) ? theta : sigma;
    ctx->history.insert(ctx->history.end(),
                        {(double)outer, (double)k, rel, theta.real(), theta.imag(), rel <= o.fix ? 1.0 : 0.0});
    // GMRES on the device for the projected preconditioned operator; vectors in the
    // precision of V (double2 or float2); rhs in `a` (consumed), result to `tout`.
    auto gmres = [&](auto* Gbp, auto* a, auto* bw, auto* Qt0, auto* ut, auto* Yt0, int kq, int budget,
                     auto* tout, bool first) -> klst_status {
      using V = std::remove_pointer_t<decltype(Gbp)>;
      klst_status s2;
      {
        const int nch = launch_dot_partial(st, (const V*)nullptr, 0, (const V*)nullptr, 0, a, n, partial, 1,
                                           nullptr);
        launch_dot_reduce(st, partial, 0, nch, d_small, 3, nullptr, nullptr, nullptr);
      }
      launch_gmres_init(st, d_small, d_g, d_done, d_steps, d_beta, first ? 1 : 0);
      launch_scale_rsqrt(st, a, Gbp, n, d_small, d_done);
      for (int j = 0; j < budget; ++j) {
        V* gj = Gbp + (size_t)j * n;
        V* gj1 = Gbp + (size_t)(j + 1) * n;
        if ((s2 = op_v(ctx, shift, gj, bw, d_done)) != KLST_OK) return s2;
        if ((s2 = pc_v(ctx, bw, gj1, d_done)) != KLST_OK) return s2;
        // oblique projection: gj1 -= Yt Ht^{-1} Qt^H gj1
        int nch = launch_dot_partial(st, Qt0, kq, ut, 1, gj1, n, partial, 0, d_done);
        launch_subm_fused(st, Yt0, kq + 1, (const V*)nullptr, 0, partial, nch, d_Hinv, nullptr, nullptr,
                          gj1, n, nullptr, d_done);
        // Classical Gram-Schmidt against the Krylov basis, coefficients into
        // Hessenberg column j; with reorth = 1 the second pass runs only when the
        // DGKS test on the device asks for it (the first pass kept less than
        // 1/sqrt(2) of ||x||), with reorth = 0 always
        double2* hcol = d_H + (size_t)j * (gm + 1);
        nch = launch_dot_partial(st, Gbp, j + 1, (const V*)nullptr, 0, gj1, n, partial, 1, d_done);
        launch_subm_fused(st, Gbp, j + 1, (const V*)nullptr, 0, partial, nch, nullptr, hcol, nullptr, gj1, n,
                          npart, d_done);
        const int* skip2 = d_done;
        if (o.reorth == 1) {
          launch_reorth_test(st, partial, j + 1, nch, n, npart, 0.5, d_done, d_reorth);
          skip2 = d_reorth;
        }
        nch = launch_dot_partial(st, Gbp, j + 1, (const V*)nullptr, 0, gj1, n, partial, 0, skip2);
        launch_subm_fused(st, Gbp, j + 1, (const V*)nullptr, 0, partial, nch, nullptr, nullptr, hcol, gj1, n,
                          npart, skip2);
        // h[j+1] = ||gj1||, Givens update, gj1 /= ||gj1||
        launch_scale_norm(st, gj1, (V*)nullptr, n, npart, d_small + 2, d_H, gm + 1, j, d_cs, d_sn, d_g,
                          d_done, d_steps, d_beta, o.inner_rtol);
      }
      launch_gmres_solve(st, d_H, gm + 1, d_g, d_steps, d_yk);
      launch_combine(st, Gbp, budget, n, d_yk, 1, 1, tout, d_steps);
      HIPCHK(hipGetLastError());
      return KLST_OK;
    };
    // The same GMRES in FP64 arithmetic with the Krylov basis stored in FP32 (half
    // the bytes of every Gram-Schmidt pass); the current basis vector is kept in
    // FP64 in wk, and the operator and preconditioner act on it.
    auto gmres_kb32 = [&](double2* a, double2* bw, const double2* Qt0, const double2* ut, const double2* Yt0,
                          int kq, int budget, double2* tout, bool first) -> klst_status {
      klst_status s2;
      {
        const int nch = launch_dot_partial(st, (const double2*)nullptr, 0, (const double2*)nullptr, 0, a, n,
                                           partial, 1, nullptr);
        launch_dot_reduce(st, partial, 0, nch, d_small, 3, nullptr, nullptr, nullptr);
      }
      launch_gmres_init(st, d_small, d_g, d_done, d_steps, d_beta, first ? 1 : 0);
      launch_scale_rsqrt(st, a, wk, n, d_small, d_done, Gk32);
      const float2* nul32 = nullptr;
      for (int j = 0; j < budget; ++j) {
        if ((s2 = op_v(ctx, shift, wk, bw, d_done)) != KLST_OK) return s2;
        if ((s2 = pc_v(ctx, bw, wk, d_done)) != KLST_OK) return s2;
        int nch = launch_dot_partial(st, Qt0, kq, ut, 1, wk, n, partial, 0, d_done);
        launch_subm_fused(st, Yt0, kq + 1, (const double2*)nullptr, 0, partial, nch, d_Hinv, nullptr, nullptr,
                          wk, n, nullptr, d_done);
        double2* hcol = d_H + (size_t)j * (gm + 1);
        nch = launch_dot_partial(st, (const float2*)Gk32, j + 1, nul32, 0, (const double2*)wk, n, partial, 1,
                                 d_done);
        launch_subm_fused(st, (const float2*)Gk32, j + 1, nul32, 0, partial, nch, nullptr, hcol, nullptr, wk, n,
                          npart, d_done);
        const int* skip2 = d_done;
        if (o.reorth == 1) {
          launch_reorth_test(st, partial, j + 1, nch, n, npart, 0.5, d_done, d_reorth);
          skip2 = d_reorth;
        }
        nch = launch_dot_partial(st, (const float2*)Gk32, j + 1, nul32, 0, (const double2*)wk, n, partial, 0,
                                 skip2);
        launch_subm_fused(st, (const float2*)Gk32, j + 1, nul32, 0, partial, nch, nullptr, nullptr, hcol, wk, n,
                          npart, skip2);
        launch_scale_norm(st, wk, Gk32 + (size_t)(j + 1) * n, n, npart, d_small + 2, d_H, gm + 1, j, d_cs, d_sn,
                          d_g, d_done, d_steps, d_beta, o.inner_rtol);
      }
      launch_gmres_solve(st, d_H, gm + 1, d_g, d_steps, d_yk);
      launch_combine(st, (const float2*)Gk32, budget, n, d_yk, 1, 1, tout, d_steps);
      HIPCHK(hipGetLastError());
      return KLST_OK;
    };
    auto set_hinv = [&](const std::vector<cd>& HQ, const double2* col, const double2* row) -> klst_status {
      const int kt = k + 1;
      std::vector<cd> Ht((size_t)kt * kt), Hi((size_t)kt * kt);
      for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) Ht[(size_t)i * kt + j] = HQ[(size_t)i * k + j];
      for (int i = 0; i < kt; ++i) Ht[(size_t)i * kt + k] = cd(col[i].x, col[i].y);
      for (int j = 0; j < k; ++j) Ht[(size_t)k * kt + j] = std::conj(cd(row[j].x, row[j].y));
      if (!klst::invert(kt, Ht.data(), Hi.data()))
        return fail(ctx, KLST_ENOCONV, "singular projected preconditioner (Q^H K^-1 Z)");
      return upload(d_Hinv, Hi);
    };
    if (!mixed) {
      double2* ynew = Yb + (size_t)k * n;
      if ((s = pc_apply(ctx, zv, ynew, nullptr)) != KLST_OK) return s;
      dot(Qb, k, uv, 1, ynew, d_small + 0, 0);                  // Qt^H y_new  (k + 1)
      if (k > 0) dot(Yb, k, nullptr, 0, uv, d_small + 128, 0);  // Y^H u (k)
      if ((s = fetch(128 + k)) != KLST_OK) return s;
      if ((s = set_hinv(HQY, hsmall.data(), hsmall.data() + 128)) != KLST_OK) return s;
      // rhs = -(I - Yt Ht^{-1} Qt^H) K^{-1} r
      if ((s = pc_apply(ctx, rv, av, nullptr)) != KLST_OK) return s;
      dot(Qb, k, uv, 1, av, d_c, 2, d_Hinv);
      sub(Yb, k + 1, nullptr, 0, d_c, av);
      launch_axpby(st, av, av, n, -1.0, 0.0, 0);
      // Restarted GMRES(gm): cycles of at most gm steps until the projected
      // preconditioned residual is below inner_rtol times its initial norm or
      // inner_max_it steps are spent; each restart recomputes the residual from t.
      if ((s = kb32 ? gmres_kb32(av, bv, Qb, uv, Yb, k, std::min(gm, imax), tv, true)
                    : gmres(Gb, av, bv, (const double2*)Qb, (const double2*)uv, (const double2*)Yb, k,
                            std::min(gm, imax), tv, true)) != KLST_OK)
        return s;
      if (imax > gm) {
        double2* resv = Tmp;                 // the rotation buffer is free here
        double2* dt = Tmp + (size_t)n;
        int used = 0;
        while (true) {
          int flags[2] = {0, 0};
          HIPCHK(hipMemcpyAsync(&flags[0], d_done, sizeof(int), hipMemcpyDeviceToHost, st));
          HIPCHK(hipMemcpyAsync(&flags[1], d_steps, sizeof(int), hipMemcpyDeviceToHost, st));
          HIPCHK(hipStreamSynchronize(st));
          used += std::max(flags[1], 1);
          if (flags[0] || used >= imax) break;
          // resv = rhs - (I - Yt Ht^{-1} Qt^H) K^{-1} (A - shift B) t
          if ((s = op_apply(ctx, shift, tv, bv, 1, o.op_mode, nullptr)) != KLST_OK) return s;
          if ((s = pc_apply(ctx, bv, resv, nullptr)) != KLST_OK) return s;
          dot(Qb, k, uv, 1, resv, d_c, 2, d_Hinv);
          sub(Yb, k + 1, nullptr, 0, d_c, resv);
          launch_axpby(st, resv, resv, n, -1.0, 0.0, 0);
          launch_axpby(st, av, resv, n, 1.0, 0.0, 1);
          if ((s = kb32 ? gmres_kb32(resv, bv, Qb, uv, Yb, k, std::min(gm, imax - used), dt, false)
                        : gmres(Gb, resv, bv, (const double2*)Qb, (const double2*)uv, (const double2*)Yb, k,
                                std::min(gm, imax - used), dt, false)) != KLST_OK)
            return s;
          launch_axpby(st, dt, tv, n, 1.0, 0.0, 1);
        }
        launch_set_int(st, d_steps, used);
      }
    } else {
      // Mixed precision: FP64 iterative refinement of the correction equation around
      // FP32 GMRES solves (FP32 operator, preconditioner, Krylov vectors, FP32
      // accumulation); the residual of the correction equation stays FP64.  Each
      // refinement sweep is one GMRES cycle of at most gmres_m steps, so the sweeps
      // form a restarted GMRES whose restarts use the FP64 residual.
      float2* u32 = Q32 + (size_t)k * n;
      float2* ynew = Y32 + (size_t)k * n;
      launch_narrow(st, uv, u32, n);
      launch_narrow(st, zv, a32, n);
      if ((s = pc_v(ctx, a32, ynew, nullptr)) != KLST_OK) return s;
      dot32(Q32, k, u32, 1, ynew, d_small + 0, 0);
      if (k > 0)
        dot32(Y32, k, nullptr, 0, u32, d_small + 128, 0);
      // r <- (I - z z^H) r  (r is already orthogonal to Z)
      dot(zv, 1, nullptr, 0, rv, d_c, 0);
      sub(zv, 1, nullptr, 0, d_c, rv);
      dot(nullptr, 0, nullptr, 0, rv, d_small + 300, 3);
      if ((s = fetch(301)) != KLST_OK) return s;
      if ((s = set_hinv(HQY32, hsmall.data(), hsmall.data() + 128)) != KLST_OK) return s;
      const double rnorm = std::sqrt(hsmall[300].x);
      HIPCHK(hipMemsetAsync(tv, 0, sizeof(double2) * n, st));
      launch_axpby(st, rv, rho64, n, -1.0, 0.0, 0);               // rho = -r
      int used = 0;
      while (used < imax) {
        launch_narrow(st, rho64, a32, n);
        if ((s = pc_v(ctx, a32, b32, nullptr)) != KLST_OK) return s;
        dot32(Q32, k, u32, 1, b32, d_c, 2, d_Hinv);
        launch_subm(st, Y32, k + 1, (const float2*)nullptr, 0, d_c, b32, (float2*)nullptr, n, 1.0, nullptr);
        if ((s = gmres(Gb32, b32, a32, (const float2*)Q32, (const float2*)u32, (const float2*)Y32, k,
                       std::min(gm, imax - used), d32, true)) != KLST_OK)
          return s;
        launch_widen(st, d32, tv, n, 1);                          // t += delta
        int stp = 0;
        HIPCHK(hipMemcpyAsync(&stp, d_steps, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        used += std::max(stp, 1);
        if (used >= imax) break;
        // FP64 residual of the correction equation: rho = -r - Zt-proj (A - shift B) Qt-proj t
        HIPCHK(hipMemcpyAsync(av, tv, sizeof(double2) * n, hipMemcpyDeviceToDevice, st));
        dot(Qb, k, uv, 1, av, d_c, 0);
        sub(Qb, k, uv, 1, d_c, av);
        if ((s = op_apply(ctx, shift, av, bv, 1, o.op_mode, nullptr)) != KLST_OK) return s;
        dot(Zb, k, zv, 1, bv, d_c, 0);
        sub(Zb, k, zv, 1, d_c, bv);
        launch_axpby(st, rv, rho64, n, -1.0, 0.0, 0);
        launch_axpby(st, bv, rho64, n, -1.0, 0.0, 1);
        dot(nullptr, 0, nullptr, 0, rho64, d_small, 3);
        if ((s = fetch(1)) != KLST_OK) return s;
        if (std::sqrt(hsmall[0].x) <= o.inner_rtol * rnorm) break;
      }
      launch_set_int(st, d_steps, used);
    }
  }
  HIPCHK(hipStreamSynchronize(st));
  {
    int st_prev = 0;
    HIPCHK(hipMemcpy(&st_prev, d_steps, sizeof(int), hipMemcpyDeviceToHost));
    if (status == KLST_ENOCONV && !need_fresh) inner += st_prev;
  }

  // nev converged pairs count as success even if max_it stopped the completion check
  if (status == KLST_ENOCONV && k >= nev) status = KLST_OK;
  // ---- eigenpairs of the triangular pencil (S_A, S_B), x_i = Q s_i, of all k locked
  std::vector<cd> lam_all(k), Sv((size_t)k * k, 0.0);
  for (int i = 0; i < k; ++i) {
    lam_all[i] = SA[(size_t)i * k + i] / SB[(size_t)i * k + i];
    Sv[(size_t)i * k + i] = 1.0;
    for (int q = i - 1; q >= 0; --q) {
      cd acc = 0.0;
      for (int t = q + 1; t <= i; ++t)
        acc += (SA[(size_t)q * k + t] - lam_all[i] * SB[(size_t)q * k + t]) * Sv[(size_t)t * k + i];
      const cd d = SA[(size_t)q * k + q] - lam_all[i] * SB[(size_t)q * k + q];
      Sv[(size_t)q * k + i] = (std::abs(d) > 0) ? -acc / d : cd(0.0);
    }
  }
  // Every locked eigenvector x_i = Q s_i on the device.  For a real target on a
  // problem symmetric under the xi_y reflection R (velocity table closed under
  // xi_y -> -xi_y; coupling columns and moment functionals even in xi_y except
  // the v moment's, which is odd: then R A R = conj(A) entry by entry), the
  // partner (conj(lambda), R conj(x)) of a locked complex eigenvalue is an exact
  // eigenpair at the same distance from the target; which locked pairs are each
  // other's partners is read from the overlaps <R conj(x_i), x_j>.
  std::vector<int> mk;
  auto mirror_symmetric = [&]() {
    for (int j = 0; j < p.Ny; ++j)
      for (int f = 0; f < 2; ++f)
        for (int a = 0; a < p.r; ++a) {
          const double sg = (p.r == 4 && a == 2) ? -1.0 : 1.0;
          const double* u = &p.U[(((size_t)j * 2 + f) * p.r + a) * p.Nxi];
          const double* m = &p.M[(((size_t)j * p.r + a) * 2 + f) * p.Nxi];
          for (int kk = 0; kk < p.Nxi; ++kk)
            if (u[mk[kk]] != sg * u[kk] || m[mk[kk]] != sg * m[kk]) return false;
        }
    return true;
  };
  const bool mirror = k > 0 && sigma.imag() == 0.0 && klst::mirror_nodes(p.xi_x, p.xi_y, mk) && mirror_symmetric();
  double2* Xall = ws.vec(std::max(1, k));
  double2* Mall = mirror ? ws.vec(k) : nullptr;
  double2* d_sv = ws.small<double2>((size_t)std::max(1, k) * std::max(1, k));
  double2* d_gram = mirror ? ws.small<double2>((size_t)k * (k + 1)) : nullptr;
  int* d_mk = mirror ? ws.small<int>(p.Nxi) : nullptr;
  if (!Xall || !d_sv || (mirror && (!Mall || !d_gram || !d_mk))) return KLST_ENOMEM;
  if (k > 0) {
    if ((s = upload(d_sv, Sv)) != KLST_OK) return s;
    launch_combine(st, Qb, k, n, d_sv, k, k, Xall, nullptr);
  }
  std::vector<cd> gram;
  std::vector<double> nrm2;
  if (mirror) {
    HIPCHK(hipMemcpyAsync(d_mk, mk.data(), sizeof(int) * p.Nxi, hipMemcpyHostToDevice, st));
    launch_mirror_conj(st, Xall, Mall, n, k, p.Nxi, d_mk);
    for (int j = 0; j < k; ++j) dot(Mall, k, nullptr, 0, Xall + (size_t)j * n, d_gram + (size_t)j * (k + 1), 3);
    std::vector<double2> hg((size_t)k * (k + 1));
    const auto tw = std::chrono::steady_clock::now();
    HIPCHK(hipMemcpyAsync(hg.data(), d_gram, sizeof(double2) * hg.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    t_wait += since(tw);
    gram.assign((size_t)k * k, 0.0);
    nrm2.assign(k, 0.0);
    for (int j = 0; j < k; ++j) {
      for (int i = 0; i < k; ++i) gram[(size_t)i * k + j] = cd(hg[(size_t)j * (k + 1) + i].x, hg[(size_t)j * (k + 1) + i].y);
      nrm2[j] = hg[(size_t)j * (k + 1) + k].x;
    }
  }
  const std::vector<klst::OutputCandidate> sel =
      klst::select_output(lam_all, mirror ? gram.data() : nullptr, mirror ? nrm2.data() : nullptr, sigma, nev);
  const int nconv = (int)sel.size();
  std::vector<cd> lam(nconv);
  for (int o2 = 0; o2 < nconv; ++o2) lam[o2] = sel[o2].lam;
  std::vector<double> res(nconv, 0.0);
  if (nconv > 0) {
    double2* Xd = ws.vec(nconv);
    if (!Xd) return KLST_ENOMEM;
    for (int o2 = 0; o2 < nconv; ++o2)
      HIPCHK(hipMemcpyAsync(Xd + (size_t)o2 * n, (sel[o2].mirrored ? Mall : Xall) + (size_t)sel[o2].src * n,
                            sizeof(double2) * n, hipMemcpyDeviceToDevice, st));
    std::vector<cd> hx((size_t)nconv * n);
    HIPCHK(hipMemcpyAsync(hx.data(), Xd, sizeof(double2) * hx.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    // unit 2-norm, largest entry real positive
    for (int o2 = 0; o2 < nconv; ++o2) {
      cd* xi = &hx[(size_t)o2 * n];
      double nrm = 0.0, big = -1.0;
      int64_t ib = 0;
      for (int64_t t = 0; t < n; ++t) {
        const double a = std::norm(xi[t]);
        nrm += a;
        if (a > big * (1.0 + 1e-12)) { big = a; ib = t; }
      }
      const cd ph = std::conj(xi[ib]) / std::abs(xi[ib]) / std::sqrt(nrm);
      for (int64_t t = 0; t < n; ++t) xi[t] *= ph;
    }
    HIPCHK(hipMemcpyAsync(Xd, hx.data(), sizeof(double2) * hx.size(), hipMemcpyHostToDevice, st));
    for (int i = 0; i < nconv; ++i) {
      if ((s = op_apply(ctx, lam[i], Xd + (size_t)i * n, av, 1, o.op_mode, nullptr)) != KLST_OK) return s;
      dot(nullptr, 0, nullptr, 0, av, d_small + i, 3);
    }
    if ((s = fetch(nconv)) != KLST_OK) return s;
    for (int i = 0; i < nconv; ++i) {
      const double sc = std::abs(lam[i]) >= 1e-6 ? std::abs(lam[i]) : 1.0;
      res[i] = std::sqrt(hsmall[i].x) / sc;
    }
    if (X) {
      if (X_on_device) {
        HIPCHK(hipMemcpyAsync(X, Xd, sizeof(double2) * (size_t)nconv * n, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
      } else {
        std::memcpy(X, hx.data(), sizeof(double2) * hx.size());
      }
    }
  }
  for (int i = 0; i < nconv; ++i) {
    lambda[2 * i] = lam[i].real();
    lambda[2 * i + 1] = lam[i].imag();
    if (resid) resid[i] = res[i];
  }
  if (nconv_out) *nconv_out = nconv;
  ctx->stats.outer_iterations = outer;
  ctx->stats.inner_iterations = inner;
  ctx->stats.restarts = restarts;
  ctx->stats.nconv = nconv;
  ctx->stats.seconds_setup = t_setup;
  ctx->stats.seconds_host = t_host;
  ctx->stats.seconds_wait = t_wait;
  ctx->stats.seconds_total =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  return status;
}

// ===================================================== shift-invert solver ===
//
// Krylov-Schur iteration on S = (A - sigma B)^{-1} B (the paper's Method 1,
// Sec. 4.1, with the exact structured inverse in place of a sparse LU).  Arnoldi
// steps run on the device, CGS2 coefficients and norms collect in device memory;
// at each restart the host forms the Schur form of the Rayleigh quotient sorted by
// |mu| (mu = 1 / (lambda - sigma)), keeps the leading Schur vectors and the next
// Arnoldi vector (S V_k = V_k T_k + v_{m+1} b^T), and accepts the nev leading Ritz
// pairs once their FP64 pencil residuals are below tol.
extern "C" klst_status klst_solve_shift_invert(klst_ctx* ctx, const double sigma_in[2], int nev,
                                               double* lambda, void* X, int X_on_device, double* resid,
                                               int* nconv_out) {
  using namespace klst::dev;
  if (!ctx || !sigma_in || !lambda) return KLST_EINVAL;
  if (!ctx->assembled) return fail(ctx, KLST_ESTATE, "klst_solve_shift_invert before klst_assemble");
  HIPCHK(hipSetDevice(ctx->opt.device));
  const auto t_start = std::chrono::steady_clock::now();
  const klst::Problem& p = ctx->prob;
  const klst_options& o = ctx->opt;
  const int64_t n = p.n();
  const int ncv = std::max(o.m_max, nev + 2);
  if (nev < 1 || nev > 100 || nev > n - p.n_bc || ncv > 250 || ncv > n - p.n_bc)
    return fail(ctx, KLST_EINVAL, "nev or search-space size out of range");
  const cd sigma(sigma_in[0], sigma_in[1]);
  hipStream_t st = ctx->stream;
  ctx->stats = klst_stats{};
  ctx->history.clear();
  klst_status s = pc_setup(ctx, sigma, 2);
  if (s != KLST_OK) return s;
  const double t_setup = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();

  Workspace ws{ctx, n, {}};
  double2* V = ws.vec(ncv + 1);
  double2* av = ws.vec(1);
  double2* Tmp = ws.vec(ncv);
  double2* d_H = ws.small<double2>((size_t)(ncv + 1) * ncv);   // column j at d_H + j (ncv + 1)
  double2* d_nrm = ws.small<double2>(ncv + 1);
  double2* d_coef = ws.small<double2>((size_t)ncv * ncv);
  double2* d_small = ws.small<double2>(256);
  if (!V || !av || !Tmp || !d_H || !d_nrm || !d_coef || !d_small) return KLST_ENOMEM;
  double2* partial = ctx->d_partial;
  double2* npart = ctx->d_npart;
  if (n > 256LL * 65536) return fail(ctx, KLST_EINVAL, "problem too large for the norm partial table");
  double t_host = 0.0, t_wait = 0.0;
  auto now = [] { return std::chrono::steady_clock::now(); };
  auto secs = [](std::chrono::steady_clock::time_point a, std::chrono::steady_clock::time_point b) {
    return std::chrono::duration<double>(b - a).count();
  };
  auto cgs2 = [&](int m0, double2* x, double2* c, double2* nrm) {
    int nch = launch_dot_partial(st, V, m0, (const double2*)nullptr, 0, x, n, partial, 0, nullptr);
    launch_subm_fused(st, V, m0, (const double2*)nullptr, 0, partial, nch, nullptr, c, nullptr, x, n, nullptr,
                      nullptr);
    nch = launch_dot_partial(st, V, m0, (const double2*)nullptr, 0, x, n, partial, 0, nullptr);
    launch_subm_fused(st, V, m0, (const double2*)nullptr, 0, partial, nch, nullptr, nullptr, c, x, n, npart,
                      nullptr);
    launch_scale_norm(st, x, (double2*)nullptr, n, npart, nrm, nullptr, 0, 0, nullptr, nullptr, nullptr,
                      nullptr, nullptr, nullptr, 0.0);
  };
  auto apply_S = [&](const double2* x, double2* y) -> klst_status {
    launch_mask_bc(st, x, av, n, p.Ny, p.Nxi, ctx->d_xix);
    return pc_apply(ctx, av, y, nullptr);
  };
  // start: S applied to a seeded vector (no component in the null space of B)
  {
    std::vector<cd> h;
    start_vector(p, o.seed, 0, h);
    HIPCHK(hipMemcpyAsync(V + n, h.data(), sizeof(double2) * n, hipMemcpyHostToDevice, st));
    if ((s = apply_S(V + n, V)) != KLST_OK) return s;
    launch_subm_fused(st, V, 0, (const double2*)nullptr, 0, partial, 1, nullptr, nullptr, nullptr, V, n, npart,
                      nullptr);
    launch_scale_norm(st, V, (double2*)nullptr, n, npart, d_nrm, nullptr, 0, 0, nullptr, nullptr, nullptr,
                      nullptr, nullptr, nullptr, 0.0);
  }
  std::vector<cd> Hm((size_t)ncv * ncv, 0.0), U, T, Y, Z, lam;
  std::vector<double2> hH((size_t)(ncv + 1) * ncv), hn(ncv + 1);
  const int kkeep = std::min(ncv - 2, nev + (ncv - nev) / 2);
  int kcur = 0, restarts = 0, steps = 0;
  bool done = false;
  klst_status status = KLST_OK;
  std::vector<double> res(nev, 0.0);
  double2* Xd = Tmp;   // candidate Ritz vectors (nev <= ncv - 2 columns of the scratch)
  while (!done) {
    if (restarts >= o.max_it) { status = KLST_ENOCONV; break; }
    if (ctx->cancel && *ctx->cancel) { status = KLST_ECANCELLED; break; }
    // ---- Arnoldi steps kcur .. ncv - 1
    for (int j = kcur; j < ncv; ++j) {
      double2* w = V + (size_t)(j + 1) * n;
      if ((s = apply_S(V + (size_t)j * n, w)) != KLST_OK) return s;
      cgs2(j + 1, w, d_H + (size_t)j * (ncv + 1), d_nrm + j);
      ++steps;
    }
    {
      const auto t0 = now();
      HIPCHK(hipMemcpyAsync(hH.data(), d_H, sizeof(double2) * hH.size(), hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(hn.data(), d_nrm, sizeof(double2) * hn.size(), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      t_wait += secs(t0, now());
    }
    for (int j = kcur; j < ncv; ++j)
      if (!(hn[j].x > 0) || !std::isfinite(hn[j].x))
        return fail(ctx, KLST_ENOCONV, "Krylov space breakdown (zero or non-finite Arnoldi vector)");
    const auto th = now();
    for (int j = kcur; j < ncv; ++j) {
      for (int i = 0; i <= j; ++i) Hm[(size_t)i * ncv + j] = cd(hH[(size_t)j * (ncv + 1) + i].x, hH[(size_t)j * (ncv + 1) + i].y);
      if (j + 1 < ncv) Hm[(size_t)(j + 1) * ncv + j] = std::sqrt(hn[j].x);
    }
    const double beta = std::sqrt(hn[ncv - 1].x);
    U.assign((size_t)ncv * ncv, 0.0);
    T.assign((size_t)ncv * ncv, 0.0);
    if (!klst::sorted_schur(ncv, Hm.data(), U.data(), T.data(), kkeep))
      return fail(ctx, KLST_ENOCONV, "Rayleigh quotient Schur form did not converge");
    // eigenvectors of the leading triangular block, Ritz residual estimates
    Y.assign((size_t)nev * nev, 0.0);
    lam.assign(nev, 0.0);
    double est = 0.0;
    for (int i = 0; i < nev; ++i) {
      const cd mu = T[(size_t)i * ncv + i];
      Y[(size_t)i * nev + i] = 1.0;
      for (int q = i - 1; q >= 0; --q) {
        cd acc = 0.0;
        for (int t = q + 1; t <= i; ++t) acc += T[(size_t)q * ncv + t] * Y[(size_t)t * nev + i];
        const cd d = T[(size_t)q * ncv + q] - mu;
        Y[(size_t)q * nev + i] = (std::abs(d) > 0) ? -acc / d : cd(0.0);
      }
      cd zl = 0.0;
      double zn = 0.0;
      for (int q = 0; q <= i; ++q) zl += U[(size_t)(ncv - 1) * ncv + q] * Y[(size_t)q * nev + i];
      for (int r2 = 0; r2 < ncv; ++r2) {
        cd zr = 0.0;
        for (int q = 0; q <= i; ++q) zr += U[(size_t)r2 * ncv + q] * Y[(size_t)q * nev + i];
        zn += std::norm(zr);
      }
      est = std::max(est, beta * std::abs(zl) / (std::abs(mu) * std::sqrt(zn)));
      lam[i] = sigma + 1.0 / mu;
    }
    t_host += secs(th, now());
    ctx->history.insert(ctx->history.end(),
                        {(double)restarts, 0.0, est, lam[0].real(), lam[0].imag(), 0.0});
    if (est <= 1e-10) {
      // explicit FP64 pencil residuals of the candidates x_i = V U Y[:, i]
      Z.assign((size_t)ncv * nev, 0.0);
      for (int r2 = 0; r2 < ncv; ++r2)
        for (int i = 0; i < nev; ++i) {
          cd acc = 0.0;
          for (int q = 0; q <= i; ++q) acc += U[(size_t)r2 * ncv + q] * Y[(size_t)q * nev + i];
          Z[(size_t)r2 * nev + i] = acc;
        }
      HIPCHK(hipMemcpyAsync(d_coef, Z.data(), sizeof(double2) * Z.size(), hipMemcpyHostToDevice, st));
      launch_combine(st, V, ncv, n, d_coef, nev, nev, Xd, nullptr);
      for (int i = 0; i < nev; ++i) {
        if ((s = op_apply(ctx, lam[i], Xd + (size_t)i * n, av, 1, o.op_mode, nullptr)) != KLST_OK) return s;
        int nch = launch_dot_partial(st, (const double2*)nullptr, 0, (const double2*)nullptr, 0, av, n, partial,
                                     1, nullptr);
        launch_dot_reduce(st, partial, 0, nch, d_small + 2 * i, 3, nullptr, nullptr, nullptr);
        nch = launch_dot_partial(st, (const double2*)nullptr, 0, (const double2*)nullptr, 0, Xd + (size_t)i * n,
                                 n, partial, 1, nullptr);
        launch_dot_reduce(st, partial, 0, nch, d_small + 2 * i + 1, 3, nullptr, nullptr, nullptr);
      }
      std::vector<double2> hs(2 * nev);
      const auto t0 = now();
      HIPCHK(hipMemcpyAsync(hs.data(), d_small, sizeof(double2) * 2 * nev, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      t_wait += secs(t0, now());
      bool ok = true;
      for (int i = 0; i < nev; ++i) {
        const double sc = std::abs(lam[i]) >= 1e-6 ? std::abs(lam[i]) : 1.0;
        res[i] = std::sqrt(hs[2 * i].x) / (sc * std::sqrt(hs[2 * i + 1].x));
        ok = ok && (res[i] <= o.tol);
      }
      if (ok) { done = true; break; }
    }
    // ---- restart: keep the kkeep leading Schur vectors and the next Arnoldi vector
    ++restarts;
    {
      std::vector<cd> cf((size_t)ncv * kkeep);
      for (int r2 = 0; r2 < ncv; ++r2)
        for (int c2 = 0; c2 < kkeep; ++c2) cf[(size_t)r2 * kkeep + c2] = U[(size_t)r2 * ncv + c2];
      HIPCHK(hipMemcpyAsync(d_coef, cf.data(), sizeof(double2) * cf.size(), hipMemcpyHostToDevice, st));
      launch_combine(st, V, ncv, n, d_coef, kkeep, kkeep, Tmp, nullptr);
      HIPCHK(hipMemcpyAsync(V, Tmp, sizeof(double2) * (size_t)kkeep * n, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(V + (size_t)kkeep * n, V + (size_t)ncv * n, sizeof(double2) * n,
                            hipMemcpyDeviceToDevice, st));
      std::vector<cd> Hn((size_t)ncv * ncv, 0.0);
      for (int i = 0; i < kkeep; ++i)
        for (int j = i; j < kkeep; ++j) Hn[(size_t)i * ncv + j] = T[(size_t)i * ncv + j];
      for (int j = 0; j < kkeep; ++j) Hn[(size_t)kkeep * ncv + j] = beta * U[(size_t)(ncv - 1) * ncv + j];
      Hm.swap(Hn);
      kcur = kkeep;
    }
  }
  // ---- output: the converged candidates (or the current ones), nearest first
  const int nconv = done ? nev : 0;
  std::vector<int> order(nconv);
  for (int i = 0; i < nconv; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const double da = std::abs(lam[a] - sigma), db = std::abs(lam[b] - sigma);
    if (std::abs(da - db) > 1e-12 * std::max(da, db)) return da < db;
    return (lam[a].imag() > 0) && !(lam[b].imag() > 0);
  });
  if (nconv > 0) {
    std::vector<cd> hx((size_t)nconv * n);
    HIPCHK(hipMemcpyAsync(hx.data(), Xd, sizeof(double2) * hx.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::vector<cd> ho((size_t)nconv * n);
    for (int o2 = 0; o2 < nconv; ++o2) {
      const cd* xi = &hx[(size_t)order[o2] * n];
      double nrm = 0.0, big = -1.0;
      int64_t ib = 0;
      for (int64_t t = 0; t < n; ++t) {
        const double a = std::norm(xi[t]);
        nrm += a;
        if (a > big * (1.0 + 1e-12)) { big = a; ib = t; }
      }
      const cd ph = std::conj(xi[ib]) / std::abs(xi[ib]) / std::sqrt(nrm);
      cd* xo = &ho[(size_t)o2 * n];
      for (int64_t t = 0; t < n; ++t) xo[t] = xi[t] * ph;
      lambda[2 * o2] = lam[order[o2]].real();
      lambda[2 * o2 + 1] = lam[order[o2]].imag();
      if (resid) resid[o2] = res[order[o2]];
    }
    if (X) {
      if (X_on_device) {
        HIPCHK(hipMemcpyAsync(X, ho.data(), sizeof(double2) * ho.size(), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
      } else {
        std::memcpy(X, ho.data(), sizeof(double2) * ho.size());
      }
    }
  }
  if (nconv_out) *nconv_out = nconv;
  ctx->stats.outer_iterations = restarts;
  ctx->stats.inner_iterations = steps;
  ctx->stats.restarts = restarts;
  ctx->stats.nconv = nconv;
  ctx->stats.seconds_setup = t_setup;
  ctx->stats.seconds_host = t_host;
  ctx->stats.seconds_wait = t_wait;
  ctx->stats.seconds_total = secs(t_start, now());
  return status;
}

// ================================================================ server ===
//
// Continuous batching of independent solves (stability sweeps).  `slots`
// workers each own a context on their own non-blocking stream, so admitted
// solves overlap on the device and their host-side work overlaps on the CPU.
// A request is admitted (FIFO) when a worker is free and its modelled HBM
// footprint fits under the budget; it then runs assemble + solve and keeps
// its results until fetched.  Each request runs alone on its context with
// deterministic kernels, so its result does not depend on what else is running.

namespace {

struct Request {
  uint64_t ticket = 0;
  klst_grid grid{};
  int Nxi = 0, Dv = 2;
  std::vector<double> xi_x, xi_y, w, rho, u, T, g_c, h_c;
  int mode = 0;
  double s_visc = 0, nu_inf = 0, beta = 0, sigma[2] = {0, 0};
  int nev = 0;
  size_t footprint = 0;
  std::atomic<int> state{0};   // 0 queued, 1 running, 2 done, 3 failed, 4 cancelled
  volatile int cancel = 0;
  klst_status status = KLST_OK;
  std::string err;
  std::vector<double> lambda, resid, X;
  int nconv = 0;
  klst_stats stats{};
  double t_submit = 0, t_start = 0, t_done = 0;
};

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct klst_server {
  klst_options opt{};
  int slots = 1;
  size_t budget = 0, in_use = 0, peak_bytes = 0;
  int running = 0, peak_running = 0;
  int max_queue = 1 << 16;
  int want_vectors = 1;
  std::mutex mu;
  std::condition_variable cv, done_cv;
  std::deque<std::shared_ptr<Request>> queue;
  std::unordered_map<uint64_t, std::shared_ptr<Request>> all;
  std::vector<std::thread> workers;
  std::vector<klst_ctx*> ctxs;
  std::vector<hipStream_t> streams;
  bool stop = false;
  uint64_t next = 1;
};

extern "C" size_t klst_footprint_bytes(int Ny, int Nxi, int nev, const klst_options* opt) {
  klst_options o;
  if (opt) o = *opt; else klst_default_options(&o);
  if (Ny < 1 || Nxi < 1 || nev < 1) return 0;
  const size_t n = 2ull * Ny * Nxi, r = 4, cvec = 16 * n;
  const int m_max = std::max(o.m_max, o.m_min + 2), gm = o.gmres_m;
  const int kcap = std::max(nev, std::min({2 * nev, 100, 250 - m_max}));
  const int nl = std::max(1, std::min(o.lines_per_block, 2 * Nxi));
  const size_t nblocks = (2ull * Nxi + nl - 1) / nl;
  size_t b = 0;
  b += 8ull * (2 * Ny * Ny + 2 * Nxi + Ny) + 2 * 8ull * Ny * 2 * r * Nxi + 16ull * Ny * r * 8;  // tables
  const size_t Rd = r * (size_t)Ny;
  if (o.method == 1) {   // shift-invert: structured inverse, basis, scratch
    const int ncv = std::max(o.m_max, nev + 2);
    b += 16ull * Nxi * Ny * Ny + 16ull * Rd * Rd + 16ull * Rd;
    if (o.op_mode == 1) b += 20 * n * (Ny - 1 + 2ull * Nxi) + 8 * (n + 1);
    b += cvec * (2ull * ncv + 2 + nev) + 16ull * ((size_t)(ncv + 1) * ncv + ncv * ncv + 512);
    b += 16ull * 512 * 256;
    return b;
  }
  if (o.pc_kernel == 2) {
    b += 16ull * Nxi * Ny * Ny + 16ull * Rd * Rd + 16ull * Rd;                          // P^-1, S^-1, d
  } else {
    b += 16ull * 2 * Nxi * Ny * Ny + 16ull * nblocks * nl * nl * Ny;                     // ILU factors
    if (o.pc_kernel == 1) b += 16ull * nblocks * (size_t)(nl * Ny) * (nl * Ny) + 8 * (nblocks + 1);
  }
  if (o.precision == 1) {
    b += 4ull * (2 * Ny * Ny + 2 * Nxi + Ny) + 2 * 4ull * Ny * 2 * r * Nxi + 8ull * Ny * r * 8;
    if (o.pc_kernel == 2) b += 8ull * Nxi * Ny * Ny + 8ull * Rd * Rd + 8ull * Rd;
    else b += 8ull * nblocks * (size_t)(nl * Ny) * (nl * Ny);
    b += 8ull * n * ((gm + 1) + 2 * (kcap + 1) + 3) + cvec;
  }
  if (o.op_mode == 1) {
    const size_t nnz = n * (Ny - 1 + 2ull * Nxi);
    b += 20 * nnz + 8 * (n + 1);
  }
  b += cvec * (2ull * (m_max + 1) + 3ull * (kcap + 1) + (gm + 1) + m_max + 6 + nev);    // JD workspace
  if (o.precision == 0 && o.krylov32 == 1) b += 8ull * n * (gm + 1) + cvec;            // FP32 Krylov basis
  const size_t ncoef = std::max({(size_t)m_max * m_max, (size_t)2 * m_max, (size_t)kcap * nev});
  b += 16ull * 512 * 256 + 16ull * (4 * 1024 + ncoef + (size_t)(kcap + 1) * (kcap + 1) +
                                    (gm + 1) * (gm + 3));                           // reductions, small
  return b;
}

namespace {

void serve_one(klst_server* sv, klst_ctx* ctx, Request& r) {
  klst_vel vel{r.Nxi, r.xi_x.data(), r.xi_y.data(), r.w.data(), r.Dv};
  klst_base base{};
  base.mode = r.mode;
  base.s_visc = r.s_visc;
  base.nu_inf = r.nu_inf;
  if (r.mode == 0) { base.rho = r.rho.data(); base.u = r.u.data(); base.T = r.T.data(); }
  else { base.g_c = r.g_c.data(); base.h_c = r.h_c.data(); }
  ctx->cancel = &r.cancel;
  klst_status st = klst_assemble(ctx, &r.grid, &vel, &base, r.beta);
  if (st == KLST_OK) {
    r.lambda.assign(2 * r.nev, 0.0);
    r.resid.assign(r.nev, 0.0);
    if (sv->want_vectors) r.X.assign((size_t)2 * r.nev * ctx->prob.n(), 0.0);
    st = klst_solve(ctx, r.sigma, r.nev, r.lambda.data(), sv->want_vectors ? r.X.data() : nullptr, 0,
                    r.resid.data(), &r.nconv);
    r.stats = ctx->stats;
  }
  if (st != KLST_OK) r.err = ctx->err;
  ctx->cancel = nullptr;
  r.status = st;
}

void worker_main(klst_server* sv, int wi) {
  klst_ctx* ctx = sv->ctxs[wi];
  hipSetDevice(sv->opt.device);
  for (;;) {
    std::shared_ptr<Request> r;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv.wait(lk, [&] {
        return sv->stop ||
               (!sv->queue.empty() && sv->in_use + sv->queue.front()->footprint <= sv->budget);
      });
      if (sv->stop) return;
      r = sv->queue.front();
      sv->queue.pop_front();
      if (r->cancel) {
        r->state = 4;
        r->status = KLST_ECANCELLED;
        r->t_done = now_s();
        sv->done_cv.notify_all();
        sv->cv.notify_all();
        continue;
      }
      sv->in_use += r->footprint;
      sv->running += 1;
      sv->peak_bytes = std::max(sv->peak_bytes, sv->in_use);
      sv->peak_running = std::max(sv->peak_running, sv->running);
      r->t_start = now_s();
      r->state = 1;
    }
    serve_one(sv, ctx, *r);
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->in_use -= r->footprint;
      sv->running -= 1;
      r->t_done = now_s();
      r->state = (r->status == KLST_OK || r->status == KLST_ENOCONV) ? 2
                 : (r->status == KLST_ECANCELLED ? 4 : 3);
    }
    sv->done_cv.notify_all();
    sv->cv.notify_all();
  }
}

}  // namespace

extern "C" klst_status klst_server_create(klst_server** out, const klst_options* opt, int slots,
                                          size_t hbm_budget_bytes, int want_vectors) {
  if (!out || slots < 1 || slots > 64) return KLST_EINVAL;
  *out = nullptr;
  klst_server* sv = new klst_server();
  if (opt) sv->opt = *opt; else klst_default_options(&sv->opt);
  sv->slots = slots;
  sv->want_vectors = want_vectors ? 1 : 0;
  if (hipSetDevice(sv->opt.device) != hipSuccess) { delete sv; return KLST_EDEVICE; }
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) { delete sv; return KLST_EDEVICE; }
  sv->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.8 * (double)free_b);
  for (int i = 0; i < slots; ++i) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) { klst_server_destroy(sv); return KLST_EDEVICE; }
    sv->streams.push_back(s);
    klst_options o = sv->opt;
    o.stream = s;
    klst_ctx* c = nullptr;
    const klst_status st = klst_create(&c, &o);
    if (st != KLST_OK) { klst_server_destroy(sv); return st; }
    sv->ctxs.push_back(c);
  }
  for (int i = 0; i < slots; ++i) sv->workers.emplace_back(worker_main, sv, i);
  *out = sv;
  return KLST_OK;
}

extern "C" void klst_server_destroy(klst_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    for (auto& q : sv->queue) q->cancel = 1;
    for (auto& kv : sv->all) kv.second->cancel = 1;
  }
  sv->cv.notify_all();
  for (auto& t : sv->workers) t.join();
  for (klst_ctx* c : sv->ctxs) klst_destroy(c);
  for (hipStream_t s : sv->streams) hipStreamDestroy(s);
  delete sv;
}

extern "C" klst_status klst_submit(klst_server* sv, const klst_grid* grid, const klst_vel* vel,
                                   const klst_base* base, double beta, const double sigma[2], int nev,
                                   uint64_t* ticket) {
  if (!sv || !grid || !vel || !base || !sigma || !ticket || nev < 1) return KLST_EINVAL;
  // validate the inputs once on the host (same checks as klst_assemble)
  {
    klst::Problem p;
    if (!klst::build_problem(grid, vel, base, beta, p).empty()) return KLST_EINVAL;
    if (nev > p.n() - p.n_bc) return KLST_EINVAL;
  }
  auto r = std::make_shared<Request>();
  r->grid = *grid;
  r->Nxi = vel->Nxi;
  r->Dv = vel->Dv;
  r->xi_x.assign(vel->xi_x, vel->xi_x + vel->Nxi);
  r->xi_y.assign(vel->xi_y, vel->xi_y + vel->Nxi);
  r->w.assign(vel->w, vel->w + vel->Nxi);
  r->mode = base->mode;
  if (base->mode == 0) {
    r->rho.assign(base->rho, base->rho + grid->Ny);
    r->u.assign(base->u, base->u + grid->Ny);
    r->T.assign(base->T, base->T + grid->Ny);
  } else {
    r->g_c.assign(base->g_c, base->g_c + (size_t)grid->Ny * vel->Nxi);
    r->h_c.assign(base->h_c, base->h_c + (size_t)grid->Ny * vel->Nxi);
  }
  r->s_visc = base->s_visc;
  r->nu_inf = base->nu_inf;
  r->beta = beta;
  r->sigma[0] = sigma[0];
  r->sigma[1] = sigma[1];
  r->nev = nev;
  r->footprint = klst_footprint_bytes(grid->Ny, vel->Nxi, nev, &sv->opt);
  if (r->footprint > sv->budget) return KLST_ENOMEM;   // would never be admitted
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if ((int)sv->queue.size() >= sv->max_queue) return KLST_EBUSY;
    r->ticket = sv->next++;
    r->t_submit = now_s();
    sv->queue.push_back(r);
    sv->all[r->ticket] = r;
    *ticket = r->ticket;
  }
  sv->cv.notify_all();
  return KLST_OK;
}

extern "C" klst_status klst_poll(klst_server* sv, uint64_t ticket, int* state) {
  if (!sv || !state) return KLST_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->all.find(ticket);
  if (it == sv->all.end()) return KLST_EINVAL;
  *state = it->second->state.load();
  return KLST_OK;
}

extern "C" klst_status klst_wait(klst_server* sv, uint64_t ticket, double timeout_s) {
  if (!sv) return KLST_EINVAL;
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->all.find(ticket);
  if (it == sv->all.end()) return KLST_EINVAL;
  auto r = it->second;
  auto pred = [&] { return r->state.load() >= 2; };
  if (timeout_s < 0) sv->done_cv.wait(lk, pred);
  else if (!sv->done_cv.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) return KLST_EBUSY;
  return KLST_OK;
}

extern "C" klst_status klst_cancel(klst_server* sv, uint64_t ticket) {
  if (!sv) return KLST_EINVAL;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->all.find(ticket);
    if (it == sv->all.end()) return KLST_EINVAL;
    it->second->cancel = 1;
  }
  sv->cv.notify_all();
  return KLST_OK;
}

extern "C" klst_status klst_fetch(klst_server* sv, uint64_t ticket, double* lambda, void* X,
                                  double* resid, int* nconv, double timing[3], klst_stats* stats) {
  if (!sv) return KLST_EINVAL;
  std::shared_ptr<Request> r;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->all.find(ticket);
    if (it == sv->all.end()) return KLST_EINVAL;
    r = it->second;
    if (r->state.load() < 2) return KLST_EBUSY;
    sv->all.erase(it);
  }
  const int k = r->nconv;
  if (lambda && !r->lambda.empty()) std::memcpy(lambda, r->lambda.data(), sizeof(double) * 2 * k);
  if (resid && !r->resid.empty()) std::memcpy(resid, r->resid.data(), sizeof(double) * k);
  if (X && !r->X.empty()) {
    const size_t nn = 2ull * r->grid.Ny * r->Nxi;
    std::memcpy(X, r->X.data(), sizeof(double) * 2 * nn * k);
  }
  if (nconv) *nconv = k;
  if (timing) {
    timing[0] = r->t_start > 0 ? r->t_start - r->t_submit : 0.0;   // queueing
    timing[1] = r->t_start > 0 ? r->t_done - r->t_start : 0.0;     // service
    timing[2] = r->t_done - r->t_submit;                           // latency
  }
  if (stats) *stats = r->stats;
  return r->status;
}

extern "C" klst_status klst_server_stats(klst_server* sv, int* peak_running, size_t* peak_bytes,
                                         size_t* budget) {
  if (!sv) return KLST_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  if (peak_running) *peak_running = sv->peak_running;
  if (peak_bytes) *peak_bytes = sv->peak_bytes;
  if (budget) *budget = sv->budget;
  return KLST_OK;
}
