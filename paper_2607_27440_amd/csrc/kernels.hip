// HIP kernels for gfx950 (CDNA4, 64-wide wavefronts).
//
// Vectors are complex FP64 stored as double2 (re, im), unknown (j, f, k) at
// (2 j + f) * Nxi + k.  All reductions are deterministic: fixed partitions whose
// partial sums are combined in a fixed order by the kernel that consumes them,
// with no cross-workgroup synchronisation.
#include <hip/hip_runtime.h>
#include <atomic>
#include <algorithm>
#include <array>
#include <cstdint>
#include <map>
#include <mutex>
#include <type_traits>
#include <vector>

#include "kernels.hpp"

namespace klst {
namespace dev {

// complex vector type of a real type
template <class R> struct cvec;
template <> struct cvec<double> { using type = double2; };
template <> struct cvec<float> { using type = float2; };
template <class R> using cv = typename cvec<R>::type;

template <class R> __device__ __forceinline__ cv<R> mk(R a, R b) { cv<R> v; v.x = a; v.y = b; return v; }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
template <class R> __device__ __forceinline__ cv<R> narrow(double2 c) { return mk<R>((R)c.x, (R)c.y); }

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {   // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

// Entry of a stored vector of real type RS in arithmetic type R.
template <class R, class RS>
__device__ __forceinline__ cv<R> as_cv(cv<RS> v) { return mk<R>((R)v.x, (R)v.y); }

// sum_{i < m} S_i[t] c[i * cstride] with the loads of eight vectors issued before
// their products are accumulated (c indices are wave-uniform: scalar loads).
// Vectors stored in real type RS, coefficients in FP64 (narrowed to R),
// accumulation in R.
template <class R, class RS = R>
__device__ __forceinline__ cv<R> lincomb(const cv<RS>* __restrict__ S, int m, int64_t n, int64_t t,
                                         const double2* __restrict__ c, int cstride) {
  cv<R> acc = mk<R>(0, 0);
  int i = 0;
  for (; i + 8 <= m; i += 8) {
    cv<RS> sv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) sv[u] = S[(int64_t)(i + u) * n + t];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      acc = cadd(acc, cmul(as_cv<R, RS>(sv[u]), narrow<R>(c[(int64_t)(i + u) * cstride])));
  }
  for (; i < m; ++i) acc = cadd(acc, cmul(as_cv<R, RS>(S[(int64_t)i * n + t]), narrow<R>(c[(int64_t)i * cstride])));
  return acc;
}

// 64-bit value of lane l' for each lane l, l' given by a DPP lane pattern
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wavefront (all lanes active), the same value in
// every lane.  A fixed butterfly: lane pairs l ^ 1 and l ^ 2 (quad
// permutations), then the two quads of each 8 (half-row mirror), the two halves
// of each 16 (row mirror), the two rows of each 32 (swizzle swap 16), each
// stage adding two equal-shaped partial sums, and finally the two 32-lane
// halves read from lanes 0 and 32.  Addition is commutative in IEEE
// arithmetic, so every lane of a group holds the same bits after each stage and
// the result is deterministic.  The lane moves run on the VALU (DPP) and the
// LDS crossbar without memory traffic, unlike 64-lane permutes.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xB1>(v);    // quad_perm [1, 0, 3, 2]
  v += dpp_f64<0x4E>(v);    // quad_perm [2, 3, 0, 1]
  v += dpp_f64<0x141>(v);   // row_half_mirror
  v += dpp_f64<0x140>(v);   // row_mirror
  {
    const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), 0x401F);   // lane ^ 16 within 32
    const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), 0x401F);
    v += __hiloint2double(hi, lo);
  }
  const double h0 = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 0),
                                     __builtin_amdgcn_readlane(__double2loint(v), 0));
  const double h1 = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 32),
                                     __builtin_amdgcn_readlane(__double2loint(v), 32));
  return h0 + h1;
}

// lane ^ 4 within each row of 16: lanes 0-3 and 8-11 read lane + 4 (row_shl:4),
// lanes 4-7 and 12-15 read lane - 4 (row_shr:4)
__device__ __forceinline__ double dpp_xor4_f64(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  int rlo = __builtin_amdgcn_update_dpp(0, lo, 0x104, 0xF, 0x5, false);
  int rhi = __builtin_amdgcn_update_dpp(0, hi, 0x104, 0xF, 0x5, false);
  rlo = __builtin_amdgcn_update_dpp(rlo, lo, 0x114, 0xF, 0xA, false);
  rhi = __builtin_amdgcn_update_dpp(rhi, hi, 0x114, 0xF, 0xA, false);
  return __hiloint2double(rhi, rlo);
}

// Eight wavefront sums at once, each bit for bit the one wave_sum gives: the
// same pairs at every level (lanes l ^ 1, l ^ 2, l ^ 4, l ^ 8, l ^ 16, then the
// two 32-lane halves), but at each of the first three levels a lane keeps half
// of its values and adds its partner's copies of just those, so the later
// levels move one value instead of eight.  Lane l returns the sum of
// p[4 (l & 1) + 2 ((l >> 1) & 1) + ((l >> 2) & 1)].  All lanes active.
__device__ __forceinline__ double wave_sum8(const double (&p)[8]) {
  const int lane = threadIdx.x & 63;
  const bool b0 = (lane & 1) != 0, b1 = (lane & 2) != 0, b2 = (lane & 4) != 0;
  double q[4], t[2];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double keep = b0 ? p[4 + i] : p[i], send = b0 ? p[i] : p[4 + i];
    q[i] = keep + dpp_f64<0xB1>(send);         // quad_perm [1, 0, 3, 2]
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double keep = b1 ? q[2 + i] : q[i], send = b1 ? q[i] : q[2 + i];
    t[i] = keep + dpp_f64<0x4E>(send);         // quad_perm [2, 3, 0, 1]
  }
  double v;
  {
    const double keep = b2 ? t[1] : t[0], send = b2 ? t[0] : t[1];
    v = keep + dpp_xor4_f64(send);
  }
  v += dpp_f64<0x128>(v);                      // row_ror:8 = lane ^ 8 within 16
  {
    const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), 0x401F);   // lane ^ 16 within 32
    const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), 0x401F);
    v += __hiloint2double(hi, lo);
  }
  {
    const int addr = (lane ^ 32) << 2;
    const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(v));
    v += __hiloint2double(hi, lo);
  }
  return v;
}

// Sum of a double2 over a 256-thread block, result valid in thread 0.
__device__ __forceinline__ double2 block_sum256(double2 v, double2* sh /*[4]*/) {
  v.x = wave_sum(v.x);
  v.y = wave_sum(v.y);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double2 r = make_double2(0.0, 0.0);
  if (threadIdx.x == 0) {
    for (int i = 0; i < 4; ++i) r = cadd(r, sh[i]);
  }
  __syncthreads();
  return r;
}

// Item of workgroup L in a 1-D grid of N workgroups such that each XCD takes a
// contiguous range of items, balanced to within one.  Workgroups are dispatched
// round robin over the 8 XCDs (L runs on XCD L mod 8), each XCD with its own
// L2: XCD x runs L = x, x + 8, ..., i.e. items x q + min(x, N mod 8) + i, q =
// N / 8.  Items that share tables (the same column tile of U, the same node of
// M, for consecutive vectors) then meet in one L2.
__device__ __forceinline__ int64_t xcd_item(int64_t L, int64_t N) {
  const int64_t x = L & 7, i = L >> 3, q = N >> 3, rm = N & 7;
  return x * q + (x < rm ? x : rm) + i;
}

// ------------------------------------------------------------ operator ----

// One output entry of y = (A - tau B) x from its streaming sum (sr, si) =
// (D_x x)(j, c): xi_x times the sum plus the diagonal (dre + i dim) times x(j,
// c); then op_moment subtracts each rank-r moment term.  Written as explicit
// fused multiply-adds so that every operator kernel rounds an entry the same
// way, whatever contractions the compiler would pick in each.
__device__ __forceinline__ double2 op_out(double xik, double sr, double si, double dre, double dim,
                                          double2 xjc) {
  double2 o;
  o.x = fma(xik, sr, fma(dre, xjc.x, -(dim * xjc.y)));
  o.y = fma(xik, si, fma(dre, xjc.y, dim * xjc.x));
  return o;
}
__device__ __forceinline__ void op_moment(double2& o, double ua, double2 ma) {
  o.x = fma(-ua, ma.x, o.x);
  o.y = fma(-ua, ma.y, o.y);
}
// The same entry in FP32 (the mixed solve's operator), as k_apply_mfma32 forms it.
__device__ __forceinline__ float2 op_out(float xik, float sr, float si, float dre, float dim, float2 xjc) {
  float2 o;
  o.x = fmaf(xik, sr, fmaf(dre, xjc.x, -(dim * xjc.y)));
  o.y = fmaf(xik, si, fmaf(dre, xjc.y, dim * xjc.x));
  return o;
}
__device__ __forceinline__ void op_moment(float2& o, float ua, float2 ma) {
  o.x = fmaf(-ua, ma.x, o.x);
  o.y = fmaf(-ua, ma.y, o.y);
}

// Perturbation moments m_a(j) = sum_{f,p} M[j][a][f][p] x[j][f][p] (rank r <= 4)
// for each node j and vector v, split over S column parts: workgroup
// (j * S + part, v) writes the partial sums of its part to mom[((v Ny + j) S +
// part) r + a]; the operator kernels add the S parts in fixed order.
template <class R>
__global__ void __launch_bounds__(256) k_moments(const cv<R>* __restrict__ x, int64_t n, int Ny,
                                                 int Nxi, int r, const R* __restrict__ M,
                                                 cv<R>* __restrict__ mom, int S,
                                                 const int* __restrict__ skip, int vmaj) {
  __shared__ double2 sh[4][4];
  const int sk = skip ? *skip : 0;
  // vmaj > 0: a 1-D grid of Ny S vmaj workgroups ordered node-part major, vector
  // minor, spread over the XCDs by xcd_item (a node's M rows are read from one
  // L2 for all vectors); else grid (Ny S, nvec)
  int j, part, v;
  if (vmaj > 0) {
    const int64_t item = xcd_item(blockIdx.x, gridDim.x);
    v = (int)(item % vmaj);
    const int q = (int)(item / vmaj);
    j = q / S;
    part = q - j * S;
  } else {
    j = blockIdx.x / S;
    part = blockIdx.x - j * S;
    v = blockIdx.y;
  }
  const int nc = 2 * Nxi;
  const int per = (nc + S - 1) / S;
  const int cbeg = part * per, cend = min(nc, cbeg + per);
  const cv<R>* xj = x + (int64_t)v * n + (int64_t)j * nc;
  R ar[4] = {0, 0, 0, 0}, ai[4] = {0, 0, 0, 0};
  // columns c, c + 256, ... in order; four of them (x and the r M rows) loaded
  // together, the first four before the skip flag is tested
  const R* Mj = M + (int64_t)j * r * nc;
  cv<R> xv[4];
  R mw[4][4];
  auto load = [&](int c0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = c0 + 256 * u;
      const bool ok = c < cend;
      xv[u] = ok ? xj[c] : mk<R>(0, 0);
#pragma unroll
      for (int a = 0; a < 4; ++a) mw[u][a] = (ok && a < r) ? Mj[(int64_t)a * nc + c] : (R)0;
    }
  };
  int c0 = cbeg + threadIdx.x;
  load(c0);
  if (sk) return;
  for (;;) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (c0 + 256 * u < cend) {
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          if (a < r) {
            ar[a] += mw[u][a] * xv[u].x;
            ai[a] += mw[u][a] * xv[u].y;
          }
        }
      }
    }
    c0 += 1024;
    if (c0 >= cend) break;
    load(c0);
  }
  // all r sums of the four wavefronts in one exchange: the eight wave sums
  // together (wave_sum8, lane l < 8 holding entry q(l) of sh[wv] read as 8
  // doubles), one barrier, then thread a adds the four waves' values in wave
  // order
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double pv[8];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    pv[2 * a] = (a < r) ? (double)ar[a] : 0.0;
    pv[2 * a + 1] = (a < r) ? (double)ai[a] : 0.0;
  }
  const double ws = wave_sum8(pv);
  if (lane < 8) {
    const int q = 4 * (lane & 1) + 2 * ((lane >> 1) & 1) + ((lane >> 2) & 1);
    if ((q >> 1) < r) reinterpret_cast<double*>(&sh[wv][0])[q] = ws;
  }
  __syncthreads();
  if (threadIdx.x < r) {
    double2 sres = make_double2(0.0, 0.0);
    for (int w = 0; w < 4; ++w) sres = cadd(sres, sh[w][threadIdx.x]);
    mom[(((int64_t)v * Ny + j) * S + part) * r + threadIdx.x] = mk<R>((R)sres.x, (R)sres.y);
  }
}

// m_a(j) of vector v from the S <= 8 partial sums (fixed order); the parts are
// loaded together, then added in part order.
template <class R>
__device__ __forceinline__ cv<R> mom_at(const cv<R>* __restrict__ mom, int64_t v, int Ny, int j, int a, int r,
                                        int S) {
  const cv<R>* p = mom + ((v * Ny + j) * S) * r + a;
  cv<R> part[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) part[q] = (q < S) ? p[(int64_t)q * r] : mk<R>(0, 0);
  cv<R> s = part[0];
#pragma unroll
  for (int q = 1; q < 8; ++q)
    if (q < S) s = cadd(s, part[q]);
  return s;
}

// y = (A - tau B) x, matrix-free.  The streaming term is a real GEMM
// Y[j, c] = sum_m D_x[j, m] X[m, c] over the 2 Nxi complex columns c = (f, k);
// a workgroup stages an Ny x TC column tile of X in LDS once and computes the
// rows [row0, row1) of the tile.  Epilogue per entry: xi_x scaling, diagonal
// (nu_j + i beta xi_y - tau), rank-r moment update, identity inflow rows.
// grid (col tiles, row groups, nvec), block 256, dynamic LDS Ny * TC * 16 B.
template <class R, int RB>
__global__ void __launch_bounds__(256) k_apply(const cv<R>* __restrict__ x, cv<R>* __restrict__ y,
                                               int64_t n, int Ny, int Nxi, int r, R tau_re,
                                               R tau_im, R beta,
                                               const R* __restrict__ DxT,
                                               const R* __restrict__ xi_x,
                                               const R* __restrict__ xi_y,
                                               const R* __restrict__ nu,
                                               const R* __restrict__ U,
                                               const cv<R>* __restrict__ mom, int S,
                                               const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int nc = 2 * Nxi;
  const int c = blockIdx.x * 256 + threadIdx.x;
  const int j0 = blockIdx.y * RB;
  const int v = blockIdx.z;
  if (c >= nc) return;
  const cv<R>* xv = x + (int64_t)v * n;
  cv<R>* yv = y + (int64_t)v * n;
  // streaming: acc[rr] = sum_m D_x[j0 + rr, m] X[m, c]; the D_x column slice is
  // wave-uniform (scalar loads from the transposed table), X is read once per
  // row group and reused for all RB rows from registers
  R ar[RB], ai[RB];
#pragma unroll
  for (int rr = 0; rr < RB; ++rr) { ar[rr] = 0; ai[rr] = 0; }
  const int jn = min(RB, Ny - j0);
  int m = 0;
  for (; m + 4 <= Ny; m += 4) {
    cv<R> xm[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) xm[u] = xv[(int64_t)(m + u) * nc + c];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const R* dcol = DxT + (int64_t)(m + u) * Ny + j0;
#pragma unroll
      for (int rr = 0; rr < RB; ++rr) {
        const R d = (rr < jn) ? dcol[rr] : (R)0;
        ar[rr] = fma(d, xm[u].x, ar[rr]);
        ai[rr] = fma(d, xm[u].y, ai[rr]);
      }
    }
  }
  for (; m < Ny; ++m) {
    const cv<R> xm = xv[(int64_t)m * nc + c];
    const R* dcol = DxT + (int64_t)m * Ny + j0;
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) {
      const R d = (rr < jn) ? dcol[rr] : (R)0;
      ar[rr] = fma(d, xm.x, ar[rr]);
      ai[rr] = fma(d, xm.y, ai[rr]);
    }
  }
  // epilogue: xi_x scaling, diagonal, rank-r moment update, identity inflow rows
  const int f = c / Nxi, k = c - f * Nxi;
  const R xik = xi_x[k], bxy = beta * xi_y[k];
#pragma unroll
  for (int rr = 0; rr < RB; ++rr) {
    const int j = j0 + rr;
    if (j >= Ny) break;
    const cv<R> xjc = xv[(int64_t)j * nc + c];
    const bool bc = (j == Ny - 1 && xik > 0) || (j == 0 && xik < 0);
    cv<R> out;
    if (bc) {
      out = xjc;
    } else {
      const R dre = nu[j] - tau_re, dim = bxy - tau_im;
      out.x = xik * ar[rr] + dre * xjc.x - dim * xjc.y;
      out.y = xik * ai[rr] + dre * xjc.y + dim * xjc.x;
      const R* Uj = U + ((int64_t)(j * 2 + f) * r) * Nxi + k;
      for (int a = 0; a < r; ++a) {
        const R ua = Uj[(int64_t)a * Nxi];
        const cv<R> ma = mom_at<R>(mom, v, Ny, j, a, r, S);
        out.x -= ua * ma.x;
        out.y -= ua * ma.y;
      }
    }
    yv[(int64_t)j * nc + c] = out;
  }
}

// y = (A - tau B) x with the streaming GEMM on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64).  One wavefront per tile of 16 complex columns x RT*16
// rows; the real and imaginary parts of X are two B operands sharing the D_x
// fragment.  Operand layouts (gfx950): A[i][k] in lane i + 16k, B[k][j] in lane
// j + 16k, D[i][j] for lane l, register q at i = l/16 + 4q, j = l%16.
// 1-D grid of gx gy nvec workgroups, gx = ceil(ceil(2 Nxi / 16) / NW), gy =
// ceil(ceil(Ny / 16) / RT), block 64 NW.
typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));
// One matrix-core step acc += A B of a 16 x 16 x 4 tile in precision R, and the
// tile row that register q of lane group lk (lane / 16) holds: rows lk + 4 q for
// v_mfma_f64_16x16x4f64, rows 4 lk + q for v_mfma_f32_16x16x4f32.
template <class R> struct mfma_acc { typedef dbl4 type; };
template <> struct mfma_acc<float> { typedef flt4 type; };
__device__ __forceinline__ dbl4 mfma4(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ flt4 mfma4(float a, float b, flt4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <class R>
__device__ __forceinline__ int acc_row(int lk, int q) {
  return sizeof(R) == 8 ? lk + 4 * q : 4 * lk + q;
}
// NW wavefronts per workgroup, each a column tile of 16; with NW > 1 the D_x^T
// row slice of the workgroup is staged once in LDS and shared.  The moments of
// the workgroup's rows are summed from their S parts once into LDS.
template <int RT, int NW>
__global__ void __launch_bounds__(64 * NW) k_apply_mfma(const double2* __restrict__ x,
                                                        double2* __restrict__ y, int64_t n, int Ny,
                                                        int Nxi, int r, double tau_re, double tau_im,
                                                        double beta, const double* __restrict__ DxT,
                                                        const double* __restrict__ xi_x,
                                                        const double* __restrict__ xi_y,
                                                        const double* __restrict__ nu,
                                                        const double* __restrict__ U,
                                                        const double2* __restrict__ mom, int S,
                                                        const int* __restrict__ skip, int gx, int gy,
                                                        int vmaj) {
  extern __shared__ unsigned char lds_raw[];
  double2* ms = reinterpret_cast<double2*>(lds_raw);                 // [RT*16][4] moments
  double* As = reinterpret_cast<double*>(lds_raw + RT * 16 * 4 * sizeof(double2));  // [Ny4][RT*16]
  const int sk = skip ? *skip : 0;
  const int nc = 2 * Nxi;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nrt = (Ny + 15) / 16;
  // A 1-D grid spread over the XCDs by xcd_item.  vmaj > 0: gx gy vmaj
  // workgroups ordered tile major, vector minor (a column tile's U entries and
  // D_x rows are read from one L2 for all vectors).  vmaj == 0 (one vector):
  // gx gy workgroups ordered column tile major, row group minor (the row groups
  // of a column tile read its x strip from one L2).
  int bx, by, v;
  const int64_t item = xcd_item(blockIdx.x, gridDim.x);
  if (vmaj > 0) {
    v = (int)(item % vmaj);
    const int q = (int)(item / vmaj);
    bx = q % gx;
    by = q / gx;
  } else {
    v = 0;
    by = (int)(item % gy);
    bx = (int)(item / gy);
  }
  const int rt0 = by * RT;
  const int W = RT * 16;
  const int c0 = (bx * NW + wv) * 16;
  const double2* xv = x + (int64_t)v * n;
  double2* yv = y + (int64_t)v * n;
  const int li = lane & 15, lk = lane >> 4;
  const int cb = c0 + li;
  // Loads that need neither the moments nor the D_x slice are issued first, so
  // they are in flight while those are staged: with one row tile (the
  // single-vector launches) the epilogue's operands (x at the tile's rows, nu,
  // the U columns), and in every tiling the first block of the x strip.
  constexpr bool kPre = (RT == 1);
  double2 pre_x[4];
  double pre_nu[4], pre_u[4][4];
  if constexpr (kPre) {
    const bool cok = cb < nc;
    const int fp = cok ? cb / Nxi : 0, kp = cok ? cb - fp * Nxi : 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = rt0 * 16 + lk + 4 * q;
      const bool ok = cok && j < Ny;
      pre_x[q] = ok ? xv[(int64_t)j * nc + cb] : make_double2(0.0, 0.0);
      pre_nu[q] = ok ? nu[j] : 0.0;
#pragma unroll
      for (int a = 0; a < 4; ++a)
        pre_u[q][a] = (ok && a < r) ? U[((int64_t)(j * 2 + fp) * r + a) * Nxi + kp] : 0.0;
    }
  }
  // The K loop runs in blocks of XB steps of 4 rows, the next block's x strip
  // loading while the current block's MFMAs run (XB loads in flight per lane).
  // One-wavefront workgroups (small launches) take 8 steps per block; the wide
  // path, already at 2 waves per SIMD from its LDS slice and accumulators,
  // takes 4 (measured at the M = 4 shape, 64 vectors: 374 us per launch against
  // 446 us with one step of prefetch and 581 us with 8).
  constexpr int XB = (NW == 1) ? 8 : 4;
  auto load_block = [&](int mb, double2* dst) {
#pragma unroll
    for (int p = 0; p < XB; ++p) {
      const int m = mb + 4 * p + lk;
      dst[p] = (m < Ny && cb < nc) ? xv[(int64_t)m * nc + cb] : make_double2(0.0, 0.0);
    }
  };
  double2 xc[XB], xn[XB];
  load_block(0, xc);
  if (sk) return;
  for (int idx = threadIdx.x; idx < W * r; idx += 64 * NW) {
    const int jl = idx / r, a = idx - jl * r;
    const int j = rt0 * 16 + jl;
    ms[jl * 4 + a] = (j < Ny) ? mom_at<double>(mom, v, Ny, j, a, r, S) : make_double2(0.0, 0.0);
  }
  if (NW > 1) {
    const int Ny4 = (Ny + 3) & ~3;
    for (int idx = threadIdx.x; idx < Ny4 * W; idx += 64 * NW) {
      const int m = idx / W, rl = idx - m * W;
      const int row = rt0 * 16 + rl;
      As[idx] = (m < Ny && row < Ny) ? DxT[(int64_t)m * Ny + row] : 0.0;
    }
  }
  __syncthreads();
  if (c0 >= nc) return;
  dbl4 are[RT], aim[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t) { are[t] = dbl4{0, 0, 0, 0}; aim[t] = dbl4{0, 0, 0, 0}; }
  for (int mb = 0; mb < Ny; mb += 4 * XB) {
    if (mb + 4 * XB < Ny) load_block(mb + 4 * XB, xn);
#pragma unroll
    for (int p = 0; p < XB; ++p) {
      const int m = mb + 4 * p + lk;
      if (mb + 4 * p >= Ny) break;
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        double a;
        if (NW > 1) {
          a = As[m * W + t * 16 + li];
        } else {
          const int row = (rt0 + t) * 16 + li;
          a = (row < Ny && m < Ny) ? DxT[(int64_t)m * Ny + row] : 0.0;
        }
        are[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, xc[p].x, are[t], 0, 0, 0);
        aim[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, xc[p].y, aim[t], 0, 0, 0);
      }
    }
#pragma unroll
    for (int p = 0; p < XB; ++p) xc[p] = xn[p];
  }
  // epilogue on the accumulator layout: column c, rows j = tile*16 + lk + 4q
  const int c = c0 + li;
  if (c >= nc) return;
  const int f = c / Nxi, k = c - f * Nxi;
  const double xik = xi_x[k], bxy = beta * xi_y[k];
#pragma unroll
  for (int t = 0; t < RT; ++t) {
    if (rt0 + t >= nrt) break;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int jl = t * 16 + lk + 4 * q;
      const int j = rt0 * 16 + jl;
      if (j >= Ny) continue;
      const double2 xjc = kPre ? pre_x[q] : xv[(int64_t)j * nc + c];
      const bool bc = (j == Ny - 1 && xik > 0.0) || (j == 0 && xik < 0.0);
      double2 out;
      if (bc) {
        out = xjc;
      } else {
        const double dre = (kPre ? pre_nu[q] : nu[j]) - tau_re, dim = bxy - tau_im;
        out = op_out(xik, are[t][q], aim[t][q], dre, dim, xjc);
        if constexpr (kPre) {
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            if (a < r) {
              const double2 ma = ms[jl * 4 + a];
              op_moment(out, pre_u[q][a], ma);
            }
          }
        } else {
          // (a rolled loop keeps the wide path at 2 waves per SIMD)
          const double* Uj = U + ((int64_t)(j * 2 + f) * r) * Nxi + k;
          for (int a = 0; a < r; ++a) {
            const double ua = Uj[(int64_t)a * Nxi];
            const double2 ma = ms[jl * 4 + a];
            op_moment(out, ua, ma);
          }
        }
      }
      yv[(int64_t)j * nc + c] = out;
    }
  }
}

// FP32 operator for the mixed-precision inner solve: y = (A - tau B) x with the
// streaming GEMM on the FP32 matrix cores (v_mfma_f32_16x16x4f32).  One
// wavefront per tile of 16 complex columns x RT 16 rows, NW wavefronts per
// workgroup sharing an LDS copy of their D_x row slice (NW > 1); the real and
// imaginary parts of X are two B operands sharing the D_x fragment.  Operand
// layouts (gfx950): A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k; the
// result D[i][j] sits in lane j + 16 (i / 4), register i % 4 (rows held four
// to a lane, unlike the FP64 instruction).  Accumulation in FP32; the
// epilogue's moments are the FP32 totals of the S column parts.
// 1-D grid of gx gy nvec workgroups, gx = ceil(ceil(2 Nxi / 16) / NW), gy =
// ceil(ceil(Ny / 16) / RT), block 64 NW.
template <int RT, int NW>
__global__ void __launch_bounds__(64 * NW) k_apply_mfma32(const float2* __restrict__ x, float2* __restrict__ y,
                                                          int64_t n, int Ny, int Nxi, int r, float tau_re,
                                                          float tau_im, float beta, const float* __restrict__ DxT,
                                                          const float* __restrict__ xi_x,
                                                          const float* __restrict__ xi_y,
                                                          const float* __restrict__ nu,
                                                          const float* __restrict__ U,
                                                          const float2* __restrict__ mom, int S,
                                                          const int* __restrict__ skip, int gx, int gy) {
  extern __shared__ unsigned char lds_raw[];
  float2* ms = reinterpret_cast<float2*>(lds_raw);                          // [RT*16][4] moments
  float* As = reinterpret_cast<float*>(lds_raw + RT * 16 * 4 * sizeof(float2));  // [Ny4][RT*16]
  if (skip && *skip) return;
  const int nc = 2 * Nxi;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // 1-D grid over the XCDs, ordered column tile, vector, row group (fastest):
  // the row groups of a column tile read its x strip from one L2, and the
  // vectors of a column tile its U columns
  const int64_t item = xcd_item(blockIdx.x, gridDim.x);
  const int nv = (int)(gridDim.x / ((int64_t)gx * gy));
  const int by = (int)(item % gy);
  const int64_t rest = item / gy;
  const int v = (int)(rest % nv);
  const int bx = (int)(rest / nv);
  const int rt0 = by * RT;
  const int W = RT * 16;
  for (int idx = threadIdx.x; idx < W * r; idx += 64 * NW) {
    const int jl = idx / r, a = idx - jl * r;
    const int j = rt0 * 16 + jl;
    ms[jl * 4 + a] = (j < Ny) ? mom_at<float>(mom, v, Ny, j, a, r, S) : make_float2(0.f, 0.f);
  }
  if (NW > 1) {
    const int Ny4 = (Ny + 3) & ~3;
    for (int idx = threadIdx.x; idx < Ny4 * W; idx += 64 * NW) {
      const int m = idx / W, rl = idx - m * W;
      const int row = rt0 * 16 + rl;
      As[idx] = (m < Ny && row < Ny) ? DxT[(int64_t)m * Ny + row] : 0.f;
    }
  }
  __syncthreads();
  const int c0 = (bx * NW + wv) * 16;
  if (c0 >= nc) return;
  const float2* xv = x + (int64_t)v * n;
  float2* yv = y + (int64_t)v * n;
  const int li = lane & 15, lk = lane >> 4;
  const int cb = c0 + li;
  flt4 are[RT], aim[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t) { are[t] = flt4{0, 0, 0, 0}; aim[t] = flt4{0, 0, 0, 0}; }
  // K loop in blocks of XB steps of 4 rows; the next block's x strip loads
  // while the current block's MFMAs run
  {
    constexpr int XB = 8;
    auto load_block = [&](int mb, float2* dst) {
#pragma unroll
      for (int p = 0; p < XB; ++p) {
        const int m = mb + 4 * p + lk;
        dst[p] = (m < Ny && cb < nc) ? xv[(int64_t)m * nc + cb] : make_float2(0.f, 0.f);
      }
    };
    float2 xc[XB], xn[XB];
    load_block(0, xc);
    for (int mb = 0; mb < Ny; mb += 4 * XB) {
      if (mb + 4 * XB < Ny) load_block(mb + 4 * XB, xn);
#pragma unroll
      for (int p = 0; p < XB; ++p) {
        const int m = mb + 4 * p + lk;
        if (mb + 4 * p >= Ny) break;
#pragma unroll
        for (int t = 0; t < RT; ++t) {
          float a;
          if (NW > 1) {
            a = As[m * W + t * 16 + li];
          } else {
            const int row = (rt0 + t) * 16 + li;
            a = (row < Ny && m < Ny) ? DxT[(int64_t)m * Ny + row] : 0.f;
          }
          are[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, xc[p].x, are[t], 0, 0, 0);
          aim[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, xc[p].y, aim[t], 0, 0, 0);
        }
      }
#pragma unroll
      for (int p = 0; p < XB; ++p) xc[p] = xn[p];
    }
  }
  // epilogue on the accumulator layout: column c, rows j = tile 16 + 4 lk + q
  const int c = cb;
  if (c >= nc) return;
  const int f = c / Nxi, k = c - f * Nxi;
  const float xik = xi_x[k], bxy = beta * xi_y[k];
#pragma unroll
  for (int t = 0; t < RT; ++t) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int jl = t * 16 + 4 * lk + q;
      const int j = rt0 * 16 + jl;
      if (j >= Ny) continue;
      const float2 xjc = xv[(int64_t)j * nc + c];
      const bool bc = (j == Ny - 1 && xik > 0.f) || (j == 0 && xik < 0.f);
      float2 out;
      if (bc) {
        out = xjc;
      } else {
        const float dre = nu[j] - tau_re, dim = bxy - tau_im;
        out.x = fmaf(xik, are[t][q], fmaf(dre, xjc.x, -(dim * xjc.y)));
        out.y = fmaf(xik, aim[t][q], fmaf(dre, xjc.y, dim * xjc.x));
        const float* Uj = U + ((int64_t)(j * 2 + f) * r) * Nxi + k;
        for (int a = 0; a < r; ++a) {
          const float ua = Uj[(int64_t)a * Nxi];
          const float2 ma = ms[jl * 4 + a];
          out.x = fmaf(-ua, ma.x, out.x);
          out.y = fmaf(-ua, ma.y, out.y);
        }
      }
      yv[(int64_t)j * nc + c] = out;
    }
  }
}

// Load / store at a uniform base plus a 32-bit byte offset (the global_load
// form with a scalar base and a 32-bit vector offset).
template <class T>
__device__ __forceinline__ T ld_off(const T* __restrict__ base, uint32_t byte_off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const unsigned char*>(base) + byte_off);
}
template <class T>
__device__ __forceinline__ void st_off(T* base, uint32_t byte_off, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<unsigned char*>(base) + byte_off) = v;
}

// Totals of the S moment parts of nvec vectors, in the order of mom_at:
// tot[(v Ny + j) r + a].  One thread per entry.
template <class R>
__global__ void __launch_bounds__(256) k_mom_total(const cv<R>* __restrict__ mom, cv<R>* __restrict__ tot,
                                                   int64_t count, int r, int S) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= count) return;
  const int64_t vj = e / r, a = e - vj * r;
  const cv<R>* p = mom + vj * S * r + a;
  cv<R> part[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) part[q] = (q < S) ? p[(int64_t)q * r] : mk<R>(0, 0);
  cv<R> s = part[0];
#pragma unroll
  for (int q = 1; q < 8; ++q)
    if (q < S) s = cadd(s, part[q]);
  tot[e] = s;
}

// Many-vector operator as a stream of work items, y_v = (A - tau B) x_v.  An
// item is (group of WPG 16-column tiles, vector v); wavefront w computes the
// whole output strip (all N_y rows) of column tile WPG g + w for vector v.
// * The D_x fragments of every row tile (the A operands of
//   v_mfma_f64_16x16x4f64, or of v_mfma_f32_16x16x4f32 for R = float, the
//   mixed solve's operator) sit in LDS in lane order, so each K step reads them
//   conflict-free with one load per lane and row tile.
// * The x strip streams from memory into registers in chunks of XB K steps;
//   the next chunk, of this item or of the next, loads while the current
//   chunk's MFMAs run.  The one barrier per item orders only LDS (an LDS-only
//   fence), so these loads stay in flight across it.
// * The item's moments (totals over the column parts, summed in fixed order by
//   k_mom_total) are staged in LDS, double buffered; the next item's load
//   during the current epilogue.
// * Loads and stores within one vector or table address it as a uniform base
//   plus a 32-bit byte offset (each vector and table is under 4 GiB, checked by
//   the launcher), which keeps the address arithmetic in few registers.
// Every output entry is accumulated as in k_apply_mfma (K in steps of 4 from 0,
// then op_out and op_moment), so the results are bit-identical to it (to
// k_apply_mfma32 for R = float).
// Workgroup b takes a contiguous range of items, ordered column group major and
// vector minor, at its XCD-ordered index, so the U entries and tables of a
// column group are reused from one L2.  A wavefront whose tile lies past the
// last column (in the last group) only relays the next item's first chunk.
// grid ceil(items / per), block 64 WPG; items = ceil(ceil(2 Nxi / 16) / WPG) nvec.
template <class R, int NRT, int WPG, int RR>
__global__ void __launch_bounds__(64 * WPG) k_apply_stream(const cv<R>* __restrict__ x,
                                                          cv<R>* __restrict__ y, int64_t n, int Ny,
                                                          int Nxi, R tau_re, R tau_im,
                                                          R beta, const R* __restrict__ DxT,
                                                          const R* __restrict__ xi_x,
                                                          const R* __restrict__ xi_y,
                                                          const R* __restrict__ nu,
                                                          const R* __restrict__ U,
                                                          const cv<R>* __restrict__ mtot, int nvec,
                                                          int64_t nitems, int per) {
  typedef typename mfma_acc<R>::type acc4;
  constexpr uint32_t XS = sizeof(cv<R>), RS = sizeof(R);   // bytes per entry
  constexpr int K4 = 4 * NRT;             // K steps of 4 rows, N_y <= 16 NRT
  constexpr int XB = 4;                   // K steps per chunk: one row tile of x
  static_assert(XB * 4 == 16, "a chunk of x rows is one row tile");
  constexpr int NMOM = NRT * 16 * 4;      // moments of one vector: rows x 4
  __shared__ R afs[K4 * NRT * 64];        // [step][row tile][lane]
  __shared__ cv<R> ms[2][NMOM];          // [buffer][row * 4 + a]
  // The x entries of the first KEEP row tiles, as the chunk loop loads them
  // (chunk t is row tile t), kept per wavefront for the epilogue in the LDS that
  // the one workgroup per CU leaves free: [tile][wavefront][K step][lane]
  constexpr int LDS_WG = 160 * 1024;
  constexpr int USED = K4 * NRT * 64 * (int)sizeof(R) + 2 * NMOM * (int)sizeof(cv<R>);
  constexpr int PER_TILE = WPG * XB * 64 * (int)sizeof(cv<R>);
  constexpr int KEEP = ((LDS_WG - USED) / PER_TILE < NRT) ? (LDS_WG - USED) / PER_TILE : NRT;
  __shared__ cv<R> xk[(KEEP > 0 ? KEEP : 1) * WPG * XB * 64];
  const int nc = 2 * Nxi;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t i0 = xcd_item(blockIdx.x, gridDim.x) * per;
  const int64_t i1 = min(nitems, i0 + per);
  if (i0 >= i1) return;                   // uniform over the workgroup
  // fragment (s, t, l) = D_x[t 16 + l % 16][4 s + l / 16] = DxT[(4 s + l / 16) Ny + t 16 + l % 16]
  for (int idx = threadIdx.x; idx < K4 * NRT * 64; idx += 64 * WPG) {
    const int l = idx & 63, st = idx >> 6;
    const int t = st % NRT, s = st / NRT;
    const int m = 4 * s + (l >> 4), row = t * 16 + (l & 15);
    afs[idx] = (m < Ny && row < Ny) ? DxT[(int64_t)m * Ny + row] : (R)0;
  }
  const int nsteps = (Ny + 3) >> 2;
  const int nch = (nsteps + XB - 1) / XB;
  const bool mthr = threadIdx.x < NMOM;
  const int mj = threadIdx.x >> 2, ma = threadIdx.x & 3;
  // moment entry (mj, ma) of vector v
  auto mom_load = [&](int v) {
    return (mthr && mj < Ny && ma < RR) ? mtot[((int64_t)v * Ny + mj) * RR + ma] : mk<R>(0, 0);
  };
  auto load_chunk = [&](int v, int c, int ch, cv<R>* dst) {
    const cv<R>* xv = x + (int64_t)v * n;
#pragma unroll
    for (int p = 0; p < XB; ++p) {
      const int m = 4 * (ch * XB + p) + lk;
      dst[p] = (m < Ny && c < nc) ? ld_off(xv, (uint32_t)(m * nc + c) * XS) : mk<R>(0, 0);
    }
  };
  int v = (int)(i0 % nvec), g = (int)(i0 / nvec);
  if (mthr) ms[0][threadIdx.x] = mom_load(v);
  cv<R> xa[XB], xb[XB];
  load_chunk(v, (g * WPG + w) * 16 + li, 0, xa);
  __syncthreads();
  int buf = 0;
  for (int64_t it = i0; it < i1; ++it, buf ^= 1) {
    const int c = (g * WPG + w) * 16 + li;
    const bool more = it + 1 < i1;
    const int vn = (v + 1 == nvec) ? 0 : v + 1, gn = (v + 1 == nvec) ? g + 1 : g;
    const int cn = (gn * WPG + w) * 16 + li;
    acc4 are[NRT], aim[NRT];
#pragma unroll
    for (int t = 0; t < NRT; ++t) { are[t] = acc4{0, 0, 0, 0}; aim[t] = acc4{0, 0, 0, 0}; }
    if ((g * WPG + w) * 16 < nc) {
      for (int ch = 0; ch < nch; ++ch) {
        if (ch + 1 < nch) load_chunk(v, c, ch + 1, xb);
        else if (more) load_chunk(vn, cn, 0, xb);
        if (ch < KEEP) {
#pragma unroll
          for (int p = 0; p < XB; ++p) xk[((ch * WPG + w) * XB + p) * 64 + lane] = xa[p];
        }
#pragma unroll
        for (int p = 0; p < XB; ++p) {
          const int s = ch * XB + p;
          if (s < nsteps) {
#pragma unroll
            for (int t = 0; t < NRT; ++t) {
              const R a = afs[(s * NRT + t) * 64 + lane];
              are[t] = mfma4(a, xa[p].x, are[t]);
              aim[t] = mfma4(a, xa[p].y, aim[t]);
            }
          }
        }
#pragma unroll
        for (int p = 0; p < XB; ++p) xa[p] = xb[p];
      }
    } else if (more) {
      load_chunk(vn, cn, 0, xa);
    }
    // the next item's moments load during the epilogue
    const cv<R> mnext = more ? mom_load(vn) : mk<R>(0, 0);
    // epilogue on the accumulator layout: column c, rows j = t 16 + lk + 4 q.
    // The row index is made opaque per item so the compiler keeps no
    // per-row masks or offsets live across items; loads take clamped rows and
    // only the stores are guarded.
    int lko = lk;
    asm volatile("" : "+v"(lko));
    // the kept entries were written by other lanes of this wavefront (FP32 layout)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
    if (c < nc) {
      const int f = c / Nxi, k = c - f * Nxi;
      const R xik = xi_x[k], bxy = beta * xi_y[k];
      const cv<R>* xv = x + (int64_t)v * n;
      cv<R>* yv = y + (int64_t)v * n;
      const cv<R>* mb = ms[buf];
#pragma unroll
      for (int t = 0; t < NRT; ++t) {
        if (t * 16 < Ny) {
          cv<R> xq[4];
          R nq[4], uq[4][RR];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int rho = acc_row<R>(lko, q), jc = min(t * 16 + rho, Ny - 1);
            // row 16 t + rho was the B operand of K step 4 t + rho / 4 in lane
            // li + 16 (rho % 4)
            if (t < KEEP)
              xq[q] = xk[((t * WPG + w) * XB + (rho >> 2)) * 64 + li + 16 * (rho & 3)];
            else
              xq[q] = ld_off(xv, (uint32_t)(jc * nc + c) * XS);
            nq[q] = nu[jc];
#pragma unroll
            for (int a = 0; a < RR; ++a)
              uq[q][a] = ld_off(U + (int64_t)a * Nxi, (uint32_t)((jc * 2 + f) * RR * Nxi + k) * RS);
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int j = t * 16 + acc_row<R>(lko, q);
            if (j < Ny) {
              const cv<R> xjc = xq[q];
              const bool bc = (j == Ny - 1 && xik > (R)0) || (j == 0 && xik < (R)0);
              cv<R> out;
              if (bc) {
                out = xjc;
              } else {
                const R dre = nq[q] - tau_re, dim = bxy - tau_im;
                out = op_out(xik, are[t][q], aim[t][q], dre, dim, xjc);
#pragma unroll
                for (int a = 0; a < RR; ++a) op_moment(out, uq[q][a], mb[j * 4 + a]);
              }
              st_off(yv, (uint32_t)(j * nc + c) * XS, out);
            }
          }
        }
        // one row tile's epilogue loads in flight at a time (keeps the
        // accumulators, the prefetched chunk and these loads in registers)
        asm volatile("" ::: "memory");
      }
    }
    if (more && mthr) ms[buf ^ 1][threadIdx.x] = mnext;
    // LDS-only barrier: the next item's first x chunk stays in flight
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    v = vn;
    g = gn;
  }
}

// Moment partials of a group of vectors per workgroup (node j, column part):
// each thread holds the M entries of its columns (the columns k_moments gives
// it) in registers and sums every vector of the group in the order of
// k_moments, so the partials are bit-identical to it (the eight wavefront sums
// of a vector together, by wave_sum8).  The next two vectors' x entries load
// while the current one is reduced; the per-vector exchange of wavefront sums
// is double buffered with one LDS-only barrier, so those loads stay in flight
// across it.  grid (Ny S, vector groups), block 256; CPT =
// columns per thread (the part has <= 256 CPT).  R: FP64, or FP32 for the
// mixed solve's tables (sums in R per thread, wavefront sums in FP64, as in
// k_moments).
template <class R, int CPT>
__global__ void __launch_bounds__(256) k_moments_batch(const cv<R>* __restrict__ x, int64_t n, int Ny, int Nxi,
                                                       int r, const R* __restrict__ M,
                                                       cv<R>* __restrict__ mom, int S, int nvec, int VG) {
  __shared__ double2 sh[2][4][4];
  const int j = blockIdx.x / S, part = blockIdx.x - j * S;
  const int v0 = blockIdx.y * VG, v1 = min(nvec, v0 + VG);
  const int nc = 2 * Nxi;
  const int per = (nc + S - 1) / S;
  const int cbeg = part * per, cend = min(nc, cbeg + per);
  R mw[CPT][4];
#pragma unroll
  for (int i = 0; i < CPT; ++i) {
    const int cc = cbeg + threadIdx.x + 256 * i;
#pragma unroll
    for (int a = 0; a < 4; ++a) mw[i][a] = (cc < cend && a < r) ? M[((int64_t)j * r + a) * nc + cc] : (R)0;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  auto load = [&](int v, cv<R>* xr) {
    const cv<R>* xj = x + (int64_t)v * n + (int64_t)j * nc;
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      const int cc = cbeg + threadIdx.x + 256 * i;
      xr[i] = (cc < cend) ? xj[cc] : mk<R>(0, 0);
    }
  };
  cv<R> xc[CPT], xn[CPT], xn2[CPT];
  if (v0 < v1) load(v0, xc);
  if (v0 + 1 < v1) load(v0 + 1, xn);
  for (int v = v0; v < v1; ++v) {
    const int buf = (v - v0) & 1;
    if (v + 2 < v1) load(v + 2, xn2);
    R ar[4] = {0, 0, 0, 0}, ai[4] = {0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      const int cc = cbeg + threadIdx.x + 256 * i;
      if (cc < cend) {
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          if (a < r) {
            ar[a] += mw[i][a] * xc[i].x;
            ai[a] += mw[i][a] * xc[i].y;
          }
        }
      }
    }
    // the wavefront sums of (re, im) of every moment at once; lane l < 8 holds
    // entry q(l) of sh[buf][wv] read as 8 doubles
    double pv[8];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      pv[2 * a] = (a < r) ? (double)ar[a] : 0.0;
      pv[2 * a + 1] = (a < r) ? (double)ai[a] : 0.0;
    }
    const double ws = wave_sum8(pv);
    if (lane < 8) {
      const int q = 4 * (lane & 1) + 2 * ((lane >> 1) & 1) + ((lane >> 2) & 1);
      if ((q >> 1) < r) reinterpret_cast<double*>(&sh[buf][wv][0])[q] = ws;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    if (threadIdx.x < r) {
      double2 sres = make_double2(0.0, 0.0);
      for (int w = 0; w < 4; ++w) sres = cadd(sres, sh[buf][w][threadIdx.x]);
      mom[(((int64_t)v * Ny + j) * S + part) * r + threadIdx.x] = mk<R>((R)sres.x, (R)sres.y);
    }
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      xc[i] = xn[i];
      xn[i] = xn2[i];
    }
  }
}

// ----------------------------------------------------------------- CSR -----

// Row pointer of the explicit matrix: uniform length Ny - 1 + 2 Nxi for
// non-inflow rows, 1 for inflow rows.  One thread per row writes rowptr[i+1];
// the prefix is closed-form because row lengths are known: rows before i in
// node order j' < j contribute per-node counts.
__global__ void k_csr_rowptr(int64_t* __restrict__ rowptr, int Ny, int Nxi,
                             const double* __restrict__ xi_x, int npos_x, int nneg_x) {
  const int64_t n = 2LL * Ny * Nxi;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t L = Ny - 1 + 2LL * Nxi;
  const int nc = 2 * Nxi;
  const int j = (int)(i / nc);
  const int c = (int)(i - (int64_t)j * nc);
  const int k = c % Nxi, f = c / Nxi;
  // inflow rows strictly before row i
  int64_t nbc_before = 0;
  if (j > 0) nbc_before += 2LL * nneg_x;                 // node 0, both fields
  if (j == Ny - 1 && j > 0) {
    // node Ny-1: inflow rows are xi_x > 0; count those before column c
    int cnt = 0;
    for (int cc = 0; cc < c; ++cc) cnt += (xi_x[cc % Nxi] > 0.0) ? 1 : 0;
    nbc_before += cnt;
  } else if (j == 0) {
    int cnt = 0;
    for (int cc = 0; cc < c; ++cc) cnt += (xi_x[cc % Nxi] < 0.0) ? 1 : 0;
    nbc_before = cnt;
  }
  (void)f;
  const bool bc = (j == Ny - 1 && xi_x[k] > 0.0) || (j == 0 && xi_x[k] < 0.0);
  const int64_t before = i - nbc_before;   // non-inflow rows before i
  const int64_t start = before * L + nbc_before;
  rowptr[i + 1] = start + (bc ? 1 : L);
  if (i == 0) rowptr[0] = 0;
  (void)npos_x;
}

// Values and columns of the explicit matrix, one wavefront per row; columns in
// ascending order: (m, f, k) for m < j, the 2 Nxi entries of node j, (m, f, k)
// for m > j.
__global__ void __launch_bounds__(256) k_csr_fill(const int64_t* __restrict__ rowptr,
                                                  int32_t* __restrict__ col, double2* __restrict__ val,
                                                  int Ny, int Nxi, int r, double beta,
                                                  const double* __restrict__ Dx,
                                                  const double* __restrict__ xi_x,
                                                  const double* __restrict__ xi_y,
                                                  const double* __restrict__ nu,
                                                  const double* __restrict__ U,
                                                  const double* __restrict__ M) {
  const int64_t n = 2LL * Ny * Nxi;
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  const int nc = 2 * Nxi;
  const int j = (int)(i / nc);
  const int c = (int)(i - (int64_t)j * nc);
  const int f = c / Nxi, k = c - f * Nxi;
  const int64_t s = rowptr[i];
  const bool bc = (j == Ny - 1 && xi_x[k] > 0.0) || (j == 0 && xi_x[k] < 0.0);
  if (bc) {
    if (lane == 0) { col[s] = (int32_t)i; val[s] = make_double2(1.0, 0.0); }
    return;
  }
  const int L = Ny - 1 + nc;
  const double xik = xi_x[k];
  for (int e = lane; e < L; e += 64) {
    int32_t cidx;
    double2 v;
    if (e < j) {                                 // streaming, m = e < j
      cidx = (int32_t)((2LL * e + f) * Nxi + k);
      v = make_double2(xik * Dx[(int64_t)j * Ny + e], 0.0);
    } else if (e < j + nc) {                     // node block
      const int cb = e - j;
      const int fb = cb / Nxi, kb = cb - fb * Nxi;
      cidx = (int32_t)((int64_t)j * nc + cb);
      double cp = 0.0;
      for (int a = 0; a < r; ++a)
        cp += U[(((int64_t)j * 2 + f) * r + a) * Nxi + k] * M[(((int64_t)j * r + a) * 2 + fb) * Nxi + kb];
      v = make_double2(-cp, 0.0);
      if (cb == c) { v.x += xik * Dx[(int64_t)j * Ny + j] + nu[j]; v.y += beta * xi_y[k]; }
    } else {                                     // streaming, m > j
      const int m = e - nc + 1;
      cidx = (int32_t)((2LL * m + f) * Nxi + k);
      v = make_double2(xik * Dx[(int64_t)j * Ny + m], 0.0);
    }
    col[s + e] = cidx;
    val[s + e] = v;
  }
}

// y = A x - tau B x with the CSR matrix, one wavefront per row.
__global__ void __launch_bounds__(256) k_csr_spmv(const int64_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ col,
                                                  const double2* __restrict__ val,
                                                  const double2* __restrict__ x, double2* __restrict__ y,
                                                  int64_t n, int Ny, int Nxi,
                                                  const double* __restrict__ xi_x, double tau_re,
                                                  double tau_im, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  const int64_t s = rowptr[i], e = rowptr[i + 1];
  double sr = 0.0, si = 0.0;
  for (int64_t p = s + lane; p < e; p += 64) {
    const double2 a = val[p];
    const double2 b = x[col[p]];
    sr = fma(a.x, b.x, sr); sr = fma(-a.y, b.y, sr);
    si = fma(a.x, b.y, si); si = fma(a.y, b.x, si);
  }
  sr = wave_sum(sr);
  si = wave_sum(si);
  if (lane == 0) {
    const int nc = 2 * Nxi;
    const int j = (int)(i / nc);
    const int k = (int)(i - (int64_t)j * nc) % Nxi;
    const bool bc = (j == Ny - 1 && xi_x[k] > 0.0) || (j == 0 && xi_x[k] < 0.0);
    if (!bc) {
      const double2 xi = x[i];
      sr -= tau_re * xi.x - tau_im * xi.y;
      si -= tau_re * xi.y + tau_im * xi.x;
    }
    y[i] = make_double2(sr, si);
  }
}

// ------------------------------------------------- block-Jacobi ILU(0) -----

// y = (L U)^{-1} x for every block of `nl` whole velocity lines.  One workgroup
// per block, one wavefront per line; lane q holds the rows j = q + 64 s of its
// line in registers.  Forward sweep: at step t, wavefront l finalises row
// j = t - l (the level set l + j = t of the lower factor), taking the coupling
// entries of earlier lines of the block at the same node from LDS, then updates
// its later rows with column j of L (right-looking).  Backward sweep mirrors it.
// The factor column and coupling entries of step t + 2 are loaded during step t,
// so the per-step critical path is the barrier and the shuffles, not memory.
// F is stored column-major per line (Fc[line][col][row]); C as in the host set-up.
template <int NPL>
__device__ __forceinline__ void load_col(double2 (&f)[NPL], const double2* __restrict__ col, int Ny,
                                         int lane) {
#pragma unroll
  for (int s = 0; s < NPL; ++s) {
    const int q = lane + 64 * s;
    f[s] = (q < Ny) ? col[q] : make_double2(0.0, 0.0);
  }
}

// Broadcast lane `src` (wave-uniform) of a double2 to the whole wavefront.
__device__ __forceinline__ double2 bcast(double2 v, int src) {
  double2 r;
  const unsigned lo_x = __builtin_amdgcn_readlane((unsigned)(__double_as_longlong(v.x) & 0xffffffffULL), src);
  const unsigned hi_x = __builtin_amdgcn_readlane((unsigned)((unsigned long long)__double_as_longlong(v.x) >> 32), src);
  const unsigned lo_y = __builtin_amdgcn_readlane((unsigned)(__double_as_longlong(v.y) & 0xffffffffULL), src);
  const unsigned hi_y = __builtin_amdgcn_readlane((unsigned)((unsigned long long)__double_as_longlong(v.y) >> 32), src);
  r.x = __longlong_as_double((long long)(((unsigned long long)hi_x << 32) | lo_x));
  r.y = __longlong_as_double((long long)(((unsigned long long)hi_y << 32) | lo_y));
  return r;
}

template <int NPL, int PD>
__global__ void __launch_bounds__(1024) k_ilu_apply(const double2* __restrict__ x,
                                                    double2* __restrict__ y, int Ny, int Nxi,
                                                    int nl, const double2* __restrict__ Fc,
                                                    const double2* __restrict__ C,
                                                    const int* __restrict__ skip) {
  extern __shared__ double2 ys[];   // [nl][Ny]
  if (skip && *skip) return;
  const int b = blockIdx.x;
  const int l = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nlines = 2 * Nxi;
  const int nl_blk = min(nl, nlines - b * nl);
  const bool active = l < nl_blk;
  const int lg = b * nl + l;
  const int f = active ? lg / Nxi : 0, k = active ? lg - f * Nxi : 0;
  const double2* Fl = Fc + (int64_t)(active ? lg : 0) * Ny * Ny;
  const double2* Cl = C + (((int64_t)b * nl + l) * nl) * Ny;   // Cl[l2 * Ny + j]
  double2 v[NPL];
#pragma unroll
  for (int s = 0; s < NPL; ++s) {
    const int j = lane + 64 * s;
    v[s] = (active && j < Ny) ? x[((int64_t)2 * j + f) * Nxi + k] : make_double2(0.0, 0.0);
  }
  const int steps = Ny + nl_blk - 1;
  // ring of the factor columns (and lane-l2 coupling entries) of the next PD steps
  double2 fr[PD][NPL], cr[PD];
  const bool cl = active && lane < nl_blk && lane != l;
  // ---- forward sweep, unit lower factor
  if (active) {
#pragma unroll
    for (int d = 0; d < PD; ++d) {
      if (d < Ny) {
        load_col<NPL>(fr[d], Fl + (int64_t)d * Ny, Ny, lane);
        cr[d] = cl ? Cl[(int64_t)lane * Ny + d] : make_double2(0.0, 0.0);
      }
    }
  }
  for (int t = 0; t < steps; ++t) {
    const int j = t - l;
    if (active && j >= 0 && j < Ny) {
      double2 f0[NPL];
#pragma unroll
      for (int s2 = 0; s2 < NPL; ++s2) f0[s2] = fr[0][s2];
      const double2 c0 = cr[0];
#pragma unroll
      for (int d = 0; d + 1 < PD; ++d) {
#pragma unroll
        for (int s2 = 0; s2 < NPL; ++s2) fr[d][s2] = fr[d + 1][s2];
        cr[d] = cr[d + 1];
      }
      if (j + PD < Ny) {
        load_col<NPL>(fr[PD - 1], Fl + (int64_t)(j + PD) * Ny, Ny, lane);
        cr[PD - 1] = cl ? Cl[(int64_t)lane * Ny + j + PD] : make_double2(0.0, 0.0);
      }
      // coupling with earlier lines of the block at node j (same value in every lane)
      double2 cpl = make_double2(0.0, 0.0);
      for (int l2 = 0; l2 < l; ++l2) cpl = cadd(cpl, cmul(bcast(c0, l2), ys[l2 * Ny + j]));
      const int owner = j & 63, slot = j >> 6;
      double2 mine = make_double2(0.0, 0.0);
#pragma unroll
      for (int s = 0; s < NPL; ++s)
        if (s == slot) mine = v[s];
      const double2 yj = csub(bcast(mine, owner), cpl);
      if (lane == owner && nl_blk > 1) ys[l * Ny + j] = yj;
#pragma unroll
      for (int s = 0; s < NPL; ++s) {
        const int q = lane + 64 * s;
        if (q == j) v[s] = yj;
        else if (q > j && q < Ny) v[s] = csub(v[s], cmul(f0[s], yj));
      }
    }
    if (nl_blk > 1) __syncthreads();
  }
  // ---- backward sweep, upper factor; its diagonal is stored as the reciprocal
  if (active) {
#pragma unroll
    for (int d = 0; d < PD; ++d) {
      if (Ny - 1 - d >= 0) {
        load_col<NPL>(fr[d], Fl + (int64_t)(Ny - 1 - d) * Ny, Ny, lane);
        cr[d] = cl ? Cl[(int64_t)lane * Ny + Ny - 1 - d] : make_double2(0.0, 0.0);
      }
    }
  }
  for (int t = 0; t < steps; ++t) {
    const int j = (Ny - 1) - (t - (nl_blk - 1 - l));
    if (active && j >= 0 && j < Ny) {
      double2 f0[NPL];
#pragma unroll
      for (int s2 = 0; s2 < NPL; ++s2) f0[s2] = fr[0][s2];
      const double2 c0 = cr[0];
#pragma unroll
      for (int d = 0; d + 1 < PD; ++d) {
#pragma unroll
        for (int s2 = 0; s2 < NPL; ++s2) fr[d][s2] = fr[d + 1][s2];
        cr[d] = cr[d + 1];
      }
      if (j - PD >= 0) {
        load_col<NPL>(fr[PD - 1], Fl + (int64_t)(j - PD) * Ny, Ny, lane);
        cr[PD - 1] = cl ? Cl[(int64_t)lane * Ny + j - PD] : make_double2(0.0, 0.0);
      }
      double2 cpl = make_double2(0.0, 0.0);
      for (int l2 = l + 1; l2 < nl_blk; ++l2) cpl = cadd(cpl, cmul(bcast(c0, l2), ys[l2 * Ny + j]));
      const int owner = j & 63, slot = j >> 6;
      double2 mine = make_double2(0.0, 0.0), dmine = make_double2(0.0, 0.0);
#pragma unroll
      for (int s = 0; s < NPL; ++s)
        if (s == slot) { mine = v[s]; dmine = f0[s]; }
      const double2 xj = cmul(csub(bcast(mine, owner), cpl), bcast(dmine, owner));
      if (lane == owner && nl_blk > 1) ys[l * Ny + j] = xj;
#pragma unroll
      for (int s = 0; s < NPL; ++s) {
        const int q = lane + 64 * s;
        if (q == j) v[s] = xj;
        else if (q < j) v[s] = csub(v[s], cmul(f0[s], xj));
      }
    }
    if (nl_blk > 1) __syncthreads();
  }
  if (active) {
#pragma unroll
    for (int s = 0; s < NPL; ++s) {
      const int j = lane + 64 * s;
      if (j < Ny) y[((int64_t)2 * j + f) * Nxi + k] = v[s];
    }
  }
}

// y_b = Kinv_b x_b for every block-Jacobi block b, with Kinv_b = (L_b U_b)^{-1}
// the dense inverse of the block's ILU(0) factors (same preconditioner as the
// sweeps above, applied as a bandwidth-bound batched GEMV).  Kinv_b is stored
// column-major over the block's rows in velocity-major order (line, node).
// grid (row tiles of 64, blocks), block 256: the 4 wavefronts split the columns,
// lanes own rows (coalesced column reads), partial sums meet in LDS.
// XCD-aware workgroup order.  Workgroups are dispatched round-robin over the 8
// XCDs (linear id L runs on XCD L mod 8), each with its own L2.  Mapping L to the
// logical index q = (L mod 8) * (nfull / 8) + L / 8 (a bijection on the first
// nfull = 8 floor(nwg / 8) ids, identity on the tail) gives every XCD a contiguous
// range of logical workgroups, so neighbouring velocity nodes, whose strided 16 B
// vector entries share 128 B lines, are served by the same L2.
__device__ __forceinline__ int xcd_logical_id() {
  const int nwg = gridDim.x * gridDim.y;
  const int L = blockIdx.y * gridDim.x + blockIdx.x;
  const int nfull = nwg & ~7;
  return (L < nfull) ? (L & 7) * (nfull >> 3) + (L >> 3) : L;
}

template <class R, int NW>
__global__ void __launch_bounds__(64 * NW) k_blockinv_apply(const cv<R>* __restrict__ x,
                                                            cv<R>* __restrict__ y, int Ny, int Nxi,
                                                            int nl, const cv<R>* __restrict__ Kinv,
                                                            const int64_t* __restrict__ koff,
                                                            const int* __restrict__ skip) {
  extern __shared__ unsigned char lds_raw[];
  cv<R>* xsb = reinterpret_cast<cv<R>*>(lds_raw);   // [nb] block input, then [NW][64] partials
  if (skip && *skip) return;
  const int q = xcd_logical_id();
  const int b = q / gridDim.x, tile = q - b * gridDim.x;
  const int nlines = 2 * Nxi;
  const int nl_blk = min(nl, nlines - b * nl);
  const int nb = nl_blk * Ny;
  const int l0 = b * nl;
  for (int c = threadIdx.x; c < nb; c += 64 * NW) {
    const int lg = l0 + c / Ny, j = c % Ny;
    const int f = lg / Nxi, k = lg - f * Nxi;
    xsb[c] = x[((int64_t)2 * j + f) * Nxi + k];
  }
  __syncthreads();
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = tile * 64 + lane;
  const cv<R>* K = Kinv + koff[b];
  cv<R> acc = mk<R>(0, 0);
  if (row < nb) {
    const int cper = (nb + NW - 1) / NW;
    const int cb = wv * cper, ce = min(nb, cb + cper);
    int c = cb;
    for (; c + 8 <= ce; c += 8) {
      cv<R> kv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) kv[u] = K[(int64_t)(c + u) * nb + row];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc = cadd(acc, cmul(kv[u], xsb[c + u]));
    }
    for (; c < ce; ++c) acc = cadd(acc, cmul(K[(int64_t)c * nb + row], xsb[c]));
  }
  __syncthreads();
  cv<R>* part = xsb + nb;
  part[wv * 64 + lane] = acc;
  __syncthreads();
  if (wv == 0 && row < nb) {
    cv<R> rr = part[lane];
#pragma unroll
    for (int w = 1; w < NW; ++w) rr = cadd(rr, part[w * 64 + lane]);
    const int lg = l0 + row / Ny, j = row % Ny;
    const int f = lg / Nxi, k = lg - f * Nxi;
    y[((int64_t)2 * j + f) * Nxi + k] = rr;
  }
}

// ------------------------------------- structured exact (A - sigma B)^{-1} ----
//
// A - sigma B = P - Ut M: P is block diagonal over the velocity lines and its
// block depends on the velocity node k only, P_k = xi_x,k D_x + diag(nu_j + i beta
// xi_y,k - sigma) with unit inflow rows; Ut M is the rank-r moment coupling of
// every node j (U with inflow rows zeroed).  By the Woodbury identity
//   (A - sigma B)^{-1} x = P^{-1} (x + Ut d),  d = S^{-1} M P^{-1} x,
// with the (r Ny) x (r Ny) capacitance S = I - M P^{-1} Ut (index q = j r + a).

// y = P^{-1} (x + Ut d) for both fields of the nodes of one slot, reading the
// slot's inverse once: P_k^{-1} for node k = slot_node[s] and, with sigma real,
// conj(P_k^{-1}) = P_k'^{-1} for its mirror k' = slot_mate[s] (same xi_x, xi_y
// negated), so up to four right-hand sides per read.  d == nullptr skips the rank
// update.  Pinv: [slots][Ny x Ny] column-major.  Lanes own rows, the NW
// wavefronts split the columns and their partial sums are added in fixed order.
// grid ((Ny + 63) / 64, slots), block 64 NW, dynamic LDS (cmax Ny + cmax 64 NW)
// * sizeof(cv<R>), cmax = 4 when any slot has a mate, else 2.
template <class R, int NW, bool PAIR>
__global__ void __launch_bounds__(64 * NW) k_line_inverse(const cv<R>* __restrict__ x,
                                                          cv<R>* __restrict__ y, int Ny, int Nxi,
                                                          int r, const cv<R>* __restrict__ Pinv,
                                                          const int* __restrict__ slot_node,
                                                          const int* __restrict__ slot_mate, int cmax,
                                                          const R* __restrict__ U,
                                                          const R* __restrict__ xix,
                                                          const cv<R>* __restrict__ d,
                                                          const int* __restrict__ skip) {
  extern __shared__ unsigned char lds_raw[];
  cv<R>* xs = reinterpret_cast<cv<R>*>(lds_raw);   // [cmax][Ny]: node (g, h), mate (g, h)
  cv<R>* part = xs + cmax * Ny;                     // [cmax][NW][64]
  if (skip && *skip) return;
  const int q = xcd_logical_id();
  const int sl = q / gridDim.x, tile = q - sl * gridDim.x;
  const int k = slot_node[sl], km = PAIR ? slot_mate[sl] : -1;
  const bool pair = PAIR && km >= 0;
  const int ncol = pair ? 4 : 2;
  const R xk = xix[k];                              // the mate has the same xi_x
  for (int c = threadIdx.x; c < ncol * Ny; c += 64 * NW) {
    const int col = c / Ny, m = c - col * Ny;
    const int f = col & 1, kk = (col < 2) ? k : km;
    cv<R> v = x[((int64_t)2 * m + f) * Nxi + kk];
    const bool inflow = (m == Ny - 1 && xk > 0) || (m == 0 && xk < 0);
    if (d && !inflow) {
      for (int b = 0; b < r; ++b) {
        const R u = U[(((int64_t)m * 2 + f) * r + b) * Nxi + kk];
        const cv<R> db = d[m * r + b];
        v.x += u * db.x;
        v.y += u * db.y;
      }
    }
    xs[c] = v;
  }
  __syncthreads();
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = tile * 64 + lane;
  const cv<R>* K = Pinv + (int64_t)sl * Ny * Ny;
  // a: P x at the node; b: conj(P) x at the mate, conj(p) v = (p.x v.x + p.y v.y, p.x v.y - p.y v.x)
  cv<R> a0 = mk<R>(0, 0), a1 = mk<R>(0, 0), b0 = mk<R>(0, 0), b1 = mk<R>(0, 0);
  auto cjmul = [](cv<R> p, cv<R> v) { return mk<R>(p.x * v.x + p.y * v.y, p.x * v.y - p.y * v.x); };
  if (row < Ny) {
    const int cper = (Ny + NW - 1) / NW;
    const int cb = wv * cper, ce = min(Ny, cb + cper);
    int c = cb;
    for (; c + 8 <= ce; c += 8) {
      cv<R> kv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) kv[u] = K[(int64_t)(c + u) * Ny + row];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        a0 = cadd(a0, cmul(kv[u], xs[c + u]));
        a1 = cadd(a1, cmul(kv[u], xs[Ny + c + u]));
      }
      if (pair) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          b0 = cadd(b0, cjmul(kv[u], xs[2 * Ny + c + u]));
          b1 = cadd(b1, cjmul(kv[u], xs[3 * Ny + c + u]));
        }
      }
    }
    for (; c < ce; ++c) {
      const cv<R> kv = K[(int64_t)c * Ny + row];
      a0 = cadd(a0, cmul(kv, xs[c]));
      a1 = cadd(a1, cmul(kv, xs[Ny + c]));
      if (pair) {
        b0 = cadd(b0, cjmul(kv, xs[2 * Ny + c]));
        b1 = cadd(b1, cjmul(kv, xs[3 * Ny + c]));
      }
    }
  }
  part[(0 * NW + wv) * 64 + lane] = a0;
  part[(1 * NW + wv) * 64 + lane] = a1;
  if (pair) {
    part[(2 * NW + wv) * 64 + lane] = b0;
    part[(3 * NW + wv) * 64 + lane] = b1;
  }
  __syncthreads();
  if (wv < ncol && row < Ny) {
    const cv<R>* pf = part + wv * NW * 64;
    cv<R> rr = pf[lane];
#pragma unroll
    for (int w = 1; w < NW; ++w) rr = cadd(rr, pf[w * 64 + lane]);
    y[((int64_t)2 * row + (wv & 1)) * Nxi + (wv < 2 ? k : km)] = rr;
  }
}

// d = S^{-1} c with c_q = m_a(j), q = j r + a, summed from the moment partials in
// fixed order.  One wavefront per row of S^{-1} (row-major, Rd x Rd, Rd = r Ny),
// FP64 accumulation.  grid ceil(Rd / 4), block 256, dynamic LDS Rd * sizeof(cv<R>).
template <class R>
__global__ void __launch_bounds__(256) k_capacitance(const cv<R>* __restrict__ mom, int Ny, int r,
                                                     int S, const cv<R>* __restrict__ Sinv,
                                                     cv<R>* __restrict__ d,
                                                     const int* __restrict__ skip) {
  extern __shared__ unsigned char lds_raw[];
  cv<R>* cs = reinterpret_cast<cv<R>*>(lds_raw);
  if (skip && *skip) return;
  const int Rd = r * Ny;
  for (int q = threadIdx.x; q < Rd; q += 256) {
    const int j = q / r, a = q - j * r;
    cs[q] = mom_at<R>(mom, 0, Ny, j, a, r, S);
  }
  __syncthreads();
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int q = blockIdx.x * 4 + wv;
  if (q >= Rd) return;
  double dr = 0.0, di = 0.0;
  const cv<R>* srow = Sinv + (int64_t)q * Rd;
  for (int c = lane; c < Rd; c += 64) {
    const cv<R> sv = srow[c], xv = cs[c];
    dr += (double)sv.x * xv.x - (double)sv.y * xv.y;
    di += (double)sv.x * xv.y + (double)sv.y * xv.x;
  }
  dr = wave_sum(dr);
  di = wave_sum(di);
  if (lane == 0) d[q] = mk<R>((R)dr, (R)di);
}

// ------------------------------------ structured inverse set-up (device) ----
//
// In-place inversion of one N x N complex matrix in global memory by one
// workgroup: Gauss-Jordan elimination with partial (row) pivoting, the pivot
// the entry of largest modulus in the column (the first on ties), the row
// interchanges undone as column interchanges in reverse order at the end.
// Column-major storage, (i, j) at j N + i; on a row-major matrix the same steps
// invert the transpose, which is the row-major inverse.  The matrix stays in
// the workgroup's caches; each step stages the scaled pivot row and the old
// pivot column in LDS.  Returns false (uniformly) for an exactly singular matrix.
// lds: [N] scaled pivot row, [N] pivot column, [N] pivot rows (int).
__device__ bool gj_invert(double2* __restrict__ a, int N, double2* srow, double2* fcol, int* piv) {
  __shared__ int s_p, s_sing;
  const int NN = N * N;
  for (int c = 0; c < N; ++c) {
    if (threadIdx.x < 64) {
      double best = -1.0;
      int bi = N;
      for (int i = c + (int)threadIdx.x; i < N; i += 64) {
        const double2 v = a[(int64_t)c * N + i];
        const double m = v.x * v.x + v.y * v.y;
        if (m > best) { best = m; bi = i; }
      }
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (threadIdx.x == 0) {
        s_p = bi;
        piv[c] = bi;
        s_sing = (best > 0.0) ? 0 : 1;
      }
    }
    __syncthreads();
    if (s_sing) return false;
    const int p = s_p;
    if (p != c) {
      for (int j = threadIdx.x; j < N; j += blockDim.x) {
        const double2 t = a[(int64_t)j * N + c];
        a[(int64_t)j * N + c] = a[(int64_t)j * N + p];
        a[(int64_t)j * N + p] = t;
      }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < N; t += blockDim.x) {
      srow[t] = a[(int64_t)t * N + c];
      fcol[t] = a[(int64_t)c * N + t];
    }
    __syncthreads();
    const double2 pv = srow[c];
    const double pm = 1.0 / (pv.x * pv.x + pv.y * pv.y);
    const double2 inv = make_double2(pv.x * pm, -pv.y * pm);
    __syncthreads();
    for (int t = threadIdx.x; t < N; t += blockDim.x) srow[t] = (t == c) ? inv : cmul(srow[t], inv);
    __syncthreads();
    for (int e = threadIdx.x; e < NN; e += blockDim.x) {
      const int j = e / N, i = e - j * N;
      double2 v;
      if (i == c) {
        v = srow[j];
      } else {
        const double2 f = fcol[i];
        if (j == c) {
          v = cmul(f, inv);
          v.x = -v.x;
          v.y = -v.y;
        } else {
          v = csub(a[e], cmul(f, srow[j]));
        }
      }
      a[e] = v;
    }
    __syncthreads();
  }
  for (int c = N - 1; c >= 0; --c) {
    const int p = piv[c];
    if (p != c) {
      for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const double2 t = a[(int64_t)c * N + i];
        a[(int64_t)c * N + i] = a[(int64_t)p * N + i];
        a[(int64_t)p * N + i] = t;
      }
    }
    __syncthreads();
  }
  return true;
}

// The velocity-line block of slot sl, P_k = xi_x,k D_x + diag(nu_j + i beta
// xi_y,k - sigma) with unit inflow rows (k = slot_node[sl]), written
// column-major into the slot and inverted in place.  One workgroup per slot;
// status[sl] = 1 for an exactly singular block, else 0.  Dx row-major.
// Dynamic LDS: 2 Ny double2 + Ny int.
__global__ void __launch_bounds__(256) k_line_blocks_invert(double2* __restrict__ Pinv, int Ny,
                                                            const int* __restrict__ slot_node,
                                                            const double* __restrict__ Dx,
                                                            const double* __restrict__ xix,
                                                            const double* __restrict__ xiy,
                                                            const double* __restrict__ nu, double beta,
                                                            double sre, double sim, int* __restrict__ status) {
  extern __shared__ unsigned char lds_raw[];
  double2* srow = reinterpret_cast<double2*>(lds_raw);
  double2* fcol = srow + Ny;
  int* piv = reinterpret_cast<int*>(fcol + Ny);
  const int sl = blockIdx.x;
  const int k = slot_node[sl];
  double2* a = Pinv + (int64_t)sl * Ny * Ny;
  const double xk = xix[k], by = beta * xiy[k];
  for (int e = threadIdx.x; e < Ny * Ny; e += blockDim.x) {
    const int j = e / Ny, i = e - j * Ny;
    const bool bc = (i == Ny - 1 && xk > 0.0) || (i == 0 && xk < 0.0);
    double2 v;
    if (bc) {
      v = make_double2(i == j ? 1.0 : 0.0, 0.0);
    } else {
      v = make_double2(xk * Dx[(int64_t)i * Ny + j], 0.0);
      if (i == j) {
        v.x += nu[i] - sre;
        v.y += by - sim;
      }
    }
    a[e] = v;
  }
  __syncthreads();
  const bool ok = gj_invert(a, Ny, srow, fcol, piv);
  if (threadIdx.x == 0) status[sl] = ok ? 0 : 1;
}

// The same for Ny <= 96 with the block held in LDS (147 KB at Ny = 96, one
// workgroup per CU): built there, inverted by the same Gauss-Jordan steps, and
// written out once; the global-memory version rewrites the whole block at every
// step.  Results are bit-identical to it (same operations in the same order).
constexpr int kLdsLineMax = 96;
__global__ void __launch_bounds__(256) k_line_blocks_invert_lds(double2* __restrict__ Pinv, int Ny,
                                                                const int* __restrict__ slot_node,
                                                                const double* __restrict__ Dx,
                                                                const double* __restrict__ xix,
                                                                const double* __restrict__ xiy,
                                                                const double* __restrict__ nu, double beta,
                                                                double sre, double sim, int* __restrict__ status) {
  __shared__ double2 mat[kLdsLineMax * kLdsLineMax];
  __shared__ double2 srow[kLdsLineMax], fcol[kLdsLineMax];
  __shared__ int piv[kLdsLineMax];
  const int sl = blockIdx.x;
  const int k = slot_node[sl];
  const double xk = xix[k], by = beta * xiy[k];
  for (int e = threadIdx.x; e < Ny * Ny; e += blockDim.x) {
    const int j = e / Ny, i = e - j * Ny;
    const bool bc = (i == Ny - 1 && xk > 0.0) || (i == 0 && xk < 0.0);
    double2 v;
    if (bc) {
      v = make_double2(i == j ? 1.0 : 0.0, 0.0);
    } else {
      v = make_double2(xk * Dx[(int64_t)i * Ny + j], 0.0);
      if (i == j) {
        v.x += nu[i] - sre;
        v.y += by - sim;
      }
    }
    mat[e] = v;
  }
  __syncthreads();
  const bool ok = gj_invert(mat, Ny, srow, fcol, piv);
  double2* a = Pinv + (int64_t)sl * Ny * Ny;
  for (int e = threadIdx.x; e < Ny * Ny; e += blockDim.x) a[e] = mat[e];
  if (threadIdx.x == 0) status[sl] = ok ? 0 : 1;
}

// Partial sums of the moment capacitance's coupling part
//   G[(j, a), (j', b)] = sum_k P_k^{-1}(j, j') sum_f M_a(j, f, k) Ut_b(j', f, k)
// (Ut = U with inflow rows zeroed) over the node range of part ks: grid (Ny [j'],
// KS), one thread per row j; slot_of[k] / conj_of[k] give node k's stored
// inverse (conjugated for a mirrored node).  part [KS][Rd][Rd], Rd = r Ny,
// row-major over q = j r + a.
__global__ void __launch_bounds__(128) k_cap_partial(const double2* __restrict__ Pinv, int Ny, int Nxi,
                                                     int r, const int* __restrict__ slot_of,
                                                     const int* __restrict__ conj_of,
                                                     const double* __restrict__ M,
                                                     const double* __restrict__ U,
                                                     const double* __restrict__ xix,
                                                     double2* __restrict__ part) {
  const int jp = blockIdx.x, ks = blockIdx.y, KS = gridDim.y;
  const int per = (Nxi + KS - 1) / KS;
  const int k0 = ks * per, k1 = min(Nxi, k0 + per);
  const int Rd = r * Ny;
  for (int j = threadIdx.x; j < Ny; j += blockDim.x) {
    double2 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = make_double2(0.0, 0.0);
    for (int k = k0; k < k1; ++k) {
      const double xk = xix[k];
      if ((jp == Ny - 1 && xk > 0.0) || (jp == 0 && xk < 0.0)) continue;
      double2 w = Pinv[((int64_t)slot_of[k] * Ny + jp) * Ny + j];
      if (conj_of[k]) w.y = -w.y;
      double g[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) g[a][b] = 0.0;
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        double ma[4], ub[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          ma[a] = (a < r) ? M[(((int64_t)j * r + a) * 2 + f) * Nxi + k] : 0.0;
          ub[a] = (a < r) ? U[(((int64_t)jp * 2 + f) * r + a) * Nxi + k] : 0.0;
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) g[a][b] = fma(ma[a], ub[b], g[a][b]);
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          acc[a][b].x = fma(w.x, g[a][b], acc[a][b].x);
          acc[a][b].y = fma(w.y, g[a][b], acc[a][b].y);
        }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if (a < r && b < r) part[((int64_t)ks * Rd + j * r + a) * Rd + jp * r + b] = acc[a][b];
  }
}

// S = I - sum over the KS parts (added in part order), row-major Rd x Rd.
__global__ void __launch_bounds__(256) k_cap_finish(const double2* __restrict__ part, int KS, int Rd,
                                                    double2* __restrict__ S) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t RR = (int64_t)Rd * Rd;
  if (e >= RR) return;
  double2 v = part[e];
  for (int ks = 1; ks < KS; ++ks) v = cadd(v, part[(int64_t)ks * RR + e]);
  const int q = (int)(e / Rd), qc = (int)(e - (int64_t)q * Rd);
  S[e] = make_double2((q == qc ? 1.0 : 0.0) - v.x, -v.y);
}

// Gauss-Jordan inversion of an N x N row-major matrix across many workgroups,
// one pivot step per launch: step c reads A and writes the next iterate to B
// (separate buffers, so no workgroup reads what another writes in the launch).
// Every workgroup finds the pivot of column c itself (largest modulus among rows
// >= c, the first on ties; the same result everywhere), and writes its rows of
// the row-interchanged, eliminated matrix: row c = pivot row / pivot (entry c:
// 1 / pivot), row p = old row c, and every row i != c gets row_i - a_ic row_c'
// (entry c: -a_ic / pivot), exactly the in-place Gauss-Jordan update.  The
// pivot row index is recorded in piv[c]; status[0] = 1 for a zero pivot.
// grid ceil(N / 4), block 256 (4 rows per workgroup, lanes over columns).
__global__ void __launch_bounds__(256) k_gj_step(const double2* __restrict__ A, double2* __restrict__ B, int N,
                                                 int c, int* __restrict__ piv, int* __restrict__ status) {
  __shared__ int s_p;
  __shared__ double2 s_inv;
  if (threadIdx.x < 64) {
    double best = -1.0;
    int bi = N;
    for (int i = c + (int)threadIdx.x; i < N; i += 64) {
      const double2 v = A[(int64_t)i * N + c];
      const double mm = v.x * v.x + v.y * v.y;
      if (mm > best) { best = mm; bi = i; }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    if (threadIdx.x == 0) {
      s_p = (best > 0.0) ? bi : c;
      const double2 pv = A[(int64_t)s_p * N + c];
      const double pm = (best > 0.0) ? 1.0 / best : 0.0;
      s_inv = make_double2(pv.x * pm, -pv.y * pm);
      if (blockIdx.x == 0) {
        piv[c] = s_p;
        if (!(best > 0.0)) status[0] = 1;
        else if (c == 0) status[0] = 0;
      }
    }
  }
  __syncthreads();
  const int p = s_p;
  const double2 inv = s_inv;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + wv;
  if (i >= N) return;
  const int src = (i == c) ? p : (i == p ? c : i);
  const double2* arow = A + (int64_t)src * N;
  const double2* prow = A + (int64_t)p * N;
  double2* brow = B + (int64_t)i * N;
  if (i == c) {
    for (int j = lane; j < N; j += 64) brow[j] = (j == c) ? inv : cmul(prow[j], inv);
  } else {
    const double2 f = arow[c];
    const double2 fi = cmul(f, inv);
    for (int j = lane; j < N; j += 64) {
      if (j == c) {
        brow[j] = make_double2(-fi.x, -fi.y);
      } else {
        brow[j] = csub(arow[j], cmul(f, cmul(prow[j], inv)));
      }
    }
  }
}

// out[i][j] = X[i][pi(j)] with pi the composition of the interchanges of rows c
// and piv[c], c = 0 .. N-1 (the inverse of the interchanged matrix times the
// permutation).  grid ceil(N / 4), block 256.
__global__ void __launch_bounds__(256) k_gj_unpermute(const double2* __restrict__ X, double2* __restrict__ out,
                                                      int N, const int* __restrict__ piv) {
  extern __shared__ int s_pi[];
  for (int j = threadIdx.x; j < N; j += blockDim.x) {
    int pos = j;
    for (int c = 0; c < N; ++c) {
      const int q = piv[c];
      if (pos == c) pos = q;
      else if (pos == q) pos = c;
    }
    s_pi[j] = pos;
  }
  __syncthreads();
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + wv;
  if (i >= N) return;
  for (int j = lane; j < N; j += 64) out[(int64_t)i * N + j] = X[(int64_t)i * N + s_pi[j]];
}


// ------------------------------------------------------- vector kernels ----

// ---- two-phase deterministic reductions (no cross-workgroup synchronisation) ----
//
// Phase 1 (k_dot_partial): one wavefront per (vector, chunk of t) writes the
// chunk's partial sum.  Phase 2 happens in the consumer: every workgroup of the
// next kernel reduces the partials of each vector with one wavefront in a fixed
// order, so all workgroups obtain bit-identical coefficients.

// partial[q * nch + chunk] = sum_{t in chunk} conj(S_q[t]) x[t] for q < m; with
// with_norm, row q = m holds sum |x[t]|^2.  1-D grid of nch ceil(mtot / 4)
// workgroups, block 256: item (chunk, row group) in chunk-major XCD order, so
// the row groups that read one chunk of x do so from one L2.
// The vectors S_q are stored in real type RS (the Krylov basis may be FP32
// under FP64 arithmetic), x and the arithmetic in R.
template <class R, class RS = R>
__global__ void __launch_bounds__(256) k_dot_partial(const cv<RS>* __restrict__ s0, int m0,
                                                     const cv<RS>* __restrict__ s1, int m1,
                                                     const cv<R>* __restrict__ x, int64_t n, int chunk,
                                                     double2* __restrict__ partial, int with_norm,
                                                     const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int m = m0 + m1;
  const int mtot = m + (with_norm ? 1 : 0);
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int gy = (mtot + 3) / 4;
  const int64_t item = xcd_item(blockIdx.x, gridDim.x);
  const int bx = (int)(item / gy), by = (int)(item - (int64_t)bx * gy);
  const int nch = gridDim.x / gy;
  const int i = by * 4 + wv;
  if (i >= mtot) return;
  const int64_t t0 = (int64_t)bx * chunk;
  const int64_t t1 = min(n, t0 + chunk);
  R ar = 0, ai = 0;
  auto accumulate = [&](const auto* __restrict__ sv) {
    using SV = std::remove_cv_t<std::remove_reference_t<decltype(sv[0])>>;
    int64_t t = t0 + lane;
    for (; t + 192 < t1; t += 256) {
      SV a0[4];
      cv<R> b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) { a0[u] = sv[t + 64 * u]; b[u] = x[t + 64 * u]; }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const cv<R> a = mk<R>((R)a0[u].x, (R)a0[u].y);
        ar = fma(a.x, b[u].x, ar); ar = fma(a.y, b[u].y, ar);
        ai = fma(a.x, b[u].y, ai); ai = fma(-a.y, b[u].x, ai);
      }
    }
    for (; t < t1; t += 64) {
      const cv<R> a = mk<R>((R)sv[t].x, (R)sv[t].y), b = x[t];
      ar = fma(a.x, b.x, ar); ar = fma(a.y, b.y, ar);
      ai = fma(a.x, b.y, ai); ai = fma(-a.y, b.x, ai);
    }
  };
  if (i < m) accumulate((i < m0) ? s0 + (int64_t)i * n : s1 + (int64_t)(i - m0) * n);
  else accumulate(x);
  if (i >= m) ai = 0;
  const double dr = wave_sum((double)ar);
  const double di = wave_sum((double)ai);
  if (lane == 0) partial[(int64_t)i * nch + bx] = make_double2(dr, di);
}

// c[q] = sum over chunks of partial[q * nch + chunk], q < mtot, into LDS; one
// wavefront per q, lanes over chunks, fixed tree: identical in every workgroup.
// With stage (dynamic LDS of mtot * nch entries) the partials are first copied in
// with all loads in flight, so the per-q rounds wait on LDS instead of on L2.
__device__ __forceinline__ void reduce_partials(const double2* __restrict__ partial, int mtot, int nch,
                                                double2* c, double2* stage) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  const double2* src = partial;
  if (stage) {
    const int tot = mtot * nch;
#pragma unroll 8
    for (int e = threadIdx.x; e < tot; e += blockDim.x) stage[e] = partial[e];
    __syncthreads();
    src = stage;
  }
  // each lane adds its chunks in order lane, lane + 64, ...; four of them are
  // loaded together (a chunk count that is not a multiple of 64 is predicated)
  for (int q = wv; q < mtot; q += nw) {
    const double2* pq = src + (int64_t)q * nch;
    double sr = 0.0, si = 0.0;
    for (int c0 = lane; c0 < nch; c0 += 256) {
      double2 pv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) pv[i] = (c0 + 64 * i < nch) ? pq[c0 + 64 * i] : make_double2(0.0, 0.0);
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (c0 + 64 * i < nch) { sr += pv[i].x; si += pv[i].y; }
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
    if (lane == 0) c[q] = make_double2(sr, si);
  }
  __syncthreads();
}

// Final reduction of k_dot_partial into out (single workgroup).  mode 0 out = c,
// 1 out += c, 2 out = Hinv c, 3 as 0 plus out[m] = ||x||^2; out2 (optional) += c.
__global__ void __launch_bounds__(256) k_dot_reduce(const double2* __restrict__ partial, int m, int nch,
                                                    double2* __restrict__ out, int mode,
                                                    const double2* __restrict__ Hinv,
                                                    double2* __restrict__ out2, int staged,
                                                    const int* __restrict__ skip) {
  __shared__ double2 c[256];
  extern __shared__ double2 stage_dyn[];
  if (skip && *skip) return;
  const int mtot = (mode == 3) ? m + 1 : m;
  reduce_partials(partial, mtot, nch, c, staged ? stage_dyn : nullptr);
  for (int q = threadIdx.x; q < mtot; q += 256) {
    double2 v = c[q];
    if (mode == 2) {
      v = make_double2(0.0, 0.0);
      for (int p = 0; p < m; ++p) v = cadd(v, cmul(Hinv[q * m + p], c[p]));
      out[q] = v;
    } else if (mode == 1) {
      out[q] = cadd(out[q], v);
    } else {
      out[q] = v;
    }
    if (out2 && q < m) out2[q] = cadd(out2[q], c[q]);
  }
}

// x -= sum_i S_i c_i where c comes from the dot partials of the previous kernel
// (c = Hinv * sums when Hinv != nullptr).  Workgroup 0 stores c to coef_set
// and/or adds it to coef_add.  With norm_part, each workgroup writes the partial
// ||x_new||^2 of its slice.  grid ceil(n / 256), block 256.
template <class R, class RS = R>
__global__ void __launch_bounds__(256) k_subm_fused(const cv<RS>* __restrict__ s0, int m0,
                                                    const cv<RS>* __restrict__ s1, int m1,
                                                    const double2* __restrict__ partial, int nch,
                                                    const double2* __restrict__ Hinv,
                                                    double2* __restrict__ coef_set,
                                                    double2* __restrict__ coef_add, cv<R>* x, int64_t n,
                                                    double2* __restrict__ norm_part, int staged,
                                                    const int* __restrict__ skip) {
  __shared__ double2 cr[256], cc[256];
  __shared__ double2 sh[4];
  extern __shared__ double2 stage_dyn[];
  if (skip && *skip) return;
  const int m = m0 + m1;
  reduce_partials(partial, m, nch, cr, staged ? stage_dyn : nullptr);
  const double2* c = cr;
  if (Hinv) {
    for (int q = threadIdx.x; q < m; q += 256) {
      double2 v = make_double2(0.0, 0.0);
      for (int p = 0; p < m; ++p) v = cadd(v, cmul(Hinv[q * m + p], cr[p]));
      cc[q] = v;
    }
    __syncthreads();
    c = cc;
  }
  if (blockIdx.x == 0) {
    for (int q = threadIdx.x; q < m; q += 256) {
      if (coef_set) coef_set[q] = c[q];
      if (coef_add) coef_add[q] = cadd(coef_add[q], c[q]);
    }
  }
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  R a2 = 0;
  if (t < n) {
    const cv<R> acc = cadd(lincomb<R, RS>(s0, m0, n, t, c, 1), lincomb<R, RS>(s1, m1, n, t, c + m0, 1));
    const cv<R> xv = csub(x[t], acc);
    x[t] = xv;
    a2 = xv.x * xv.x + xv.y * xv.y;
  }
  if (norm_part) {
    const double2 bs = block_sum256(make_double2((double)a2, 0.0), sh);
    if (threadIdx.x == 0) norm_part[blockIdx.x] = bs;
  }
}

// Is a second Gram-Schmidt pass needed?  DGKS criterion (Daniel, Gragg, Kaufman
// and Stewart 1976): reorthogonalise when the first pass leaves less than eta of
// the norm, ||x_after||^2 < eta2 ||x_before||^2.  before^2 is row m of the dot
// partials (nch chunks, written with with_norm), after^2 the first pass's norm
// partials (nb workgroups).  *skip_out = done || not needed.  grid 1, block 256.
__global__ void __launch_bounds__(256) k_reorth_test(const double2* __restrict__ partial, int m, int nch,
                                                     const double2* __restrict__ norm_part, int nb,
                                                     double eta2, const int* __restrict__ done,
                                                     int* __restrict__ skip_out) {
  __shared__ double2 sh[4];
  if (done && *done) {
    if (threadIdx.x == 0) *skip_out = 1;
    return;
  }
  double before = 0.0, after = 0.0;
  for (int c = threadIdx.x; c < nch; c += 256) before += partial[(int64_t)m * nch + c].x;
  for (int c = threadIdx.x; c < nb; c += 256) after += norm_part[c].x;
  const double2 s = block_sum256(make_double2(before, after), sh);
  if (threadIdx.x == 0) *skip_out = (s.y >= eta2 * s.x) ? 1 : 0;
}

// nrm2 = sum of the nb norm partials (fixed order, every workgroup); x (or dst)
// = x / sqrt(nrm2).  Workgroup 0 stores nrm2 and, when H is given, performs the
// GMRES Givens update of column j (which may set *done).
__device__ void gmres_givens_body(double2* __restrict__ H, int ldh, int j, double nrm2,
                                  double* __restrict__ cs, double2* __restrict__ sn,
                                  double2* __restrict__ g, int* __restrict__ done,
                                  int* __restrict__ steps, const double* __restrict__ beta,
                                  double rtol);
template <class R, class R2 = R>
__global__ void __launch_bounds__(256) k_scale_norm(cv<R>* x, cv<R>* dst, cv<R2>* dst2, int64_t n,
                                                    const double2* __restrict__ norm_part, int nb,
                                                    double2* __restrict__ nrm2_out,
                                                    double2* __restrict__ H, int ldh, int j,
                                                    double* __restrict__ cs, double2* __restrict__ sn,
                                                    double2* __restrict__ g, int* done,
                                                    int* __restrict__ steps,
                                                    const double* __restrict__ beta, double rtol) {
  __shared__ double2 sh[4];
  __shared__ double tot;
  if (done && *done) return;
  // each thread adds its partials b = tid, tid + 256, ... in order, four loaded together
  double ps = 0.0;
  for (int b0 = threadIdx.x; b0 < nb; b0 += 1024) {
    double pv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) pv[i] = (b0 + 256 * i < nb) ? norm_part[b0 + 256 * i].x : 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (b0 + 256 * i < nb) ps += pv[i];
  }
  const double2 s2 = block_sum256(make_double2(ps, 0.0), sh);
  if (threadIdx.x == 0) {
    tot = s2.x;
    if (blockIdx.x == 0) {
      *nrm2_out = make_double2(s2.x, 0.0);
      if (H) gmres_givens_body(H, ldh, j, s2.x, cs, sn, g, done, steps, beta, rtol);
    }
  }
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const R sc = (R)(1.0 / sqrt(tot));
  const cv<R> v = x[t];
  const cv<R> w = mk<R>(v.x * sc, v.y * sc);
  (dst ? dst : x)[t] = w;
  if (dst2) dst2[t] = mk<R2>((R2)w.x, (R2)w.y);
}

// x[t] -= sum_i S_i[t] c[i] over two segments (c on device; c[0..m0) for seg0,
// c[m0..m0+m1) for seg1).  If dst != nullptr the result goes to dst instead.
template <class R>
__global__ void __launch_bounds__(256) k_subm(const cv<R>* __restrict__ s0, int m0,
                                              const cv<R>* __restrict__ s1, int m1,
                                              const double2* __restrict__ c, cv<R>* x,
                                              cv<R>* dst, int64_t n, R sign,
                                              const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const cv<R> acc = cadd(lincomb<R>(s0, m0, n, t, c, 1), lincomb<R>(s1, m1, n, t, c + m0, 1));
  const cv<R> xv = x[t];
  const cv<R> r = mk<R>(xv.x - sign * acc.x, xv.y - sign * acc.y);
  (dst ? dst : x)[t] = r;
}

// out_j[t] = sum_i S_i[t] coef[i * ldc + j] for j < k (basis rotation V <- V U),
// coefficients on the device.  grid.y = output vector j.
template <class R, class RS = R>
__global__ void __launch_bounds__(256) k_combine(const cv<RS>* __restrict__ S, int m, int64_t n,
                                                 const double2* __restrict__ coef, int ldc,
                                                 cv<R>* __restrict__ out,
                                                 const int* __restrict__ count) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (t >= n) return;
  const int mm = count ? min(m, *count) : m;
  out[(int64_t)j * n + t] = lincomb<R, RS>(S, mm, n, t, coef + j, ldc);
}

// The same rotation for CB outputs per pass: every input entry S_i[t] is read
// once per group of CB outputs instead of once per output; each output is
// accumulated in the order of k_combine (i = 0, 1, ...), so the results are
// bit-identical to it.  1-D grid of ceil(n / 256) ceil(k / CB) workgroups.
template <class R, int CB>
__global__ void __launch_bounds__(256) k_combine_multi(const cv<R>* __restrict__ S, int m, int64_t n,
                                                       const double2* __restrict__ coef, int ldc, int k,
                                                       cv<R>* __restrict__ out, const int* __restrict__ count) {
  // 1-D grid, item (entry block, output group) in entry-block-major XCD order:
  // the groups that read the same entries of S do so from one L2
  const int ng = (k + CB - 1) / CB;
  const int64_t item = xcd_item(blockIdx.x, gridDim.x);
  const int64_t tb = item / ng;
  const int64_t t = tb * blockDim.x + threadIdx.x;
  const int j0 = (int)(item - tb * ng) * CB;
  if (t >= n) return;
  const int mm = count ? min(m, *count) : m;
  cv<R> acc[CB];
#pragma unroll
  for (int q = 0; q < CB; ++q) acc[q] = mk<R>(0, 0);
  int i = 0;
  for (; i + 4 <= mm; i += 4) {
    cv<R> sv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) sv[u] = S[(int64_t)(i + u) * n + t];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double2* cr = coef + (int64_t)(i + u) * ldc + j0;
#pragma unroll
      for (int q = 0; q < CB; ++q)
        if (j0 + q < k) acc[q] = cadd(acc[q], cmul(sv[u], narrow<R>(cr[q])));
    }
  }
  for (; i < mm; ++i) {
    const cv<R> sv = S[(int64_t)i * n + t];
    const double2* cr = coef + (int64_t)i * ldc + j0;
#pragma unroll
    for (int q = 0; q < CB; ++q)
      if (j0 + q < k) acc[q] = cadd(acc[q], cmul(sv, narrow<R>(cr[q])));
  }
#pragma unroll
  for (int q = 0; q < CB; ++q)
    if (j0 + q < k) out[(int64_t)(j0 + q) * n + t] = acc[q];
}

// x *= 1 / sqrt(*nrm2) (nrm2 on device), optionally into dst.
template <class R>
__global__ void k_scale_rsqrt(cv<R>* x, cv<R>* dst, float2* dst32, int64_t n, const double2* __restrict__ nrm2,
                              const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const R sc = (R)(1.0 / sqrt(nrm2->x));
  const cv<R> v = x[t];
  const cv<R> w = mk<R>(v.x * sc, v.y * sc);
  (dst ? dst : x)[t] = w;
  if (dst32) dst32[t] = make_float2((float)w.x, (float)w.y);
}

// y = a x (+ y if accum), a host scalar.
template <class R>
__global__ void k_axpby(const cv<R>* __restrict__ x, cv<R>* y, int64_t n, R are, R aim, int accum) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const cv<R> xv = x[t];
  cv<R> r = mk<R>(are * xv.x - aim * xv.y, are * xv.y + aim * xv.x);
  if (accum) r = cadd(r, y[t]);
  y[t] = r;
}

// out_v = R conj(x_v) for nvec vectors: entry (j, f, k) takes conj of entry
// (j, f, mk[k]), mk the xi_y reflection of the velocity nodes.  grid (ceil(n /
// 256), nvec).
__global__ void k_mirror_conj(const double2* __restrict__ x, double2* __restrict__ out, int64_t n, int Nxi,
                              const int* __restrict__ mk) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int64_t v = blockIdx.y;
  const int64_t row = t / Nxi;
  const int k = (int)(t - row * Nxi);
  const double2 a = x[v * n + row * Nxi + mk[k]];
  out[v * n + t] = make_double2(a.x, -a.y);
}

// Precision conversion: y32 = (float) x64, or y64 (+)= (double) x32.
__global__ void k_narrow(const double2* __restrict__ x, float2* __restrict__ y, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double2 v = x[t];
  y[t] = make_float2((float)v.x, (float)v.y);
}
__global__ void k_widen(const float2* __restrict__ x, double2* __restrict__ y, int64_t n, int accum) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float2 v = x[t];
  double2 r = make_double2((double)v.x, (double)v.y);
  if (accum) r = cadd(r, y[t]);
  y[t] = r;
}

// GMRES bookkeeping on the device (one thread): column j of the Hessenberg
// (h[0..j] from Gram-Schmidt, h[j+1] = sqrt(nrm2)) gets the previous Givens
// rotations, a new rotation zeroes h[j+1], g is rotated, and the residual
// estimate |g[j+1]| decides whether the cycle is done.
__device__ void gmres_givens_body(double2* __restrict__ H, int ldh, int j, double nrm2,
                                  double* __restrict__ cs, double2* __restrict__ sn,
                                  double2* __restrict__ g, int* __restrict__ done,
                                  int* __restrict__ steps, const double* __restrict__ beta,
                                  double rtol) {
  const double tol_abs = rtol * (*beta);
  double2* h = H + (int64_t)j * ldh;
  h[j + 1] = make_double2(sqrt(nrm2), 0.0);
  for (int i = 0; i < j; ++i) {
    const double2 a = h[i], b = h[i + 1];
    const double2 sb = cmul(sn[i], b);
    const double2 csa = cscale(a, cs[i]);
    const double2 nsa = cmul(make_double2(-sn[i].x, sn[i].y), a);   // -conj(s) a
    h[i] = cadd(csa, sb);
    h[i + 1] = cadd(nsa, cscale(b, cs[i]));
  }
  const double2 a = h[j], b = h[j + 1];
  const double af = sqrt(a.x * a.x + a.y * a.y), ag = sqrt(b.x * b.x + b.y * b.y);
  double c;
  double2 s;
  if (ag == 0.0) { c = 1.0; s = make_double2(0.0, 0.0); }
  else if (af == 0.0) { c = 0.0; s = make_double2(b.x / ag, -b.y / ag); }
  else {
    const double nrm = hypot(af, ag);
    c = af / nrm;
    const double2 ph = make_double2(a.x / af, a.y / af);
    s = cscale(cmul(ph, make_double2(b.x, -b.y)), 1.0 / nrm);
  }
  cs[j] = c;
  sn[j] = s;
  h[j] = cadd(cscale(a, c), cmul(s, b));
  h[j + 1] = make_double2(0.0, 0.0);
  const double2 gj = g[j];
  g[j] = cscale(gj, c);
  g[j + 1] = cmul(make_double2(-s.x, s.y), gj);
  *steps = j + 1;
  const double res = sqrt(g[j + 1].x * g[j + 1].x + g[j + 1].y * g[j + 1].y);
  if (res <= tol_abs || ag == 0.0) *done = 1;
}

// g[0] = sqrt(*nrm2); done = (g[0] == 0); steps = 0.  The first cycle of a
// restarted solve records its initial residual norm in *beta_out, which later
// cycles keep, so that every cycle stops at rtol times the initial residual.
__global__ void k_gmres_init(const double2* __restrict__ nrm2, double2* __restrict__ g, int* done,
                             int* steps, double* beta_out, int first) {
  const double b = sqrt(nrm2->x);
  g[0] = make_double2(b, 0.0);
  *done = (b == 0.0) ? 1 : 0;
  *steps = 0;
  if (first) *beta_out = b;
}

// Back substitution R y = g with the rotated Hessenberg (steps x steps upper).
__global__ void k_gmres_solve(const double2* __restrict__ H, int ldh, const double2* __restrict__ g,
                              const int* __restrict__ steps, double2* __restrict__ yk) {
  const int s = *steps;
  for (int i = s - 1; i >= 0; --i) {
    double2 acc = g[i];
    for (int q = i + 1; q < s; ++q) acc = csub(acc, cmul(H[(int64_t)q * ldh + i], yk[q]));
    const double2 d = H[(int64_t)i * ldh + i];
    const double dd = d.x * d.x + d.y * d.y;
    yk[i] = make_double2((acc.x * d.x + acc.y * d.y) / dd, (acc.y * d.x - acc.x * d.y) / dd);
  }
}

// y = B x: copy with inflow entries zeroed.
__global__ void k_mask_bc(const double2* __restrict__ x, double2* __restrict__ y, int64_t n, int Ny,
                          int Nxi, const double* __restrict__ xi_x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int nc = 2 * Nxi;
  const int j = (int)(i / nc);
  const int k = (int)(i - (int64_t)j * nc) % Nxi;
  const bool bc = (j == Ny - 1 && xi_x[k] > 0.0) || (j == 0 && xi_x[k] < 0.0);
  y[i] = bc ? make_double2(0.0, 0.0) : x[i];
}

// Reset a flag.
__global__ void k_set_int(int* p, int v) { *p = v; }

// ------------------------------------------------------------- launchers ---

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// Column parts of the moment reduction: enough workgroups per vector to fill
// the chip.  A function of the grid only (not of the batch size), so a vector
// gets bit-identical results alone and in a batch.
// Column parts per node for k_moments: one per 512 columns and, from 512
// columns on, enough for about 256 workgroups, with no part under 128 columns;
// at most 8.  (Below 512 columns, splitting measured slower: the consumers then
// add more parts.)
namespace {
std::mutex g_tune_mu;
std::map<std::array<int, 4>, Tuning> g_tune;   // (Ny, Nxi, nvec, precision) -> launch choices
}  // namespace

void tune_set(int Ny, int Nxi, int nvec, int prec, const Tuning& t) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[{Ny, Nxi, nvec, prec}] = t;
}
bool tune_get(int Ny, int Nxi, int nvec, int prec, Tuning* t) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find({Ny, Nxi, nvec, prec});
  if (it == g_tune.end()) return false;
  if (t) *t = it->second;
  return true;
}
void tune_erase(int Ny, int Nxi, int nvec, int prec) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.erase({Ny, Nxi, nvec, prec});
}
void tune_clear() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
}
std::vector<std::pair<std::array<int, 4>, Tuning>> tune_all() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return std::vector<std::pair<std::array<int, 4>, Tuning>>(g_tune.begin(), g_tune.end());
}

int moment_splits(int Ny, int nvec, int Nxi, int prec) {
  (void)nvec;
  const int nc = 2 * Nxi;
  // a tuned split belongs to the shape (the single-vector entry), never to a
  // batch size, so a vector's moments are summed the same way alone and in a batch
  Tuning t;
  if (tune_get(Ny, Nxi, 1, prec, &t) && t.msplit > 0) return std::max(1, std::min({8, t.msplit, nc}));
  if (nc < 512) return 1;
  const int fill = (256 + Ny - 1) / Ny;
  return std::max(1, std::min({8, std::max(nc / 512, fill), nc / 128}));
}

// ------------------------------------------------------- post-processing ----

// Macroscopic perturbations of vector v (blockIdx.x) at every node from the S
// moment partials of k_moments: macros[(v Ny + j) 5 + (rho, u, v, E, T)], with
// T_hat = (4/3)(E_hat - u u_hat), the linearisation of T = (4/3)(E - |u|^2/2)
// about v = 0; umag[v Ny + j] = |U_hat| / max over j, |U_hat| = sqrt(|u_hat|^2 +
// |v_hat|^2).  Each thread rescales the entries it wrote.  grid nvec, block 256.
__global__ void __launch_bounds__(256) k_pert_macros(const double2* __restrict__ mom, int Ny, int r, int S,
                                                     const double* __restrict__ base,
                                                     double2* __restrict__ macros,
                                                     double* __restrict__ umag) {
  __shared__ double smax[256];
  const int v = blockIdx.x;
  double lmax = 0.0;
  for (int j = threadIdx.x; j < Ny; j += 256) {
    const double2 rh = mom_at<double>(mom, v, Ny, j, 0, r, S);
    const double2 uh = mom_at<double>(mom, v, Ny, j, 1, r, S);
    const double2 vh = (r == 4) ? mom_at<double>(mom, v, Ny, j, 2, r, S) : make_double2(0.0, 0.0);
    const double2 eh = mom_at<double>(mom, v, Ny, j, r - 1, r, S);
    const double u = base[(int64_t)j * 4 + 1];
    const double2 th = make_double2((4.0 / 3.0) * (eh.x - u * uh.x), (4.0 / 3.0) * (eh.y - u * uh.y));
    double2* o = macros + ((int64_t)v * Ny + j) * 5;
    o[0] = rh;
    o[1] = uh;
    o[2] = vh;
    o[3] = eh;
    o[4] = th;
    const double a = sqrt(uh.x * uh.x + uh.y * uh.y + vh.x * vh.x + vh.y * vh.y);
    umag[(int64_t)v * Ny + j] = a;
    lmax = fmax(lmax, a);
  }
  smax[threadIdx.x] = lmax;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
    __syncthreads();
  }
  const double mx = smax[0];
  if (mx > 0.0)
    for (int j = threadIdx.x; j < Ny; j += 256) umag[(int64_t)v * Ny + j] /= mx;
}

// Non-equilibrium level of the base flow at node j (blockIdx.x):
// sqrt(sum_k w_k (g_c - g^e)^2), g^e the reduced Maxwellian rho / (pi T)^(Dv/2)
// exp(-((xi_x - u)^2 + xi_y^2) / T) at the node's macros; gc == nullptr (an EQ
// base, g_c = g^e) gives 0.  grid Ny, block 256.
__global__ void __launch_bounds__(256) k_noneq_level(const double* __restrict__ gc,
                                                     const double* __restrict__ base,
                                                     const double* __restrict__ xix,
                                                     const double* __restrict__ xiy,
                                                     const double* __restrict__ w, int Nxi, int Dv,
                                                     double* __restrict__ eneq) {
  __shared__ double2 sh[4];
  const int j = blockIdx.x;
  double acc = 0.0;
  if (gc) {
    const double rho = base[(int64_t)j * 4], u = base[(int64_t)j * 4 + 1], T = base[(int64_t)j * 4 + 3];
    const double pre = rho / (Dv == 2 ? M_PI * T : sqrt(M_PI * T));
    for (int k = threadIdx.x; k < Nxi; k += 256) {
      const double cx = xix[k] - u, cy = xiy[k];
      const double d = gc[(int64_t)j * Nxi + k] - pre * exp(-(cx * cx + cy * cy) / T);
      acc += w[k] * d * d;
    }
  }
  const double2 t = block_sum256(make_double2(acc, 0.0), sh);
  if (threadIdx.x == 0) eneq[j] = sqrt(t.x);
}

// --------------------------------------------- BE-BGK base-flow relaxation ----

// Interface value between x-ascending nodes i and i+1 from the values at i-1, i,
// i+1, i+2: MUSCL upwinded on the sign of xi_x, minmod limiter evaluated as
// (sgn a + sgn b)/2 min(|a|, |b|) of the two one-sided differences.
__device__ __forceinline__ double muscl_face(double pm, double p0, double pp, double ppp, double xi) {
  auto mm = [](double a, double b) {
    return 0.5 * ((a > 0) - (a < 0) + (b > 0) - (b < 0)) * fmin(fabs(a), fabs(b));
  };
  return xi >= 0.0 ? p0 + 0.5 * mm(p0 - pm, pp - p0) : pp - 0.5 * mm(ppp - pp, pp - p0);
}

// One Runge-Kutta stage of the reduced BGK equations at node j (blockIdx.x) of
// the grid order (node 0 at x = +s_inf), state layout q[(2 j + f) Nxi + k]:
//   stage state  Q = q + a kprev (kprev == nullptr: Q = q)
//   kout         = nu (Q^e - Q) - xi_x (Q_{i+1/2} - Q_{i-1/2}) inv_dx_j at the
//                  interior nodes (x-ascending index i = Ny - 1 - j, values beyond
//                  the ends repeat the end node), 0 at the two held end nodes
//   acc          = kout (stage 1) or acc + 2 kout (stages 2, 3)
//   qout         = q + dt6 (acc + kout) (stage 4)
// with Q^e the reduced Maxwellian pair at node j's macros of Q.  The node's 2 Nxi
// columns are split over gridDim.y workgroups, each of which forms the node's
// macros itself (same sums in the same order, so the copies agree bit for bit).
// resid (optional) receives max |kout| over the workgroup's columns at
// resid[j gridDim.y + blockIdx.y].  grid (Ny, parts), block 256.
__global__ void __launch_bounds__(256) k_bgk_stage(const double* __restrict__ q,
                                                   const double* __restrict__ kprev, double a,
                                                   double* __restrict__ kout, double* __restrict__ acc,
                                                   double* __restrict__ qout, double dt6, int stage, int Ny,
                                                   int Nxi, int Dv, const double* __restrict__ xix,
                                                   const double* __restrict__ xiy,
                                                   const double* __restrict__ w,
                                                   const double* __restrict__ inv_dx, double nu_inf,
                                                   double s_visc, double* __restrict__ resid) {
  __shared__ double red[3][256];
  const int j = blockIdx.x, tid = threadIdx.x;
  const int nc = 2 * Nxi;
  const bool held = (j == 0 || j == Ny - 1);
  auto Q = [&](int jj, int c) {
    const int64_t e = (int64_t)jj * nc + c;
    return kprev ? q[e] + a * kprev[e] : q[e];
  };
  // macros of the stage state at node j
  double m0 = 0.0, m1 = 0.0, m2 = 0.0;
  if (!held) {
    for (int k = tid; k < Nxi; k += 256) {
      const double gv = Q(j, k), hv = Q(j, Nxi + k), xx = xix[k], yy = xiy[k];
      m0 += w[k] * gv;
      m1 += w[k] * xx * gv;
      m2 += w[k] * ((xx * xx + yy * yy) * gv + hv);
    }
  }
  red[0][tid] = m0;
  red[1][tid] = m1;
  red[2][tid] = m2;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) {
      red[0][tid] += red[0][tid + st];
      red[1][tid] += red[1][tid + st];
      red[2][tid] += red[2][tid + st];
    }
    __syncthreads();
  }
  const double rho = red[0][0], u = red[1][0] / rho, E = 0.5 * red[2][0] / rho;
  const double T = (4.0 / 3.0) * (E - 0.5 * u * u);
  const double nu = nu_inf * rho * pow(T, 1.0 - s_visc);
  const double pre = rho / (Dv == 2 ? M_PI * T : sqrt(M_PI * T));
  const double hfac = 0.5 * (3 - Dv) * T;
  // neighbours in x-ascending order: i - 1 <-> j + 1, i + 1 <-> j - 1 (clamped)
  const int jm2 = min(j + 2, Ny - 1), jm1 = min(j + 1, Ny - 1), jp1 = max(j - 1, 0), jp2 = max(j - 2, 0);
  const double idx = inv_dx[j];
  const int per = (nc + gridDim.y - 1) / gridDim.y;
  const int cbeg = blockIdx.y * per, cend = min(nc, cbeg + per);
  double rmax = 0.0;
  for (int c = cbeg + tid; c < cend; c += 256) {
    const int64_t e = (int64_t)j * nc + c;
    double r = 0.0;
    if (!held) {
      const int k = (c < Nxi) ? c : c - Nxi;
      const double xx = xix[k], cx = xx - u, cy = xiy[k];
      const double ge = pre * exp(-(cx * cx + cy * cy) / T);
      const double eq = (c < Nxi) ? ge : hfac * ge;
      const double v0 = Q(j, c), vm1 = Q(jm1, c), vm2 = Q(jm2, c), vp1 = Q(jp1, c), vp2 = Q(jp2, c);
      const double fr = muscl_face(vm1, v0, vp1, vp2, xx);    // i + 1/2
      const double fl = muscl_face(vm2, vm1, v0, vp1, xx);    // i - 1/2
      r = nu * (eq - v0) - xx * (fr - fl) * idx;
    }
    kout[e] = r;
    if (stage == 1) acc[e] = r;
    else if (stage < 4) acc[e] += 2.0 * r;
    else qout[e] = q[e] + dt6 * (acc[e] + r);
    const double ar = fabs(r);
    rmax = (ar > rmax || ar != ar) ? ar : rmax;   // a NaN propagates (fmax would drop it)
  }
  if (resid) {
    __syncthreads();
    red[0][tid] = rmax;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (tid < st) {
        const double o = red[0][tid + st];
        if (o > red[0][tid] || o != o) red[0][tid] = o;
      }
      __syncthreads();
    }
    if (tid == 0) resid[(int64_t)j * gridDim.y + blockIdx.y] = red[0][0];
  }
}

// Compute units of the current device (cached per device).
static int64_t device_cus() {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int c = cache[dev].load(std::memory_order_relaxed);
  if (c <= 0) {
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0) c = 256;
    cache[dev].store(c, std::memory_order_relaxed);
  }
  return c;
}

// Vector groups for the many-vector kernels: enough workgroups to fill the chip
// (about `want` of them over `per_group` workgroups per group).
static void vector_groups(int nvec, int64_t per_group, int64_t want, int* VG, int* nvg) {
  int g = (int)std::max<int64_t>(1, std::min<int64_t>(nvec, (want + per_group - 1) / per_group));
  *VG = (nvec + g - 1) / g;
  *nvg = (nvec + *VG - 1) / *VG;
}
//: batch sizes from which the many-vector operator and moment kernels take over
constexpr int kBatchMin = 8;

template <class R>
static void moments_t(hipStream_t st, const cv<R>* x, int64_t n, int nvec, int Ny, int Nxi, int r,
                      const R* M, cv<R>* mom, const int* skip) {
  const int S = moment_splits(Ny, nvec, Nxi, sizeof(R) == 4 ? 1 : 0);
  {
    const int per = (2 * Nxi + S - 1) / S;
    if (nvec >= kBatchMin && !skip && per <= 3 * 256) {
      // about 4,096 workgroups (M = 4 shape, 128 FP32 vectors: 370 against
      // 388 us for the whole operator with 2,048; no change beyond)
      int VG, nvg;
      vector_groups(nvec, (int64_t)Ny * S, 4096, &VG, &nvg);
      const dim3 g(Ny * S, nvg);
      if (per <= 256)
        hipLaunchKernelGGL((k_moments_batch<R, 1>), g, dim3(256), 0, st, x, n, Ny, Nxi, r, M, mom, S, nvec, VG);
      else if (per <= 512)
        hipLaunchKernelGGL((k_moments_batch<R, 2>), g, dim3(256), 0, st, x, n, Ny, Nxi, r, M, mom, S, nvec, VG);
      else
        hipLaunchKernelGGL((k_moments_batch<R, 3>), g, dim3(256), 0, st, x, n, Ny, Nxi, r, M, mom, S, nvec, VG);
      return;
    }
  }
  if (nvec > 1)
    hipLaunchKernelGGL((k_moments<R>), dim3(Ny * S * nvec), dim3(256), 0, st, x, n, Ny, Nxi, r, M, mom, S, skip,
                       nvec);
  else
    hipLaunchKernelGGL((k_moments<R>), dim3(Ny * S, nvec), dim3(256), 0, st, x, n, Ny, Nxi, r, M, mom, S, skip, 0);
}
void launch_moments(hipStream_t st, const double2* x, int64_t n, int nvec, int Ny, int Nxi, int r,
                    const double* M, double2* mom, const int* skip) {
  moments_t<double>(st, x, n, nvec, Ny, Nxi, r, M, mom, skip);
}
void launch_moments(hipStream_t st, const float2* x, int64_t n, int nvec, int Ny, int Nxi, int r,
                    const float* M, float2* mom, const int* skip) {
  moments_t<float>(st, x, n, nvec, Ny, Nxi, r, M, mom, skip);
}

// FP32 operator (the mixed-precision inner solve).  Default: the FP32 matrix-
// core kernel, row tiles per wavefront chosen for >= ~1024 wavefronts and 4
// wavefronts per workgroup when there are enough of them.  The launch table can
// select other tilings of it (apply_waves 1 or 4) or the scalar kernel with 4,
// 8 or 16 rows per thread (apply_waves 0); each gives its own FP32 rounding.
static void apply_f32(hipStream_t st, const float2* x, float2* y, int64_t n, int nvec, int Ny, int Nxi, int r,
                      double tre, double tim, double beta, const float* DxT, const float* xix, const float* xiy,
                      const float* nu, const float* U, float2* mom, const int* skip) {
  const int nc = 2 * Nxi;
  const int cblocks = (nc + 255) / 256;
  const int S = moment_splits(Ny, nvec, Nxi, 1);
  Tuning tn;
  const bool tuned = tune_get(Ny, Nxi, nvec, 1, &tn);
  if (tuned && tn.apply_nw == 0 && (tn.apply_rt == 4 || tn.apply_rt == 8 || tn.apply_rt == 16)) {
    if (tn.apply_rt == 16)
      hipLaunchKernelGGL((k_apply<float, 16>), dim3(cblocks, (Ny + 15) / 16, nvec), dim3(256), 0, st, x, y, n, Ny,
                         Nxi, r, (float)tre, (float)tim, (float)beta, DxT, xix, xiy, nu, U, mom, S, skip);
    else if (tn.apply_rt == 8)
      hipLaunchKernelGGL((k_apply<float, 8>), dim3(cblocks, (Ny + 7) / 8, nvec), dim3(256), 0, st, x, y, n, Ny,
                         Nxi, r, (float)tre, (float)tim, (float)beta, DxT, xix, xiy, nu, U, mom, S, skip);
    else
      hipLaunchKernelGGL((k_apply<float, 4>), dim3(cblocks, (Ny + 3) / 4, nvec), dim3(256), 0, st, x, y, n, Ny,
                         Nxi, r, (float)tre, (float)tim, (float)beta, DxT, xix, xiy, nu, U, mom, S, skip);
    return;
  }
  const int ctiles = (nc + 15) / 16, nrt = (Ny + 15) / 16;
  // many vectors: the streaming kernel, as for FP64 (the moment totals after the
  // partials: mom holds nvec Ny r 9 entries)
  const bool off32 = (uint64_t)n * sizeof(float2) < ((uint64_t)1 << 32) &&
                     (uint64_t)Ny * 2 * r * Nxi * sizeof(float) < ((uint64_t)1 << 32);
  const int64_t sgroups = (ctiles + 7) / 8;
  const bool stream_fits = sgroups >= 4 && sgroups * nvec >= device_cus() / 2;
  if (nvec >= kBatchMin && !skip && nrt <= 6 && off32 && (r == 3 || r == 4) &&
      (tuned ? (tn.apply_nw == 8 || (tn.apply_nw == 0 && stream_fits)) : stream_fits)) {
    constexpr int WPG = 8;
    float2* tot = mom + (size_t)nvec * Ny * r * 8;
    const int64_t ntot = (int64_t)nvec * Ny * r;
    hipLaunchKernelGGL(k_mom_total<float>, dim3(nblk(ntot, 256)), dim3(256), 0, st, mom, tot, ntot, r, S);
    const int64_t items = sgroups * nvec;
    const int64_t slots = device_cus();
    const int per = (int)std::max<int64_t>(1, (items + slots - 1) / slots);
    const int nwg = (int)((items + per - 1) / per);
#define KLST_MS32(NRT_)                                                                                      \
  do {                                                                                                       \
    if (r == 4)                                                                                              \
      hipLaunchKernelGGL((k_apply_stream<float, NRT_, WPG, 4>), dim3(nwg), dim3(64 * WPG), 0, st, x, y, n, Ny, \
                         Nxi, (float)tre, (float)tim, (float)beta, DxT, xix, xiy, nu, U, tot, nvec, items, per); \
    else                                                                                                     \
      hipLaunchKernelGGL((k_apply_stream<float, NRT_, WPG, 3>), dim3(nwg), dim3(64 * WPG), 0, st, x, y, n, Ny, \
                         Nxi, (float)tre, (float)tim, (float)beta, DxT, xix, xiy, nu, U, tot, nvec, items, per); \
  } while (0)
    switch (nrt) {
      case 1: KLST_MS32(1); break;
      case 2: KLST_MS32(2); break;
      case 3: KLST_MS32(3); break;
      case 4: KLST_MS32(4); break;
      case 5: KLST_MS32(5); break;
      default: KLST_MS32(6); break;
    }
#undef KLST_MS32
    return;
  }
  int rt = 6;
  while (rt > 1 && (int64_t)ctiles * ((nrt + rt - 1) / rt) * nvec < 1024) rt = (rt == 6) ? 3 : (rt == 3 ? 2 : 1);
  // many vectors on the tiled kernel: at most two row tiles per wavefront (M = 4
  // shape, 128 vectors: 345 us against 405 us with six)
  if (nvec >= kBatchMin) rt = std::min(rt, 2);
  bool wide = (int64_t)((ctiles + 3) / 4) * ((nrt + rt - 1) / rt) * nvec >= 512;
  if (tuned && (tn.apply_nw == 1 || tn.apply_nw == 4) &&
      (tn.apply_rt == 1 || tn.apply_rt == 2 || tn.apply_rt == 3 || tn.apply_rt == 6)) {
    rt = tn.apply_rt;
    wide = tn.apply_nw == 4;
  }
  wide = wide && (size_t)((Ny + 3) & ~3) * rt * 16 * sizeof(float) <= 96 * 1024;
  const size_t lds = (size_t)rt * 16 * 4 * sizeof(float2) + (wide ? (size_t)((Ny + 3) & ~3) * rt * 16 * sizeof(float) : 0);
  const int gx = wide ? (ctiles + 3) / 4 : ctiles, gy = (nrt + rt - 1) / rt;
  const dim3 g((unsigned)((int64_t)gx * gy * nvec));
#define KLST_M32(RT_, NW_) hipLaunchKernelGGL((k_apply_mfma32<RT_, NW_>), g, dim3(64 * NW_), lds, st, x, y, n, Ny, \
                                              Nxi, r, (float)tre, (float)tim, (float)beta, DxT, xix, xiy, nu, U, \
                                              mom, S, skip, gx, gy)
  if (wide) {
    if (rt == 6) KLST_M32(6, 4); else if (rt == 3) KLST_M32(3, 4); else if (rt == 2) KLST_M32(2, 4); else KLST_M32(1, 4);
  } else {
    if (rt == 6) KLST_M32(6, 1); else if (rt == 3) KLST_M32(3, 1); else if (rt == 2) KLST_M32(2, 1); else KLST_M32(1, 1);
  }
#undef KLST_M32
}
void launch_apply(hipStream_t st, const double2* x, double2* y, int64_t n, int nvec, int Ny, int Nxi,
                  int r, double tre, double tim, double beta, const double* Dx, const double* xix,
                  const double* xiy, const double* nu, const double* U, double2* mom,
                  const int* skip) {
  // FP64: streaming GEMM on the matrix cores.  Large launches use workgroups of
  // 4 wavefronts sharing an LDS copy of their D_x row slice; small ones use one
  // wavefront per workgroup (more workgroups, D_x from L2).  Row tiles per
  // workgroup are chosen for >= ~1024 wavefronts when the problem allows it.
  const int nc = 2 * Nxi;
  const int ctiles = (nc + 15) / 16, nrt = (Ny + 15) / 16;
  const int S = moment_splits(Ny, nvec, Nxi, 0);
  Tuning tq;
  const bool tq_ok = tune_get(Ny, Nxi, nvec, 0, &tq);
  // the streaming kernel addresses each vector and the U table with 32-bit byte offsets
  const bool off32 = (uint64_t)n * sizeof(double2) < ((uint64_t)1 << 32) &&
                     (uint64_t)Ny * 2 * r * Nxi * sizeof(double) < ((uint64_t)1 << 32);
  // the streaming kernel needs enough column groups to spread items over the CUs
  // (at 12 column tiles, 2 groups, the tiled kernel is faster at 64 vectors)
  const int64_t sgroups = (ctiles + 7) / 8;
  const bool stream_fits = sgroups >= 4 && sgroups * nvec >= device_cus() / 2;
  if (nvec >= kBatchMin && !skip && nrt <= 6 && off32 && (r == 3 || r == 4) &&
      (tq_ok ? (tq.apply_nw == 8 || (tq.apply_nw == 0 && stream_fits)) : stream_fits)) {
    constexpr int WPG = 8;
    // moment totals after the partials (mom holds nvec Ny r 9 entries)
    double2* tot = mom + (size_t)nvec * Ny * r * 8;
    const int64_t ntot = (int64_t)nvec * Ny * r;
    hipLaunchKernelGGL(k_mom_total<double>, dim3(nblk(ntot, 256)), dim3(256), 0, st, mom, tot, ntot, r, S);
    const int64_t groups = (ctiles + WPG - 1) / WPG;
    const int64_t items = groups * nvec;
    const int64_t slots = device_cus();                  // one 8-wavefront workgroup per CU
    const int per = (int)std::max<int64_t>(1, (items + slots - 1) / slots);
    const int nwg = (int)((items + per - 1) / per);
#define KLST_MS(NRT_)                                                                                        \
  do {                                                                                                       \
    if (r == 4)                                                                                              \
      hipLaunchKernelGGL((k_apply_stream<double, NRT_, WPG, 4>), dim3(nwg), dim3(64 * WPG), 0, st, x, y, n, Ny, Nxi, \
                         tre, tim, beta, Dx, xix, xiy, nu, U, tot, nvec, items, per);                        \
    else                                                                                                     \
      hipLaunchKernelGGL((k_apply_stream<double, NRT_, WPG, 3>), dim3(nwg), dim3(64 * WPG), 0, st, x, y, n, Ny, Nxi, \
                         tre, tim, beta, Dx, xix, xiy, nu, U, tot, nvec, items, per);                        \
  } while (0)
    switch (nrt) {
      case 1: KLST_MS(1); break;
      case 2: KLST_MS(2); break;
      case 3: KLST_MS(3); break;
      case 4: KLST_MS(4); break;
      case 5: KLST_MS(5); break;
      default: KLST_MS(6); break;
    }
#undef KLST_MS
    return;
  }
  int rt = 6;
  while (rt > 1 && (int64_t)ctiles * ((nrt + rt - 1) / rt) * nvec < 1024) rt = (rt == 6) ? 3 : (rt == 3 ? 2 : 1);
  // a single vector takes 4 wavefronts per workgroup sharing the D_x slice from
  // LDS once it has 4 column tiles (M = 4 shape: 22.4 against 23.7 us per
  // moments + operator; the tuned launch tables of the sweep shapes pick it too)
  bool wide = (int64_t)((ctiles + 3) / 4) * ((nrt + rt - 1) / rt) * nvec >= 512 || (nvec == 1 && ctiles >= 4);
  // tuned row tiles and waves per workgroup (every output entry is accumulated
  // in the same order whatever the tiling, so the choice does not change results)
  Tuning tn;
  if (tune_get(Ny, Nxi, nvec, 0, &tn)) {
    if (tn.apply_rt == 1 || tn.apply_rt == 2 || tn.apply_rt == 3 || tn.apply_rt == 6) rt = tn.apply_rt;
    if (tn.apply_nw == 1 || tn.apply_nw == 4) wide = (tn.apply_nw == 4);
  }
  wide = wide && (size_t)((Ny + 3) & ~3) * rt * 16 * sizeof(double) <= 96 * 1024;
  const size_t lds_m = (size_t)rt * 16 * 4 * sizeof(double2);
  const size_t lds = lds_m + (wide ? (size_t)((Ny + 3) & ~3) * rt * 16 * sizeof(double) : 0);
  const int gx = wide ? (ctiles + 3) / 4 : ctiles, gy = (nrt + rt - 1) / rt;
  const dim3 g(gx * gy * nvec);
  const int vmaj = nvec > 1 ? nvec : 0;
#define KLST_MF(RT_, NW_) hipLaunchKernelGGL((k_apply_mfma<RT_, NW_>), g, dim3(64 * NW_), lds, st, x, y, n, Ny, \
                                             Nxi, r, tre, tim, beta, Dx, xix, xiy, nu, U, mom, S, skip, gx, gy, vmaj)
  if (wide) {
    if (rt == 6) KLST_MF(6, 4); else if (rt == 3) KLST_MF(3, 4); else if (rt == 2) KLST_MF(2, 4); else KLST_MF(1, 4);
  } else {
    if (rt == 6) KLST_MF(6, 1); else if (rt == 3) KLST_MF(3, 1); else if (rt == 2) KLST_MF(2, 1); else KLST_MF(1, 1);
  }
#undef KLST_MF
}
void launch_apply(hipStream_t st, const float2* x, float2* y, int64_t n, int nvec, int Ny, int Nxi,
                  int r, double tre, double tim, double beta, const float* Dx, const float* xix,
                  const float* xiy, const float* nu, const float* U, float2* mom,
                  const int* skip) {
  apply_f32(st, x, y, n, nvec, Ny, Nxi, r, tre, tim, beta, Dx, xix, xiy, nu, U, mom, skip);
}

void launch_csr_build(hipStream_t st, int64_t* rowptr, int32_t* col, double2* val, int Ny, int Nxi,
                      int r, double beta, const double* Dx, const double* xix, const double* xiy,
                      const double* nu, const double* U, const double* M, int npos, int nneg) {
  const int64_t n = 2LL * Ny * Nxi;
  hipLaunchKernelGGL(k_csr_rowptr, dim3(nblk(n, 256)), dim3(256), 0, st, rowptr, Ny, Nxi, xix, npos, nneg);
  hipLaunchKernelGGL(k_csr_fill, dim3(nblk(n * 64, 256)), dim3(256), 0, st, rowptr, col, val, Ny, Nxi, r,
                     beta, Dx, xix, xiy, nu, U, M);
}

void launch_csr_spmv(hipStream_t st, const int64_t* rowptr, const int32_t* col, const double2* val,
                     const double2* x, double2* y, int64_t n, int Ny, int Nxi, const double* xix,
                     double tre, double tim, const int* skip) {
  hipLaunchKernelGGL(k_csr_spmv, dim3(nblk(n * 64, 256)), dim3(256), 0, st, rowptr, col, val, x, y, n,
                     Ny, Nxi, xix, tre, tim, skip);
}

void launch_ilu_apply(hipStream_t st, const double2* x, double2* y, int Ny, int Nxi, int nl,
                      int nblocks, const double2* Fc, const double2* C, const int* skip) {
  const size_t lds = (size_t)nl * Ny * sizeof(double2);
  const dim3 blk(64 * nl);
  if (Ny <= 64)
    hipLaunchKernelGGL((k_ilu_apply<1, 4>), dim3(nblocks), blk, lds, st, x, y, Ny, Nxi, nl, Fc, C, skip);
  else if (Ny <= 128)
    hipLaunchKernelGGL((k_ilu_apply<2, 3>), dim3(nblocks), blk, lds, st, x, y, Ny, Nxi, nl, Fc, C, skip);
  else
    hipLaunchKernelGGL((k_ilu_apply<4, 2>), dim3(nblocks), blk, lds, st, x, y, Ny, Nxi, nl, Fc, C, skip);
}

// Wavefronts per workgroup for the block GEMVs: enough loads in flight when the
// grid alone cannot fill the 256 CUs (few or small blocks).
static int gemv_waves(int64_t workgroups) {
  return workgroups >= 1024 ? 4 : (workgroups >= 512 ? 8 : 16);
}

template <class R>
static void blockinv_t(hipStream_t st, const cv<R>* x, cv<R>* y, int Ny, int Nxi, int nl, int nblocks,
                       const cv<R>* Kinv, const int64_t* koff, const int* skip) {
  const int nb = nl * Ny;
  const dim3 grid((nb + 63) / 64, nblocks);
  int nw = gemv_waves((int64_t)grid.x * grid.y);
  Tuning tn;
  if (tune_get(Ny, Nxi, 1, sizeof(R) == 4 ? 1 : 0, &tn) && (tn.gemv == 4 || tn.gemv == 8 || tn.gemv == 16)) nw = tn.gemv;
  const size_t lds = (size_t)(nb + 64 * nw) * sizeof(cv<R>);
  if (nw == 4)
    hipLaunchKernelGGL((k_blockinv_apply<R, 4>), grid, dim3(256), lds, st, x, y, Ny, Nxi, nl, Kinv, koff, skip);
  else if (nw == 8)
    hipLaunchKernelGGL((k_blockinv_apply<R, 8>), grid, dim3(512), lds, st, x, y, Ny, Nxi, nl, Kinv, koff, skip);
  else
    hipLaunchKernelGGL((k_blockinv_apply<R, 16>), grid, dim3(1024), lds, st, x, y, Ny, Nxi, nl, Kinv, koff,
                       skip);
}
void launch_blockinv_apply(hipStream_t st, const double2* x, double2* y, int Ny, int Nxi, int nl,
                           int nblocks, const double2* Kinv, const int64_t* koff, const int* skip) {
  blockinv_t<double>(st, x, y, Ny, Nxi, nl, nblocks, Kinv, koff, skip);
}
void launch_blockinv_apply(hipStream_t st, const float2* x, float2* y, int Ny, int Nxi, int nl,
                           int nblocks, const float2* Kinv, const int64_t* koff, const int* skip) {
  blockinv_t<float>(st, x, y, Ny, Nxi, nl, nblocks, Kinv, koff, skip);
}

// One pass y = P^{-1} (x + Ut d) over all stored line inverses (d == nullptr:
// y = P^{-1} x).
template <class R>
static void line_pass_t(hipStream_t st, const cv<R>* x, cv<R>* y, int Ny, int Nxi, int r, const cv<R>* Pinv,
                        const int* slot_node, const int* slot_mate, int nslots, const R* U, const R* xix,
                        const cv<R>* dd, const int* skip) {
  const dim3 grid((Ny + 63) / 64, nslots);
  // slots that serve a mirrored node apply their inverse to 4 columns; the LDS
  // then holds 4 Ny inputs and 4 x NW x 64 partial sums, which caps NW at 8
  const int cmax = nslots < Nxi ? 4 : 2;
  int nw = gemv_waves((int64_t)grid.x * grid.y);
  Tuning tn;
  if (tune_get(Ny, Nxi, 1, sizeof(R) == 4 ? 1 : 0, &tn) && (tn.gemv == 4 || tn.gemv == 8 || tn.gemv == 16)) nw = tn.gemv;
  if (cmax == 4 && nw > 8) nw = 8;
  const size_t lds = (size_t)(cmax * Ny + cmax * 64 * nw) * sizeof(cv<R>);
#define KLST_LI(NW_, P_) hipLaunchKernelGGL((k_line_inverse<R, NW_, P_>), grid, dim3(64 * NW_), lds, st, x, y, Ny, \
                                            Nxi, r, Pinv, slot_node, slot_mate, cmax, U, xix, dd, skip)
  if (cmax == 4) {
    if (nw == 4) KLST_LI(4, true); else KLST_LI(8, true);
  } else {
    if (nw == 4) KLST_LI(4, false); else if (nw == 8) KLST_LI(8, false); else KLST_LI(16, false);
  }
#undef KLST_LI
}

template <class R>
static void structured_t(hipStream_t st, const cv<R>* x, cv<R>* y, int Ny, int Nxi, int r,
                         const cv<R>* Pinv, const int* slot_node, const int* slot_mate, int nslots,
                         const cv<R>* Sinv, const R* M, const R* U, const R* xix, cv<R>* mom, cv<R>* d,
                         const int* skip) {
  line_pass_t<R>(st, x, y, Ny, Nxi, r, Pinv, slot_node, slot_mate, nslots, U, xix, nullptr, skip);
  const int64_t n = 2LL * Ny * Nxi;
  moments_t<R>(st, y, n, 1, Ny, Nxi, r, M, mom, skip);
  const int Rd = r * Ny;
  const int S = moment_splits(Ny, 1, Nxi, sizeof(R) == 4 ? 1 : 0);
  hipLaunchKernelGGL((k_capacitance<R>), dim3((Rd + 3) / 4), dim3(256), (size_t)Rd * sizeof(cv<R>), st, mom,
                     Ny, r, S, Sinv, d, skip);
  line_pass_t<R>(st, x, y, Ny, Nxi, r, Pinv, slot_node, slot_mate, nslots, U, xix, d, skip);
}
void launch_structured_setup(hipStream_t st, double2* Pinv, double2* Sinv, double2* part, int Ny, int Nxi, int r,
                             const int* slot_node, int nslots, const int* slot_of, const int* conj_of,
                             const double* Dx, const double* xix, const double* xiy, const double* nu,
                             const double* U, const double* M, double beta, double sre, double sim,
                             int* status) {
  const size_t lds_line = (size_t)Ny * (2 * sizeof(double2) + sizeof(int));
  if (Ny <= kLdsLineMax)
    hipLaunchKernelGGL(k_line_blocks_invert_lds, dim3(nslots), dim3(256), 0, st, Pinv, Ny, slot_node, Dx, xix, xiy,
                       nu, beta, sre, sim, status + 1);
  else
    hipLaunchKernelGGL(k_line_blocks_invert, dim3(nslots), dim3(256), lds_line, st, Pinv, Ny, slot_node, Dx, xix,
                       xiy, nu, beta, sre, sim, status + 1);
  const int Rd = r * Ny;
  hipLaunchKernelGGL(k_cap_partial, dim3(Ny, kCapParts), dim3(128), 0, st, Pinv, Ny, Nxi, r, slot_of, conj_of, M,
                     U, xix, part);
  hipLaunchKernelGGL(k_cap_finish, dim3(nblk((int64_t)Rd * Rd, 256)), dim3(256), 0, st, part, kCapParts, Rd,
                     Sinv);
  // the capacitance is assembled into part (free again after k_cap_finish has
  // read it) and inverted by one Gauss-Jordan step per launch, ping-ponging
  // between part and Sinv; piv sits after the two matrices in part
  const int64_t RR = (int64_t)Rd * Rd;
  double2* bufA = Sinv;
  double2* bufB = part;
  int* piv = reinterpret_cast<int*>(part + RR);
  const unsigned rows = (unsigned)((Rd + 3) / 4);
  for (int c = 0; c < Rd; ++c) {
    hipLaunchKernelGGL(k_gj_step, dim3(rows), dim3(256), 0, st, bufA, bufB, Rd, c, piv, status);
    std::swap(bufA, bufB);
  }
  // the final iterate is in bufA; undo the interchanges into Sinv
  if (bufA == Sinv) {
    hipLaunchKernelGGL(k_gj_unpermute, dim3(rows), dim3(256), (size_t)Rd * sizeof(int), st, Sinv, part, Rd, piv);
    hipMemcpyAsync(Sinv, part, sizeof(double2) * RR, hipMemcpyDeviceToDevice, st);
  } else {
    hipLaunchKernelGGL(k_gj_unpermute, dim3(rows), dim3(256), (size_t)Rd * sizeof(int), st, part, Sinv, Rd, piv);
  }
}
void launch_line_inverse(hipStream_t st, const double2* x, double2* y, int Ny, int Nxi, int r,
                         const double2* Pinv, const int* slot_node, const int* slot_mate, int nslots,
                         const double* U, const double* xix) {
  line_pass_t<double>(st, x, y, Ny, Nxi, r, Pinv, slot_node, slot_mate, nslots, U, xix, nullptr, nullptr);
}
void launch_structured_inverse(hipStream_t st, const double2* x, double2* y, int Ny, int Nxi, int r,
                               const double2* Pinv, const int* slot_node, const int* slot_mate, int nslots,
                               const double2* Sinv, const double* M, const double* U, const double* xix,
                               double2* mom, double2* d, const int* skip) {
  structured_t<double>(st, x, y, Ny, Nxi, r, Pinv, slot_node, slot_mate, nslots, Sinv, M, U, xix, mom, d, skip);
}
void launch_structured_inverse(hipStream_t st, const float2* x, float2* y, int Ny, int Nxi, int r,
                               const float2* Pinv, const int* slot_node, const int* slot_mate, int nslots,
                               const float2* Sinv, const float* M, const float* U, const float* xix,
                               float2* mom, float2* d, const int* skip) {
  structured_t<float>(st, x, y, Ny, Nxi, r, Pinv, slot_node, slot_mate, nslots, Sinv, M, U, xix, mom, d, skip);
}

// Chunking for k_dot_partial: about 2048 wavefronts in total, at least 256
// entries per chunk, at most 512 chunks.
int partial_chunks(int64_t n, int mtot, int* chunk) {
  int64_t want = std::max<int64_t>(1, 2048 / std::max(1, mtot));
  want = std::min<int64_t>(want, 512);
  int64_t c = std::max<int64_t>(256, (n + want - 1) / want);
  c = (c + 63) / 64 * 64;
  while ((n + c - 1) / c > 512) c += 64;
  *chunk = (int)c;
  return (int)((n + c - 1) / c);
}

template <class R, class RS = R>
static int dot_partial_t(hipStream_t st, const cv<RS>* s0, int m0, const cv<RS>* s1, int m1, const cv<R>* x,
                         int64_t n, double2* partial, int with_norm, const int* skip) {
  const int mtot = m0 + m1 + (with_norm ? 1 : 0);
  int chunk;
  const int nch = partial_chunks(n, mtot, &chunk);
  if (mtot > 0)
    hipLaunchKernelGGL((k_dot_partial<R, RS>), dim3(nch * ((mtot + 3) / 4)), dim3(256), 0, st, s0, m0, s1, m1, x,
                       n, chunk, partial, with_norm, skip);
  return nch;
}
int launch_dot_partial(hipStream_t st, const double2* s0, int m0, const double2* s1, int m1,
                       const double2* x, int64_t n, double2* partial, int with_norm, const int* skip) {
  return dot_partial_t<double>(st, s0, m0, s1, m1, x, n, partial, with_norm, skip);
}
int launch_dot_partial(hipStream_t st, const float2* s0, int m0, const float2* s1, int m1,
                       const float2* x, int64_t n, double2* partial, int with_norm, const int* skip) {
  return dot_partial_t<float>(st, s0, m0, s1, m1, x, n, partial, with_norm, skip);
}
int launch_dot_partial(hipStream_t st, const float2* s0, int m0, const float2* s1, int m1,
                       const double2* x, int64_t n, double2* partial, int with_norm, const int* skip) {
  return dot_partial_t<double, float>(st, s0, m0, s1, m1, x, n, partial, with_norm, skip);
}
// Dynamic LDS for staging the dot partials in the consumer kernels: used when
// they fit in 16 KB (mtot x nch <= 1024), which keeps 6 workgroups per CU for
// the streaming part of k_subm_fused.
static size_t partial_stage_bytes(int mtot, int nch) {
  const int64_t tot = (int64_t)mtot * nch;
  return (tot > 0 && tot <= 1024) ? (size_t)tot * sizeof(double2) : 0;
}
void launch_dot_reduce(hipStream_t st, const double2* partial, int m, int nch, double2* out, int mode,
                       const double2* Hinv, double2* out2, const int* skip) {
  const size_t lds = partial_stage_bytes(mode == 3 ? m + 1 : m, nch);
  hipLaunchKernelGGL(k_dot_reduce, dim3(1), dim3(256), lds, st, partial, m, nch, out, mode, Hinv, out2,
                     lds > 0 ? 1 : 0, skip);
}
template <class R, class RS = R>
static void subm_fused_t(hipStream_t st, const cv<RS>* s0, int m0, const cv<RS>* s1, int m1,
                         const double2* partial, int nch, const double2* Hinv, double2* coef_set,
                         double2* coef_add, cv<R>* x, int64_t n, double2* norm_part, const int* skip) {
  const size_t lds = partial_stage_bytes(m0 + m1, nch);
  hipLaunchKernelGGL((k_subm_fused<R, RS>), dim3(nblk(n, 256)), dim3(256), lds, st, s0, m0, s1, m1, partial, nch,
                     Hinv, coef_set, coef_add, x, n, norm_part, lds > 0 ? 1 : 0, skip);
}
void launch_subm_fused(hipStream_t st, const double2* s0, int m0, const double2* s1, int m1,
                       const double2* partial, int nch, const double2* Hinv, double2* coef_set,
                       double2* coef_add, double2* x, int64_t n, double2* norm_part, const int* skip) {
  subm_fused_t<double>(st, s0, m0, s1, m1, partial, nch, Hinv, coef_set, coef_add, x, n, norm_part, skip);
}
void launch_subm_fused(hipStream_t st, const float2* s0, int m0, const float2* s1, int m1,
                       const double2* partial, int nch, const double2* Hinv, double2* coef_set,
                       double2* coef_add, float2* x, int64_t n, double2* norm_part, const int* skip) {
  subm_fused_t<float>(st, s0, m0, s1, m1, partial, nch, Hinv, coef_set, coef_add, x, n, norm_part, skip);
}
void launch_subm_fused(hipStream_t st, const float2* s0, int m0, const float2* s1, int m1,
                       const double2* partial, int nch, const double2* Hinv, double2* coef_set,
                       double2* coef_add, double2* x, int64_t n, double2* norm_part, const int* skip) {
  subm_fused_t<double, float>(st, s0, m0, s1, m1, partial, nch, Hinv, coef_set, coef_add, x, n, norm_part, skip);
}

template <class R, class R2 = R>
static void scale_norm_t(hipStream_t st, cv<R>* x, cv<R>* dst, cv<R2>* dst2, int64_t n, const double2* norm_part,
                         double2* nrm2_out, double2* H, int ldh, int j, double* cs, double2* sn, double2* g,
                         int* done, int* steps, const double* beta, double rtol) {
  hipLaunchKernelGGL((k_scale_norm<R, R2>), dim3(nblk(n, 256)), dim3(256), 0, st, x, dst, dst2, n, norm_part,
                     (int)nblk(n, 256), nrm2_out, H, ldh, j, cs, sn, g, done, steps, beta, rtol);
}
void launch_scale_norm(hipStream_t st, double2* x, double2* dst, int64_t n, const double2* norm_part,
                       double2* nrm2_out, double2* H, int ldh, int j, double* cs, double2* sn, double2* g,
                       int* done, int* steps, const double* beta, double rtol) {
  scale_norm_t<double>(st, x, dst, (double2*)nullptr, n, norm_part, nrm2_out, H, ldh, j, cs, sn, g, done, steps,
                       beta, rtol);
}
void launch_scale_norm(hipStream_t st, double2* x, float2* dst32, int64_t n, const double2* norm_part,
                       double2* nrm2_out, double2* H, int ldh, int j, double* cs, double2* sn, double2* g,
                       int* done, int* steps, const double* beta, double rtol) {
  scale_norm_t<double, float>(st, x, (double2*)nullptr, dst32, n, norm_part, nrm2_out, H, ldh, j, cs, sn, g, done,
                              steps, beta, rtol);
}
void launch_scale_norm(hipStream_t st, float2* x, float2* dst, int64_t n, const double2* norm_part,
                       double2* nrm2_out, double2* H, int ldh, int j, double* cs, double2* sn, double2* g,
                       int* done, int* steps, const double* beta, double rtol) {
  scale_norm_t<float>(st, x, dst, (float2*)nullptr, n, norm_part, nrm2_out, H, ldh, j, cs, sn, g, done, steps,
                      beta, rtol);
}

void launch_subm(hipStream_t st, const double2* s0, int m0, const double2* s1, int m1,
                 const double2* c, double2* x, double2* dst, int64_t n, double sign, const int* skip) {
  hipLaunchKernelGGL((k_subm<double>), dim3(nblk(n, 256)), dim3(256), 0, st, s0, m0, s1, m1, c, x, dst, n,
                     sign, skip);
}
void launch_subm(hipStream_t st, const float2* s0, int m0, const float2* s1, int m1,
                 const double2* c, float2* x, float2* dst, int64_t n, double sign, const int* skip) {
  hipLaunchKernelGGL((k_subm<float>), dim3(nblk(n, 256)), dim3(256), 0, st, s0, m0, s1, m1, c, x, dst, n,
                     (float)sign, skip);
}

void launch_combine(hipStream_t st, const double2* S, int m, int64_t n, const double2* coef, int ldc,
                    int k, double2* out, const int* count) {
  if (k >= 2)
    hipLaunchKernelGGL((k_combine_multi<double, 8>), dim3(nblk(n, 256) * ((k + 7) / 8)), dim3(256), 0, st, S, m, n,
                       coef, ldc, k, out, count);
  else
    hipLaunchKernelGGL((k_combine<double>), dim3(nblk(n, 256), k), dim3(256), 0, st, S, m, n, coef, ldc, out,
                       count);
}
void launch_combine(hipStream_t st, const float2* S, int m, int64_t n, const double2* coef, int ldc,
                    int k, float2* out, const int* count) {
  hipLaunchKernelGGL((k_combine<float>), dim3(nblk(n, 256), k), dim3(256), 0, st, S, m, n, coef, ldc, out,
                     count);
}
void launch_combine(hipStream_t st, const float2* S, int m, int64_t n, const double2* coef, int ldc,
                    int k, double2* out, const int* count) {
  hipLaunchKernelGGL((k_combine<double, float>), dim3(nblk(n, 256), k), dim3(256), 0, st, S, m, n, coef, ldc, out,
                     count);
}

void launch_scale_rsqrt(hipStream_t st, double2* x, double2* dst, int64_t n, const double2* nrm2,
                        const int* skip, float2* dst32) {
  hipLaunchKernelGGL((k_scale_rsqrt<double>), dim3(nblk(n, 256)), dim3(256), 0, st, x, dst, dst32, n, nrm2,
                     skip);
}
void launch_scale_rsqrt(hipStream_t st, float2* x, float2* dst, int64_t n, const double2* nrm2,
                        const int* skip) {
  hipLaunchKernelGGL((k_scale_rsqrt<float>), dim3(nblk(n, 256)), dim3(256), 0, st, x, dst, (float2*)nullptr, n,
                     nrm2, skip);
}

void launch_axpby(hipStream_t st, const double2* x, double2* y, int64_t n, double are, double aim,
                  int accum) {
  hipLaunchKernelGGL((k_axpby<double>), dim3(nblk(n, 256)), dim3(256), 0, st, x, y, n, are, aim, accum);
}
void launch_axpby(hipStream_t st, const float2* x, float2* y, int64_t n, double are, double aim,
                  int accum) {
  hipLaunchKernelGGL((k_axpby<float>), dim3(nblk(n, 256)), dim3(256), 0, st, x, y, n, (float)are,
                     (float)aim, accum);
}

void launch_mirror_conj(hipStream_t st, const double2* x, double2* out, int64_t n, int nvec, int Nxi,
                        const int* mk) {
  hipLaunchKernelGGL(k_mirror_conj, dim3(nblk(n, 256), nvec), dim3(256), 0, st, x, out, n, Nxi, mk);
}
void launch_narrow(hipStream_t st, const double2* x, float2* y, int64_t n) {
  hipLaunchKernelGGL(k_narrow, dim3(nblk(n, 256)), dim3(256), 0, st, x, y, n);
}
void launch_widen(hipStream_t st, const float2* x, double2* y, int64_t n, int accum) {
  hipLaunchKernelGGL(k_widen, dim3(nblk(n, 256)), dim3(256), 0, st, x, y, n, accum);
}

void launch_reorth_test(hipStream_t st, const double2* partial, int m, int nch, int64_t n,
                        const double2* norm_part, double eta2, const int* done, int* skip_out) {
  hipLaunchKernelGGL(k_reorth_test, dim3(1), dim3(256), 0, st, partial, m, nch, norm_part, (int)nblk(n, 256),
                     eta2, done, skip_out);
}

void launch_gmres_init(hipStream_t st, const double2* nrm2, double2* g, int* done, int* steps,
                       double* beta, int first) {
  hipLaunchKernelGGL(k_gmres_init, dim3(1), dim3(1), 0, st, nrm2, g, done, steps, beta, first);
}

void launch_gmres_solve(hipStream_t st, const double2* H, int ldh, const double2* g, const int* steps,
                        double2* yk) {
  hipLaunchKernelGGL(k_gmres_solve, dim3(1), dim3(1), 0, st, H, ldh, g, steps, yk);
}

void launch_mask_bc(hipStream_t st, const double2* x, double2* y, int64_t n, int Ny, int Nxi,
                    const double* xix) {
  hipLaunchKernelGGL(k_mask_bc, dim3(nblk(n, 256)), dim3(256), 0, st, x, y, n, Ny, Nxi, xix);
}

void launch_set_int(hipStream_t st, int* p, int v) {
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, st, p, v);
}

void launch_perturbation_macros(hipStream_t st, const double2* x, int64_t n, int nvec, int Ny, int Nxi, int r,
                                const double* M, double2* mom, const double* base, double2* macros,
                                double* umag) {
  const int S = moment_splits(Ny, nvec, Nxi, 0);
  hipLaunchKernelGGL((k_moments<double>), dim3(Ny * S, nvec), dim3(256), 0, st, x, n, Ny, Nxi, r, M, mom, S,
                     nullptr, 0);
  hipLaunchKernelGGL(k_pert_macros, dim3(nvec), dim3(256), 0, st, mom, Ny, r, S, base, macros, umag);
}

void launch_noneq_level(hipStream_t st, const double* gc, const double* base, const double* xix,
                        const double* xiy, const double* w, int Ny, int Nxi, int Dv, double* eneq) {
  hipLaunchKernelGGL(k_noneq_level, dim3(Ny), dim3(256), 0, st, gc, base, xix, xiy, w, Nxi, Dv, eneq);
}

int bgk_parts(int Nxi) { return std::max(1, std::min(32, (2 * Nxi + 255) / 256)); }

void launch_bgk_stage(hipStream_t st, const double* q, const double* kprev, double a, double* kout, double* acc,
                      double* qout, double dt6, int stage, int Ny, int Nxi, int Dv, const double* xix,
                      const double* xiy, const double* w, const double* inv_dx, double nu_inf, double s_visc,
                      double* resid) {
  hipLaunchKernelGGL(k_bgk_stage, dim3(Ny, bgk_parts(Nxi)), dim3(256), 0, st, q, kprev, a, kout, acc, qout, dt6,
                     stage, Ny, Nxi, Dv, xix, xiy, w, inv_dx, nu_inf, s_visc, resid);
}

}  // namespace dev
}  // namespace klst
