// Host-side problem tables, block-Jacobi ILU(0) set-up and small dense
// complex linear algebra.  See host.hpp.
#include "host.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <thread>

namespace klst {

namespace {

bool finite_all(const double* a, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

}  // namespace

// Grid: Chebyshev-Gauss-Lobatto nodes y_i = cos(i pi / N) (eq. ChebPoints), the
// derivative matrix of eqs. ChebOffDiag / ChebDiag / ChebBC, and the algebraic map
// x = L y / sqrt(1 + s - y^2), dy/dx = sqrt(1+s) L^2 / (L^2 + x^2)^{3/2}
// (eq. Chebmapping), giving D_x = diag(dy/dx) D_y.
//
// Operator coefficients: linearisation of the discrete BGK relaxation
// nu(m) (f^e(m) - f) about the base state (eq. CompBGKtilde), in units where
// 2RT -> T and P = rho T / 2, with macros a = (rho, u, v, E) and
// T = (4/3)(E - (u^2 + v^2)/2):
//   g^e = rho / (pi T)^{Dv/2} exp(-|xi - u e_x|^2 / T),  h^e = ((3 - Dv)/2) T g^e,
//   G_a = nu (dg^e/da + (g^e - g_c) dln(nu)/da),  H_a likewise with h,
// and the perturbation moments of the discrete rows (eq. comp_ghat1Dshock):
//   m_rho = sum W g, m_u = sum W (xi_x - u) g / rho, m_v = sum W xi_y g / rho,
//   m_E = sum W ((|xi|^2 - 2E) g + h) / (2 rho).
void mapped_nodes(int Ny, double L, double s_inf, double* x) {
  const int N = Ny - 1;
  const double pi = 3.14159265358979323846;
  const double s = (L / s_inf) * (L / s_inf);
  for (int i = 0; i < Ny; ++i) {
    const double y = std::cos(pi * i / N);
    x[i] = L * y / std::sqrt(1.0 + s - y * y);
  }
}

bool mirror_nodes(const std::vector<double>& xi_x, const std::vector<double>& xi_y, std::vector<int>& mk) {
  const int Nxi = (int)xi_x.size();
  std::map<std::pair<double, double>, int> where;
  for (int k = 0; k < Nxi; ++k) where[{xi_x[k], xi_y[k]}] = k;
  mk.assign(Nxi, -1);
  for (int k = 0; k < Nxi; ++k) {
    auto it = where.find({xi_x[k], -xi_y[k]});
    if (it == where.end()) { mk.clear(); return false; }
    mk[k] = it->second;
  }
  return true;
}

std::string build_problem(const klst_grid* g, const klst_vel* v, const klst_base* b,
                          double beta, Problem& p) {
  if (!g || !v || !b) return "null grid, velocity table or base flow";
  if (g->Ny < 3) return "Ny must be >= 3";
  if (v->Nxi < 1) return "Nxi must be >= 1";
  if (v->Dv != 1 && v->Dv != 2) return "Dv must be 1 or 2";
  if (!v->xi_x || !v->xi_y || !v->w) return "velocity table pointers must be non-null";
  if (!(g->L > 0) || !(g->s_inf > 0) || !std::isfinite(g->L) || !std::isfinite(g->s_inf))
    return "L and s_inf must be finite and > 0";
  if (!std::isfinite(beta) || !std::isfinite(b->s_visc) || !std::isfinite(b->nu_inf) ||
      b->nu_inf < 0)
    return "beta, s_visc, nu_inf must be finite (nu_inf >= 0)";
  const int Ny = g->Ny, Nxi = v->Nxi, Dv = v->Dv;
  const int r = (Dv == 2) ? 4 : 3;
  if (!finite_all(v->xi_x, Nxi) || !finite_all(v->xi_y, Nxi) || !finite_all(v->w, Nxi))
    return "non-finite velocity table";
  for (int k = 0; k < Nxi; ++k) {
    if (!(v->w[k] > 0)) return "velocity weights must be > 0";
    if (Dv == 1 && v->xi_y[k] != 0.0) return "Dv = 1 requires xi_y == 0";
  }
  p = Problem();
  p.Ny = Ny; p.Nxi = Nxi; p.r = r; p.Dv = Dv;
  p.beta = beta; p.L = g->L; p.s_inf = g->s_inf; p.s_visc = b->s_visc; p.nu_inf = b->nu_inf;
  p.xi_x.assign(v->xi_x, v->xi_x + Nxi);
  p.xi_y.assign(v->xi_y, v->xi_y + Nxi);
  p.w.assign(v->w, v->w + Nxi);

  // --- grid and mapped derivative
  const int N = Ny - 1;
  const double pi = 3.14159265358979323846;
  std::vector<double> y(Ny), x(Ny), dydx(Ny);
  const double s = (g->L / g->s_inf) * (g->L / g->s_inf);
  for (int i = 0; i < Ny; ++i) {
    y[i] = std::cos(pi * i / N);
    x[i] = g->L * y[i] / std::sqrt(1.0 + s - y[i] * y[i]);
    const double q = g->L * g->L + x[i] * x[i];
    dydx[i] = std::sqrt(1.0 + s) * g->L * g->L / (q * std::sqrt(q));
  }
  p.Dx.assign((size_t)Ny * Ny, 0.0);
  for (int j = 0; j < Ny; ++j) {
    const double cj = (j == 0 || j == N) ? 2.0 : 1.0;
    for (int m = 0; m < Ny; ++m) {
      double d;
      if (j != m) {
        const double cm = (m == 0 || m == N) ? 2.0 : 1.0;
        const double sgn = ((j + m) % 2 == 0) ? 1.0 : -1.0;
        d = cj / cm * sgn / (y[j] - y[m]);
      } else if (j == 0) {
        d = (2.0 * N * N + 1.0) / 6.0;
      } else if (j == N) {
        d = -(2.0 * N * N + 1.0) / 6.0;
      } else {
        d = -y[j] / (2.0 * (1.0 - y[j] * y[j]));
      }
      p.Dx[(size_t)j * Ny + m] = dydx[j] * d;
    }
  }

  // --- base macros and VDFs
  p.rho.resize(Ny); p.u.resize(Ny); p.E.resize(Ny); p.T.resize(Ny); p.nu.resize(Ny);
  std::vector<double> ge((size_t)Ny * Nxi), he((size_t)Ny * Nxi), gc((size_t)Ny * Nxi),
      hc((size_t)Ny * Nxi);
  const double hfac = 0.5 * (3 - Dv);
  auto maxwell = [&](int j) {
    const double T = p.T[j], rho = p.rho[j], u = p.u[j];
    const double pre = rho / std::pow(pi * T, 0.5 * Dv);
    for (int k = 0; k < Nxi; ++k) {
      const double cx = p.xi_x[k] - u, cy = p.xi_y[k];
      const double gv = pre * std::exp(-(cx * cx + cy * cy) / T);
      ge[(size_t)j * Nxi + k] = gv;
      he[(size_t)j * Nxi + k] = hfac * T * gv;
    }
  };
  if (b->mode == 0) {
    if (!b->rho || !b->u || !b->T) return "EQ base flow needs rho, u, T";
    if (!finite_all(b->rho, Ny) || !finite_all(b->u, Ny) || !finite_all(b->T, Ny))
      return "non-finite base macros";
    for (int j = 0; j < Ny; ++j) {
      p.rho[j] = b->rho[j]; p.u[j] = b->u[j]; p.T[j] = b->T[j];
      if (!(p.rho[j] > 0) || !(p.T[j] > 0)) return "base rho and T must be > 0";
      p.E[j] = 0.5 * p.u[j] * p.u[j] + 0.75 * p.T[j];
      maxwell(j);
    }
    gc = ge; hc = he;
  } else if (b->mode == 1) {
    if (!b->g_c || !b->h_c) return "NONEQ base flow needs g_c, h_c";
    if (!finite_all(b->g_c, (size_t)Ny * Nxi) || !finite_all(b->h_c, (size_t)Ny * Nxi))
      return "non-finite base VDF";
    gc.assign(b->g_c, b->g_c + (size_t)Ny * Nxi);
    hc.assign(b->h_c, b->h_c + (size_t)Ny * Nxi);
    p.gc = gc;
    for (int j = 0; j < Ny; ++j) {
      double m0 = 0, m1 = 0, m2 = 0;
      for (int k = 0; k < Nxi; ++k) {
        const double gv = gc[(size_t)j * Nxi + k], hv = hc[(size_t)j * Nxi + k];
        const double xx = p.xi_x[k], yy = p.xi_y[k];
        m0 += p.w[k] * gv;
        m1 += p.w[k] * xx * gv;
        m2 += p.w[k] * ((xx * xx + yy * yy) * gv + hv);
      }
      if (!(m0 > 0)) return "base density must be > 0";
      p.rho[j] = m0;
      p.u[j] = m1 / m0;
      p.E[j] = 0.5 * m2 / m0;
      p.T[j] = (4.0 / 3.0) * (p.E[j] - 0.5 * p.u[j] * p.u[j]);
      if (!(p.T[j] > 0)) return "base temperature must be > 0";
      maxwell(j);
    }
  } else {
    return "base mode must be 0 (EQ) or 1 (NONEQ)";
  }
  for (int j = 0; j < Ny; ++j) p.nu[j] = b->nu_inf * p.rho[j] * std::pow(p.T[j], 1.0 - b->s_visc);

  // --- coefficients U[j][f][a][k] and functionals M[j][a][f][k]
  p.U.assign((size_t)Ny * 2 * r * Nxi, 0.0);
  p.M.assign((size_t)Ny * r * 2 * Nxi, 0.0);
  const double sv = b->s_visc;
  for (int j = 0; j < Ny; ++j) {
    const double rho = p.rho[j], u = p.u[j], T = p.T[j], E = p.E[j], nu = p.nu[j];
    // d T / d a for a = rho, u, v, E at v = 0
    const double dT[4] = {0.0, -4.0 * u / 3.0, 0.0, 4.0 / 3.0};
    // d ln(nu) / d a = d ln P / d a - d ln mu / d a, nu = P / mu, P = rho T / 2, mu ~ T^s
    const double dlnu[4] = {1.0 / rho, (1.0 - sv) * dT[1] / T, 0.0, (1.0 - sv) * dT[3] / T};
    const int amap3[3] = {0, 1, 3};   // Dv = 1: (rho, u, E)
    for (int k = 0; k < Nxi; ++k) {
      const size_t jk = (size_t)j * Nxi + k;
      const double gev = ge[jk], hev = he[jk];
      const double cx = p.xi_x[k] - u, cy = p.xi_y[k];
      const double c2 = cx * cx + cy * cy;
      const double dlng_dT = c2 / (T * T) - 0.5 * Dv / T;
      double dg[4];
      dg[0] = gev / rho;
      dg[1] = gev * (2.0 * cx / T + dlng_dT * dT[1]);
      dg[2] = gev * (2.0 * cy / T);
      dg[3] = gev * dlng_dT * dT[3];
      for (int ia = 0; ia < r; ++ia) {
        const int a = (r == 4) ? ia : amap3[ia];
        const double dh = hfac * (T * dg[a] + gev * dT[a]);
        p.U[(((size_t)j * 2 + 0) * r + ia) * Nxi + k] = nu * (dg[a] + (gev - gc[jk]) * dlnu[a]);
        p.U[(((size_t)j * 2 + 1) * r + ia) * Nxi + k] = nu * (dh + (hev - hc[jk]) * dlnu[a]);
        double mg = 0, mh = 0;
        switch (a) {
          case 0: mg = p.w[k]; break;
          case 1: mg = p.w[k] * cx / rho; break;
          case 2: mg = p.w[k] * p.xi_y[k] / rho; break;
          default:
            mg = p.w[k] * (p.xi_x[k] * p.xi_x[k] + p.xi_y[k] * p.xi_y[k] - 2.0 * E) / (2.0 * rho);
            mh = p.w[k] / (2.0 * rho);
        }
        p.M[(((size_t)j * r + ia) * 2 + 0) * Nxi + k] = mg;
        p.M[(((size_t)j * r + ia) * 2 + 1) * Nxi + k] = mh;
      }
    }
  }
  // --- inflow rows: x = -s_inf (j = N) with xi_x > 0, x = +s_inf (j = 0) with xi_x < 0
  p.bc.assign((size_t)Ny * 2 * Nxi, 0);
  p.n_bc = 0;
  for (int f = 0; f < 2; ++f)
    for (int k = 0; k < Nxi; ++k) {
      if (p.xi_x[k] > 0) { p.bc[((size_t)N * 2 + f) * Nxi + k] = 1; ++p.n_bc; }
      if (p.xi_x[k] < 0) { p.bc[((size_t)0 * 2 + f) * Nxi + k] = 1; ++p.n_bc; }
    }
  return std::string();
}

// ILU(0) of one block of whole velocity lines, rows ordered (line, node).  The
// pattern of a non-inflow row (l, j) is {(l, m): all m} (streaming along the
// line, D_x is dense) and {(l2, j): all block lines l2} (moment coupling at node
// j); an inflow row holds its diagonal only.  Eliminating in column order, the
// coupling columns (l2 < l, j) come first and only update the coupling entries
// and the diagonal of row (l, j); the line columns (l, m < j) then update the
// line part, and the fill they would create in (l2, m) is dropped.
static void ilu0_block(const Problem& p, cd sigma, int b, int nl_blk, int nl, ILU0& f,
                       std::vector<double>& rownorm, int& floored) {
  const int Ny = p.Ny, Nxi = p.Nxi, r = p.r;
  const int l0 = b * nl;
  auto line_fk = [&](int lg, int& fo, int& ko) { fo = lg / Nxi; ko = lg % Nxi; };
  auto coupling = [&](int j, int fa, int ka, int fb, int kb) {
    double s = 0;
    for (int a = 0; a < r; ++a)
      s += p.U[(((size_t)j * 2 + fa) * r + a) * Nxi + ka] * p.M[(((size_t)j * r + a) * 2 + fb) * Nxi + kb];
    return s;
  };
  for (int l = 0; l < nl_blk; ++l) {
    int fl, kl;
    line_fk(l0 + l, fl, kl);
    cd* F = &f.F[(size_t)(l0 + l) * Ny * Ny];
    cd* Cl = &f.C[(((size_t)b * nl + l) * nl) * Ny];   // Cl[l2 * Ny + j]
    // initial values
    for (int j = 0; j < Ny; ++j) {
      const bool bcr = p.is_bc(j, kl);
      for (int m = 0; m < Ny; ++m) F[(size_t)j * Ny + m] = 0.0;
      for (int l2 = 0; l2 < nl; ++l2) Cl[(size_t)l2 * Ny + j] = 0.0;
      if (bcr) { F[(size_t)j * Ny + j] = 1.0; rownorm[j] = 1.0; continue; }
      const double xi = p.xi_x[kl];
      double nrm = 0;
      for (int m = 0; m < Ny; ++m) F[(size_t)j * Ny + m] = xi * p.Dx[(size_t)j * Ny + m];
      F[(size_t)j * Ny + j] += cd(p.nu[j], p.beta * p.xi_y[kl]) - sigma - coupling(j, fl, kl, fl, kl);
      for (int m = 0; m < Ny; ++m) nrm += std::abs(F[(size_t)j * Ny + m]);
      for (int l2 = 0; l2 < nl_blk; ++l2) {
        if (l2 == l) continue;
        int f2, k2;
        line_fk(l0 + l2, f2, k2);
        Cl[(size_t)l2 * Ny + j] = -coupling(j, fl, kl, f2, k2);
        nrm += std::abs(Cl[(size_t)l2 * Ny + j]);
      }
      // the row also couples to block-external lines; count them in the norm
      for (int lg = 0; lg < 2 * Nxi; ++lg) {
        if (lg >= l0 && lg < l0 + nl_blk) continue;
        int f2, k2;
        line_fk(lg, f2, k2);
        nrm += std::abs(coupling(j, fl, kl, f2, k2));
      }
      rownorm[j] = nrm;
    }
    for (int j = 0; j < Ny; ++j) {
      if (p.is_bc(j, kl)) continue;
      cd* Fj = F + (size_t)j * Ny;
      // coupling columns (l2, j), l2 < l
      for (int l2 = 0; l2 < l; ++l2) {
        int f2, k2;
        line_fk(l0 + l2, f2, k2);
        const bool bc2 = p.is_bc(j, k2);
        const cd piv = bc2 ? cd(1.0) : f.F[((size_t)(l0 + l2) * Ny + j) * Ny + j];
        const cd lc = Cl[(size_t)l2 * Ny + j] / piv;
        Cl[(size_t)l2 * Ny + j] = lc;
        if (bc2) continue;   // an inflow row has no entries right of its diagonal
        const cd* C2 = &f.C[(((size_t)b * nl + l2) * nl) * Ny];
        for (int l3 = l2 + 1; l3 < nl_blk; ++l3) {
          if (l3 == l) Fj[j] -= lc * C2[(size_t)l3 * Ny + j];
          else Cl[(size_t)l3 * Ny + j] -= lc * C2[(size_t)l3 * Ny + j];
        }
      }
      // line columns (l, m), m < j
      for (int m = 0; m < j; ++m) {
        if (p.is_bc(m, kl)) continue;   // row m is e_m: L entry stays, no update
        const cd lm = Fj[m] / F[(size_t)m * Ny + m];
        Fj[m] = lm;
        const cd* Fm = F + (size_t)m * Ny;
        for (int q = m + 1; q < Ny; ++q) Fj[q] -= lm * Fm[q];
      }
      // pivot floor: |u_jj| >= 1e-12 x the row's 1-norm in A - sigma B
      const double fl_abs = 1e-12 * rownorm[j];
      const double a = std::abs(Fj[j]);
      if (a < fl_abs) {
        Fj[j] = (a > 0) ? Fj[j] * (fl_abs / a) : cd(fl_abs);
        ++floored;
      }
    }
  }
}

void build_ilu0(const Problem& p, cd sigma, int lines_per_block, ILU0& f, int nthreads) {
  const int nlines = 2 * p.Nxi;
  const int nl = std::max(1, std::min(lines_per_block, nlines));
  f.nl = nl;
  f.Ny = p.Ny;
  f.nlines = nlines;
  f.nblocks = (nlines + nl - 1) / nl;
  f.F.assign((size_t)nlines * p.Ny * p.Ny, cd(0.0));
  f.C.assign((size_t)f.nblocks * nl * nl * p.Ny, cd(0.0));
  nthreads = std::max(1, std::min(nthreads, f.nblocks));
  std::vector<int> floored(nthreads, 0);
  auto work = [&](int t) {
    std::vector<double> rownorm(p.Ny);
    for (int b = t; b < f.nblocks; b += nthreads) {
      const int nb = std::min(nl, nlines - b * nl);
      ilu0_block(p, sigma, b, nb, nl, f, rownorm, floored[t]);
    }
  };
  if (nthreads == 1) {
    work(0);
  } else {
    std::vector<std::thread> th;
    for (int t = 0; t < nthreads; ++t) th.emplace_back(work, t);
    for (auto& x : th) x.join();
  }
  f.floored = 0;
  for (int v : floored) f.floored += v;
}

void build_block_inverse(const ILU0& f, std::vector<cd>& Kinv, std::vector<int64_t>& off,
                         int nthreads) {
  const int Ny = f.Ny, nl = f.nl;
  off.assign(f.nblocks + 1, 0);
  for (int b = 0; b < f.nblocks; ++b) {
    const int nb = std::min(nl, f.nlines - b * nl) * Ny;
    off[b + 1] = off[b] + (int64_t)nb * nb;
  }
  Kinv.assign(off[f.nblocks], cd(0.0));
  auto work = [&](int t) {
    std::vector<cd> L, U, col;
    for (int b = t; b < f.nblocks; b += nthreads) {
      const int nlb = std::min(nl, f.nlines - b * nl);
      const int nb = nlb * Ny;
      L.assign((size_t)nb * nb, cd(0.0));
      U.assign((size_t)nb * nb, cd(0.0));
      for (int l = 0; l < nlb; ++l) {
        const cd* F = &f.F[(size_t)(b * nl + l) * Ny * Ny];
        const cd* Cl = &f.C[(((size_t)b * nl + l) * nl) * Ny];
        for (int j = 0; j < Ny; ++j) {
          const size_t r = (size_t)(l * Ny + j) * nb;
          for (int m = 0; m < Ny; ++m) {
            if (m < j) L[r + l * Ny + m] = F[(size_t)j * Ny + m];
            else U[r + l * Ny + m] = F[(size_t)j * Ny + m];
          }
          L[r + l * Ny + j] = 1.0;
          for (int l2 = 0; l2 < nlb; ++l2) {
            if (l2 < l) L[r + l2 * Ny + j] = Cl[(size_t)l2 * Ny + j];
            else if (l2 > l) U[r + l2 * Ny + j] = Cl[(size_t)l2 * Ny + j];
          }
        }
      }
      cd* K = &Kinv[off[b]];
      col.resize(nb);
      for (int c = 0; c < nb; ++c) {
        for (int i = 0; i < nb; ++i) col[i] = (i == c) ? cd(1.0) : cd(0.0);
        for (int i = 0; i < nb; ++i) {               // L z = e_c
          cd acc = col[i];
          const cd* Li = &L[(size_t)i * nb];
          for (int q = c; q < i; ++q) acc -= Li[q] * col[q];
          col[i] = acc;
        }
        for (int i = nb - 1; i >= 0; --i) {          // U w = z
          cd acc = col[i];
          const cd* Ui = &U[(size_t)i * nb];
          for (int q = i + 1; q < nb; ++q) acc -= Ui[q] * col[q];
          col[i] = acc / Ui[i];
        }
        for (int i = 0; i < nb; ++i) K[(size_t)c * nb + i] = col[i];
      }
    }
  };
  nthreads = std::max(1, std::min(nthreads, f.nblocks));
  if (nthreads == 1) {
    work(0);
  } else {
    std::vector<std::thread> th;
    for (int t = 0; t < nthreads; ++t) th.emplace_back(work, t);
    for (auto& x : th) x.join();
  }
}

// ---------------------------------------------------------------- dense ----

namespace {

// Givens rotation (c real, s complex) with [c s; -conj(s) c] [f; g] = [r; 0].
void givens(cd f, cd g, double& c, cd& s) {
  // squared moduli and sqrt instead of hypot: the projected problems hold values
  // far from the over/underflow range
  const double f2 = std::norm(f), g2 = std::norm(g);
  if (g2 == 0.0) { c = 1.0; s = 0.0; return; }
  if (f2 == 0.0) { c = 0.0; s = std::conj(g) / std::sqrt(g2); return; }
  const double af = std::sqrt(f2), nrm = std::sqrt(f2 + g2);
  c = af / nrm;
  s = (f / af) * std::conj(g) / nrm;
}

}  // namespace

void qr_square(int m, const cd* A, cd* Qm, cd* Rm) {
  std::vector<cd> R(A, A + (size_t)m * m), Q((size_t)m * m, cd(0.0));
  for (int i = 0; i < m; ++i) Q[(size_t)i * m + i] = 1.0;
  std::vector<cd> v(m);
  for (int k = 0; k < m - 1; ++k) {
    double nrm = 0;
    for (int i = k; i < m; ++i) nrm += std::norm(R[(size_t)i * m + k]);
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) continue;
    const cd x0 = R[(size_t)k * m + k];
    const cd ph = (std::abs(x0) > 0) ? x0 / std::abs(x0) : cd(1.0);
    const cd alpha = -ph * nrm;
    for (int i = k; i < m; ++i) v[i] = R[(size_t)i * m + k];
    v[k] -= alpha;
    double vn = 0;
    for (int i = k; i < m; ++i) vn += std::norm(v[i]);
    if (vn == 0.0) continue;
    // R <- (I - 2 v v^H / v^H v) R ; Q <- Q (I - 2 v v^H / v^H v)
    for (int jc = 0; jc < m; ++jc) {
      cd s = 0;
      for (int i = k; i < m; ++i) s += std::conj(v[i]) * R[(size_t)i * m + jc];
      s *= 2.0 / vn;
      for (int i = k; i < m; ++i) R[(size_t)i * m + jc] -= s * v[i];
    }
    for (int ir = 0; ir < m; ++ir) {
      cd s = 0;
      for (int i = k; i < m; ++i) s += Q[(size_t)ir * m + i] * v[i];
      s *= 2.0 / vn;
      for (int i = k; i < m; ++i) Q[(size_t)ir * m + i] -= s * std::conj(v[i]);
    }
  }
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < i; ++j) R[(size_t)i * m + j] = 0.0;
  std::copy(Q.begin(), Q.end(), Qm);
  std::copy(R.begin(), R.end(), Rm);
}

// Complex Schur form by Householder reduction to Hessenberg form followed by
// single-shift QR iterations with Wilkinson shifts and Givens rotations
// (Golub & Van Loan, Matrix Computations, Sec. 7.4-7.5), then a selection sort
// of the diagonal by adjacent swaps of 1x1 blocks (the exchange of Bai & Demmel
// used by LAPACK's ZTREXC).
static inline double cabs1(cd z) { return std::fabs(z.real()) + std::fabs(z.imag()); }

bool sorted_schur(int m, const cd* G, cd* Uo, cd* To, int nsort) {
  // H row-major (row operations contiguous); the Schur vectors are kept
  // column-major in Uc so that rotating two columns is contiguous.
  std::vector<cd> H(G, G + (size_t)m * m), Uc((size_t)m * m, cd(0.0));
  for (int i = 0; i < m; ++i) Uc[(size_t)i * m + i] = 1.0;
  auto h = [&](int i, int j) -> cd& { return H[(size_t)i * m + j]; };
  auto ucol = [&](int j) -> cd* { return &Uc[(size_t)j * m]; };
  auto rot_cols = [&](int k, double cs, cd sn) {   // U[:, k], U[:, k+1] <- (x, y) G^H
    cd* x = ucol(k);
    cd* y = ucol(k + 1);
    const cd snc = std::conj(sn);
    for (int ir = 0; ir < m; ++ir) {
      const cd a = x[ir], b = y[ir];
      x[ir] = cs * a + snc * b;
      y[ir] = -sn * a + cs * b;
    }
  };
  // Hessenberg reduction by Householder reflectors P = I - 2 v v^H / (v^H v)
  std::vector<cd> v(m), t(m);
  for (int k = 0; k < m - 2; ++k) {
    double nrm = 0;
    for (int i = k + 1; i < m; ++i) nrm += std::norm(h(i, k));
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) continue;
    const cd x0 = h(k + 1, k);
    const cd ph = (std::abs(x0) > 0) ? x0 / std::abs(x0) : cd(1.0);
    const cd alpha = -ph * nrm;
    for (int i = k + 1; i < m; ++i) v[i] = h(i, k);
    v[k + 1] -= alpha;
    double vn = 0;
    for (int i = k + 1; i < m; ++i) vn += std::norm(v[i]);
    if (vn == 0.0) continue;
    const double f = 2.0 / vn;
    // H <- P H: t = v^H H (row vector), H -= v t
    std::fill(t.begin(), t.end(), cd(0.0));
    for (int i = k + 1; i < m; ++i) {
      const cd vc = std::conj(v[i]);
      const cd* hi = &h(i, 0);
      for (int jc = 0; jc < m; ++jc) t[jc] += vc * hi[jc];
    }
    for (int i = k + 1; i < m; ++i) {
      const cd vi = v[i] * f;
      cd* hi = &h(i, 0);
      for (int jc = 0; jc < m; ++jc) hi[jc] -= vi * t[jc];
    }
    // H <- H P (rows), U <- U P (columns of Uc)
    for (int ir = 0; ir < m; ++ir) {
      cd sum = 0;
      cd* hr = &h(ir, 0);
      for (int i = k + 1; i < m; ++i) sum += hr[i] * v[i];
      sum *= f;
      for (int i = k + 1; i < m; ++i) hr[i] -= sum * std::conj(v[i]);
    }
    std::fill(t.begin(), t.end(), cd(0.0));
    for (int i = k + 1; i < m; ++i) {
      const cd vi = v[i];
      const cd* ui = ucol(i);
      for (int ir = 0; ir < m; ++ir) t[ir] += ui[ir] * vi;
    }
    for (int i = k + 1; i < m; ++i) {
      const cd vc = std::conj(v[i]) * f;
      cd* ui = ucol(i);
      for (int ir = 0; ir < m; ++ir) ui[ir] -= t[ir] * vc;
    }
    for (int i = k + 2; i < m; ++i) h(i, k) = 0.0;
  }
  // QR iterations on the active window [lo, hi]
  const double eps = 2.220446049250313e-16;
  int hi = m - 1;
  int iter = 0, since = 0;
  while (hi > 0) {
    if (++iter > 100 * m + 1000) return false;
    int lo = hi;
    while (lo > 0) {
      // |re| + |im| as the magnitude in the deflation test (as LAPACK does)
      const double sub = cabs1(h(lo, lo - 1));
      double scale = cabs1(h(lo, lo)) + cabs1(h(lo - 1, lo - 1));
      if (scale == 0.0) scale = 1.0;
      if (sub <= eps * scale) { h(lo, lo - 1) = 0.0; break; }
      --lo;
    }
    if (lo == hi) { --hi; since = 0; continue; }
    ++since;
    // Wilkinson shift from the trailing 2x2 block; exceptional shift now and then
    cd mu;
    const cd a = h(hi - 1, hi - 1), bb = h(hi - 1, hi), c = h(hi, hi - 1), d = h(hi, hi);
    if (since % 11 == 10) {
      mu = d + cd(0.75 * std::abs(c), 0.0);
    } else {
      const cd tr = 0.5 * (a - d);
      const cd disc = std::sqrt(tr * tr + bb * c);
      const cd e1 = d - (bb * c) / (tr + disc), e2 = d - (bb * c) / (tr - disc);
      const bool ok1 = std::abs(tr + disc) > 0, ok2 = std::abs(tr - disc) > 0;
      if (ok1 && ok2) mu = (std::abs(e1 - d) < std::abs(e2 - d)) ? e1 : e2;
      else if (ok1) mu = e1;
      else if (ok2) mu = e2;
      else mu = d;
    }
    // implicit single-shift step via the explicit first rotation and chasing
    for (int k = lo; k < hi; ++k) {
      cd f0, g0;
      if (k == lo) { f0 = h(lo, lo) - mu; g0 = h(lo + 1, lo); }
      else { f0 = h(k, k - 1); g0 = h(k + 1, k - 1); }
      double cs; cd sn;
      givens(f0, g0, cs, sn);
      const cd snc = std::conj(sn);
      // rows k, k+1 from column (k == lo ? lo : k-1)
      cd* rk = &h(k, 0);
      cd* rk1 = &h(k + 1, 0);
      for (int jc = (k == lo ? lo : k - 1); jc < m; ++jc) {
        const cd x = rk[jc], y = rk1[jc];
        rk[jc] = cs * x + sn * y;
        rk1[jc] = -snc * x + cs * y;
      }
      if (k > lo) h(k + 1, k - 1) = 0.0;
      // columns k, k+1 of H rows 0..min(k+2, hi), and of U
      const int rmax = std::min(k + 2, hi);
      for (int ir = 0; ir <= rmax; ++ir) {
        const cd x = h(ir, k), y = h(ir, k + 1);
        h(ir, k) = cs * x + snc * y;
        h(ir, k + 1) = -sn * x + cs * y;
      }
      rot_cols(k, cs, sn);
    }
  }
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < i; ++j) h(i, j) = 0.0;
  // swap the 1x1 blocks at positions k, k+1 of the triangular T
  auto swap_adj = [&](int k) {
    const cd t11 = h(k, k), t22 = h(k + 1, k + 1);
    double cs; cd sn;
    givens(h(k, k + 1), t22 - t11, cs, sn);
    const cd snc = std::conj(sn);
    cd* rk = &h(k, 0);
    cd* rk1 = &h(k + 1, 0);
    for (int jc = k + 2; jc < m; ++jc) {       // rows k, k+1
      const cd x = rk[jc], y = rk1[jc];
      rk[jc] = cs * x + sn * y;
      rk1[jc] = -snc * x + cs * y;
    }
    for (int ir = 0; ir < k; ++ir) {           // columns k, k+1
      const cd x = h(ir, k), y = h(ir, k + 1);
      h(ir, k) = cs * x + snc * y;
      h(ir, k + 1) = -sn * x + cs * y;
    }
    h(k, k) = t22;
    h(k + 1, k + 1) = t11;
    rot_cols(k, cs, sn);
  };
  // selection by adjacent swaps: the largest |T_ii| into position 0, 1, ...,
  // for the first nsort positions (all when nsort <= 0 or >= m)
  const int npos = (nsort <= 0 || nsort >= m) ? m : nsort;
  for (int pos = 0; pos < npos; ++pos) {
    int best = pos;
    for (int i = pos + 1; i < m; ++i)
      if (std::norm(h(i, i)) > std::norm(h(best, best))) best = i;
    for (int k = best - 1; k >= pos; --k) swap_adj(k);
  }
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < i; ++j) h(i, j) = 0.0;
  std::copy(H.begin(), H.end(), To);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) Uo[(size_t)i * m + j] = Uc[(size_t)j * m + i];
  return true;
}

bool dominant_eig(int m, const cd* G, cd& mu, cd* x) {
  // Real and imaginary parts in separate row-major arrays, so that the row
  // sweeps of every step run over contiguous doubles; each complex product is
  // written out as (a c - b d, a d + b c), the formula of the complex type.
  const size_t mm = (size_t)m * m;
  std::vector<double> Hr(mm), Hi(mm);
  for (size_t q = 0; q < mm; ++q) { Hr[q] = G[q].real(); Hi[q] = G[q].imag(); }
  auto hr = [&](int i) { return &Hr[(size_t)i * m]; };
  auto hi_ = [&](int i) { return &Hi[(size_t)i * m]; };
  auto h = [&](int i, int j) { return cd(Hr[(size_t)i * m + j], Hi[(size_t)i * m + j]); };
  auto set = [&](int i, int j, cd z) { Hr[(size_t)i * m + j] = z.real(); Hi[(size_t)i * m + j] = z.imag(); };
  // Hessenberg reduction (similarity only: no transformation is kept)
  std::vector<double> vr(m), vi(m), tr(m), ti(m), wr(m), wi(m);
  for (int k = 0; k < m - 2; ++k) {
    double nrm = 0;
    for (int i = k + 1; i < m; ++i) nrm += std::norm(h(i, k));
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) continue;
    const cd x0 = h(k + 1, k);
    const cd ph = (std::abs(x0) > 0) ? x0 / std::abs(x0) : cd(1.0);
    for (int i = k + 1; i < m; ++i) { vr[i] = Hr[(size_t)i * m + k]; vi[i] = Hi[(size_t)i * m + k]; }
    {
      const cd v1 = cd(vr[k + 1], vi[k + 1]) + ph * nrm;
      vr[k + 1] = v1.real();
      vi[k + 1] = v1.imag();
    }
    double vn = 0;
    for (int i = k + 1; i < m; ++i) vn += std::norm(cd(vr[i], vi[i]));
    if (vn == 0.0) continue;
    const double f = 2.0 / vn;
    // H <- P H: t = v^H H over columns k.., H -= v t
    for (int jc = k; jc < m; ++jc) { tr[jc] = 0.0; ti[jc] = 0.0; }
    for (int i = k + 1; i < m; ++i) {
      const double a = vr[i], b = -vi[i];
      const double* r = hr(i);
      const double* s = hi_(i);
      for (int jc = k; jc < m; ++jc) {
        tr[jc] += a * r[jc] - b * s[jc];
        ti[jc] += a * s[jc] + b * r[jc];
      }
    }
    for (int i = k + 1; i < m; ++i) {
      const double a = vr[i] * f, b = vi[i] * f;
      double* r = hr(i);
      double* s = hi_(i);
      for (int jc = k; jc < m; ++jc) {
        r[jc] -= a * tr[jc] - b * ti[jc];
        s[jc] -= a * ti[jc] + b * tr[jc];
      }
    }
    // H <- H P (rows).  The row sums (H v)_ir, four rows at a time: four
    // independent chains, each summed in the same order as alone
    int ir = 0;
    for (; ir + 4 <= m; ir += 4) {
      double sr[4] = {0.0, 0.0, 0.0, 0.0}, si[4] = {0.0, 0.0, 0.0, 0.0};
      for (int i = k + 1; i < m; ++i) {
        const double a = vr[i], b = vi[i];
        for (int q = 0; q < 4; ++q) {
          const double xr = Hr[(size_t)(ir + q) * m + i], xi = Hi[(size_t)(ir + q) * m + i];
          sr[q] += xr * a - xi * b;
          si[q] += xr * b + xi * a;
        }
      }
      for (int q = 0; q < 4; ++q) { wr[ir + q] = sr[q] * f; wi[ir + q] = si[q] * f; }
    }
    for (; ir < m; ++ir) {
      const double* r = hr(ir);
      const double* s = hi_(ir);
      double sr = 0.0, si = 0.0;
      for (int i = k + 1; i < m; ++i) {
        sr += r[i] * vr[i] - s[i] * vi[i];
        si += r[i] * vi[i] + s[i] * vr[i];
      }
      wr[ir] = sr * f;
      wi[ir] = si * f;
    }
    for (ir = 0; ir < m; ++ir) {
      double* r = hr(ir);
      double* s = hi_(ir);
      const double sr = wr[ir], si = wi[ir];
      for (int i = k + 1; i < m; ++i) {
        // sum conj(v_i) = (sr vr + si vi, si vr - sr vi)
        r[i] -= sr * vr[i] - si * (-vi[i]);
        s[i] -= sr * (-vi[i]) + si * vr[i];
      }
    }
    for (int i = k + 2; i < m; ++i) { Hr[(size_t)i * m + k] = 0.0; Hi[(size_t)i * m + k] = 0.0; }
  }
  // eigenvalues only: single-shift QR restricted to the active window
  const double eps = 2.220446049250313e-16;
  int hi = m - 1, iter = 0, since = 0;
  while (hi > 0) {
    if (++iter > 100 * m + 1000) return false;
    int lo = hi;
    while (lo > 0) {
      // |re| + |im| as the magnitude in the deflation test (as LAPACK does)
      const double sub = cabs1(h(lo, lo - 1));
      double scale = cabs1(h(lo, lo)) + cabs1(h(lo - 1, lo - 1));
      if (scale == 0.0) scale = 1.0;
      if (sub <= eps * scale) { set(lo, lo - 1, 0.0); break; }
      --lo;
    }
    if (lo == hi) { --hi; since = 0; continue; }
    ++since;
    cd sh;
    const cd a = h(hi - 1, hi - 1), bb = h(hi - 1, hi), c = h(hi, hi - 1), d = h(hi, hi);
    if (since % 11 == 10) {
      sh = d + cd(0.75 * std::abs(c), 0.0);
    } else {
      const cd tr2 = 0.5 * (a - d);
      const cd disc = std::sqrt(tr2 * tr2 + bb * c);
      const cd e1 = d - (bb * c) / (tr2 + disc), e2 = d - (bb * c) / (tr2 - disc);
      const bool ok1 = std::abs(tr2 + disc) > 0, ok2 = std::abs(tr2 - disc) > 0;
      if (ok1 && ok2) sh = (std::abs(e1 - d) < std::abs(e2 - d)) ? e1 : e2;
      else if (ok1) sh = e1;
      else if (ok2) sh = e2;
      else sh = d;
    }
    for (int k = lo; k < hi; ++k) {
      cd f0, g0;
      if (k == lo) { f0 = h(lo, lo) - sh; g0 = h(lo + 1, lo); }
      else { f0 = h(k, k - 1); g0 = h(k + 1, k - 1); }
      double cs; cd sn;
      givens(f0, g0, cs, sn);
      const double snr = sn.real(), sni = sn.imag();
      // rows k, k+1: (cs x + sn y, -conj(sn) x + cs y)
      double* rk = hr(k);
      double* ik = hi_(k);
      double* rk1 = hr(k + 1);
      double* ik1 = hi_(k + 1);
      for (int jc = (k == lo ? lo : k - 1); jc <= hi; ++jc) {
        const double xr = rk[jc], xi = ik[jc], yr = rk1[jc], yi = ik1[jc];
        rk[jc] = cs * xr + (snr * yr - sni * yi);
        ik[jc] = cs * xi + (snr * yi + sni * yr);
        rk1[jc] = (-snr * xr - sni * xi) + cs * yr;
        ik1[jc] = (-snr * xi + sni * xr) + cs * yi;
      }
      if (k > lo) set(k + 1, k - 1, 0.0);
      // columns k, k+1: (cs x + conj(sn) y, -sn x + cs y)
      const int rmax = std::min(k + 2, hi);
      for (int ir = lo; ir <= rmax; ++ir) {
        double* r = hr(ir);
        double* s = hi_(ir);
        const double xr = r[k], xi = s[k], yr = r[k + 1], yi = s[k + 1];
        r[k] = cs * xr + (snr * yr - (-sni) * yi);
        s[k] = cs * xi + (snr * yi + (-sni) * yr);
        r[k + 1] = (-snr * xr - (-sni) * xi) + cs * yr;
        s[k + 1] = (-snr * xi + (-sni) * xr) + cs * yi;
      }
    }
  }
  int best = 0;
  for (int i = 1; i < m; ++i)
    if (std::norm(h(i, i)) > std::norm(h(best, best))) best = i;
  mu = h(best, best);
  // eigenvector by inverse iteration with G - mu I (LU, partial pivoting; an
  // exactly zero pivot is replaced by eps ||G||)
  double gn = 0;
  for (size_t q = 0; q < mm; ++q) gn = std::max(gn, std::abs(G[q]));
  std::vector<double> Lr(mm), Li(mm);
  for (size_t q = 0; q < mm; ++q) { Lr[q] = G[q].real(); Li[q] = G[q].imag(); }
  for (int i = 0; i < m; ++i) {
    const cd dd = cd(Lr[(size_t)i * m + i], Li[(size_t)i * m + i]) - mu;
    Lr[(size_t)i * m + i] = dd.real();
    Li[(size_t)i * m + i] = dd.imag();
  }
  auto L = [&](int i, int j) { return cd(Lr[(size_t)i * m + j], Li[(size_t)i * m + j]); };
  std::vector<int> piv(m);
  for (int k = 0; k < m; ++k) {
    int p = k;
    for (int i = k + 1; i < m; ++i)
      if (std::abs(L(i, k)) > std::abs(L(p, k))) p = i;
    piv[k] = p;
    if (p != k)
      for (int j = 0; j < m; ++j) {
        std::swap(Lr[(size_t)p * m + j], Lr[(size_t)k * m + j]);
        std::swap(Li[(size_t)p * m + j], Li[(size_t)k * m + j]);
      }
    cd pk = L(k, k);
    if (std::abs(pk) == 0.0) {
      pk = eps * std::max(gn, 1e-300);
      Lr[(size_t)k * m + k] = pk.real();
      Li[(size_t)k * m + k] = pk.imag();
    }
    const double* ur = &Lr[(size_t)k * m];
    const double* ui = &Li[(size_t)k * m];
    for (int i = k + 1; i < m; ++i) {
      const cd l = L(i, k) / pk;
      Lr[(size_t)i * m + k] = l.real();
      Li[(size_t)i * m + k] = l.imag();
      if (l == 0.0) continue;
      const double a = l.real(), b = l.imag();
      double* r = &Lr[(size_t)i * m];
      double* s = &Li[(size_t)i * m];
      for (int j = k + 1; j < m; ++j) {
        r[j] -= a * ur[j] - b * ui[j];
        s[j] -= a * ui[j] + b * ur[j];
      }
    }
  }
  std::vector<cd> y(m, cd(1.0));
  for (int it = 0; it < 2; ++it) {
    for (int k = 0; k < m; ++k) std::swap(y[k], y[piv[k]]);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < i; ++j) y[i] -= L(i, j) * y[j];
    for (int i = m - 1; i >= 0; --i) {
      for (int j = i + 1; j < m; ++j) y[i] -= L(i, j) * y[j];
      y[i] /= L(i, i);
    }
    double nn = 0;
    for (int i = 0; i < m; ++i) nn += std::norm(y[i]);
    nn = std::sqrt(nn);
    if (!(nn > 0) || !std::isfinite(nn)) return false;
    for (int i = 0; i < m; ++i) y[i] /= nn;
  }
  std::copy(y.begin(), y.end(), x);
  return true;
}

void structured_slots(const Problem& p, cd sigma, std::vector<int>& slot_node, std::vector<int>& slot_mate,
                      std::vector<int>& slot_of, std::vector<int>& conj_of) {
  const int Nxi = p.Nxi;
  slot_node.clear();
  slot_mate.clear();
  slot_of.assign(Nxi, -1);
  conj_of.assign(Nxi, 0);
  // a node and its xi_y mirror share one inverse when sigma is real
  std::map<std::pair<double, double>, int> where;
  for (int k = 0; k < Nxi; ++k) where[{p.xi_x[k], p.xi_y[k]}] = k;
  for (int k = 0; k < Nxi; ++k) {
    if (slot_of[k] >= 0) continue;
    int mate = -1;
    if (sigma.imag() == 0.0 && p.xi_y[k] != 0.0) {
      auto it = where.find({p.xi_x[k], -p.xi_y[k]});
      if (it != where.end() && it->second != k && slot_of[it->second] < 0) mate = it->second;
    }
    slot_of[k] = (int)slot_node.size();
    if (mate >= 0) { slot_of[mate] = slot_of[k]; conj_of[mate] = 1; }
    slot_node.push_back(k);
    slot_mate.push_back(mate);
  }
}

std::string build_structured_inverse(const Problem& p, cd sigma, StructuredInverse& si, int nthreads) {
  const int Ny = p.Ny, Nxi = p.Nxi, r = p.r, Rd = r * Ny;
  si.Ny = Ny;
  si.Nxi = Nxi;
  si.r = r;
  const size_t blk = (size_t)Ny * Ny;
  std::vector<int> slot_of, conj_of;
  structured_slots(p, sigma, si.slot_node, si.slot_mate, slot_of, conj_of);
  const int nslots = (int)si.slot_node.size();
  std::vector<cd> Prow((size_t)nslots * blk);   // row-major line inverses
  si.Pinv.assign((size_t)nslots * blk, cd(0.0));
  auto run = [&](int count, const std::function<void(int, int)>& work) {
    const int nt = std::max(1, std::min(nthreads, count));
    if (nt == 1) { work(0, 1); return; }
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) th.emplace_back(work, t, nt);
    for (auto& x : th) x.join();
  };
  std::vector<int> singular(nslots, 0);
  run(nslots, [&](int t, int nt) {
    std::vector<cd> a(blk);
    for (int sl = t; sl < nslots; sl += nt) {
      const int k = si.slot_node[sl];
      std::fill(a.begin(), a.end(), cd(0.0));
      for (int j = 0; j < Ny; ++j) {
        cd* aj = &a[(size_t)j * Ny];
        if (p.is_bc(j, k)) { aj[j] = 1.0; continue; }
        for (int m = 0; m < Ny; ++m) aj[m] = p.xi_x[k] * p.Dx[(size_t)j * Ny + m];
        aj[j] += cd(p.nu[j], p.beta * p.xi_y[k]) - sigma;
      }
      cd* inv = &Prow[(size_t)sl * blk];
      if (!invert(Ny, a.data(), inv)) { singular[sl] = 1; continue; }
      cd* col = &si.Pinv[(size_t)sl * blk];
      for (int j = 0; j < Ny; ++j)
        for (int m = 0; m < Ny; ++m) col[(size_t)m * Ny + j] = inv[(size_t)j * Ny + m];
    }
  });
  for (int sl = 0; sl < nslots; ++sl)
    if (singular[sl]) return "singular velocity-line block at node " + std::to_string(si.slot_node[sl]);
  // G = M P^{-1} Ut:  G[(j,a),(j',b)] = sum_k P_k^{-1}[j][j'] sum_f M_a(j,f,k) Ut_b(j',f,k).
  // Node-major copies of M and U keep the inner loops contiguous.
  std::vector<double> Mt((size_t)Nxi * Ny * 2 * r), Ut((size_t)Nxi * Ny * 2 * r, 0.0);
  for (int k = 0; k < Nxi; ++k)
    for (int j = 0; j < Ny; ++j)
      for (int f = 0; f < 2; ++f)
        for (int a = 0; a < r; ++a) {
          const size_t o = (((size_t)k * Ny + j) * 2 + f) * r + a;
          Mt[o] = p.M[(((size_t)j * r + a) * 2 + f) * Nxi + k];
          if (!p.is_bc(j, k)) Ut[o] = p.U[(((size_t)j * 2 + f) * r + a) * Nxi + k];
        }
  std::vector<cd> S((size_t)Rd * Rd, cd(0.0));
  run(Ny, [&](int t, int nt) {
    std::vector<double> g((size_t)r * r);
    for (int j = t; j < Ny; j += nt) {
      for (int k = 0; k < Nxi; ++k) {
        const cd* prow = &Prow[(size_t)slot_of[k] * blk + (size_t)j * Ny];
        const bool cj = conj_of[k] != 0;
        const double* mj = &Mt[((size_t)k * Ny + j) * 2 * r];
        for (int jp = 0; jp < Ny; ++jp) {
          const double* uj = &Ut[((size_t)k * Ny + jp) * 2 * r];
          for (int a = 0; a < r; ++a)
            for (int b = 0; b < r; ++b) g[(size_t)a * r + b] = mj[a] * uj[b] + mj[r + a] * uj[r + b];
          const cd w = cj ? std::conj(prow[jp]) : prow[jp];
          for (int a = 0; a < r; ++a) {
            cd* srow = &S[((size_t)j * r + a) * Rd + (size_t)jp * r];
            for (int b = 0; b < r; ++b) srow[b] += w * g[(size_t)a * r + b];
          }
        }
      }
    }
  });
  for (auto& v : S) v = -v;
  for (int q = 0; q < Rd; ++q) S[(size_t)q * Rd + q] += 1.0;
  si.Sinv.assign((size_t)Rd * Rd, cd(0.0));
  if (!invert(Rd, S.data(), si.Sinv.data(), nthreads)) return "singular moment capacitance matrix";
  return std::string();
}

bool invert(int m, const cd* A, cd* Ainv, int nthreads) {
  // P A = L U in place (row-major; L unit lower below the diagonal)
  std::vector<cd> a(A, A + (size_t)m * m);
  std::vector<int> perm(m);
  for (int i = 0; i < m; ++i) perm[i] = i;
  for (int k = 0; k < m; ++k) {
    int p = k;
    double best = std::abs(a[(size_t)k * m + k]);
    for (int i = k + 1; i < m; ++i) {
      const double v = std::abs(a[(size_t)i * m + k]);
      if (v > best) { best = v; p = i; }
    }
    if (best == 0.0) return false;
    if (p != k) {
      std::swap_ranges(a.begin() + (size_t)p * m, a.begin() + (size_t)(p + 1) * m, a.begin() + (size_t)k * m);
      std::swap(perm[p], perm[k]);
    }
    const cd* ak = &a[(size_t)k * m];
    const cd rpiv = 1.0 / ak[k];
    for (int i = k + 1; i < m; ++i) {
      cd* ai = &a[(size_t)i * m];
      const cd f = ai[k] * rpiv;
      ai[k] = f;
      if (f == 0.0) continue;
      for (int j = k + 1; j < m; ++j) ai[j] -= f * ak[j];
    }
  }
  // column c of A^{-1} solves L U x = P e_c, whose one nonzero sits at row i
  // with perm[i] = c; the forward sweep starts there
  std::vector<int> row_of(m);
  for (int i = 0; i < m; ++i) row_of[perm[i]] = i;
  auto solve_cols = [&](int c0, int c1) {
    std::vector<cd> x(m);
    for (int c = c0; c < c1; ++c) {
      const int s0 = row_of[c];
      std::fill(x.begin(), x.end(), cd(0.0));
      x[s0] = 1.0;
      for (int i = s0 + 1; i < m; ++i) {
        const cd* ai = &a[(size_t)i * m];
        cd acc = 0.0;
        for (int q = s0; q < i; ++q) acc += ai[q] * x[q];
        x[i] = -acc;
      }
      for (int i = m - 1; i >= 0; --i) {
        const cd* ai = &a[(size_t)i * m];
        cd acc = x[i];
        for (int q = i + 1; q < m; ++q) acc -= ai[q] * x[q];
        x[i] = acc / ai[i];
      }
      for (int i = 0; i < m; ++i) Ainv[(size_t)i * m + c] = x[i];
    }
  };
  const int nt = std::max(1, std::min(nthreads, m / 32));
  if (nt == 1) {
    solve_cols(0, m);
  } else {
    std::vector<std::thread> th;
    const int per = (m + nt - 1) / nt;
    for (int t = 0; t < nt; ++t) th.emplace_back(solve_cols, t * per, std::min(m, (t + 1) * per));
    for (auto& x : th) x.join();
  }
  return true;
}


std::vector<OutputCandidate> select_output(const std::vector<cd>& lam, const cd* G, const double* nrm2, cd sigma,
                                           int nev) {
  const int k = (int)lam.size();
  std::vector<OutputCandidate> cand;
  for (int i = 0; i < k; ++i) cand.push_back({lam[i], i, false});
  if (G && k > 0) {
    auto align = [&](int i, int j) {
      const double d = std::sqrt(nrm2[i] * nrm2[j]);
      return d > 0 ? std::abs(G[(size_t)i * k + j]) / d : 0.0;
    };
    std::vector<int> partner(k, -1);
    for (int i = 0; i < k; ++i)
      if (align(i, i) >= 1.0 - kSelfAlign) partner[i] = i;
    for (int i = 0; i < k; ++i) {
      if (partner[i] >= 0) continue;
      int best = -1;
      double ba = 0.0;
      for (int j = 0; j < k; ++j) {
        if (j == i || partner[j] >= 0) continue;
        const double a = align(i, j);
        if (a > ba) { ba = a; best = j; }
      }
      if (best >= 0 && ba >= 1.0 - kPairAlign &&
          std::abs(lam[best] - std::conj(lam[i])) <= kPairTol * std::abs(lam[i])) {
        partner[i] = best;
        partner[best] = i;
      } else {
        cand.push_back({std::conj(lam[i]), i, true});
      }
    }
  }
  std::vector<int> order(cand.size());
  for (size_t i = 0; i < cand.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const double da = std::abs(cand[a].lam - sigma), db = std::abs(cand[b].lam - sigma);
    if (std::abs(da - db) > 1e-12 * std::max(da, db)) return da < db;
    return (cand[a].lam.imag() > 0) && !(cand[b].lam.imag() > 0);
  });
  std::vector<OutputCandidate> out;
  for (int o = 0; o < (int)order.size() && o < nev; ++o) out.push_back(cand[order[o]]);
  return out;
}


// Gilbarg-Paolucci structure.  Normalised velocity W = m u / P and temperature
// th = m^2 R T / P^2 (m, P the mass and momentum fluxes), shock strength
// alpha = 2 E m^2 / P^2 - 1 (E the total enthalpy), g = (gamma - 1) / 2:
//   (4/3) mu_h dW/dz = W + th/W - 1,   (gamma mu_h / Pr) dth/dz = th - g((1 - W)^2 + alpha),
// mu_h = mu_h_inf (th / th_inf)^s, mu_h_inf = (delta / 16) sqrt(2 pi / gamma) / M.
// The shock is the separatrix of the downstream saddle.  It is traced in the
// phase plane th(W) by classical RK4 from the saddle (along its falling
// eigendirection) to the upstream node; z(W) then follows from the scalar ODE
// dW/dz on that curve, integrated by RK4 from the steepest point outward (on the
// curve the ODE is one-dimensional, so both directions are stable).
std::string gp_shock(double mach, double gamma, double Pr, double s_visc, double delta, int nz, const double* z,
                     double* rho, double* u, double* T, double* thickness) {
  if (!(mach > 1.0) || !(gamma > 1.0) || !(Pr > 0.0) || !(delta > 0.0) || !std::isfinite(mach) ||
      !std::isfinite(s_visc) || nz < 0)
    return "gp_shock: need mach > 1, gamma > 1, Pr > 0, delta > 0";
  const double g = 0.5 * (gamma - 1.0);
  const double u0 = mach * std::sqrt(gamma);            // rho_inf = 1, R T_inf = 1
  const double m = u0, P = 1.0 + u0 * u0, E = gamma / (gamma - 1.0) + 0.5 * u0 * u0;
  const double alpha = 2.0 * E * m * m / (P * P) - 1.0;
  const double Wi = m * u0 / P, ti = m * m / (P * P);
  // both zeros of the right-hand sides solve (1 + g) W^2 - (1 + 2 g) W + g (1 + alpha) = 0
  const double qa = 1.0 + g, qb = -(1.0 + 2.0 * g), qc = g * (1.0 + alpha);
  const double disc = std::sqrt(std::max(0.0, qb * qb - 4.0 * qa * qc));
  const double r1 = (-qb - disc) / (2.0 * qa), r2 = (-qb + disc) / (2.0 * qa);
  const double W1 = (std::abs(r1 - Wi) > std::abs(r2 - Wi)) ? r1 : r2;
  const double t1 = W1 * (1.0 - W1);
  const double muinf = (delta / 16.0) * std::sqrt(2.0 * M_PI / gamma) / mach;
  const double c = 4.0 * Pr / (3.0 * gamma);
  auto mu_h = [&](double th) { return muinf * std::pow(th / ti, s_visc); };
  auto Fth = [&](double W, double th) { return th - g * ((1.0 - W) * (1.0 - W) + alpha); };
  auto slope = [&](double W, double th) { return c * W * Fth(W, th) / (W * W - W + th); };
  auto dWdz = [&](double W, double th) { return (W + th / W - 1.0) / (4.0 / 3.0 * mu_h(th)); };
  // falling eigendirection at the saddle: k^2 + (2 W1 - 1 - c W1) k - 2 c g W1 (1 - W1) = 0
  const double B = 2.0 * W1 - 1.0 - c * W1, C = -2.0 * c * g * W1 * (1.0 - W1);
  const double k = 0.5 * (-B - std::sqrt(B * B - 4.0 * C));
  const double span = Wi - W1;
  // the curve is traced in t with W = W1 + span (1 + tanh t) / 2, whose steps
  // shrink geometrically toward both singular end points (RK4 stages then stay
  // close to the curve, where dth/dW is smooth)
  const int N = 1 << 16;
  const double ta = std::atanh(2.0 * 1e-9 - 1.0), tb = std::atanh(1.0 - 2.0 * 1e-10);
  const double dt = (tb - ta) / N;
  auto Wof = [&](double t) { return W1 + span * 0.5 * (1.0 + std::tanh(t)); };
  auto dWdt = [&](double t) { const double th_ = std::tanh(t); return span * 0.5 * (1.0 - th_ * th_); };
  std::vector<double> Ws(N + 1), ts(N + 1), ds(N + 1);
  Ws[0] = Wof(ta);
  ts[0] = t1 + k * (Ws[0] - W1);
  for (int i = 0; i < N; ++i) {
    const double t0 = ta + i * dt, th0 = ts[i];
    auto F = [&](double tt, double th_) { return slope(Wof(tt), th_) * dWdt(tt); };
    const double k1 = F(t0, th0), k2 = F(t0 + 0.5 * dt, th0 + 0.5 * dt * k1);
    const double k3 = F(t0 + 0.5 * dt, th0 + 0.5 * dt * k2), k4 = F(t0 + dt, th0 + dt * k3);
    Ws[i + 1] = Wof(t0 + dt);
    ts[i + 1] = th0 + dt * (k1 + 2.0 * k2 + 2.0 * k3 + k4) / 6.0;
  }
  for (int i = 0; i <= N; ++i) ds[i] = slope(Ws[i], ts[i]);
  const double Wa = Ws[0], Wb = Ws[N];
  // th(W) on the curve: cubic Hermite interpolation with the ODE's own slopes
  auto theta = [&](double W) {
    int i = (int)(std::upper_bound(Ws.begin(), Ws.end(), W) - Ws.begin()) - 1;
    i = std::max(0, std::min(N - 1, i));
    const double h = Ws[i + 1] - Ws[i];
    const double tq = (W - Ws[i]) / h;
    const double h00 = (1 + 2 * tq) * (1 - tq) * (1 - tq), h10 = tq * (1 - tq) * (1 - tq);
    const double h01 = tq * tq * (3 - 2 * tq), h11 = tq * tq * (tq - 1);
    return h00 * ts[i] + h10 * h * ds[i] + h01 * ts[i + 1] + h11 * h * ds[i + 1];
  };
  // steepest point: largest |dW/dz| on the samples, refined by golden section
  int ib = 0;
  double best = -1.0;
  for (int i = 0; i <= N; ++i) {
    const double v = std::abs(dWdz(Ws[i], ts[i]));
    if (v > best) { best = v; ib = i; }
  }
  double lo = Ws[std::max(0, ib - 1)], hi = Ws[std::min(N, ib + 1)];
  const double gr = 0.5 * (std::sqrt(5.0) - 1.0);
  auto f = [&](double W) { return -std::abs(dWdz(W, theta(W))); };
  double xa = hi - gr * (hi - lo), xb = lo + gr * (hi - lo), fa = f(xa), fb = f(xb);
  for (int it = 0; it < 200 && hi - lo > 1e-15 * span; ++it) {
    if (fa < fb) { hi = xb; xb = xa; fb = fa; xa = hi - gr * (hi - lo); fa = f(xa); }
    else { lo = xa; xa = xb; fa = fb; xb = lo + gr * (hi - lo); fb = f(xb); }
  }
  const double Wstar = 0.5 * (lo + hi);
  const double maxs = -f(Wstar);
  const double Delta = span / maxs;
  if (thickness) *thickness = Delta;
  if (nz == 0) return std::string();
  // z(W): RK4 on dW/dz along the curve from the steepest point, outward on each side
  auto rhs = [&](double W) {
    const double Wc = std::min(std::max(W, Wa), Wb);
    return dWdz(Wc, theta(Wc));
  };
  std::vector<int> ord(nz);
  for (int i = 0; i < nz; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return z[a] < z[b]; });
  const double hz = Delta / 4000.0;
  auto march = [&](double W, double z0, double z1) {
    const int steps = std::max(1, (int)std::ceil(std::abs(z1 - z0) / hz));
    const double dz = (z1 - z0) / steps;
    for (int s = 0; s < steps; ++s) {
      const double k1 = rhs(W), k2 = rhs(W + 0.5 * dz * k1), k3 = rhs(W + 0.5 * dz * k2), k4 = rhs(W + dz * k3);
      W += dz * (k1 + 2.0 * k2 + 2.0 * k3 + k4) / 6.0;
    }
    return W;
  };
  auto put = [&](int idx, double W) {
    const double Wc = std::min(std::max(W, Wa), Wb);
    const double th = theta(Wc);
    u[idx] = Wc / Wi;
    rho[idx] = Wi / Wc;
    T[idx] = th / ti;
  };
  // downstream side (z >= 0, W falls toward W1), nearest first
  {
    double W = Wstar, zc = 0.0;
    for (int q = 0; q < nz; ++q) {
      const int idx = ord[q];
      if (z[idx] < 0.0) continue;
      W = march(W, zc, z[idx]);
      zc = z[idx];
      put(idx, W);
    }
  }
  // upstream side (z < 0, W rises toward W_inf), nearest first
  {
    double W = Wstar, zc = 0.0;
    for (int q = nz - 1; q >= 0; --q) {
      const int idx = ord[q];
      if (z[idx] >= 0.0) continue;
      W = march(W, zc, z[idx]);
      zc = z[idx];
      put(idx, W);
    }
  }
  return std::string();
}

}  // namespace klst
