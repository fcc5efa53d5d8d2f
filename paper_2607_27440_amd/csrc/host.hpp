// Host-side pieces of the kLST library: problem tables, block-Jacobi ILU(0)
// factorisation, and small dense complex linear algebra for projected problems.
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "klst.h"

namespace klst {

using cd = std::complex<double>;

// Discrete operator tables (Sec. 2.2 with the grid of Sec. 3.1).
struct Problem {
  int Ny = 0, Nxi = 0, r = 0, Dv = 2;
  double beta = 0, L = 0, s_inf = 0, s_visc = 0, nu_inf = 0;
  std::vector<double> xi_x, xi_y, w;   // [Nxi]
  std::vector<double> Dx;              // [Ny*Ny] row-major, mapped derivative
  std::vector<double> rho, u, E, T, nu;
  std::vector<double> gc;              // [Ny][Nxi] NONEQ base g (empty for EQ bases)
  std::vector<double> U;               // [Ny][2][r][Nxi] coupling columns G_a / H_a
  std::vector<double> M;               // [Ny][r][2][Nxi] moment functionals
  std::vector<uint8_t> bc;             // [Ny][2][Nxi] inflow rows
  int n_bc = 0;
  int64_t n() const { return 2LL * Ny * Nxi; }
  int64_t nnz() const {
    return n() * (Ny - 1 + 2LL * Nxi) - (int64_t)n_bc * (Ny - 2 + 2LL * Nxi);
  }
  bool is_bc(int j, int k) const { return bc[((size_t)j * 2) * Nxi + k] != 0; }
};

// Mapped Chebyshev-Gauss-Lobatto node positions x_j = L y_j / sqrt(1 + s - y_j^2),
// y_j = cos(j pi / (Ny - 1)), s = (L / s_inf)^2 (node 0 at x = +s_inf).
void mapped_nodes(int Ny, double L, double s_inf, double* x);

// Mirror of every velocity node in xi_y (same xi_x, xi_y negated; a node with
// xi_y = 0 is its own), when the table has all of them exactly: mk[k] = mirror.
// Returns false (mk cleared) when some node has none.
bool mirror_nodes(const std::vector<double>& xi_x, const std::vector<double>& xi_y, std::vector<int>& mk);

// Fills `p`; returns an empty string on success, else a description of the error.
std::string build_problem(const klst_grid* g, const klst_vel* v, const klst_base* b,
                          double beta, Problem& p);

// Block-Jacobi ILU(0) of (A - sigma B) over blocks of whole velocity lines in
// the velocity-major ordering.  Line l = f * Nxi + k; block = lines
// [b*nl, min((b+1)*nl, 2 Nxi)).  For every line, F holds the combined unit-lower
// L and upper U factors of its dense Ny x Ny diagonal block; C holds, per block,
// the factor entries that couple two lines of the block at the same node j:
// C[((b*nl + l)*nl + l2)*Ny + j], l2 < l in L, l2 > l in U (l, l2 block-local).
struct ILU0 {
  int nl = 1, nblocks = 0, Ny = 0, nlines = 0;
  std::vector<cd> F;    // [nlines][Ny][Ny]
  std::vector<cd> C;    // [nblocks][nl][nl][Ny]
  int floored = 0;
};
void build_ilu0(const Problem& p, cd sigma, int lines_per_block, ILU0& f, int nthreads);
// Dense inverse (L_b U_b)^{-1} of every block's ILU(0) factors, column-major over
// the block's rows in (line, node) order; block b starts at Kinv[off[b]].
void build_block_inverse(const ILU0& f, std::vector<cd>& Kinv, std::vector<int64_t>& off,
                         int nthreads);

// Exact inverse of (A - sigma B) in structured form (Woodbury identity):
// A - sigma B = P - Ut M, P block diagonal over the velocity lines with a block
// that depends on the velocity node only, P_k = xi_x,k D_x + diag(nu_j + i beta
// xi_y,k - sigma) with unit inflow rows, and Ut M the rank-(r Ny) moment coupling
// (coupling columns U with inflow rows zeroed).  Then
// (A - sigma B)^{-1} = P^{-1} + P^{-1} Ut S^{-1} M P^{-1}, S = I - M P^{-1} Ut.
struct StructuredInverse {
  int Ny = 0, Nxi = 0, r = 0;
  // Line inverses are stored per slot.  With sigma real, the block of the node
  // mirrored in xi_y (same xi_x, opposite xi_y) is the complex conjugate of the
  // node's block, so one slot serves both: slot s holds P_k^{-1} for k =
  // slot_node[s] and stands for conj(P_k^{-1}) at slot_mate[s] (-1: no mate).
  std::vector<int> slot_node, slot_mate;
  std::vector<cd> Pinv;   // [slots][Ny x Ny], column-major: entry (j, m) at m Ny + j
  std::vector<cd> Sinv;   // [(r Ny) x (r Ny)], row-major, index q = j r + a
};
// Slot assignment of the structured inverse: slot s stores node slot_node[s]
// and, with sigma real, serves its xi_y mirror slot_mate[s] (-1: none) by
// conjugation; slot_of[k] / conj_of[k] per node.
void structured_slots(const Problem& p, cd sigma, std::vector<int>& slot_node, std::vector<int>& slot_mate,
                      std::vector<int>& slot_of, std::vector<int>& conj_of);
// Returns an empty string on success, else why (a singular line block or capacitance).
std::string build_structured_inverse(const Problem& p, cd sigma, StructuredInverse& si, int nthreads);

// ---- continuum normal-shock structure (Gilbarg-Paolucci, Sec. 2.1) ----
// Steady 1-D Navier-Stokes shock of a gas with ratio of specific heats gamma,
// Prandtl number Pr, viscosity mu ~ T^s, lengths in upstream mean free paths
// l_inf = (16/delta) mu_inf / (rho_inf sqrt(2 pi R T_inf)).  Fills, at the nz
// positions z (measured from the point of steepest velocity gradient, positive
// downstream), rho / rho_inf, u / u_inf, T / T_inf, and returns the thickness
// Delta / l_inf of eq. ShockThickness.  Returns an empty string on success.
std::string gp_shock(double mach, double gamma, double Pr, double s_visc, double delta, int nz, const double* z,
                     double* rho, double* u, double* T, double* thickness);

// ---- returned eigenpairs of a Jacobi-Davidson solve ----
struct OutputCandidate {
  cd lam;
  int src;         // locked pair whose eigenvector the candidate uses
  bool mirrored;   // (conj(lambda_src), R conj(x_src)) rather than the pair itself
};
// Candidates for the returned set: every locked pair and, when G != nullptr (a
// real target on a problem symmetric under the xi_y reflection R), the partner
// (conj(lambda_i), R conj(x_i)) of each locked complex eigenvalue whose partner
// was not locked.  G [k x k] row-major, G[i k + j] = <R conj(x_i), x_j>, and
// nrm2[i] = ||x_i||^2.  Partnership is read from the eigenvectors: lambda_i is
// real (its own partner) when |G_ii| >= (1 - kSelfAlign) ||x_i||^2, and locked
// x_j is the partner of x_i when |G_ij| >= (1 - kPairAlign) ||x_i|| ||x_j|| and
// |lambda_j - conj(lambda_i)| <= kPairTol |lambda_i| (one to one, best
// alignment first).  Returns at most nev candidates ordered by |lambda - sigma|
// (ties within 1e-12 relative: Im lambda > 0 first, then locking order).
constexpr double kSelfAlign = 1e-10;
constexpr double kPairAlign = 1e-6;
constexpr double kPairTol = 1e-6;
std::vector<OutputCandidate> select_output(const std::vector<cd>& lam, const cd* G, const double* nrm2, cd sigma,
                                           int nev);

// ---- small dense complex matrices, row-major m x m ----
// Schur form G U = U T, T upper triangular, with the diagonal ordered by
// decreasing |T_ii| in the first nsort positions (each holds the largest
// remaining magnitude; all positions when nsort <= 0).  U row-major.
// Returns false if the QR iteration failed to converge.
bool sorted_schur(int m, const cd* G, cd* U, cd* T, int nsort = 0);
// The eigenvalue mu of G of largest modulus (first on ties in the QR order) and
// a unit eigenvector x (inverse iteration): the first column of a sorted Schur
// form, without computing the rest of it.  Returns false on failure.
bool dominant_eig(int m, const cd* G, cd& mu, cd* x);
// Householder QR of an m x m matrix A = Qm Rm.
void qr_square(int m, const cd* A, cd* Qm, cd* Rm);
// Inverse of an m x m matrix by LU with partial pivoting, then one forward and
// one backward sweep per column (columns split over up to nthreads threads);
// false if singular.
bool invert(int m, const cd* A, cd* Ainv, int nthreads = 1);

}  // namespace klst
