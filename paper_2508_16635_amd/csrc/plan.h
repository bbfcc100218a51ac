// Host-side plan data of the rotating-shell IMEX step: grids, tables and the FP64
// block factorization of the implicit operator.  Internal to libshellconv.
#pragma once
#include <complex>
#include <string>
#include <vector>

namespace sc {

typedef std::complex<double> cplx;

// Discretization sizes and node sets.
struct HostGrid {
  int L = 0, M = 0, m0 = 1, N = 0, Np = 0, nth = 0, nphi = 0, K = 0, S = 0;
  double ri = 0, ro = 0;
  std::vector<int> ms, nl, lmbase;            // per m-index k
  std::vector<int> lm_k, lm_l;                // per packed (k,l) index
  std::vector<double> x, r, xp, rp;           // radial nodes (N) and dealiasing nodes (Np)
  // radial matrices, row-major
  std::vector<double> D, D2, D4;              // N x N, d/dr powers
  std::vector<double> E, ED, ED2;             // Np x N: evaluation of u, u', u'' on the Np nodes
  std::vector<double> P;                      // N x Np: truncation to N Chebyshev modes
  std::vector<double> Dp;                     // Np x Np: d/dr on the Np nodes
  std::vector<double> ct, st, wt;             // Gauss-Legendre cos/sin(theta), weights
  // Legendre tables per k, [l - m][theta]
  std::vector<std::vector<double>> Pb, dPb, mPs;
};

// Builds every table above; throws std::runtime_error on bad sizes.
void build_grid(HostGrid& g, int L, int M, int m0, int N, double eta, int Np, int nth, int nphi);

// One chain of the block-tridiagonal implicit operator: unknown blocks along l at fixed m,
// alternating e and f.  Factor data (equilibrated block LU):
//   global scalings Rg, Cg (A~ = diag(Rg) A diag(Cg)),
//   per block: Sinv = inverse of the Ruiz-equilibrated Schur complement diag(sr) S diag(sc),
//              Lo = A~_{i,i-1},  H = S_i^{-1} A~_{i,i+1}.
//   segmented scan (segments of `seg` blocks): with z_i the forward unknowns and x_i the
//   backward ones, z_i = zeta_i + Phi_i z_{a-1} inside a segment starting at a, and
//   x_i = xi_i + Psi_i x_{e+1} inside a segment ending at e; Phi_i = -S_i^{-1} Lo_i Phi_{i-1},
//   Psi_i = -H_i Psi_{i+1} (zero in the first / last segment where they are not used).
struct ChainFactor {
  int k = 0, m = 0, cls = 0, n = 0, l0 = 0;
  std::vector<int> field, l;                  // per block: 0 = e, 1 = f
  std::vector<double> Rg, Cg;                 // n*N
  std::vector<double> sr, sc;                 // n*N
  std::vector<cplx> Sinv, Lo, H;              // n*N*N each (row-major blocks)
  std::vector<cplx> Phi, Psi;                 // n*N*N each
  std::vector<cplx> G;                        // n*N*N: S_i^{-1} Lo_i (forward recurrence matrix)
};

struct TFactor {                              // temperature block per l (real)
  std::vector<double> Tinv, tr, tc;           // N*N, N, N
};

struct OpParams {
  double Ek, Pr, dt;
  double cor = 1.0;   // weight of the Coriolis terms of K: 1 implicit, 0 explicit-Coriolis variant
};

// Builds and factors every chain and temperature block; nthreads host threads.
void factor_all(const HostGrid& g, const OpParams& op, std::vector<ChainFactor>& chains,
                std::vector<TFactor>& tf, int nthreads, int seg);

}  // namespace sc
