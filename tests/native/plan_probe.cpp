// CPU probe of libshellconv's host-side plan (grids, tables, FP64 block factorization):
// writes the tables and solves A x = b with the factors by host block substitution, so the
// tests can compare them with the oracle without a GPU.
//   plan_probe L M m0 N Ek Pr dt out.bin rhs.bin
// rhs.bin: packed chain right-hand sides in the canonical (field, lm, j, ri) layout.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_2508_16635_amd/csrc/plan.h"

using namespace sc;

static void put(FILE* f, const std::vector<double>& v) {
  long long n = (long long)v.size();
  fwrite(&n, sizeof(n), 1, f);
  fwrite(v.data(), sizeof(double), v.size(), f);
}

int main(int argc, char** argv) {
  if (argc < 10) return 2;
  int L = atoi(argv[1]), M = atoi(argv[2]), m0 = atoi(argv[3]), N = atoi(argv[4]);
  double Ek = atof(argv[5]), Pr = atof(argv[6]), dt = atof(argv[7]);
  HostGrid g;
  build_grid(g, L, M, m0, N, 0.35, 0, 0, 0);
  std::vector<ChainFactor> ch;
  std::vector<TFactor> tf;
  factor_all(g, OpParams{Ek, Pr, dt}, ch, tf, 4, 8);
  // read rhs
  long long nreal = 6LL * N * g.S;
  std::vector<double> b(nreal), x(nreal, 0.0);
  FILE* fr = fopen(argv[9], "rb");
  if (!fr || fread(b.data(), sizeof(double), nreal, fr) != (size_t)nreal) return 3;
  fclose(fr);
  auto at = [&](std::vector<double>& v, int fld, int lm, int j) -> cplx* {
    return reinterpret_cast<cplx*>(&v[2LL * ((long long)N * ((long long)fld * g.S + lm) + j)]);
  };
  for (auto& c : ch) {
    int n = c.n;
    std::vector<cplx> z((size_t)n * N), t(N);
    for (int i = 0; i < n; ++i) {
      int lm = g.lmbase[c.k] + c.l[i] - c.m;
      for (int j = 0; j < N; ++j) {
        cplx r = c.Rg[(size_t)i * N + j] * *at(b, c.field[i], lm, j);
        if (i > 0)
          for (int q = 0; q < N; ++q) r -= c.Lo[((size_t)i * N + j) * N + q] * z[(size_t)(i - 1) * N + q];
        t[j] = c.sr[(size_t)i * N + j] * r;
      }
      for (int j = 0; j < N; ++j) {
        cplx a = 0;
        for (int q = 0; q < N; ++q) a += c.Sinv[((size_t)i * N + j) * N + q] * t[q];
        z[(size_t)i * N + j] = c.sc[(size_t)i * N + j] * a;
      }
    }
    for (int i = n - 2; i >= 0; --i)
      for (int j = 0; j < N; ++j) {
        cplx a = z[(size_t)i * N + j];
        for (int q = 0; q < N; ++q) a -= c.H[((size_t)i * N + j) * N + q] * z[(size_t)(i + 1) * N + q];
        z[(size_t)i * N + j] = a;  // rows of block i only read block i+1 (already final)
      }
    for (int i = 0; i < n; ++i) {
      int lm = g.lmbase[c.k] + c.l[i] - c.m;
      for (int j = 0; j < N; ++j) *at(x, c.field[i], lm, j) = c.Cg[(size_t)i * N + j] * z[(size_t)i * N + j];
    }
  }
  for (int lm = 0; lm < g.S; ++lm) {
    int l = g.lm_l[lm];
    for (int j = 0; j < N; ++j) {
      cplx a = 0;
      for (int q = 0; q < N; ++q) a += tf[l].Tinv[(size_t)j * N + q] * tf[l].tr[q] * *at(b, 2, lm, q);
      *at(x, 2, lm, j) = tf[l].tc[j] * a;
    }
  }
  FILE* f = fopen(argv[8], "wb");
  put(f, g.x);
  put(f, g.r);
  put(f, g.rp);
  put(f, g.D);
  put(f, g.E);
  put(f, g.P);
  put(f, g.Dp);
  put(f, g.ct);
  put(f, g.wt);
  std::vector<double> Pb, dP, mP;
  for (int k = 0; k <= g.K; ++k) {
    Pb.insert(Pb.end(), g.Pb[k].begin(), g.Pb[k].end());
    dP.insert(dP.end(), g.dPb[k].begin(), g.dPb[k].end());
    mP.insert(mP.end(), g.mPs[k].begin(), g.mPs[k].end());
  }
  put(f, Pb);
  put(f, dP);
  put(f, mP);
  put(f, x);
  fclose(f);
  return 0;
}
