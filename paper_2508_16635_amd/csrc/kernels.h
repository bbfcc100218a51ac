// Device kernels of the rotating-shell IMEX step / Jacobian action (gfx950).
// Internal to libshellconv; included by api.hip only.
//
// Data layouts (nv = vectors in the batch, q = field component, ri = Re/Im):
//   canonical state  v[vec][field e,f,T][lm][j][ri]          (FP64; lm packs (m, l))
//   synthesis input  Gs[k][(vec, rp, q<3, ri)][l-m]  Gv[k][(vec, rp, q<5, ri)][l-m]
//   synthesis output Cs[k][(vec, rp, q<3, ri)][theta]  Cv[k][(vec, rp, q<5, ri)][2 nth]
//   analysis input   Fs[k][(vec, rp, q<2, ri)][theta]  Fv[k][(vec, rp, q<2, ri)][2 nth]
//   analysis output  As[k][(vec, rp, q<2, ri)][l-m]    Av[k][(vec, rp, q<2, ri)][l-m]
//   base fields      base[rp][field<9][phi][theta]
// The Legendre transforms are the contractions C[i][j] = sum_k A[i][k] B[j][k] with both
// operands contiguous in k (gemm_batched).
#pragma once
#include <hip/hip_runtime.h>

namespace sc {

struct GemmProb {
  long long a_off, b_off, c_off;  // element offsets: A, C in the workspace, B in the tables
  int Mper, N, K, lda, ldb, ldc;  // M = Mper * nvec
};

struct DevGrid {
  int L, m0, N, Np, nth, nphi, K, S;
  int vcap;           // vector capacity of the workspaces (block strides use it)
  const int* lm_k;    // [S]
  const int* lm_l;    // [S]
  const int* lmbase;  // [K+1]
  const double* r;    // [N]
  const double* rp;   // [Np]
  const double* E;    // [Np][N]
  const double* ED;
  const double* ED2;
  const double* P;    // [N][Np]
  const double* Dp;   // [Np][Np]
  const double* D;    // [N][N]
  const double* D2;
  const double* D4;
};

struct PhysParams {
  double Ek, Ra, Pr, dt, ro;
};

// ------------------------------------------------------------------------------------------
// K1: radial preparation.  For each (vec, r_p, lm): the eight spectral profiles
//   ur = lam f/r^2, wr = lam e/r^2, dT = T'   (scalar synthesis with Pbar)
//   Su = f'/r, Tu = e/r, Sw = e'/r, Tw = -(f'' - lam f/r^2)/r, ST = T/r  (vector synthesis)
// evaluated at the N_p nodes as diag(r^-k) E D^j u, in FP64, stored in precision T.
// Input cleaning: Im at m = 0, e/f at l = 0 and the phase slot J are read as 0.
template <class T>
__global__ void k_radial_prep(DevGrid g, const double* __restrict__ v, long long ldv, long long J,
                              int nvec, T* __restrict__ Gs, T* __restrict__ Gv) {
  long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long total = (long long)nvec * g.Np * g.S;
  if (tid >= total) return;
  int lm = (int)(tid % g.S);
  long long t2 = tid / g.S;
  int rp = (int)(t2 % g.Np);
  int vec = (int)(t2 / g.Np);
  int k = g.lm_k[lm], l = g.lm_l[lm];
  int m = k * g.m0;
  const int N = g.N;
  const double* vb = v + (long long)vec * ldv;
  double acc[7][2];
#pragma unroll
  for (int a = 0; a < 7; ++a) acc[a][0] = acc[a][1] = 0.0;
  const double* Er = g.E + (long long)rp * N;
  const double* EDr = g.ED + (long long)rp * N;
  const double* ED2r = g.ED2 + (long long)rp * N;
  long long base_e = 2LL * ((long long)N * (0LL * g.S + lm));
  long long base_f = 2LL * ((long long)N * (1LL * g.S + lm));
  long long base_t = 2LL * ((long long)N * (2LL * g.S + lm));
  bool ef_ok = (l > 0);
  for (int j = 0; j < N; ++j) {
    double e0 = 0, e1 = 0, f0 = 0, f1 = 0, t0, t1;
    long long ie = base_e + 2 * j, jf = base_f + 2 * j, it = base_t + 2 * j;
    if (ef_ok) {
      e0 = (ie == J) ? 0.0 : vb[ie];
      e1 = (k == 0 || ie + 1 == J) ? 0.0 : vb[ie + 1];
      f0 = (jf == J) ? 0.0 : vb[jf];
      f1 = (k == 0 || jf + 1 == J) ? 0.0 : vb[jf + 1];
    }
    t0 = (it == J) ? 0.0 : vb[it];
    t1 = (k == 0 || it + 1 == J) ? 0.0 : vb[it + 1];
    double E0 = Er[j], E1 = EDr[j], E2 = ED2r[j];
    acc[0][0] += E0 * f0; acc[0][1] += E0 * f1;   // E f
    acc[1][0] += E1 * f0; acc[1][1] += E1 * f1;   // E D f
    acc[2][0] += E2 * f0; acc[2][1] += E2 * f1;   // E D^2 f
    acc[3][0] += E0 * e0; acc[3][1] += E0 * e1;   // E e
    acc[4][0] += E1 * e0; acc[4][1] += E1 * e1;   // E D e
    acc[5][0] += E0 * t0; acc[5][1] += E0 * t1;   // E T
    acc[6][0] += E1 * t0; acc[6][1] += E1 * t1;   // E D T
  }
  double lam = (double)l * (l + 1);
  double ri = 1.0 / g.rp[rp];
  double ri2 = ri * ri;
  int nl = g.L - m + 1;
  int il = l - m;
  long long rowS = ((long long)vec * g.Np + rp) * 6;
  long long rowV = ((long long)vec * g.Np + rp) * 10;
  long long offS = 6LL * g.Np * g.vcap * g.lmbase[k];  // block k of Gs (rows x nl)
  long long offV = 10LL * g.Np * g.vcap * g.lmbase[k];
  T* gs = Gs + offS + rowS * nl + il;
  T* gv = Gv + offV + rowV * nl + il;
  for (int c = 0; c < 2; ++c) {
    gs[(0 + c) * nl] = (T)(lam * ri2 * acc[0][c]);                 // ur
    gs[(2 + c) * nl] = (T)(lam * ri2 * acc[3][c]);                 // wr
    gs[(4 + c) * nl] = (T)(acc[6][c]);                             // dT
    gv[(0 + c) * nl] = (T)(acc[1][c] * ri);                        // Su
    gv[(2 + c) * nl] = (T)(acc[3][c] * ri);                        // Tu
    gv[(4 + c) * nl] = (T)(acc[4][c] * ri);                        // Sw
    gv[(6 + c) * nl] = (T)(-acc[2][c] * ri + lam * ri2 * ri * acc[0][c]);  // Tw
    gv[(8 + c) * nl] = (T)(acc[5][c] * ri);                        // ST
  }
}

// ------------------------------------------------------------------------------------------
// K2/K6: batched contractions C[i][j] = sum_k A[i][k] B[j][k], 64x64 tiles, LDS-staged.
template <class T>
__global__ void __launch_bounds__(256) k_gemm_batched(const GemmProb* __restrict__ probs, int nprob, int nvec,
                                                      const T* __restrict__ ws_in, const T* __restrict__ tab,
                                                      T* __restrict__ ws_out) {
  constexpr int BM = 64, BN = 64, BK = 16;
  __shared__ T As[BK][BM + 1];
  __shared__ T Bs[BK][BN + 1];
  // locate this tile's problem
  int tile = blockIdx.x;
  int p = 0;
  GemmProb pr;
  int tm = 0, tn = 0;
  for (p = 0; p < nprob; ++p) {
    pr = probs[p];
    int M = pr.Mper * nvec;
    int nt_m = (M + BM - 1) / BM, nt_n = (pr.N + BN - 1) / BN;
    int nt = nt_m * nt_n;
    if (tile < nt) {
      tm = tile / nt_n;
      tn = tile % nt_n;
      break;
    }
    tile -= nt;
  }
  if (p >= nprob) return;
  const int M = pr.Mper * nvec, N = pr.N, K = pr.K;
  const T* A = ws_in + pr.a_off;
  const T* B = tab + pr.b_off;
  T* C = ws_out + pr.c_off;
  const int tid = threadIdx.x;
  const int tx = tid % 16, ty = tid / 16;  // 16 x 16 threads, 4 x 4 outputs each
  T acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = (T)0;
  const int i0 = tm * BM, j0 = tn * BN;
  for (int k0 = 0; k0 < K; k0 += BK) {
    // load A tile: 64 rows x 16 k; thread -> row tid/4, k (tid%4)*4 .. +3
    {
      int r = tid / 4, kk = (tid % 4) * 4;
      int gi = i0 + r;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        int gk = k0 + kk + q;
        As[kk + q][r] = (gi < M && gk < K) ? A[(long long)gi * pr.lda + gk] : (T)0;
      }
      int gj = j0 + r;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        int gk = k0 + kk + q;
        Bs[kk + q][r] = (gj < N && gk < K) ? B[(long long)gj * pr.ldb + gk] : (T)0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; ++kk) {
      T a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = As[kk][ty + 16 * q];
        b[q] = Bs[kk][tx + 16 * q];
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] += a[x] * b[y];
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    int gi = i0 + ty + 16 * x;
    if (gi >= M) continue;
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      int gj = j0 + tx + 16 * y;
      if (gj < N) C[(long long)gi * pr.ldc + gj] = acc[x][y];
    }
  }
}

// ------------------------------------------------------------------------------------------
// K3/K4/K5: per ring (vec, r_p, theta): combine the synthesized Legendre sums into the
// Fourier coefficients of the 9 physical fields (U, omega, grad T), inverse DFT along phi,
// pointwise products, forward DFT of (W_r, W_theta, W_phi, Q), and write the analysis inputs.
// MODE 0: linearized products about the cached base fields,
// MODE 1: nonlinear products of the fields themselves,
// MODE 2: synthesis only, the 9 fields are written to base (and base32 if non-null).
enum { RING_LINEAR = 0, RING_NONLINEAR = 1, RING_SYNTH = 2 };

template <class T, int MODE, int RT>
__global__ void __launch_bounds__(256) k_ring(DevGrid g, int nvec, const T* __restrict__ Cs, const T* __restrict__ Cv,
                                              const T* __restrict__ base, const T* __restrict__ twc,
                                              const T* __restrict__ tws, T Ek, T* __restrict__ Fs,
                                              T* __restrict__ Fv, double* __restrict__ base_out64,
                                              float* __restrict__ base_out32) {
  extern __shared__ unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const int K1 = g.K + 1, nphi = g.nphi, nth = g.nth;
  T* coef = sm;                                  // [9][K1][RT] complex -> 2 arrays
  T* coefr = coef;                               // [(f*K1 + k)*RT + tt]
  T* coefi = coef + 9 * K1 * RT;
  T* vals = coefi + 9 * K1 * RT;                 // [4][nphi][RT]
  T* tc = vals + 4 * nphi * RT;                  // [K1][nphi]
  T* ts = tc + K1 * nphi;
  const int ntile = (nth + RT - 1) / RT;
  int blk = blockIdx.x;
  int tile = blk % ntile;
  int vr = blk / ntile;  // vec * Np + rp
  int rp = vr % g.Np;
  const int th0 = tile * RT;
  const int tid = threadIdx.x;
  for (int i = tid; i < K1 * nphi; i += blockDim.x) {
    tc[i] = twc[i];
    ts[i] = tws[i];
  }
  // step A: gather coefficients
  const long long Ms = (long long)6 * g.Np * g.vcap, Mv = (long long)10 * g.Np * g.vcap;
  for (int idx = tid; idx < K1 * RT; idx += blockDim.x) {
    int tt = idx % RT, k = idx / RT;
    int th = th0 + tt;
    T c[26];
    if (th < nth) {
      const T* cs = Cs + (long long)k * Ms * nth + ((long long)vr * 6) * nth + th;
#pragma unroll
      for (int q = 0; q < 6; ++q) c[q] = cs[(long long)q * nth];
      const T* cv = Cv + (long long)k * Mv * 2 * nth + ((long long)vr * 10) * 2 * nth + th;
#pragma unroll
      for (int q = 0; q < 10; ++q) {
        c[6 + q] = cv[(long long)q * 2 * nth];         // dP part
        c[16 + q] = cv[(long long)q * 2 * nth + nth];  // mPs part
      }
    } else {
#pragma unroll
      for (int q = 0; q < 26; ++q) c[q] = (T)0;
    }
    // scalar parts: ur(0,1) wr(2,3) dT(4,5); vector parts q: Su 0, Tu 1, Sw 2, Tw 3, ST 4
    auto dPr = [&](int q) { return c[6 + 2 * q]; };
    auto dPi = [&](int q) { return c[7 + 2 * q]; };
    auto mPr = [&](int q) { return c[16 + 2 * q]; };
    auto mPi = [&](int q) { return c[17 + 2 * q]; };
    T fr[9], fi[9];
    fr[0] = c[0]; fi[0] = c[1];                                   // U_r
    fr[1] = dPr(0) - mPi(1); fi[1] = dPi(0) + mPr(1);              // U_th = dP Su + i mPs Tu
    fr[2] = -mPi(0) - dPr(1); fi[2] = mPr(0) - dPi(1);             // U_ph = i mPs Su - dP Tu
    fr[3] = c[2]; fi[3] = c[3];                                   // w_r
    fr[4] = dPr(2) - mPi(3); fi[4] = dPi(2) + mPr(3);              // w_th
    fr[5] = -mPi(2) - dPr(3); fi[5] = mPr(2) - dPi(3);             // w_ph
    fr[6] = c[4]; fi[6] = c[5];                                   // G_r
    fr[7] = dPr(4); fi[7] = dPi(4);                               // G_th = dP ST
    fr[8] = -mPi(4); fi[8] = mPr(4);                              // G_ph = i mPs ST
#pragma unroll
    for (int f = 0; f < 9; ++f) {
      coefr[(f * K1 + k) * RT + tt] = fr[f];
      coefi[(f * K1 + k) * RT + tt] = fi[f];
    }
  }
  __syncthreads();
  // step B: inverse DFT and pointwise products
  for (int idx = tid; idx < nphi * RT; idx += blockDim.x) {
    int tt = idx % RT, p = idx / RT;
    int th = th0 + tt;
    T f[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) f[q] = (T)0;
    for (int k = 0; k < K1; ++k) {
      T cr = tc[k * nphi + p], si = ts[k * nphi + p];
#pragma unroll
      for (int q = 0; q < 9; ++q) f[q] += coefr[(q * K1 + k) * RT + tt] * cr - coefi[(q * K1 + k) * RT + tt] * si;
    }
    if (MODE == RING_SYNTH) {
      if (th < nth) {
#pragma unroll
        for (int q = 0; q < 9; ++q) {
          long long o = (((long long)rp * 9 + q) * nphi + p) * nth + th;
          base_out64[o] = (double)f[q];
          if (base_out32) base_out32[o] = (float)f[q];
        }
      }
      continue;
    }
    T W0, W1, W2, Q;
    if (MODE == RING_NONLINEAR) {
      // W = Ek U x w, Q = -U . grad T
      W0 = Ek * (f[1] * f[5] - f[2] * f[4]);
      W1 = Ek * (f[2] * f[3] - f[0] * f[5]);
      W2 = Ek * (f[0] * f[4] - f[1] * f[3]);
      Q = -(f[0] * f[6] + f[1] * f[7] + f[2] * f[8]);
    } else {
      T b[9];
      if (th < nth) {
#pragma unroll
        for (int q = 0; q < 9; ++q) b[q] = base[(((long long)rp * 9 + q) * nphi + p) * nth + th];
      } else {
#pragma unroll
        for (int q = 0; q < 9; ++q) b[q] = (T)0;
      }
      // W' = Ek (U x w_u + u x Omega), Q' = -(U . grad tau + u . grad T)
      W0 = Ek * ((b[1] * f[5] - b[2] * f[4]) + (f[1] * b[5] - f[2] * b[4]));
      W1 = Ek * ((b[2] * f[3] - b[0] * f[5]) + (f[2] * b[3] - f[0] * b[5]));
      W2 = Ek * ((b[0] * f[4] - b[1] * f[3]) + (f[0] * b[4] - f[1] * b[3]));
      Q = -((b[0] * f[6] + b[1] * f[7] + b[2] * f[8]) + (f[0] * b[6] + f[1] * b[7] + f[2] * b[8]));
    }
    vals[(0 * nphi + p) * RT + tt] = W0;
    vals[(1 * nphi + p) * RT + tt] = W1;
    vals[(2 * nphi + p) * RT + tt] = W2;
    vals[(3 * nphi + p) * RT + tt] = Q;
  }
  if (MODE == RING_SYNTH) return;
  __syncthreads();
  // step C: forward DFT, scale (2 - d_k0)/nphi, write analysis inputs
  const long long Ma = (long long)4 * g.Np * g.vcap;
  for (int idx = tid; idx < 3 * K1 * RT; idx += blockDim.x) {
    int tt = idx % RT;
    int o = (idx / RT) % 3;
    int k = idx / (3 * RT);
    int th = th0 + tt;
    if (th >= nth) continue;
    T sc = (k == 0 ? (T)1 : (T)2) / (T)nphi;
    if (o < 2) {
      int src = (o == 0) ? 0 : 3;  // W_r or Q
      T ar = 0, ai = 0;
      for (int p = 0; p < nphi; ++p) {
        T x = vals[(src * nphi + p) * RT + tt];
        ar += x * tc[k * nphi + p];
        ai -= x * ts[k * nphi + p];
      }
      T* out = Fs + (long long)k * Ma * nth + ((long long)vr * 4 + 2 * o) * nth + th;
      out[0] = ar * sc;
      out[nth] = ai * sc;
    } else {
      T ar = 0, ai = 0, br = 0, bi = 0;  // W_th, W_ph
      for (int p = 0; p < nphi; ++p) {
        T x = vals[(1 * nphi + p) * RT + tt], y = vals[(2 * nphi + p) * RT + tt];
        T cc = tc[k * nphi + p], ss = ts[k * nphi + p];
        ar += x * cc;
        ai -= x * ss;
        br += y * cc;
        bi -= y * ss;
      }
      ar *= sc; ai *= sc; br *= sc; bi *= sc;
      T* out = Fv + (long long)k * Ma * 2 * nth + ((long long)vr * 4) * 2 * nth + th;
      // dP rows: (W_th, -W_ph); mPs rows: (-i W_ph, -i W_th)
      out[0 * 2 * nth] = ar;
      out[1 * 2 * nth] = ai;
      out[2 * 2 * nth] = -br;
      out[3 * 2 * nth] = -bi;
      out[0 * 2 * nth + nth] = bi;
      out[1 * 2 * nth + nth] = -br;
      out[2 * 2 * nth + nth] = ai;
      out[3 * 2 * nth + nth] = -ar;
    }
  }
}

// ------------------------------------------------------------------------------------------
// K7: curl projections back to the N nodes and assembly of the right-hand side
//   b = M u + dt (N(u) + Ra lam T/(r r_o) [f only] + C i m M u + c i m M X)
// with M_e = Ek lam/r^2, M_f = -Ek lam/r^2 (D^2 - lam/r^2), M_T = 1, and boundary rows.
// MODE_STEP: inhomogeneous T_00 rows, no c-term.  One block per (vec, lm).
template <class T, bool STEP>
__global__ void __launch_bounds__(128) k_project_rhs(DevGrid g, PhysParams ph, int nvec, const T* __restrict__ As,
                                                     const T* __restrict__ Av, const double* __restrict__ v,
                                                     long long ldv, long long J, double C,
                                                     const double* __restrict__ MX, double* __restrict__ b) {
  __shared__ double sWr[2][128], sQ[2][128], sS[2][128], sTor[2][128], sTf[2][128];
  __shared__ double su[3][2][64];
  int blk = blockIdx.x;
  int lm = blk % g.S, vec = blk / g.S;
  int k = g.lm_k[lm], l = g.lm_l[lm];
  int m = k * g.m0;
  int nl = g.L - m + 1, il = l - m;
  const int N = g.N, Np = g.Np;
  const int tid = threadIdx.x;
  double lam = (double)l * (l + 1);
  const long long Ma = (long long)4 * Np * g.vcap;
  const double* vb = v + (long long)vec * ldv;
  double* bb = b + (long long)vec * 6LL * N * g.S;
  // phase-slot value c
  double cval = 0.0;
  if (!STEP && J >= 0) cval = v[(long long)vec * ldv + J];
  const T* as = As + Ma * g.lmbase[k];
  const T* av = Av + Ma * g.lmbase[k];
  for (int rp = tid; rp < Np; rp += blockDim.x) {
    long long row = ((long long)vec * Np + rp) * 4;
    for (int c = 0; c < 2; ++c) {
      sWr[c][rp] = (double)as[(row + 0 + c) * nl + il];
      sQ[c][rp] = (double)as[(row + 2 + c) * nl + il];
      sS[c][rp] = (double)av[(row + 0 + c) * nl + il] * g.rp[rp];  // r S
      sTor[c][rp] = (double)av[(row + 2 + c) * nl + il];
    }
  }
  // cleaned state u at the N nodes
  for (int j = tid; j < N; j += blockDim.x) {
    for (int f = 0; f < 3; ++f) {
      long long o = 2LL * ((long long)N * ((long long)f * g.S + lm) + j);
      double re = (o == J) ? 0.0 : vb[o];
      double im = (k == 0 || o + 1 == J) ? 0.0 : vb[o + 1];
      if (f < 2 && l == 0) re = im = 0.0;
      su[f][0][j] = re;
      su[f][1][j] = im;
    }
  }
  __syncthreads();
  for (int rp = tid; rp < Np; rp += blockDim.x) {
    double r = g.rp[rp];
    for (int c = 0; c < 2; ++c) {
      double d = 0.0;
      for (int q = 0; q < Np; ++q) d += g.Dp[(long long)rp * Np + q] * sS[c][q];
      sTf[c][rp] = lam / (r * r) * (sWr[c][rp] - d);
      sTor[c][rp] = lam / r * sTor[c][rp];
    }
  }
  __syncthreads();
  for (int j = tid; j < N; j += blockDim.x) {
    double ne[2] = {0, 0}, nf[2] = {0, 0}, nt[2] = {0, 0};
    const double* Pr = g.P + (long long)j * Np;
    for (int q = 0; q < Np; ++q) {
      double pw = Pr[q];
      for (int c = 0; c < 2; ++c) {
        ne[c] += pw * sTor[c][q];
        nf[c] += pw * sTf[c][q];
        nt[c] += pw * sQ[c][q];
      }
    }
    double r = g.r[j];
    double a = ph.Ek * lam / (r * r);
    double d2f[2] = {0, 0};
    const double* D2r = g.D2 + (long long)j * N;
    for (int i = 0; i < N; ++i) {
      d2f[0] += D2r[i] * su[1][0][i];
      d2f[1] += D2r[i] * su[1][1][i];
    }
    double Mu[3][2];
    for (int c = 0; c < 2; ++c) {
      Mu[0][c] = a * su[0][c][j];
      Mu[1][c] = -a * (d2f[c] - lam / (r * r) * su[1][c][j]);
      Mu[2][c] = su[2][c][j];
    }
    double nn[3][2] = {{ne[0], ne[1]}, {nf[0], nf[1]}, {nt[0], nt[1]}};
    // buoyancy on the f-equation
    nn[1][0] += ph.Ra * lam * su[2][0][j] / (r * ph.ro);
    nn[1][1] += ph.Ra * lam * su[2][1][j] / (r * ph.ro);
    for (int f = 0; f < 3; ++f) {
      long long o = 2LL * ((long long)N * ((long long)f * g.S + lm) + j);
      // i m C M u  +  i m c M X
      double tr = -m * C * Mu[f][1], ti = m * C * Mu[f][0];
      if (!STEP) {
        tr += -m * cval * MX[o + 1];
        ti += m * cval * MX[o];
      }
      double br = Mu[f][0] + ph.dt * (nn[f][0] + tr);
      double bi = Mu[f][1] + ph.dt * (nn[f][1] + ti);
      bool bc;
      if (f == 1) bc = (j == 0 || j == 1 || j == N - 2 || j == N - 1);
      else bc = (j == 0 || j == N - 1);
      if (bc) {
        br = 0.0;
        bi = 0.0;
        if (STEP && f == 2 && lm == 0 && j == N - 1) br = 1.0;  // T_00(r_i) = 1
      }
      if (f < 2 && l == 0) br = bi = 0.0;
      bb[o] = br;
      bb[o + 1] = bi;
    }
  }
}

// M X for the drift-speed column of the Jacobian: M_e e, M_f f, M_T T on the cleaned state.
__global__ void k_apply_M(DevGrid g, PhysParams ph, const double* __restrict__ X, double* __restrict__ MX) {
  long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int N = g.N;
  long long total = 3LL * g.S * N;
  if (tid >= total) return;
  int j = (int)(tid % N);
  int lm = (int)((tid / N) % g.S);
  int f = (int)(tid / ((long long)N * g.S));
  int k = g.lm_k[lm], l = g.lm_l[lm];
  double lam = (double)l * (l + 1);
  long long o0 = 2LL * ((long long)N * ((long long)f * g.S + lm));
  double r = g.r[j];
  double a = ph.Ek * lam / (r * r);
  double re, im;
  auto rd = [&](int i, int c) -> double {
    if (f < 2 && l == 0) return 0.0;
    if (c == 1 && k == 0) return 0.0;
    return X[o0 + 2 * i + c];
  };
  if (f == 0) {
    re = a * rd(j, 0);
    im = a * rd(j, 1);
  } else if (f == 1) {
    double d0 = 0, d1 = 0;
    for (int i = 0; i < N; ++i) {
      d0 += g.D2[(long long)j * N + i] * rd(i, 0);
      d1 += g.D2[(long long)j * N + i] * rd(i, 1);
    }
    re = -a * (d0 - lam / (r * r) * rd(j, 0));
    im = -a * (d1 - lam / (r * r) * rd(j, 1));
  } else {
    re = rd(j, 0);
    im = rd(j, 1);
  }
  MX[o0 + 2 * j] = re;
  MX[o0 + 2 * j + 1] = im;
}

// ------------------------------------------------------------------------------------------
// K8: block-tridiagonal solve along each (m, class) chain with the equilibrated block LU,
// organised as a segmented scan so that the sequential part is short:
//   forward  z_i = D_i (t_i - Lo_i z_{i-1}),  t = Rg b,  D_i = diag(sc_i) Shat_i^{-1} diag(sr_i)
//   backward x_i = z_i - H_i x_{i+1},         result Cg x
// Inside a segment [a, e]: z_i = zeta_i + Phi_i z_{a-1}, x_i = xi_i + Psi_i x_{e+1}, where zeta
// and xi are the local recurrences started from zero.  Five launches: local forward (per
// segment), forward boundary pass (per chain), local backward with the forward fix-up (per
// segment), backward boundary pass (per chain), final fix-up and output (per block).
// Work vectors live in W[(block*N + j)*vcap + vec] (complex, precision F, scaled space).
struct ChainMeta {
  int start, n, k, first_seg, nseg, pad0, pad1, pad2;
};
struct SegMeta {
  int first_block, len, chain, pidx;
};

template <class F>
struct cpx {
  F re, im;
};

// Stage an N x N complex block (row-major, interleaved) into LDS with coalesced loads.
template <class F>
__device__ inline void stage_block(const F* __restrict__ gmat, cpx<F>* sm, int N) {
  const cpx<F>* src = reinterpret_cast<const cpx<F>*>(gmat);
  for (int i = threadIdx.x; i < N * N; i += blockDim.x) sm[i] = src[i];
}

// acc(j, vv) += sign * sum_q M[j][q] v[q][vv] for the thread's own (j, vv) entries.
template <class F, int VG>
__device__ inline void mv_acc(const cpx<F>* M, const cpx<F>* v, cpx<F>* acc, int N, int nv, F sign) {
  for (int idx = threadIdx.x; idx < N * VG; idx += blockDim.x) {
    int vv = idx % VG, j = idx / VG;
    if (vv >= nv) continue;
    F ar = 0, ai = 0;
    const cpx<F>* Mr = M + j * N;
    for (int q = 0; q < N; ++q) {
      cpx<F> m = Mr[q], x = v[q * VG + vv];
      ar += m.re * x.re - m.im * x.im;
      ai += m.re * x.im + m.im * x.re;
    }
    acc[j * VG + vv].re += sign * ar;
    acc[j * VG + vv].im += sign * ai;
  }
}

template <class F, int VG>
__device__ inline void load_w(const F* __restrict__ W, int vcap, int b, int v0, cpx<F>* dst, int N, int nv) {
  const cpx<F>* src = reinterpret_cast<const cpx<F>*>(W);
  for (int idx = threadIdx.x; idx < N * VG; idx += blockDim.x) {
    int vv = idx % VG, j = idx / VG;
    if (vv < nv) dst[idx] = src[((long long)b * N + j) * vcap + v0 + vv];
  }
}

template <class F, int VG>
__device__ inline void store_w(F* __restrict__ W, int vcap, int b, int v0, const cpx<F>* srcv, int N, int nv) {
  cpx<F>* dst = reinterpret_cast<cpx<F>*>(W);
  for (int idx = threadIdx.x; idx < N * VG; idx += blockDim.x) {
    int vv = idx % VG, j = idx / VG;
    if (vv < nv) dst[((long long)b * N + j) * vcap + v0 + vv] = srcv[idx];
  }
}

template <class F, int VG>
__global__ void __launch_bounds__(256) k_scan_fwd_local(DevGrid g, int nvec, const SegMeta* __restrict__ segs,
                                                        const int* __restrict__ blk_field, const int* __restrict__ blk_lm,
                                                        const F* __restrict__ Sinv, const F* __restrict__ Lo,
                                                        const F* __restrict__ sr, const F* __restrict__ scl,
                                                        const F* __restrict__ Rg, const double* __restrict__ bvec,
                                                        F* __restrict__ W) {
  extern __shared__ unsigned char smem_raw[];
  const int N = g.N;
  cpx<F>* Ms = reinterpret_cast<cpx<F>*>(smem_raw);
  cpx<F>* prev = Ms + N * N;
  cpx<F>* tmp = prev + N * VG;
  const SegMeta sg = segs[blockIdx.x];
  const int v0 = blockIdx.y * VG, nv = min(VG, nvec - v0);
  const long long NN2 = 2LL * N * N, ld = 6LL * N * g.S;
  for (int i = 0; i < sg.len; ++i) {
    const int b = sg.first_block + i;
    const long long o = 2LL * ((long long)N * ((long long)blk_field[b] * g.S + blk_lm[b]));
    __syncthreads();
    for (int idx = threadIdx.x; idx < N * VG; idx += blockDim.x) {
      int vv = idx % VG, j = idx / VG;
      if (vv >= nv) continue;
      const double* bp = bvec + (long long)(v0 + vv) * ld + o + 2 * j;
      F rg = Rg[(long long)b * N + j];
      tmp[idx].re = rg * (F)bp[0];
      tmp[idx].im = rg * (F)bp[1];
    }
    if (i > 0) {
      stage_block(Lo + NN2 * b, Ms, N);
      __syncthreads();
      mv_acc<F, VG>(Ms, prev, tmp, N, nv, (F)-1);
    }
    for (int idx = threadIdx.x; idx < N * VG; idx += blockDim.x) {
      int j = idx / VG;
      F s = sr[(long long)b * N + j];
      tmp[idx].re *= s;
      tmp[idx].im *= s;
    }
    __syncthreads();
    stage_block(Sinv + NN2 * b, Ms, N);
    for (int idx = threadIdx.x; idx < N * VG; idx += blockDim.x) prev[idx].re = prev[idx].im = 0;
    __syncthreads();
    mv_acc<F, VG>(Ms, tmp, prev, N, nv, (F)1);
    for (int idx = threadIdx.x; idx < N * VG; idx += blockDim.x) {
      int j = idx / VG;
      F c = scl[(long long)b * N + j];
      prev[idx].re *= c;
      prev[idx].im *= c;
    }
    __syncthreads();
    store_w<F, VG>(W, g.vcap, b, v0, prev, N, nv);
  }
}

// z at the end of each segment: z_e(p) = zeta_e(p) + Phi_e(p) z_e(p-1), sequential over p.
template <class F, int VG>
__global__ void __launch_bounds__(256) k_scan_fwd_bound(DevGrid g, int nvec, const ChainMeta* __restrict__ chains,
                                                        const SegMeta* __restrict__ segs, const F* __restrict__ Phi,
                                                        F* __restrict__ W) {
  extern __shared__ unsigned char smem_raw[];
  const int N = g.N;
  cpx<F>* Ms = reinterpret_cast<cpx<F>*>(smem_raw);
  cpx<F>* zb = Ms + N * N;
  cpx<F>* tmp = zb + N * VG;
  const ChainMeta ch = chains[blockIdx.x];
  const int v0 = blockIdx.y * VG, nv = min(VG, nvec - v0);
  if (ch.nseg <= 1) return;
  const long long NN2 = 2LL * N * N;
  SegMeta s0 = segs[ch.first_seg];
  load_w<F, VG>(W, g.vcap, s0.first_block + s0.len - 1, v0, zb, N, nv);
  for (int p = 1; p < ch.nseg; ++p) {
    SegMeta sp = segs[ch.first_seg + p];
    int e = sp.first_block + sp.len - 1;
    __syncthreads();
    load_w<F, VG>(W, g.vcap, e, v0, tmp, N, nv);
    stage_block(Phi + NN2 * e, Ms, N);
    __syncthreads();
    mv_acc<F, VG>(Ms, zb, tmp, N, nv, (F)1);
    __syncthreads();
    for (int idx = threadIdx.x; idx < N * VG; idx += blockDim.x) zb[idx] = tmp[idx];
    store_w<F, VG>(W, g.vcap, e, v0, tmp, N, nv);
  }
}

// Per segment, top-down: z_i = zeta_i + Phi_i z_{a-1} (segments after the first), then the
// local backward recurrence xi_i = z_i - H_i xi_{i+1} started from xi_e = z_e.
template <class F, int VG>
__global__ void __launch_bounds__(256) k_scan_bwd_local(DevGrid g, int nvec, const ChainMeta* __restrict__ chains,
                                                        const SegMeta* __restrict__ segs, const F* __restrict__ Phi,
                                                        const F* __restrict__ H, F* __restrict__ W) {
  extern __shared__ unsigned char smem_raw[];
  const int N = g.N;
  cpx<F>* Ms = reinterpret_cast<cpx<F>*>(smem_raw);
  cpx<F>* prev = Ms + N * N;
  cpx<F>* tmp = prev + N * VG;
  cpx<F>* zin = tmp + N * VG;
  const SegMeta sg = segs[blockIdx.x];
  const int v0 = blockIdx.y * VG, nv = min(VG, nvec - v0);
  const long long NN2 = 2LL * N * N;
  const int e = sg.first_block + sg.len - 1;
  const bool fix = sg.pidx > 0;
  if (fix) load_w<F, VG>(W, g.vcap, sg.first_block - 1, v0, zin, N, nv);  // z_{a-1}: end of previous segment
  load_w<F, VG>(W, g.vcap, e, v0, prev, N, nv);                               // xi_e = z_e
  for (int b = e - 1; b >= sg.first_block; --b) {
    __syncthreads();
    load_w<F, VG>(W, g.vcap, b, v0, tmp, N, nv);
    if (fix) {
      stage_block(Phi + NN2 * b, Ms, N);
      __syncthreads();
      mv_acc<F, VG>(Ms, zin, tmp, N, nv, (F)1);
      __syncthreads();
    }
    stage_block(H + NN2 * b, Ms, N);
    __syncthreads();
    mv_acc<F, VG>(Ms, prev, tmp, N, nv, (F)-1);
    __syncthreads();
    for (int idx = threadIdx.x; idx < N * VG; idx += blockDim.x) prev[idx] = tmp[idx];
    store_w<F, VG>(W, g.vcap, b, v0, tmp, N, nv);
  }
}

// x at the start of each segment: x_a(p) = xi_a(p) + Psi_a(p) x_a(p+1), sequential from the end.
template <class F, int VG>
__global__ void __launch_bounds__(256) k_scan_bwd_bound(DevGrid g, int nvec, const ChainMeta* __restrict__ chains,
                                                        const SegMeta* __restrict__ segs, const F* __restrict__ Psi,
                                                        F* __restrict__ W) {
  extern __shared__ unsigned char smem_raw[];
  const int N = g.N;
  cpx<F>* Ms = reinterpret_cast<cpx<F>*>(smem_raw);
  cpx<F>* xb = Ms + N * N;
  cpx<F>* tmp = xb + N * VG;
  const ChainMeta ch = chains[blockIdx.x];
  const int v0 = blockIdx.y * VG, nv = min(VG, nvec - v0);
  if (ch.nseg <= 1) return;
  const long long NN2 = 2LL * N * N;
  load_w<F, VG>(W, g.vcap, segs[ch.first_seg + ch.nseg - 1].first_block, v0, xb, N, nv);
  for (int p = ch.nseg - 2; p >= 0; --p) {
    int a = segs[ch.first_seg + p].first_block;
    __syncthreads();
    load_w<F, VG>(W, g.vcap, a, v0, tmp, N, nv);
    stage_block(Psi + NN2 * a, Ms, N);
    __syncthreads();
    mv_acc<F, VG>(Ms, xb, tmp, N, nv, (F)1);
    __syncthreads();
    for (int idx = threadIdx.x; idx < N * VG; idx += blockDim.x) xb[idx] = tmp[idx];
    store_w<F, VG>(W, g.vcap, a, v0, tmp, N, nv);
  }
}

// x_i = xi_i + Psi_i x_{a(p+1)} for the blocks not yet final, then x = Cg x~ into the
// canonical output.  One workgroup per (block, vector group).
template <class F, int VG>
__global__ void __launch_bounds__(256) k_scan_out(DevGrid g, int nvec, const int* __restrict__ blk_field,
                                                  const int* __restrict__ blk_lm, const int* __restrict__ blk_next,
                                                  const F* __restrict__ Psi, const F* __restrict__ Cg,
                                                  const F* __restrict__ W, double* __restrict__ xvec) {
  extern __shared__ unsigned char smem_raw[];
  const int N = g.N;
  cpx<F>* Ms = reinterpret_cast<cpx<F>*>(smem_raw);
  cpx<F>* xn = Ms + N * N;
  cpx<F>* acc = xn + N * VG;
  const int b = blockIdx.x;
  const int v0 = blockIdx.y * VG, nv = min(VG, nvec - v0);
  const long long NN2 = 2LL * N * N, ld = 6LL * N * g.S;
  const int nx = blk_next[b];
  load_w<F, VG>(W, g.vcap, b, v0, acc, N, nv);
  if (nx >= 0) {
    load_w<F, VG>(W, g.vcap, nx, v0, xn, N, nv);
    stage_block(Psi + NN2 * b, Ms, N);
    __syncthreads();
    mv_acc<F, VG>(Ms, xn, acc, N, nv, (F)1);
  }
  const long long o = 2LL * ((long long)N * ((long long)blk_field[b] * g.S + blk_lm[b]));
  for (int idx = threadIdx.x; idx < N * VG; idx += blockDim.x) {
    int vv = idx % VG, j = idx / VG;
    if (vv >= nv) continue;
    double c = (double)Cg[(long long)b * N + j];
    double* xp = xvec + (long long)(v0 + vv) * ld + o + 2 * j;
    xp[0] = c * (double)acc[idx].re;
    xp[1] = c * (double)acc[idx].im;
  }
}

// Temperature blocks: x = tc * Tinv (tr * b) per l, for every (vec, k, l), both Re and Im.
template <class F>
__global__ void k_T_solve(DevGrid g, int nvec, const F* __restrict__ Tinv, const F* __restrict__ tr,
                          const F* __restrict__ tc, const double* __restrict__ bvec, double* __restrict__ xvec) {
  long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int N = g.N;
  long long total = (long long)nvec * g.S * N;
  if (tid >= total) return;
  int j = (int)(tid % N);
  int lm = (int)((tid / N) % g.S);
  int vec = (int)(tid / ((long long)N * g.S));
  int l = g.lm_l[lm];
  long long ld = 6LL * N * g.S;
  long long o = (long long)vec * ld + 2LL * ((long long)N * (2LL * g.S + lm));
  const F* Ti = Tinv + (long long)l * N * N + (long long)j * N;
  const F* trl = tr + (long long)l * N;
  F ar = 0, ai = 0;
  for (int i = 0; i < N; ++i) {
    F w = Ti[i] * trl[i];
    ar += w * (F)bvec[o + 2 * i];
    ai += w * (F)bvec[o + 2 * i + 1];
  }
  F c = tc[(long long)l * N + j];
  xvec[o + 2 * j] = (double)(c * ar);
  xvec[o + 2 * j + 1] = (double)(c * ai);
}

// ------------------------------------------------------------------------------------------
// K9: FP64 residual r = b - A x of the implicit operator, applied through the shared radial
// matrices (D, D^2, D^4) rather than stored blocks.  One thread per (vec, field, lm, j).
__device__ inline double kappa_dev(int l, int m) {
  if (l <= 1 || l <= m) return 0.0;
  double ll = l;
  return (ll * ll - 1.0) * sqrt((ll * ll - (double)m * m) / (4.0 * ll * ll - 1.0));
}

__global__ void k_residual64(DevGrid g, PhysParams ph, int nvec, const double* __restrict__ bvec,
                             const double* __restrict__ xvec, double* __restrict__ rvec) {
  long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int N = g.N;
  long long total = (long long)nvec * 3 * g.S * N;
  if (tid >= total) return;
  int j = (int)(tid % N);
  long long t2 = tid / N;
  int lm = (int)(t2 % g.S);
  long long t3 = t2 / g.S;
  int f = (int)(t3 % 3);
  int vec = (int)(t3 / 3);
  int k = g.lm_k[lm], l = g.lm_l[lm];
  int m = k * g.m0;
  long long ld = 6LL * N * g.S;
  const double* x = xvec + (long long)vec * ld;
  long long o = 2LL * ((long long)N * ((long long)f * g.S + lm));
  double br = bvec[(long long)vec * ld + o + 2 * j], bi = bvec[(long long)vec * ld + o + 2 * j + 1];
  double* rr = rvec + (long long)vec * ld + o + 2 * j;
  if (f < 2 && l == 0) {
    rr[0] = 0.0;
    rr[1] = 0.0;
    return;
  }
  const double* xs = x + o;
  double r = g.r[j], r2 = r * r;
  double lam = (double)l * (l + 1);
  const double* Dr = g.D + (long long)j * N;
  const double* D2r = g.D2 + (long long)j * N;
  double ar, ai;
  if (f == 2) {
    if (j == 0 || j == N - 1) {
      ar = xs[2 * j];
      ai = xs[2 * j + 1];
    } else {
      double d1r = 0, d1i = 0, d2r = 0, d2i = 0;
      for (int i = 0; i < N; ++i) {
        d1r += Dr[i] * xs[2 * i];
        d1i += Dr[i] * xs[2 * i + 1];
        d2r += D2r[i] * xs[2 * i];
        d2i += D2r[i] * xs[2 * i + 1];
      }
      double Kr = (d2r + 2.0 / r * d1r - lam / r2 * xs[2 * j]) / ph.Pr;
      double Ki = (d2i + 2.0 / r * d1i - lam / r2 * xs[2 * j + 1]) / ph.Pr;
      ar = xs[2 * j] - ph.dt * Kr;
      ai = xs[2 * j + 1] - ph.dt * Ki;
    }
  } else {
    bool bc = (f == 0) ? (j == 0 || j == N - 1) : (j == 0 || j == 1 || j == N - 2 || j == N - 1);
    if (bc) {
      if (j == 0 || j == N - 1) {
        ar = xs[2 * j];
        ai = xs[2 * j + 1];
      } else {
        const double* Db = g.D + (long long)((j == 1) ? 0 : N - 1) * N;
        ar = ai = 0.0;
        for (int i = 0; i < N; ++i) {
          ar += Db[i] * xs[2 * i];
          ai += Db[i] * xs[2 * i + 1];
        }
      }
    } else {
      double a = ph.Ek * lam / r2;
      double cr, ci;  // self part
      if (f == 0) {
        double d2r = 0, d2i = 0;
        for (int i = 0; i < N; ++i) {
          d2r += D2r[i] * xs[2 * i];
          d2i += D2r[i] * xs[2 * i + 1];
        }
        double Lr = d2r - lam / r2 * xs[2 * j], Li = d2i - lam / r2 * xs[2 * j + 1];
        // a e - dt (a L e + (2 i m / r^2) e)
        cr = a * xs[2 * j] - ph.dt * (a * Lr - 2.0 * m / r2 * xs[2 * j + 1]);
        ci = a * xs[2 * j + 1] - ph.dt * (a * Li + 2.0 * m / r2 * xs[2 * j]);
      } else {
        const double* D4r = g.D4 + (long long)j * N;
        double d2r = 0, d2i = 0, d4r = 0, d4i = 0, q2r = 0, q2i = 0;
        for (int i = 0; i < N; ++i) {
          double xr = xs[2 * i], xi = xs[2 * i + 1];
          double ir2 = 1.0 / (g.r[i] * g.r[i]);
          d2r += D2r[i] * xr;
          d2i += D2r[i] * xi;
          d4r += D4r[i] * xr;
          d4i += D4r[i] * xi;
          q2r += D2r[i] * xr * ir2;
          q2i += D2r[i] * xi * ir2;
        }
        double xr = xs[2 * j], xi = xs[2 * j + 1];
        double Lr = d2r - lam / r2 * xr, Li = d2i - lam / r2 * xi;
        double L2r = d4r - lam * q2r - lam / r2 * d2r + lam * lam / (r2 * r2) * xr;
        double L2i = d4i - lam * q2i - lam / r2 * d2i + lam * lam / (r2 * r2) * xi;
        // -a L f - dt(-a L^2 f - (2 i m/r^2) L f)
        cr = -a * Lr + ph.dt * (a * L2r - 2.0 * m / r2 * Li);
        ci = -a * Li + ph.dt * (a * L2i + 2.0 * m / r2 * Lr);
      }
      // Coriolis coupling to the other potential at l-1 and l+1 (same m)
      int fo = 1 - f;
      for (int nb = -1; nb <= 1; nb += 2) {
        int ln = l + nb;
        if (ln < max(m, 1) || ln > g.L) continue;
        double kap = (nb < 0) ? kappa_dev(l, m) : kappa_dev(l + 1, m);
        if (kap == 0.0) continue;
        double c = (nb < 0) ? (double)l : -(l + 1.0);
        const double* xn = x + 2LL * ((long long)N * ((long long)fo * g.S + lm + nb));
        double dr = 0, di = 0;
        for (int i = 0; i < N; ++i) {
          dr += Dr[i] * xn[2 * i];
          di += Dr[i] * xn[2 * i + 1];
        }
        double pre = ph.dt * 2.0 / r2 * kap;
        cr += pre * (c / r * xn[2 * j] - dr);
        ci += pre * (c / r * xn[2 * j + 1] - di);
      }
      ar = cr;
      ai = ci;
    }
  }
  rr[0] = br - ar;
  rr[1] = bi - ai;
}

// x += d (FP64), over n elements
__global__ void k_axpy1(long long n, const double* __restrict__ d, double* __restrict__ x) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] += d[i];
}

// y = clean(x) - u, u = v with u_J = 0; clean(x) zeroes e/f at l=0 and Im at m=0.
__global__ void k_finalize(DevGrid g, int nvec, const double* __restrict__ x, const double* __restrict__ v,
                           long long ldv, long long J, double* __restrict__ y, long long ldy, int subtract) {
  long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long ld = 6LL * g.N * g.S;
  long long total = (long long)nvec * ld;
  if (tid >= total) return;
  long long i = tid % ld;
  int vec = (int)(tid / ld);
  int c = (int)(i & 1);
  long long node = i / 2;
  int lm = (int)((node / g.N) % g.S);
  int f = (int)(node / ((long long)g.N * g.S));
  int k = g.lm_k[lm], l = g.lm_l[lm];
  double xv = x[(long long)vec * ld + i];
  if ((f < 2 && l == 0) || (c == 1 && k == 0)) xv = 0.0;
  double u = 0.0;
  if (subtract) u = (i == J) ? 0.0 : v[(long long)vec * ldv + i];
  y[(long long)vec * ldy + i] = xv - u;
}

// Sum of squares per vector into out[vec] (deterministic: one block per vector).
__global__ void k_sumsq(long long n, const double* __restrict__ x, long long ld, double* __restrict__ out) {
  __shared__ double red[256];
  const double* xv = x + (long long)blockIdx.x * ld;
  double s = 0.0;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) s += xv[i] * xv[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

}  // namespace sc
