// Device kernels of the rotating-shell IMEX step / Jacobian action (gfx950).
// Internal to libshellconv; included by api.hip only.
//
// Data layouts (nv = vectors in the batch, q = field component, ri = Re/Im):
//   canonical state  v[vec][field e,f,T][lm][j][ri]          (FP64; lm packs (m, l))
//   synthesis input  Gs[k][(vec, q<3, ri, rp)][l-m]  Gv[k][groups of four rows, syn_vec_row][l-m]
//                    (operand order)
//   synthesis output Cs[k][(vec, q<3, ri, rp)][theta]  Cv[k][(vec, f<12, rp)][theta] (the six
//                    vector fields U_th, U_ph, w_th, w_ph, dT/dth, dT/dph, Re and Im)
//   analysis input   Fs[k][(vec, rp, q<2, ri)][theta]  Fv[k][(vec, rp, q<2, ri)][2 nth] (dP half,
//                    m P/sin half; only the dP half is written while the folded analysis runs)
//   analysis output  As[k][(l-m)/8][(vec, rp, q<2, ri)][(l-m)%8]  (likewise Av; the GEMM
//                    fallback writes As[k][(vec, rp, q<2, ri)][l-m])
//   base fields      base[rp][field<9][phi][theta]
// The Legendre transforms are the contractions C[i][j] = sum_k A[i][k] B[j][k] with both
// operands contiguous in k (gemm_batched).
#pragma once
#include <hip/hip_runtime.h>
#include <type_traits>

namespace sc {

struct GemmProb {
  long long a_off, b_off, c_off;  // element offsets: A, C in the workspace, B in the tables
  int Mper, N, K, lda, ldb, ldc;  // M = Mper * nvec
};

struct DevGrid {
  int L, m0, N, Np, nth, nphi, K, S;
  int vcap;           // vector capacity of the workspaces (block strides use it)
  int wcap;           // column stride of the chain-solve work vectors (vcap rounded up to 16)
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
  // transposed copies ([column][row]) for coalesced row-parallel products
  const double* ET;   // [N][Np]: E^T
  const double* EDT;
  const double* ED2T;
  const double* DT;   // [N][N]
  const double* D2T;
  const double* D4T;
  const int2* rtiles; // radial-prep tiles: (k, first l-m), up to 16 l
  int nrtiles;
  const double* PT;   // [Np][N]: P^T
  const double* DpT;  // [Np][Np]: Dp^T
  const int2* ptiles; // projection tiles: (k, first l-m)
  int nptiles;
  const int2* qtiles; // residual tiles: (k, first l-m)
  int nqtiles;
  const double* DF;   // D (N x N), operand order
  const double* D4F;  // D^4 (N x N), operand order
  const long long* gsoff;  // per m: offsets of the synthesis inputs in operand order, from Gs and from Gv
  int rtcS, rtcV;     // row tiles of the scalar / vector synthesis inputs at vector capacity
  const double* EF;   // E, ED, ED2 (N_p x N each) in 16x16x4 MFMA operand order, k padded to 16 ceil(N/16)
  const double* PF;   // P diag(1/r), P diag(1/r^2), P diag(1/r^2) Dp diag(r), P (N x N_p each), operand order
  const double* D2F;  // D^2 (N x N), operand order
  int fft_nr;         // azimuthal FFT: number of passes and their radices (each 2, 3, 4 or 5)
  int fft_r[8];
  // analysis outputs: tiled ([m][l-m tile of 8][row][8], m blocks at lmbase8) when ana_tiled,
  // else [m][row][l-m] at lmbase
  int ana_tiled;
  const int* lmbase8;
  // the vector analysis inputs hold only their dP half: the m P/sin half of a row group
  // (-D3, D2, D1, -D0) is a signed permutation of its dP half (D0..D3), and the folded analysis
  // takes it from there
  int fv_dp_only;
  // explicit-Coriolis variant (Sec. 3.1, eq:defineFexp): the ring products add -2 e_z x U to the
  // force; cst holds cos(theta_j), sin(theta_j) of the Gauss-Legendre nodes ([2][nth])
  int cor_explicit;
  const double* cst;
};

struct PhysParams {
  double Ek, Ra, Pr, dt, ro;
  double cor;   // weight of the Coriolis terms of the implicit operator (1, or 0 when explicit)
};

// Final output of a Jacobian action, written by the last solve: y = clean(x) - u, where clean
// zeroes e, f at l = 0 and Im at m = 0, and u = v with the phase slot J read as 0.
struct FinalOut {
  const double* v;
  long long ldv, J;
  double* y;
  long long ldy;
};

__device__ inline double final_value(const FinalOut& fo, int vec, long long o, double x) {
  const double u = (o == fo.J) ? 0.0 : fo.v[(long long)vec * fo.ldv + o];
  return x - u;
}

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on XCD b % 8), each
// with its own L2.  This maps blockIdx.x to a linear id such that every XCD receives one
// contiguous range of ids (a bijection on [0, gridDim.x)).
__device__ inline int xcd_linear_id() {
  const int b = blockIdx.x, G = gridDim.x;
  const int x = b & 7, q = G >> 3, r = G & 7;
  return x * q + min(x, r) + (b >> 3);
}

// Calls f(std::integral_constant<int, n>) for the runtime count 1 <= n <= NMAX (wave-uniform), so
// that loops over n tiles have a compile-time trip count and no per-tile branch.
template <int NMAX, class Fn>
__device__ inline void with_count(int n, Fn&& f) {
  if constexpr (NMAX >= 1) {
    if (n == NMAX) {
      f(std::integral_constant<int, NMAX>());
      return;
    }
    with_count<NMAX - 1>(n, f);
  }
}

// Cooperative copy into LDS by the workgroup: element i (i = tid, tid + blockDim, ... < total)
// is ld(i) stored by st(i, value).  The loads of CH consecutive rounds are all issued before the
// first store, so a thread waits for memory once per CH elements, not per element.
template <int CH, class V, class LoadF, class StoreF>
__device__ inline void staged_copy(int total, LoadF ld, StoreF st) {
  const int nt = blockDim.x;
  for (int b = threadIdx.x; b < total; b += CH * nt) {
    V v[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int i = b + u * nt;
      v[u] = (i < total) ? ld(i) : V{};
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int i = b + u * nt;
      if (i < total) st(i, v[u]);
    }
  }
}

// Matrix-core (MFMA) 16x16x4 tile per wavefront: D[16][16] += A[16][4] B[4][16].
// Lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; element q of its 4-vector holds
// D[out_row(l, q)][l % 16], with out_row = 4 (l / 16) + q for FP32 and l / 16 + 4 q for FP64
// (both checked on gfx950 with a probe kernel).
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
template <class T>
struct Mfma;
template <>
struct Mfma<float> {
  typedef f32x4 acc_t;
  static __device__ inline acc_t step(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static __device__ inline int out_row(int lane, int q) { return 4 * (lane >> 4) + q; }
};
template <>
struct Mfma<double> {
  typedef f64x4 acc_t;
  static __device__ inline acc_t step(double a, double b, acc_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  static __device__ inline int out_row(int lane, int q) { return (lane >> 4) + 4 * q; }
};

// ------------------------------------------------------------------------------------------
// Real matrices in 16x16x4 MFMA operand order: for R row tiles and KS k-steps, lane l of
// (row tile t, k-step s) holds M[16t + l%16][4s + l/16] (zero outside the matrix), at
// ((t KS + s) 64 + l).  A wavefront then loads its A operands with unit-stride loads.

// acc[p] += M_p X_p over k < 16 KB for NPR independent products on one 16-row tile: Mp[p] is
// this lane's element of k-step 0 of the tile (k-step stride 64), Xp[p] the LDS column of X_p
// (row k at Xp[p][k ldx]).  The operands of the next 16-wide k block load while the current
// block multiplies.
template <int NPR, class TX>
__device__ inline void mfma_f64_products(const double* const (&Mp)[NPR], const TX* const (&Xp)[NPR], int ldx, int KB,
                                         int l, f64x4 (&acc)[NPR]) {
  double a0[NPR][4], a1[NPR][4];
  auto load = [&](int kb, double (&a)[NPR][4]) {
    kb = kb < KB ? kb : KB - 1;
#pragma unroll
    for (int p = 0; p < NPR; ++p)
#pragma unroll
      for (int st = 0; st < 4; ++st) a[p][st] = Mp[p][(4 * kb + st) * 64];
  };
  auto run = [&](int kb, const double (&a)[NPR][4]) {
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int row = 16 * kb + 4 * st + (l >> 4);
#pragma unroll
      for (int p = 0; p < NPR; ++p) acc[p] = Mfma<double>::step(a[p][st], (double)Xp[p][row * ldx], acc[p]);
    }
  };
  // k blocks in pairs with no branch inside (a load used only in a conditional block is sunk
  // into it, behind the products it should overlap); an odd last block runs after the loop
  load(0, a0);
  int kb = 0;
  for (; kb + 1 < KB; kb += 2) {
    load(kb + 1, a1);
    __builtin_amdgcn_sched_barrier(0);
    run(kb, a0);
    load(kb + 2, a0);
    __builtin_amdgcn_sched_barrier(0);
    run(kb + 1, a1);
  }
  if (kb < KB) run(kb, a0);
}

// ------------------------------------------------------------------------------------------
// Rows of the vector synthesis operand.  The five complex vector profiles (S_u, T_u, S_w, T_w,
// T) form groups of four real rows (members): per vector, groups [0, N_p) are (S_u, T_u) and
// [N_p, 2 N_p) are (S_w, T_w) at r_p = G mod N_p, and groups [2 N_p, 2 N_p + ceil(N_p/2)) are
// (T at r_p = 2 j, T at r_p = 2 j + 1); syn_vec_groups(N_p) groups per vector.  Sixteen
// consecutive groups share four 16-row tiles, member q in tile 4 (G/16) + q at row G % 16: a
// synthesis workgroup owns such a set of four row tiles, so every lane holds the four members
// of its groups at the same output position and combines them into the physical fields
// (U_th, U_ph), (w_th, w_ph) or (dT/dth, dT/dph) in registers; consecutive r_p stay
// consecutive rows.
__host__ __device__ inline long long syn_vec_row(long long G, int q) {
  return ((G >> 4) * 4 + q) * 16 + (G & 15);
}
__host__ __device__ inline int syn_vec_groups(int Np) { return 2 * Np + (Np + 1) / 2; }
// Row tiles of the vector synthesis operand for n groups.
__host__ __device__ inline int syn_vec_tiles(long long n) { return (int)(4 * ((n + 15) / 16)); }

// K1: radial preparation.  For each (vec, r_p, lm): the eight spectral profiles
//   ur = lam f/r^2, wr = lam e/r^2, dT = T'   (scalar synthesis with Pbar)
//   Su = f'/r, Tu = e/r, Sw = e'/r, Tw = -(f'' - lam f/r^2)/r, ST = T/r  (vector synthesis)
// evaluated at the N_p nodes as diag(r^-k) E D^j u, in FP64, stored in precision T.
// Input cleaning: Im at m = 0, e/f at l = 0 and the phase slot J are read as 0.
constexpr int kRPT = 16;      // l per radial-prep tile

// The work of one wavefront: NT column tiles (ct0, ct0 + 4) of one field class, NP products
// each (E, ED and, for f, ED2).  Kept separate per wave kind so that each holds only its own
// operands.
template <class T, int RTN, int NT, int NP>
__device__ inline void radial_prep_wave(const DevGrid& g, const double* __restrict__ vb, long long J, int vec, int k,
                                        int il0, int ct0, T* __restrict__ Gs, T* __restrict__ Gv) {
  constexpr int KS = 4 * RTN;           // k-steps over the N nodes
  constexpr int QB = KS / 4;            // k-steps per operand block (a quarter row tile)
  const int N = g.N, Np = g.Np;
  const int RTP = (Np + 15) / 16;
  const int m = k * g.m0, nl = g.L - m + 1;
  const int nt = min(kRPT, nl - il0);
  const int lm0 = g.lmbase[k] + il0;
  const int l = threadIdx.x & 63, t = l & 15;
  // X^T operands: lane l of k-step s holds X[4 s + l/16][column t] of its tile
  double xb[NT][KS];
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    const int ct = ct0 + 4 * u, f = ct >> 1, c = ct & 1;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int j = 4 * s + (l >> 4);
      double val = 0.0;
      if (j < N && t < nt) {
        const long long o = 2LL * ((long long)N * ((long long)f * g.S + lm0 + t) + j) + c;
        val = vb[o];
        if (o == J || (c == 1 && k == 0) || (f < 2 && m + il0 + t == 0)) val = 0.0;
      }
      xb[u][s] = val;
    }
  }
  const long long mstride = (long long)RTP * KS * 64;
  // Synthesis operand order: row r = (vec ns + slot) Np + r_p of the sums, depth column kc of
  // degree il (even l - m at il/2, odd ones at 4 KSe + il/2) at
  // ((r/16) KSl + kc/4) 64 + (kc%4) 16 + r%16.
  const long long offS = g.gsoff[2 * k], offV = g.gsoff[2 * k + 1];
  const int KSe = ((nl + 1) / 2 + 3) >> 2, KSo = (nl / 2 + 3) >> 2, KSl = KSe + KSo;
  // E operands in quarter row tiles, the next block loading while the current one multiplies:
  // block b = 4 rt + h
  double ea[NP][QB], eb[NP][QB];
  auto load_blk = [&](int b, double (&a)[NP][QB]) {
    b = b < 4 * RTP ? b : 4 * RTP - 1;
    const double* F = g.EF + (long long)(b >> 2) * KS * 64 + (b & 3) * QB * 64 + l;
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int s = 0; s < QB; ++s) a[p][s] = F[p * mstride + s * 64];
  };
  f64x4 acc[NT][NP];
  auto run_blk = [&](int h, const double (&a)[NP][QB]) {
#pragma unroll
    for (int s = 0; s < QB; ++s)
#pragma unroll
      for (int u = 0; u < NT; ++u)
#pragma unroll
        for (int p = 0; p < NP; ++p) acc[u][p] = Mfma<double>::step(xb[u][h * QB + s], a[p][s], acc[u][p]);
  };
  load_blk(0, ea);
  for (int rt = 0; rt < RTP; ++rt) {
#pragma unroll
    for (int u = 0; u < NT; ++u)
#pragma unroll
      for (int p = 0; p < NP; ++p) acc[u][p] = f64x4{0, 0, 0, 0};
#pragma unroll
    for (int h = 0; h < 4; h += 2) {
      load_blk(4 * rt + h + 1, eb);
      __builtin_amdgcn_sched_barrier(0);
      run_blk(h, ea);
      load_blk(4 * rt + h + 2, ea);
      __builtin_amdgcn_sched_barrier(0);
      run_blk(h + 1, eb);
    }
    // epilogue: this lane's r_p, four degrees (element q: degree il0 + l/16 + 4 q)
    const int rp = 16 * rt + t;
    if (rp >= Np) continue;
    const double ri1 = 1.0 / g.rp[rp], ri2 = ri1 * ri1;
    const long long rs = (long long)vec * 6 * Np + rp, gv0 = (long long)vec * syn_vec_groups(Np);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int tq = Mfma<double>::out_row(l, q), il = il0 + tq, lw = m + il;
      if (tq >= nt) continue;
      const int kc = (il & 1) ? 4 * KSe + (il >> 1) : (il >> 1);
      const long long kofs = (kc >> 2) * 64 + (kc & 3) * 16;
      const double lam = (double)lw * (lw + 1);
      auto gs = [&](int slot, double val) {
        const long long r = rs + (long long)slot * Np;
        Gs[offS + (r >> 4) * KSl * 64 + kofs + (r & 15)] = (T)val;
      };
      auto gv = [&](int slot, double val) {
        const long long r = slot < 8 ? syn_vec_row(gv0 + (long long)(slot >> 2) * Np + rp, slot & 3)
                                     : syn_vec_row(gv0 + 2LL * Np + (rp >> 1), 2 * (rp & 1) + (slot & 1));
        Gv[offV + (r >> 4) * KSl * 64 + kofs + (r & 15)] = (T)val;
      };
#pragma unroll
      for (int u = 0; u < NT; ++u) {
        const int ct = ct0 + 4 * u, f = ct >> 1, c = ct & 1;
        const double y0 = acc[u][0][q], y1 = acc[u][1][q], y2 = (NP == 3) ? acc[u][NP - 1][q] : 0.0;
        if (f == 0) {          // e
          gs(2 + c, lam * ri2 * y0);                                   // wr
          gv(2 + c, y0 * ri1);                                         // Tu
          gv(4 + c, y1 * ri1);                                         // Sw
        } else if (f == 1) {   // f
          gs(0 + c, lam * ri2 * y0);                                   // ur
          gv(0 + c, y1 * ri1);                                         // Su
          gv(6 + c, -y2 * ri1 + lam * ri2 * ri1 * y0);                 // Tw
        } else {               // T
          gs(4 + c, y1);                                               // dT
          gv(8 + c, y0 * ri1);                                         // ST
        }
      }
    }
  }
}

// K1: one workgroup per (tile of up to 16 consecutive l at one m, vector).  The tile's
// profiles form six 16-column tiles (field, Re/Im) of X; wavefront w owns column tiles w and
// (w < 2) w + 4 (waves 0, 1: an e and a T tile, products E and ED; waves 2, 3: an f tile,
// products E, ED, ED2) and holds their X operands in registers (read once from the state).
// Row tile by row tile it forms (E X)^T = X^T E^T etc. on the FP64 matrix cores, with the E
// operands streamed from L2 a quarter row tile ahead.  A lane then holds 16 consecutive r_p
// of one degree, which are consecutive rows of the synthesis operands (scalar rows ordered
// (vec, slot, r_p); vector rows of consecutive groups, syn_vec_row): the stores write runs of
// 16 contiguous elements (two runs where a vector run crosses a tile).
template <class T, int RTN>
__global__ void __launch_bounds__(256) k_radial_prep(DevGrid g, const double* __restrict__ v, long long ldv,
                                                     long long J, int nvec, T* __restrict__ Gs, T* __restrict__ Gv) {
  const int2 tl = g.rtiles[blockIdx.x];
  const int vec = blockIdx.y;
  const double* vb = v + (long long)vec * ldv;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (w >= 2) radial_prep_wave<T, RTN, 1, 3>(g, vb, J, vec, tl.x, tl.y, w, Gs, Gv);
  else radial_prep_wave<T, RTN, 2, 2>(g, vb, J, vec, tl.x, tl.y, w, Gs, Gv);
}

// ------------------------------------------------------------------------------------------
// K2: Legendre synthesis per m with the equatorial symmetry.  Nodes nth-1-j mirror j; P and
// m P/sin have the parity (-1)^(l-m) under the mirror, dP/dtheta the opposite one.  For the
// northern nodes the sums over even l - m (S_e) and over odd l - m (S_o) are two products
// C_e = A_e B_e, C_o = A_o B_o with half the columns and half the depth; the outputs are then
// S_e + S_o at the node and S_e - S_o (P, m P/sin) or S_o - S_e (dP/dtheta) at its mirror.
// A (spectral profiles, depth [even l | odd l]; scalar rows (vec, q, r_p), vector rows in groups,
// syn_vec_row) and B (tables, northern columns) are stored in MFMA operand order, so every
// wavefront streams its operands from L2 into registers with unit-stride loads, one k-step
// ahead, with no LDS.  A workgroup owns kSynTM row tiles and 4 kSynTN column tiles: for the
// scalar problem wavefront w takes the column tiles w, w+4 and writes C[row][theta]; for the
// vector problem it takes the dP and the m P/sin tile of the same nodes and writes the six
// fields C[(vec, field row, r_p)][theta].
constexpr int kSynTM = 4;
constexpr int kSynTN = 2;

struct SynProb {
  long long a_off, b_off, c_off;  // A, C in the workspace; B in the tables (even part, then odd)
  int rper;                        // rows per vector (6 N_p; vector: 4 syn_vec_groups(N_p))
  int kse, kso;                    // k-steps of the even and odd parts
  int cth;                         // column tiles of one part (ceil(nth/2 / 16))
  int parts;                       // 1 (scalar: P) or 2 (vector: dP, m P/sin)
  int nth;                         // theta nodes; C rows have parts * nth columns
  int np;                          // N_p
};

__host__ __device__ inline int syn_row_tiles(const SynProb& p, int nvec) {
  return p.parts == 2 ? syn_vec_tiles((long long)syn_vec_groups(p.np) * nvec) : (p.rper * nvec + 15) / 16;
}

__host__ __device__ inline int syn_tiles(const SynProb& p, int nvec) {
  const int rt = syn_row_tiles(p, nvec);
  return ((rt + kSynTM - 1) / kSynTM) * ((p.parts * p.cth + 4 * kSynTN - 1) / (4 * kSynTN));
}

template <class T>
__global__ void __launch_bounds__(256) k_synth(const SynProb* __restrict__ probs, int nprob,
                                               const int2* __restrict__ lut, int nvec,
                                               const T* __restrict__ ws_in, const T* __restrict__ tab,
                                               T* __restrict__ ws_out) {
  typedef typename Mfma<T>::acc_t acc_t;
  int tile = blockIdx.x, p = 0;
  if (lut) {   // (problem, tile) of this workgroup, one load
    const int2 pt = lut[blockIdx.x];
    p = pt.x;
    tile = pt.y;
  } else {
    for (; p < nprob; ++p) {
      const int nt = syn_tiles(probs[p], nvec);
      if (tile < nt) break;
      tile -= nt;
    }
    if (p >= nprob) return;
  }
  const SynProb pr = probs[p];
  const int ct = pr.parts * pr.cth, ks = pr.kse + pr.kso;
  const int ncg = (ct + 4 * kSynTN - 1) / (4 * kSynTN);
  const int rg = tile / ncg, cg = tile - rg * ncg;
  const int rows = pr.rper * nvec, rtu = syn_row_tiles(pr, nvec);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const T* A[kSynTM];
  const T* Be[kSynTN];
  const T* Bo[kSynTN];
  int rt[kSynTM], ctl[kSynTN];
#pragma unroll
  for (int i = 0; i < kSynTM; ++i) {
    rt[i] = rg * kSynTM + i;
    A[i] = ws_in + pr.a_off + (long long)min(rt[i], rtu - 1) * ks * 64 + l;
  }
  int ncol = 0;
  const long long bodd = (long long)ct * pr.kse * 64;  // odd tables follow the even ones
  // vector problems: the wavefront's two column tiles are the dP and the m P/sin tile of the
  // same nodes (both parts of a field meet in one lane)
  const bool vec2 = pr.parts == 2;
  static_assert(kSynTN == 2, "column tile pairs of the vector problems");
#pragma unroll
  for (int j = 0; j < kSynTN; ++j) {
    ctl[j] = vec2 ? j * pr.cth + cg * 4 + w : cg * 4 * kSynTN + w + 4 * j;
    if (vec2 ? (cg * 4 + w < pr.cth) : (ctl[j] < ct)) ncol = j + 1;
    const int cc = min(ctl[j], ct - 1);
    Be[j] = tab + pr.b_off + (long long)cc * pr.kse * 64 + l;
    Bo[j] = tab + pr.b_off + bodd + (long long)cc * pr.kso * 64 + l;
  }
  acc_t ce[kSynTM][kSynTN], co[kSynTM][kSynTN];
#pragma unroll
  for (int i = 0; i < kSynTM; ++i)
#pragma unroll
    for (int j = 0; j < kSynTN; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        ce[i][j][q] = (T)0;
        co[i][j][q] = (T)0;
      }
  // one pipelined pass over a part: A k-steps [k0, k0 + n), tables B.  The loop takes the
  // k-steps in pairs with no branch on the k-step inside (a load used only in a conditional
  // block is sunk into it, behind the products it should overlap, and a select on a loaded value
  // waits for it); an odd last k-step runs after the loop.  In FP32 the column tiles beyond ncol
  // multiply clamped table operands into sums that are never stored (cheaper than the branch,
  // measured); in FP64, where a product costs twice as much, they are skipped.
  auto pass = [&](int k0, int n, const T* const* B, acc_t (&acc)[kSynTM][kSynTN]) {
    if (n <= 0) return;
    T a0[kSynTM], b0[kSynTN], a1[kSynTM], b1[kSynTN];
    auto load = [&](int st, T* a, T* b) {
      st = st < n ? st : n - 1;
#pragma unroll
      for (int i = 0; i < kSynTM; ++i) a[i] = A[i][(k0 + st) * 64];
#pragma unroll
      for (int j = 0; j < kSynTN; ++j) b[j] = B[j][st * 64];
    };
    auto run = [&](const T* a, const T* b) {
#pragma unroll
      for (int j = 0; j < kSynTN; ++j)
        if (sizeof(T) == 4 || j < ncol) {
#pragma unroll
          for (int i = 0; i < kSynTM; ++i) acc[i][j] = Mfma<T>::step(a[i], b[j], acc[i][j]);
        }
    };
    load(0, a0, b0);
    int st = 0;
    for (; st + 1 < n; st += 2) {
      load(st + 1, a1, b1);
      __builtin_amdgcn_sched_barrier(0);
      run(a0, b0);
      load(st + 2, a0, b0);
      __builtin_amdgcn_sched_barrier(0);
      run(a1, b1);
    }
    if (st < n) run(a0, b0);
  };
  pass(0, pr.kse, Be, ce);
  pass(pr.kse, pr.kso, Bo, co);
  T* C = ws_out + pr.c_off;
  const int nh = pr.nth >> 1, ncolC = pr.parts * pr.nth;
  if (vec2) {
    // the four row tiles of this workgroup hold the members q = 0..3 of sixteen groups; element
    // e of a lane is group 16 rg + out_row(l, e).  With D the dP sums and M the m P/sin sums:
    // a group (a, b) of two profiles gives the fields (D a + i M b, i M a - D b), i.e.
    // (U_th, U_ph) from (S_u, T_u) and (w_th, w_ph) from (S_w, T_w); a group (T, T') of two
    // nodes gives (dT/dth, dT/dph) = (D T, i M T) at both.  Output rows (vec, field row
    // 0..11, r_p), nth columns.
    static_assert(kSynTM == 4, "one row tile per member");
    if (ncol == 0) return;
    const int tn = (cg * 4 + w) * 16 + (l & 15);  // northern node
    if (tn >= nh) return;
    const int ts = pr.nth - 1 - tn, Np = pr.np, GP = syn_vec_groups(Np);
    const long long fs = (long long)Np * pr.nth;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int G = rg * 16 + Mfma<T>::out_row(l, e);
      if (G >= GP * nvec) continue;
      const int vec = G / GP, rem = G - vec * GP;
      T Dn[4], Ds[4], Mn[4], Ms[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const T de = ce[q][0][e], dd = co[q][0][e], me = ce[q][1][e], mo = co[q][1][e];
        Dn[q] = de + dd;   // dP: north e + o, south o - e
        Ds[q] = dd - de;
        Mn[q] = me + mo;   // m P/sin: north e + o, south e - o
        Ms[q] = me - mo;
      }
      if (rem < 2 * Np) {
        const int gg = rem >= Np ? 1 : 0, rp = rem - gg * Np;
        T* cr = C + ((long long)(vec * 12 + 4 * gg) * Np + rp) * pr.nth;
        cr[0 * fs + tn] = Dn[0] - Mn[3];
        cr[1 * fs + tn] = Dn[1] + Mn[2];
        cr[2 * fs + tn] = -Mn[1] - Dn[2];
        cr[3 * fs + tn] = Mn[0] - Dn[3];
        cr[0 * fs + ts] = Ds[0] - Ms[3];
        cr[1 * fs + ts] = Ds[1] + Ms[2];
        cr[2 * fs + ts] = -Ms[1] - Ds[2];
        cr[3 * fs + ts] = Ms[0] - Ds[3];
      } else {
        const int rp = 2 * (rem - 2 * Np);
        T* cr = C + ((long long)(vec * 12 + 8) * Np + rp) * pr.nth;
        cr[0 * fs + tn] = Dn[0];
        cr[1 * fs + tn] = Dn[1];
        cr[2 * fs + tn] = -Mn[1];
        cr[3 * fs + tn] = Mn[0];
        cr[0 * fs + ts] = Ds[0];
        cr[1 * fs + ts] = Ds[1];
        cr[2 * fs + ts] = -Ms[1];
        cr[3 * fs + ts] = Ms[0];
        if (rp + 1 < Np) {
          cr += pr.nth;
          cr[0 * fs + tn] = Dn[2];
          cr[1 * fs + tn] = Dn[3];
          cr[2 * fs + tn] = -Mn[3];
          cr[3 * fs + tn] = Mn[2];
          cr[0 * fs + ts] = Ds[2];
          cr[1 * fs + ts] = Ds[3];
          cr[2 * fs + ts] = -Ms[3];
          cr[3 * fs + ts] = Ms[2];
        }
      }
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < kSynTN; ++j) {
    if (j >= ncol) continue;
    const int part = ctl[j] / pr.cth;
    const int tn = (ctl[j] - part * pr.cth) * 16 + (l & 15);  // northern node
    if (tn >= nh) continue;
    const int cn = part * pr.nth + tn, cs = part * pr.nth + pr.nth - 1 - tn;
    const bool dp = (pr.parts == 2 && part == 0);   // mirror value: e - o, or o - e for dP/dtheta
    const T sge = dp ? (T)-1 : (T)1, sgo = dp ? (T)1 : (T)-1;
#pragma unroll
    for (int i = 0; i < kSynTM; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = rt[i] * 16 + Mfma<T>::out_row(l, q);
        if (row >= rows) continue;
        const T e = ce[i][j][q], o = co[i][j][q];
        T* cr = C + (long long)row * ncolC;
        cr[cn] = e + o;
        cr[cs] = sge * e + sgo * o;
      }
  }
}

// ------------------------------------------------------------------------------------------
// K6: Legendre analysis per m with the equatorial symmetry.  The quadrature over the N_theta
// Gauss-Legendre nodes pairs node j with its mirror nth-1-j (equal weights); Pbar and
// m Pbar/sin have parity (-1)^(l-m) under the mirror, dPbar/dtheta the opposite one.  So the
// even-degree outputs contract the folded inputs F(j) + s F(nth-1-j) and the odd-degree ones
// F(j) - s F(nth-1-j) over the northern nodes only, s = +1 for Pbar and m Pbar/sin, -1 for
// dPbar/dtheta: half the depth for each half of the degrees.
// A workgroup owns ROWS rows (vec, r_p, q, Re/Im) of one m and part set (scalar: P; vector:
// the dP part, then the m P/sin part, accumulated).  It folds its rows into LDS ([parity][row]
// [node], rows padded to an odd stride), then wavefront w multiplies row tile w%2 against all
// column tiles of parity w/2, the tables streamed from L2 in MFMA operand order one k-step
// ahead.  Only the dP half of a vector row is stored (the ring kernels skip the other half when
// this kernel runs): the m P/sin operand is a signed row permutation of the dP fold.  Each
// input row is read once.
struct AnaProb {
  long long f_off;   // first input row of this m and part set (Fs or Fv), elements
  long long t_off;   // tables of this m and part set: [part][parity][column tile][k-step][lane]
  long long c_off;   // output (As or Av of this m), rows of nl degrees
  int parts;         // 1 (scalar) or 2 (vector: dP, m P/sin)
  int nl, ldf;       // degrees; input row length (nth or 2 nth)
  int cte, cto;      // column tiles of the even and odd degrees
  int rper;          // rows per vector (4 N_p)
  int rcap;          // rows of an output tile of 8 degrees (4 N_p times the vector capacity)
};
constexpr int kAnaRows = 32;

__host__ __device__ inline int ana_tiles(const AnaProb& p, int nvec) {
  return (p.rper * nvec + kAnaRows - 1) / kAnaRows;
}

template <class T>
__host__ __device__ inline size_t ana_lds_bytes(int nth, int nlmax) {
  // the folded rows, then (reused) the output block of kAnaRows rows x nlmax degrees padded to 8
  const int ksa = (nth / 2 + 3) / 4;
  const size_t fold = (size_t)2 * kAnaRows * (4 * ksa + 1), out = (size_t)kAnaRows * ((nlmax + 7) & ~7);
  return sizeof(T) * (fold > out ? fold : out);
}

template <class T, int CT>
__global__ void __launch_bounds__(256) k_anal(const AnaProb* __restrict__ probs, int nprob,
                                              const int2* __restrict__ lut, int nvec, int nth,
                                              const T* __restrict__ ws_in, const T* __restrict__ tab,
                                              T* __restrict__ ws_out) {
  typedef typename Mfma<T>::acc_t acc_t;
  extern __shared__ unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  int tile = blockIdx.x, p = 0;
  if (lut) {   // (problem, tile) of this workgroup, one load
    const int2 pt = lut[blockIdx.x];
    p = pt.x;
    tile = pt.y;
  } else {
    for (; p < nprob; ++p) {
      const int nt = ana_tiles(probs[p], nvec);
      if (tile < nt) break;
      tile -= nt;
    }
    if (p >= nprob) return;
  }
  const AnaProb pr = probs[p];
  const int nh = nth / 2, KSa = (nh + 3) >> 2, pitch = 4 * KSa + 1;
  const int rows = pr.rper * nvec, r0 = tile * kAnaRows;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), l = threadIdx.x & 63;
  const int rt = w & 1, par = w >> 1;
  const int nct = par ? pr.cto : pr.cte;
  acc_t acc[CT];
#pragma unroll
  for (int c = 0; c < CT; ++c)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[c][q] = (T)0;
  for (int part = 0; part < pr.parts; ++part) {
    // the m P/sin part (part 1) of the vector rows is not stored: within a group of four rows
    // it is (-D3, D2, D1, -D0) of the dP part D, and its fold (sign +1) is the dP fold (sign -1)
    // with the parities exchanged, so its operand is read from the dP fold at the permuted row
    // of the other parity, with that sign
    const bool derived = part == 1;
    if (!derived) {
      // fold this part of the rows into [parity][row][node]: wave w takes rows w, w + 4, ...,
      // lane l nodes l and l + 64 (nh <= 128); all loads of a thread are issued before use
      const T sg = (pr.parts == 2 && part == 0) ? (T)-1 : (T)1;
      constexpr int NI = kAnaRows / 4;
      T va[NI][2], vb[NI][2];
#pragma unroll
      for (int i = 0; i < NI; ++i) {
        const int row = r0 + w + 4 * i;
        const T* fr = ws_in + pr.f_off + (long long)row * pr.ldf + part * nth;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int j = l + 64 * h;
          va[i][h] = (T)0;
          vb[i][h] = (T)0;
          if (row < rows && j < nh) {
            va[i][h] = fr[j];
            vb[i][h] = fr[nth - 1 - j];
          }
        }
      }
#pragma unroll
      for (int i = 0; i < NI; ++i) {
        const int rr = w + 4 * i;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int j = l + 64 * h;
          if (j < 4 * KSa) {
            lds[rr * pitch + j] = va[i][h] + sg * vb[i][h];
            lds[(kAnaRows + rr) * pitch + j] = va[i][h] - sg * vb[i][h];
          }
        }
      }
      __syncthreads();
    }
    if (nct > 0) {
      const int R = 16 * rt + (l & 15), q4 = R & 3;
      const T* Ab = derived ? lds + ((1 - par) * kAnaRows + (R - q4) + (3 - q4)) * pitch + (l >> 4)
                            : lds + (par * kAnaRows + R) * pitch + (l >> 4);
      const T asg = (derived && (q4 == 0 || q4 == 3)) ? (T)-1 : (T)1;
      const T* Bb = tab + pr.t_off + (long long)(part * (pr.cte + pr.cto) + (par ? pr.cte : 0)) * KSa * 64 + l;
      // operands of PD k-steps are in flight: slot u holds k-step s + u while it is multiplied
      // and is then refilled with k-step s + u + PD.  Nothing touches a table operand between
      // its load and its product, and no product sits under a branch (either makes the compiler
      // wait for every load in flight): the sign and the zero of a padded k-step past KSa are
      // applied to the LDS operand at its use.
      constexpr int PD = 4;
      with_count<CT>(nct, [&](auto ncc) {
        constexpr int NC = decltype(ncc)::value;
        T aq[PD], bq[PD][NC];
        auto load = [&](int s, T& a, T (&b)[NC]) {
          s = s < KSa ? s : KSa - 1;
          a = Ab[4 * s];
#pragma unroll
          for (int c = 0; c < NC; ++c) b[c] = Bb[((long long)c * KSa + s) * 64];
        };
#pragma unroll
        for (int u = 0; u < PD; ++u) load(u, aq[u], bq[u]);
        for (int s = 0; s < KSa; s += PD) {
#pragma unroll
          for (int u = 0; u < PD; ++u) {
            __builtin_amdgcn_sched_barrier(0);
            const T a = (s + u < KSa) ? asg * aq[u] : (T)0;
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[c] = Mfma<T>::step(a, bq[u][c], acc[c]);
            load(s + u + PD, aq[u], bq[u]);
          }
        }
      });
    }
    if (!(part == 0 && pr.parts == 2)) __syncthreads();   // the fold stays for the derived part
  }
  // degree il = 2 (16 c + l%16) + parity; the block [row][il] is gathered in LDS (the fold
  // buffer is free) and written in tiles of 8 degrees, [il/8][row][il%8], each tile of the
  // block one contiguous run
  const int nlp = (pr.nl + 7) & ~7;
#pragma unroll
  for (int c = 0; c < CT; ++c) {
    if (c >= nct) continue;
    const int il = 2 * (16 * c + (l & 15)) + par;
    if (il >= pr.nl) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) lds[(16 * rt + Mfma<T>::out_row(l, q)) * nlp + il] = acc[c][q];
  }
  __syncthreads();
  T* C = ws_out + pr.c_off;
  const int nrow = min(kAnaRows, rows - r0);
  for (int idx = threadIdx.x; idx < kAnaRows * nlp; idx += 256) {
    const int it = idx / (8 * kAnaRows), rem = idx - it * 8 * kAnaRows, row = rem >> 3, e = rem & 7;
    if (row < nrow && it * 8 + e < pr.nl) C[((long long)it * pr.rcap + r0 + row) * 8 + e] = lds[row * nlp + it * 8 + e];
  }
}

// ------------------------------------------------------------------------------------------
// K6: batched contractions C[i][j] = sum_k A[i][k] B[j][k] on the matrix cores.
// Output tile BM x 64 per workgroup (BM = 128 in FP32, 64 in FP64); the four wavefronts
// form a 2 x 2 grid, each owning (BM/2) x 32 as (BM/32) x 2 MFMA 16x16 tiles.  k is staged
// through LDS 32 at a time, and the next k-slice is fetched into registers while the current
// one is multiplied.  Problems of one launch are enumerated tile by tile.
template <class T>
struct GemmCfg {
  static constexpr int BM = (sizeof(T) == 4) ? 128 : 64;
  static constexpr int BN = 64, BK = 32, LDK = BK + 1;
  static constexpr int TM = BM / 32;                 // MFMA row tiles per wavefront
  static constexpr int AL = BM * BK / 256;           // A elements loaded per thread
  static constexpr int BL = BN * BK / 256;           // B elements loaded per thread
};

template <class T>
__global__ void __launch_bounds__(256) k_gemm_batched(const GemmProb* __restrict__ probs, int nprob, int nvec,
                                                      const T* __restrict__ ws_in, const T* __restrict__ tab,
                                                      T* __restrict__ ws_out) {
  typedef GemmCfg<T> G;
  __shared__ T As[G::BM * G::LDK];
  __shared__ T Bs[G::BN * G::LDK];
  int tile = blockIdx.x;
  int p = 0;
  GemmProb pr;
  int tm = 0, tn = 0;
  for (p = 0; p < nprob; ++p) {
    pr = probs[p];
    int M = pr.Mper * nvec;
    int nt_m = (M + G::BM - 1) / G::BM, nt_n = (pr.N + G::BN - 1) / G::BN;
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
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * (G::BM / 2), wn = (wave & 1) * 32;
  typename Mfma<T>::acc_t acc[G::TM][2];
#pragma unroll
  for (int x = 0; x < G::TM; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[x][y][q] = (T)0;
  const int i0 = tm * G::BM, j0 = tn * G::BN;
  // loader mapping: element e = tid + 256 u of the tile, row = e / BK, k = e % BK
  T ra[G::AL], rb[G::BL];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < G::AL; ++u) {
      const int e = tid + 256 * u, r = e / G::BK, kk = k0 + e % G::BK, gi = i0 + r;
      ra[u] = (gi < M && kk < K) ? A[(long long)gi * pr.lda + kk] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < G::BL; ++u) {
      const int e = tid + 256 * u, r = e / G::BK, kk = k0 + e % G::BK, gj = j0 + r;
      rb[u] = (gj < N && kk < K) ? B[(long long)gj * pr.ldb + kk] : (T)0;
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < K; k0 += G::BK) {
#pragma unroll
    for (int u = 0; u < G::AL; ++u) {
      const int e = tid + 256 * u;
      As[(e / G::BK) * G::LDK + e % G::BK] = ra[u];
    }
#pragma unroll
    for (int u = 0; u < G::BL; ++u) {
      const int e = tid + 256 * u;
      Bs[(e / G::BK) * G::LDK + e % G::BK] = rb[u];
    }
    __syncthreads();
    if (k0 + G::BK < K) fetch(k0 + G::BK);
#pragma unroll
    for (int ks = 0; ks < G::BK / 4; ++ks) {
      const int kk = ks * 4 + (lane >> 4);
      T a[G::TM], b[2];
#pragma unroll
      for (int x = 0; x < G::TM; ++x) a[x] = As[(wm + x * 16 + (lane & 15)) * G::LDK + kk];
#pragma unroll
      for (int y = 0; y < 2; ++y) b[y] = Bs[(wn + y * 16 + (lane & 15)) * G::LDK + kk];
#pragma unroll
      for (int x = 0; x < G::TM; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = Mfma<T>::step(a[x], b[y], acc[x][y]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < G::TM; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gi = i0 + wm + x * 16 + Mfma<T>::out_row(lane, q);
        const int gj = j0 + wn + y * 16 + (lane & 15);
        if (gi < M && gj < N) C[(long long)gi * pr.ldc + gj] = acc[x][y][q];
      }
}

// ------------------------------------------------------------------------------------------
// K3/K4/K5: per ring (vec, r_p, theta): take the synthesized Legendre sums as the
// Fourier coefficients of the 9 physical fields (U, omega, grad T), inverse real FFT along
// phi, pointwise products, forward real FFT of (W_r, W_theta, W_phi, Q), and write the
// analysis inputs.  The FFTs are mixed-radix Stockham passes (radix 4, 2, 3, 5) between two
// LDS buffers; two real signals travel as the real and imaginary parts of one complex
// transform, so a ring needs 5 inverse and 2 forward complex transforms of length N_phi.
// A workgroup holds 2^rt_log2 rings of one (vec, r_p).
// MODE 0: linearized products about the cached base fields,
// MODE 1: nonlinear products of the fields themselves,
// MODE 2: synthesis only, the 9 fields are written to base (and base32 if non-null).
enum { RING_LINEAR = 0, RING_NONLINEAR = 1, RING_SYNTH = 2 };

// Explicit-Coriolis variant: adds -2 e_z x u to the force (W_r, W_th, W_ph) at Gauss-Legendre node
// th, where u = (f[0], f[1], f[2]) is the velocity of the products (U in the nonlinear step, the
// perturbation u in the Jacobian action: the force is linear).  e_z x u = (-sin u_ph, -cos u_ph,
// cos u_th + sin u_r).  Rings beyond the last node (never written) use the last node.
template <class T>
__device__ inline void coriolis_force(const DevGrid& g, int th, const T* f, T& W0, T& W1, T& W2) {
  const int j = th < g.nth ? th : g.nth - 1;
  const T c = (T)g.cst[j], s = (T)g.cst[g.nth + j];
  W0 += (T)2 * s * f[2];
  W1 += (T)2 * c * f[2];
  W2 -= (T)2 * (c * f[1] + s * f[0]);
}

// Rows of the Legendre sums a ring reads per harmonic: 0..5 the scalar sums (U_r, w_r, dT/dr;
// Re, Im), 6..17 the vector fields (U_th, U_ph, w_th, w_ph, (1/r) dT/dth, (1/(r sin)) dT/dph;
// Re, Im).  Field f = 0..9 of the transforms (U_r, U_th, U_ph, w_r, w_th, w_ph, dT/dr, dT/dth,
// dT/dph, zero) starts at row kRingFieldRow[f].
__device__ constexpr int kRingFieldRow[10] = {0, 6, 8, 2, 10, 12, 4, 14, 16, 0};
constexpr int kRingRows = 18;

template <class T>
struct cz {
  T re, im;
};

// In-place R-point DFT X_k = sum_n v_n exp(sgn 2 pi i n k / R), sgn = +-1.
template <class T, int R>
__device__ inline void small_dft(cz<T>* v, T sgn) {
  if (R == 2) {
    const cz<T> a = v[0], b = v[1];
    v[0] = {a.re + b.re, a.im + b.im};
    v[1] = {a.re - b.re, a.im - b.im};
  } else if (R == 4) {
    const cz<T> a = v[0], b = v[1], c = v[2], d = v[3];
    const cz<T> s0 = {a.re + c.re, a.im + c.im}, s1 = {a.re - c.re, a.im - c.im};
    const cz<T> s2 = {b.re + d.re, b.im + d.im}, s3 = {b.re - d.re, b.im - d.im};
    const cz<T> is3 = {-sgn * s3.im, sgn * s3.re};  // sgn i s3
    v[0] = {s0.re + s2.re, s0.im + s2.im};
    v[2] = {s0.re - s2.re, s0.im - s2.im};
    v[1] = {s1.re + is3.re, s1.im + is3.im};
    v[3] = {s1.re - is3.re, s1.im - is3.im};
  } else if (R == 8) {
    // two radix-4 transforms of the even and odd samples, combined with w^k, w = exp(sgn 2 pi i/8)
    const T c8 = (T)0.70710678118654752440;
    cz<T> e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
    small_dft<T, 4>(e, sgn);
    small_dft<T, 4>(o, sgn);
    const cz<T> t1 = {c8 * (o[1].re - sgn * o[1].im), c8 * (o[1].im + sgn * o[1].re)};
    const cz<T> t2 = {-sgn * o[2].im, sgn * o[2].re};
    const cz<T> t3 = {c8 * (-o[3].re - sgn * o[3].im), c8 * (-o[3].im + sgn * o[3].re)};
    const cz<T> tw[4] = {o[0], t1, t2, t3};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = {e[k].re + tw[k].re, e[k].im + tw[k].im};
      v[k + 4] = {e[k].re - tw[k].re, e[k].im - tw[k].im};
    }
  } else if (R == 3) {
    const T h = (T)0.86602540378443864676;  // sin(2 pi / 3)
    const cz<T> a = v[0], t = {v[1].re + v[2].re, v[1].im + v[2].im}, u = {v[1].re - v[2].re, v[1].im - v[2].im};
    const cz<T> m = {a.re - (T)0.5 * t.re, a.im - (T)0.5 * t.im};
    const cz<T> iu = {-sgn * h * u.im, sgn * h * u.re};
    v[0] = {a.re + t.re, a.im + t.im};
    v[1] = {m.re + iu.re, m.im + iu.im};
    v[2] = {m.re - iu.re, m.im - iu.im};
  } else {  // R == 5
    const T c1 = (T)0.30901699437494742410, s1 = (T)0.95105651629515357212;   // cos, sin(2 pi/5)
    const T c2 = (T)-0.80901699437494742410, s2 = (T)0.58778525229247312917;  // cos, sin(4 pi/5)
    const cz<T> a = v[0];
    const cz<T> t1 = {v[1].re + v[4].re, v[1].im + v[4].im}, u1 = {v[1].re - v[4].re, v[1].im - v[4].im};
    const cz<T> t2 = {v[2].re + v[3].re, v[2].im + v[3].im}, u2 = {v[2].re - v[3].re, v[2].im - v[3].im};
    const cz<T> p1 = {a.re + c1 * t1.re + c2 * t2.re, a.im + c1 * t1.im + c2 * t2.im};
    const cz<T> p2 = {a.re + c2 * t1.re + c1 * t2.re, a.im + c2 * t1.im + c1 * t2.im};
    const cz<T> q1 = {s1 * u1.re + s2 * u2.re, s1 * u1.im + s2 * u2.im};
    const cz<T> q2 = {s2 * u1.re - s1 * u2.re, s2 * u1.im - s1 * u2.im};
    const cz<T> iq1 = {-sgn * q1.im, sgn * q1.re}, iq2 = {-sgn * q2.im, sgn * q2.re};
    v[0] = {a.re + t1.re + t2.re, a.im + t1.im + t2.im};
    v[1] = {p1.re + iq1.re, p1.im + iq1.im};
    v[4] = {p1.re - iq1.re, p1.im - iq1.im};
    v[2] = {p2.re + iq2.re, p2.im + iq2.im};
    v[3] = {p2.re - iq2.re, p2.im - iq2.im};
  }
}

// LDS slot of complex entry i of the ring buffer: one pad entry after every 16 breaks the
// power-of-two strides of the butterflies and of the (ring, point) accesses across banks.
__device__ inline int lp(int i) { return i + (i >> 4); }

// Layout of the transforms of a workgroup in LDS: transform t lives at
// (t / PER) * stride + (t % PER) * N (PER transforms of each ring, consecutive).
struct FftSet {
  int ntr, stride;
};

constexpr int kRingThreads = 256;

// Most complex values a k_ring workgroup transforms at once (5 spectra of 2^rt_log2 rings of
// N_phi points); bounds the butterflies each thread holds in registers during a pass.
template <class T>
__host__ __device__ constexpr int ring_cap() {
  return sizeof(T) == 4 ? 4096 : 2048;
}

// Exact quotient a / b for 0 <= a < 2^13 and 1 <= b < 2^12 through a single-precision
// reciprocal (rcp_b = 1/b rounded): the error of (a + 1/2) rcp_b stays far below the 1/(2b)
// margin to the next integer, so no integer division is issued.
__device__ inline int fdiv_small(int a, float rcp_b) { return (int)(((float)a + 0.5f) * rcp_b); }

// One radix-R Stockham pass (Ns = product of the radices of the earlier passes), in place:
// every thread first reads and transforms its butterflies into registers, then, after a
// barrier, all of them write.  w[m] = exp(-2 pi i m / N); the inverse (sgn = +1) uses its
// conjugate.  Requires fs.ntr * N <= ring_cap<T>().  Kept out of line so that the register
// staging of the four radices is not allocated side by side in the caller.
template <class T, int R, int PER>
__device__ __attribute__((noinline)) void stockham_pass(cz<T>* buf, int N, int Ns, FftSet fs, const cz<T>* __restrict__ w,
                                                        T sgn) {
  constexpr int MAXB = (ring_cap<T>() + R * kRingThreads - 1) / (R * kRingThreads);
  const int nb = N / R, step = N / (Ns * R), total = fs.ntr * nb;
  const float rnb = 1.0f / (float)nb, rNs = 1.0f / (float)Ns;
  cz<T> v[MAXB][R];
  int dst[MAXB];
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int idx = threadIdx.x + b * kRingThreads;
    dst[b] = -1;
    if (idx < total) {
      const int t = fdiv_small(idx, rnb), j = idx - t * nb;
      const int o = (t / PER) * fs.stride + (t % PER) * N;
      const int qq = fdiv_small(j, rNs), k = j - qq * Ns;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        cz<T> a = buf[lp(o + j + r * nb)];
        if (r > 0) {
          const cz<T> tw = w[k * r * step];
          const T twi = (sgn < 0) ? tw.im : -tw.im;
          a = {a.re * tw.re - a.im * twi, a.re * twi + a.im * tw.re};
        }
        v[b][r] = a;
      }
      small_dft<T, R>(v[b], sgn);
      dst[b] = o + qq * Ns * R + k;
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < MAXB; ++b)
    if (dst[b] >= 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) buf[lp(dst[b] + r * Ns)] = v[b][r];
    }
  __syncthreads();
}

// All passes of the plan's radices over the set, in place.
template <class T, int PER>
__device__ inline void fft_run(const DevGrid& g, cz<T>* buf, FftSet fs, const cz<T>* w, T sgn) {
  int Ns = 1;
  for (int s = 0; s < g.fft_nr; ++s) {
    const int R = g.fft_r[s];
    if (R == 8) stockham_pass<T, 8, PER>(buf, g.nphi, Ns, fs, w, sgn);
    else if (R == 4) stockham_pass<T, 4, PER>(buf, g.nphi, Ns, fs, w, sgn);
    else if (R == 2) stockham_pass<T, 2, PER>(buf, g.nphi, Ns, fs, w, sgn);
    else if (R == 3) stockham_pass<T, 3, PER>(buf, g.nphi, Ns, fs, w, sgn);
    else stockham_pass<T, 5, PER>(buf, g.nphi, Ns, fs, w, sgn);
    Ns *= R;
  }
}

// LDS bytes of k_ring for 2^rt_log2 rings per workgroup.
template <class T>
__host__ __device__ inline size_t ring_lds_bytes(int nphi, int rt_log2) {
  const size_t n = (size_t)5 * nphi * ((size_t)1 << rt_log2);
  return sizeof(cz<T>) * ((size_t)nphi + n + n / 16 + 1);
}

template <class T, int MODE>
__global__ void __launch_bounds__(kRingThreads) k_ring(DevGrid g, int nvec, int rt_log2, const T* __restrict__ Cs,
                                              const T* __restrict__ Cv, const T* __restrict__ base,
                                              const T* __restrict__ fw, T Ek, T* __restrict__ Fs, T* __restrict__ Fv,
                                              double* __restrict__ base_out64, float* __restrict__ base_out32) {
  extern __shared__ unsigned char smem_raw[];
  const int K1 = g.K + 1, N = g.nphi, nth = g.nth;
  const int RT = 1 << rt_log2, rmask = RT - 1;
  cz<T>* w = reinterpret_cast<cz<T>*>(smem_raw);  // [N] twiddles exp(-2 pi i m / N)
  cz<T>* X = w + N;                                // [RT][5][N]
  const int ntile = (nth + RT - 1) >> rt_log2;
  // logical order (r_p, vec, tile) in contiguous runs per XCD, so that the tiles of one ring
  // row and the vectors sharing one base radius reuse the same L2
  const int lid = xcd_linear_id();
  const int tile = lid % ntile;
  const int rv = lid / ntile;  // rp * nvec + vec
  const int rp = rv / nvec;
  const int vr = (rv - rp * nvec) * g.Np + rp;  // vec * Np + rp: row index of the sums
  const int th0 = tile << rt_log2;
  const int tid = threadIdx.x;
  // the linearized products read the base fields at the points this thread owns in step C:
  // issue those loads first so that they overlap the gathers and transforms
  constexpr int NPT = (ring_cap<T>() / 5 + kRingThreads - 1) / kRingThreads;
  T bpre[NPT][9];
  if (MODE == RING_LINEAR) {
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
      const int idx = tid + u * kRingThreads;
      const int tt = idx & rmask, p = idx >> rt_log2;
      const int th = th0 + tt;
#pragma unroll
      for (int q = 0; q < 9; ++q)
        bpre[u][q] = (idx < N * RT && th < nth) ? base[(((long long)rp * 9 + q) * N + p) * nth + th] : (T)0;
    }
  }
  for (int i = tid; i < N; i += kRingThreads) w[i] = {fw[2 * i], fw[2 * i + 1]};
  // spectra entries K < k < N - K stay zero
  for (int i = tid; i < lp(RT * 5 * N); i += kRingThreads) X[i] = {(T)0, (T)0};
  __syncthreads();
  // step A: gather the Legendre sums and form the Fourier coefficients of the 9 fields,
  // packing fields (2q, 2q+1) into spectrum q: Z_k = (A_k + i B_k)/2, Z_{N-k} = conj(A_k)/2 +
  // i conj(B_k)/2 for k >= 1 and Z_0 = Re A_0 + i Re B_0.
  const long long Ms = (long long)6 * g.Np * g.vcap, Mv = (long long)12 * g.Np * g.vcap;
  const int vq = rv - rp * nvec;  // vector index
  for (int idx = tid; idx < K1 * RT; idx += kRingThreads) {
    const int tt = idx & rmask, k = idx >> rt_log2;
    const int th = th0 + tt;
    if (th >= nth) continue;
    T c[kRingRows];
    // rows of the sums: (vec, slot, r_p); scalar U_r, w_r, dT/dr, vector fields U_th, U_ph,
    // w_th, w_ph, (1/r) dT/dth, (1/(r sin)) dT/dph (Re, Im each)
    const T* cs = Cs + (long long)k * Ms * nth + ((long long)vq * 6 * g.Np + rp) * nth + th;
#pragma unroll
    for (int q = 0; q < 6; ++q) c[q] = cs[(long long)q * g.Np * nth];
    const T* cv = Cv + (long long)k * Mv * nth + ((long long)vq * 12 * g.Np + rp) * nth + th;
#pragma unroll
    for (int q = 0; q < 12; ++q) c[6 + q] = cv[(long long)q * g.Np * nth];
    T fr[10], fi[10];
#pragma unroll
    for (int f = 0; f < 9; ++f) {
      fr[f] = c[kRingFieldRow[f]];
      fi[f] = c[kRingFieldRow[f] + 1];
    }
    fr[9] = 0; fi[9] = 0;
    const int zb = tt * 5 * N;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const T ar = fr[2 * q], ai = fi[2 * q], br = fr[2 * q + 1], bi = fi[2 * q + 1];
      if (k == 0) {
        X[lp(zb + q * N)] = {ar, br};
      } else {
        X[lp(zb + q * N + k)] = {(T)0.5 * (ar - bi), (T)0.5 * (ai + br)};
        X[lp(zb + q * N + N - k)] = {(T)0.5 * (ar + bi), (T)0.5 * (br - ai)};
      }
    }
  }
  __syncthreads();
  // step B: inverse transforms; spectrum q of a ring becomes field 2q + i field 2q+1
  fft_run<T, 5>(g, X, FftSet{5 * RT, 5 * N}, w, (T)1);
  // step C: pointwise products, written in place as slot 0 = W_r + i Q, slot 1 = W_th + i W_ph
#pragma unroll
  for (int u = 0; u < NPT; ++u) {
    const int idx = tid + u * kRingThreads;
    if (idx >= N * RT) continue;
    const int tt = idx & rmask, p = idx >> rt_log2;
    const int th = th0 + tt;
    const int zb = tt * 5 * N;
    T f[10];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const cz<T> zq = X[lp(zb + q * N + p)];
      f[2 * q] = zq.re;
      f[2 * q + 1] = zq.im;
    }
    if (MODE == RING_SYNTH) {
      if (th < nth) {
#pragma unroll
        for (int q = 0; q < 9; ++q) {
          const long long o = (((long long)rp * 9 + q) * N + p) * nth + th;
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
      const T* b = bpre[u];
      // W' = Ek (U x w_u + u x Omega), Q' = -(U . grad tau + u . grad T)
      W0 = Ek * ((b[1] * f[5] - b[2] * f[4]) + (f[1] * b[5] - f[2] * b[4]));
      W1 = Ek * ((b[2] * f[3] - b[0] * f[5]) + (f[2] * b[3] - f[0] * b[5]));
      W2 = Ek * ((b[0] * f[4] - b[1] * f[3]) + (f[0] * b[4] - f[1] * b[3]));
      Q = -((b[0] * f[6] + b[1] * f[7] + b[2] * f[8]) + (f[0] * b[6] + f[1] * b[7] + f[2] * b[8]));
    }
    if (g.cor_explicit) coriolis_force<T>(g, th, f, W0, W1, W2);
    X[lp(zb + p)] = {W0, Q};
    X[lp(zb + N + p)] = {W1, W2};
  }
  if (MODE == RING_SYNTH) return;
  __syncthreads();
  // step D: forward transforms of slots 0 and 1 of every ring
  fft_run<T, 2>(g, X, FftSet{2 * RT, 5 * N}, w, (T)-1);
  // step E: split the packed pair, scale by (2 - delta_k0)/N_phi, write analysis inputs
  const long long Ma = (long long)4 * g.Np * g.vcap;
  for (int idx = tid; idx < 2 * K1 * RT; idx += kRingThreads) {
    const int tt = idx & rmask;
    const int o = (idx >> rt_log2) & 1;
    const int k = idx >> (rt_log2 + 1);
    const int th = th0 + tt;
    if (th >= nth) continue;
    const int zb = tt * 5 * N + o * N;
    const T sc = (k == 0 ? (T)1 : (T)2) / (T)N;
    T ar, ai, br, bi;
    if (k == 0) {
      const cz<T> z0 = X[lp(zb)];
      ar = z0.re; ai = 0; br = z0.im; bi = 0;
    } else {
      const cz<T> zk = X[lp(zb + k)], zm = X[lp(zb + N - k)];
      ar = (T)0.5 * (zk.re + zm.re);
      ai = (T)0.5 * (zk.im - zm.im);
      br = (T)0.5 * (zk.im + zm.im);
      bi = (T)0.5 * (zm.re - zk.re);
    }
    ar *= sc; ai *= sc; br *= sc; bi *= sc;
    if (o == 0) {  // (W_r, Q)
      T* out = Fs + (long long)k * Ma * nth + ((long long)vr * 4) * nth + th;
      out[0 * nth] = ar;
      out[1 * nth] = ai;
      out[2 * nth] = br;
      out[3 * nth] = bi;
    } else {       // (W_th, W_ph): dP rows (W_th, -W_ph); mPs rows (-i W_ph, -i W_th)
      T* out = Fv + (long long)k * Ma * 2 * nth + ((long long)vr * 4) * 2 * nth + th;
      out[0 * 2 * nth] = ar;
      out[1 * 2 * nth] = ai;
      out[2 * 2 * nth] = -br;
      out[3 * 2 * nth] = -bi;
      if (!g.fv_dp_only) {
        out[0 * 2 * nth + nth] = bi;
        out[1 * 2 * nth + nth] = -br;
        out[2 * 2 * nth + nth] = ai;
        out[3 * 2 * nth + nth] = -ar;
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// K3/K4/K5 with register-resident transforms, for N_phi = N1 N2 (N1, N2 in {2, 3, 4, 5, 8}).
// Every thread owns one complex transform of one ring and runs it entirely in registers as a
// four-step FFT with compile-time indices: N2 DFTs of length N1 over n1 (inputs n = N2 n1 + n2),
// twiddles w^(n2 k1), N1 DFTs of length N2 over n2.  Both steps work in place, so output k
// = k1 + N1 k2 ends at position N2 k1 + k2 (fft_pos).  LDS only carries the fields from the
// inverse transforms to the pointwise products and the products to the forward transforms.
template <int N1, int N2>
__host__ __device__ constexpr int fft_pos(int k) {
  return N2 * (k % N1) + k / N1;
}

// x: natural order in, x[fft_pos(k)] = sum_n x_n exp(SGN 2 pi i n k / N) out; fw[2e], fw[2e+1]
// = cos, -sin(2 pi e / N).
template <class T, int N1, int N2, int SGN>
__device__ inline void fft_reg(cz<T> (&x)[N1 * N2], const T* __restrict__ fw) {
  constexpr int N = N1 * N2;
#pragma unroll
  for (int n2 = 0; n2 < N2; ++n2) {
    cz<T> v[N1];
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) v[n1] = x[N2 * n1 + n2];
    small_dft<T, N1>(v, (T)SGN);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) {
      cz<T> a = v[k1];
      const int e = (n2 * k1) % N;
      if (e != 0) {
        const T c = fw[2 * e], sn = (SGN < 0) ? fw[2 * e + 1] : -fw[2 * e + 1];
        a = {a.re * c - a.im * sn, a.re * sn + a.im * c};
      }
      x[N2 * k1 + n2] = a;
    }
  }
#pragma unroll
  for (int k1 = 0; k1 < N1; ++k1) {
    cz<T> u[N2];
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) u[n2] = x[N2 * k1 + n2];
    small_dft<T, N2>(u, (T)SGN);
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) x[N2 * k1 + k2] = u[k2];
  }
}

// Spectrum of transform q = fields (2q, 2q+1) of one ring, packed as in k_ring; g points at
// the ring's column of the LDS copy, laid out [row][k][ring] (row stride rs, k stride ks).  The
// same code serves every q (row indices per lane), so the lanes of a wave that hold different
// transforms do not diverge.
template <class T, int N>
__device__ inline void ring_spectrum(cz<T> (&z)[N], const T* g, int rs, int ks, int K1, int q) {
  constexpr int KM = (N - 1) / 3 + 1;   // K1 <= KM (N_phi >= 3K + 1)
  const int fb = 2 * q + 1;
  // kRingFieldRow[2q] and [2q+1] by selects: a lookup in the table would be a memory load, and
  // waiting for it would wait for every load issued before it (the base fields in flight)
  const int ra = q == 0 ? 0 : q == 1 ? 8 : q == 2 ? 10 : q == 3 ? 4 : 16;
  const int rb = q == 0 ? 6 : q == 1 ? 2 : q == 2 ? 12 : q == 3 ? 14 : 0;
  const T* a = g + ra * rs;
  const T* b = g + rb * rs;
  const T bon = fb == 9 ? (T)0 : (T)1;
#pragma unroll
  for (int k = 0; k < KM; ++k) {
    T ar = 0, ai = 0, br = 0, bi = 0;
    if (k < K1) {
      const int o = k * ks;
      ar = a[o];
      ai = a[o + rs];
      br = bon * b[o];
      bi = bon * b[o + rs];
    }
    if (k == 0) {
      z[0] = {ar, br};
    } else {
      z[k] = {(T)0.5 * (ar - bi), (T)0.5 * (ai + br)};
      z[N - k] = {(T)0.5 * (ar + bi), (T)0.5 * (br - ai)};
    }
  }
}

// Buffer loads (raw, byte offsets: per-lane vo plus wave-uniform so).  The third descriptor word
// selects 32-bit data with bounds checking, so a load past num_records returns zero.
constexpr int kBufferDword3 = 0x00020000;

template <class T>
__device__ __forceinline__ T buffer_load1(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so);
template <>
__device__ __forceinline__ float buffer_load1<float>(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
}
template <>
__device__ __forceinline__ double buffer_load1<double>(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
}
template <class T>
__device__ __forceinline__ void buffer_store1(T x, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so);
template <>
__device__ __forceinline__ void buffer_store1<float>(float x, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), r, vo, so, 0);
}
template <>
__device__ __forceinline__ void buffer_store1<double>(double x, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, x), r, vo, so,
                                        0);
}
template <class V>
__device__ __forceinline__ V buffer_load8(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
  static_assert(sizeof(V) == 8, "an 8-byte piece");
  return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
}

// Rings per workgroup of k_ring_reg: the variants a plan may choose, per precision (the first
// is the default), and the threads of a workgroup of RR rings: eight per ring (five hold the
// inverse transforms, two the forward ones; 8 RR is a whole number of wavefronts).  Fewer rings
// give smaller workgroups (less LDS each, more of them per compute unit) at the same number of
// waves per compute unit, and fewer rings past the last node in the last tile.
template <class T>
__host__ __device__ constexpr int ring_reg_variants() {
  return sizeof(T) == 4 ? 3 : 2;
}
template <class T>
__host__ __device__ constexpr int ring_reg_rings(int variant) {
  return sizeof(T) == 4 ? (variant == 0 ? 32 : variant == 1 ? 24 : 16) : (variant == 0 ? 16 : 8);
}
__host__ __device__ constexpr int ring_reg_threads(int rr) { return 8 * rr; }

template <class T, int MODE, int N1, int N2, int RR>
__global__ void __launch_bounds__(ring_reg_threads(RR)) k_ring_reg(DevGrid g, int nvec, const T* __restrict__ Cs, const T* __restrict__ Cv,
                                                  const T* __restrict__ base, const T* __restrict__ fw, T Ek,
                                                  T* __restrict__ Fs, T* __restrict__ Fv, double* __restrict__ base_out64,
                                                  float* __restrict__ base_out32) {
  constexpr int N = N1 * N2, LS = N + 1;  // LS: LDS stride of one (slot, ring)
  constexpr int NT = ring_reg_threads(RR);  // threads per workgroup
  static_assert(5 * RR <= NT && NT % 64 == 0, "a thread per inverse transform");
  constexpr int NPT = (RR * N + NT - 1) / NT;                       // product points per thread
  // the fields of the transforms; first the copy of the Legendre sums [18 rows][K1][RR rings]
  __shared__ cz<T> X[5 * RR * LS];
  T* Gl = reinterpret_cast<T*>(X);
  const int K1 = g.K + 1, nth = g.nth, Np = g.Np;
  const int ntile = (nth + RR - 1) / RR;
  const int lid = xcd_linear_id();
  const int tile = lid % ntile, rv = lid / ntile, rp = rv / nvec, vq = rv - rp * nvec;
  const int th0 = tile * RR, tid = threadIdx.x;
  // The loads go through buffer resources with 32-bit byte offsets (the launch checks that the
  // sums of every vector, 18 (K+1) N_p vcap N_theta values from Cs on, and the base fields fit
  // in 2^31 bytes): one add per load instead of 64-bit address arithmetic, and a load past a
  // resource returns zero.
  const unsigned szT = sizeof(T);
  // base fields of this thread's product points; points of rings beyond the last node read that
  // node (their results are never written).  They are loaded right after the sums: the memory
  // counter completes in issue order, so loads issued before the sums would be waited for with
  // them, while loads issued after them stay in flight through the FFTs
  T bpre[NPT][9];
  auto load_base = [&] {
    const __amdgpu_buffer_rsrc_t rb =
        __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)(9u * N * nth * Np * szT), kBufferDword3);
    const unsigned qs = (unsigned)N * nth * szT;   // byte stride of the nine fields
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
      const int idx = tid + NT * u, r = idx % RR, pt = min(idx / RR, N - 1), th = min(th0 + r, nth - 1);
      const unsigned vo = ((unsigned)(rp * 9 * N + pt) * nth + th) * szT;
#pragma unroll
      for (int q = 0; q < 9; ++q) bpre[u][q] = buffer_load1<T>(rb, vo, q * qs);
    }
  };
  // copy of the sums of this workgroup's rings into LDS, [18 rows][K1][RR rings]: every (row, k)
  // is a run of RR consecutive theta, read as 8-byte pieces (nth and th0 are even, so a piece
  // lies wholly inside or wholly beyond the last node).  Thread (group, piece) owns rows group,
  // group + NG, ... and reads them for every k (K1 <= KM = (N - 1)/3 + 1, a compile-time trip
  // count), all loads issued before the first store.
  {
    constexpr int EPL = 8 / sizeof(T), PPR = RR / EPL, NG = NT / PPR;   // elements per piece, pieces per run, groups
    constexpr int KM = (N - 1) / 3 + 1, NRW = (kRingRows + NG - 1) / NG; // rows per group
    typedef T pT __attribute__((ext_vector_type(EPL)));
    const unsigned kS = 6u * Np * g.vcap * nth * szT, kV = 2 * kS;        // bytes per harmonic
    const unsigned sR = (unsigned)Np * nth * szT;                          // bytes per row
    const unsigned offV = (unsigned)(Cv - Cs) * szT;                       // Cv follows Cs
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void*)Cs, (short)0, (int)(3u * K1 * kS), kBufferDword3);
    // a piece beyond the last node reads the last one (that ring's results are never written),
    // k >= K1 reads past the rows of K1 harmonics (not stored); rows beyond the last are
    // skipped (whole wavefronts but one)
    const int e = tid % PPR, grp = tid / PPR, th = min(th0 + e * EPL, nth - EPL);
    const unsigned vs = ((unsigned)(vq * 6 * Np + rp) * nth + th) * szT;
    const unsigned vv = offV + ((unsigned)(vq * 12 * Np + rp) * nth + th) * szT;
    pT val[NRW][KM];
#pragma unroll
    for (int i = 0; i < NRW; ++i) {
      const int row = grp + i * NG;
      if (i > 0 && row >= kRingRows) continue;
      unsigned o = row < 6 ? vs + row * sR : vv + (row - 6) * sR;
      const unsigned kst = row < 6 ? kS : kV;
#pragma unroll
      for (int k = 0; k < KM; ++k, o += kst) val[i][k] = buffer_load8<pT>(rs, o, 0);
    }
    if (MODE == RING_LINEAR) {
      __builtin_amdgcn_sched_barrier(0);
      load_base();
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int i = 0; i < NRW; ++i) {
      const int row = grp + i * NG;
#pragma unroll
      for (int k = 0; k < KM; ++k)
        if (row < kRingRows && k < K1) *reinterpret_cast<pT*>(Gl + (row * K1 + k) * RR + e * EPL) = val[i][k];
    }
  }
  __syncthreads();
  // inverse transforms: thread (q, r) owns transform q of ring r
  {
    const int q = tid / RR, r = tid % RR;
    cz<T> z[N];
#pragma unroll
    for (int p = 0; p < N; ++p) z[p] = {(T)0, (T)0};
    if (q < 5) ring_spectrum<T, N>(z, Gl + r, K1 * RR, RR, K1, q);
    __syncthreads();   // the copy of the sums is dead from here on; X reuses its space
    if (q < 5) {
      fft_reg<T, N1, N2, 1>(z, fw);
      cz<T>* xo = X + (q * RR + r) * LS;
#pragma unroll
      for (int p = 0; p < N; ++p) xo[p] = z[fft_pos<N1, N2>(p)];
    }
  }
  __syncthreads();
  // pointwise products at (ring, point), in place as slot 0 = W_r + i Q, slot 1 = W_th + i W_ph
#pragma unroll
  for (int u = 0; u < NPT; ++u) {
    const int idx = tid + NT * u, r = idx % RR, pt = idx / RR, th = th0 + r;
    if (pt >= N) continue;
    T f[10];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const cz<T> zq = X[(q * RR + r) * LS + pt];
      f[2 * q] = zq.re;
      f[2 * q + 1] = zq.im;
    }
    if (MODE == RING_SYNTH) {
      if (th < nth) {
#pragma unroll
        for (int q = 0; q < 9; ++q) {
          const long long o = (((long long)rp * 9 + q) * N + pt) * nth + th;
          base_out64[o] = (double)f[q];
          if (base_out32) base_out32[o] = (float)f[q];
        }
      }
      continue;
    }
    T W0, W1, W2, Q;
    if (MODE == RING_NONLINEAR) {
      W0 = Ek * (f[1] * f[5] - f[2] * f[4]);
      W1 = Ek * (f[2] * f[3] - f[0] * f[5]);
      W2 = Ek * (f[0] * f[4] - f[1] * f[3]);
      Q = -(f[0] * f[6] + f[1] * f[7] + f[2] * f[8]);
    } else {
      const T* b = bpre[u];
      W0 = Ek * ((b[1] * f[5] - b[2] * f[4]) + (f[1] * b[5] - f[2] * b[4]));
      W1 = Ek * ((b[2] * f[3] - b[0] * f[5]) + (f[2] * b[3] - f[0] * b[5]));
      W2 = Ek * ((b[0] * f[4] - b[1] * f[3]) + (f[0] * b[4] - f[1] * b[3]));
      Q = -((b[0] * f[6] + b[1] * f[7] + b[2] * f[8]) + (f[0] * b[6] + f[1] * b[7] + f[2] * b[8]));
    }
    if (g.cor_explicit) coriolis_force<T>(g, th, f, W0, W1, W2);
    X[(0 * RR + r) * LS + pt] = {W0, Q};
    X[(1 * RR + r) * LS + pt] = {W1, W2};
  }
  if (MODE == RING_SYNTH) return;
  __syncthreads();
  // forward transforms of slots 0 and 1, spread over the eight threads (j, r) of every ring as
  // a four-step FFT through LDS: the 2 N2 column DFTs of length N1 (inputs n = N2 n1 + n2),
  // written to slot 2 + o at N2 k1 + n2; then the 2 N1 row DFTs of length N2, their inputs
  // twiddled by w^(n2 k1), output k = k1 + N1 k2 written to slot o at k; then the 2 KM
  // harmonics (o, k): split the packed pair, scale by (2 - delta_k0)/N_phi and write the
  // analysis inputs.  Slots 2..4 are free after the products.
  {
    const int r = tid % RR, j = tid / RR, th = th0 + r;
#pragma unroll
    for (int i = 0; i < (2 * N2 + 7) / 8; ++i) {
      const int c = j + 8 * i;
      if (c < 2 * N2) {
        const int o = c / N2, n2 = c - o * N2;
        const cz<T>* xi = X + (o * RR + r) * LS + n2;
        cz<T> v[N1];
#pragma unroll
        for (int n1 = 0; n1 < N1; ++n1) v[n1] = xi[N2 * n1];
        small_dft<T, N1>(v, (T)-1);
        cz<T>* xo = X + ((2 + o) * RR + r) * LS + n2;
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) xo[N2 * k1] = v[k1];
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < (2 * N1 + 7) / 8; ++i) {
      const int c = j + 8 * i;
      if (c < 2 * N1) {
        const int o = c / N1, k1 = c - o * N1;
        const cz<T>* xi = X + ((2 + o) * RR + r) * LS + N2 * k1;
        cz<T> u[N2];
        T tc[N2], ts[N2];
#pragma unroll
        for (int n2 = 1; n2 < N2; ++n2) {
          const int e = (n2 * k1) % N;   // fw[2e], fw[2e+1] = cos, -sin(2 pi e / N)
          tc[n2] = fw[2 * e];
          ts[n2] = fw[2 * e + 1];
        }
#pragma unroll
        for (int n2 = 0; n2 < N2; ++n2) u[n2] = xi[n2];
#pragma unroll
        for (int n2 = 1; n2 < N2; ++n2) {
          const cz<T> a = u[n2];
          u[n2] = {a.re * tc[n2] - a.im * ts[n2], a.re * ts[n2] + a.im * tc[n2]};
        }
        small_dft<T, N2>(u, (T)-1);
        cz<T>* xo = X + (o * RR + r) * LS + k1;
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) xo[N1 * k2] = u[k2];
      }
    }
    __syncthreads();
    if (th < nth) {
      constexpr int KM = (N - 1) / 3 + 1;
      const int vr = vq * Np + rp;  // row (vec, r_p) of the analysis inputs
      // buffer stores from Fs (Fv follows it; 3 (K+1) 4 N_p vcap N_theta values in all): per
      // lane the byte offset of its output row and harmonic, per row a wave-uniform offset
      const unsigned Ma = 4u * Np * g.vcap, ns = (unsigned)nth * szT;
      const __amdgpu_buffer_rsrc_t rf =
          __builtin_amdgcn_make_buffer_rsrc((void*)Fs, (short)0, (int)(3u * K1 * Ma * ns), kBufferDword3);
      const unsigned vsb = ((unsigned)vr * 4 * nth + th) * szT;
      const unsigned vvb = (unsigned)(Fv - Fs) * szT + ((unsigned)vr * 4 * 2 * nth + th) * szT;
      const unsigned dS = Ma * ns, dV = 2 * Ma * ns;
      auto st = [&](unsigned vo, unsigned so, T x) { buffer_store1<T>(x, rf, vo, so); };
#pragma unroll
      for (int i = 0; i < (2 * KM + 7) / 8; ++i) {
        const int c = j + 8 * i, o = c / KM, k = c - o * KM;
        if (c >= 2 * KM || k >= K1) continue;
        const cz<T>* z = X + (o * RR + r) * LS;
        const cz<T> zk = z[k], zm = z[k == 0 ? 0 : N - k];
        const T sc = (T)1 / (T)N;   // (2 - delta_k0)/N_phi with the 1/2 of the unpacking
        T ar, ai, br, bi;
        if (k == 0) {
          ar = zk.re * sc; ai = 0; br = zk.im * sc; bi = 0;
        } else {
          ar = (zk.re + zm.re) * sc;
          ai = (zk.im - zm.im) * sc;
          br = (zk.im + zm.im) * sc;
          bi = (zm.re - zk.re) * sc;
        }
        if (o == 0) {  // (W_r, Q)
          const unsigned vo = vsb + k * dS;
          st(vo, 0, ar);
          st(vo, ns, ai);
          st(vo, 2 * ns, br);
          st(vo, 3 * ns, bi);
        } else {       // (W_th, W_ph): dP rows (W_th, -W_ph); mPs rows (-i W_ph, -i W_th)
          const unsigned vo = vvb + k * dV;
          st(vo, 0, ar);
          st(vo, 2 * ns, ai);
          st(vo, 4 * ns, -br);
          st(vo, 6 * ns, -bi);
          if (!g.fv_dp_only) {
            st(vo, ns, bi);
            st(vo, 3 * ns, -br);
            st(vo, 5 * ns, ai);
            st(vo, 7 * ns, -ar);
          }
        }
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// K7: curl projections back to the N nodes and assembly of the right-hand side
//   b = M u + dt (N(u) + Ra lam T/(r r_o) [f only] + C i m M u + c i m M X)
// with M_e = Ek lam/r^2, M_f = -Ek lam/r^2 (D^2 - lam/r^2), M_T = 1, and boundary rows.
// The e-row force P((lam/r) Tor), the f-row force P((lam/r^2)(W_r - d_r(r S))) and the T-row
// force P(Q) are products with fixed N x N_p matrices (P diag(1/r), P diag(1/r^2),
// P diag(1/r^2) Dp diag(r), P), so every output of the tile comes from five FP64 MFMA
// products (the fifth is D^2 on f) and a pointwise epilogue in registers.
// STEP: inhomogeneous T_00 rows, no c-term.  One workgroup per (tile of up to 8 consecutive l
// at one m, vector); columns (Re/Im, l); wavefront w owns output rows 16w..16w+15.
constexpr int kPT = 8;  // l per projection tile

template <class T>
__host__ __device__ inline size_t project_lds_bytes(int Np, int N) {
  const int rp = 16 * ((Np + 15) / 16), rn = 16 * ((N + 15) / 16);
  return (size_t)4 * rp * 16 * sizeof(T) + (size_t)3 * rn * 16 * sizeof(double);
}

template <class T, bool STEP, int RTN>
__global__ void __launch_bounds__(256) k_project_rhs(DevGrid g, PhysParams ph, int nvec, const T* __restrict__ As,
                                                     const T* __restrict__ Av, const double* __restrict__ v,
                                                     long long ldv, long long J, double C,
                                                     const double* __restrict__ Cdev,
                                                     const double* __restrict__ MX, double* __restrict__ b) {
  extern __shared__ unsigned char smem_raw[];
  const int N = g.N, Np = g.Np;
  const int KBP = (Np + 15) / 16, rowsP = 16 * KBP;
  constexpr int rowsN = 16 * RTN;
  T* Xa = reinterpret_cast<T*>(smem_raw);                                             // [4][rowsP][16]: Tor, W_r, S, Q
  double* Xu = reinterpret_cast<double*>(smem_raw + (size_t)4 * rowsP * 16 * sizeof(T));  // [3][rowsN][16]: e, f, T
  const int2 tl = g.ptiles[blockIdx.x];
  const int vec = blockIdx.y;
  const int k = tl.x, il0 = tl.y;
  const int m = k * g.m0, nl = g.L - m + 1;
  const int nt = min(kPT, nl - il0);
  const int lm0 = g.lmbase[k] + il0;
  const long long Ma = 4LL * Np * g.vcap;
  const long long mb = Ma * (g.ana_tiled ? g.lmbase8[k] : g.lmbase[k]);
  const T* as = As + mb;
  const T* av = Av + mb;
  const double* vb = v + (long long)vec * ldv;
  double* bb = b + (long long)vec * 6LL * N * g.S;
  double cval = 0.0;
  if (!STEP && J >= 0) cval = v[(long long)vec * ldv + J];
  // the drift speed of the base state is read from device memory in the Jacobian action, so a
  // captured graph of it stays valid when only the base state changes
  if (!STEP) C = Cdev[0];
  // analysis outputs on the N_p nodes: column (c, t) = c * 8 + t
  staged_copy<10, T>(
      4 * rowsP * 16,
      [&](int idx) -> T {
        const int col = idx & 15, rp = (idx >> 4) % rowsP, which = idx / (16 * rowsP);
        const int c = col >> 3, t = col & 7;
        if (rp >= Np || t >= nt) return (T)0;
        // which: 0 Tor (vector slot 2), 1 W_r (scalar slot 0), 2 S (vector slot 0), 3 Q (scalar slot 2)
        const T* src = (which == 1 || which == 3) ? as : av;
        const int slot = (which == 0 || which == 3) ? 2 : 0;
        const long long row = ((long long)vec * Np + rp) * 4 + slot + c;
        return g.ana_tiled ? src[((il0 >> 3) * Ma + row) * 8 + t] : src[row * nl + il0 + t];
      },
      [&](int idx, T val) { Xa[idx] = val; });
  // cleaned state u at the N nodes (coalesced over (j, c) of one profile)
  staged_copy<10, double>(
      3 * kPT * 2 * rowsN,
      [&](int idx) -> double {
        const int cj = idx % (2 * rowsN), t = (idx / (2 * rowsN)) % kPT, f = idx / (2 * rowsN * kPT);
        const int jj = cj >> 1, c = cj & 1;
        if (jj >= N || t >= nt) return 0.0;
        const long long o = 2LL * ((long long)N * ((long long)f * g.S + lm0 + t) + jj) + c;
        const int l = m + il0 + t;
        if (o == J || (c == 1 && k == 0) || (f < 2 && l == 0)) return 0.0;
        return vb[o];
      },
      [&](int idx, double val) {
        const int cj = idx % (2 * rowsN), t = (idx / (2 * rowsN)) % kPT, f = idx / (2 * rowsN * kPT);
        Xu[(f * rowsN + (cj >> 1)) * 16 + (cj & 1) * 8 + t] = val;
      });
  __syncthreads();
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (w >= RTN) return;
  const int col = l & 15, c = col >> 3, t = col & 7;
  // the four N x N_p products
  f64x4 acc[4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
  {
    const long long ms = (long long)RTN * 4 * KBP * 64;
    const double* base = g.PF + (long long)w * 4 * KBP * 64 + l;
    const double* const Mp[4] = {base, base + ms, base + 2 * ms, base + 3 * ms};
    const T* const Xp[4] = {Xa + col, Xa + rowsP * 16 + col, Xa + 2 * rowsP * 16 + col, Xa + 3 * rowsP * 16 + col};
    mfma_f64_products<4, T>(Mp, Xp, 16, KBP, l, acc);
  }
  f64x4 dacc[1] = {{0, 0, 0, 0}};
  {
    const double* const Mp[1] = {g.D2F + (long long)w * 4 * RTN * 64 + l};
    const double* const Xp[1] = {Xu + rowsN * 16 + col};
    mfma_f64_products<1, double>(Mp, Xp, 16, RTN, l, dacc);
  }
  const int il = il0 + t, lw = m + il;
  const double lam = (double)lw * (lw + 1);
  const double sgn = (c == 0) ? -1.0 : 1.0;  // i z: Re <- -Im, Im <- +Re
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double d2f = dacc[0][q];
    const double d2f_o = __shfl_xor(d2f, 8);  // the other component of the same (j, l)
    const int jj = 16 * w + Mfma<double>::out_row(l, q);
    if (jj >= N || t >= nt) continue;
    const double r = g.r[jj], r2 = r * r;
    const double a = ph.Ek * lam / r2;
    const double* ue = Xu + jj * 16 + 8 * c + t;
    const double* uo = Xu + jj * 16 + 8 * (1 - c) + t;
    const double u_e = ue[0], u_f = ue[rowsN * 16], u_T = ue[2 * rowsN * 16];
    const double o_e = uo[0], o_f = uo[rowsN * 16], o_T = uo[2 * rowsN * 16];
    const double Mu[3] = {a * u_e, -a * (d2f - lam / r2 * u_f), u_T};
    const double Mo[3] = {a * o_e, -a * (d2f_o - lam / r2 * o_f), o_T};
    const double nn[3] = {lam * acc[0][q], lam * (acc[1][q] - acc[2][q]) + ph.Ra * lam * u_T / (r * ph.ro), acc[3][q]};
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const long long o = 2LL * ((long long)N * ((long long)f * g.S + lm0 + t) + jj);
      double tv = sgn * m * C * Mo[f];
      if (!STEP) tv += sgn * m * cval * MX[o + 1 - c];
      double bv = Mu[f] + ph.dt * (nn[f] + tv);
      const bool bc = (f == 1) ? (jj == 0 || jj == 1 || jj == N - 2 || jj == N - 1) : (jj == 0 || jj == N - 1);
      if (bc) bv = (STEP && f == 2 && lw == 0 && jj == N - 1 && c == 0) ? 1.0 : 0.0;  // T_00(r_i) = 1
      if (f < 2 && lw == 0) bv = 0.0;
      bb[o + c] = bv;
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
// organised as a segmented scan so that the sequential part is short.  In scaled space
// (t = Rg b, result x = Cg x~), with D_i = S_i^{-1} = diag(sc_i) Shat_i^{-1} diag(sr_i):
//   forward  z_i = c_i - G_i z_{i-1},   c_i = D_i t_i,  G_i = D_i Lo_i
//   backward x_i = z_i - H_i x_{i+1}
// Inside a segment [a, e]: z_i = zeta_i + Phi_i z_{a-1}, x_i = xi_i + Psi_i x_{e+1}, with zeta
// and xi the local recurrences started from zero.  Launches: local forward with c (per
// segment), forward boundary pass (per chain), forward fix-up with the local backward (per
// segment), backward boundary pass (per chain), backward fix-up and output (all blocks).
//
// Every step is y = w + sign M x for one complex N x N block M (or the sum of two such
// products) and 16 right-hand sides, done as three real 16x16x4 MFMA products per k-step
// (Gauss's form of the complex product).  The blocks are stored in the MFMA operand order:
// with RT = ceil(N/16) row tiles and 4 RT k-steps, lane l of (row tile t, k-step s) holds
// M[16t + l%16][4s + l/16] (zero outside N x N), so a wave streams the operands of its k-steps
// with fully coalesced loads straight into registers, ahead of their use (the walks split the
// k-steps of a row tile over several waves; see KqWave).  The output kernel stages x in LDS
// (64 rows x 16 columns, rows >= N zero).  Work vectors live in W[(block*N + j)*wcap + vec]
// (complex, precision F, scaled space); wcap is a multiple of 16 and the columns beyond nvec
// carry zeros.
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

constexpr int kSolveThreads = 256;
constexpr int kVG = 16;  // right-hand sides per workgroup (the MFMA column count)

// complex entries of one block in MFMA operand order
__host__ __device__ constexpr int frag_block_size(int rt) { return 256 * rt * rt; }

template <class F, int RT>
struct ChainOps {
  static constexpr int KS = 4 * RT;
  static constexpr int FB = 256 * RT * RT;
  typedef typename Mfma<F>::acc_t acc_t;

  // registers of one step: operand fragments of this wave's row tile and its w rows
  struct Set {
    F ar[KS], ai[KS];
    cpx<F> w[4];
  };

  int N, wcap, w, l, col;
  int rowc[4];  // output rows of this lane, clamped into [0, N)

  __device__ ChainOps(int N_, int wcap_) : N(N_), wcap(wcap_) {
    w = threadIdx.x >> 6;
    l = threadIdx.x & 63;
    col = l & 15;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = 16 * w + Mfma<F>::out_row(l, q);
      rowc[q] = row < N ? row : N - 1;
    }
  }
  __device__ inline bool active() const { return w < RT; }
  __device__ inline int row(int q) const { return 16 * w + Mfma<F>::out_row(l, q); }

  __device__ inline void load_frag(const cpx<F>* __restrict__ frags, long long blk, Set& S) const {
    const cpx<F>* p = frags + blk * FB + (long long)w * KS * 64 + l;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const cpx<F> v = p[ks * 64];
      S.ar[ks] = v.re;
      S.ai[ks] = v.im;
    }
  }
  __device__ inline void load_w(const cpx<F>* __restrict__ W, long long blk, int v0, Set& S) const {
#pragma unroll
    for (int q = 0; q < 4; ++q) S.w[q] = W[(blk * N + rowc[q]) * wcap + v0 + col];
  }
  // acc = M x for this wave's row tile; x = 64 x 16 complex in LDS.  M = A + iB, x = c + id in
  // three real products (Gauss): P1 = A c, P2 = B d, P3 = (A + B)(c + d); Re = P1 - P2,
  // Im = P3 - P1 - P2.
  __device__ inline void apply(const Set& S, const cpx<F>* x, acc_t& yr, acc_t& yi) const {
    acc_t p1 = {0, 0, 0, 0}, p2 = {0, 0, 0, 0}, p3 = {0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const cpx<F> xv = x[(4 * ks + (l >> 4)) * kVG + col];
      p1 = Mfma<F>::step(S.ar[ks], xv.re, p1);
      p2 = Mfma<F>::step(S.ai[ks], xv.im, p2);
      p3 = Mfma<F>::step(S.ar[ks] + S.ai[ks], xv.re + xv.im, p3);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      yr[q] = p1[q] - p2[q];
      yi[q] = p3[q] - p1[q] - p2[q];
    }
  }
  // The Gauss sums of M x added into (p1, p2, p3), x = sgn * (LDS buffer), or x in registers in
  // the B-operand layout (xv[ks] = x[4 ks + l/16][l % 16]); several products summed this way
  // share one set of sums, finished by yr = p1 - p2, yi = p3 - p1 - p2.
  __device__ inline void acc_lds(const F (&ar)[KS], const F (&ai)[KS], const cpx<F>* x, F sgn, acc_t& p1, acc_t& p2,
                                 acc_t& p3) const {
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const cpx<F> xv = x[(4 * ks + (l >> 4)) * kVG + col];
      const F c = sgn * xv.re, d = sgn * xv.im;
      p1 = Mfma<F>::step(ar[ks], c, p1);
      p2 = Mfma<F>::step(ai[ks], d, p2);
      p3 = Mfma<F>::step(ar[ks] + ai[ks], c + d, p3);
    }
  }
  __device__ inline void acc_reg(const F (&ar)[KS], const F (&ai)[KS], const cpx<F> (&xv)[KS], acc_t& p1, acc_t& p2,
                                 acc_t& p3) const {
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      p1 = Mfma<F>::step(ar[ks], xv[ks].re, p1);
      p2 = Mfma<F>::step(ai[ks], xv[ks].im, p2);
      p3 = Mfma<F>::step(ar[ks] + ai[ks], xv[ks].re + xv[ks].im, p3);
    }
  }
  __device__ inline void load_ops(const cpx<F>* __restrict__ frags, long long blk, F (&ar)[KS], F (&ai)[KS]) const {
    const cpx<F>* p = frags + blk * FB + (long long)w * KS * 64 + l;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const cpx<F> v = p[ks * 64];
      ar[ks] = v.re;
      ai[ks] = v.im;
    }
  }
};

// x block of W (or zero) into a 64 x 16 LDS buffer; the second buffer (if any) is zeroed.
template <class F>
__device__ inline void stage_x(const cpx<F>* __restrict__ W, int N, int wcap, long long blk, int v0, cpx<F>* xa,
                               cpx<F>* xb_zero) {
  staged_copy<64 * kVG / kSolveThreads, cpx<F>>(
      64 * kVG,
      [&](int idx) -> cpx<F> {
        const int r = idx / kVG, c = idx % kVG;
        return (r < N && blk >= 0) ? W[(blk * N + r) * wcap + v0 + c] : cpx<F>{0, 0};
      },
      [&](int idx, cpx<F> v) {
        xa[idx] = v;
        if (xb_zero) xb_zero[idx] = cpx<F>{0, 0};
      });
}

// Walks with the k-steps of each row tile split over four waves.  One CU's matrix cores bound a
// walk step (a complex N x N by N x 16 product per chain or segment), so the step's products
// are spread over all four SIMDs: the 4 RT k-steps of each row tile are split into KQ groups
// (four, two at four row tiles, whose 8 waves then keep 256 VGPRs each), wave (rt, kq) of the
// RT KQ waves multiplies the KW = 4 RT / KQ k-steps of group kq of row tile rt (the Gauss sums
// of 3 KW matrix-core products instead of 12 RT), writes its partial product to LDS, and after
// one barrier every wave sums the KQ partials of the x rows its own k-steps read next,
// x[4 s + l/16][l % 16], straight into registers in the B-operand layout (xrow[j] for its
// k-step j); the waves of row tile 0 store the result.  The partials are double-buffered, so one barrier per step suffices: a buffer is
// written again only after the barrier that every reader of its previous contents has passed.
// Operands are loaded PD steps ahead into a ring of register sets, unconditionally (indices
// clamped), and steps past the end (padding to a multiple of PD) store nothing.
__host__ __device__ constexpr int walk_kq(int rt) { return rt >= 4 ? 2 : 4; }
__host__ __device__ constexpr int walk_threads(int rt) { return 64 * rt * walk_kq(rt); }
template <int RT>
constexpr int walk_part_entries() {  // two buffers of [kq][row][column] partials
  return 2 * walk_kq(RT) * 16 * RT * kVG;
}
// operand sets in flight in a boundary walk: three, two at four row tiles (eight k-steps per wave)
template <int RT>
constexpr int walk_depth() {
  return RT >= 4 ? 2 : 3;
}

template <class F, int RT>
struct KqWave {
  static constexpr int KQ = walk_kq(RT), KW = 4 * RT / KQ, KS = 4 * RT, FB = 256 * RT * RT,
                       PBUF = KQ * 16 * RT * kVG;
  typedef typename Mfma<F>::acc_t acc_t;
  int rt, kq, l, col;
  int xrow[KW], xrowc[KW];  // x rows of this lane's B operands (clamped into [0, N))
  __device__ explicit KqWave(int N) {
    const int wv = threadIdx.x >> 6;
    rt = wv / KQ;
    kq = wv % KQ;
    l = threadIdx.x & 63;
    col = l & 15;
#pragma unroll
    for (int j = 0; j < KW; ++j) {
      xrow[j] = 4 * (kq * KW + j) + (l >> 4);
      xrowc[j] = xrow[j] < N ? xrow[j] : N - 1;
    }
  }
  __device__ inline void load(const cpx<F>* __restrict__ frags, long long blk, F (&ar)[KW], F (&ai)[KW]) const {
    const cpx<F>* p = frags + blk * FB + (long long)(rt * KS + kq * KW) * 64 + l;
#pragma unroll
    for (int j = 0; j < KW; ++j) {
      const cpx<F> v = p[j * 64];
      ar[j] = v.re;
      ai[j] = v.im;
    }
  }
  // Gauss sums of M x over this wave's k-steps added into (p1, p2, p3)
  __device__ inline void gauss(const F (&ar)[KW], const F (&ai)[KW], const cpx<F> (&x)[KW], acc_t& p1, acc_t& p2,
                               acc_t& p3) const {
#pragma unroll
    for (int j = 0; j < KW; ++j) {
      p1 = Mfma<F>::step(ar[j], x[j].re, p1);
      p2 = Mfma<F>::step(ai[j], x[j].im, p2);
      p3 = Mfma<F>::step(ar[j] + ai[j], x[j].re + x[j].im, p3);
    }
  }
  __device__ inline void put(cpx<F>* buf, const acc_t& p1, const acc_t& p2, const acc_t& p3) const {
    cpx<F>* pw = buf + kq * (16 * RT * kVG);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = 16 * rt + Mfma<F>::out_row(l, q);
      pw[r * kVG + col] = cpx<F>{p1[q] - p2[q], p3[q] - p1[q] - p2[q]};
    }
  }
  __device__ inline cpx<F> sum(const cpx<F>* buf, int j) const {
    const int o = xrow[j] * kVG + col;
    constexpr int S = 16 * RT * kVG;
    if (KQ == 2) {
      const cpx<F> s0 = buf[o], s1 = buf[S + o];
      return cpx<F>{s0.re + s1.re, s0.im + s1.im};
    }
    const cpx<F> s0 = buf[o], s1 = buf[S + o], s2 = buf[2 * S + o], s3 = buf[3 * S + o];
    return cpx<F>{(s0.re + s1.re) + (s2.re + s3.re), (s0.im + s1.im) + (s2.im + s3.im)};
  }
};

// Boundary walk: x_0 = W[blk(0)]; for t = 1..nsteps: W[blk(t)] = W[blk(t)] + sign M_blk(t) x_{t-1},
// x_t = that result.
template <class F, int RT, int PD, class BlockOf>
__device__ inline void chain_walk_kq(int N, int wcap, const cpx<F>* __restrict__ frags, cpx<F>* __restrict__ W, int v0,
                                     int nsteps, BlockOf blk_of, F sign, cpx<F>* part) {
  typedef KqWave<F, RT> Kw;
  typedef typename Kw::acc_t acc_t;
  const Kw kw(N);
  struct Set {
    F ar[Kw::KW], ai[Kw::KW];
    cpx<F> wx[Kw::KW];
  };
  auto load = [&](int t, Set& S) {
    const long long b = blk_of(t < nsteps ? t : nsteps);
    kw.load(frags, b, S.ar, S.ai);
#pragma unroll
    for (int j = 0; j < Kw::KW; ++j) S.wx[j] = W[(b * N + kw.xrowc[j]) * wcap + v0 + kw.col];
  };
  cpx<F> x[Kw::KW];
  {
    const long long b0 = blk_of(0);
#pragma unroll
    for (int j = 0; j < Kw::KW; ++j) {
      const cpx<F> v = W[(b0 * N + kw.xrowc[j]) * wcap + v0 + kw.col];
      x[j] = kw.xrow[j] < N ? v : cpx<F>{0, 0};
    }
  }
  Set S[PD];
#pragma unroll
  for (int d = 0; d < PD; ++d) {
    load(1 + d, S[d]);
    __builtin_amdgcn_sched_barrier(0);  // the sets in issue order (the waits count in order)
  }
  int pb = 0;
  auto body = [&](int t, Set& cur) {
    acc_t p1 = {0, 0, 0, 0}, p2 = {0, 0, 0, 0}, p3 = {0, 0, 0, 0};
    kw.gauss(cur.ar, cur.ai, x, p1, p2, p3);
    kw.put(part + pb * Kw::PBUF, p1, p2, p3);
    __syncthreads();
    const long long b = blk_of(t <= nsteps ? t : nsteps);
#pragma unroll
    for (int j = 0; j < Kw::KW; ++j) {
      const cpx<F> sm = kw.sum(part + pb * Kw::PBUF, j);
      const cpx<F> y = {cur.wx[j].re + sign * sm.re, cur.wx[j].im + sign * sm.im};
      x[j] = kw.xrow[j] < N ? y : cpx<F>{0, 0};
      if (kw.rt == 0 && kw.xrow[j] < N && t <= nsteps) W[(b * N + kw.xrow[j]) * wcap + v0 + kw.col] = y;
    }
    load(t + PD, cur);
    pb ^= 1;
  };
  for (int t = 1; t <= nsteps; t += PD) {
#pragma unroll
    for (int d = 0; d < PD; ++d) body(t + d, S[d]);
  }
}

// Forward pass of one segment [a, e] with its right-hand side: c_i = D_i b_i for every block
// of the segment (D_i = diag(sc_i) Shat_i^{-1} diag(sr_i) diag(Rg_i), the scalings folded into
// the stored blocks) and the local recurrence zeta_a = c_a, zeta_i = c_i - G_i zeta_{i-1},
// stored in W (zero columns beyond nvec).  Each step sums both products in one set of Gauss
// sums on the k-split waves (see KqWave); b is read from the FP64 input straight into the
// B-operand layout (rows and vectors clamped, masked at use), and the operands of the next two
// steps are in flight (local_sets).  One workgroup of RT KQ waves per (segment, vector group).
// Operand sets of a local walk: the loads of step t + NS - 1 are issued (behind a scheduling
// barrier, so that the compiler keeps them there) before the products of step t; two sets at
// three row tiles (three would spill there), one at four (eight k-steps of two blocks per wave).
template <int RT>
constexpr int local_sets() {
  return RT >= 4 ? 1 : RT >= 3 ? 2 : 3;
}
template <class F, int RT>
__global__ void __launch_bounds__(walk_threads(RT), 1) k_cs_fwd_rhs(DevGrid g, int nvec, const SegMeta* __restrict__ segs,
                                                                     const int* __restrict__ blk_field,
                                                                     const int* __restrict__ blk_lm,
                                                                     const cpx<F>* __restrict__ Dm,
                                                                     const cpx<F>* __restrict__ Gm,
                                                                     const double* __restrict__ bvec,
                                                                     cpx<F>* __restrict__ W) {
  __shared__ cpx<F> part[walk_part_entries<RT>()];
  typedef KqWave<F, RT> Kw;
  typedef typename Kw::acc_t acc_t;
  const SegMeta sg = segs[blockIdx.x];
  const int N = g.N, a = sg.first_block, len = sg.len, v0 = blockIdx.y * kVG, nv = min(kVG, nvec - v0);
  const Kw kw(N);
  const long long ld = 6LL * N * g.S;
  const long long vrow = (long long)(v0 + min(kw.col, nv - 1)) * ld;  // this lane's vector, clamped
  bool bok[Kw::KW];
#pragma unroll
  for (int j = 0; j < Kw::KW; ++j) bok[j] = kw.xrow[j] < N && kw.col < nv;
  struct Set {
    F dr[Kw::KW], di[Kw::KW], gr[Kw::KW], gi[Kw::KW];
    double2 b[Kw::KW];
  };
  auto load = [&](int t, Set& S) {
    const long long blk = a + (t < len ? t : len - 1);
    kw.load(Dm, blk, S.dr, S.di);
    kw.load(Gm, blk, S.gr, S.gi);
    const double* bp = bvec + vrow + 2LL * ((long long)N * ((long long)blk_field[blk] * g.S + blk_lm[blk]));
#pragma unroll
    for (int j = 0; j < Kw::KW; ++j) S.b[j] = *reinterpret_cast<const double2*>(bp + 2 * kw.xrowc[j]);
  };
  cpx<F> x[Kw::KW];  // -zeta_{i-1} in the B-operand layout (zero before the first step)
#pragma unroll
  for (int j = 0; j < Kw::KW; ++j) x[j] = cpx<F>{0, 0};
  constexpr int NS = local_sets<RT>();
  Set S[NS];
#pragma unroll
  for (int d = 0; d + 1 < NS; ++d) {
    load(d, S[d]);
    __builtin_amdgcn_sched_barrier(0);  // the sets in issue order (the waits count in order)
  }
  int pb = 0;
  // steps past the segment (padding to a multiple of NS) skip the products and store nothing
  auto body = [&](int t, Set& cur, Set& ahead) {
    load(t + NS - 1, ahead);
    __builtin_amdgcn_sched_barrier(0);
    if (t < len) {
      acc_t p1 = {0, 0, 0, 0}, p2 = {0, 0, 0, 0}, p3 = {0, 0, 0, 0};
      cpx<F> bv[Kw::KW];
#pragma unroll
      for (int j = 0; j < Kw::KW; ++j) bv[j] = bok[j] ? cpx<F>{(F)cur.b[j].x, (F)cur.b[j].y} : cpx<F>{0, 0};
      kw.gauss(cur.dr, cur.di, bv, p1, p2, p3);
      kw.gauss(cur.gr, cur.gi, x, p1, p2, p3);
      kw.put(part + pb * Kw::PBUF, p1, p2, p3);
    }
    __syncthreads();
    if (t < len) {
      const long long blk = a + t;
#pragma unroll
      for (int j = 0; j < Kw::KW; ++j) {
        const cpx<F> y = kw.sum(part + pb * Kw::PBUF, j);
        x[j] = kw.xrow[j] < N ? cpx<F>{-y.re, -y.im} : cpx<F>{0, 0};
        if (kw.rt == 0 && kw.xrow[j] < N) W[(blk * N + kw.xrow[j]) * g.wcap + v0 + kw.col] = y;
      }
    }
    pb ^= 1;
  };
  for (int t = 0; t < len; t += NS) {
#pragma unroll
    for (int d = 0; d < NS; ++d) body(t + d, S[d], S[(d + NS - 1) % NS]);
  }
}

// Block product for one right-hand side (nvec = 1) on the vector units, the output kernel's
// layout: lane l of wave w (w < RT) holds M[16 w + l%16][4 s + l/16] for every k-step s, forms
// that row's partial sum over the columns = l/16 (mod 4), and the four partial sums of a row
// meet by lane exchanges (rowsum4).  Waves beyond the row tiles load the last tile's operands
// and write nothing.
template <class F, int RT>
struct Lane1 {
  static constexpr int KS = 4 * RT, FB = 256 * RT * RT;
  int w, l, c0, row, rowc;
  bool writer;
  __device__ Lane1(int N) {
    w = min((int)(threadIdx.x >> 6), RT - 1);
    l = threadIdx.x & 63;
    c0 = l >> 4;
    row = 16 * w + (l & 15);
    rowc = row < N ? row : N - 1;
    writer = (int)(threadIdx.x >> 6) < RT && c0 == 0 && row < N;
  }
  __device__ inline void load(const cpx<F>* __restrict__ frags, long long blk, F (&ar)[KS], F (&ai)[KS]) const {
    const cpx<F>* p = frags + blk * FB + (long long)w * KS * 64 + l;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const cpx<F> v = p[ks * 64];
      ar[ks] = v.re;
      ai[ks] = v.im;
    }
  }
  __device__ static inline void rowsum4(F& re, F& im) {
    re += __shfl_xor(re, 16);
    im += __shfl_xor(im, 16);
    re += __shfl_xor(re, 32);
    im += __shfl_xor(im, 32);
  }
};

// Walks for one right-hand side (nvec = 1) on the vector units, with the waves of KqWave: lane l
// of wave (rt, kq) holds the operands M[16 rt + l%16][4 s + l/16] of its group's k-steps s
// (the stored MFMA operand order) and the entries x[4 s + l/16] they multiply, forms its part
// of row 16 rt + l%16, and the four parts of a row meet by lane exchanges; the groups' sums meet
// through LDS (double-buffered, one barrier per step), and every lane then sums the x entries
// its own k-steps read next straight into registers.  A 16-column matrix-core product would
// spend 15 of its columns on padding.  A lane's operand set is KW fragments per block plus KW
// right-hand-side or w entries, so the sets of several steps stay within the 63 loads the
// memory counter tracks.
template <class F, int RT>
struct Kq1 {
  static constexpr int KQ = walk_kq(RT), KW = 4 * RT / KQ, KS = 4 * RT, FB = 256 * RT * RT, PBUF = KQ * 64;
  int rt, kq, l, c0, row;
  int xrow[KW], xrowc[KW];
  bool writer;  // column-0 lanes of row tile 0 store the x entries they hold
  __device__ explicit Kq1(int N) {
    const int wv = threadIdx.x >> 6;
    rt = wv / KQ;
    kq = wv % KQ;
    l = threadIdx.x & 63;
    c0 = l >> 4;
    row = 16 * rt + (l & 15);
#pragma unroll
    for (int j = 0; j < KW; ++j) {
      xrow[j] = 4 * (kq * KW + j) + c0;
      xrowc[j] = xrow[j] < N ? xrow[j] : N - 1;
    }
    writer = rt == 0 && (l & 15) == 0;
  }
  __device__ inline void load(const cpx<F>* __restrict__ frags, long long blk, F (&ar)[KW], F (&ai)[KW]) const {
    const cpx<F>* p = frags + blk * FB + (long long)(rt * KS + kq * KW) * 64 + l;
#pragma unroll
    for (int j = 0; j < KW; ++j) {
      const cpx<F> v = p[j * 64];
      ar[j] = v.re;
      ai[j] = v.im;
    }
  }
  // (re, im) += this lane's part of row M x
  __device__ static inline void dot(const F (&ar)[KW], const F (&ai)[KW], const cpx<F> (&x)[KW], F& re, F& im) {
#pragma unroll
    for (int j = 0; j < KW; ++j) {
      re += ar[j] * x[j].re - ai[j] * x[j].im;
      im += ar[j] * x[j].im + ai[j] * x[j].re;
    }
  }
  // the row's sum over this group's k-steps into buf[kq][row]
  __device__ inline void put(cpx<F>* buf, F re, F im) const {
    re += __shfl_xor(re, 16);
    im += __shfl_xor(im, 16);
    re += __shfl_xor(re, 32);
    im += __shfl_xor(im, 32);
    if (c0 == 0) buf[kq * 64 + row] = cpx<F>{re, im};
  }
  __device__ inline cpx<F> sum(const cpx<F>* buf, int j) const {
    const int o = xrow[j];
    if (KQ == 2) return cpx<F>{buf[o].re + buf[64 + o].re, buf[o].im + buf[64 + o].im};
    const cpx<F> s0 = buf[o], s1 = buf[64 + o], s2 = buf[128 + o], s3 = buf[192 + o];
    return cpx<F>{(s0.re + s1.re) + (s2.re + s3.re), (s0.im + s1.im) + (s2.im + s3.im)};
  }
};

// Operand sets of the one-vector walks: the loads of step t + NS - 1 are issued (behind a
// scheduling barrier) before the products of step t; steps past the end skip the products.
// One set at four row tiles (eight k-steps of two blocks per lane: two sets would spill).
template <int RT>
constexpr int walk1_sets() {
  return RT >= 4 ? 1 : 3;
}

// Boundary walk for one right-hand side: x_0 = W[blk(0)]; for t = 1..nsteps:
// W[blk(t)] = W[blk(t)] + M_blk(t) x_{t-1}, x_t = that result.
template <class F, int RT, class BlockOf>
__device__ inline void chain_walk1(int N, int wcap, const cpx<F>* __restrict__ frags, cpx<F>* __restrict__ W,
                                   int nsteps, BlockOf blk_of, cpx<F>* part) {
  typedef Kq1<F, RT> Kw;
  constexpr int KW = Kw::KW, NS = walk1_sets<RT>();
  const Kw kw(N);
  struct Set {
    F ar[KW], ai[KW];
    cpx<F> w[KW];
  };
  auto load = [&](int t, Set& S) {
    const long long b = blk_of(t < nsteps ? t : nsteps);
    kw.load(frags, b, S.ar, S.ai);
#pragma unroll
    for (int j = 0; j < KW; ++j) S.w[j] = W[(b * N + kw.xrowc[j]) * wcap];
  };
  cpx<F> x[KW];
  {
    const long long b0 = blk_of(0);
#pragma unroll
    for (int j = 0; j < KW; ++j) {
      const cpx<F> v = W[(b0 * N + kw.xrowc[j]) * wcap];
      x[j] = kw.xrow[j] < N ? v : cpx<F>{0, 0};
    }
  }
  Set S[NS];
#pragma unroll
  for (int d = 0; d + 1 < NS; ++d) {
    load(1 + d, S[d]);
    __builtin_amdgcn_sched_barrier(0);  // the sets in issue order (the waits count in order)
  }
  int pb = 0;
  auto body = [&](int t, Set& cur, Set& ahead) {
    load(t + NS - 1, ahead);
    __builtin_amdgcn_sched_barrier(0);
    if (t <= nsteps) {
      F re = 0, im = 0;
      Kw::dot(cur.ar, cur.ai, x, re, im);
      kw.put(part + pb * Kw::PBUF, re, im);
    }
    __syncthreads();
    if (t <= nsteps) {
      const long long b = blk_of(t);
#pragma unroll
      for (int j = 0; j < KW; ++j) {
        const cpx<F> sm = kw.sum(part + pb * Kw::PBUF, j);
        const cpx<F> y = {cur.w[j].re + sm.re, cur.w[j].im + sm.im};
        x[j] = kw.xrow[j] < N ? y : cpx<F>{0, 0};
        if (kw.writer && kw.xrow[j] < N) W[(b * N + kw.xrow[j]) * wcap] = y;
      }
    }
    pb ^= 1;
  };
  for (int t = 1; t <= nsteps; t += NS) {
#pragma unroll
    for (int d = 0; d < NS; ++d) body(t + d, S[d], S[(d + NS - 1) % NS]);
  }
}

// Boundary passes for one right-hand side: one workgroup of RT KQ waves per chain.
template <class F, int RT>
__global__ void __launch_bounds__(walk_threads(RT), 1) k_cs1_fwd_bound(DevGrid g, const ChainMeta* __restrict__ chains,
                                                                      int seg, const cpx<F>* __restrict__ Phi,
                                                                      cpx<F>* __restrict__ W) {
  __shared__ cpx<F> part[2 * Kq1<F, RT>::PBUF];
  const ChainMeta ch = chains[blockIdx.x];
  if (ch.nseg <= 1) return;
  const int st = ch.start, n = ch.n;
  chain_walk1<F, RT>(g.N, g.wcap, Phi, W, ch.nseg - 1,
                     [&](int p) { return (long long)(st + min((p + 1) * seg, n) - 1); }, part);
}

template <class F, int RT>
__global__ void __launch_bounds__(walk_threads(RT), 1) k_cs1_bwd_bound(DevGrid g, const ChainMeta* __restrict__ chains,
                                                                      int seg, const cpx<F>* __restrict__ Psi,
                                                                      cpx<F>* __restrict__ W) {
  __shared__ cpx<F> part[2 * Kq1<F, RT>::PBUF];
  const ChainMeta ch = chains[blockIdx.x];
  if (ch.nseg <= 1) return;
  const int st = ch.start, last = ch.nseg - 1;
  chain_walk1<F, RT>(g.N, g.wcap, Psi, W, ch.nseg - 1, [&](int t) { return (long long)(st + (last - t) * seg); },
                     part);
}

// Local walks for one right-hand side (as k_cs_fwd_rhs and k_cs_bwd_fix): one workgroup of
// RT KQ waves per segment.  The results stay in LDS until the walk ends (no store inside the
// loop, whose conditional form would make the compiler wait on the prefetched operands) and are
// then written out together.
constexpr int kSegMax = 16;  // longest scan segment the one-vector local walks hold in LDS
template <class F, int RT>
__global__ void __launch_bounds__(walk_threads(RT), 1) k_cs1_fwd_rhs(DevGrid g, const SegMeta* __restrict__ segs,
                                                                    const int* __restrict__ blk_field,
                                                                    const int* __restrict__ blk_lm,
                                                                    const cpx<F>* __restrict__ Dm,
                                                                    const cpx<F>* __restrict__ Gm,
                                                                    const double* __restrict__ bvec,
                                                                    cpx<F>* __restrict__ W) {
  typedef Kq1<F, RT> Kw;
  constexpr int KW = Kw::KW, NS = walk1_sets<RT>();
  __shared__ cpx<F> part[2 * Kw::PBUF];
  __shared__ cpx<F> ys[kSegMax * 64];  // the segment's results, stored after the walk
  const SegMeta sg = segs[blockIdx.x];
  const int N = g.N, a = sg.first_block, len = sg.len, wcap = g.wcap;
  const Kw kw(N);
  struct Set {
    F dr[KW], di[KW], gr[KW], gi[KW];
    double2 b[KW];
  };
  auto load = [&](int t, Set& S) {
    const long long blk = a + (t < len ? t : len - 1);
    kw.load(Dm, blk, S.dr, S.di);
    kw.load(Gm, blk, S.gr, S.gi);
    const double* bp = bvec + 2LL * ((long long)N * ((long long)blk_field[blk] * g.S + blk_lm[blk]));
#pragma unroll
    for (int j = 0; j < KW; ++j) S.b[j] = *reinterpret_cast<const double2*>(bp + 2 * kw.xrowc[j]);
  };
  cpx<F> x[KW];  // -zeta_{i-1} (zero before the first step)
#pragma unroll
  for (int j = 0; j < KW; ++j) x[j] = cpx<F>{0, 0};
  Set S[NS];
#pragma unroll
  for (int d = 0; d + 1 < NS; ++d) {
    load(d, S[d]);
    __builtin_amdgcn_sched_barrier(0);  // the sets in issue order (the waits count in order)
  }
  int pb = 0;
  auto body = [&](int t, Set& cur, Set& ahead) {
    load(t + NS - 1, ahead);
    __builtin_amdgcn_sched_barrier(0);
    if (t < len) {
      cpx<F> bv[KW];
#pragma unroll
      for (int j = 0; j < KW; ++j) bv[j] = kw.xrow[j] < N ? cpx<F>{(F)cur.b[j].x, (F)cur.b[j].y} : cpx<F>{0, 0};
      F re = 0, im = 0;
      Kw::dot(cur.dr, cur.di, bv, re, im);
      Kw::dot(cur.gr, cur.gi, x, re, im);
      kw.put(part + pb * Kw::PBUF, re, im);
    }
    __syncthreads();
    if (t < len) {
#pragma unroll
      for (int j = 0; j < KW; ++j) {
        const cpx<F> y = kw.sum(part + pb * Kw::PBUF, j);
        x[j] = kw.xrow[j] < N ? cpx<F>{-y.re, -y.im} : cpx<F>{0, 0};
        if (kw.writer) ys[t * 64 + kw.xrow[j]] = y;
      }
    }
    pb ^= 1;
  };
  for (int t = 0; t < len; t += NS) {
#pragma unroll
    for (int d = 0; d < NS; ++d) body(t + d, S[d], S[(d + NS - 1) % NS]);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < len * N; i += blockDim.x) {
    const int t = i / N, r = i - t * N;
    W[((long long)(a + t) * N + r) * wcap] = ys[t * 64 + r];
  }
}

template <class F, int RT>
__global__ void __launch_bounds__(walk_threads(RT), 1) k_cs1_bwd_fix(DevGrid g, const SegMeta* __restrict__ segs,
                                                                    const cpx<F>* __restrict__ Phi,
                                                                    const cpx<F>* __restrict__ H, cpx<F>* __restrict__ W) {
  typedef Kq1<F, RT> Kw;
  constexpr int KW = Kw::KW, NS = walk1_sets<RT>();
  __shared__ cpx<F> part[2 * Kw::PBUF];
  __shared__ cpx<F> ys[kSegMax * 64];  // the segment's results, stored after the walk
  const SegMeta sg = segs[blockIdx.x];
  if (sg.len <= 1) return;
  const int N = g.N, a = sg.first_block, len = sg.len, e = a + len - 1, wcap = g.wcap;
  const bool fix = sg.pidx > 0;
  const Kw kw(N);
  const long long ap = a > 0 ? a - 1 : 0;
  cpx<F> x[KW], zs[KW];  // -xi_{i+1} and z_{a-1} (zero in a chain's first segment)
#pragma unroll
  for (int j = 0; j < KW; ++j) {
    const cpx<F> v = W[((long long)e * N + kw.xrowc[j]) * wcap];
    const cpx<F> z = W[(ap * N + kw.xrowc[j]) * wcap];
    x[j] = kw.xrow[j] < N ? cpx<F>{-v.re, -v.im} : cpx<F>{0, 0};
    zs[j] = (fix && kw.xrow[j] < N) ? z : cpx<F>{0, 0};
  }
  struct Set {
    F hr[KW], hi[KW], pr[KW], pi[KW];
    cpx<F> w[KW];
  };
  auto load = [&](int t, Set& S) {
    const long long blk = e - (t < len ? t : len - 1);
    kw.load(H, blk, S.hr, S.hi);
    kw.load(Phi, blk, S.pr, S.pi);
#pragma unroll
    for (int j = 0; j < KW; ++j) S.w[j] = W[(blk * N + kw.xrowc[j]) * wcap];
  };
  Set S[NS];
#pragma unroll
  for (int d = 0; d + 1 < NS; ++d) {
    load(1 + d, S[d]);
    __builtin_amdgcn_sched_barrier(0);  // the sets in issue order (the waits count in order)
  }
  int pb = 0;
  auto body = [&](int t, Set& cur, Set& ahead) {
    load(t + NS - 1, ahead);
    __builtin_amdgcn_sched_barrier(0);
    if (t < len) {
      F re = 0, im = 0;
      Kw::dot(cur.pr, cur.pi, zs, re, im);
      Kw::dot(cur.hr, cur.hi, x, re, im);
      kw.put(part + pb * Kw::PBUF, re, im);
    }
    __syncthreads();
    if (t < len) {
#pragma unroll
      for (int j = 0; j < KW; ++j) {
        const cpx<F> sm = kw.sum(part + pb * Kw::PBUF, j);
        const cpx<F> y = {cur.w[j].re + sm.re, cur.w[j].im + sm.im};
        x[j] = kw.xrow[j] < N ? cpx<F>{-y.re, -y.im} : cpx<F>{0, 0};
        if (kw.writer) ys[t * 64 + kw.xrow[j]] = y;
      }
    }
    pb ^= 1;
  };
  for (int t = 1; t < len; t += NS) {
#pragma unroll
    for (int d = 0; d < NS; ++d) body(t + d, S[d], S[(d + NS - 1) % NS]);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < (len - 1) * N; i += blockDim.x) {
    const int t = 1 + i / N, r = i - (t - 1) * N;
    W[((long long)(e - t) * N + r) * wcap] = ys[t * 64 + r];
  }
}

// Boundary pass of the forward recurrence: z_e(p) = zeta_e(p) + Phi_e(p) z_e(p-1).
// One workgroup of RT KQ waves per (chain, vector group).
template <class F, int RT>
__global__ void __launch_bounds__(walk_threads(RT), 1) k_cs_fwd_bound(DevGrid g, int nvec, const ChainMeta* __restrict__ chains,
                                                                       int seg, const cpx<F>* __restrict__ Phi,
                                                                       cpx<F>* __restrict__ W) {
  __shared__ cpx<F> part[walk_part_entries<RT>()];
  const ChainMeta ch = chains[blockIdx.x];
  if (ch.nseg <= 1) return;
  const int st = ch.start, n = ch.n;
  chain_walk_kq<F, RT, walk_depth<RT>()>(g.N, g.wcap, Phi, W, blockIdx.y * kVG, ch.nseg - 1,
                                   [&](int p) { return (long long)(st + min((p + 1) * seg, n) - 1); }, (F)1, part);
}

// Backward pass of one segment [a, e] with the forward fix-up: the forward values of a segment
// p > 0 are completed on the way, z_i = zeta_i + Phi_i z_{a-1} (z_{a-1}, the previous segment's
// last value, and z_e are final after the forward boundary pass), and the local backward
// recurrence xi_e = z_e, xi_i = z_i - H_i xi_{i+1} runs from e down to a, stored in W.  Each
// step sums both products in one set of Gauss sums on the k-split waves (see KqWave); z_{a-1}
// is held in registers in the B-operand layout (zero in a chain's first segment, whose Phi
// blocks are then multiplied by zero), and the operands of the next two steps are in flight.
template <class F, int RT>
__global__ void __launch_bounds__(walk_threads(RT), 1) k_cs_bwd_fix(DevGrid g, int nvec, const SegMeta* __restrict__ segs,
                                                                     const cpx<F>* __restrict__ Phi,
                                                                     const cpx<F>* __restrict__ H, cpx<F>* __restrict__ W) {
  __shared__ cpx<F> part[walk_part_entries<RT>()];
  typedef KqWave<F, RT> Kw;
  typedef typename Kw::acc_t acc_t;
  const SegMeta sg = segs[blockIdx.x];
  if (sg.len <= 1) return;
  const int N = g.N, a = sg.first_block, len = sg.len, e = a + len - 1, v0 = blockIdx.y * kVG;
  const bool fix = sg.pidx > 0;
  const Kw kw(N);
  const long long ap = a > 0 ? a - 1 : 0;
  cpx<F> x[Kw::KW], zs[Kw::KW];  // -xi_{i+1} and z_{a-1}
#pragma unroll
  for (int j = 0; j < Kw::KW; ++j) {
    const cpx<F> v = W[((long long)e * N + kw.xrowc[j]) * g.wcap + v0 + kw.col];
    const cpx<F> z = W[(ap * N + kw.xrowc[j]) * g.wcap + v0 + kw.col];
    x[j] = kw.xrow[j] < N ? cpx<F>{-v.re, -v.im} : cpx<F>{0, 0};
    zs[j] = (fix && kw.xrow[j] < N) ? z : cpx<F>{0, 0};
  }
  struct Set {
    F hr[Kw::KW], hi[Kw::KW], pr[Kw::KW], pi[Kw::KW];
    cpx<F> w[Kw::KW];
  };
  auto load = [&](int t, Set& S) {
    const long long blk = e - (t < len ? t : len - 1);
    kw.load(H, blk, S.hr, S.hi);
    kw.load(Phi, blk, S.pr, S.pi);
#pragma unroll
    for (int j = 0; j < Kw::KW; ++j) S.w[j] = W[(blk * N + kw.xrowc[j]) * g.wcap + v0 + kw.col];
  };
  constexpr int NS = local_sets<RT>();
  Set S[NS];
#pragma unroll
  for (int d = 0; d + 1 < NS; ++d) {
    load(1 + d, S[d]);
    __builtin_amdgcn_sched_barrier(0);  // the sets in issue order (the waits count in order)
  }
  int pb = 0;
  auto body = [&](int t, Set& cur, Set& ahead) {
    load(t + NS - 1, ahead);
    __builtin_amdgcn_sched_barrier(0);
    if (t < len) {
      acc_t p1 = {0, 0, 0, 0}, p2 = {0, 0, 0, 0}, p3 = {0, 0, 0, 0};
      kw.gauss(cur.pr, cur.pi, zs, p1, p2, p3);
      kw.gauss(cur.hr, cur.hi, x, p1, p2, p3);
      kw.put(part + pb * Kw::PBUF, p1, p2, p3);
    }
    __syncthreads();
    if (t < len) {
      const long long blk = e - t;
#pragma unroll
      for (int j = 0; j < Kw::KW; ++j) {
        const cpx<F> sm = kw.sum(part + pb * Kw::PBUF, j);
        const cpx<F> y = {cur.w[j].re + sm.re, cur.w[j].im + sm.im};
        x[j] = kw.xrow[j] < N ? cpx<F>{-y.re, -y.im} : cpx<F>{0, 0};
        if (kw.rt == 0 && kw.xrow[j] < N) W[(blk * N + kw.xrow[j]) * g.wcap + v0 + kw.col] = y;
      }
    }
    pb ^= 1;
  };
  for (int t = 1; t < len; t += NS) {
#pragma unroll
    for (int d = 0; d < NS; ++d) body(t + d, S[d], S[(d + NS - 1) % NS]);
  }
}

// Boundary pass of the backward recurrence: x_a(p) = xi_a(p) + Psi_a(p) x_a(p+1).
template <class F, int RT>
__global__ void __launch_bounds__(walk_threads(RT), 1) k_cs_bwd_bound(DevGrid g, int nvec, const ChainMeta* __restrict__ chains,
                                                                       int seg, const cpx<F>* __restrict__ Psi,
                                                                       cpx<F>* __restrict__ W) {
  __shared__ cpx<F> part[walk_part_entries<RT>()];
  const ChainMeta ch = chains[blockIdx.x];
  if (ch.nseg <= 1) return;
  const int st = ch.start, last = ch.nseg - 1;
  chain_walk_kq<F, RT, walk_depth<RT>()>(g.N, g.wcap, Psi, W, blockIdx.y * kVG, ch.nseg - 1,
                                   [&](int t) { return (long long)(st + (last - t) * seg); }, (F)1, part);
}

// x_i = xi_i + Psi_i x_{a(p+1)} for the blocks not yet final, then x = Cg x~ into the
// canonical FP64 output (ACC: added to it, the update of a refinement pass; FIN: the sum is
// not stored but turned into the Jacobian action y = clean(x) - u).  One workgroup per
// (block, vector group).
template <class F, int RT, bool ACC, bool FIN>
__global__ void __launch_bounds__(kSolveThreads) k_cs_out(DevGrid g, int nvec, const int* __restrict__ blk_field,
                                                         const int* __restrict__ blk_lm, const int* __restrict__ blk_next,
                                                         const cpx<F>* __restrict__ Psi, const F* __restrict__ Cg,
                                                         const cpx<F>* __restrict__ W, double* __restrict__ xvec,
                                                         FinalOut fo) {
  __shared__ cpx<F> xs[64 * kVG];
  typedef ChainOps<F, RT> Ops;
  const int N = g.N;
  Ops op(N, g.wcap);
  const int blk = blockIdx.x, v0 = blockIdx.y * kVG, nv = min(kVG, nvec - v0);
  const int nx = blk_next[blk];
  typename Ops::Set S;
  if (op.active()) {
    if (nx >= 0) op.load_frag(Psi, blk, S);
    op.load_w(W, blk, v0, S);
  }
  if (nx >= 0) stage_x<F>(W, N, g.wcap, nx, v0, xs, nullptr);
  // the output's other operands (scaling, accumulated x, u) load before the product
  const long long ld = 6LL * N * g.S;
  const int lm = blk_lm[blk];
  const long long o = 2LL * ((long long)N * ((long long)blk_field[blk] * g.S + lm));
  double cq[4], xa[4][2], ua[4][2];
  if (op.active()) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = op.row(q);
      const bool ok = r < N && op.col < nv;
      const long long oo = o + 2 * r;
      cq[q] = ok ? (double)Cg[(long long)blk * N + r] : 0.0;
      xa[q][0] = xa[q][1] = ua[q][0] = ua[q][1] = 0.0;
      if (ACC && ok) {
        const double* xp = xvec + (long long)(v0 + op.col) * ld + oo;
        xa[q][0] = xp[0];
        xa[q][1] = xp[1];
      }
      if (FIN && ok) {
        const double* vp = fo.v + (long long)(v0 + op.col) * fo.ldv + oo;
        ua[q][0] = (oo == fo.J) ? 0.0 : vp[0];
        ua[q][1] = (oo + 1 == fo.J) ? 0.0 : vp[1];
      }
    }
  }
  __syncthreads();
  if (op.active()) {
    typename Ops::acc_t yr = {0, 0, 0, 0}, yi = {0, 0, 0, 0};
    if (nx >= 0) op.apply(S, xs, yr, yi);
    const bool mzero = (g.lm_k[lm] == 0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = op.row(q);
      if (r < N && op.col < nv) {
        const double c = cq[q];
        const long long oo = o + 2 * r;
        double x0 = c * (double)(S.w[q].re + yr[q]) + xa[q][0], x1 = c * (double)(S.w[q].im + yi[q]) + xa[q][1];
        if (FIN) {
          double* yp = fo.y + (long long)(v0 + op.col) * fo.ldy + oo;
          yp[0] = x0 - ua[q][0];
          yp[1] = (mzero ? 0.0 : x1) - ua[q][1];
        } else {
          double* xp = xvec + (long long)(v0 + op.col) * ld + oo;
          xp[0] = x0;
          xp[1] = x1;
        }
      }
    }
  }
}

// Backward fix-up and output for one right-hand side (as k_cs_out, on the vector units; see
// Lane1): the 16-column kernel would also stage the 15 unused columns of W.  One workgroup per
// block; the operands of the product, and x_{a(p+1)}, are read in the B-operand layout and
// masked at their use.
template <class F, int RT, bool ACC, bool FIN>
__global__ void __launch_bounds__(kSolveThreads) k_cs1_out(DevGrid g, const int* __restrict__ blk_field,
                                                          const int* __restrict__ blk_lm,
                                                          const int* __restrict__ blk_next,
                                                          const cpx<F>* __restrict__ Psi, const F* __restrict__ Cg,
                                                          const cpx<F>* __restrict__ W, double* __restrict__ xvec,
                                                          FinalOut fo) {
  typedef Lane1<F, RT> Ln;
  constexpr int KS = Ln::KS;
  const int N = g.N, wcap = g.wcap, blk = blockIdx.x, nx = blk_next[blk];
  const Ln ln(N);
  F ar[KS], ai[KS];
  ln.load(Psi, blk, ar, ai);
  cpx<F> xv[KS];
  {
    const long long bx = nx >= 0 ? nx : blk;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int r = 4 * ks + ln.c0, rr = r < N ? r : N - 1;
      xv[ks] = W[(bx * N + rr) * wcap];
    }
  }
  const cpx<F> wv = W[((long long)blk * N + ln.rowc) * wcap];
  const int lm = blk_lm[blk];
  const long long oo = 2LL * ((long long)N * ((long long)blk_field[blk] * g.S + lm)) + 2 * ln.rowc;
  const double cq = (double)Cg[(long long)blk * N + ln.rowc];
  double xa0 = 0.0, xa1 = 0.0, ua0 = 0.0, ua1 = 0.0;
  if (ACC) {
    xa0 = xvec[oo];
    xa1 = xvec[oo + 1];
  }
  if (FIN) {
    ua0 = fo.v[oo];
    ua1 = fo.v[oo + 1];
  }
  F re = 0, im = 0;
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const bool ok = nx >= 0 && 4 * ks + ln.c0 < N;
    const F xr = ok ? xv[ks].re : (F)0, xi = ok ? xv[ks].im : (F)0;
    re += ar[ks] * xr - ai[ks] * xi;
    im += ar[ks] * xi + ai[ks] * xr;
  }
  Ln::rowsum4(re, im);
  if (ln.writer) {
    const double x0 = cq * (double)(wv.re + re) + xa0, x1 = cq * (double)(wv.im + im) + xa1;
    if (FIN) {
      const bool mzero = (g.lm_k[lm] == 0);
      fo.y[oo] = x0 - (oo == fo.J ? 0.0 : ua0);
      fo.y[oo + 1] = (mzero ? 0.0 : x1) - (oo + 1 == fo.J ? 0.0 : ua1);
    } else {
      xvec[oo] = x0;
      xvec[oo + 1] = x1;
    }
  }
}

// Temperature blocks: x = tc * Tinv (tr * b) per l, for every (vec, k, l), both Re and Im
// (ACC: added to x; FIN: y = clean(x) - u is written instead of x, and the workgroups of l = 0
// also write y = -u on the e, f slots at l = 0, which no chain covers).  One workgroup per
// (l, group of kTV vectors): Tinv_l and the columns (vec, k, Re/Im) staged in LDS, the product
// on the matrix cores.
constexpr int kTV = 4;

template <class F, bool ACC, bool FIN>
__global__ void __launch_bounds__(256) k_T_solve(DevGrid g, int nvec, const F* __restrict__ Tinv,
                                                 const F* __restrict__ tr, const F* __restrict__ tc,
                                                 const double* __restrict__ bvec, double* __restrict__ xvec,
                                                 FinalOut fo) {
  typedef typename Mfma<F>::acc_t acc_t;
  extern __shared__ unsigned char smem_raw[];
  const int N = g.N, NP1 = N + 1;                 // padded LDS row stride
  F* Ts = reinterpret_cast<F*>(smem_raw);         // [N][N + 1]: Ts[r * NP1 + k] = Tinv[r][k]
  F* bs = Ts + N * NP1;                           // [ncol][N + 1]: right-hand side columns
  const int l = blockIdx.x;
  const int v0 = blockIdx.y * kTV, nv = min(kTV, nvec - v0);
  const int nk = min(g.K, l / g.m0) + 1;          // m = k m0 <= l
  const int ncol = nv * nk * 2;
  const long long ld = 6LL * N * g.S;
  for (int i = threadIdx.x; i < N * N; i += blockDim.x) Ts[(i / N) * NP1 + i % N] = Tinv[(long long)l * N * N + i];
  for (int idx = threadIdx.x; idx < ncol * N; idx += blockDim.x) {
    int jj = idx % N, col = idx / N;
    int ri = col & 1, kk = (col >> 1) % nk, vv = (col >> 1) / nk;
    int lm = g.lmbase[kk] + l - kk * g.m0;
    long long o = (long long)(v0 + vv) * ld + 2LL * ((long long)N * (2LL * g.S + lm) + jj) + ri;
    bs[col * NP1 + jj] = tr[(long long)l * N + jj] * (F)bvec[o];
  }
  __syncthreads();
  // Tinv (N x N) times the columns (N x ncol) on the matrix cores: 16 x 16 output tiles,
  // wavefront w takes tiles w, w + 4, ...; operands read from LDS (zero beyond N and ncol)
  const int RTt = (N + 15) / 16, KS = (N + 3) / 4, CT = (ncol + 15) / 16;
  const int w = threadIdx.x >> 6, ln = threadIdx.x & 63;
  for (int tile = w; tile < RTt * CT; tile += 4) {
    const int rt = tile % RTt, ct = tile / RTt;
    const int ar = 16 * rt + (ln & 15), bc = 16 * ct + (ln & 15);
    acc_t acc;
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = (F)0;
    for (int s = 0; s < KS; ++s) {
      const int k = 4 * s + (ln >> 4);
      const F a = (ar < N && k < N) ? Ts[ar * NP1 + k] : (F)0;
      const F b = (bc < ncol && k < N) ? bs[bc * NP1 + k] : (F)0;
      acc = Mfma<F>::step(a, b, acc);
    }
    const int col = bc;
    if (col >= ncol) continue;
    const int ri = col & 1, kk = (col >> 1) % nk, vv = (col >> 1) / nk;
    const int lm = g.lmbase[kk] + l - kk * g.m0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int jj = 16 * rt + Mfma<F>::out_row(ln, q);
      if (jj >= N) continue;
      const F a = acc[q];
      long long o = (long long)(v0 + vv) * ld + 2LL * ((long long)N * (2LL * g.S + lm) + jj) + ri;
      double xv = (double)(tc[(long long)l * N + jj] * a);
      if (ACC) xv += xvec[o];
      if (FIN) {
        const long long oo = 2LL * ((long long)N * (2LL * g.S + lm) + jj) + ri;
        fo.y[(long long)(v0 + vv) * fo.ldy + oo] = final_value(fo, v0 + vv, oo, (kk == 0 && ri == 1) ? 0.0 : xv);
      } else {
        xvec[o] = xv;
      }
    }
  }
  if (FIN && l == 0) {
    // e, f at (m, l) = (0, 0): lm = 0
    for (int idx = threadIdx.x; idx < nv * 2 * 2 * N; idx += blockDim.x) {
      const int ri = idx & 1, jj = (idx >> 1) % N, f = (idx / (2 * N)) & 1, vv = idx / (4 * N);
      const long long oo = 2LL * ((long long)N * ((long long)f * g.S) + jj) + ri;
      fo.y[(long long)(v0 + vv) * fo.ldy + oo] = final_value(fo, v0 + vv, oo, 0.0);
    }
  }
}

// ------------------------------------------------------------------------------------------
// K9: FP64 residual r = b - A x of the implicit operator, applied through the shared radial
// matrices (D, D^2, D^4) rather than stored blocks.  One thread per (vec, field, lm, j).
__device__ inline double kappa_dev(int l, int m) {
  if (l <= 1 || l <= m) return 0.0;
  double ll = l;
  return (ll * ll - 1.0) * sqrt((ll * ll - (double)m * m) / (4.0 * ll * ll - 1.0));
}

// One workgroup per (tile of up to 6 consecutive l at one m, vector).  The columns
// (Re/Im, t = 0..7) hold l0-1 .. l0+6: the outer two only feed the Coriolis coupling of their
// neighbours.  The products D e, D^2 e, D f, D^2 f, D^4 f, D^2 (f/r^2), D T, D^2 T run on the FP64
// matrix cores (wavefront w owns rows 16w..16w+15); the coupling reads its neighbours'
// products from the adjacent lanes and the other Re/Im component from lane ^ 8.
constexpr int kRLT = 6;  // own l per residual tile

template <int RTN>
__global__ void __launch_bounds__(256) k_residual64(DevGrid g, PhysParams ph, int nvec, const double* __restrict__ bvec,
                                                    const double* __restrict__ xvec, double* __restrict__ rvec) {
  constexpr int rowsN = 16 * RTN;
  __shared__ double xs[4][rowsN][16];   // e, f, q = f/r^2, T; column c*8 + t
  __shared__ double dfb[2][16];         // (D f) at rows 0 and N-1 per column
  const int N = g.N;
  const int2 tl = g.qtiles[blockIdx.x];
  const int vec = blockIdx.y;
  const int k = tl.x, il0 = tl.y;
  const int m = k * g.m0, nl = g.L - m + 1;
  const int nown = min(kRLT, nl - il0);
  const int lmb = g.lmbase[k];
  const long long ld = 6LL * N * g.S;
  const double* x = xvec + (long long)vec * ld;
  staged_copy<9, double>(
      3 * 8 * 2 * rowsN,
      [&](int idx) -> double {
        const int cj = idx % (2 * rowsN), t = (idx / (2 * rowsN)) % 8, f = idx / (2 * rowsN * 8);
        const int jj = cj >> 1, c = cj & 1;
        const int il = il0 - 1 + t;
        if (jj >= N || il < 0 || il >= nl) return 0.0;
        return x[2LL * ((long long)N * ((long long)f * g.S + lmb + il) + jj) + c];
      },
      [&](int idx, double val) {
        const int cj = idx % (2 * rowsN), t = (idx / (2 * rowsN)) % 8, f = idx / (2 * rowsN * 8);
        const int jj = cj >> 1, c = cj & 1;
        const int fs = (f == 2) ? 3 : f;
        xs[fs][jj][c * 8 + t] = val;
        if (f == 1) {
          const double r = (jj < N) ? g.r[jj] : 1.0;
          xs[2][jj][c * 8 + t] = val / (r * r);
        }
      });
  __syncthreads();
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int col = l & 15, c = col >> 3, t = col & 7;
  // products: 0 De, 1 D2e, 2 Df, 3 D2f, 4 D4f, 5 D2q, 6 DT, 7 D2T
  f64x4 y[8];
#pragma unroll
  for (int p = 0; p < 8; ++p) y[p] = f64x4{0, 0, 0, 0};
  if (w < RTN) {
    const double* A0 = g.DF + (long long)w * 4 * RTN * 64 + l;
    const double* A1 = g.D2F + (long long)w * 4 * RTN * 64 + l;
    const double* A2 = g.D4F + (long long)w * 4 * RTN * 64 + l;
#pragma unroll
    for (int st = 0; st < 4 * RTN; ++st) {
      const double d1 = A0[st * 64], d2 = A1[st * 64], d4 = A2[st * 64];
      const int row = 4 * st + (l >> 4);
      const double xe = xs[0][row][col], xf = xs[1][row][col], xq = xs[2][row][col], xt = xs[3][row][col];
      y[0] = Mfma<double>::step(d1, xe, y[0]);
      y[1] = Mfma<double>::step(d2, xe, y[1]);
      y[2] = Mfma<double>::step(d1, xf, y[2]);
      y[3] = Mfma<double>::step(d2, xf, y[3]);
      y[4] = Mfma<double>::step(d4, xf, y[4]);
      y[5] = Mfma<double>::step(d2, xq, y[5]);
      y[6] = Mfma<double>::step(d1, xt, y[6]);
      y[7] = Mfma<double>::step(d2, xt, y[7]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int jj = 16 * w + Mfma<double>::out_row(l, q);
      if (jj == 0) dfb[0][col] = y[2][q];
      if (jj == N - 1) dfb[1][col] = y[2][q];
    }
  }
  __syncthreads();
  if (w >= RTN) return;
  const int il = il0 - 1 + t, lw = m + il;
  const bool own = (t >= 1 && t <= nown);
  const bool has_lo = (lw - 1 >= max(m, 1)), has_hi = (lw + 1 <= g.L);
  const double lam = (double)lw * (lw + 1);
  const double sg = (c == 0) ? -1.0 : 1.0;
  const double* b = bvec + (long long)vec * ld;
  double* rr = rvec + (long long)vec * ld;
  const double kap_lo = ph.cor * kappa_dev(lw, m), kap_hi = ph.cor * kappa_dev(lw + 1, m);
  const double cm = ph.cor * 2.0 * m;   // 2 m of the diagonal Coriolis term (0 when explicit)
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    // values from other lanes first (every lane takes part)
    const double De_lo = __shfl(y[0][q], l - 1), De_hi = __shfl(y[0][q], l + 1);
    const double Df_lo = __shfl(y[2][q], l - 1), Df_hi = __shfl(y[2][q], l + 1);
    const double D2f_o = __shfl_xor(y[3][q], 8);
    const int jj = 16 * w + Mfma<double>::out_row(l, q);
    if (!own || jj >= N) continue;
    const double r = g.r[jj], r2 = r * r;
    const double a = ph.Ek * lam / r2;
    const int co = col ^ 8;
    for (int f = 0; f < 3; ++f) {
      const long long o = 2LL * ((long long)N * ((long long)f * g.S + lmb + il) + jj) + c;
      if (f < 2 && lw == 0) {
        rr[o] = 0.0;
        continue;
      }
      double av;
      if (f == 2) {
        const double xt = xs[3][jj][col];
        if (jj == 0 || jj == N - 1) av = xt;
        else av = xt - ph.dt * (y[7][q] + 2.0 / r * y[6][q] - lam / r2 * xt) / ph.Pr;
      } else {
        const double xv = xs[f][jj][col], xo = xs[f][jj][co];
        const bool bc = (f == 0) ? (jj == 0 || jj == N - 1) : (jj == 0 || jj == 1 || jj == N - 2 || jj == N - 1);
        if (bc) {
          if (jj == 0 || jj == N - 1) av = xv;
          else av = dfb[jj == 1 ? 0 : 1][col];
        } else {
          double cv;
          if (f == 0) {
            const double L_ = y[1][q] - lam / r2 * xv;
            cv = a * xv - ph.dt * (a * L_ + sg * cm / r2 * xo);
          } else {
            const double L_ = y[3][q] - lam / r2 * xv, Lo = D2f_o - lam / r2 * xo;
            const double L2 = y[4][q] - lam * y[5][q] - lam / r2 * y[3][q] + lam * lam / (r2 * r2) * xv;
            cv = -a * L_ + ph.dt * (a * L2 + sg * cm / r2 * Lo);
          }
          // Coriolis coupling to the other potential at l-1 and l+1
          const int fo = 1 - f;
          if (has_lo && kap_lo != 0.0) {
            const double xn = xs[fo][jj][col - 1], Dn = (f == 0) ? Df_lo : De_lo;
            cv += ph.dt * 2.0 / r2 * kap_lo * ((double)lw / r * xn - Dn);
          }
          if (has_hi && kap_hi != 0.0) {
            const double xn = xs[fo][jj][col + 1], Dn = (f == 0) ? Df_hi : De_hi;
            cv += ph.dt * 2.0 / r2 * kap_hi * (-(lw + 1.0) / r * xn - Dn);
          }
          av = cv;
        }
      }
      rr[o] = b[o] - av;
    }
  }
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

// Sum over the 64 lanes of a wavefront by a fixed shuffle tree (reproducible results).
__device__ inline double wave_sum_fixed(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// ------------------------------------------------------------------------------------------
// K13: Krylov helpers (FP64).  Partial dot products part[i * nchunk + chunk] of V_i with w over
// fixed chunks (summed on the host in a fixed order, so results are reproducible).
__global__ void __launch_bounds__(256) k_dots_partial(const double* __restrict__ V, long long ldv, int k,
                                                      const double* __restrict__ w, long long n, int nchunk,
                                                      double* __restrict__ part) {
  __shared__ double red[256];
  const int chunk = blockIdx.x, i = blockIdx.y;
  const long long len = (n + nchunk - 1) / nchunk;
  const long long a = (long long)chunk * len, b = min(n, a + len);
  const double* v = V + (long long)i * ldv;
  double s = 0.0;
  for (long long t = a + threadIdx.x; t < b; t += blockDim.x) s += v[t] * w[t];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(long long)i * nchunk + chunk] = red[0];
}

// w = alpha * w - sum_i h_i V_i   (alpha = 1: Gram-Schmidt update; the sum runs over i < k, in
// order).  The vectors go in groups of kCombineGroup, the loads of the next group in flight while
// the current one is summed (a bandwidth-bound stream needs many loads in flight per wave); the
// loop takes groups in pairs with an odd last group after it, and no load sits under a branch
// (the compiler would wait for it at once).  Lanes past n load the last element and store
// nothing.
constexpr int kCombineGroup = 8;
__global__ void __launch_bounds__(256) k_combine(double* __restrict__ w, double alpha, const double* __restrict__ V,
                                                 long long ldv, int k, const double* __restrict__ h, long long n) {
  constexpr int G = kCombineGroup;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x, tc = t < n ? t : n - 1;
  const int ng = k / G;
  double acc = alpha * w[tc];
  double va[G], vb[G];
  auto load = [&](int gi, double (&v)[G]) {
    gi = gi < ng ? gi : ng - 1;
#pragma unroll
    for (int g = 0; g < G; ++g) v[g] = V[(long long)(gi * G + g) * ldv + tc];
  };
  auto use = [&](int gi, const double (&v)[G]) {
#pragma unroll
    for (int g = 0; g < G; ++g) acc -= h[gi * G + g] * v[g];
  };
  if (ng > 0) {
    load(0, va);
    int gi = 0;
    for (; gi + 1 < ng; gi += 2) {
      load(gi + 1, vb);
      use(gi, va);
      load(gi + 2, va);
      use(gi + 1, vb);
    }
    if (gi < ng) use(gi, va);
  }
  for (int i = ng * G; i < k; ++i) acc -= h[i] * V[(long long)i * ldv + tc];
  if (t < n) w[t] = acc;
}

// Arnoldi step with delayed reorthogonalization (classical Gram-Schmidt applied twice, the second
// pass of step j done at step j + 1 together with the first pass of step j + 1: one pass over the
// basis for the dot products and one for the update per step, instead of two each; the method
// of the low-synchronization Gram-Schmidt variants for GMRES, restated here from its algebra).
// At step j the basis vectors V_0..V_{j-1} are final and V_j holds u, orthogonalized once against
// them and normalized once; w = A u.  With s = V^T u, alpha = u.u, p = V^T w, q = u.w (one pass):
//   rho = sqrt(alpha - s.s),  v_j = (u - V s) / rho                  (u orthogonalized again)
//   H[0:j, j-1] += H[j, j-1] s,  H[j, j-1] *= rho                      (column j-1 final)
//   A v_j = (w - [V, v_j] t) / rho with t = H[0:j+1, 0:j] s          (the Arnoldi relation)
//   c = v_j.w = (q - s.p) / rho
//   column j: h_r = (p_r - t_r) / rho (r < j), h_j = (c - t_j) / rho
//   w1 = A v_j - [V, v_j] h = (w - (c/rho) u - V (p - (c/rho) s)) / rho    (one pass)
// then H[j+1, j] = ||w1|| and V_{j+1} = w1 / ||w1||, orthogonalized once (finished at step j + 1).
// k_dcgs_coef (one workgroup): sp = the reduced dot products (s_0..s_{j-1}, alpha, then
// p_0..p_{j-1}, q); finishes column j-1 of Hc and writes coef = (1/rho, c/rho, s_0..s_{j-1},
// g_0..g_{j-1}, c), g = p - (c/rho) s, for the update pass; column j (the product with H) is
// k_hess_col's.  With fin it only finishes column j-1 (sp = s, alpha of V_j against
// V_0..V_{j-1}: the end of a cycle).  The sums are taken in a fixed order; rho = 0 (u in the span
// of V: a breakdown) gives zero coefficients.
__global__ void __launch_bounds__(256) k_dcgs_coef(int j, int ld, const double* __restrict__ sp, int fin,
                                                   double* __restrict__ Hc, double* __restrict__ coef) {
  __shared__ double red[2][256];
  __shared__ double sh[2];
  const int tid = threadIdx.x;
  const double* sv = sp;
  const double* pv = sp + (j + 1);
  double a1 = 0.0, a2 = 0.0;
  for (int i = tid; i < j; i += 256) {
    a1 += sv[i] * sv[i];
    if (!fin) a2 += sv[i] * pv[i];
  }
  red[0][tid] = a1;
  red[1][tid] = a2;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) {
      red[0][tid] += red[0][tid + h];
      red[1][tid] += red[1][tid + h];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double r2 = sv[j] - red[0][0];
    const double rho = r2 > 0.0 ? sqrt(r2) : 0.0;
    sh[0] = rho;
    sh[1] = (!fin && rho > 0.0) ? (pv[j] - red[1][0]) / rho : 0.0;
  }
  __syncthreads();
  const double rho = sh[0], c = sh[1], ir = rho > 0.0 ? 1.0 / rho : 0.0;
  if (j >= 1) {
    double* col = Hc + (long long)(j - 1) * ld;
    const double hj = col[j];
    for (int i = tid; i < j; i += 256) col[i] += hj * sv[i];
    __syncthreads();
    if (tid == 0) col[j] = hj * rho;
  }
  if (fin) return;
  const double cu = c * ir;
  for (int i = tid; i < j; i += 256) {
    coef[2 + i] = sv[i];
    coef[2 + j + i] = pv[i] - cu * sv[i];
  }
  if (tid == 0) {
    coef[0] = ir;
    coef[1] = cu;
    coef[2 + 2 * j] = c;
  }
}

// Column j of the delayed step (after k_dcgs_coef): h_r = (p_r - t_r) / rho for r < j,
// h_j = (c - t_j) / rho, t = H[0:j+1, 0:j] s (H upper Hessenberg: row r from column r - 1 on).
// Workgroup b owns rows 64 b .. 64 b + 63; wave q of it the columns = q (mod 4) of each row, with
// the loads of eight columns issued together; the four partial sums meet in LDS in a fixed order.
__global__ void __launch_bounds__(256) k_hess_col(int j, int ld, const double* __restrict__ sp,
                                                  const double* __restrict__ coef, double* __restrict__ Hc) {
  __shared__ double red[4][64];
  const int tid = threadIdx.x, q = tid >> 6, r = blockIdx.x * 64 + (tid & 63);
  const double* sv = sp;
  const double* pv = sp + (j + 1);
  double t = 0.0;
  if (r <= j) {
    int cl = (r > 0 ? r - 1 : 0);
    cl += (q - cl % 4 + 4) % 4;   // the first column = q (mod 4) from r - 1 on
    for (; cl + 28 < j; cl += 32) {
      double hv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) hv[u] = Hc[r + (long long)(cl + 4 * u) * ld];
#pragma unroll
      for (int u = 0; u < 8; ++u) t += hv[u] * sv[cl + 4 * u];
    }
    for (; cl < j; cl += 4) t += Hc[r + (long long)cl * ld] * sv[cl];
  }
  red[q][tid & 63] = t;
  __syncthreads();
  if (q == 0 && r <= j) {
    const int i = tid & 63;
    const double tt = ((red[0][i] + red[1][i]) + red[2][i]) + red[3][i];
    const double ir = coef[0], c = coef[2 + 2 * j];
    Hc[r + (long long)j * ld] = (r < j ? pv[r] - tt : c - tt) * ir;
  }
}

// The update pass of the delayed step (see k_dcgs_coef), reading V_0..V_{j-1} once for both
// outputs: V_j <- (u - V s) / rho and w <- (w - cu u - V g) / rho, u = V_j, coef = (1/rho, cu, s,
// g); pn[b] = the part of ||w||^2 of workgroup b.  Basis loads in groups of kCombineGroup with the
// next group in flight (as in k_combine).
__global__ void __launch_bounds__(256) k_combine2(double* __restrict__ w, double* __restrict__ V, long long ldv, int j,
                                                  const double* __restrict__ coef, long long n, double* __restrict__ pn) {
  constexpr int G = kCombineGroup;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x, tc = t < n ? t : n - 1;
  const int ng = j / G;
  const double ir = coef[0], cu = coef[1];
  const double* sv = coef + 2;
  const double* gv = coef + 2 + j;
  double* u = V + (long long)j * ldv;
  const double uu = u[tc];
  double av = uu, aw = w[tc] - cu * uu;
  double va[G], vb[G];
  auto load = [&](int gi, double (&v)[G]) {
    gi = gi < ng ? gi : ng - 1;
#pragma unroll
    for (int g = 0; g < G; ++g) v[g] = V[(long long)(gi * G + g) * ldv + tc];
  };
  auto use = [&](int gi, const double (&v)[G]) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
      av -= sv[gi * G + g] * v[g];
      aw -= gv[gi * G + g] * v[g];
    }
  };
  if (ng > 0) {
    load(0, va);
    int gi = 0;
    for (; gi + 1 < ng; gi += 2) {
      load(gi + 1, vb);
      use(gi, va);
      load(gi + 2, va);
      use(gi + 1, vb);
    }
    if (gi < ng) use(gi, va);
  }
  for (int i = ng * G; i < j; ++i) {
    const double v = V[(long long)i * ldv + tc];
    av -= sv[i] * v;
    aw -= gv[i] * v;
  }
  const double w1 = aw * ir;
  if (t < n) {
    u[t] = av * ir;
    w[t] = w1;
  }
  // ||w1||^2 partial of this workgroup (fixed order), for k_scale_norm
  __shared__ double red[4];
  double ss = t < n ? w1 * w1 : 0.0;
  ss = wave_sum_fixed(ss);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ss;
  __syncthreads();
  if (threadIdx.x == 0) pn[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// dst = alpha * src
__global__ void k_scale(double* __restrict__ dst, const double* __restrict__ src, double alpha, long long n) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) dst[t] = alpha * src[t];
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

// Partial sums of squares: parts[b] = sum of x[i]^2 over chunk b = [b chunk, (b + 1) chunk) of
// [0, n), one workgroup per chunk, fixed summation order.
__global__ void __launch_bounds__(256) k_sumsq_parts(long long n, const double* __restrict__ x, long long chunk,
                                                     double* __restrict__ parts) {
  __shared__ double red[256];
  const long long b0 = (long long)blockIdx.x * chunk;
  const long long b1 = b0 + chunk < n ? b0 + chunk : n;
  double s = 0.0;
  for (long long i = b0 + threadIdx.x; i < b1; i += blockDim.x) s += x[i] * x[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) parts[blockIdx.x] = red[0];
}

// out[0] = sqrt(sum of parts[0..nparts)), one workgroup, fixed summation order.
__global__ void __launch_bounds__(256) k_sqrt_sum(int nparts, const double* __restrict__ parts,
                                                  double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) s += parts[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sqrt(red[0]);
}

// ------------------------------------------------------------------------------------------
// Continuation and grid refinement (Sec. 3.5, 4.2).
// out = w0 x0 + w1 x1 + w2 x2 (the quadratic Lagrange prediction; unused terms have weight 0
// and may repeat a valid pointer).
__global__ void k_lincomb3(long long n, double w0, const double* __restrict__ x0, double w1,
                           const double* __restrict__ x1, double w2, const double* __restrict__ x2,
                           double* __restrict__ out) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) out[t] = w0 * x0[t] + w1 * x1[t] + w2 * x2[t];
}

// Index and magnitude of the largest |x| over chunk b of `chunk` elements: one workgroup per
// chunk, ties to the lower index.
__global__ void __launch_bounds__(256) k_absmax_parts(long long n, const double* __restrict__ x, long long chunk,
                                                      double* __restrict__ pval, long long* __restrict__ pidx) {
  __shared__ double sv[256];
  __shared__ long long si[256];
  const long long b0 = (long long)blockIdx.x * chunk;
  const long long b1 = b0 + chunk < n ? b0 + chunk : n;
  double bv = -1.0;
  long long bi = b0;
  for (long long i = b0 + threadIdx.x; i < b1; i += blockDim.x) {
    const double a = fabs(x[i]);
    if (a > bv) {
      bv = a;
      bi = i;
    }
  }
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      const double ov = sv[threadIdx.x + w];
      const long long oi = si[threadIdx.x + w];
      if (ov > sv[threadIdx.x] || (ov == sv[threadIdx.x] && oi < si[threadIdx.x])) {
        sv[threadIdx.x] = ov;
        si[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pval[blockIdx.x] = sv[0];
    pidx[blockIdx.x] = si[0];
  }
}

// Refinement: y (new layout) from x (old layout) with the same m0.  Every (field, l, m) profile
// present in both layouts is carried by the interpolation matrix Ip (N_new x N_old, row-major:
// the old interpolating polynomial evaluated at the new nodes); new degrees and orders are zero.
// One thread per (field, packed lm of the new layout, new node, Re/Im).
struct InterpMap {
  int N_old, N_new, S_old, S_new, L_old, K_old, m0;
  const int* lmbase_old;   // [K_old + 1]
  const int* lm_k_new;     // [S_new]
  const int* lm_l_new;     // [S_new]
  const double* Ip;        // [N_new][N_old]
};

__global__ void k_interp(InterpMap im, const double* __restrict__ x, double* __restrict__ y) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = 3LL * im.S_new * im.N_new * 2;
  if (t >= total) return;
  const int c = (int)(t & 1);
  const long long q = t >> 1;
  const int jn = (int)(q % im.N_new);
  const long long fl = q / im.N_new;
  const int lm = (int)(fl % im.S_new), f = (int)(fl / im.S_new);
  const int k = im.lm_k_new[lm], l = im.lm_l_new[lm];
  double acc = 0.0;
  if (k <= im.K_old && l <= im.L_old) {
    const int lmo = im.lmbase_old[k] + (l - k * im.m0);
    const double* src = x + 2LL * ((long long)im.N_old * ((long long)f * im.S_old + lmo)) + c;
    const double* row = im.Ip + (long long)jn * im.N_old;
    for (int j = 0; j < im.N_old; ++j) acc += row[j] * src[2LL * j];
  }
  y[t] = acc;
}

// Device-side Arnoldi (restarted GMRES without a host round trip per step).
// out[i] = sum over c of part[i * nchunk + c], i < k: one wavefront per i, lane l adds the
// entries c = l, l + 64, ... in order, then a fixed shuffle tree (reproducible results).
__global__ void __launch_bounds__(256) k_dots_reduce(const double* __restrict__ part, int k, int nchunk,
                                                     double* __restrict__ out) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (i >= k) return;
  double s = 0.0;
  for (int c = lane; c < nchunk; c += 64) s += part[(long long)i * nchunk + c];
  s = wave_sum_fixed(s);
  if (lane == 0) out[i] = s;
}

// 1 / ||r|| from its chunk partials (0 if r = 0), one wavefront.
__global__ void k_inv_norm(const double* __restrict__ pn, int nchunk, double* __restrict__ hinv) {
  double ss = 0.0;
  for (int c = threadIdx.x; c < nchunk; c += 64) ss += pn[c];
  ss = wave_sum_fixed(ss);
  if (threadIdx.x == 0) hinv[0] = ss > 0.0 ? 1.0 / sqrt(ss) : 0.0;
}

// V_{j+1} = w / ||w|| with ||w||^2 the sum of the nchunk parts pn (every workgroup sums them in
// the same fixed order, so all use the same norm); workgroup 0 also writes H[j+1, j] = ||w||.
// ||w|| = 0 (a breakdown) gives V_{j+1} = 0.
__global__ void __launch_bounds__(256) k_scale_norm(int j, int ld, const double* __restrict__ pn, int nchunk,
                                                    const double* __restrict__ w, double* __restrict__ vout,
                                                    long long n, double* __restrict__ Hc) {
  __shared__ double sh;
  if (threadIdx.x < 64) {
    double ss = 0.0;
    for (int c = threadIdx.x; c < nchunk; c += 64) ss += pn[c];
    ss = wave_sum_fixed(ss);
    if (threadIdx.x == 0) {
      const double hn = sqrt(ss);
      sh = hn > 0.0 ? 1.0 / hn : 0.0;
      if (blockIdx.x == 0) Hc[(j + 1) + (long long)j * ld] = hn;
    }
  }
  __syncthreads();
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) vout[t] = sh * w[t];
}

// Dot products of x_r (r < NX right vectors) with V_i, i < k: workgroup (b, c) owns the elements
// [b len, (b + 1) len) (len = 256 kDotsPerThread; thread t the pairs 2 (t + 256 q),
// q < kDotsPerThread / 2, read as 16-byte loads; n is even) and the vectors i = 8 c .. 8 c + 7,
// all of whose loads are issued together; part[(r k + i) * nchunk + b] is the partial sum of
// <V_i, x_r> (summed in a fixed order by k_dots_reduce).  Pairs past n read the last pair
// (clamped, no load under a branch) and are masked at use.
constexpr int kDotsPerThread = 8;
constexpr int kDotsGroup = 8;
template <int NX>
__device__ __forceinline__ void dots_multi_dev(const double* __restrict__ V, long long ldv, int k,
                                               const double* __restrict__ x0, const double* __restrict__ x1,
                                               long long n, int nchunk, double* __restrict__ part) {
  constexpr int NP = kDotsPerThread / 2;
  __shared__ double red[4][NX][kDotsGroup];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const long long base = (long long)blockIdx.x * (256 * kDotsPerThread);
  const int i0 = blockIdx.y * kDotsGroup;
  double2 xr[NX][NP];
  double msk[NP];
  long long idx[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    const long long e = base + 2 * (tid + 256LL * q);
    idx[q] = e < n ? e : n - 2;
    msk[q] = e < n ? 1.0 : 0.0;
    xr[0][q] = *reinterpret_cast<const double2*>(x0 + idx[q]);
    if (NX > 1) xr[NX - 1][q] = *reinterpret_cast<const double2*>(x1 + idx[q]);
  }
  double2 vv[kDotsGroup][NP];
#pragma unroll
  for (int g = 0; g < kDotsGroup; ++g) {
    const int i = min(i0 + g, k - 1);   // rows beyond k repeat the last one and are not stored
    const double* v = V + (long long)i * ldv;
#pragma unroll
    for (int q = 0; q < NP; ++q) vv[g][q] = *reinterpret_cast<const double2*>(v + idx[q]);
  }
  double s[NX][kDotsGroup];
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int g = 0; g < kDotsGroup; ++g) {
      double a = 0.0;
#pragma unroll
      for (int q = 0; q < NP; ++q) a += msk[q] * (vv[g][q].x * xr[r][q].x + vv[g][q].y * xr[r][q].y);
      s[r][g] = a;
    }
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int g = 0; g < kDotsGroup; ++g) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) s[r][g] += __shfl_xor(s[r][g], off);
    }
  if (lane == 0) {
#pragma unroll
    for (int r = 0; r < NX; ++r)
#pragma unroll
      for (int g = 0; g < kDotsGroup; ++g) red[wave][r][g] = s[r][g];
  }
  __syncthreads();
  if (tid < NX * kDotsGroup) {
    const int r = tid / kDotsGroup, g = tid % kDotsGroup;
    if (i0 + g < k)
      part[((long long)r * k + i0 + g) * nchunk + blockIdx.x] =
          ((red[0][r][g] + red[1][r][g]) + red[2][r][g]) + red[3][r][g];
  }
}

// One right vector (norms, Gram-Schmidt dot products) and two (the delayed reorthogonalization).
__global__ void __launch_bounds__(256) k_dots_multi(const double* __restrict__ V, long long ldv, int k,
                                                    const double* __restrict__ w, long long n, int nchunk,
                                                    double* __restrict__ part) {
  dots_multi_dev<1>(V, ldv, k, w, w, n, nchunk, part);
}
__global__ void __launch_bounds__(256) k_dots_multi2(const double* __restrict__ V, long long ldv, int k,
                                                     const double* __restrict__ x0, const double* __restrict__ x1,
                                                     long long n, int nchunk, double* __restrict__ part) {
  dots_multi_dev<2>(V, ldv, k, x0, x1, n, nchunk, part);
}

// x[0] = v (a device scalar written in stream order)
__global__ void k_set1(double* __restrict__ x, double v) {
  if (blockIdx.x == 0 && threadIdx.x == 0) x[0] = v;
}

// dst = alpha[0] * src (alpha read from device memory)
__global__ void k_scale_dev(double* __restrict__ dst, const double* __restrict__ src, const double* __restrict__ alpha,
                            long long n) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) dst[t] = alpha[0] * src[t];
}

}  // namespace sc
