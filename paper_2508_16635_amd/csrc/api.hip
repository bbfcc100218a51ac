// C-ABI of libshellconv: plan creation, factorization, IMEX step, Newton residual and the
// batched Jacobian action on one GPU.  See include/shellconv.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "../../include/shellconv.h"
#include "kernels.h"
#include "plan.h"

namespace {

thread_local std::string g_last_error;

struct Fail {
  int code;
  std::string msg;
};

#define HIPCHK(expr)                                                                      \
  do {                                                                                    \
    hipError_t _e = (expr);                                                               \
    if (_e != hipSuccess)                                                                 \
      throw Fail{_e == hipErrorOutOfMemory ? SC_ERR_NOMEM : SC_ERR_HIP,                   \
                 std::string(#expr) + ": " + hipGetErrorString(_e)};                      \
  } while (0)

// Device allocation that frees itself.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  void alloc(size_t n) {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = n;
    if (n) HIPCHK(hipMalloc(&p, n));
  }
  template <class T>
  T* as() const {
    return reinterpret_cast<T*>(p);
  }
};

template <class T>
void upload(DevBuf& b, const std::vector<T>& h) {
  b.alloc(h.size() * sizeof(T));
  if (!h.empty()) HIPCHK(hipMemcpy(b.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
}

// Rows of (problem, tile within the problem) for every workgroup of a grouped launch, one row per
// vector count nv = 1..vcap (row nv starts at off[nv]), so that a workgroup finds its problem
// with one load instead of walking the problem list.  Left empty (off all -1) beyond 4M entries.
template <class Prob, class TilesOf>
void build_tile_lut(const std::vector<Prob>& probs, int vcap, TilesOf tiles_of, DevBuf& buf,
                    std::vector<long long>& off) {
  off.assign(vcap + 1, -1);
  long long total = 0;
  for (int nv = 1; nv <= vcap; ++nv)
    for (const Prob& q : probs) total += tiles_of(q, nv);
  if (total > (4LL << 20)) return;
  std::vector<int2> h;
  h.reserve((size_t)total);
  for (int nv = 1; nv <= vcap; ++nv) {
    off[nv] = (long long)h.size();
    for (int p = 0; p < (int)probs.size(); ++p) {
      const int nt = tiles_of(probs[p], nv);
      for (int t = 0; t < nt; ++t) {
        int2 e;
        e.x = p;
        e.y = t;
        h.push_back(e);
      }
    }
  }
  upload(buf, h);
}

// Workspace offsets (elements) of one precision.
struct WsLayout {
  long long Gs, Gv, Cs, Cv, Fs, Fv, As, Av, total;
};

struct TabLayout {
  std::vector<long long> synS, synV, anaS, anaV, anfS, anfV;
  long long fw, total;
};

}  // namespace

struct sc_plan {
  sc_params prm{};
  sc::HostGrid hg;
  int vcap = 16, wcap = 16;
  int refine64 = 1, refine32 = 1;
  bool mixed_fp32_solve = false;  // SC_MIXED_SOLVE_FP32
  bool ring_reg32 = true, ring_reg64 = false;  // register-transform ring kernel where N_phi has one
  int ring_rtl32 = -1, ring_rtl64 = -1;         // LDS ring kernel: log2 rings per workgroup (-1: the LDS limit)
  int ring_rv32 = 0, ring_rv64 = 0;             // register ring kernel: shape variant (rings per workgroup)
  int fft_nr = 0, fft_r[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  long long n_real = 0;
  bool factored = false, have_base = false;
  unsigned long long gen = 0;  // bumped by every change of factor, base or parameters
  unsigned long long graph_epoch = 0;  // bumped by every change baked into captured graphs
  double baseC = 0.0;
  long long baseJ = -1;
  // grid / radial data
  DevBuf d_lmk, d_lml, d_lmbase, d_r, d_rp, d_E, d_ED, d_ED2, d_P, d_Dp, d_D, d_D2, d_D4;
  DevBuf d_ET, d_EDT, d_ED2T, d_DT, d_D2T, d_D4T, d_rtiles, d_PT, d_DpT, d_ptiles;
  DevBuf d_EF, d_PF, d_D2F, d_DF, d_D4F, d_qtiles, d_cst;
  int nqtiles = 0;
  int nrtiles = 0, nptiles = 0;
  // tables and workspaces per precision
  TabLayout tl;
  WsLayout wl;
  DevBuf tab64, tab32, ws64, ws32;
  DevBuf probs_syn, probs_ana, probs_anf, d_gsoff, d_lmb8;
  std::vector<int> h_lmb8;                 // per m: first tile-padded degree slot of the analysis outputs
  int nprob_syn = 0, nprob_ana = 0, nprob_anf = 0;
  int ana_ct = 0;                          // column tiles of the folded analysis kernel (0: GEMM path)
  int ana_ct_fold = 0;                     // the folded kernel's column tiles where it can run (0: it cannot)
  std::vector<sc::AnaProb> h_anf;
  std::vector<sc::SynProb> h_syn;
  // tile -> (problem, tile within it) of the synthesis and folded-analysis launches, one row per
  // vector count 1..vcap starting at lut_*_off[nvec] (empty when the rows would be too large:
  // the kernels then search the problem list themselves)
  DevBuf lut_syn, lut_anf;
  std::vector<long long> lut_syn_off, lut_anf_off;
  std::vector<sc::GemmProb> h_ana;
  std::vector<long long> h_gsoff;         // per m: operand-order offsets of Gs, Gv
  int rtcS = 0, rtcV = 0;
  // canonical FP64 vectors
  DevBuf bbuf, xbuf, rbuf, dbuf, norms;
  // base state (dC: its drift speed, read by the Jacobian action's right-hand side)
  DevBuf base64, base32, MX, dC;
  // factors
  DevBuf chains, segs, blk_field, blk_lm, blk_next;
  int nchains = 0, nblocks = 0, nsegs = 0;
  DevBuf D64, G64, H64, Phi64, Psi64, Cg64;
  DevBuf D32, G32, H32, Phi32, Psi32, Cg32;
  DevBuf wscan;  // scan work vectors, capacity vcap x nblocks x N complex doubles
  DevBuf Tinv64, tr64, tc64, Tinv32, tr32, tc32;
  // Newton-GMRES workspace (allocated by the first sc_newton call)
  DevBuf kV, kW, kR, kDu, kPart, kH;
  DevBuf kHc, kGiv, kRes;  // device Arnoldi: Hessenberg columns; the two Gram-Schmidt columns and 1/h;
                           // norm partials
  int krylov_cap = 0;
  // stage profiler: pairs of events recorded around launches while enabled
  bool prof_on = false;
  std::vector<hipEvent_t> ev;           // 2 * capacity
  std::vector<int> ev_stage;            // stage of each recorded pair
  int ev_used = 0;

  // side stream (default priority) for the temperature solve, which runs beside the chains
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // HIP graphs of Krylov chunks (graph_capture): captured on `cap`, a stream of the plan, and
  // launched there between two events; cached per launch configuration until graph_epoch moves
  hipStream_t cap = nullptr;
  hipEvent_t ev_gin = nullptr, ev_gout = nullptr;
  std::map<std::vector<long long>, hipGraphExec_t> graphs;
  unsigned long long graphs_epoch = 0;

  void drop_graphs() {
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    graphs.clear();
  }
  ~sc_plan() {
    drop_graphs();
    for (auto e : ev) (void)hipEventDestroy(e);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (ev_gin) (void)hipEventDestroy(ev_gin);
    if (ev_gout) (void)hipEventDestroy(ev_gout);
    if (side) (void)hipStreamDestroy(side);
    if (cap) (void)hipStreamDestroy(cap);
  }

  sc::DevGrid dg() const {
    sc::DevGrid g;
    g.L = hg.L;
    g.m0 = hg.m0;
    g.N = hg.N;
    g.Np = hg.Np;
    g.nth = hg.nth;
    g.nphi = hg.nphi;
    g.fft_nr = fft_nr;
    for (int i = 0; i < 8; ++i) g.fft_r[i] = fft_r[i];
    g.K = hg.K;
    g.S = hg.S;
    g.vcap = vcap;
    g.wcap = wcap;
    g.lm_k = d_lmk.as<int>();
    g.lm_l = d_lml.as<int>();
    g.lmbase = d_lmbase.as<int>();
    g.r = d_r.as<double>();
    g.rp = d_rp.as<double>();
    g.E = d_E.as<double>();
    g.ED = d_ED.as<double>();
    g.ED2 = d_ED2.as<double>();
    g.P = d_P.as<double>();
    g.Dp = d_Dp.as<double>();
    g.D = d_D.as<double>();
    g.D2 = d_D2.as<double>();
    g.D4 = d_D4.as<double>();
    g.ET = d_ET.as<double>();
    g.EF = d_EF.as<double>();
    g.gsoff = d_gsoff.as<long long>();
    g.rtcS = rtcS;
    g.rtcV = rtcV;
    g.PF = d_PF.as<double>();
    g.D2F = d_D2F.as<double>();
    g.DF = d_DF.as<double>();
    g.D4F = d_D4F.as<double>();
    g.qtiles = d_qtiles.as<int2>();
    g.nqtiles = nqtiles;
    g.EDT = d_EDT.as<double>();
    g.ED2T = d_ED2T.as<double>();
    g.DT = d_DT.as<double>();
    g.D2T = d_D2T.as<double>();
    g.D4T = d_D4T.as<double>();
    g.rtiles = d_rtiles.as<int2>();
    g.nrtiles = nrtiles;
    g.PT = d_PT.as<double>();
    g.DpT = d_DpT.as<double>();
    g.ptiles = d_ptiles.as<int2>();
    g.nptiles = nptiles;
    g.ana_tiled = ana_ct > 0 ? 1 : 0;
    g.lmbase8 = d_lmb8.as<int>();
    g.fv_dp_only = g.ana_tiled;   // the folded analysis derives the m P/sin half
    g.cor_explicit = prm.coriolis == SC_CORIOLIS_EXPLICIT ? 1 : 0;
    g.cst = d_cst.as<double>();
    return g;
  }
  sc::PhysParams pp() const {
    sc::PhysParams p;
    p.Ek = prm.Ek;
    p.Ra = prm.Ra;
    p.Pr = prm.Pr;
    p.dt = prm.dt;
    p.ro = hg.ro;
    p.cor = prm.coriolis == SC_CORIOLIS_EXPLICIT ? 0.0 : 1.0;
    return p;
  }
};

namespace {

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

template <class F>
int guarded(F&& f) {
  try {
    f();
    return SC_OK;
  } catch (const Fail& e) {
    return fail(e.code, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(SC_ERR_NOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(SC_ERR_INTERNAL, e.what());
  }
}

inline unsigned nblk(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// Scratch of the allocation-free residual (sc_newton_residual_noalloc): partial sums of squares,
// one per chunk of kNoAllocChunk elements, in a file-scope device array that every GPU the
// library runs on holds until the process ends.  Host code never passes the array's name to a
// kernel: its device address on each device is looked up once, with that device current, when
// the first plan is created there, and kept in g_scratch_dev.
constexpr int kNoAllocParts = 1024;
constexpr long long kNoAllocChunk = 8192;
static __device__ __align__(256) double scratch[kNoAllocParts];
std::mutex g_scratch_mu;
std::vector<double*> g_scratch_dev;   // indexed by device ordinal

void resolve_scratch(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_dev.size() <= dev) g_scratch_dev.resize(dev + 1, nullptr);
  if (g_scratch_dev[dev]) return;
  void* p = nullptr;
  HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) throw Fail{SC_ERR_HIP, "hipGetSymbolAddress returned a null address for the scratch array"};
  g_scratch_dev[dev] = static_cast<double*>(p);
}

double* scratch_on(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return dev >= 0 && dev < (int)g_scratch_dev.size() ? g_scratch_dev[dev] : nullptr;
}

// Stage profiler: brackets one launch with events on its stream (no effect when disabled).
struct Prof {
  sc_plan* P;
  int pair = -1;
  hipStream_t s;
  Prof(sc_plan* p, int stage, hipStream_t st) : P(p), s(st) {
    if (!P->prof_on || P->ev_used * 2 >= (int)P->ev.size()) return;
    pair = P->ev_used++;
    P->ev_stage[pair] = stage;
    HIPCHK(hipEventRecord(P->ev[2 * pair], s));
  }
  ~Prof() noexcept(false) {
    if (pair >= 0) HIPCHK(hipEventRecord(P->ev[2 * pair + 1], s));
  }
};

// Stream capture of the work `enqueue(stream)` puts on `cap` (a non-blocking stream of the
// library, never the caller's: the legacy default stream cannot be captured), in relaxed mode
// (other host threads may use HIP meanwhile), instantiated; every return and handle is checked.
template <class F>
hipGraphExec_t capture_graph(hipStream_t cap, F&& enqueue) {
  HIPCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed));
  try {
    enqueue(cap);
  } catch (...) {
    hipGraph_t broken = nullptr;
    (void)hipStreamEndCapture(cap, &broken);
    if (broken) (void)hipGraphDestroy(broken);
    throw;
  }
  hipGraph_t graph = nullptr;
  HIPCHK(hipStreamEndCapture(cap, &graph));
  if (!graph) throw Fail{SC_ERR_HIP, "stream capture returned no graph"};
  hipGraphExec_t exec = nullptr;
  const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) throw Fail{SC_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)};
  if (!exec) throw Fail{SC_ERR_HIP, "hipGraphInstantiate returned no executable graph"};
  return exec;
}

// Runs `exec` on `cap` after the work already on `s`, and makes `s` wait for it.
void launch_graph(hipGraphExec_t exec, hipStream_t cap, hipEvent_t ein, hipEvent_t eout, hipStream_t s) {
  HIPCHK(hipEventRecord(ein, s));
  HIPCHK(hipStreamWaitEvent(cap, ein, 0));
  HIPCHK(hipGraphLaunch(exec, cap));
  HIPCHK(hipEventRecord(eout, cap));
  HIPCHK(hipStreamWaitEvent(s, eout, 0));
}

// The plan's cached graph for `key`, captured by `enqueue` on first use; the cache is dropped
// whenever graph_epoch has moved (factor, parameters, kernel choices, phase slot, workspaces).
template <class F>
hipGraphExec_t plan_graph(sc_plan* P, const std::vector<long long>& key, F&& enqueue) {
  if (P->graphs_epoch != P->graph_epoch) {
    P->drop_graphs();
    P->graphs_epoch = P->graph_epoch;
  }
  auto it = P->graphs.find(key);
  if (it != P->graphs.end()) return it->second;
  hipGraphExec_t ex = capture_graph(P->cap, enqueue);
  P->graphs[key] = ex;
  return ex;
}

void build_tables(sc_plan* P) {
  const sc::HostGrid& g = P->hg;
  TabLayout& t = P->tl;
  const int K1 = g.K + 1, nth = g.nth;
  t.synS.resize(K1);
  t.synV.resize(K1);
  t.anaS.resize(K1);
  t.anaV.resize(K1);
  t.anfS.resize(K1);
  t.anfV.resize(K1);
  // synthesis tables on the northern nodes, in MFMA B-operand order: for the even l - m then
  // the odd ones, [column tile][k-step][lane], lane l of (c, s) holding
  // B[degree 4s + lane/16 of the part][node 16c' + lane%16], zero outside; vector tables have
  // the dP/dtheta column tiles first, then the m P/sin ones (c' = c mod cth)
  const long long cth = (nth / 2 + 15) / 16;
  long long off = 0;
  for (int k = 0; k < K1; ++k) {
    const long long nl = g.nl[k], kse = ((nl + 1) / 2 + 3) / 4, kso = (nl / 2 + 3) / 4;
    t.synS[k] = off; off += cth * (kse + kso) * 64;
    t.synV[k] = off; off += 2 * cth * (kse + kso) * 64;
    t.anaS[k] = off; off += nth * nl;
    t.anaV[k] = off; off += 2LL * nth * nl;
    // folded analysis tables in MFMA B-operand order: [part][parity][column tile][k-step][lane],
    // lane l of (c, s) holding table[degree 2 (16c + l%16) + parity][northern node 4s + l/16]
    const long long ksa = (nth / 2 + 3) / 4, cte = ((nl + 1) / 2 + 15) / 16, cto = (nl / 2 + 15) / 16;
    t.anfS[k] = off; off += (cte + cto) * ksa * 64;
    t.anfV[k] = off; off += 2 * (cte + cto) * ksa * 64;
  }
  t.fw = off; off += 2LL * g.nphi;
  t.total = off;
  std::vector<double> h(off, 0.0);
  for (int k = 0; k < K1; ++k) {
    int m = g.ms[k], nl = g.nl[k];
    double dm = (m == 0) ? 1.0 : 2.0;
    for (int il = 0; il < nl; ++il) {
      int l = m + il;
      double lam = (double)l * (l + 1);
      for (int j = 0; j < nth; ++j) {
        double Pb = g.Pb[k][(size_t)il * nth + j], dP = g.dPb[k][(size_t)il * nth + j],
               mP = g.mPs[k][(size_t)il * nth + j];
        if (j < nth / 2) {
          const long long kse = ((nl + 1) / 2 + 3) / 4, kso = (nl / 2 + 3) / 4;
          const bool odd = il & 1;
          const long long kp = odd ? kso : kse, ie = il >> 1;
          const long long kpos = (ie >> 2) * 64 + (ie & 3) * 16 + (j & 15);
          // scalar: cth tiles; vector: 2 cth tiles (dP first)
          const long long sS = t.synS[k] + (odd ? cth * kse * 64 : 0);
          const long long sV = t.synV[k] + (odd ? 2 * cth * kse * 64 : 0);
          h[sS + (long long)(j >> 4) * kp * 64 + kpos] = Pb;
          h[sV + (long long)(j >> 4) * kp * 64 + kpos] = dP;
          h[sV + (long long)(cth + (j >> 4)) * kp * 64 + kpos] = mP;
        }
        double w = g.wt[j];
        h[t.anaS[k] + (long long)il * nth + j] = w * Pb / (2.0 * dm);
        double wv = (l > 0) ? w / (2.0 * dm * lam) : 0.0;
        h[t.anaV[k] + (long long)il * 2 * nth + j] = wv * dP;
        h[t.anaV[k] + (long long)il * 2 * nth + nth + j] = wv * mP;
        if (j < nth / 2) {
          const long long ksa = (nth / 2 + 3) / 4, cte = ((nl + 1) / 2 + 15) / 16, cto = (nl / 2 + 15) / 16;
          const int par = il & 1, ie = il >> 1;
          const long long blk = (par ? cte : 0) + ie / 16;          // column tile within the part
          const long long pos = (blk * ksa + j / 4) * 64 + (j % 4) * 16 + ie % 16;
          h[t.anfS[k] + pos] = w * Pb / (2.0 * dm);
          h[t.anfV[k] + pos] = wv * dP;
          h[t.anfV[k] + (cte + cto) * ksa * 64 + pos] = wv * mP;
        }
      }
    }
  }
  const double twopi = 6.283185307179586476925286766559;
  for (int q = 0; q < g.nphi; ++q) {  // FFT twiddles exp(-2 pi i q / nphi)
    h[t.fw + 2LL * q] = std::cos(twopi * (double)q / g.nphi);
    h[t.fw + 2LL * q + 1] = -std::sin(twopi * (double)q / g.nphi);
  }
  upload(P->tab64, h);
  std::vector<float> hf(h.begin(), h.end());
  upload(P->tab32, hf);
}

void build_workspaces(sc_plan* P) {
  const sc::HostGrid& g = P->hg;
  WsLayout& w = P->wl;
  const long long V = P->vcap, Np = g.Np, S = g.S, K1 = g.K + 1, nth = g.nth;
  long long off = 0;
  // synthesis inputs in MFMA A-operand order per m: [row tile][k-step][lane]
  P->rtcS = (int)((6 * Np * V + 15) / 16);
  P->rtcV = sc::syn_vec_tiles((long long)sc::syn_vec_groups((int)Np) * V);
  P->h_gsoff.assign(2 * K1, 0);
  long long gsz = 0, gvz = 0;
  for (int k = 0; k < K1; ++k) {
    const long long ks = ((g.nl[k] + 1) / 2 + 3) / 4 + (g.nl[k] / 2 + 3) / 4;
    P->h_gsoff[2 * k] = gsz;
    P->h_gsoff[2 * k + 1] = gvz;
    gsz += (long long)P->rtcS * ks * 64;
    gvz += (long long)P->rtcV * ks * 64;
  }
  w.Gs = off; off += gsz;   // h_gsoff: relative to Gs and Gv
  w.Gv = off; off += gvz;
  w.Cs = off; off += K1 * 6 * Np * V * nth;
  w.Cv = off; off += K1 * 12 * Np * V * nth;
  w.Fs = off; off += K1 * 4 * Np * V * nth;
  w.Fv = off; off += K1 * 4 * Np * V * 2 * nth;
  // analysis outputs sized for both layouts: natural (S degrees) and tiled (degrees of every m
  // padded to a multiple of 8)
  P->h_lmb8.assign(K1, 0);
  long long S8 = 0;
  for (int k = 0; k < K1; ++k) {
    P->h_lmb8[k] = (int)S8;
    S8 += (g.nl[k] + 7) / 8 * 8;
  }
  upload(P->d_lmb8, P->h_lmb8);
  w.As = off; off += 4 * Np * V * std::max(S, S8);
  w.Av = off; off += 4 * Np * V * std::max(S, S8);
  w.total = off;
  P->ws64.alloc(off * sizeof(double));
  P->ws32.alloc(off * sizeof(float));
  // the operand-order padding (k beyond n_l) is never written and must read as zero
  HIPCHK(hipMemset(P->ws64.p, 0, off * sizeof(double)));
  HIPCHK(hipMemset(P->ws32.p, 0, off * sizeof(float)));
  upload(P->d_gsoff, P->h_gsoff);
  // contraction problems (offsets are in elements, so they serve both precisions)
  P->h_syn.clear();
  P->h_ana.clear();
  const TabLayout& t = P->tl;
  for (int k = 0; k < K1; ++k) {
    int nl = g.nl[k];
    long long lb = g.lmbase[k];
    const int kse = ((nl + 1) / 2 + 3) / 4, kso = (nl / 2 + 3) / 4, cth = (int)((nth / 2 + 15) / 16);
    P->h_syn.push_back(sc::SynProb{w.Gs + P->h_gsoff[2 * k], t.synS[k], w.Cs + k * 6 * Np * V * nth, (int)(6 * Np), kse,
                                   kso, cth, 1, (int)nth, (int)Np});
    P->h_syn.push_back(sc::SynProb{w.Gv + P->h_gsoff[2 * k + 1], t.synV[k], w.Cv + k * 12 * Np * V * nth,
                                   4 * sc::syn_vec_groups((int)Np), kse, kso, cth, 2, (int)nth, (int)Np});
    sc::GemmProb c{w.Fs + k * 4 * Np * V * nth, t.anaS[k], w.As + 4 * Np * V * lb, (int)(4 * Np), nl, (int)nth, (int)nth, (int)nth, nl};
    sc::GemmProb d{w.Fv + k * 4 * Np * V * 2 * nth, t.anaV[k], w.Av + 4 * Np * V * lb, (int)(4 * Np), nl, (int)(2 * nth), (int)(2 * nth), (int)(2 * nth), nl};
    P->h_ana.push_back(c);
    P->h_ana.push_back(d);
    const int cte = ((nl + 1) / 2 + 15) / 16, cto = (nl / 2 + 15) / 16;
    const long long lb8 = P->h_lmb8[k];
    P->h_anf.push_back(sc::AnaProb{w.Fs + k * 4 * Np * V * nth, t.anfS[k], w.As + 4 * Np * V * lb8, 1, nl, (int)nth, cte, cto,
                                   (int)(4 * Np), (int)(4 * Np * V)});
    P->h_anf.push_back(sc::AnaProb{w.Fv + k * 4 * Np * V * 2 * nth, t.anfV[k], w.Av + 4 * Np * V * lb8, 2, nl, (int)(2 * nth),
                                   cte, cto, (int)(4 * Np), (int)(4 * Np * V)});
  }
  upload(P->probs_syn, P->h_syn);
  upload(P->probs_ana, P->h_ana);
  upload(P->probs_anf, P->h_anf);
  P->nprob_syn = (int)P->h_syn.size();
  P->nprob_ana = (int)P->h_ana.size();
  P->nprob_anf = (int)P->h_anf.size();
  build_tile_lut(P->h_syn, P->vcap, [](const sc::SynProb& q, int nv) { return sc::syn_tiles(q, nv); }, P->lut_syn,
                 P->lut_syn_off);
  build_tile_lut(P->h_anf, P->vcap, [](const sc::AnaProb& q, int nv) { return sc::ana_tiles(q, nv); }, P->lut_anf,
                 P->lut_anf_off);
  {
    // the smallest instantiated column-tile count that covers every m (0: keep the GEMM path)
    int ct = 0;
    for (const auto& a : P->h_anf) ct = std::max(ct, std::max(a.cte, a.cto));
    P->ana_ct = 0;
    for (int c : {1, 2, 3, 5, 8})
      if (ct <= c) {
        P->ana_ct = c;
        break;
      }
  }
  const long long nr = P->n_real;
  P->bbuf.alloc(V * nr * sizeof(double));
  P->xbuf.alloc(V * nr * sizeof(double));
  P->rbuf.alloc(V * nr * sizeof(double));
  P->dbuf.alloc(V * nr * sizeof(double));
  P->norms.alloc(V * sizeof(double));
  long long nbase = 9LL * Np * g.nphi * nth;
  P->base64.alloc(nbase * sizeof(double));
  P->base32.alloc(nbase * sizeof(float));
  P->MX.alloc(nr * sizeof(double));
  P->dC.alloc(sizeof(double));
  HIPCHK(hipMemset(P->dC.p, 0, sizeof(double)));
}

template <class T>
long long gemm_tiles(const std::vector<sc::GemmProb>& pr, int nvec) {
  const int BM = sc::GemmCfg<T>::BM, BN = sc::GemmCfg<T>::BN;
  long long t = 0;
  for (const auto& p : pr) t += (long long)((p.Mper * nvec + BM - 1) / BM) * ((p.N + BN - 1) / BN);
  return t;
}

// ---- pipeline stages ---------------------------------------------------------------------
template <class T>
T* ws_ptr(sc_plan* P);
template <>
double* ws_ptr<double>(sc_plan* P) { return P->ws64.as<double>(); }
template <>
float* ws_ptr<float>(sc_plan* P) { return P->ws32.as<float>(); }
template <class T>
const T* tab_ptr(sc_plan* P);
template <>
const double* tab_ptr<double>(sc_plan* P) { return P->tab64.as<double>(); }
template <>
const float* tab_ptr<float>(sc_plan* P) { return P->tab32.as<float>(); }

// Rings per k_ring workgroup: the largest power of two up to 16 whose 5 spectra fit the
// register staging bound of the in-place FFT passes (-1 if even one ring does not).
template <class T>
int ring_rt_log2(const sc::HostGrid& g) {
  int lg = 4;
  while (lg >= 0 && 5LL * g.nphi * (1LL << lg) > sc::ring_cap<T>()) --lg;
  return lg;
}

// Whether the register-transform ring kernel serves this grid: N_phi = N1 N2 with an
// instantiation below, N_phi >= 3K + 1 (its loops over harmonics have the compile-time bound
// (N_phi - 1)/3 + 1, and the LDS copy of the sums, 18 (K+1) values per ring, fits the field
// buffer of 10 (N_phi + 1)), and its buffer loads and stores reach every sum, base field and
// output with 32-bit byte offsets (each range below 2^31 bytes in FP64).
static bool ring_reg_available(const sc::DevGrid& d) {
  const int nphi = d.nphi, K = d.K;
  if (3 * K + 1 > nphi) return false;
  const long long lim = 1LL << 31;
  if (18LL * (K + 1) * d.Np * d.vcap * d.nth * 8 >= lim || 9LL * d.N * d.nth * d.Np * 8 >= lim ||
      12LL * (K + 1) * d.Np * d.vcap * d.nth * 8 >= lim)
    return false;
  switch (nphi) {
    case 10: case 15: case 20: case 32: case 40: return true;
    default: return false;
  }
}

// Arguments of a register-transform ring launch.
template <class T>
struct RingRegArgs {
  hipStream_t s;
  sc::DevGrid dg;
  int nvec;
  const T *Cs, *Cv, *base, *fw;
  T Ek;
  T *Fs, *Fv;
  double* b64;
  float* b32;
};

template <class T, int MODE, int N1, int N2, int V>
void launch_ring_reg_v(const RingRegArgs<T>& a) {
  constexpr int RR = sc::ring_reg_rings<T>(V);
  const dim3 grid((unsigned)((long long)a.nvec * a.dg.Np * ((a.dg.nth + RR - 1) / RR)));
  hipLaunchKernelGGL((sc::k_ring_reg<T, MODE, N1, N2, RR>), grid, dim3(sc::ring_reg_threads(RR)), 0, a.s, a.dg,
                     a.nvec, a.Cs, a.Cv, a.base, a.fw, a.Ek, a.Fs, a.Fv, a.b64, a.b32);
}

template <class T, int MODE, int N1, int N2>
void launch_ring_reg_n(int variant, const RingRegArgs<T>& a) {
  if (variant == 1) launch_ring_reg_v<T, MODE, N1, N2, 1>(a);
  else if constexpr (sc::ring_reg_variants<T>() > 2) {
    if (variant == 2) launch_ring_reg_v<T, MODE, N1, N2, 2>(a);
    else launch_ring_reg_v<T, MODE, N1, N2, 0>(a);
  } else {
    launch_ring_reg_v<T, MODE, N1, N2, 0>(a);
  }
}

// Register-transform ring kernel (shape `variant`, see ring_reg_rings) for N_phi = N1 N2, if this
// N_phi has one and N_phi >= 3K + 1.  Returns false if not.
template <class T, int MODE>
bool launch_ring_reg(int nphi, int variant, const RingRegArgs<T>& a) {
  if (!ring_reg_available(a.dg)) return false;
  switch (nphi) {
    case 10: launch_ring_reg_n<T, MODE, 2, 5>(variant, a); return true;
    case 15: launch_ring_reg_n<T, MODE, 3, 5>(variant, a); return true;
    case 20: launch_ring_reg_n<T, MODE, 4, 5>(variant, a); return true;
    case 32: launch_ring_reg_n<T, MODE, 8, 4>(variant, a); return true;
    case 40: launch_ring_reg_n<T, MODE, 8, 5>(variant, a); return true;
    default: return false;
  }
}

// Spectral state -> analysed forces (As, Av) in precision T.  mode: linear/nonlinear/synth.
template <class T>
void transforms(sc_plan* P, int mode, int nvec, const double* v, long long ldv, long long J, hipStream_t s) {
  const sc::HostGrid& g = P->hg;
  sc::DevGrid dg = P->dg();
  T* ws = ws_ptr<T>(P);
  const T* tab = tab_ptr<T>(P);
  const WsLayout& w = P->wl;
  {
    Prof _p(P, SC_STAGE_RADIAL_PREP, s);
    const dim3 grid(P->nrtiles, nvec);
    switch ((g.N + 15) / 16) {
      case 1: hipLaunchKernelGGL((sc::k_radial_prep<T, 1>), grid, dim3(256), 0, s, dg, v, ldv, J, nvec, ws + w.Gs, ws + w.Gv); break;
      case 2: hipLaunchKernelGGL((sc::k_radial_prep<T, 2>), grid, dim3(256), 0, s, dg, v, ldv, J, nvec, ws + w.Gs, ws + w.Gv); break;
      case 3: hipLaunchKernelGGL((sc::k_radial_prep<T, 3>), grid, dim3(256), 0, s, dg, v, ldv, J, nvec, ws + w.Gs, ws + w.Gv); break;
      default: hipLaunchKernelGGL((sc::k_radial_prep<T, 4>), grid, dim3(256), 0, s, dg, v, ldv, J, nvec, ws + w.Gs, ws + w.Gv); break;
    }
  }
  HIPCHK(hipGetLastError());
  long long nt = 0;
  for (const auto& pr : P->h_syn) nt += sc::syn_tiles(pr, nvec);
  {
    Prof _p(P, SC_STAGE_LEGENDRE_SYNTH, s);
    const int2* lut = P->lut_syn_off[nvec] >= 0 ? P->lut_syn.as<int2>() + P->lut_syn_off[nvec] : nullptr;
    hipLaunchKernelGGL(sc::k_synth<T>, dim3((unsigned)nt), dim3(256), 0, s, P->probs_syn.as<sc::SynProb>(),
                       P->nprob_syn, lut, nvec, (const T*)ws, tab, ws);
  }
  HIPCHK(hipGetLastError());
  const int rtl_set = std::is_same<T, float>::value ? P->ring_rtl32 : P->ring_rtl64;
  const int rtl = rtl_set >= 0 ? std::min(rtl_set, ring_rt_log2<T>(g)) : ring_rt_log2<T>(g);
  const int ntile = (g.nth + (1 << rtl) - 1) >> rtl;
  dim3 grid((unsigned)((long long)nvec * g.Np * ntile));
  size_t smem = sc::ring_lds_bytes<T>(g.nphi, rtl);
  const T* base = std::is_same<T, double>::value ? (const T*)P->base64.p : (const T*)P->base32.p;
  const T* fw = tab + P->tl.fw;
  T Ek = (T)P->prm.Ek;
  const bool use_reg = std::is_same<T, float>::value ? P->ring_reg32 : P->ring_reg64;
  const int rvar = std::is_same<T, float>::value ? P->ring_rv32 : P->ring_rv64;
  {
    Prof _p(P, SC_STAGE_RING, s);
    bool done = false;
    if (use_reg) {
      RingRegArgs<T> a = {s, dg, nvec, ws + w.Cs, ws + w.Cv, base, fw, Ek, ws + w.Fs, ws + w.Fv, nullptr, nullptr};
      if (mode == sc::RING_LINEAR) {
        done = launch_ring_reg<T, sc::RING_LINEAR>(g.nphi, rvar, a);
      } else if (mode == sc::RING_NONLINEAR) {
        done = launch_ring_reg<T, sc::RING_NONLINEAR>(g.nphi, rvar, a);
      } else {
        a.b64 = P->base64.as<double>();
        a.b32 = P->base32.as<float>();
        done = launch_ring_reg<T, sc::RING_SYNTH>(g.nphi, rvar, a);
      }
    }
    if (done) {
    } else if (mode == sc::RING_LINEAR)
      hipLaunchKernelGGL((sc::k_ring<T, sc::RING_LINEAR>), grid, dim3(256), smem, s, dg, nvec, rtl, ws + w.Cs, ws + w.Cv,
                         base, fw, Ek, ws + w.Fs, ws + w.Fv, (double*)nullptr, (float*)nullptr);
    else if (mode == sc::RING_NONLINEAR)
      hipLaunchKernelGGL((sc::k_ring<T, sc::RING_NONLINEAR>), grid, dim3(256), smem, s, dg, nvec, rtl, ws + w.Cs,
                         ws + w.Cv, base, fw, Ek, ws + w.Fs, ws + w.Fv, (double*)nullptr, (float*)nullptr);
    else
      hipLaunchKernelGGL((sc::k_ring<T, sc::RING_SYNTH>), grid, dim3(256), smem, s, dg, nvec, rtl, ws + w.Cs, ws + w.Cv,
                         base, fw, Ek, ws + w.Fs, ws + w.Fv, P->base64.as<double>(), P->base32.as<float>());
  }
  if (mode == sc::RING_SYNTH) {
    HIPCHK(hipGetLastError());
    return;
  }
  HIPCHK(hipGetLastError());
  if (P->ana_ct > 0) {
    long long na = 0;
    for (const auto& a : P->h_anf) na += sc::ana_tiles(a, nvec);
    const size_t lds = sc::ana_lds_bytes<T>(g.nth, g.L + 1);
    const int2* lut = P->lut_anf_off[nvec] >= 0 ? P->lut_anf.as<int2>() + P->lut_anf_off[nvec] : nullptr;
    Prof _p(P, SC_STAGE_LEGENDRE_ANAL, s);
#define SC_ANAL(CT)                                                                                              \
  hipLaunchKernelGGL((sc::k_anal<T, CT>), dim3((unsigned)na), dim3(256), lds, s, P->probs_anf.as<sc::AnaProb>(), \
                     P->nprob_anf, lut, nvec, g.nth, (const T*)ws, tab, ws)
    switch (P->ana_ct) {
      case 1: SC_ANAL(1); break;
      case 2: SC_ANAL(2); break;
      case 3: SC_ANAL(3); break;
      case 5: SC_ANAL(5); break;
      default: SC_ANAL(8); break;
    }
#undef SC_ANAL
  } else {
    nt = gemm_tiles<T>(P->h_ana, nvec);
    Prof _p(P, SC_STAGE_LEGENDRE_ANAL, s);
    hipLaunchKernelGGL(sc::k_gemm_batched<T>, dim3((unsigned)nt), dim3(256), 0, s, P->probs_ana.as<sc::GemmProb>(),
                       P->nprob_ana, nvec, (const T*)ws, tab, ws);
  }
  HIPCHK(hipGetLastError());
}

constexpr int kSeg = 10;  // blocks per scan segment
static_assert(kSeg <= sc::kSegMax, "the one-vector local walks hold a segment in LDS");
using sc::kVG;            // vectors per workgroup in the chain solves

// Projection launch for RT = ceil(N/16) output row tiles.
template <class T, bool STEP>
void launch_project(sc_plan* P, int nvec, const T* As, const T* Av, const double* v, long long ldv, long long J, double C,
                    const double* MX, double* b, hipStream_t s) {
  const double* Cd = P->dC.as<const double>();
  const sc::HostGrid& g = P->hg;
  const dim3 grid(P->nptiles, nvec);
  const size_t smem = sc::project_lds_bytes<T>(g.Np, g.N);
  sc::DevGrid dg = P->dg();
  switch ((g.N + 15) / 16) {
    case 1: hipLaunchKernelGGL((sc::k_project_rhs<T, STEP, 1>), grid, dim3(256), smem, s, dg, P->pp(), nvec, As, Av, v, ldv, J, C, Cd, MX, b); break;
    case 2: hipLaunchKernelGGL((sc::k_project_rhs<T, STEP, 2>), grid, dim3(256), smem, s, dg, P->pp(), nvec, As, Av, v, ldv, J, C, Cd, MX, b); break;
    case 3: hipLaunchKernelGGL((sc::k_project_rhs<T, STEP, 3>), grid, dim3(256), smem, s, dg, P->pp(), nvec, As, Av, v, ldv, J, C, Cd, MX, b); break;
    default: hipLaunchKernelGGL((sc::k_project_rhs<T, STEP, 4>), grid, dim3(256), smem, s, dg, P->pp(), nvec, As, Av, v, ldv, J, C, Cd, MX, b); break;
  }
  HIPCHK(hipGetLastError());
}

template <class T, bool STEP, int RT>
void project_attr() {
  HIPCHK(hipFuncSetAttribute((const void*)sc::k_project_rhs<T, STEP, RT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)sc::project_lds_bytes<double>(128, 64)));
}

template <class F>
size_t tsolve_smem(const sc::HostGrid& g) {
  return sizeof(F) * ((size_t)g.N * (g.N + 1) + (size_t)sc::kTV * (g.K + 1) * 2 * (g.N + 1));
}

// The five chain-solve launches for RT = ceil(N/16) row tiles.
template <class F, int RT, bool ACC, bool FIN>
void chain_solve_rt(sc_plan* P, int nvec, const double* b, double* x, const sc::FinalOut& fo, hipStream_t s) {
  sc::DevGrid dg = P->dg();
  const int nvg = (nvec + kVG - 1) / kVG;
  const bool d = std::is_same<F, double>::value;
  typedef sc::cpx<F> C;
  const C* Dm = (const C*)(d ? P->D64.p : P->D32.p);
  const C* Gm = (const C*)(d ? P->G64.p : P->G32.p);
  const C* H = (const C*)(d ? P->H64.p : P->H32.p);
  const C* Phi = (const C*)(d ? P->Phi64.p : P->Phi32.p);
  const C* Psi = (const C*)(d ? P->Psi64.p : P->Psi32.p);
  const F* Cg = (const F*)(d ? P->Cg64.p : P->Cg32.p);
  C* W = (C*)P->wscan.p;
  const sc::ChainMeta* ch = P->chains.as<sc::ChainMeta>();
  const sc::SegMeta* sg = P->segs.as<sc::SegMeta>();
  const dim3 blk(sc::kSolveThreads);
  if (nvec == 1) {
    // one right-hand side: the walks on the vector units with deeper operand prefetch (a
    // 16-column matrix-core step would carry 15 columns of padding)
    const dim3 wblk(sc::walk_threads(RT));
    hipLaunchKernelGGL((sc::k_cs1_fwd_rhs<F, RT>), dim3(P->nsegs), wblk, 0, s, dg, sg, P->blk_field.as<int>(),
                       P->blk_lm.as<int>(), Dm, Gm, b, W);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL((sc::k_cs1_fwd_bound<F, RT>), dim3(P->nchains), wblk, 0, s, dg, ch, kSeg, Phi, W);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL((sc::k_cs1_bwd_fix<F, RT>), dim3(P->nsegs), wblk, 0, s, dg, sg, Phi, H, W);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL((sc::k_cs1_bwd_bound<F, RT>), dim3(P->nchains), wblk, 0, s, dg, ch, kSeg, Psi, W);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL((sc::k_cs1_out<F, RT, ACC, FIN>), dim3(P->nblocks), blk, 0, s, dg, P->blk_field.as<int>(),
                       P->blk_lm.as<int>(), P->blk_next.as<int>(), Psi, Cg, (const C*)W, x, fo);
  } else {
    hipLaunchKernelGGL((sc::k_cs_fwd_rhs<F, RT>), dim3(P->nsegs, nvg), dim3(sc::walk_threads(RT)), 0, s, dg, nvec, sg, P->blk_field.as<int>(),
                       P->blk_lm.as<int>(), Dm, Gm, b, W);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL((sc::k_cs_fwd_bound<F, RT>), dim3(P->nchains, nvg), dim3(sc::walk_threads(RT)), 0, s, dg, nvec, ch, kSeg, Phi, W);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL((sc::k_cs_bwd_fix<F, RT>), dim3(P->nsegs, nvg), dim3(sc::walk_threads(RT)), 0, s, dg, nvec, sg, Phi, H, W);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL((sc::k_cs_bwd_bound<F, RT>), dim3(P->nchains, nvg), dim3(sc::walk_threads(RT)), 0, s, dg, nvec, ch, kSeg, Psi, W);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL((sc::k_cs_out<F, RT, ACC, FIN>), dim3(P->nblocks, nvg), blk, 0, s, dg, nvec,
                       P->blk_field.as<int>(), P->blk_lm.as<int>(), P->blk_next.as<int>(), Psi, Cg, (const C*)W, x,
                       fo);
  }
  HIPCHK(hipGetLastError());
}

// Implicit solve x = A^{-1} b (ACC: x += A^{-1} b) with factors in precision F (all vectors
// in canonical FP64).  With FIN the result is not stored in x: the output kernels write the
// Jacobian action fo.y = clean(x) - u instead.
template <class F, bool ACC, bool FIN>
void implicit_solve(sc_plan* P, int nvec, const double* b, double* x, const sc::FinalOut& fo, hipStream_t s) {
  sc::DevGrid dg = P->dg();
  const bool d = std::is_same<F, double>::value;
  // the temperature blocks are independent of the chains: solve them on the side stream
  HIPCHK(hipEventRecord(P->ev_fork, s));
  HIPCHK(hipStreamWaitEvent(P->side, P->ev_fork, 0));
  {
    const F* Ti = (const F*)(d ? P->Tinv64.p : P->Tinv32.p);
    const F* tr = (const F*)(d ? P->tr64.p : P->tr32.p);
    const F* tc = (const F*)(d ? P->tc64.p : P->tc32.p);
    Prof _p(P, SC_STAGE_T_SOLVE, P->side);
    hipLaunchKernelGGL((sc::k_T_solve<F, ACC, FIN>), dim3(P->hg.L + 1, (nvec + sc::kTV - 1) / sc::kTV), dim3(256),
                       tsolve_smem<F>(P->hg), P->side, dg, nvec, Ti, tr, tc, b, x, fo);
    HIPCHK(hipGetLastError());
  }
  {
    Prof _p(P, SC_STAGE_CHAIN_SOLVE, s);
    switch ((P->hg.N + 15) / 16) {
      case 1: chain_solve_rt<F, 1, ACC, FIN>(P, nvec, b, x, fo, s); break;
      case 2: chain_solve_rt<F, 2, ACC, FIN>(P, nvec, b, x, fo, s); break;
      case 3: chain_solve_rt<F, 3, ACC, FIN>(P, nvec, b, x, fo, s); break;
      default: chain_solve_rt<F, 4, ACC, FIN>(P, nvec, b, x, fo, s); break;
    }
  }
  HIPCHK(hipEventRecord(P->ev_join, P->side));
  HIPCHK(hipStreamWaitEvent(s, P->ev_join, 0));
}

// x = A^{-1} b: a solve with the factors in precision F, then `passes` FP64 refinement passes
// (FP64 residual r = b - A x, FP64 correction solve added to x).  With fo the last solve writes
// the Jacobian action fo->y = clean(x) - u instead of updating x.
template <class F>
void refined_solve(sc_plan* P, int nvec, const double* b, double* x, int passes, const sc::FinalOut* fo,
                   hipStream_t s) {
  const sc::FinalOut none = {nullptr, 0, -1, nullptr, 0};
  if (fo && passes == 0) {
    implicit_solve<F, false, true>(P, nvec, b, x, *fo, s);
    return;
  }
  implicit_solve<F, false, false>(P, nvec, b, x, none, s);
  sc::DevGrid dg = P->dg();
  for (int it = 0; it < passes; ++it) {
    {
      Prof _p(P, SC_STAGE_RESIDUAL, s);
      const dim3 grid(P->nqtiles, nvec);
      double* r = P->rbuf.as<double>();
      switch ((P->hg.N + 15) / 16) {
        case 1: hipLaunchKernelGGL((sc::k_residual64<1>), grid, dim3(256), 0, s, dg, P->pp(), nvec, b, x, r); break;
        case 2: hipLaunchKernelGGL((sc::k_residual64<2>), grid, dim3(256), 0, s, dg, P->pp(), nvec, b, x, r); break;
        case 3: hipLaunchKernelGGL((sc::k_residual64<3>), grid, dim3(256), 0, s, dg, P->pp(), nvec, b, x, r); break;
        default: hipLaunchKernelGGL((sc::k_residual64<4>), grid, dim3(256), 0, s, dg, P->pp(), nvec, b, x, r); break;
      }
    }
    HIPCHK(hipGetLastError());
    if (fo && it == passes - 1) implicit_solve<double, true, true>(P, nvec, P->rbuf.as<double>(), x, *fo, s);
    else implicit_solve<double, true, false>(P, nvec, P->rbuf.as<double>(), x, none, s);
  }
}

// Nonlinear step: P->xbuf <- B_C(x) (uncleaned solve output).
void step_into_xbuf(sc_plan* P, const double* x, double C, hipStream_t s) {
  transforms<double>(P, sc::RING_NONLINEAR, 1, x, P->n_real, -1, s);
  {
    Prof _p(P, SC_STAGE_PROJECT_RHS, s);
    launch_project<double, true>(P, 1, (const double*)(P->ws64.as<double>() + P->wl.As),
                                 (const double*)(P->ws64.as<double>() + P->wl.Av), x, P->n_real, (long long)-1, C,
                                 (const double*)nullptr, P->bbuf.as<double>(), s);
  }
  refined_solve<double>(P, 1, P->bbuf.as<double>(), P->xbuf.as<double>(), P->refine64, nullptr, s);
}

void check_plan(sc_plan* P) {
  if (!P) throw Fail{SC_ERR_ARG, "null plan"};
  HIPCHK(hipSetDevice(P->prm.device));
}


long long check_slot(sc_plan* P, long long J) {
  if (J < 0) return -1;
  const sc::HostGrid& g = P->hg;
  if (J >= P->n_real || (J % 2) == 0) throw Fail{SC_ERR_ARG, "phase slot must be an Im entry"};
  long long node = J / 2;
  int lm = (int)((node / g.N) % g.S);
  if (g.lm_k[lm] == 0) throw Fail{SC_ERR_ARG, "phase slot must have m > 0"};
  return J;
}

void set_base_impl(sc_plan* P, const double* x, double C, long long J, hipStream_t s) {
  const sc::HostGrid& g = P->hg;
  transforms<double>(P, sc::RING_SYNTH, 1, x, P->n_real, -1, s);
  long long n3 = 3LL * g.S * g.N;
  hipLaunchKernelGGL(sc::k_apply_M, dim3(nblk(n3, 256)), dim3(256), 0, s, P->dg(), P->pp(), x, P->MX.as<double>());
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(sc::k_set1, dim3(1), dim3(64), 0, s, P->dC.as<double>(), C);
  HIPCHK(hipGetLastError());
  if (J != P->baseJ) ++P->graph_epoch;   // the phase slot is a launch argument of captured graphs
  P->baseC = C;
  P->baseJ = J;
  P->have_base = true;
  ++P->gen;
}

void jvp_impl(sc_plan* P, int nvec, const double* v, long long ldv, double* y, long long ldy, int prec, hipStream_t s) {
  const long long J = P->baseJ;
  // the last solve writes y = clean(x) - u, u = v with slot J zeroed
  const sc::FinalOut fo = {v, ldv, J, y, ldy};
  if (prec == SC_FP64) {
    transforms<double>(P, sc::RING_LINEAR, nvec, v, ldv, J, s);
    {
      Prof _p(P, SC_STAGE_PROJECT_RHS, s);
      launch_project<double, false>(P, nvec, (const double*)(P->ws64.as<double>() + P->wl.As),
                                    (const double*)(P->ws64.as<double>() + P->wl.Av), v, ldv, J, P->baseC,
                                    P->MX.as<const double>(), P->bbuf.as<double>(), s);
    }
    refined_solve<double>(P, nvec, P->bbuf.as<double>(), P->xbuf.as<double>(), P->refine64, &fo, s);
  } else {
    transforms<float>(P, sc::RING_LINEAR, nvec, v, ldv, J, s);
    {
      Prof _p(P, SC_STAGE_PROJECT_RHS, s);
      launch_project<float, false>(P, nvec, (const float*)(P->ws32.as<float>() + P->wl.As),
                                   (const float*)(P->ws32.as<float>() + P->wl.Av), v, ldv, J, P->baseC,
                                   P->MX.as<const double>(), P->bbuf.as<double>(), s);
    }
    if (P->mixed_fp32_solve)
      refined_solve<float>(P, nvec, P->bbuf.as<double>(), P->xbuf.as<double>(), P->refine32, &fo, s);
    else
      refined_solve<double>(P, nvec, P->bbuf.as<double>(), P->xbuf.as<double>(), 0, &fo, s);
  }
}

// ---- Krylov / Newton (host control, device vectors) ----------------------------------------
constexpr int kDotChunks = 64;

// workgroups of k_dots_multi for vectors of n elements
inline long long dots_chunks(long long n) { return (n + 256LL * sc::kDotsPerThread - 1) / (256LL * sc::kDotsPerThread); }

void ensure_krylov(sc_plan* P, int restart) {
  if (P->krylov_cap >= restart) return;
  const long long n = P->n_real;
  P->kV.alloc((size_t)(restart + 1) * n * sizeof(double));
  P->kW.alloc(n * sizeof(double));
  P->kR.alloc(n * sizeof(double));
  P->kDu.alloc(n * sizeof(double));
  P->kPart.alloc((size_t)2 * (restart + 1) * std::max<long long>(kDotChunks, dots_chunks(n)) * sizeof(double));
  P->kH.alloc((size_t)(restart + 1) * sizeof(double));
  P->kHc.alloc((size_t)(restart + 1) * restart * sizeof(double));
  P->kGiv.alloc((size_t)(5 * (restart + 1) + 4) * sizeof(double));
  P->kRes.alloc((size_t)std::max<long long>(std::max<long long>(kDotChunks, dots_chunks(n)), nblk(n, 256)) *
                sizeof(double));
  P->krylov_cap = restart;
  ++P->graph_epoch;
}

// h[i] = <V_i, w> for i < k (device vectors, fixed-order host summation of fixed chunks)
void dots(sc_plan* P, const double* V, long long ldv, int k, const double* w, std::vector<double>& h, hipStream_t s) {
  const long long n = P->n_real;
  hipLaunchKernelGGL(sc::k_dots_partial, dim3(kDotChunks, k), dim3(256), 0, s, V, ldv, k, w, n, kDotChunks,
                     P->kPart.as<double>());
  HIPCHK(hipGetLastError());
  std::vector<double> part((size_t)k * kDotChunks);
  HIPCHK(hipMemcpyAsync(part.data(), P->kPart.p, part.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  h.assign(k, 0.0);
  for (int i = 0; i < k; ++i)
    for (int c = 0; c < kDotChunks; ++c) h[i] += part[(size_t)i * kDotChunks + c];
}

double norm2(sc_plan* P, const double* w, hipStream_t s) {
  std::vector<double> h;
  dots(P, w, P->n_real, 1, w, h, s);
  return std::sqrt(h[0]);
}

// w = alpha w - sum_{i<k} h_i V_i
void combine(sc_plan* P, double* w, double alpha, const double* V, long long ldv, int k, const std::vector<double>& h,
             hipStream_t s) {
  const long long n = P->n_real;
  if (k > 0) HIPCHK(hipMemcpyAsync(P->kH.p, h.data(), k * sizeof(double), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(sc::k_combine, dim3(nblk(n, 256)), dim3(256), 0, s, w, alpha, V, ldv, k, P->kH.as<const double>(), n);
  HIPCHK(hipGetLastError());
}

// Device Arnoldi workspace views (capacity krylov_cap).
struct ArnoldiWs {
  double *Hc, *h1, *h2, *pn, *hinv, *coef;   // h1, h2 contiguous: the 2 (R + 1) reduced dot products
  int ld;
};
ArnoldiWs arnoldi_ws(sc_plan* P) {
  const int R = P->krylov_cap;
  double* b = P->kGiv.as<double>();
  ArnoldiWs a;
  a.ld = R + 1;
  a.Hc = P->kHc.as<double>();
  a.h1 = b;
  a.h2 = b + (R + 1);
  a.hinv = b + 2 * (R + 1);
  a.coef = b + 2 * (R + 1) + 2;   // 2 + 2 R coefficients of the delayed step
  a.pn = P->kRes.as<double>();   // norm partials (capacity: chunks of n, workgroups of the update)
  return a;
}

constexpr int kArnoldiChunk = 8;   // Arnoldi steps enqueued between two host checks

// ||x||^2 partials of x into pn (one pass, dots_chunks(n) workgroups)
void norm_parts(sc_plan* P, const double* x, double* pn, hipStream_t s) {
  const long long n = P->n_real;
  const int nch = (int)dots_chunks(n);
  hipLaunchKernelGGL(sc::k_dots_multi, dim3(nch, 1), dim3(256), 0, s, x, n, 1, x, n, nch, pn);
}

// One Arnoldi step j on the device, no host synchronization, with the second Gram-Schmidt pass
// delayed to the next step (k_dcgs_coef): w = J u with u = V_j (orthogonalized once); one pass of
// dot products of V_0..V_j with u and w; the coefficients and column j - 1 finished; one update
// pass giving the final V_j, w1 and the parts of ||w1||^2; column j; H[j+1, j] = ||w1|| and
// V_{j+1} = w1 / ||w1|| in one pass.
void arnoldi_step(sc_plan* P, int j, int prec, hipStream_t s) {
  const long long n = P->n_real;
  double* V = P->kV.as<double>();
  double* w = P->kW.as<double>();
  double* part = P->kPart.as<double>();
  const ArnoldiWs a = arnoldi_ws(P);
  double* u = V + (long long)j * n;
  jvp_impl(P, 1, u, n, w, n, prec, s);
  const int nch = (int)dots_chunks(n);
  hipLaunchKernelGGL(sc::k_dots_multi2, dim3(nch, (j + 1 + sc::kDotsGroup - 1) / sc::kDotsGroup), dim3(256), 0, s,
                     (const double*)V, n, j + 1, (const double*)u, (const double*)w, n, nch, part);
  hipLaunchKernelGGL(sc::k_dots_reduce, dim3(nblk(2 * (j + 1), 4)), dim3(256), 0, s, (const double*)part, 2 * (j + 1),
                     nch, a.h1);
  hipLaunchKernelGGL(sc::k_dcgs_coef, dim3(1), dim3(256), 0, s, j, a.ld, (const double*)a.h1, 0, a.Hc, a.coef);
  const int nwg = (int)nblk(n, 256);
  hipLaunchKernelGGL(sc::k_combine2, dim3(nwg), dim3(256), 0, s, w, V, n, j, (const double*)a.coef, n, a.pn);
  hipLaunchKernelGGL(sc::k_hess_col, dim3((j + 1 + 63) / 64), dim3(256), 0, s, j, a.ld, (const double*)a.h1,
                     (const double*)a.coef, a.Hc);
  hipLaunchKernelGGL(sc::k_scale_norm, dim3(nwg), dim3(256), 0, s, j, a.ld, (const double*)a.pn, nwg, (const double*)w,
                     V + (long long)(j + 1) * n, n, a.Hc);
  HIPCHK(hipGetLastError());
}

// Finishes column k - 1 after the last step of a cycle: the dot products of V_k (orthogonalized
// once) with V_0..V_k give the second pass's coefficients (no new Jacobian action).
void arnoldi_finish(sc_plan* P, int k, hipStream_t s) {
  const long long n = P->n_real;
  double* V = P->kV.as<double>();
  double* part = P->kPart.as<double>();
  const ArnoldiWs a = arnoldi_ws(P);
  const int nch = (int)dots_chunks(n);
  hipLaunchKernelGGL(sc::k_dots_multi, dim3(nch, (k + 1 + sc::kDotsGroup - 1) / sc::kDotsGroup), dim3(256), 0, s,
                     (const double*)V, n, k + 1, (const double*)(V + (long long)k * n), n, nch, part);
  hipLaunchKernelGGL(sc::k_dots_reduce, dim3(nblk(k + 1, 4)), dim3(256), 0, s, (const double*)part, k + 1, nch, a.h1);
  hipLaunchKernelGGL(sc::k_dcgs_coef, dim3(1), dim3(256), 0, s, k, a.ld, (const double*)a.h1, 1, a.Hc, a.coef);
  HIPCHK(hipGetLastError());
}

// Restarted GMRES for (B_X - I) du = b with the current base; returns the number of jvps.
// The Arnoldi steps run on the device in chunks of kArnoldiChunk; after each chunk the host reads
// the new Hessenberg columns, applies the Givens rotations and checks the residual estimates, so
// up to kArnoldiChunk - 1 steps beyond convergence may be computed (and counted); the solution
// uses the steps up to the first converged one.
int gmres(sc_plan* P, const double* b, double* du, double rtol, int restart, int maxmv, int prec, hipStream_t s) {
  const long long n = P->n_real;
  double* V = P->kV.as<double>();
  double* w = P->kW.as<double>();
  const ArnoldiWs a = arnoldi_ws(P);
  const int nch = (int)dots_chunks(n);
  const double bn = norm2(P, b, s);
  hipLaunchKernelGGL(sc::k_scale, dim3(nblk(n, 256)), dim3(256), 0, s, du, b, 0.0, n);
  HIPCHK(hipGetLastError());
  if (bn == 0.0) return 0;
  // r = b (x0 = 0) in V_0 before normalization
  hipLaunchKernelGGL(sc::k_scale, dim3(nblk(n, 256)), dim3(256), 0, s, V, b, 1.0, n);
  HIPCHK(hipGetLastError());
  int mv = 0;
  double beta = bn;
  std::vector<double> H((size_t)a.ld * restart), cs(restart), sn(restart), g(restart + 1);
  while (true) {
    if (beta <= rtol * bn || mv >= maxmv) break;
    norm_parts(P, V, a.pn, s);
    hipLaunchKernelGGL(sc::k_inv_norm, dim3(1), dim3(64), 0, s, (const double*)a.pn, nch, a.hinv);
    hipLaunchKernelGGL(sc::k_scale_dev, dim3(nblk(n, 256)), dim3(256), 0, s, V, (const double*)V,
                       (const double*)a.hinv, n);
    HIPCHK(hipGetLastError());
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    // column j - 1 of the Hessenberg matrix is finished by step j (the delayed second
    // Gram-Schmidt pass), so the host takes the columns one step behind the device and the last
    // column of a cycle is finished by arnoldi_finish
    int j = 0, jend = 0, jq = 0;
    bool done = false, cycle = true;   // done: converged, broken down or out of actions
    while (cycle) {
      const int cnt = std::min(std::min(kArnoldiChunk, restart - j), maxmv - mv);
      if (cnt > 0) {
        for (int q = 0; q < cnt; ++q) arnoldi_step(P, j + q, prec, s);
        mv += cnt;
        j += cnt;
      }
      const bool last = cnt <= 0 || j >= restart || mv >= maxmv;
      if (last && j > jq) arnoldi_finish(P, j, s);
      const int jfin = last ? j : j - 1;   // columns [jq, jfin) are final
      if (jfin > jq) {
        HIPCHK(hipMemcpyAsync(H.data() + (size_t)jq * a.ld, a.Hc + (size_t)jq * a.ld,
                              (size_t)(jfin - jq) * a.ld * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int jj = jq; jj < jfin && !done; ++jj) {
          double* col = H.data() + (size_t)jj * a.ld;
          const double hn = col[jj + 1];
          if (!std::isfinite(hn)) throw Fail{SC_ERR_NONFINITE, "GMRES: non-finite Hessenberg entry"};
          for (int i = 0; i < jj; ++i) {
            const double x0 = col[i], x1 = col[i + 1];
            col[i] = cs[i] * x0 + sn[i] * x1;
            col[i + 1] = -sn[i] * x0 + cs[i] * x1;
          }
          const double x0 = col[jj], den = std::hypot(x0, hn);
          cs[jj] = den > 0 ? x0 / den : 1.0;
          sn[jj] = den > 0 ? hn / den : 0.0;
          col[jj] = den;
          col[jj + 1] = 0.0;
          g[jj + 1] = -sn[jj] * g[jj];
          g[jj] = cs[jj] * g[jj];
          if (std::fabs(g[jj + 1]) <= rtol * bn || hn == 0.0) {
            jend = jj + 1;
            done = true;
          }
        }
        jq = jfin;
      }
      if (done) {
        cycle = false;
      } else if (last) {
        jend = j;
        cycle = false;
        if (cnt <= 0 || mv >= maxmv) done = true;
      }
    }
    if (jend == 0) break;
    // y = R^{-1} g from the first jend rotated columns, du -= V y
    std::vector<double> y(jend, 0.0);
    for (int i = jend - 1; i >= 0; --i) {
      double acc = g[i];
      for (int q = i + 1; q < jend; ++q) acc -= H[(size_t)q * a.ld + i] * y[q];
      y[i] = acc / H[(size_t)i * a.ld + i];
    }
    for (auto& v : y) v = -v;
    combine(P, du, 1.0, V, n, jend, y, s);
    if (done || mv >= maxmv) break;
    // restart: r = b - J du, stored in V_0
    jvp_impl(P, 1, du, n, w, n, prec, s);
    ++mv;
    hipLaunchKernelGGL(sc::k_scale, dim3(nblk(n, 256)), dim3(256), 0, s, V, b, 1.0, n);
    HIPCHK(hipGetLastError());
    std::vector<double> one{1.0};
    combine(P, V, 1.0, w, n, 1, one, s);
    beta = norm2(P, V, s);
  }
  return mv;
}

void newton_impl(sc_plan* P, double* x, double* C, const sc_newton_opts& o, long long J, sc_newton_report* rep,
                 hipStream_t s) {
  ensure_krylov(P, o.restart);
  const long long n = P->n_real;
  std::memset(rep, 0, sizeof(*rep));
  double* R = P->kR.as<double>();
  double* du = P->kDu.as<double>();
  for (int it = 0;; ++it) {
    step_into_xbuf(P, x, *C, s);
    hipLaunchKernelGGL(sc::k_finalize, dim3(nblk(n, 256)), dim3(256), 0, s, P->dg(), 1, P->xbuf.as<const double>(), x, n,
                       (long long)-1, R, n, 1);
    HIPCHK(hipGetLastError());
    if (o.forcing) {
      hipLaunchKernelGGL(sc::k_axpy1, dim3(nblk(n, 256)), dim3(256), 0, s, n, o.forcing, R);
      HIPCHK(hipGetLastError());
    }
    const double rn = norm2(P, R, s);
    rep->rnorm[it] = rn;
    rep->newton_steps = it;
    rep->C = *C;
    if (!std::isfinite(rn)) throw Fail{SC_ERR_NONFINITE, "Newton residual is not finite"};
    if (rn <= o.tol) {
      rep->converged = 1;
      return;
    }
    if (it >= o.max_newton) return;
    set_base_impl(P, x, *C, J, s);
    const int mv = gmres(P, R, du, o.gmres_tol, o.restart, o.max_matvec, o.prec, s);
    rep->step_matvecs[it] = mv;
    rep->matvecs += mv;
    if (J >= 0) {
      double c = 0.0, zero = 0.0;
      HIPCHK(hipMemcpyAsync(&c, du + J, sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      HIPCHK(hipMemcpyAsync(du + J, &zero, sizeof(double), hipMemcpyHostToDevice, s));
      HIPCHK(hipStreamSynchronize(s));
      *C -= c;
    }
    std::vector<double> one{1.0};
    combine(P, x, 1.0, du, n, 1, one, s);
  }
}

}  // namespace

// ==========================================================================================
extern "C" {

const char* sc_last_error(void) { return g_last_error.c_str(); }

int sc_plan_create(sc_plan** out, const sc_params* params) {
  if (!out || !params) return fail(SC_ERR_ARG, "null argument");
  *out = nullptr;
  return guarded([&] {
    std::unique_ptr<sc_plan> P(new sc_plan());
    P->prm = *params;
    const sc_params& p = *params;
    if (p.L < 1 || p.m0 < 1 || p.M < 0 || p.N < 6 || p.N > 64) throw Fail{SC_ERR_ARG, "need L >= 1, m0 >= 1, M >= 0, 6 <= N <= 64"};
    if (!(p.radius_ratio > 0 && p.radius_ratio < 1)) throw Fail{SC_ERR_ARG, "radius_ratio must lie in (0, 1)"};
    if (!(p.Ek > 0) || !(p.Pr > 0) || !(p.dt > 0) || !std::isfinite(p.Ra)) throw Fail{SC_ERR_ARG, "need Ek, Pr, dt > 0 and finite Ra"};
    P->vcap = p.nvec_max > 0 ? p.nvec_max : 16;
    P->wcap = (P->vcap + kVG - 1) / kVG * kVG;
    P->refine64 = p.refine_fp64 >= 0 ? p.refine_fp64 : 1;
    P->refine32 = p.refine_mixed >= 0 ? p.refine_mixed : 1;
    if (p.mixed_solve != 0 && p.mixed_solve != SC_MIXED_SOLVE_FP64 && p.mixed_solve != SC_MIXED_SOLVE_FP32)
      throw Fail{SC_ERR_ARG, "mixed_solve must be 0, SC_MIXED_SOLVE_FP64 or SC_MIXED_SOLVE_FP32"};
    P->mixed_fp32_solve = (p.mixed_solve == SC_MIXED_SOLVE_FP32);
    if (p.coriolis != SC_CORIOLIS_IMPLICIT && p.coriolis != SC_CORIOLIS_EXPLICIT)
      throw Fail{SC_ERR_ARG, "coriolis must be SC_CORIOLIS_IMPLICIT or SC_CORIOLIS_EXPLICIT"};
    // HIP graph capture is switched off: the first captured batch call ended the process with a
    // host segmentation fault inside the HIP runtime, on the caller's stream and again on a
    // library stream with every return code checked; the cause is not found, so no plan takes
    // the captured path (the capture code below stays, unreachable, for that investigation)
    if (p.graph_capture != 0)
      throw Fail{SC_ERR_ARG, "graph_capture is switched off in this build (a captured batch call crashed the host "
                             "process; cause not found): pass 0"};
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (p.device < 0 || p.device >= ndev) throw Fail{SC_ERR_ARG, "bad device ordinal"};
    HIPCHK(hipSetDevice(p.device));
    resolve_scratch(p.device);
    HIPCHK(hipStreamCreateWithFlags(&P->side, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&P->ev_join, hipEventDisableTiming));
    HIPCHK(hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&P->ev_gin, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&P->ev_gout, hipEventDisableTiming));
    try {
      sc::build_grid(P->hg, p.L, p.M, p.m0, p.N, p.radius_ratio, p.nr_phys, p.ntheta, p.nphi);
    } catch (const std::runtime_error& e) {
      throw Fail{SC_ERR_ARG, e.what()};
    }
    const sc::HostGrid& g = P->hg;
    if (g.Np > 128) throw Fail{SC_ERR_ARG, "N_p > 128 unsupported"};
    if (g.nth % 2) throw Fail{SC_ERR_ARG, "ntheta must be even (mirror pairs of Gauss-Legendre nodes)"};
    P->n_real = 6LL * g.N * g.S;
    upload(P->d_lmk, g.lm_k);
    upload(P->d_lml, g.lm_l);
    upload(P->d_lmbase, g.lmbase);
    upload(P->d_r, g.r);
    upload(P->d_rp, g.rp);
    upload(P->d_E, g.E);
    upload(P->d_ED, g.ED);
    upload(P->d_ED2, g.ED2);
    upload(P->d_P, g.P);
    upload(P->d_Dp, g.Dp);
    upload(P->d_D, g.D);
    upload(P->d_D2, g.D2);
    upload(P->d_D4, g.D4);
    {
      std::vector<double> cst(2 * (size_t)g.nth);
      for (int j = 0; j < g.nth; ++j) {
        cst[j] = g.ct[j];
        cst[g.nth + j] = g.st[j];
      }
      upload(P->d_cst, cst);
    }
    auto transpose = [](const std::vector<double>& A, int rows, int cols) {
      std::vector<double> T((size_t)rows * cols);
      for (int i = 0; i < rows; ++i)
        for (int j = 0; j < cols; ++j) T[(size_t)j * rows + i] = A[(size_t)i * cols + j];
      return T;
    };
    {
      // E, ED, ED2 in MFMA operand order, k (the N nodes) padded to 16 ceil(N/16)
      const int rtp = (g.Np + 15) / 16, ks = 4 * ((g.N + 15) / 16);
      const size_t ms = (size_t)rtp * ks * 64;
      std::vector<double> F(3 * ms, 0.0);
      const std::vector<double>* mats[3] = {&g.E, &g.ED, &g.ED2};
      for (int a = 0; a < 3; ++a)
        for (int t = 0; t < rtp; ++t)
          for (int sk = 0; sk < ks; ++sk)
            for (int l = 0; l < 64; ++l) {
              const int row = 16 * t + l % 16, col = 4 * sk + l / 16;
              if (row < g.Np && col < g.N) F[a * ms + ((size_t)t * ks + sk) * 64 + l] = (*mats[a])[(size_t)row * g.N + col];
            }
      upload(P->d_EF, F);
    }
    {
      // projection matrices (N x N_p) and D^2 (N x N) in MFMA operand order
      const int rtn = (g.N + 15) / 16, ksp = 4 * ((g.Np + 15) / 16), ksn = 4 * rtn;
      auto frag = [](const std::vector<double>& M, int rows, int cols, int rt, int ks, double* out) {
        for (int t = 0; t < rt; ++t)
          for (int sk = 0; sk < ks; ++sk)
            for (int l = 0; l < 64; ++l) {
              const int row = 16 * t + l % 16, col = 4 * sk + l / 16;
              out[((size_t)t * ks + sk) * 64 + l] = (row < rows && col < cols) ? M[(size_t)row * cols + col] : 0.0;
            }
      };
      const int N = g.N, Np = g.Np;
      std::vector<double> P1((size_t)N * Np), P2((size_t)N * Np), PDr((size_t)N * Np, 0.0);
      for (int j = 0; j < N; ++j)
        for (int q = 0; q < Np; ++q) {
          const double pr = g.P[(size_t)j * Np + q], r = g.rp[q];
          P1[(size_t)j * Np + q] = pr / r;
          P2[(size_t)j * Np + q] = pr / (r * r);
        }
      for (int j = 0; j < N; ++j)          // P diag(1/r^2) Dp diag(r)
        for (int i = 0; i < Np; ++i) {
          const double a = P2[(size_t)j * Np + i];
          for (int q = 0; q < Np; ++q) PDr[(size_t)j * Np + q] += a * g.Dp[(size_t)i * Np + q] * g.rp[q];
        }
      const size_t ms = (size_t)rtn * ksp * 64;
      std::vector<double> F(4 * ms);
      frag(P1, N, Np, rtn, ksp, F.data());
      frag(P2, N, Np, rtn, ksp, F.data() + ms);
      frag(PDr, N, Np, rtn, ksp, F.data() + 2 * ms);
      frag(g.P, N, Np, rtn, ksp, F.data() + 3 * ms);
      upload(P->d_PF, F);
      std::vector<double> F2((size_t)rtn * ksn * 64);
      frag(g.D2, N, N, rtn, ksn, F2.data());
      upload(P->d_D2F, F2);
      frag(g.D, N, N, rtn, ksn, F2.data());
      upload(P->d_DF, F2);
      frag(g.D4, N, N, rtn, ksn, F2.data());
      upload(P->d_D4F, F2);
      std::vector<int2> tiles;
      for (int k = 0; k <= g.K; ++k)
        for (int il = 0; il < g.nl[k]; il += sc::kRLT) tiles.push_back(make_int2(k, il));
      upload(P->d_qtiles, tiles);
      P->nqtiles = (int)tiles.size();
    }
    upload(P->d_ET, transpose(g.E, g.Np, g.N));
    upload(P->d_EDT, transpose(g.ED, g.Np, g.N));
    upload(P->d_ED2T, transpose(g.ED2, g.Np, g.N));
    upload(P->d_DT, transpose(g.D, g.N, g.N));
    upload(P->d_D2T, transpose(g.D2, g.N, g.N));
    upload(P->d_D4T, transpose(g.D4, g.N, g.N));
    upload(P->d_PT, transpose(g.P, g.N, g.Np));
    upload(P->d_DpT, transpose(g.Dp, g.Np, g.Np));
    {
      std::vector<int2> tiles;
      for (int k = 0; k <= g.K; ++k)
        for (int il = 0; il < g.nl[k]; il += sc::kPT) tiles.push_back(make_int2(k, il));
      upload(P->d_ptiles, tiles);
      P->nptiles = (int)tiles.size();
    }
    {
      std::vector<int2> tiles;
      for (int k = 0; k <= g.K; ++k)
        for (int il = 0; il < g.nl[k]; il += sc::kRPT) tiles.push_back(make_int2(k, il));
      upload(P->d_rtiles, tiles);
      P->nrtiles = (int)tiles.size();
    }
    build_tables(P.get());
    build_workspaces(P.get());
    {
      // azimuthal FFT plan: radices 8, then 4, 2, 3, 5
      int n = g.nphi, nr = 0;
      P->fft_nr = 0;
      for (int R : {8, 4, 2, 3, 5})
        while (n % R == 0) {
          if (nr == 8) throw Fail{SC_ERR_ARG, "nphi needs more than 8 FFT passes"};
          P->fft_r[nr++] = R;
          n /= R;
        }
      if (n != 1) throw Fail{SC_ERR_ARG, "nphi must be a product of powers of 2, 3 and 5"};
      P->fft_nr = nr;
      if (ring_rt_log2<double>(g) < 0 || ring_rt_log2<float>(g) < 0)
        throw Fail{SC_ERR_ARG, "nphi too large for the ring kernel"};
      const size_t smem64 = sc::ring_lds_bytes<double>(g.nphi, ring_rt_log2<double>(g));
      const size_t smem32 = sc::ring_lds_bytes<float>(g.nphi, ring_rt_log2<float>(g));
      if (smem64 > 64 * 1024 || smem32 > 64 * 1024) throw Fail{SC_ERR_INTERNAL, "ring LDS above 64 KB"};
    }
    if (sc::project_lds_bytes<double>(g.Np, g.N) > 64 * 1024) {
      project_attr<double, true, 1>(); project_attr<double, true, 2>(); project_attr<double, true, 3>(); project_attr<double, true, 4>();
      project_attr<double, false, 1>(); project_attr<double, false, 2>(); project_attr<double, false, 3>(); project_attr<double, false, 4>();
      project_attr<float, false, 1>(); project_attr<float, false, 2>(); project_attr<float, false, 3>(); project_attr<float, false, 4>();
    }
    {
      const size_t t64 = tsolve_smem<double>(g), t32 = tsolve_smem<float>(g);
      if (t64 > 160 * 1024) throw Fail{SC_ERR_ARG, "too many m for the temperature solve"};
      auto attr = [](const void* f, size_t b) {
        HIPCHK(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)b));
      };
      if (t64 > 64 * 1024) {
        attr((const void*)sc::k_T_solve<double, false, false>, t64);
        attr((const void*)sc::k_T_solve<double, false, true>, t64);
        attr((const void*)sc::k_T_solve<double, true, false>, t64);
        attr((const void*)sc::k_T_solve<double, true, true>, t64);
      }
      if (t32 > 64 * 1024) {
        attr((const void*)sc::k_T_solve<float, false, false>, t32);
        attr((const void*)sc::k_T_solve<float, false, true>, t32);
      }
      // folded analysis: LDS grows with N_theta; beyond the CU's 160 KiB the GEMM path is used
      const size_t a64 = sc::ana_lds_bytes<double>(g.nth, g.L + 1), a32 = sc::ana_lds_bytes<float>(g.nth, g.L + 1);
      if (a64 > 160 * 1024 || g.nth > 256) P->ana_ct = 0;   // the fold covers nth/2 <= 128 nodes
      P->ana_ct_fold = P->ana_ct;
      if (P->ana_ct > 0 && a64 > 64 * 1024) {
        for (const void* f : {(const void*)sc::k_anal<double, 1>, (const void*)sc::k_anal<double, 2>,
                              (const void*)sc::k_anal<double, 3>, (const void*)sc::k_anal<double, 5>,
                              (const void*)sc::k_anal<double, 8>})
          attr(f, a64);
        if (a32 > 64 * 1024)
          for (const void* f : {(const void*)sc::k_anal<float, 1>, (const void*)sc::k_anal<float, 2>,
                                (const void*)sc::k_anal<float, 3>, (const void*)sc::k_anal<float, 5>,
                                (const void*)sc::k_anal<float, 8>})
            attr(f, a32);
      }
    }
    // deterministic contents for slots the solves never write (e, f at l = 0)
    HIPCHK(hipMemset(P->xbuf.p, 0, P->xbuf.bytes));
    HIPCHK(hipMemset(P->dbuf.p, 0, P->dbuf.bytes));
    HIPCHK(hipMemset(P->rbuf.p, 0, P->rbuf.bytes));
    HIPCHK(hipDeviceSynchronize());
    *out = P.release();
  });
}

int sc_plan_destroy(sc_plan* plan) {
  if (!plan) return SC_OK;
  (void)hipSetDevice(plan->prm.device);
  (void)hipDeviceSynchronize();
  delete plan;
  return SC_OK;
}

int sc_layout(const sc_plan* P, sc_layout_info* out) {
  if (!P || !out) return fail(SC_ERR_ARG, "null argument");
  const sc::HostGrid& g = P->hg;
  out->n_real = P->n_real;
  out->L = g.L;
  out->M = g.M;
  out->m0 = g.m0;
  out->N = g.N;
  out->K = g.K;
  out->S = g.S;
  out->Np = g.Np;
  out->ntheta = g.nth;
  out->nphi = g.nphi;
  out->nvec_max = P->vcap;
  return SC_OK;
}

int sc_set_params(sc_plan* P, double Ra, double Ek, double dt) {
  if (!P) return fail(SC_ERR_ARG, "null plan");
  if (!(Ek > 0) || !(dt > 0) || !std::isfinite(Ra)) return fail(SC_ERR_ARG, "need Ek, dt > 0 and finite Ra");
  if (Ek != P->prm.Ek || dt != P->prm.dt) P->factored = false;
  ++P->gen;
  ++P->graph_epoch;
  P->prm.Ra = Ra;
  P->prm.Ek = Ek;
  P->prm.dt = dt;
  return SC_OK;
}

int sc_factor(sc_plan* P, void* stream) {
  return guarded([&] {
    check_plan(P);
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipStreamSynchronize(s));
    const sc::HostGrid& g = P->hg;
    std::vector<sc::ChainFactor> ch;
    std::vector<sc::TFactor> tf;
    sc::OpParams op{P->prm.Ek, P->prm.Pr, P->prm.dt, P->prm.coriolis == SC_CORIOLIS_EXPLICIT ? 0.0 : 1.0};
    int nth = (int)std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
    sc::factor_all(g, op, ch, tf, nth, kSeg);
    const int N = g.N;
    std::vector<sc::ChainMeta> meta;
    std::vector<sc::SegMeta> segv;
    std::vector<int> bf, blm, bnext;
    long long nb = 0;
    for (auto& c : ch) nb += c.n;
    const long long NN = (long long)N * N;
    // blocks in MFMA operand order (see the chain-solve kernels): RT row tiles, 4 RT k-steps,
    // lane l of (t, s) holds M[16 t + l % 16][4 s + l / 16], zero outside N x N
    const int RT = (N + 15) / 16, KS = 4 * RT;
    const long long FB = sc::frag_block_size(RT);
    std::vector<double> Dm(2 * nb * FB, 0.0), Gm(2 * nb * FB, 0.0), H(2 * nb * FB, 0.0), Phi(2 * nb * FB, 0.0),
        Psi(2 * nb * FB, 0.0);
    std::vector<double> Cg(nb * N);
    std::vector<sc::cplx> Dblk((size_t)NN);
    long long b = 0;
    auto put = [&](std::vector<double>& dst, const std::vector<sc::cplx>& src, long long bb, int i) {
      for (int t = 0; t < RT; ++t)
        for (int ks = 0; ks < KS; ++ks)
          for (int l = 0; l < 64; ++l) {
            const int row = 16 * t + l % 16, col = 4 * ks + l / 16;
            if (row >= N || col >= N) continue;
            const long long o = bb * FB + ((long long)t * KS + ks) * 64 + l;
            const sc::cplx v = src[(size_t)i * NN + (size_t)row * N + col];
            dst[2 * o] = v.real();
            dst[2 * o + 1] = v.imag();
          }
    };
    for (int ci = 0; ci < (int)ch.size(); ++ci) {
      auto& c = ch[ci];
      int nseg = (c.n + kSeg - 1) / kSeg;
      meta.push_back(sc::ChainMeta{(int)b, c.n, c.k, (int)segv.size(), nseg, 0, 0, 0});
      for (int p = 0; p < nseg; ++p) segv.push_back(sc::SegMeta{(int)b + p * kSeg, std::min(kSeg, c.n - p * kSeg), ci, p});
      for (int i = 0; i < c.n; ++i, ++b) {
        bf.push_back(c.field[i]);
        blm.push_back(g.lmbase[c.k] + (c.l[i] - c.m));
        int p = i / kSeg;
        bool fixup = (p < nseg - 1) && (i % kSeg != 0);
        bnext.push_back(fixup ? (int)(meta.back().start + (p + 1) * kSeg) : -1);
        // D_i = diag(sc_i) Shat_i^{-1} diag(sr_i) diag(Rg_i): the right-hand side's scalings
        // folded into the pivot block's inverse, so that c_i = D_i b_i
        for (int r = 0; r < N; ++r)
          for (int q = 0; q < N; ++q)
            Dblk[(size_t)r * N + q] = c.Sinv[(size_t)i * NN + (size_t)r * N + q] *
                                      (c.sc[(size_t)i * N + r] * c.sr[(size_t)i * N + q] * c.Rg[(size_t)i * N + q]);
        put(Dm, Dblk, b, 0);
        put(Gm, c.G, b, i);
        put(H, c.H, b, i);
        put(Phi, c.Phi, b, i);
        put(Psi, c.Psi, b, i);
        for (int j = 0; j < N; ++j) Cg[b * N + j] = c.Cg[(size_t)i * N + j];
      }
    }
    std::vector<double> Tinv((size_t)(g.L + 1) * N * N), tr((size_t)(g.L + 1) * N), tc((size_t)(g.L + 1) * N);
    for (int l = 0; l <= g.L; ++l) {
      std::copy(tf[l].Tinv.begin(), tf[l].Tinv.end(), Tinv.begin() + (size_t)l * N * N);
      std::copy(tf[l].tr.begin(), tf[l].tr.end(), tr.begin() + (size_t)l * N);
      std::copy(tf[l].tc.begin(), tf[l].tc.end(), tc.begin() + (size_t)l * N);
    }
    auto up2 = [](DevBuf& d64, DevBuf& d32, const std::vector<double>& h) {
      upload(d64, h);
      std::vector<float> f(h.begin(), h.end());
      upload(d32, f);
    };
    upload(P->chains, meta);
    upload(P->segs, segv);
    upload(P->blk_field, bf);
    upload(P->blk_lm, blm);
    upload(P->blk_next, bnext);
    up2(P->D64, P->D32, Dm);
    up2(P->G64, P->G32, Gm);
    up2(P->H64, P->H32, H);
    up2(P->Phi64, P->Phi32, Phi);
    up2(P->Psi64, P->Psi32, Psi);
    P->wscan.alloc((size_t)P->wcap * nb * N * 2 * sizeof(double));
    HIPCHK(hipMemset(P->wscan.p, 0, (size_t)P->wcap * nb * N * 2 * sizeof(double)));
    up2(P->Cg64, P->Cg32, Cg);
    up2(P->Tinv64, P->Tinv32, Tinv);
    up2(P->tr64, P->tr32, tr);
    up2(P->tc64, P->tc32, tc);
    P->nchains = (int)meta.size();
    P->nblocks = (int)nb;
    P->nsegs = (int)segv.size();
    P->factored = true;
    P->have_base = false;  // the cached M X depends on Ek
    ++P->gen;
    ++P->graph_epoch;
  });
}

int sc_step(sc_plan* P, const double* x, double C, double* x_next, void* stream) {
  return guarded([&] {
    check_plan(P);
    if (!x || !x_next) throw Fail{SC_ERR_ARG, "null vector"};
    if (!P->factored) throw Fail{SC_ERR_STATE, "sc_factor has not run for the current (Ek, dt)"};
    hipStream_t s = (hipStream_t)stream;
    step_into_xbuf(P, x, C, s);
    long long n = P->n_real;
    {
      Prof _p(P, SC_STAGE_FINALIZE, s);
      hipLaunchKernelGGL(sc::k_finalize, dim3(nblk(n, 256)), dim3(256), 0, s, P->dg(), 1, P->xbuf.as<const double>(), x, n,
                         (long long)-1, x_next, n, 0);
    }
    HIPCHK(hipGetLastError());
  });
}

int sc_newton_residual(sc_plan* P, const double* x, double C, double* r, double* rnorm_host, void* stream) {
  return guarded([&] {
    check_plan(P);
    if (!x || !r) throw Fail{SC_ERR_ARG, "null vector"};
    if (!P->factored) throw Fail{SC_ERR_STATE, "sc_factor has not run for the current (Ek, dt)"};
    hipStream_t s = (hipStream_t)stream;
    step_into_xbuf(P, x, C, s);
    long long n = P->n_real;
    {
      Prof _p(P, SC_STAGE_FINALIZE, s);
      hipLaunchKernelGGL(sc::k_finalize, dim3(nblk(n, 256)), dim3(256), 0, s, P->dg(), 1, P->xbuf.as<const double>(), x, n,
                         (long long)-1, r, n, 1);
    }
    HIPCHK(hipGetLastError());
    if (rnorm_host) {
      hipLaunchKernelGGL(sc::k_sumsq, dim3(1), dim3(256), 0, s, n, (const double*)r, n, P->norms.as<double>());
      HIPCHK(hipGetLastError());
      double ss = 0.0;
      HIPCHK(hipMemcpyAsync(&ss, P->norms.p, sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      *rnorm_host = std::sqrt(ss);
      if (!std::isfinite(*rnorm_host)) throw Fail{SC_ERR_NONFINITE, "residual norm is not finite"};
    }
  });
}

int sc_newton_residual_noalloc(sc_plan* P, const double* x, double C, double* r, double* rnorm_dev, void* stream) {
  return guarded([&] {
    check_plan(P);
    if (!x || !r || !rnorm_dev) throw Fail{SC_ERR_ARG, "null vector"};
    if (!P->factored) throw Fail{SC_ERR_STATE, "sc_factor has not run for the current (Ek, dt)"};
    const long long n = P->n_real;
    const long long nparts = (n + kNoAllocChunk - 1) / kNoAllocChunk;
    if (nparts > kNoAllocParts)
      throw Fail{SC_ERR_ARG, "n_real = " + std::to_string(n) + " exceeds the allocation-free limit of " +
                                 std::to_string((long long)kNoAllocParts * kNoAllocChunk) + " values"};
    double* parts = scratch_on(P->prm.device);
    if (!parts) throw Fail{SC_ERR_INTERNAL, "scratch address of the device was not resolved"};
    hipStream_t s = (hipStream_t)stream;
    step_into_xbuf(P, x, C, s);
    {
      Prof _p(P, SC_STAGE_FINALIZE, s);
      hipLaunchKernelGGL(sc::k_finalize, dim3(nblk(n, 256)), dim3(256), 0, s, P->dg(), 1, P->xbuf.as<const double>(), x, n,
                         (long long)-1, r, n, 1);
    }
    HIPCHK(hipGetLastError());
    // every partial is written before it is read: nothing needs clearing
    hipLaunchKernelGGL(sc::k_sumsq_parts, dim3((unsigned)nparts), dim3(256), 0, s, n, (const double*)r, kNoAllocChunk,
                       parts);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(sc::k_sqrt_sum, dim3(1), dim3(256), 0, s, (int)nparts, (const double*)parts, rnorm_dev);
    HIPCHK(hipGetLastError());
  });
}

int sc_set_base(sc_plan* P, const double* x, double C, long long J, void* stream) {
  return guarded([&] {
    check_plan(P);
    if (!x) throw Fail{SC_ERR_ARG, "null vector"};
    if (!P->factored) throw Fail{SC_ERR_STATE, "sc_factor has not run for the current (Ek, dt)"};
    set_base_impl(P, x, C, check_slot(P, J), (hipStream_t)stream);
  });
}

int sc_profile(sc_plan* P, int enable) {
  return guarded([&] {
    check_plan(P);
    HIPCHK(hipDeviceSynchronize());
    if (enable && P->ev.empty()) {
      const int cap = 16384;
      P->ev.resize(2 * cap);
      P->ev_stage.assign(cap, -1);
      for (auto& e : P->ev) HIPCHK(hipEventCreate(&e));
    }
    P->ev_used = 0;
    P->prof_on = enable != 0;
  });
}

int sc_profile_read(sc_plan* P, double* ms_total, long long* count, int nstages) {
  return guarded([&] {
    check_plan(P);
    if (!ms_total || !count || nstages < 0) throw Fail{SC_ERR_ARG, "null output"};
    for (int i = 0; i < nstages; ++i) {
      ms_total[i] = 0.0;
      count[i] = 0;
    }
    for (int q = 0; q < P->ev_used; ++q) {
      HIPCHK(hipEventSynchronize(P->ev[2 * q + 1]));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, P->ev[2 * q], P->ev[2 * q + 1]));
      int st = P->ev_stage[q];
      if (st >= 0 && st < nstages) {
        ms_total[st] += ms;
        count[st] += 1;
      }
    }
    P->ev_used = 0;
  });
}

}  // extern "C"

// Ring kernel choice c of precision T: -1 - v the register kernel of shape v, k >= 0 the LDS
// kernel with 2^k rings per workgroup (validated by the callers).
template <class T>
static void set_ring_choice(sc_plan* P, int c) {
  const bool reg = c < 0;
  const int rv = reg ? -1 - c : 0;
  if (std::is_same<T, float>::value) {
    P->ring_reg32 = reg;
    P->ring_rtl32 = c;
    P->ring_rv32 = rv;
  } else {
    P->ring_reg64 = reg;
    P->ring_rtl64 = c;
    P->ring_rv64 = rv;
  }
}

extern "C" {

int sc_autotune(sc_plan* P, int nvec, int reps, sc_tune_report* rep, void* stream) {
  return guarded([&] {
    check_plan(P);
    if (nvec < 1 || nvec > P->vcap || reps < 1) throw Fail{SC_ERR_ARG, "need 1 <= nvec <= nvec_max and reps >= 1"};
    if (P->prof_on) throw Fail{SC_ERR_STATE, "turn the stage profiler off before sc_autotune"};
    hipStream_t s = (hipStream_t)stream;
    const sc::HostGrid& g = P->hg;
    DevBuf vin;
    vin.alloc((size_t)nvec * P->n_real * sizeof(double));
    HIPCHK(hipMemsetAsync(vin.p, 0, vin.bytes, s));
    struct Events {
      hipEvent_t a = nullptr, b = nullptr;
      ~Events() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
      }
    } ev;
    HIPCHK(hipEventCreate(&ev.a));
    HIPCHK(hipEventCreate(&ev.b));
    int ncand = 0;
    // the jvp's products (linear mode, base fields read per point) once a base state is set,
    // else the nonlinear products of the step
    const int mode = P->have_base ? sc::RING_LINEAR : sc::RING_NONLINEAR;
    // ms per transform pass of the current choices
    auto time_pass = [&](auto tag) -> double {
      typedef decltype(tag) T;
      transforms<T>(P, mode, nvec, vin.as<double>(), P->n_real, -1, s);
      HIPCHK(hipEventRecord(ev.a, s));
      for (int i = 0; i < reps; ++i) transforms<T>(P, mode, nvec, vin.as<double>(), P->n_real, -1, s);
      HIPCHK(hipEventRecord(ev.b, s));
      HIPCHK(hipEventSynchronize(ev.b));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, ev.a, ev.b));
      return (double)ms / reps;
    };
    // ring candidates: -1 - v register kernel of shape v, k >= 0 LDS kernel with 2^k rings
    auto ring_cands = [&](auto tag) {
      typedef decltype(tag) T;
      std::vector<int> c;
      if (ring_reg_available(P->dg()))
        for (int v = 0; v < sc::ring_reg_variants<T>(); ++v) c.push_back(-1 - v);
      for (int k = 0; k <= ring_rt_log2<T>(g); ++k) c.push_back(k);
      return c;
    };
    auto set_ring = [&](auto tag, int c) { set_ring_choice<decltype(tag)>(P, c); };
    // three interleaved rounds over the candidates, each kept at its fastest round: drifts of
    // the device (clocks, caches) then touch every candidate alike, and the register ring's
    // shapes differ by only a few per cent
    auto tune_ring = [&](auto tag, double& best, int& choice) {
      const std::vector<int> cands = ring_cands(tag);
      ncand += (int)cands.size();
      std::vector<double> t(cands.size(), 1e300);
      for (int round = 0; round < 3; ++round)
        for (size_t i = 0; i < cands.size(); ++i) {
          set_ring(tag, cands[i]);
          t[i] = std::min(t[i], time_pass(tag));
        }
      best = 1e300;
      for (size_t i = 0; i < cands.size(); ++i)
        if (t[i] < best) {
          best = t[i];
          choice = cands[i];
        }
      set_ring(tag, choice);
    };
    // FP32: ring choice for each analysis path; the analysis path serves both precisions
    double best32 = 1e300, best64 = 1e300;
    int ring32 = 0, ring64 = 0, folded = 0;
    std::vector<int> paths;
    if (P->ana_ct_fold > 0) paths.push_back(1);
    paths.push_back(0);
    for (int f : paths) {
      P->ana_ct = f ? P->ana_ct_fold : 0;
      double t;
      int c = 0;
      tune_ring(0.0f, t, c);
      if (t < best32) {
        best32 = t;
        ring32 = c;
        folded = f;
      }
    }
    P->ana_ct = folded ? P->ana_ct_fold : 0;
    set_ring(0.0f, ring32);
    tune_ring(0.0, best64, ring64);
    if (rep) {
      rep->ring_fp32 = ring32;
      rep->ring_fp64 = ring64;
      rep->anal_folded = folded;
      rep->ncand = ncand;
      rep->ms_fp32 = best32;
      rep->ms_fp64 = best64;
      rep->linear_mode = mode == sc::RING_LINEAR ? 1 : 0;
    }
    ++P->graph_epoch;
  });
}

int sc_set_kernels(sc_plan* P, int ring_fp32, int ring_fp64, int anal_folded) {
  return guarded([&] {
    check_plan(P);
    const sc::HostGrid& g = P->hg;
    auto ok = [&](int c, int lim, int nvar) {
      return c < 0 ? (ring_reg_available(P->dg()) && -1 - c < nvar) : c <= lim;
    };
    if (!ok(ring_fp32, ring_rt_log2<float>(g), sc::ring_reg_variants<float>()) ||
        !ok(ring_fp64, ring_rt_log2<double>(g), sc::ring_reg_variants<double>()))
      throw Fail{SC_ERR_ARG, "ring kernel choice not available on this grid"};
    if ((anal_folded != 0 && anal_folded != 1) || (anal_folded == 1 && P->ana_ct_fold == 0))
      throw Fail{SC_ERR_ARG, "analysis kernel choice not available on this grid"};
    set_ring_choice<float>(P, ring_fp32);
    set_ring_choice<double>(P, ring_fp64);
    P->ana_ct = anal_folded ? P->ana_ct_fold : 0;
    ++P->graph_epoch;
  });
}

int sc_get_kernels(const sc_plan* P, int* ring_fp32, int* ring_fp64, int* anal_folded) {
  return guarded([&] {
    if (!P) throw Fail{SC_ERR_ARG, "null plan"};
    const sc::HostGrid& g = P->hg;
    auto cur = [&](bool reg, int rv, int rtl, int lim) {
      if (reg && ring_reg_available(P->dg())) return -1 - rv;
      return rtl >= 0 ? std::min(rtl, lim) : lim;
    };
    if (ring_fp32) *ring_fp32 = cur(P->ring_reg32, P->ring_rv32, P->ring_rtl32, ring_rt_log2<float>(g));
    if (ring_fp64) *ring_fp64 = cur(P->ring_reg64, P->ring_rv64, P->ring_rtl64, ring_rt_log2<double>(g));
    if (anal_folded) *anal_folded = P->ana_ct > 0 ? 1 : 0;
  });
}

int sc_jvp(sc_plan* P, int nvec, const double* v, long long ldv, double* y, long long ldy, sc_precision prec,
           void* stream) {
  return guarded([&] {
    check_plan(P);
    if (nvec < 0 || nvec > P->vcap) throw Fail{SC_ERR_ARG, "nvec exceeds nvec_max of the plan"};
    if (nvec == 0) return;
    if (!v || !y) throw Fail{SC_ERR_ARG, "null vector"};
    if (ldv < P->n_real || ldy < P->n_real) throw Fail{SC_ERR_ARG, "leading dimension smaller than n_real"};
    if (prec != SC_FP64 && prec != SC_MIXED) throw Fail{SC_ERR_ARG, "unknown precision"};
    if (!P->factored || !P->have_base) throw Fail{SC_ERR_STATE, "call sc_factor and sc_set_base before sc_jvp"};
    jvp_impl(P, nvec, v, ldv, y, ldy, prec, (hipStream_t)stream);
  });
}

int sc_newton(sc_plan* P, double* x, double* C, const sc_newton_opts* o, sc_newton_report* rep, void* stream) {
  return guarded([&] {
    check_plan(P);
    if (!x || !C || !o || !rep) throw Fail{SC_ERR_ARG, "null argument"};
    if (o->restart < 1 || o->restart > 1024) throw Fail{SC_ERR_ARG, "restart must lie in 1..1024"};
    if (o->max_newton < 0 || o->max_newton > 64 || o->max_matvec < 1) throw Fail{SC_ERR_ARG, "bad iteration caps"};
    if (o->prec != SC_FP64 && o->prec != SC_MIXED) throw Fail{SC_ERR_ARG, "unknown precision"};
    if (!P->factored) throw Fail{SC_ERR_STATE, "sc_factor has not run for the current (Ek, dt)"};
    const long long J = check_slot(P, o->J);
    newton_impl(P, x, C, *o, J, rep, (hipStream_t)stream);
  });
}


// ------------------------------------------------------------------------------------------
// Ragged batches: one stream branch per plan, forked from and joined into the caller's stream.
struct sc_batch {
  std::vector<sc_plan*> plans;
  int device = 0;
  std::vector<hipStream_t> br;             // one branch stream per plan
  hipEvent_t ev_start = nullptr;
  std::vector<hipEvent_t> ev_done;
  // graph of a whole batch call (when every plan has graph_capture): captured on `cap`, cached per
  // (precision, vectors) while no plan's graph_epoch moves
  hipStream_t cap = nullptr;
  hipEvent_t ev_gin = nullptr, ev_gout = nullptr;
  std::map<std::vector<long long>, hipGraphExec_t> graphs;
  std::vector<unsigned long long> epochs;

  void drop_graphs() {
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    graphs.clear();
  }
  ~sc_batch() {
    drop_graphs();
    for (auto e : ev_done) (void)hipEventDestroy(e);
    if (ev_start) (void)hipEventDestroy(ev_start);
    if (ev_gin) (void)hipEventDestroy(ev_gin);
    if (ev_gout) (void)hipEventDestroy(ev_gout);
    for (auto st : br) (void)hipStreamDestroy(st);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

int sc_batch_create(sc_batch** out, sc_plan* const* plans, int nplans) {
  if (!out || !plans || nplans < 1) return fail(SC_ERR_ARG, "need at least one plan");
  *out = nullptr;
  return guarded([&] {
    std::unique_ptr<sc_batch> B(new sc_batch());
    for (int i = 0; i < nplans; ++i) {
      if (!plans[i]) throw Fail{SC_ERR_ARG, "null plan"};
      for (int j = 0; j < i; ++j)
        if (plans[j] == plans[i]) throw Fail{SC_ERR_ARG, "a plan is listed twice"};
      if (plans[i]->prm.device != plans[0]->prm.device) throw Fail{SC_ERR_ARG, "plans on different devices"};
      B->plans.push_back(plans[i]);
    }
    B->device = plans[0]->prm.device;
    HIPCHK(hipSetDevice(B->device));
    HIPCHK(hipEventCreateWithFlags(&B->ev_start, hipEventDisableTiming));
    B->br.resize(nplans, nullptr);
    B->ev_done.resize(nplans, nullptr);
    for (int i = 0; i < nplans; ++i) {
      HIPCHK(hipStreamCreateWithFlags(&B->br[i], hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&B->ev_done[i], hipEventDisableTiming));
    }
    HIPCHK(hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&B->ev_gin, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&B->ev_gout, hipEventDisableTiming));
    *out = B.release();
  });
}

int sc_batch_destroy(sc_batch* b) {
  if (!b) return SC_OK;
  (void)hipSetDevice(b->device);
  (void)hipDeviceSynchronize();
  delete b;
  return SC_OK;
}

int sc_batch_jvp(sc_batch* b, const int* nvec, const double* const* v, double* const* y, sc_precision prec,
                 void* stream) {
  return guarded([&] {
    if (!b || !nvec || !v || !y) throw Fail{SC_ERR_ARG, "null argument"};
    if (prec != SC_FP64 && prec != SC_MIXED) throw Fail{SC_ERR_ARG, "unknown precision"};
    HIPCHK(hipSetDevice(b->device));
    const int n = (int)b->plans.size();
    for (int i = 0; i < n; ++i) {
      sc_plan* P = b->plans[i];
      if (nvec[i] < 0 || nvec[i] > P->vcap) throw Fail{SC_ERR_ARG, "nvec exceeds nvec_max of a plan"};
      if (nvec[i] > 0 && (!v[i] || !y[i])) throw Fail{SC_ERR_ARG, "null vector"};
      if (!P->factored || !P->have_base) throw Fail{SC_ERR_STATE, "every plan needs sc_factor and sc_set_base"};
      if (P->prof_on) throw Fail{SC_ERR_STATE, "turn the stage profiler off before a batch call"};
    }
    hipStream_t s = (hipStream_t)stream;
    // the branches fork from and join into `origin`
    auto enqueue = [&](hipStream_t origin) {
      HIPCHK(hipEventRecord(b->ev_start, origin));
      for (int i = 0; i < n; ++i) {
        if (nvec[i] == 0) continue;
        HIPCHK(hipStreamWaitEvent(b->br[i], b->ev_start, 0));
        jvp_impl(b->plans[i], nvec[i], v[i], b->plans[i]->n_real, y[i], b->plans[i]->n_real, prec, b->br[i]);
        HIPCHK(hipEventRecord(b->ev_done[i], b->br[i]));
        HIPCHK(hipStreamWaitEvent(origin, b->ev_done[i], 0));
      }
    };
    bool graphs = true;
    for (int i = 0; i < n; ++i) graphs = graphs && b->plans[i]->prm.graph_capture;
    if (!graphs) {
      enqueue(s);
      return;
    }
    std::vector<unsigned long long> ep(n);
    for (int i = 0; i < n; ++i) ep[i] = b->plans[i]->graph_epoch;
    if (ep != b->epochs) {
      b->drop_graphs();
      b->epochs = ep;
    }
    std::vector<long long> key{(long long)prec};
    for (int i = 0; i < n; ++i) {
      key.push_back(nvec[i]);
      key.push_back((long long)(uintptr_t)v[i]);
      key.push_back((long long)(uintptr_t)y[i]);
    }
    hipGraphExec_t ex;
    auto it = b->graphs.find(key);
    if (it != b->graphs.end()) {
      ex = it->second;
    } else {
      ex = capture_graph(b->cap, enqueue);
      b->graphs[key] = ex;
    }
    launch_graph(ex, b->cap, b->ev_gin, b->ev_gout, s);
  });
}

int sc_batch_newton(sc_batch* b, double* const* x, double* C, const sc_newton_opts* opts, sc_newton_report* reps,
                    void* stream) {
  return guarded([&] {
    if (!b || !x || !C || !opts || !reps) throw Fail{SC_ERR_ARG, "null argument"};
    HIPCHK(hipSetDevice(b->device));
    const int n = (int)b->plans.size();
    std::vector<long long> J(n);
    for (int i = 0; i < n; ++i) {
      sc_plan* P = b->plans[i];
      const sc_newton_opts& o = opts[i];
      if (!x[i]) throw Fail{SC_ERR_ARG, "null state"};
      if (o.restart < 1 || o.restart > 1024) throw Fail{SC_ERR_ARG, "restart must lie in 1..1024"};
      if (o.max_newton < 0 || o.max_newton > 64 || o.max_matvec < 1) throw Fail{SC_ERR_ARG, "bad iteration caps"};
      if (o.prec != SC_FP64 && o.prec != SC_MIXED) throw Fail{SC_ERR_ARG, "unknown precision"};
      if (!P->factored) throw Fail{SC_ERR_STATE, "every plan needs sc_factor for its current (Ek, dt)"};
      if (P->prof_on) throw Fail{SC_ERR_STATE, "turn the stage profiler off before a batch call"};
      J[i] = check_slot(P, o.J);
    }
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipEventRecord(b->ev_start, s));
    for (int i = 0; i < n; ++i) HIPCHK(hipStreamWaitEvent(b->br[i], b->ev_start, 0));
    // one host thread per plan: each Newton-GMRES reads its norms back on its own branch
    std::vector<int> code(n, SC_OK);
    std::vector<std::string> msg(n);
    std::vector<std::thread> th;
    for (int i = 0; i < n; ++i)
      th.emplace_back([&, i] {
        try {
          HIPCHK(hipSetDevice(b->device));
          newton_impl(b->plans[i], x[i], &C[i], opts[i], J[i], &reps[i], b->br[i]);
        } catch (const Fail& f) {
          code[i] = f.code;
          msg[i] = f.msg;
        } catch (const std::exception& e) {
          code[i] = SC_ERR_INTERNAL;
          msg[i] = e.what();
        }
      });
    for (auto& t : th) t.join();
    for (int i = 0; i < n; ++i) {
      HIPCHK(hipEventRecord(b->ev_done[i], b->br[i]));
      HIPCHK(hipStreamWaitEvent(s, b->ev_done[i], 0));
    }
    for (int i = 0; i < n; ++i)
      if (code[i] != SC_OK) throw Fail{code[i], "plan " + std::to_string(i) + ": " + msg[i]};
  });
}

}  // extern "C"

// ==========================================================================================
// Grid refinement and continuation (Sec. 3.5, 3.6, 4.2).
namespace {

constexpr double kPiD = 3.14159265358979323846;

// Interpolation matrix [N_new][N_old]: the interpolating polynomial of N_old Gauss-Lobatto values
// (its discrete Chebyshev series) evaluated at the N_new Gauss-Lobatto nodes.
std::vector<double> cheb_interp_matrix(int No, int Nn) {
  std::vector<double> Cm((size_t)No * No);   // [k][j]: Chebyshev coefficient k of nodal value j
  for (int k = 0; k < No; ++k)
    for (int j = 0; j < No; ++j) {
      const double ck = (k == 0 || k == No - 1) ? 2.0 : 1.0, cj = (j == 0 || j == No - 1) ? 2.0 : 1.0;
      Cm[(size_t)k * No + j] = 2.0 / ((No - 1) * ck * cj) * std::cos(kPiD * k * j / (No - 1));
    }
  std::vector<double> Ip((size_t)Nn * No, 0.0);
  for (int i = 0; i < Nn; ++i)
    for (int k = 0; k < No; ++k) {
      const double Tk = std::cos(k * kPiD * i / (Nn - 1));   // T_k at x_i = cos(pi i/(Nn - 1))
      for (int j = 0; j < No; ++j) Ip[(size_t)i * No + j] += Tk * Cm[(size_t)k * No + j];
    }
  return Ip;
}

void interp_device(sc_plan* from, const double* x, sc_plan* to, double* y, hipStream_t s) {
  if (from->hg.m0 != to->hg.m0) throw Fail{SC_ERR_ARG, "interpolation keeps the sector: m0 must match"};
  if (from->prm.device != to->prm.device) throw Fail{SC_ERR_ARG, "plans on different devices"};
  DevBuf Ip;
  upload(Ip, cheb_interp_matrix(from->hg.N, to->hg.N));
  sc::InterpMap im;
  im.N_old = from->hg.N;
  im.N_new = to->hg.N;
  im.S_old = from->hg.S;
  im.S_new = to->hg.S;
  im.L_old = from->hg.L;
  im.K_old = from->hg.K;
  im.m0 = from->hg.m0;
  im.lmbase_old = from->d_lmbase.as<int>();
  im.lm_k_new = to->d_lmk.as<int>();
  im.lm_l_new = to->d_lml.as<int>();
  im.Ip = Ip.as<double>();
  hipLaunchKernelGGL(sc::k_interp, dim3(nblk(to->n_real, 256)), dim3(256), 0, s, im, x, y);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));   // Ip is freed on return
}

// Tail ratios of a host copy of a packed state: max |a_{N-1}| / max |a_n| over the Chebyshev
// coefficients of every radial profile, and max |X at l = L| / max |X| (complex magnitudes).
void tail_ratios_host(const sc_plan* P, const std::vector<double>& X, double& rc, double& rl) {
  const sc::HostGrid& g = P->hg;
  const int N = g.N;
  std::vector<double> Cm((size_t)N * N);
  for (int k = 0; k < N; ++k)
    for (int j = 0; j < N; ++j) {
      const double ck = (k == 0 || k == N - 1) ? 2.0 : 1.0, cj = (j == 0 || j == N - 1) ? 2.0 : 1.0;
      Cm[(size_t)k * N + j] = 2.0 / ((N - 1) * ck * cj) * std::cos(kPiD * k * j / (N - 1));
    }
  double amax = 0.0, atail = 0.0, xmax = 0.0, xl = 0.0;
  for (int f = 0; f < 3; ++f)
    for (int lm = 0; lm < g.S; ++lm) {
      const double* v = X.data() + 2LL * ((long long)N * ((long long)f * g.S + lm));
      const bool top = g.lm_l[lm] == g.L;
      for (int j = 0; j < N; ++j) {
        const double a = std::hypot(v[2 * j], v[2 * j + 1]);
        xmax = std::max(xmax, a);
        if (top) xl = std::max(xl, a);
      }
      for (int k = 0; k < N; ++k) {
        double re = 0.0, im = 0.0;
        for (int j = 0; j < N; ++j) {
          re += Cm[(size_t)k * N + j] * v[2 * j];
          im += Cm[(size_t)k * N + j] * v[2 * j + 1];
        }
        const double a = std::hypot(re, im);
        amax = std::max(amax, a);
        if (k == N - 1) atail = std::max(atail, a);
      }
    }
  rc = amax > 0 ? atail / amax : 0.0;
  rl = xmax > 0 ? xl / xmax : 0.0;
}

// Phase slot on a host copy: the Im entry of an m = m0 coefficient of f or T whose real part is
// largest in magnitude (-1 if the plan has no m > 0).
long long phase_slot_host(const sc_plan* P, const std::vector<double>& X) {
  const sc::HostGrid& g = P->hg;
  if (g.K < 1) return -1;
  long long best = -1;
  double bv = -1.0;
  for (int f = 1; f <= 2; ++f)
    for (int l = g.ms[1]; l <= g.L; ++l) {
      const int lm = g.lmbase[1] + (l - g.ms[1]);
      for (int j = 0; j < g.N; ++j) {
        const long long o = 2LL * ((long long)g.N * ((long long)f * g.S + lm) + j);
        if (std::fabs(X[o]) > bv) {
          bv = std::fabs(X[o]);
          best = o + 1;
        }
      }
    }
  return best;
}

std::vector<double> to_host(const double* x, long long n, hipStream_t s) {
  std::vector<double> h((size_t)n);
  HIPCHK(hipMemcpyAsync(h.data(), x, n * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return h;
}

double read1(const double* x, long long i, hipStream_t s) {
  double v = 0.0;
  HIPCHK(hipMemcpyAsync(&v, x + i, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return v;
}

// Index of the largest |x| (device reduction in fixed chunks, ties to the lower index).
long long argmax_abs(const double* x, long long n, hipStream_t s) {
  const long long chunk = 8192, nparts = (n + chunk - 1) / chunk;
  DevBuf pv, pi;
  pv.alloc(nparts * sizeof(double));
  pi.alloc(nparts * sizeof(long long));
  hipLaunchKernelGGL(sc::k_absmax_parts, dim3((unsigned)nparts), dim3(256), 0, s, n, x, chunk, pv.as<double>(),
                     pi.as<long long>());
  HIPCHK(hipGetLastError());
  std::vector<double> hv(nparts);
  std::vector<long long> hi(nparts);
  HIPCHK(hipMemcpyAsync(hv.data(), pv.p, nparts * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(hi.data(), pi.p, nparts * sizeof(long long), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  long long best = 0;
  double bv = -1.0;
  for (long long b = 0; b < nparts; ++b)
    if (hv[b] > bv) {
      bv = hv[b];
      best = hi[b];
    }
  return best;
}

double lagrange_w(double t, const double* ts, int n, int q) {
  double v = 1.0;
  for (int r = 0; r < n; ++r)
    if (r != q) v *= (t - ts[r]) / (ts[q] - ts[r]);
  return v;
}

}  // namespace

struct sc_cont {
  sc_plan* plan = nullptr;      // the plan of the current resolution
  sc_plan* owned = nullptr;     // a plan made by a refinement (owned by the session)
  sc_cont_opts o{};
  long long J = -1;             // phase slot in the current layout
  int n = 0;                    // converged points kept (<= 3), oldest first
  DevBuf X[3];
  double p[3] = {0, 0, 0}, C[3] = {0, 0, 0};
  int its[3] = {0, 0, 0};
  DevBuf trial;

  ~sc_cont() {
    if (owned) {
      (void)hipSetDevice(owned->prm.device);
      (void)hipDeviceSynchronize();
      delete owned;
    }
  }
  // parameters of the plan at continuation parameter value q (a new Ek re-factors: Sec. 4.2)
  void apply(double q, hipStream_t s) {
    if (o.param == SC_CONT_RA) {
      if (sc_set_params(plan, q, plan->prm.Ek, plan->prm.dt) != SC_OK) throw Fail{SC_ERR_ARG, g_last_error};
    } else {
      const double Ek = std::pow(10.0, q), Ra = o.ra_coef * std::pow(Ek, -1.0 / 3.0);
      if (sc_set_params(plan, Ra, Ek, plan->prm.dt) != SC_OK) throw Fail{SC_ERR_ARG, g_last_error};
      if (!plan->factored) {
        HIPCHK(hipStreamSynchronize(s));   // the factor buffers are replaced
        if (sc_factor(plan, s) != SC_OK) throw Fail{SC_ERR_HIP, g_last_error};
      }
    }
  }
  double param_of_plan() const {
    return o.param == SC_CONT_RA ? plan->prm.Ra : std::log10(plan->prm.Ek);
  }
  // Newton at parameter q from the iterate in x (in place); false if it did not converge
  bool solve(double q, double* x, double& Cq, sc_newton_report& rep, hipStream_t s) {
    apply(q, s);
    sc_newton_opts no = o.newton;
    no.J = J;
    try {
      newton_impl(plan, x, &Cq, no, J, &rep, s);
    } catch (const Fail& f) {
      if (f.code != SC_ERR_NONFINITE) throw;
      return false;
    }
    return rep.converged != 0;
  }
  void push(double q, const double* x, double Cq, int nits, hipStream_t s) {
    if (n == 3) {
      std::swap(X[0].p, X[1].p);
      std::swap(X[1].p, X[2].p);
      p[0] = p[1]; p[1] = p[2];
      C[0] = C[1]; C[1] = C[2];
      its[0] = its[1]; its[1] = its[2];
      n = 2;
    }
    HIPCHK(hipMemcpyAsync(X[n].p, x, plan->n_real * sizeof(double), hipMemcpyDeviceToDevice, s));
    p[n] = q;
    C[n] = Cq;
    its[n] = nits;
    ++n;
  }
};

extern "C" {

int sc_interpolate(sc_plan* from, const double* x, sc_plan* to, double* y, void* stream) {
  return guarded([&] {
    check_plan(from);
    if (!to || !x || !y) throw Fail{SC_ERR_ARG, "null argument"};
    interp_device(from, x, to, y, (hipStream_t)stream);
  });
}

int sc_tail_ratios(sc_plan* P, const double* x, double* cheb_ratio, double* sh_ratio, void* stream) {
  return guarded([&] {
    check_plan(P);
    if (!x || !cheb_ratio || !sh_ratio) throw Fail{SC_ERR_ARG, "null argument"};
    const std::vector<double> h = to_host(x, P->n_real, (hipStream_t)stream);
    tail_ratios_host(P, h, *cheb_ratio, *sh_ratio);
  });
}

int sc_cont_create(sc_cont** out, sc_plan* plan, const double* x0, double C0, const sc_cont_opts* opts,
                   sc_cont_point* first, void* stream) {
  if (!out || !plan || !x0 || !opts) return fail(SC_ERR_ARG, "null argument");
  *out = nullptr;
  return guarded([&] {
    check_plan(plan);
    const sc_cont_opts& o = *opts;
    if (o.param != SC_CONT_RA && o.param != SC_CONT_EK) throw Fail{SC_ERR_ARG, "param must be SC_CONT_RA or SC_CONT_EK"};
    if (o.n_opt < 1 || !(o.gamma > 0) || o.max_retries < 0 || o.max_retries > 16)
      throw Fail{SC_ERR_ARG, "need n_opt >= 1, gamma > 0, 0 <= max_retries <= 16"};
    if (o.param == SC_CONT_EK && !(o.ra_coef > 0)) throw Fail{SC_ERR_ARG, "SC_CONT_EK needs ra_coef > 0"};
    if (o.refine_tol > 0 && !(o.refine_growth > 1.0)) throw Fail{SC_ERR_ARG, "refine_growth must exceed 1"};
    if (o.newton.restart < 1 || o.newton.restart > 1024 || o.newton.max_newton < 0 || o.newton.max_newton > 64 ||
        o.newton.max_matvec < 1 || (o.newton.prec != SC_FP64 && o.newton.prec != SC_MIXED))
      throw Fail{SC_ERR_ARG, "bad Newton options"};
    if (o.newton.forcing) throw Fail{SC_ERR_ARG, "a continuation takes no forcing"};
    if (!plan->factored) throw Fail{SC_ERR_STATE, "sc_factor has not run for the current (Ek, dt)"};
    if (plan->prof_on) throw Fail{SC_ERR_STATE, "turn the stage profiler off before a continuation"};
    hipStream_t s = (hipStream_t)stream;
    std::unique_ptr<sc_cont> c(new sc_cont());
    c->plan = plan;
    c->o = o;
    c->J = check_slot(plan, o.newton.J);
    for (auto& b : c->X) b.alloc(plan->n_real * sizeof(double));
    c->trial.alloc(plan->n_real * sizeof(double));
    HIPCHK(hipMemcpyAsync(c->trial.p, x0, plan->n_real * sizeof(double), hipMemcpyDeviceToDevice, s));
    // the first point: converged at the plan's current parameters (Newton from x0)
    const double q0 = c->param_of_plan();
    double Cq = C0;
    sc_newton_report rep;
    const bool ok = c->solve(q0, c->trial.as<double>(), Cq, rep, s);
    if (!ok) throw Fail{SC_ERR_STATE, "Newton did not converge at the first point"};
    c->push(q0, c->trial.as<double>(), Cq, rep.newton_steps, s);
    HIPCHK(hipStreamSynchronize(s));
    if (first) {
      std::memset(first, 0, sizeof(*first));
      first->param = q0;
      first->Ra = plan->prm.Ra;
      first->Ek = plan->prm.Ek;
      first->C = Cq;
      first->unorm = norm2(plan, c->X[0].as<double>(), s);
      first->newton_steps = rep.newton_steps;
      first->matvecs = rep.matvecs;
      first->converged = 1;
      first->L = plan->hg.L;
      first->N = plan->hg.N;
    }
    *out = c.release();
  });
}

int sc_cont_step(sc_cont* c, double dp_first, sc_cont_point* pt, void* stream) {
  return guarded([&] {
    if (!c || !pt) throw Fail{SC_ERR_ARG, "null argument"};
    check_plan(c->plan);
    if (c->n == 1 && !(dp_first != 0.0 && std::isfinite(dp_first)))
      throw Fail{SC_ERR_ARG, "the first step needs a nonzero dp_first"};
    hipStream_t s = (hipStream_t)stream;
    const long long n = c->plan->n_real;
    std::memset(pt, 0, sizeof(*pt));
    double* xt = c->trial.as<double>();
    for (int r = 0; r <= c->o.max_retries; ++r) {
      const double scale = std::ldexp(1.0, -r);
      double q, Cq, w[3] = {0, 0, 0};
      bool state_mode = false;
      const int k = c->n;                       // points used by the prediction (1..3)
      if (k == 1) {
        q = c->p[0] + scale * dp_first;
        w[0] = 1.0;
      } else {
        const double alpha = scale * (c->o.n_opt + 1.0) / (std::max(c->its[k - 1], 1) + 1.0);
        // turning-point test on the last two points (eq:tp_detection_Ra)
        const long long Jt = argmax_abs(c->X[k - 1].as<double>(), n, s);
        double u[3];
        for (int i = 0; i < k; ++i) u[i] = read1(c->X[i].as<double>(), Jt, s);
        const double dU = std::fabs((u[k - 1] - u[k - 2]) / u[k - 1]);
        const double dP = std::fabs((c->p[k - 1] - c->p[k - 2]) / c->p[k - 1]);
        state_mode = dU > scale * c->o.gamma * dP;
        if (!state_mode) {
          q = c->p[k - 1] + alpha * (c->p[k - 1] - c->p[k - 2]);
          for (int i = 0; i < k; ++i) w[i] = lagrange_w(q, c->p, k, i);
        } else {
          const double un = u[k - 1] + alpha * (u[k - 1] - u[k - 2]);
          q = 0.0;
          for (int i = 0; i < k; ++i) {
            w[i] = lagrange_w(un, u, k, i);
            q += w[i] * c->p[i];
          }
        }
      }
      Cq = 0.0;
      for (int i = 0; i < k; ++i) Cq += w[i] * c->C[i];
      const double* x1 = c->X[k > 1 ? 1 : 0].as<double>();
      const double* x2 = c->X[k > 2 ? 2 : 0].as<double>();
      hipLaunchKernelGGL(sc::k_lincomb3, dim3(nblk(n, 256)), dim3(256), 0, s, n, w[0], c->X[0].as<const double>(),
                         w[1], x1, w[2], x2, xt);
      HIPCHK(hipGetLastError());
      sc_newton_report rep;
      const bool ok = c->solve(q, xt, Cq, rep, s);
      pt->retries = r;
      pt->newton_steps = rep.newton_steps;
      pt->matvecs += rep.matvecs;
      pt->param = q;
      if (!ok) continue;
      c->push(q, xt, Cq, rep.newton_steps, s);
      pt->converged = 1;
      pt->state_mode = state_mode ? 1 : 0;
      break;
    }
    if (pt->converged && c->o.param == SC_CONT_EK && c->o.refine_tol > 0) {
      // under-resolution check on the new point (Sec. 4.2): grow N and/or L, M by refine_growth
      const std::vector<double> h = to_host(c->X[c->n - 1].as<double>(), n, s);
      double rc = 0, rl = 0;
      tail_ratios_host(c->plan, h, rc, rl);
      pt->cheb_ratio = rc;
      pt->sh_ratio = rl;
      const sc::HostGrid& g = c->plan->hg;
      sc_params np = c->plan->prm;
      np.nr_phys = np.ntheta = np.nphi = 0;
      if (rc > c->o.refine_tol) np.N = std::min(64, (int)std::ceil(c->o.refine_growth * g.N));
      if (rl > c->o.refine_tol) {
        np.L = (int)std::ceil(c->o.refine_growth * g.L);
        np.M = (int)std::ceil(c->o.refine_growth * g.M);
      }
      if (np.N != g.N || np.L != g.L) {
        sc_plan* fine = nullptr;
        if (sc_plan_create(&fine, &np) != SC_OK) throw Fail{SC_ERR_ARG, "refinement: " + g_last_error};
        std::unique_ptr<sc_plan> guard(fine);
        if (sc_factor(fine, s) != SC_OK) throw Fail{SC_ERR_HIP, "refinement: " + g_last_error};
        // carry the kept points to the new grid
        DevBuf Xn[3], tn;
        for (int i = 0; i < 3; ++i) Xn[i].alloc(fine->n_real * sizeof(double));
        tn.alloc(fine->n_real * sizeof(double));
        for (int i = 0; i < c->n; ++i) interp_device(c->plan, c->X[i].as<double>(), fine, Xn[i].as<double>(), s);
        sc_plan* coarse = c->plan;
        c->plan = fine;
        for (int i = 0; i < 3; ++i) {
          std::swap(c->X[i].p, Xn[i].p);
          std::swap(c->X[i].bytes, Xn[i].bytes);
        }
        std::swap(c->trial.p, tn.p);
        std::swap(c->trial.bytes, tn.bytes);
        c->J = phase_slot_host(fine, to_host(c->X[c->n - 1].as<double>(), fine->n_real, s));
        // recompute the newest point on the new grid
        HIPCHK(hipMemcpyAsync(c->trial.p, c->X[c->n - 1].p, fine->n_real * sizeof(double), hipMemcpyDeviceToDevice, s));
        double Cq = c->C[c->n - 1];
        sc_newton_report rep;
        if (!c->solve(c->p[c->n - 1], c->trial.as<double>(), Cq, rep, s))
          throw Fail{SC_ERR_STATE, "refinement: Newton did not converge on the refined grid"};
        HIPCHK(hipMemcpyAsync(c->X[c->n - 1].p, c->trial.p, fine->n_real * sizeof(double), hipMemcpyDeviceToDevice, s));
        c->C[c->n - 1] = Cq;
        pt->matvecs += rep.matvecs;
        pt->refined = 1;
        HIPCHK(hipStreamSynchronize(s));
        guard.release();
        if (c->owned) delete c->owned;   // the previous refined plan (never the caller's)
        c->owned = fine;
        (void)coarse;
      }
    }
    if (pt->converged) {
      pt->C = c->C[c->n - 1];
      pt->Ra = c->plan->prm.Ra;
      pt->Ek = c->plan->prm.Ek;
      pt->unorm = norm2(c->plan, c->X[c->n - 1].as<double>(), s);
      pt->L = c->plan->hg.L;
      pt->N = c->plan->hg.N;
    }
  });
}

int sc_cont_layout(const sc_cont* c, sc_layout_info* out) {
  if (!c) return fail(SC_ERR_ARG, "null session");
  return sc_layout(c->plan, out);
}

int sc_cont_state(sc_cont* c, double* x, long long n, double* C, void* stream) {
  return guarded([&] {
    if (!c || !x || !C) throw Fail{SC_ERR_ARG, "null argument"};
    check_plan(c->plan);
    if (n != c->plan->n_real) throw Fail{SC_ERR_ARG, "n must equal the current n_real (sc_cont_layout)"};
    HIPCHK(hipMemcpyAsync(x, c->X[c->n - 1].p, n * sizeof(double), hipMemcpyDeviceToDevice, (hipStream_t)stream));
    *C = c->C[c->n - 1];
  });
}

int sc_cont_destroy(sc_cont* c) {
  delete c;
  return SC_OK;
}

}  // extern "C"
