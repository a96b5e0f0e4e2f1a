// Host engine shared by the translation units of the fgcg library: the
// context and its workspace, error reporting, kernel launches (plain or as
// graph nodes), the chunked CG driver and argument checks.
#pragma once
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "fgcg.h"
#include "mech_u.hpp"
#include "pointwise.hpp"
#include "scalar_cg.hpp"

namespace fgcg {

inline thread_local std::string g_err;

inline int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess) return fail(FGCG_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <typename T> using CT = typename cvec<T>::type;

// Supported axis lengths (2^a 3^b).  Each length instantiates the pass kernels.
#define FGCG_SIZES(X) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024) X(2048)

template <class F> bool with_n(int n, F&& f) {
  switch (n) {
#define FGCG_CASE(N)                       \
  case N:                                  \
    f(std::integral_constant<int, N>{});   \
    return true;
    FGCG_SIZES(FGCG_CASE)
#undef FGCG_CASE
    default:
      return false;
  }
}

inline bool size_supported(int n) {
  return with_n(n, [](auto) {});
}

}  // namespace fgcg

struct fgcg_ctx {
  int ndim = 2;
  int nx = 0, ny = 0, nz = 1, nxh = 0;
  int rows = 0;  // rows of the x-direction passes: ny (2D) or ny nz (3D)
  long long n = 0;
  double h = 0;
  int prec = FGCG_FP64;
  hipStream_t stream = nullptr;       // context-owned stream: every launch goes here
  bool own_stream = true;             // false for the groups of a batch after the first
  hipStream_t user_stream = nullptr;  // caller's stream; work on it is waited for at entry
  hipEvent_t ev_in = nullptr;
  hipEvent_t ev_done[2] = {nullptr, nullptr};
  bool use_graphs = true;
  bool building = false;            // launches become nodes of `graph`
  bool build_timed = false;         // add event-record nodes while building
  hipGraph_t graph = nullptr;
  hipGraphNode_t last = nullptr;
  int chunk = 16;  // CG iterations per captured graph
  void* twx = nullptr;    // double2[nx] twiddles
  void* twy = nullptr;    // double2[ny]
  void* twx32 = nullptr;  // float2[nx] (FP32-mixed contexts)
  void* twy32 = nullptr;  // float2[ny]
  double* xh = nullptr;   // FP32-mixed: FP64 solution (2 components)
  double* fh = nullptr;   // FP32-mixed: FP64 right-hand side (2 components)
  double* aux = nullptr;  // adjoint: forward strain (3 components) and dJ/deps (3 components)
  double2* Dx = nullptr;
  double2* Dy = nullptr;
  double2* Dz = nullptr;  // 3D
  void* twz = nullptr;    // 3D: double2[nz] twiddles
  void* twz32 = nullptr;  // 3D FP32-mixed: float2[nz]
  double* red = nullptr;  // 3D: device [8] partial sums reduced by a single block
  double* part_z = nullptr;  // 3D: partial sums of the z pass (one per block)
  int nzb = 0;               // 3D: partial-sum slots of the z pass (its most blocks: one tile per block)
  int zpt_pick = 0;          // 3D: z tiles per block of the z pass, 1 or 2 (0: tune before the next solve)
  int split3 = 0;            // 3D: 1 + (forward row pass split) + 2 (inverse split); 0: tune
  int nslab = 0;             // 3D: blocks of the stencil kernels
  void* x = nullptr;
  void* r = nullptr;
  void* p = nullptr;
  void* tmp = nullptr;
  void* spec = nullptr;
  fgcg::CgState* st = nullptr;
  fgcg::CgState* h_st = nullptr;
  dim3 sgrid;                 // grid of the stencil CG passes (8..512 blocks, a multiple of 8)
  int scalar_spectral = 0;    // 1: phase field and diffusion apply their operators by FFT
  double* part_a = nullptr;
  double* part_rr = nullptr;
  double* part_b = nullptr;
  double* part_post = nullptr;
  double* h_part = nullptr;
  int nrow = 0, ncol = 0, npost = 0, nkp = 0;
  int nkpt = 0;  // blocks of the tiled 2D stiffness pass (one partial sum each)
  int rows_pick = 0;  // 2D mechanics row passes: rows per block (0: time the candidates at the next solve)
  // 2D mechanics radix plans (1: plan 0, radix 8; 2: plan 1, radix 16; 0: time both at the next solve)
  int plan_row = 0, plan_col = 0;
  int precond = 0;          // mechanics preconditioner: 0 unit Green operator, 1 isotropic reference medium
  int gradop = 0;           // gradient operator: 0 forward, 1 central, 2 eighth-order central, 3 Fourier
  int strain_form = 0;      // 1: mechanics and homogenisation in the paper's strain / gradient form
  int sr_opt = 1;           // 1: the residual-spectrum mechanics PCG where it applies (sr_active)
  int sr_pick = 0;          // tuned form: 0 not decided, 1 residual spectrum (three passes), 2 four
                            // passes, 3 residual spectrum with the row stage fused (two passes)
  int kp_both = 1;          // residual-spectrum stiffness pass: 1 both components per block, 0 one
  int scg_onered = 1;       // stencil scalar CG on 2D grids: 1 one-reduction form (one pass), 0 textbook
  double* timing_E = nullptr;  // E = 1 field of the iteration timings (tuner), allocated on first use
  void* rhat = nullptr;     // residual-spectrum PCG: the residual's half spectra [nsamp][2][nxh][ny]
  void* p_odd = nullptr;    // two-pass form: the direction of odd iterations (p holds the even ones)
  void* spec_q = nullptr;   // two-pass form: the x spectra of K p [nsamp][2][nxh][ny]
  double* sf_buf = nullptr; // strain form: x, r, p (3 components each), allocated with the option
  void* sf_spec = nullptr;  // strain form: 3 half spectra
  double ref_lam = 0, ref_mu = 0;  // reference medium set by the caller (0, 0: from the material)
  double use_lam = 0, use_mu = 0;  // reference medium of the current solve (mu = 1)
  int nsamp = 1;            // samples of this grid size (batches)
  int ncw = 2;              // components of the x, r, p, tmp and spectrum workspace (2D: 2, 3D: 3)
  double* lm_dev = nullptr; // batches: per-sample Lame tables [nsamp][16]
  double* ems = nullptr;    // device [nsamp][3] macro strains
  bool batch = false;            // member of a batch (owns the gather buffers below)
  uint8_t* phase_buf = nullptr;  // batches: gathered phase fields [nsamp][N]
  double* strain_buf = nullptr;  // batches: strains [nsamp][3][N]
  unsigned prof_mask = 0;
  double prof_ms[FGCG_K_NKINDS] = {0};
  long long prof_n[FGCG_K_NKINDS] = {0};
  std::string kname[FGCG_K_NKINDS];
  std::vector<hipEvent_t> pool;
  struct Pending {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  hipEvent_t cur = nullptr;
  struct GraphSlot {
    hipGraphExec_t exec = nullptr;
    std::vector<Pending> ev;  // timing events recorded inside this instance
  };
  struct CgGraph {
    std::vector<char> key;
    GraphSlot slot[2];
  };
  // chunk graphs per solver: 0 mechanics, 1 phase field (spectral), 2 diffusion
  // (spectral), 3 phase field, 4 diffusion (phase tables), 5 mechanics
  // FP32-mixed, 6 diffusion (per-voxel fields), 7 diffusion homogenisation,
  // 8-11 spare
  CgGraph graphs[12];
};

namespace fgcg {

inline int prof_begin(fgcg_ctx* c, int kind) {
  if (!(c->prof_mask & (1u << kind))) return 0;
  if (c->pool.size() < 2) {
    for (int i = 0; i < 64; ++i) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      c->pool.push_back(e);
    }
  }
  c->cur = c->pool.back();
  c->pool.pop_back();
  HIPCHK(hipEventRecord(c->cur, c->stream));
  return 0;
}

inline int prof_end(fgcg_ctx* c, int kind) {
  if (!(c->prof_mask & (1u << kind))) return 0;
  hipEvent_t e = c->pool.back();
  c->pool.pop_back();
  HIPCHK(hipEventRecord(e, c->stream));
  c->pending.push_back({kind, c->cur, e});
  return 0;
}

// Call after the stream has been synchronised.
inline int prof_flush(fgcg_ctx* c) {
  for (auto& p : c->pending) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, p.a, p.b));
    c->prof_ms[p.kind] += ms;
    c->prof_n[p.kind] += 1;
    c->pool.push_back(p.a);
    c->pool.push_back(p.b);
  }
  c->pending.clear();
  return 0;
}

inline int prof_reserve(fgcg_ctx* c, size_t n) {
  while (c->pool.size() < n) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    c->pool.push_back(e);
  }
  return 0;
}

inline int prof_read_slot(fgcg_ctx* c, fgcg_ctx::GraphSlot& sl) {
  for (auto& p : sl.ev) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, p.a, p.b));
    c->prof_ms[p.kind] += ms;
    c->prof_n[p.kind] += 1;
  }
  return 0;
}

inline void release_graph(fgcg_ctx* c, fgcg_ctx::CgGraph& g) {
  for (auto& sl : g.slot) {
    if (sl.exec) (void)hipGraphExecDestroy(sl.exec);
    sl.exec = nullptr;
    for (auto& p : sl.ev) {
      c->pool.push_back(p.a);
      c->pool.push_back(p.b);
    }
    sl.ev.clear();
  }
  g.key.clear();
}

inline int enter(fgcg_ctx* c) {
  HIPCHK(hipEventRecord(c->ev_in, c->user_stream));
  HIPCHK(hipStreamWaitEvent(c->stream, c->ev_in, 0));
  return 0;
}

// Byte key of the values an iteration chunk was captured with.
struct Key {
  std::vector<char> b;
  template <typename V> Key& add(const V& v) {
    const char* p = reinterpret_cast<const char*>(&v);
    b.insert(b.end(), p, p + sizeof(V));
    return *this;
  }
};

template <typename T> const CT<T>* tw_x(const fgcg_ctx* c) {
  return (const CT<T>*)(std::is_same<T, double>::value ? c->twx : c->twx32);
}
template <typename T> const CT<T>* tw_y(const fgcg_ctx* c) {
  return (const CT<T>*)(std::is_same<T, double>::value ? c->twy : c->twy32);
}

template <typename T> const char* tname() { return std::is_same<T, double>::value ? "double" : "float"; }

inline void set_kname(fgcg_ctx* c, int kind, const char* fmt, const char* t, int n) {
  if (!c->kname[kind].empty()) return;
  char b[256];
  snprintf(b, sizeof b, fmt, t, n);
  c->kname[kind] = b;
}

// One launch: a plain stream launch (timed with events when its kind is
// profiled), or, while a chunk graph is being built, a kernel node appended to
// the chain (between two event-record nodes when profiled).
template <typename... A>
int launch_b(fgcg_ctx* c, int kind, const void* fn, dim3 grid, dim3 block, A... args) {
  void* ptrs[] = {(void*)&args...};
  const bool prof = kind >= 0 && (c->prof_mask & (1u << kind)) && (!c->building || c->build_timed);
  if (!c->building) {
    int rc = prof ? prof_begin(c, kind) : 0;
    if (rc) return rc;
    HIPCHK(hipLaunchKernel(fn, grid, block, ptrs, 0, c->stream));
    return prof ? prof_end(c, kind) : 0;
  }
  hipEvent_t ea = nullptr, eb = nullptr;
  if (prof) {
    ea = c->pool.back();
    c->pool.pop_back();
    eb = c->pool.back();
    c->pool.pop_back();
    hipGraphNode_t n;
    HIPCHK(hipGraphAddEventRecordNode(&n, c->graph, c->last ? &c->last : nullptr, c->last ? 1 : 0, ea));
    c->last = n;
  }
  hipKernelNodeParams kp{};
  kp.func = const_cast<void*>(fn);
  kp.gridDim = grid;
  kp.blockDim = block;
  kp.sharedMemBytes = 0;
  kp.kernelParams = ptrs;
  kp.extra = nullptr;
  hipGraphNode_t kn;
  HIPCHK(hipGraphAddKernelNode(&kn, c->graph, c->last ? &c->last : nullptr, c->last ? 1 : 0, &kp));
  c->last = kn;
  if (prof) {
    hipGraphNode_t n;
    HIPCHK(hipGraphAddEventRecordNode(&n, c->graph, &c->last, 1, eb));
    c->last = n;
    c->pending.push_back({kind, ea, eb});
  }
  return 0;
}

template <typename... A> int launch(fgcg_ctx* c, int kind, const void* fn, dim3 grid, A... args) {
  return launch_b(c, kind, fn, grid, dim3(NT), args...);
}

// Rows per block of the tunable row passes: rows_for(NX) times 1/2, 1 or 2,
// even, 2..16 and at most 4096 voxels per block (rows_for itself always).
constexpr bool rows_ok(int NX, int R) {
  return R == rows_for(NX) || (R >= 2 && R % 2 == 0 && R <= 16 && R * NX <= 4096);
}

template <int NX> inline std::vector<int> rows_candidates() {
  constexpr int R0 = rows_for(NX);
  std::vector<int> v;
  if (rows_ok(NX, R0 / 2)) v.push_back(R0 / 2);
  v.push_back(R0);
  if (rows_ok(NX, 2 * R0)) v.push_back(2 * R0);
  return v;
}

// Calls f(integral_constant<int, R>) with R = pick if it is a candidate, else
// the default rows_for(NX).
template <int NX, class F> void with_rows(int pick, F&& f) {
  constexpr int R0 = rows_for(NX);
  if constexpr (R0 / 2 != R0 && rows_ok(NX, R0 / 2)) {
    if (pick == R0 / 2) {
      f(std::integral_constant<int, R0 / 2>{});
      return;
    }
  }
  if constexpr (rows_ok(NX, 2 * R0)) {
    if (pick == 2 * R0) {
      f(std::integral_constant<int, 2 * R0>{});
      return;
    }
  }
  f(std::integral_constant<int, R0>{});
}

// Calls f(integral_constant<int, P>) with the radix plan of a pick (2: plan 1
// where it differs from plan 0 for length N; anything else: plan 0).
template <int N, class F> void with_plan(int pick, F&& f) {
  if constexpr (plan1_differs(N)) {
    if (pick == 2) {
      f(std::integral_constant<int, 1>{});
      return;
    }
  }
  f(std::integral_constant<int, 0>{});
}

// TUNED: the rows per block and the radix plan come from c->rows_pick and
// c->plan_row (the mechanics passes of 2D contexts); otherwise rows_for(NX)
// and plan 0.
template <typename T, int NOUT, class Pro, bool TUNED = false>
int launch_row_fwd(fgcg_ctx* c, int kind, const Pro& pro, CT<T>* spec, int nsamp = 1, long long ss = 0) {
  int rc = 0;
  with_n(c->nx, [&](auto NXc) {
    constexpr int NX = decltype(NXc)::value;
    auto go = [&](auto Rc, auto Pc) {
      constexpr int R = decltype(Rc)::value, P = decltype(Pc)::value;
      dim3 g((c->rows + R - 1) / R, nsamp);
      if (kind >= 0) set_kname(c, kind, "k_row_fwd<%s, %d", tname<T>(), NX);
      rc = launch(c, kind, (const void*)&k_row_fwd<T, NX, NOUT, Pro, R, P>, g, pro, spec, c->rows, ss,
                  tw_x<T>(c));
    };
    if constexpr (TUNED)
      with_rows<NX>(c->rows_pick, [&](auto Rc) { with_plan<NX>(c->plan_row, [&](auto Pc) { go(Rc, Pc); }); });
    else
      go(std::integral_constant<int, rows_for(NX)>{}, std::integral_constant<int, 0>{});
  });
  return rc;
}

// TUNED: the radix plan comes from c->plan_col (the mechanics Green pass):
// 1 radix 8, 2 radix 16 (k_col, 256 threads per column), 3 one wavefront per
// column (k_colw; one-component symbols and lengths 256..2048, else plan 1).
template <typename T, int NIN, int NOUT, class Sym, bool TUNED = false>
int launch_col(fgcg_ctx* c, int kind, const Sym& sym, const CT<T>* in, CT<T>* out, int nsamp = 1,
               long long ss = 0) {
  int rc = 0;
  with_n(c->ny, [&](auto NYc) {
    constexpr int NY = decltype(NYc)::value;
    if constexpr (TUNED && NIN == 1 && NOUT == 1 && wave_col_ok(NY)) {
      if (c->plan_col == 3) {
        if (kind >= 0) set_kname(c, kind, "k_colw<%s, %d", tname<T>(), NY);
        const void* fn = c->nsamp == 1 ? (const void*)&k_colw<T, NY, Sym, true> : (const void*)&k_colw<T, NY, Sym, false>;
        rc = launch_b(c, kind, fn, dim3(c->nxh, nsamp), dim3(64), sym, in, out, c->nxh, ss, ss, tw_y<T>(c));
        return;
      }
    }
    auto go = [&](auto Pc) {
      constexpr int P = decltype(Pc)::value;
      dim3 g(c->nxh, nsamp);
      if (kind >= 0) set_kname(c, kind, "k_col<%s, %d", tname<T>(), NY);
      rc = launch(c, kind, (const void*)&k_col<T, NY, NIN, NOUT, Sym, P>, g, sym, in, out, c->nxh, ss, ss,
                  tw_y<T>(c));
    };
    if constexpr (TUNED)
      with_plan<NY>(c->plan_col, go);
    else
      go(std::integral_constant<int, 0>{});
  });
  return rc;
}

template <typename T, int NIN, class Epi, bool TUNED = false>
int launch_row_inv(fgcg_ctx* c, int kind, const Epi& epi, const CT<T>* spec, int nsamp = 1,
                   long long ss = 0) {
  int rc = 0;
  with_n(c->nx, [&](auto NXc) {
    constexpr int NX = decltype(NXc)::value;
    auto go = [&](auto Rc, auto Pc) {
      constexpr int R = decltype(Rc)::value, P = decltype(Pc)::value;
      dim3 g((c->rows + R - 1) / R, nsamp);
      if (kind >= 0) set_kname(c, kind, "k_row_inv<%s, %d", tname<T>(), NX);
      rc = launch(c, kind, (const void*)&k_row_inv<T, NX, NIN, Epi, R, P>, g, epi, spec, c->rows, ss,
                  tw_x<T>(c));
    };
    if constexpr (TUNED)
      with_rows<NX>(c->rows_pick, [&](auto Rc) { with_plan<NX>(c->plan_row, [&](auto Pc) { go(Rc, Pc); }); });
    else
      go(std::integral_constant<int, rows_for(NX)>{}, std::integral_constant<int, 0>{});
  });
  return rc;
}

template <typename T, int NIN, int NOUT, class Mid>
int launch_row_mid(fgcg_ctx* c, int kind, const Mid& mid, CT<T>* spec, int nsamp = 1, long long ss = 0) {
  int rc = 0;
  with_n(c->nx, [&](auto NXc) {
    constexpr int NX = decltype(NXc)::value;
    constexpr int R = rows_for(NX);
    dim3 g((c->rows + R - 1) / R, nsamp);
    if (kind >= 0) set_kname(c, kind, "k_row_mid<%s, %d", tname<T>(), NX);
    rc = launch(c, kind, (const void*)&k_row_mid<T, NX, NIN, NOUT, Mid>, g, mid, spec, c->rows, ss,
                tw_x<T>(c));
  });
  return rc;
}

// CG drivers.  Every pass exits at once when the device state says the
// solve has ended, so chunks of iterations can be enqueued blindly and the
// host reads the state once per chunk.
//
// Graph mode (default): a chunk of K iterations is built once into two graph
// instances (rebuilt only when the values the kernels were given change); the
// instances are replayed alternately so that one is always queued while the
// host checks the state left by the other.  Event-record nodes around the
// profiled kernel nodes of the first instance time those launches inside the
// graph (an event node costs about 10 us of idle time, so the second instance
// carries none and profiling samples every other chunk).
template <class S, class F> int run_cg_plain(fgcg_ctx* c, S* dst, S* hst, F&& iter, int maxit) {
  long long k = 0;
  int chunk = 2;
  for (;;) {
    HIPCHK(hipMemcpyAsync(hst, dst, sizeof(S), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    int rc = prof_flush(c);
    if (rc) return rc;
    if (hst->done) return 0;
    if (k > (long long)maxit + 1) return fail(FGCG_EHIP, "CG driver overran the iteration limit");
    for (int j = 0; j < chunk; ++j, ++k) {
      rc = iter();
      if (rc) return rc;
    }
    HIPCHK(hipGetLastError());
    chunk = chunk < 32 ? chunk * 2 : 32;
  }
}

template <class F> int build_chunk(fgcg_ctx* c, fgcg_ctx::GraphSlot& sl, F& iter, int K, bool timed) {
  c->pending.clear();
  HIPCHK(hipGraphCreate(&c->graph, 0));
  c->building = true;
  c->build_timed = timed;
  c->last = nullptr;
  int rc = 0;
  const bool gap = timed && (c->prof_mask & (1u << FGCG_K_EVENT_GAP));
  if (gap) set_kname(c, FGCG_K_EVENT_GAP, "k_noop%.0s%.0d", "", 0);
  for (int j = 0; j < K && !rc; ++j) {
    rc = iter();
    if (!rc && gap) rc = launch(c, FGCG_K_EVENT_GAP, (const void*)&k_noop, dim3(1), 0);
  }
  c->building = false;
  hipGraph_t g = c->graph;
  c->graph = nullptr;
  if (!rc) {
    const hipError_t ei = hipGraphInstantiate(&sl.exec, g, nullptr, nullptr, 0);
    if (ei != hipSuccess) rc = fail(FGCG_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
  }
  (void)hipGraphDestroy(g);
  sl.ev.swap(c->pending);
  c->pending.clear();
  return rc;
}

template <class S, class F>
int run_cg(fgcg_ctx* c, int which, const Key& key, S* dst, S* hs, F&& iter, int maxit, int K = 0) {
  if (!c->use_graphs) return run_cg_plain(c, dst, hs, iter, maxit);
  if (K <= 0) K = c->chunk;
  HIPCHK(hipMemcpyAsync(hs, dst, sizeof(S), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  int rc = prof_flush(c);
  if (rc) return rc;
  if (hs->done) return 0;
  fgcg_ctx::CgGraph& G = c->graphs[which];
  Key full = key;
  full.add(c->prof_mask).add(K);
  if (G.key != full.b || !G.slot[0].exec || !G.slot[1].exec) {
    release_graph(c, G);
    if ((rc = prof_reserve(c, 4 * (size_t)K * FGCG_K_NKINDS))) return rc;
    for (int i = 0; i < 2; ++i)
      if ((rc = build_chunk(c, G.slot[i], iter, K, i == 0))) return rc;
    G.key = full.b;
  }
  long long launched = 0;
  auto go = [&](int i) -> int {
    HIPCHK(hipGraphLaunch(G.slot[i].exec, c->stream));
    HIPCHK(hipMemcpyAsync(hs + i, dst, sizeof(S), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipEventRecord(c->ev_done[i], c->stream));
    launched += K;
    return 0;
  };
  if ((rc = go(0)) || (rc = go(1))) return rc;
  int i = 0;
  for (;;) {
    HIPCHK(hipEventSynchronize(c->ev_done[i]));
    if ((rc = prof_read_slot(c, G.slot[i]))) return rc;
    if (hs[i].done) break;
    if (launched > (long long)maxit + 4LL * K) return fail(FGCG_EHIP, "CG driver overran the iteration limit");
    if ((rc = go(i))) return rc;
    i ^= 1;
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  if ((rc = prof_read_slot(c, G.slot[i ^ 1]))) return rc;
  if (i != 0) hs[0] = hs[i];
  return 0;
}

template <class S> int status_of(const S& s) {
  switch (s.done) {
    case 1: return FGCG_OK;
    case 2: return FGCG_NOT_CONVERGED;
    case 3: return FGCG_EBREAKDOWN;
    case 4: return FGCG_EDOMAIN;
    default: return FGCG_EHIP;
  }
}

template <class S> void fill_info(fgcg_info* info, const S& s, double secs) {
  if (!info) return;
  info->iters = s.iter;
  info->status = status_of(s);
  info->bnorm = std::sqrt(s.bnorm2);
  info->rel_res = s.bnorm2 > 0 ? std::sqrt(s.rr_final / s.bnorm2) : 0.0;
  info->seconds = secs;
}

inline double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

inline int make_mech_mat(const fgcg_ctx* c, const fgcg_material* mat, const double* d, double kappa, MechMat* m) {
  if (!mat) return fail(FGCG_EINVAL, "material is NULL");
  std::memset(m, 0, sizeof *m);
  m->d = d;
  m->kappa = kappa;
  m->ss = c->n;
  if (!(kappa >= 0.0) || !std::isfinite(kappa)) return fail(FGCG_EDOMAIN, "kappa must be finite and >= 0");
  if (mat->E_field) {
    const double nu = mat->nu_field;
    if (!(nu > -1.0 && nu < 0.5)) return fail(FGCG_EDOMAIN, "nu_field outside (-1, 0.5)");
    m->Efield = mat->E_field;
    m->lam_per_E = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    m->mu_per_E = 1.0 / (2.0 * (1.0 + nu));
    return 0;
  }
  if (!mat->phase || !mat->E_tab || !mat->nu_tab) return fail(FGCG_EINVAL, "phase/E_tab/nu_tab is NULL");
  if (mat->nphase < 1 || mat->nphase > FGCG_MAX_PHASES) return fail(FGCG_EINVAL, "nphase outside 1..8");
  m->phase = mat->phase;
  m->nphase = mat->nphase;
  for (int i = 0; i < mat->nphase; ++i) {
    const double E = mat->E_tab[i], nu = mat->nu_tab[i];
    if (!(E > 0.0) || !std::isfinite(E)) return fail(FGCG_EDOMAIN, "E <= 0 or not finite");
    if (!(nu > -1.0 && nu < 0.5)) return fail(FGCG_EDOMAIN, "nu outside (-1, 0.5)");
    m->lm.a[i] = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    m->lm.b[i] = E / (2.0 * (1.0 + nu));
  }
  return 0;
}

// A running CG state for every sample (unit r.z, no stop test), so that the
// solver's passes do their full work outside a solve (timing, test hooks).
// The residual-spectrum mechanics PCG (sr2d.hpp) runs in 2D FP64 contexts
// with the unit Green operator and the forward difference, on rows whose
// length is a multiple of 64 (of 256 for its three-pass form); every other
// mechanics solve keeps the four-pass form.
inline bool sr_eligible(const fgcg_ctx* c) {
  return c->sr_opt && c->ndim == 2 && c->prec == FGCG_FP64 && c->precond == 0 && c->gradop == 0 &&
         !c->strain_form && c->nx % 64 == 0;
}
// The three-pass form's stiffness + transform pass needs rows of a multiple
// of 256; the two-pass form's row stage one of 64.
inline bool sr3_ok(const fgcg_ctx* c) { return sr_eligible(c) && c->nx % NT == 0; }
// The form in use: 2 (four passes) where the residual spectra do not apply,
// else the tuned or pinned pick, the two-pass form (3) before tuning.
inline int sr_form(const fgcg_ctx* c) { return !sr_eligible(c) ? 2 : c->sr_pick ? c->sr_pick : 3; }
// (on grids of at least 2^18 voxels the tuner times the forms and may keep
// the four-pass form: sr_pick = 2)
inline bool sr_active(const fgcg_ctx* c) { return sr_form(c) != 2; }
inline bool fused_active(const fgcg_ctx* c) { return sr_form(c) == 3; }

inline int running_state(fgcg_ctx* c) {
  std::vector<CgState> hs(c->nsamp);
  for (CgState& t : hs) {
    std::memset(&t, 0, sizeof t);
    t.rz[0] = t.rz[1] = 1.0;
    t.bnorm2 = 1.0;
    t.maxit = 1 << 30;
  }
  HIPCHK(hipMemcpyAsync(c->st, hs.data(), sizeof(CgState) * hs.size(), hipMemcpyHostToDevice, c->stream));
  // the host vector is read by the copy: wait before it goes out of scope
  HIPCHK(hipStreamSynchronize(c->stream));
  return 0;
}

// The reference medium of the next mechanics solve: the caller's, or the
// Lame ratio of the stiffest phase (the per-voxel field's Poisson ratio).
// Only lam0 / mu0 matters to the preconditioned CG; mu0 is scaled to 1.
inline void resolve_reference(fgcg_ctx* c, const MechMat& m) {
  const int nphase = m.nphase;
  double lam = c->ref_lam, mu = c->ref_mu;
  if (!(mu > 0.0)) {
    if (m.Efield) {
      lam = m.lam_per_E;
      mu = m.mu_per_E;
    } else {
      double best = -1.0;
      for (int i = 0; i < nphase; ++i) {
        const double l = m.lm.a[i], u = m.lm.b[i];
        const double E = u * (3.0 * l + 2.0 * u) / (l + u);
        if (E > best) {
          best = E;
          lam = l;
          mu = u;
        }
      }
    }
  }
  c->use_lam = lam / mu;
  c->use_mu = 1.0;
}

// Gradient symbol D(k) on n points of spacing h for the operators of
// Sec. 2.6: forward (exp(i theta) - 1)/h; central i sin(theta)/h; eighth-order
// central (2 i / h) sum_m a_m sin(m theta), a = 4/5, -1/5, 4/105, -1/280;
// Fourier i 2 pi k / (n h) with the signed wavenumber, zero at Nyquist.
inline std::vector<double2> grad_symbol(int n, double h, int op) {
  std::vector<double2> d(n);
  for (int k = 0; k < n; ++k) {
    const double th = 2.0 * M_PI * k / n, sh = std::sin(0.5 * th);
    double re = 0.0, im = 0.0;
    if (op == 0) {
      re = -2.0 * sh * sh / h;
      im = std::sin(th) / h;
    } else if (op == 1 || op == 2) {
      // sin(m theta) is exactly zero where 2 m k is a multiple of n (k = 0 and Nyquist)
      auto sinm = [&](int m) { return (2LL * m * k) % n == 0 ? 0.0 : std::sin(m * th); };
      if (op == 1) {
        im = sinm(1) / h;
      } else {
        const double a[4] = {4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0};
        for (int m = 0; m < 4; ++m) im += 2.0 * a[m] * sinm(m + 1);
        im /= h;
      }
    } else {
      const int ks = k < (n + 1) / 2 ? k : k - n;
      im = (n % 2 == 0 && 2 * k == n) ? 0.0 : 2.0 * M_PI * ks / (n * h);
    }
    d[k] = double2{re, im};
  }
  return d;
}

inline int check_solver_args(double tol, int maxit) {
  if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(FGCG_EINVAL, "tol must be finite and >= 0");
  if (maxit < 0) return fail(FGCG_EINVAL, "maxit < 0");
  return 0;
}

// 3D grids (fgcg3d.hip).
bool size3_supported(int n);
int alloc3d(fgcg_ctx* c);
int mech3_solve(fgcg_ctx* c, const MechMat& m, const double* eig, const double* em, double tol, int maxit,
                double* strain, double* stress, double* mean_stress, double* energy, fgcg_info* info);
int history3(fgcg_ctx* c, const MechMat& m0, const double* strain, const double* e, double* H);
int debug_fft(fgcg_ctx* c, int dir, const double* in, double* out);
int debug_apply3(fgcg_ctx* c, int op, const MechMat& m, const double* in, double* out);

}  // namespace fgcg
