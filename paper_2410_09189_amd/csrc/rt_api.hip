// Runtime behind the C ABI of rt_tddft.h: workspace layout, projector tables,
// initialisation (orthonormalisation, V_ion, H_core, dipole matrices, kicks)
// and the self-consistent time loop of Algorithm 1 driving the kernels.
#include "../../include/rt_tddft.h"
#include "kernels.h"
#include "kernels_gs.h"
#include "kernels_mixed.h"
#include "kernels_mlp.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <memory>
#include <array>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <tuple>
#include <vector>

namespace {

thread_local std::string g_init_error;

// ---------------------------------------------------------------------------
// Workspace arena: the same layout code runs once to size and once to place.
// ---------------------------------------------------------------------------
struct Arena {
  char* base = nullptr;
  size_t used = 0;
  template <typename T>
  T* take(size_t count) {
    used = (used + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + used) : nullptr;
    used += count * sizeof(T);
    return p;
  }
};

// Host-side projector tables of one system (integer geometry + beta values).
struct NlTables {
  int rank = 0, n_atoms = 0, n_proj = 0;
  std::vector<int> atom_off, sph_idx;
  std::vector<double> beta, D;
  std::vector<int> u_idx, u_ptr, ent_pt, ent_atom;
};

// Sphere of each atom: every grid point whose minimum-image distance is below
// r_c, listed in increasing flat index; beta columns g, (s_x/sigma) g,
// (s_y/sigma) g, (s_z/sigma) g, each normalised to h^3 sum beta^2 = 1.
static NlTables build_nl(const rt_system& s) {
  NlTables t;
  t.rank = s.nl_rank;
  t.n_atoms = s.n_atoms;
  t.n_proj = s.n_atoms * s.nl_rank;
  if (s.nl_rank == 0) return t;
  const int nx = s.n[0], ny = s.n[1], nz = s.n[2];
  const double h = s.h, rc = s.nl_rcut, sig = s.nl_sigma;
  const double L[3] = {nx * h, ny * h, nz * h};
  const int nn[3] = {nx, ny, nz};
  t.atom_off.push_back(0);
  std::vector<std::tuple<long, int, int>> ents;  // (flat idx, atom, sphere point)
  for (int a = 0; a < s.n_atoms; ++a) {
    std::vector<int> lo(3), cnt(3);
    for (int q = 0; q < 3; ++q) {
      lo[q] = (int)std::floor((s.pos[3 * a + q] - rc) / h) - 1;
      cnt[q] = (int)std::ceil(2.0 * rc / h) + 3;
      if (cnt[q] > nn[q]) { lo[q] = 0; cnt[q] = nn[q]; }
    }
    std::vector<std::pair<long, std::vector<double>>> pts;
    for (int dz = 0; dz < cnt[2]; ++dz) {
      int iz = ((lo[2] + dz) % nz + nz) % nz;
      for (int dy = 0; dy < cnt[1]; ++dy) {
        int iy = ((lo[1] + dy) % ny + ny) % ny;
        for (int dx = 0; dx < cnt[0]; ++dx) {
          int ix = ((lo[0] + dx) % nx + nx) % nx;
          double d[3];
          const int ii[3] = {ix, iy, iz};
          for (int q = 0; q < 3; ++q) {
            double v = ii[q] * h - s.pos[3 * a + q];
            d[q] = v - L[q] * std::nearbyint(v / L[q]);
          }
          double s2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
          if (!(s2 < rc * rc)) continue;
          double g = std::exp(-s2 / (2 * sig * sig)) * (1.0 - s2 / (rc * rc)) * (1.0 - s2 / (rc * rc));
          std::vector<double> col = {g, d[0] / sig * g, d[1] / sig * g, d[2] / sig * g};
          long flat = ((long)iz * ny + iy) * nx + ix;
          pts.push_back({flat, col});
        }
      }
    }
    std::sort(pts.begin(), pts.end(), [](auto& x, auto& y) { return x.first < y.first; });
    pts.erase(std::unique(pts.begin(), pts.end(), [](auto& x, auto& y) { return x.first == y.first; }),
              pts.end());
    std::vector<double> norm(t.rank, 0.0);
    for (auto& p : pts)
      for (int r = 0; r < t.rank; ++r) norm[r] += p.second[r] * p.second[r];
    for (int r = 0; r < t.rank; ++r) norm[r] = std::sqrt(norm[r] * h * h * h);
    for (auto& p : pts) {
      int sp = (int)t.sph_idx.size();
      t.sph_idx.push_back((int)p.first);
      for (int r = 0; r < t.rank; ++r) t.beta.push_back(p.second[r] / norm[r]);
      ents.emplace_back(p.first, a, sp);
    }
    t.atom_off.push_back((int)t.sph_idx.size());
    for (int r = 0; r < t.rank; ++r) t.D.push_back(s.nl_D[a * t.rank + r]);
  }
  std::sort(ents.begin(), ents.end());
  for (size_t e = 0; e < ents.size(); ++e) {
    long flat = std::get<0>(ents[e]);
    if (t.u_idx.empty() || t.u_idx.back() != (int)flat) {
      t.u_idx.push_back((int)flat);
      t.u_ptr.push_back((int)e);
    }
    t.ent_atom.push_back(std::get<1>(ents[e]));
    t.ent_pt.push_back(std::get<2>(ents[e]));
  }
  t.u_ptr.push_back((int)ents.size());
  return t;
}

// All trajectories of one system step in lockstep: their matrices are stacked
// ([T][...]) so every stage is one launch over the active trajectories, and
// the grid kernels of different trajectories share the orbital reads.
struct SysDev {
  int nx, ny, nz, N, n_occ, n_atoms, n_images;
  long ng;
  double h, h3;
  double coef[5];
  NlTables nl;
  int n_union = 0;
  int n_split = 1, big = 0;
  long kps = 0;
  int n_split_x = 1;  // splits of the BF16x3 projection
  long kps_x = 0;
  // tuned launch shapes (0 = the built-in choice): stencil y-tile rows and z chunks
  // per element type, target block count of the FP64 projection, splits of the
  // N <= 256 BF16x3 projection
  int st_ty[2] = {0, 0}, st_nzc[2] = {0, 0}, st_hq[2] = {0, 0};
  int gemm_target = 0, tri_splits = 0;
  int n_split_cap = 1, n_split_x_cap = 1;  // partial buffers are sized for these
  bool mixed = false;
  bool nonorth = false;  // propagate in the given (non-orthogonal) basis with its overlap
  int hb = 0;            // orbitals the buffer hpsi holds (N, or the run's h_block)
  int hpsi_sets = 0;     // FP64 full updates with T > 1: T buffers of H Psi in hpsiT (else 0)
  int dcorr = 0;         // bit q: vacuum dipole correction along axis q
  int jump[3] = {0, 0, 0};  // sawtooth jump plane per axis
  double dion[3] = {0.0, 0.0, 0.0};  // ions' dipole sum_a Z_a s_q(R_a) on the corrected axes
  double *dscale = nullptr, *dfield = nullptr, *dpart = nullptr;  // [3], [T][3], [T][kRedBlocks][3]
  double* tcur = nullptr;                  // device scalar: time t_j of the step being taken
  int box_off = 0;                         // this system's mailbox slot (words): seq, then payload
  unsigned long long box_seq = 0;          // publishes of this system the host has consumed
  hipStream_t sst = nullptr;               // own stream when the context steps several systems
  hipEvent_t ev = nullptr;                 // joins sst back into the caller's stream
  unsigned long long* box_ctr = nullptr;   // device count of this system's mailbox writes
  // executable graphs of the captured launch sequences, keyed by the buffers they use
  std::map<std::vector<uintptr_t>, hipGraphExec_t> graphs;
  double *Sov = nullptr, *Sinv = nullptr, *G = nullptr;  // overlap, its inverse, [T] S^-1 Hbar
  int T = 1;          // trajectory slots of this system (>= 1)
  int step = 0;       // steps taken (lockstep)
  std::vector<int> slot_traj;  // global trajectory index of each slot (-1: none)
  std::vector<int> active_host;
  std::vector<int> zeros2T;    // host zeros for the series flags
  // orbitals and static fields
  double *psi, *hpsi, *vion, *vloc_gs, *occ;
  double* hpsiT = nullptr;  // [hpsi_sets][N][ng] (hpsi and psi trade places at init, so not hpsi)
  float* vloc32;
  double2* z;
  double2 *twx, *twy, *twz;
  double *pos, *depth, *width;
  int *atom_off, *sph_idx, *u_idx, *u_ptr, *ent_pt, *ent_atom;
  double *beta, *Dd, *cnl;
  double *hcore, *M3, *Hgs, *tmp, *tmp2, *red2, *escale, *ezero;
  int* info;
  // per-trajectory grid fields [T][ng] and weights
  double *rho, *vh, *vx, *vloc, *dv, *eparts, *W, *part;
  // mixed precision: orbitals and density weights as bf16 hi/lo, FP64 ground-state references
  unsigned short *psi_hi, *psi_lo, *w_hi, *w_lo;
  unsigned short *psiT_hi = nullptr, *psiT_lo = nullptr;  // point-major [ng][wld] (N <= 256)
  int wld = 0;                                           // leading dimension of the W split
  double *rho_gs, *S_gs;
  float *dv32, *part32;
  float* dpart32 = nullptr;                // N > 256: partial densities [T][row blocks][ng]
  // per-trajectory state [T][...]
  double *P0, *P1, *dP, *dPn, *C;          // stacked [S'; A'], 2 N^2 each
  double* gwork = nullptr;                 // Gershgorin rows [T][N][2] / observable partials [T][160]
  double* fieldp = nullptr;                // pulse parameters per slot [T][7]
  double *Bm = nullptr, *C2 = nullptr;     // fourth-order Magnus: Omega_2 [T][N^2], B . [S;A]^T [T][2N^2]
  double *A0m = nullptr, *A1m = nullptr, *Xm = nullptr;  // its scratch, [T][N^2] each
  bool field = false;                      // any slot with a nonzero pulse amplitude
  double *H0, *H1, *Hm1, *Hm2, *Hn, *Hbar;  // N^2 each
  double* hist;                            // [T][cap + 1][5]
  double* kmin;                            // [T]
  unsigned long long *slots, *resid;       // [T][max_terms + 2], [T]
  int *done, *active;                      // [T][2], [T]
  // learned predictor / training-sample recording
  bool feat = false;                       // grid edges divisible by 16: features available
  bool mlp = false;                        // RT_PRED_MLP in use
  int mom_head = -1, cd_cur = 1, cv_head = -1, n_hist = 0;
  bool x_valid = false;
  float *mom_ring, *cd_ring, *xbuf, *ybuf, *mlp_params, *mlp_work;
  double* cv_ring;                         // [T][3][4096] coarse V_loc - V_loc,gs (FP64)
  double* mom_part;
  int* mlp_mask;
  std::vector<int> mlp_on;                 // host copy of mlp_mask
  std::vector<std::vector<double>> r1_linear;
  double* rho_gs64;                        // ground-state density (all modes)
};

constexpr int kNIn = 8 * 9 + 2 * 4096, kNH = 256, kNOut = 4096;
constexpr int kMaxTraj = 256;  // trajectories per system (one series-control block)
inline rtk::MlpDims pred_dims() { return rtk::MlpDims{kNIn, kNH, kNOut}; }

struct TrajDev {
  int sys, slot, axis;
  double kappa;
  double field[7];  // a, omega, tau, phase, d_x, d_y, d_z (a = 0: no field)
};

}  // namespace

// Phase timers: hipEvents recorded around each launch of a tracked kernel class
// on the context's stream, resolved at the next synchronisation point.
enum Phase {
  PH_STENCIL = 0, PH_NONLOCAL, PH_PROJECT, PH_REDUCE, PH_DENSITY, PH_POISSON, PH_LDA, PH_SERIES_GEMM,
  PH_SERIES_UPDATE, PH_SMALL, PH_COUNT
};
static const char* kPhaseNames[PH_COUNT] = {
  "stencil_fd8", "nonlocal", "project_gemm", "reduce_partials", "density", "poisson_dft", "lda_vloc",
  "series_gemm", "series_update", "small_matrix"};

struct rt_ctx {
  hipStream_t stream = nullptr;
  bool prof = false;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  std::vector<hipEvent_t> pool;
  double prof_ms[PH_COUNT] = {0};
  long prof_n[PH_COUNT] = {0};
  rt_run run{};
  std::vector<SysDev> sys;
  std::vector<TrajDev> traj;
  std::string err;
  std::string tune_report;  // last rt_autotune's choices and timings
  int hist_cap = 0;
  float *rec_x = nullptr, *rec_y = nullptr;
  int rec_cap = 0, rec_count = 0;
  // host-mapped mailbox for the per-iteration convergence flags: the device writes them
  // with a sequence number per system slot and the host polls it (no copy, no
  // interrupt-driven wait)
  unsigned* box_host = nullptr;
  unsigned* box_dev = nullptr;
  size_t box_bytes = 0;
  // graph capture of the per-update launch sequences (rt_run.graph_capture)
  bool graphs = false;
  hipStream_t cap = nullptr;  // capture-only stream (captured work is replayed on `stream`)
  hipEvent_t join = nullptr;  // caller's stream position at the start of rt_step
  ~rt_ctx() {
    for (auto& d : sys) {
      for (auto& kv : d.graphs) (void)hipGraphExecDestroy(kv.second);
      if (d.sst) (void)hipStreamDestroy(d.sst);
      if (d.ev) (void)hipEventDestroy(d.ev);
    }
    if (join) (void)hipEventDestroy(join);
    if (cap) (void)hipStreamDestroy(cap);
    if (box_host) (void)hipHostFree(box_host);
  }
};

namespace {

#define CK(expr)                                                                    \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) return fail(c, RT_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)
#define RET(expr)                \
  do {                           \
    rt_status r_ = (expr);       \
    if (r_ != RT_OK) return r_;  \
  } while (0)

rt_status fail(rt_ctx* c, rt_status st, const std::string& msg) {
  if (c) c->err = msg; else g_init_error = msg;
  return st;
}

long nsq(int N) { return (long)N * N; }

// Waits until the mailbox holds sequence number seq.  Spins on the host-mapped word; every
// few thousand polls it asks the stream whether work is still pending, so a stream that
// drained without writing seq, or that failed, ends the wait with an error.
// Mailbox: every system owns a slot [seq (2 words)][payload], written by a publish kernel
// on the system's stream.  The host waits for the slots of several systems at once, so
// their flags are read after one round trip.
const unsigned long long* slot_seq(rt_ctx* c, const SysDev& d) {
  return reinterpret_cast<const unsigned long long*>(c->box_host + d.box_off);
}
hipStream_t stream_of(rt_ctx* c, const SysDev& d) { return d.sst ? d.sst : c->stream; }

// Waits until every listed system's slot holds its next sequence number.  Spins on the
// host-mapped words; every few thousand polls it asks the streams (the caller's and the
// system's own) whether work is still pending, so streams that drained without writing
// the slot, or failed, end the wait.
rt_status wait_slots(rt_ctx* c, const std::vector<SysDev*>& ds) {
  for (long spin = 1;; ++spin) {
    bool all = true;
    for (const SysDev* d : ds)
      if (__atomic_load_n(slot_seq(c, *d), __ATOMIC_ACQUIRE) != d->box_seq + 1) all = false;
    if (all) break;
    if ((spin & 4095) == 0) {
      for (const SysDev* d : ds) {
        if (__atomic_load_n(slot_seq(c, *d), __ATOMIC_ACQUIRE) == d->box_seq + 1) continue;
        // the publish went to the caller's stream or to the system's own one
        hipError_t e = hipStreamQuery(c->stream);
        if (e == hipSuccess && d->sst) e = hipStreamQuery(d->sst);
        if (e == hipSuccess) {
          if (__atomic_load_n(slot_seq(c, *d), __ATOMIC_ACQUIRE) == d->box_seq + 1) continue;
          return fail(c, RT_EDEVICE, "stream drained without writing the mailbox");
        }
        if (e != hipErrorNotReady) return fail(c, RT_EDEVICE, std::string("wait_slots: ") + hipGetErrorString(e));
      }
    }
    __builtin_ia32_pause();
  }
  for (SysDev* d : ds) d->box_seq += 1;
  return RT_OK;
}
rt_status wait_slot(rt_ctx* c, SysDev& d) { return wait_slots(c, std::vector<SysDev*>{&d}); }

rt_status enqueue_publish(rt_ctx* c, const SysDev& d, const void* src, size_t nbytes) {
  if (nbytes % 4 != 0 || nbytes / 4 > (size_t)(2 * d.T + 2)) return fail(c, RT_EINVAL, "mailbox slot size");
  CK(rtk::publish(c->stream, src, (int)(nbytes / 4), c->box_dev, d.box_off, d.box_ctr));
  return RT_OK;
}
void slot_read(rt_ctx* c, const SysDev& d, size_t nbytes, void* out) {
  std::memcpy(out, c->box_host + d.box_off + 2, nbytes);
}
rt_status read_back(rt_ctx* c, SysDev& d, const void* src, size_t nbytes, void* out) {
  RET(enqueue_publish(c, d, src, nbytes));
  RET(wait_slot(c, d));
  slot_read(c, d, nbytes, out);
  return RT_OK;
}

// Launches issued in its scope go to the given stream.
struct OnStream {
  rt_ctx* c;
  hipStream_t saved;
  OnStream(rt_ctx* c_, hipStream_t s) : c(c_), saved(c_->stream) { c->stream = s; }
  ~OnStream() { c->stream = saved; }
};

// Runs the launch sequence `enqueue` on the context's stream: from an executable graph
// captured once per key (the buffers the sequence uses; all changing scalars live in
// device memory), or eagerly when capture is off or the phase timers are on.  Capture
// happens on a private stream and executes nothing; the graph then runs on `stream`.
template <class F>
rt_status run_graph(rt_ctx* c, SysDev& d, const std::vector<uintptr_t>& key, F&& enqueue) {
  if (!c->graphs || c->prof) return enqueue();
  auto it = d.graphs.find(key);
  if (it == d.graphs.end() && d.graphs.size() >= 64) return enqueue();  // bounded cache
  if (it == d.graphs.end()) {
    hipStream_t user = c->stream;
    CK(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    c->stream = c->cap;
    rt_status st = enqueue();
    c->stream = user;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->cap, &g);
    if (st != RT_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return fail(c, RT_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(c, RT_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    it = d.graphs.emplace(key, ex).first;
  }
  CK(hipGraphLaunch(it->second, c->stream));
  return RT_OK;
}

hipEvent_t take_event(rt_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

struct Timed {
  rt_ctx* c;
  int ph;
  hipEvent_t a = nullptr;
  Timed(rt_ctx* c_, int ph_) : c(c_), ph(ph_) {
    if (c->prof && (a = take_event(c)) != nullptr) (void)hipEventRecord(a, c->stream);
  }
  ~Timed() {
    if (!a) return;
    hipEvent_t b = take_event(c);
    if (!b) { c->pool.push_back(a); return; }
    (void)hipEventRecord(b, c->stream);
    c->pending.push_back({ph, {a, b}});
  }
};

// Resolves recorded event pairs; the stream must have been synchronised.
void prof_collect(rt_ctx* c) {
  for (auto& p : c->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.second.first, p.second.second) == hipSuccess) {
      c->prof_ms[p.first] += ms;
      c->prof_n[p.first] += 1;
    }
    c->pool.push_back(p.second.first);
    c->pool.push_back(p.second.second);
  }
  c->pending.clear();
}

// Grid, atoms, projectors and active space of one system.
rt_status validate_system(const rt_system& s, std::string& why) {
  for (int q = 0; q < 3; ++q)
    if (s.n[q] < 8 || s.n[q] > 256) { why = "grid edge outside [8, 256]"; return RT_EINVAL; }
  for (int q = 0; q < 3; ++q) {
    int m = s.n[q];
    for (int f : {2, 3, 5})
      while (m % f == 0) m /= f;
    if (m != 1) { why = "grid edges must have no prime factor above 5 (FFT Poisson)"; return RT_EINVAL; }
  }
  if (!(s.h > 0)) { why = "h must be positive"; return RT_EINVAL; }
  if (s.n_atoms < 0 || (s.n_atoms > 0 && (!s.pos || !s.depth || !s.width))) { why = "atom arrays"; return RT_EINVAL; }
  if (s.n_images < 0 || s.n_images > 3) { why = "n_images outside [0, 3]"; return RT_EINVAL; }
  if (s.nl_rank != 0 && s.nl_rank != 4) { why = "nl_rank must be 0 or 4"; return RT_EINVAL; }
  if (s.nl_rank && (!s.nl_D || !(s.nl_rcut > 0) || !(s.nl_sigma > 0))) { why = "nonlocal parameters"; return RT_EINVAL; }
  if (s.nl_rank) {
    for (int q = 0; q < 3; ++q)
      if (2.0 * s.nl_rcut / s.h + 3 >= s.n[q]) { why = "projector sphere wider than the cell"; return RT_EINVAL; }
  }
  if (s.n_occ < 0 || s.n_virt < 0 || s.n_occ + s.n_virt < 1) { why = "active space"; return RT_EINVAL; }
  if (!s.psi0) { why = "psi0 is NULL"; return RT_EINVAL; }
  for (int q = 0; q < 3; ++q)
    if (s.saw_jump[q] < 0 || s.saw_jump[q] >= s.n[q]) { why = "saw_jump outside [0, n)"; return RT_EINVAL; }
  if (s.dipole_correction < 0 || s.dipole_correction > 7) { why = "dipole_correction mask outside [0, 7]"; return RT_EINVAL; }
  return RT_OK;
}

rt_status validate(const rt_system* sys, int n_sys, const rt_run* run, std::string& why) {
  if (!sys || n_sys < 1 || !run) { why = "null system/run or n_sys < 1"; return RT_EINVAL; }
  for (int i = 0; i < n_sys; ++i) {
    const rt_system& s = sys[i];
    RET(validate_system(s, why));
    if (s.nonorthogonal && s.orthonormalize) { why = "nonorthogonal and orthonormalize exclude each other"; return RT_EINVAL; }
    if (s.nonorthogonal && run->magnus_order == 4) { why = "magnus_order 4 needs an orthonormal basis"; return RT_EINVAL; }
    if (s.nonorthogonal && run->predictor == RT_PRED_MLP) { why = "the learned predictor needs an orthonormal basis"; return RT_EINVAL; }
  }
  if (!(run->dt != 0.0) || run->n_steps_max < 0 || run->max_scf < 1 || run->max_terms < 1 ||
      !(run->h_thrs > 0) || !(run->dp_thrs > 0)) { why = "run parameters"; return RT_EINVAL; }
  if (run->precision != RT_FP64 && run->precision != RT_MIXED) { why = "precision"; return RT_EINVAL; }
  if (run->precision == RT_MIXED) {
    for (int i = 0; i < n_sys; ++i)
      if (((long)sys[i].n[0] * sys[i].n[1] * sys[i].n[2]) % 8 != 0) {
        why = "mixed precision needs a grid point count divisible by 8"; return RT_EINVAL;
      } else if ((long)sys[i].n[0] * sys[i].n[1] * sys[i].n[2] >= (1L << 23)) {
        why = "mixed precision supports below 2^23 grid points (32-bit buffer offsets)"; return RT_EINVAL;
      }
  }
  if (run->predictor != RT_PRED_LINEAR && run->predictor != RT_PRED_MLP && run->predictor != RT_PRED_QUADRATIC) {
    why = "predictor"; return RT_EINVAL;
  }
  if (run->predictor == RT_PRED_MLP) {
    if (!run->mlp_params) { why = "RT_PRED_MLP needs mlp_params"; return RT_EINVAL; }
    for (int i = 0; i < n_sys; ++i)
      if (sys[i].n[0] % 16 || sys[i].n[1] % 16 || sys[i].n[2] % 16) {
        why = "the learned predictor needs grid edges divisible by 16"; return RT_EINVAL;
      }
  }
  if (run->hupdate != RT_HUPDATE_FULL && run->hupdate != RT_HUPDATE_LOCAL) { why = "hupdate"; return RT_EINVAL; }
  if (run->h_block < 0) { why = "h_block < 0"; return RT_EINVAL; }
  if (run->h_block > 0) {
    if (run->precision != RT_MIXED && run->hupdate != RT_HUPDATE_LOCAL) {
      why = "h_block needs RT_HUPDATE_LOCAL or RT_MIXED (the full update applies H to every orbital)"; return RT_EINVAL;
    }
    for (int i = 0; i < n_sys; ++i)
      if (sys[i].orthonormalize) { why = "h_block excludes orthonormalize"; return RT_EINVAL; }
  }
  if (run->magnus_order != 0 && run->magnus_order != 2 && run->magnus_order != 4) {
    why = "magnus_order must be 0, 2 or 4"; return RT_EINVAL;
  }
  if (run->traj_field) {
    for (int t = 0; t < run->n_traj; ++t) {
      const double* f = run->traj_field + 7L * t;
      for (int q = 0; q < 7; ++q)
        if (!std::isfinite(f[q])) { why = "traj_field must be finite"; return RT_EINVAL; }
      if (f[0] != 0.0 && !(f[2] > 0.0)) { why = "traj_field: pulse duration tau must be positive"; return RT_EINVAL; }
    }
  }
  if (run->n_traj < 0 || (run->n_traj > 0 && (!run->traj_sys || !run->traj_kappa || !run->traj_axis))) {
    why = "trajectory arrays"; return RT_EINVAL;
  }
  std::vector<int> per_sys(n_sys > 0 ? n_sys : 0, 0);
  for (int t = 0; t < run->n_traj; ++t) {
    if (run->traj_sys[t] < 0 || run->traj_sys[t] >= n_sys) { why = "traj_sys out of range"; return RT_EINVAL; }
    if (run->traj_axis[t] < 0 || run->traj_axis[t] > 2) { why = "traj_axis out of range"; return RT_EINVAL; }
    if (++per_sys[run->traj_sys[t]] > kMaxTraj) { why = "more than 256 trajectories on one system"; return RT_EINVAL; }
  }
  return RT_OK;
}

constexpr int kGemmTargets[3] = {1024, 2048, 4096};  // candidate block counts, FP64 projection
constexpr int kTriSplits[4] = {85, 128, 170, 255};   // candidate splits, BF16x3 projection (N <= 256)
// Largest extra workspace FP64 full updates take for per-trajectory H Psi buffers
// (a few percent of one device's HBM; the batched projection gains ~10 %)
constexpr long kHpsiSetsMaxBytes = 16L << 30;

void choose_split(SysDev& d) {
  // FP64 projection: 64 x 64 upper tiles, K chunks of 16, ~2048 blocks (or the tuned count)
  d.big = 0;
  int ntm = (d.N + 63) / 64;
  int tiles = ntm * (ntm + 1) / 2;
  long target = d.gemm_target > 0 ? d.gemm_target : 2048;
  long ns = (target + tiles - 1) / tiles;
  long maxs = std::max(1L, d.ng / 1024);
  ns = std::min(ns, maxs);
  const int bk = 16;
  long kps = (d.ng + ns - 1) / ns;
  kps = (kps + bk - 1) / bk * bk;
  d.kps = kps;
  d.n_split = (int)((d.ng + kps - 1) / kps);
  // room for the largest candidate count
  {
    long nsm = std::min((kGemmTargets[2] + (long)tiles - 1) / tiles, maxs);
    long km = ((d.ng + nsm - 1) / nsm + bk - 1) / bk * bk;
    d.n_split_cap = std::max(d.n_split_cap, std::max(d.n_split, (int)((d.ng + km - 1) / km)));
  }
  // BF16x3 projection: 128 x 128 upper tiles, K chunks of 64, ~4096 blocks per
  // trajectory (many rounds of two blocks per CU, so the last round's tail is short)
  int ntx = (d.N + 127) / 128;
  int tx = ntx * (ntx + 1) / 2;
  long nsx = std::min((4096L + tx - 1) / tx, std::max(1L, d.ng / 2048));
  long kx = (d.ng + nsx - 1) / nsx;
  kx = (kx + 63) / 64 * 64;
  d.kps_x = kx;
  d.n_split_x = (int)((d.ng + kx - 1) / kx);
}

// BF16x3 projection for N <= 256 (whole upper triangle per block, one block per
// CU): 85 splits of the grid, so three trajectories fill the 256 CUs of an MI355X
// in one round; each split at least four staged chunks long.  The split does not
// depend on the number of trajectories, so a trajectory's partial sums, and with
// them its results, are the same batched or alone.
void choose_split_tri(SysDev& d) {
  if (d.N > rtk::proj_tri_max_n()) return;
  const long ck = rtk::proj_tri_chunk();
  auto split = [&](long want, long& kx) {
    long ns = std::min(want, std::max(1L, d.ng / (4 * ck)));
    kx = (d.ng + ns - 1) / ns;
    kx = (kx + ck - 1) / ck * ck;
    return (int)((d.ng + kx - 1) / kx);
  };
  long kx = 0, km = 0;
  d.n_split_x = split(d.tri_splits > 0 ? d.tri_splits : kTriSplits[0], kx);
  d.kps_x = kx;
  d.n_split_x_cap = std::max(d.n_split_x, split(kTriSplits[3], km));
}

// Places every buffer; with a.base == nullptr only sizes.
void layout(Arena& a, std::vector<SysDev>& S, const rt_run& run, int hist_cap) {
  for (auto& d : S) {
    const long ng = d.ng, N = d.N, T = d.T, NN = N * N;
    d.tcur = a.take<double>(1);
    d.box_ctr = a.take<unsigned long long>(1);
    d.psi = a.take<double>(N * ng);
    d.hpsi = a.take<double>((long)d.hb * ng);
    // FP64 full updates hold every trajectory's H Psi, so that one projection launch
    // covers the trajectories and they read Psi through a shared L2; past
    // kHpsiSetsMaxBytes they share the one buffer and project one at a time
    d.hpsi_sets = (!d.mixed && run.hupdate == RT_HUPDATE_FULL && d.hb == d.N && T > 1 &&
                   T * N * ng * (long)sizeof(double) <= kHpsiSetsMaxBytes) ? (int)T : 0;
    d.hpsiT = d.hpsi_sets ? a.take<double>((long)d.hpsi_sets * N * ng) : nullptr;
    d.vion = a.take<double>(ng);
    d.vloc_gs = a.take<double>(ng);
    d.occ = a.take<double>(N);
    d.vloc32 = a.take<float>(ng);
    d.z = a.take<double2>(T * ng);
    d.twx = a.take<double2>(d.nx);
    d.twy = a.take<double2>(d.ny);
    d.twz = a.take<double2>(d.nz);
    d.pos = a.take<double>(3 * std::max(1, d.n_atoms));
    d.depth = a.take<double>(std::max(1, d.n_atoms));
    d.width = a.take<double>(std::max(1, d.n_atoms));
    d.atom_off = a.take<int>(d.nl.atom_off.size() + 1);
    d.sph_idx = a.take<int>(d.nl.sph_idx.size() + 1);
    d.beta = a.take<double>(d.nl.beta.size() + 1);
    d.Dd = a.take<double>(d.nl.D.size() + 1);
    d.u_idx = a.take<int>(d.nl.u_idx.size() + 1);
    d.u_ptr = a.take<int>(d.nl.u_ptr.size() + 1);
    d.ent_pt = a.take<int>(d.nl.ent_pt.size() + 1);
    d.ent_atom = a.take<int>(d.nl.ent_atom.size() + 1);
    d.cnl = a.take<double>(N * std::max(1, d.nl.n_proj));
    d.hcore = a.take<double>(NN);
    d.M3 = a.take<double>(3 * NN);
    d.Hgs = a.take<double>(NN);
    d.tmp = a.take<double>(NN);
    d.tmp2 = a.take<double>(NN);
    d.red2 = a.take<double>(T * 2 * rtk::kRedBlocks);
    d.gwork = a.take<double>(T * std::max(2L * N, 160L));
    d.escale = a.take<double>(2);
    d.ezero = a.take<double>(2);
    d.info = a.take<int>(4);
    d.rho = a.take<double>(T * ng);
    d.vh = a.take<double>(T * ng);
    d.vx = a.take<double>(T * ng);
    d.vloc = a.take<double>(T * ng);
    d.dv = a.take<double>(T * ng);
    d.eparts = a.take<double>(2 * T);
    d.dscale = a.take<double>(3);
    d.dfield = a.take<double>(3 * T);
    d.dpart = a.take<double>(d.dcorr ? 3 * T * rtk::kRedBlocks : 1);
    d.W = a.take<double>(T * NN);
    d.part = a.take<double>(T * std::max(d.n_split, d.n_split_cap) * NN);
    if (d.mixed) {
      // N <= 256: K-blocked for the triangle projection; else orbital-major [N][ng]
      const long npsi = d.N <= rtk::proj_tri_max_n() ? rtk::proj_tri_elems(d.N, ng) : N * ng;
      d.psi_hi = a.take<unsigned short>(npsi);
      d.psi_lo = a.take<unsigned short>(npsi);
      d.wld = rtk::density_tile_ld(d.N);
      const long WW = (long)d.wld * d.wld;
      d.w_hi = a.take<unsigned short>(T * WW);
      d.w_lo = a.take<unsigned short>(T * WW);
      if (d.N <= 256) {
        d.psiT_hi = a.take<unsigned short>(ng * d.wld);
        d.psiT_lo = a.take<unsigned short>(ng * d.wld);
      } else {
        const long nI = (d.N + rtk::density_big_rows() - 1) / rtk::density_big_rows();
        d.dpart32 = a.take<float>(T * nI * ng);
      }
      d.rho_gs = a.take<double>(ng);
      d.S_gs = a.take<double>(NN);
      d.dv32 = a.take<float>(T * ng);
      d.part32 = a.take<float>(T * std::max(d.n_split_x, d.n_split_x_cap) * NN);
    }
    d.P0 = a.take<double>(T * 2 * NN);
    d.P1 = a.take<double>(T * 2 * NN);
    d.dP = a.take<double>(T * 2 * NN);
    d.dPn = a.take<double>(T * 2 * NN);
    d.C = a.take<double>(T * rtk::series_splits(d.N) * 2 * NN);
    d.H0 = a.take<double>(T * NN);
    d.H1 = a.take<double>(T * NN);
    d.Hm1 = a.take<double>(T * NN);
    d.Hm2 = a.take<double>(T * NN);
    d.Hn = a.take<double>(T * NN);
    d.Hbar = a.take<double>(T * NN);
    d.hist = a.take<double>(T * 5L * (hist_cap + 1));
    d.fieldp = a.take<double>(T * 7L);
    if (d.nonorth) {
      d.Sov = a.take<double>(NN);
      d.Sinv = a.take<double>(NN);
      d.G = a.take<double>(T * NN);
    }
    if (run.magnus_order == 4) {
      d.Bm = a.take<double>(T * NN);
      d.C2 = a.take<double>(T * rtk::series_splits(d.N) * 2 * NN);
      d.A0m = a.take<double>(T * NN);
      d.A1m = a.take<double>(T * NN);
      d.Xm = a.take<double>(T * NN);
    }
    d.kmin = a.take<double>(T);
    d.slots = a.take<unsigned long long>(T * (run.max_terms + 2));
    d.resid = a.take<unsigned long long>(T);
    d.done = a.take<int>(2 * T);
    d.active = a.take<int>(T);
    d.rho_gs64 = a.take<double>(ng);
    if (d.feat) {
      d.mom_ring = a.take<float>(T * 72);
      d.cd_ring = a.take<float>(T * 2 * 4096);
      d.cv_ring = a.take<double>(T * 3 * 4096);
      d.xbuf = a.take<float>(T * kNIn);
      d.ybuf = a.take<float>(T * kNOut);
      d.mom_part = a.take<double>(T * 256 * 9);
      d.mlp_mask = a.take<int>(T);
    }
    if (d.mlp) {
      d.mlp_params = a.take<float>(rtk::mlp_n_params(pred_dims()));
      d.mlp_work = a.take<float>(rtk::mlp_work_floats(pred_dims(), T));
    }
  }
}

// Ions' dipole about the sawtooth, sum_a Z_a s_q(R_a), on the corrected axes: Z_a
// from ion_charge, else the electron count sum_i f_i shared equally; s_q in its
// continuous form (((x / h - j0) mod n) - (n-1)/2) h.
void ion_dipole(const rt_system& s, SysDev& d) {
  for (int q = 0; q < 3; ++q) d.dion[q] = 0.0;
  if (!s.dipole_correction || s.n_atoms < 1) return;
  double ne = 0.0;
  const int N = s.n_occ + s.n_virt;
  for (int i = 0; i < N; ++i) ne += s.occ ? s.occ[i] : (i < s.n_occ ? 2.0 : 0.0);
  for (int q = 0; q < 3; ++q) {
    if (!((s.dipole_correction >> q) & 1)) continue;
    const int n = s.n[q];
    double acc = 0.0;
    for (int a = 0; a < s.n_atoms; ++a) {
      const double z = s.ion_charge ? s.ion_charge[a] : ne / s.n_atoms;
      double u = s.pos[3 * a + q] / s.h - s.saw_jump[q];
      u -= n * std::floor(u / n);
      acc += z * ((u - 0.5 * (n - 1)) * s.h);
    }
    d.dion[q] = acc;
  }
}

void describe(const rt_system* sys, int n_sys, const rt_run* run, std::vector<SysDev>& S,
              std::vector<TrajDev>& T) {
  S.resize(n_sys);
  T.resize(run->n_traj);
  for (int i = 0; i < n_sys; ++i) {
    const rt_system& s = sys[i];
    SysDev& d = S[i];
    d.nx = s.n[0]; d.ny = s.n[1]; d.nz = s.n[2];
    d.ng = (long)d.nx * d.ny * d.nz;
    d.N = s.n_occ + s.n_virt;
    d.n_occ = s.n_occ;
    d.n_atoms = s.n_atoms;
    d.n_images = s.n_images;
    d.h = s.h;
    d.h3 = s.h * s.h * s.h;
    // 8th-order central second difference (exact for polynomials of degree <= 8)
    d.coef[0] = -205.0 / 72.0; d.coef[1] = 8.0 / 5.0; d.coef[2] = -1.0 / 5.0;
    d.coef[3] = 8.0 / 315.0; d.coef[4] = -1.0 / 560.0;
    d.nl = build_nl(s);
    d.n_union = (int)d.nl.u_idx.size();
    d.mixed = run->precision == RT_MIXED;
    d.nonorth = s.nonorthogonal != 0;
    d.hb = run->h_block > 0 && run->h_block < d.N ? run->h_block : d.N;
    d.dcorr = s.dipole_correction;
    for (int q = 0; q < 3; ++q) d.jump[q] = s.saw_jump[q];
    ion_dipole(s, d);
    d.feat = d.nx % 16 == 0 && d.ny % 16 == 0 && d.nz % 16 == 0;
    d.mlp = run->predictor == RT_PRED_MLP;
    d.slot_traj.clear();
    choose_split(d);
  }
  for (int t = 0; t < run->n_traj; ++t) {
    SysDev& d = S[run->traj_sys[t]];
    T[t].sys = run->traj_sys[t];
    T[t].slot = (int)d.slot_traj.size();
    T[t].axis = run->traj_axis[t];
    T[t].kappa = run->traj_kappa[t];
    for (int q = 0; q < 7; ++q) T[t].field[q] = run->traj_field ? run->traj_field[7L * t + q] : 0.0;
    d.slot_traj.push_back(t);
  }
  for (auto& d : S) {
    if (d.slot_traj.empty()) d.slot_traj.push_back(-1);
    d.T = (int)d.slot_traj.size();
    choose_split_tri(d);
    d.active_host.assign(d.T, 1);
    d.zeros2T.assign(2 * d.T, 0);
    d.mlp_on.assign(d.T, d.mlp ? 1 : 0);
    d.r1_linear.assign(d.T, std::vector<double>());
  }
}

template <typename V>
rt_status upload(rt_ctx* c, void* dst, const std::vector<V>& v) {
  if (v.empty()) return RT_OK;
  CK(hipMemcpyAsync(dst, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice, c->stream));
  return RT_OK;
}

// Per-trajectory 0/1 flags go to the device as kernel arguments: no pageable copy, which
// would wait for the stream to drain, inside the step loop.
rt_status upload_flags(rt_ctx* c, int* dst, const std::vector<int>& v) {
  rtk::Flags256 f{};
  for (size_t t = 0; t < v.size(); ++t)
    if (v[t]) f.w[t >> 6] |= 1ull << (t & 63);
  CK(rtk::set_flags(c->stream, dst, f, (int)v.size()));
  return RT_OK;
}

rt_status push_active(rt_ctx* c, SysDev& d) { return upload_flags(c, d.active, d.active_host); }

// ---------------------------------------------------------------------------
// Stages
// ---------------------------------------------------------------------------
// Symmetric projection out = h^3 A diag(w) B^T over the grid for one problem.
rt_status project(rt_ctx* c, SysDev& d, const double* A, const double* B, const double* w, double* out) {
  {
    Timed tm(c, PH_PROJECT);
    CK(rtk::gemm_nt_f64(c->stream, d.N, d.N, d.ng, A, d.ng, B, d.ng, w, d.part, d.kps, d.n_split, 1, d.big,
                        rtk::single()));
  }
  Timed tm(c, PH_REDUCE);
  CK(rtk::reduce_parts(c->stream, d.part, d.n_split, d.N, d.N, d.h3, out, 1, nullptr, 1, 0, 0, 0, nullptr));
  return RT_OK;
}

// hpsi = (T + vloc + V_nl) psi for n rows (FP64).
rt_status apply_h64(rt_ctx* c, SysDev& d, const double* psi, double* hpsi, const double* vloc, int n) {
  {
    Timed tm(c, PH_STENCIL);
    CK(rtk::stencil<double>(c->stream, psi, hpsi, vloc, n, d.nx, d.ny, d.nz, d.h, d.coef, d.st_ty[0], d.st_nzc[0],
                            d.st_hq[0]));
  }
  if (d.nl.rank) {
    Timed tm(c, PH_NONLOCAL);
    CK(rtk::nl_gather<double>(c->stream, psi, d.ng, n, d.n_atoms, d.nl.rank, d.atom_off, d.sph_idx,
                              d.beta, d.h3, d.cnl));
    CK(rtk::nl_scatter<double>(c->stream, hpsi, d.ng, n, d.n_union, d.u_idx, d.u_ptr, d.ent_pt,
                               d.ent_atom, d.nl.rank, d.beta, d.Dd, d.cnl, d.nl.n_proj));
  }
  return RT_OK;
}

rt_status apply_h32(rt_ctx* c, SysDev& d, const float* psi, float* hpsi, int n) {
  {
    Timed tm(c, PH_STENCIL);
    CK(rtk::stencil<float>(c->stream, psi, hpsi, d.vloc32, n, d.nx, d.ny, d.nz, d.h, d.coef, d.st_ty[1], d.st_nzc[1],
                           d.st_hq[1]));
  }
  if (d.nl.rank) {
    Timed tm(c, PH_NONLOCAL);
    CK(rtk::nl_gather<float>(c->stream, psi, d.ng, n, d.n_atoms, d.nl.rank, d.atom_off, d.sph_idx,
                             d.beta, d.h3, d.cnl));
    CK(rtk::nl_scatter<float>(c->stream, hpsi, d.ng, n, d.n_union, d.u_idx, d.u_ptr, d.ent_pt,
                              d.ent_atom, d.nl.rank, d.beta, d.Dd, d.cnl, d.nl.n_proj));
  }
  return RT_OK;
}

// Spectral Poisson + LDA for the active slots (FP64): rho_t -> V_H, v_x, V_loc, energies.
rt_status poisson_lda(rt_ctx* c, SysDev& d, int T, const int* act) {
  hipStream_t s = c->stream;
  {
    Timed tp(c, PH_POISSON);
    CK(rtk::poisson_fft(s, d.rho, d.vh, d.z, d.nx, d.ny, d.nz, d.h, d.twx, d.twy, d.twz, T));
  }
  Timed tl(c, PH_LDA);
  // vacuum dipole correction: g_q = (4 pi / Omega) h^3 sum rho s_q on the selected axes
  rtk::SawGeom sg;
  sg.nx = d.nx; sg.ny = d.ny; sg.nz = d.nz;
  sg.jx = d.jump[0]; sg.jy = d.jump[1]; sg.jz = d.jump[2];
  sg.h = d.h;
  const double gscale = 4.0 * M_PI / ((double)d.ng * d.h3);
  for (int q = 0; q < 3; ++q) {
    sg.gion[q] = gscale * d.dion[q];
    sg.dion[q] = d.dion[q] / d.h3;
  }
  if (d.dcorr) {
    CK(rtk::saw_dipole(s, d.rho, sg, d.ng, d.dpart, T, act));
    CK(rtk::reduce_cols(s, d.dpart, rtk::kRedBlocks, 3, d.dscale, d.dfield, T, act));
  }
  CK(rtk::lda_vloc(s, d.rho, d.vh, d.vion, d.vx, d.vloc, d.ng, d.red2, T, act, d.dcorr ? &sg : nullptr,
                   d.dcorr ? d.dfield : nullptr));
  CK(rtk::reduce_cols(s, d.red2, rtk::kRedBlocks, 2, d.escale, d.eparts, T, act));
  return RT_OK;
}

// Hout_t = H[P_t] for the T' slots (S_t real parts with stride sstride, Hout stride N^2).
// act: device flags (nullable = all T); act_host mirrors them.  mode_full forces the
// FP64 full apply (ground-state build).
// BF16x3 weighted projection of the orbitals against d.dv32 into d.part32
hipError_t proj_x(hipStream_t s, const SysDev& d, int T, const int* act) {
  if (d.N <= rtk::proj_tri_max_n())
    return rtk::proj_tri_bf16x3(s, d.N, d.ng, d.psi_hi, d.psi_lo, d.dv32, d.part32, d.kps_x, d.n_split_x, T, act);
  return rtk::proj_bf16x3(s, d.N, d.ng, d.psi_hi, d.psi_lo, d.dv32, d.part32, d.kps_x, d.n_split_x, T, act);
}

rt_status eval_h(rt_ctx* c, SysDev& d, int T, const int* act, const std::vector<int>& act_host,
                 const double* S, long sstride, double* Hout, bool force_full) {
  hipStream_t s = c->stream;
  const rt_run& r = c->run;
  const long NN = nsq(d.N);
  if (r.frozen_hxc && !force_full) {
    for (int t = 0; t < T; ++t)
      if (act_host[t]) CK(rtk::copy_d(s, Hout + t * NN, d.Hgs, NN));
    return RT_OK;
  }
  const bool mixed = d.mixed && !force_full;
  {
    Timed tm(c, PH_DENSITY);
    if (mixed) {
      CK(rtk::upper_weighted_delta_bf16(s, S, d.S_gs, d.w_hi, d.w_lo, d.N, d.wld, sstride, T, act, d.N <= 256));
      CK(rtk::density_bf16x3(s, d.N, d.ng, d.w_hi, d.w_lo, d.psi_hi, d.psi_lo, d.psiT_hi, d.psiT_lo, d.rho_gs,
                             d.rho, T, act, d.dpart32));
    } else {
      CK(rtk::upper_weighted(s, S, d.W, d.N, sstride, T, act));
      CK(rtk::smalltall_f64(s, d.N, d.ng, d.W, d.psi, d.rho, 1, 1, T, act));
    }
  }
  RET(poisson_lda(c, d, T, act));
  if (mixed) {
    // H = H_gs + h^3 Psi diag(V_loc - V_loc,gs) Psi^T in BF16x3
    CK(rtk::delta_f32(s, d.dv32, d.vloc, d.vloc_gs, d.ng, T, act));
    {
      Timed tm(c, PH_PROJECT);
      CK(proj_x(s, d, T, act));
    }
    Timed tr(c, PH_REDUCE);
    CK(rtk::reduce_parts_f32(s, d.part32, d.n_split_x, d.N, d.h3, d.Hgs, Hout, T, act, 0));
    return RT_OK;
  }
  if (force_full && d.hb < d.N) {
    // blocked systems: H[P] = H_core + h^3 Psi^T diag(V_loc - V_ion) Psi (no full apply)
    CK(rtk::sub_d(s, d.dv, d.vloc, d.vion, d.ng, T, act));
    const long sp = (long)d.n_split * NN;
    {
      Timed tm(c, PH_PROJECT);
      CK(rtk::gemm_nt_f64(s, d.N, d.N, d.ng, d.psi, d.ng, d.psi, d.ng, d.dv, d.part, d.kps, d.n_split, 1, d.big,
                          rtk::Batch{T, act, 0, 0, d.ng, sp}));
    }
    Timed tr(c, PH_REDUCE);
    CK(rtk::reduce_parts(s, d.part, d.n_split, d.N, d.N, d.h3, Hout, 1, d.hcore, T, sp, 0, NN, act));
    return RT_OK;
  }
  if ((r.hupdate == RT_HUPDATE_FULL || force_full) && T > 1 && d.hpsiT && d.hpsi_sets >= T) {
    // every trajectory's H Psi, then one projection launch for all of them
    const long nsz = (long)d.N * d.ng;
    for (int t = 0; t < T; ++t)
      if (act_host[t]) RET(apply_h64(c, d, d.psi, d.hpsiT + t * nsz, d.vloc + (long)t * d.ng, d.N));
    const long sp = (long)d.n_split * NN;
    {
      Timed tm(c, PH_PROJECT);
      CK(rtk::gemm_nt_f64(s, d.N, d.N, d.ng, d.psi, d.ng, d.hpsiT, d.ng, nullptr, d.part, d.kps, d.n_split, 1,
                          d.big, rtk::Batch{T, act, 0, nsz, 0, sp}));
    }
    Timed tr(c, PH_REDUCE);
    CK(rtk::reduce_parts(s, d.part, d.n_split, d.N, d.N, d.h3, Hout, 1, nullptr, T, sp, 0, NN, act));
    return RT_OK;
  }
  if (r.hupdate == RT_HUPDATE_FULL || force_full) {
    for (int t = 0; t < T; ++t) {
      if (!act_host[t]) continue;
      RET(apply_h64(c, d, d.psi, d.hpsi, d.vloc + (long)t * d.ng, d.N));
      RET(project(c, d, d.psi, d.hpsi, nullptr, Hout + t * NN));
    }
    return RT_OK;
  }
  // local update: H[P] = H_gs + h^3 Psi diag(V_loc - V_loc,gs) Psi^T (FP64)
  CK(rtk::sub_d(s, d.dv, d.vloc, d.vloc_gs, d.ng, T, act));
  const long sp = (long)d.n_split * NN;
  {
    Timed tm(c, PH_PROJECT);
    CK(rtk::gemm_nt_f64(s, d.N, d.N, d.ng, d.psi, d.ng, d.psi, d.ng, d.dv, d.part, d.kps, d.n_split, 1, d.big,
                        rtk::Batch{T, act, 0, 0, d.ng, sp}));
  }
  Timed tr(c, PH_REDUCE);
  CK(rtk::reduce_parts(s, d.part, d.n_split, d.N, d.N, d.h3, Hout, 1, d.Hgs, T, sp, 0, NN, act));
  return RT_OK;
}

// P_t -> U_t P_t U_t^dagger, U_t = exp(-i dt Hbar_t), by the commutator series, for the
// T slots starting at the given buffers (stacked [S; A], stride 2 N^2).  flags/scratch
// (kmin, slots, done, dP, dPn, C) are the system's, offset by `first`.  start() launches
// the series start with its first terms and the stop-flag publish; complete() reads the
// flags (after the caller's wait) and runs further chunks of terms until every active
// trajectory has stopped.
struct Series {
  static constexpr int CH = 8;  // terms per chunk between flag reads (even: dP/dPn end where they began)
  rt_ctx* c;
  SysDev& d;
  int first, T;
  const int* act;
  const double* Hbar;
  double dt;
  const double *Pin, *H0, *H1, *tptr;
  double* Pout;
  unsigned long long* resid;
  long NN, n2;
  int max_terms, stride;
  double thrs;
  double *dP0, *dPn0, *C, *kmin, *B, *C2;
  unsigned long long* slots;
  int* done;
  const double *fp, *Gs;
  int kend = 0;

  Series(rt_ctx* c_, SysDev& d_, int first_, int T_, const int* act_, const double* Hbar_, double dt_,
         const double* Pin_, double* Pout_, const double* H0_, const double* H1_, unsigned long long* resid_,
         const double* tptr_)
      : c(c_), d(d_), first(first_), T(T_), act(act_), Hbar(Hbar_), dt(dt_), Pin(Pin_), H0(H0_), H1(H1_),
        tptr(tptr_), Pout(Pout_), resid(resid_) {
    NN = nsq(d.N);
    n2 = 2 * NN;
    max_terms = c->run.max_terms;
    stride = max_terms + 2;
    thrs = c->run.dp_thrs;
    dP0 = d.dP + first * n2;
    dPn0 = d.dPn + first * n2;
    C = d.C + first * rtk::series_splits(d.N) * n2;
    kmin = d.kmin + first;
    slots = d.slots + (long)first * stride;
    done = d.done + 2 * first;
    // fourth-order Magnus (time steps only): Omega = -i dt Hbar + B, B = Omega_2
    B = (H0 && d.Bm) ? d.Bm + first * NN : nullptr;
    C2 = B ? d.C2 + first * rtk::series_splits(d.N) * n2 : nullptr;
    // the external field joins the midpoint Hamiltonian of a time step (H0 given):
    // + (V(t_a) + V(t_a + dt))/2, V = sum_q E_q M_q, t_a = *tptr
    fp = (H0 && d.field) ? d.fieldp + 7L * first : nullptr;
    Gs = d.nonorth ? d.G + first * NN : Hbar;
  }

  rt_status terms_k(int k_from, int k_to) {
    double* dP = dP0;
    double* dPn = dPn0;
    for (int k = k_from; k <= k_to; ++k) {
      if (!B && d.N <= rtk::series_small_max()) {
        // small N: product and update in one launch
        Timed tm(c, PH_SERIES_GEMM);
        CK(rtk::series_term_small(c->stream, d.N, T, Gs, dP, dPn, Pout, dt, k, slots, stride, kmin, thrs, done,
                                  act));
        std::swap(dP, dPn);
        continue;
      }
      {
        Timed tm(c, PH_SERIES_GEMM);
        CK(rtk::gemm_nt_f64_series(c->stream, d.N, T, Gs, dP, C, k, slots, stride, kmin, thrs, done, act));
        if (B) CK(rtk::gemm_nt_f64_series(c->stream, d.N, T, B, dP, C2, k, slots, stride, kmin, thrs, done, act));
      }
      {
        Timed tm(c, PH_SERIES_UPDATE);
        CK(rtk::series_update(c->stream, C, C2, dPn, Pout, d.N, dt, k, slots, stride, kmin, thrs, done, T, act));
      }
      std::swap(dP, dPn);
    }
    CK(rtk::series_finish(c->stream, k_to, slots, stride, kmin, thrs, done, T, act));
    return enqueue_publish(c, d, done, 2 * T * sizeof(int));
  }

  rt_status begin_chunk() {
    {
      Timed tm(c, PH_SMALL);
      if (B) CK(rtk::magnus2(c->stream, H0, H1, fp, d.M3, tptr, dt, d.A0m + first * NN, d.A1m + first * NN,
                             d.Xm + first * NN, B, d.N, T, act));
      CK(rtk::series_begin(c->stream, Pin, Pout, dP0, H0, H1, const_cast<double*>(Hbar), d.N, dt, kmin, slots,
                           stride, done, resid, d.gwork, T, act, fp, d.M3, tptr, B));
      if (d.nonorth) {
        // non-orthogonal basis: the series runs on G = S^-1 Hbar (dP_k = (1/k)(-i dt)(G dP - dP G^T)),
        // and its stop floor is the Gershgorin width of G
        CK(rtk::gemm_nt_f64(c->stream, d.N, d.N, d.N, d.Sinv, d.N, Hbar, d.N, nullptr, d.G + first * NN, d.N, 1, 0,
                            0, rtk::Batch{T, act, 0, NN, 0, NN}));
        CK(rtk::gershgorin(c->stream, d.G + first * NN, d.N, dt, kmin, d.gwork, T, act));
      }
    }
    return terms_k(1, kend);
  }

  // begin + first chunk + stop-flag publish: one captured sequence
  rt_status start() {
    kend = std::min(max_terms, CH);
    uint64_t dtb;
    std::memcpy(&dtb, &dt, sizeof(dtb));
    const std::vector<uintptr_t> key{1, (uintptr_t)first, (uintptr_t)T, (uintptr_t)act, (uintptr_t)Hbar,
                                     (uintptr_t)Pin, (uintptr_t)Pout, (uintptr_t)H0, (uintptr_t)H1,
                                     (uintptr_t)resid, (uintptr_t)tptr, (uintptr_t)dtb};
    return run_graph(c, d, key, [&]() { return begin_chunk(); });
  }

  // after the wait for start()'s publish
  rt_status complete(const std::vector<int>& act_host, std::vector<int>& terms) {
    std::vector<int> hd(2 * T);
    slot_read(c, d, 2 * T * sizeof(int), hd.data());
    while (true) {
      bool all = true;
      for (int t = 0; t < T; ++t)
        if (act_host[t] && !hd[2 * t]) all = false;
      if (all) {
        terms.assign(T, 0);
        for (int t = 0; t < T; ++t) terms[t] = act_host[t] ? hd[2 * t + 1] : 0;
        return RT_OK;
      }
      if (kend >= max_terms) return fail(c, RT_ENOCONV, "commutator series reached max_terms");
      const int k_to = std::min(max_terms, kend + CH);
      RET(terms_k(kend + 1, k_to));
      kend = k_to;
      RET(wait_slot(c, d));
      slot_read(c, d, 2 * T * sizeof(int), hd.data());
    }
  }
};

rt_status series(rt_ctx* c, SysDev& d, int first, int T, const int* act, const std::vector<int>& act_host,
                 const double* Hbar, double dt, const double* Pin, double* Pout, std::vector<int>& terms,
                 const double* H0 = nullptr, const double* H1 = nullptr, unsigned long long* resid = nullptr,
                 const double* tptr = nullptr) {
  Series sr(c, d, first, T, act, Hbar, dt, Pin, Pout, H0, H1, resid, tptr);
  RET(sr.start());
  RET(wait_slot(c, d));
  return sr.complete(act_host, terms);
}

rt_status observe(rt_ctx* c, SysDev& d, int row) {
  const double* Hc = c->run.frozen_hxc ? d.Hgs : d.hcore;
  const double* ep = c->run.frozen_hxc ? d.ezero : d.eparts;
  const int es = c->run.frozen_hxc ? 0 : 2;
  CK(rtk::observables(c->stream, d.P0, d.M3, Hc, d.nonorth ? d.Sov : nullptr, d.N, ep, es, d.hist + 5L * row, 5L * (c->hist_cap + 1), d.gwork,
                      d.T));
  return RT_OK;
}

// Appends the current (converged) state of every slot to the feature rings:
// moments of drho, R drho, R (V_loc - V_loc,gs); writes a training sample when recording;
// assembles x_j for the next prediction once 8 steps are known.
rt_status update_features(rt_ctx* c, SysDev& d) {
  if (!d.feat) return RT_OK;
  hipStream_t s = c->stream;
  const int T = d.T;
  d.mom_head = (d.mom_head + 1) % 8;
  d.cd_cur ^= 1;
  d.cv_head = (d.cv_head + 1) % 3;
  CK(rtk::moments9(s, d.rho, d.rho_gs64, d.nx, d.ny, d.nz, d.h, d.ng, d.mom_part, d.mom_ring + d.mom_head * 9, 72, T));
  CK(rtk::restrict16(s, d.rho, d.rho_gs64, d.cd_ring + d.cd_cur * 4096, d.nx, d.ny, d.nz, d.ng, 2 * 4096, T));
  CK(rtk::restrict16_f64(s, d.vloc, d.vloc_gs, d.cv_ring + d.cv_head * 4096, d.nx, d.ny, d.nz, d.ng, 3 * 4096, T));
  d.n_hist += 1;
  if (c->rec_x && d.x_valid && d.n_hist >= 3 && c->rec_count + T <= c->rec_cap) {
    int inew = d.cv_head, imid = (d.cv_head + 2) % 3, iold = (d.cv_head + 1) % 3;
    CK(rtk::second_diff(s, d.cv_ring, inew, imid, iold, c->rec_y + (long)c->rec_count * kNOut, 3 * 4096, kNOut, T));
    CK(rtk::copy_rows_f(s, d.xbuf, c->rec_x + (long)c->rec_count * kNIn, kNIn, kNIn, kNIn, T));
    c->rec_count += T;
  }
  if (d.n_hist >= 8) {
    CK(rtk::assemble_features(s, d.mom_ring, d.mom_head, d.cd_ring, d.cd_cur, d.cd_cur ^ 1, d.xbuf, kNIn, 72,
                              2 * 4096, T));
    d.x_valid = true;
  }
  return RT_OK;
}

// H1_t += h^3 Psi^T diag(P network(x_t)) Psi for the slots whose network is on.
rt_status predict_correction(rt_ctx* c, SysDev& d) {
  hipStream_t s = c->stream;
  const int T = d.T;
  const long NN = nsq(d.N);
  CK(rtk::mlp_forward(s, pred_dims(), d.mlp_params, d.xbuf, d.ybuf, T, d.mlp_work, false));
  CK(rtk::prolong16(s, d.ybuf, d.dv, d.nx, d.ny, d.nz, kNOut, d.ng, T));
  if (d.mixed) {
    CK(rtk::cast_d2f(s, d.dv32, d.dv, (long)T * d.ng));
    CK(proj_x(s, d, T, d.mlp_mask));
    CK(rtk::reduce_parts_f32(s, d.part32, d.n_split_x, d.N, d.h3, d.H1, d.H1, T, d.mlp_mask, NN));
  } else {
    const long sp = (long)d.n_split * NN;
    CK(rtk::gemm_nt_f64(s, d.N, d.N, d.ng, d.psi, d.ng, d.psi, d.ng, d.dv, d.part, d.kps, d.n_split, 1, d.big,
                        rtk::Batch{T, d.mlp_mask, 0, 0, d.ng, sp}));
    CK(rtk::reduce_parts(s, d.part, d.n_split, d.N, d.N, d.h3, d.H1, 1, d.H1, T, sp, NN, NN, d.mlp_mask));
  }
  return RT_OK;
}

// Number of NaN / infinite entries of a device array (synchronises the stream).
rt_status count_bad(rt_ctx* c, const double* v, long n, unsigned long long* scratch, unsigned long long& bad) {
  CK(rtk::fill_u64(c->stream, scratch, 1, 0ull));
  CK(rtk::count_nonfinite(c->stream, v, n, scratch));
  CK(hipMemcpyAsync(&bad, scratch, sizeof(bad), hipMemcpyDeviceToHost, c->stream));
  CK(hipStreamSynchronize(c->stream));
  return RT_OK;
}

// Scales of the dipole sums: (4 pi / Omega) h^3 on the corrected axes, 0 elsewhere.
rt_status upload_dscale(rt_ctx* c, SysDev& d) {
  const double omega = (double)d.nx * d.ny * d.nz * d.h3;
  double sc[3];
  for (int q = 0; q < 3; ++q) sc[q] = ((d.dcorr >> q) & 1) ? 4.0 * M_PI / omega * d.h3 : 0.0;
  CK(hipMemcpyAsync(d.dscale, sc, sizeof(sc), hipMemcpyHostToDevice, c->stream));
  CK(hipStreamSynchronize(c->stream));
  return RT_OK;
}

rt_status init_system(rt_ctx* c, SysDev& d, const rt_system& s) {
  hipStream_t st = c->stream;
  const long N = d.N, ng = d.ng, NN = N * N;
  CK(hipMemcpyAsync(d.psi, s.psi0, N * ng * sizeof(double),
                    s.psi0_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
  {
    unsigned long long bad = 0;
    RET(count_bad(c, d.psi, N * ng, d.resid, bad));
    if (bad) return fail(c, RT_EINVAL, "psi0 has " + std::to_string(bad) + " non-finite entries");
  }
  std::vector<double> occ(N);
  for (long i = 0; i < N; ++i) occ[i] = s.occ ? s.occ[i] : (i < s.n_occ ? 2.0 : 0.0);
  CK(hipMemcpyAsync(d.occ, occ.data(), N * sizeof(double), hipMemcpyHostToDevice, st));
  double esc[2] = {d.h3, 0.5 * d.h3}, ez[2] = {0.0, 0.0};
  CK(hipMemcpyAsync(d.escale, esc, sizeof(esc), hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(d.ezero, ez, sizeof(ez), hipMemcpyHostToDevice, st));
  RET(upload_dscale(c, d));
  if (d.n_atoms) {
    CK(hipMemcpyAsync(d.pos, s.pos, 3 * d.n_atoms * sizeof(double), hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(d.depth, s.depth, d.n_atoms * sizeof(double), hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(d.width, s.width, d.n_atoms * sizeof(double), hipMemcpyHostToDevice, st));
  }
  RET(upload(c, d.atom_off, d.nl.atom_off));
  RET(upload(c, d.sph_idx, d.nl.sph_idx));
  RET(upload(c, d.beta, d.nl.beta));
  RET(upload(c, d.Dd, d.nl.D));
  RET(upload(c, d.u_idx, d.nl.u_idx));
  RET(upload(c, d.u_ptr, d.nl.u_ptr));
  RET(upload(c, d.ent_pt, d.nl.ent_pt));
  RET(upload(c, d.ent_atom, d.nl.ent_atom));
  CK(rtk::twiddles(st, d.twx, d.nx));
  CK(rtk::twiddles(st, d.twy, d.ny));
  CK(rtk::twiddles(st, d.twz, d.nz));
  if (s.orthonormalize) {
    // S = h^3 Psi Psi^T = L L^T;  Psi <- L^-1 Psi
    RET(project(c, d, d.psi, d.psi, nullptr, d.tmp));
    CK(rtk::cholesky(st, d.tmp, d.N, d.info));
    int info = 0;
    CK(hipMemcpyAsync(&info, d.info, sizeof(int), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    if (info) return fail(c, RT_EINVAL, "orbital overlap matrix is not positive definite");
    CK(rtk::tri_inverse_lower(st, d.tmp, d.tmp2, d.N));
    CK(rtk::smalltall_f64(st, d.N, d.ng, d.tmp2, d.psi, d.hpsi, 0, 2, 1, nullptr));
    std::swap(d.psi, d.hpsi);
  }
  CK(rtk::vion(st, d.vion, d.nx, d.ny, d.nz, d.h, d.n_atoms, d.pos, d.depth, d.width, d.n_images));
  for (int q = 0; q < 3; ++q) {
    CK(rtk::coord(st, d.dv, d.nx, d.ny, d.nz, d.h, q, d.jump[q]));
    RET(project(c, d, d.psi, d.psi, d.dv, d.M3 + q * NN));
  }
  if (d.hb == d.N) {
    RET(apply_h64(c, d, d.psi, d.hpsi, d.vion, d.N));
    RET(project(c, d, d.psi, d.hpsi, nullptr, d.hcore));
  } else {
    // H_core by blocks of hb orbitals J: rows J of X = h^3 (H Psi_J) Psi^T, then
    // H_core = (X + X^T) / 2.  A block's product has few 64 x 64 tiles, so K is split
    // further (~2048 blocks), within the partial-sum buffer.
    const long tiles = (long)((d.hb + 63) / 64) * ((d.N + 63) / 64);
    const long room = (long)std::max(d.n_split, d.n_split_cap) * NN / ((long)d.hb * d.N);
    const long nsb = std::max(1L, std::min({(2048 + tiles - 1) / tiles, room, std::max(1L, ng / 1024)}));
    const long kpb = ((ng + nsb - 1) / nsb + 15) / 16 * 16;
    const int nspb = (int)((ng + kpb - 1) / kpb);
    for (int j0 = 0; j0 < d.N; j0 += d.hb) {
      const int nb = std::min(d.hb, d.N - j0);
      RET(apply_h64(c, d, d.psi + (long)j0 * ng, d.hpsi, d.vion, nb));
      {
        Timed tm(c, PH_PROJECT);
        CK(rtk::gemm_nt_f64(st, nb, d.N, ng, d.hpsi, ng, d.psi, ng, nullptr, d.part, kpb, nspb, 0, d.big,
                            rtk::single()));
      }
      CK(rtk::reduce_parts(st, d.part, nspb, nb, d.N, d.h3, d.tmp2 + (long)j0 * N, 0, nullptr, 1, 0, 0, 0,
                           nullptr));
    }
    CK(rtk::transpose(st, d.tmp2, d.tmp, d.N));
    CK(rtk::lincomb(st, d.hcore, 0.5, d.tmp2, 0.5, d.tmp, NN));
  }
  // ground-state Hamiltonian H_gs = H[P_gs] with the full FP64 apply (slot 0 fields);
  // P_gs = diag(f), or for a non-orthogonal basis with overlap S = h^3 Phi Phi^T = L L^T:
  // S^-1 = L^-T L^-1 and P_gs = L^-T diag(f) L^-1 (the occupations of the basis
  // orthonormalised by L, written in the given basis; Appendix transformation rules)
  std::vector<double> pgs(NN, 0.0);
  for (long i = 0; i < N; ++i) pgs[i * N + i] = occ[i];
  if (d.nonorth) {
    RET(project(c, d, d.psi, d.psi, nullptr, d.Sov));
    CK(rtk::copy_d(st, d.tmp, d.Sov, NN));
    CK(rtk::cholesky(st, d.tmp, d.N, d.info));
    int info = 0;
    CK(hipMemcpyAsync(&info, d.info, sizeof(int), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    if (info) return fail(c, RT_EINVAL, "basis overlap matrix is not positive definite");
    CK(rtk::tri_inverse_lower(st, d.tmp, d.tmp2, d.N));
    CK(rtk::transpose(st, d.tmp2, d.tmp, d.N));  // X = L^-T
    CK(rtk::gemm_nt_f64(st, d.N, d.N, d.N, d.tmp, d.N, d.tmp, d.N, nullptr, d.Sinv, d.N, 1, 0, 0, rtk::single()));
    CK(rtk::gemm_nt_f64(st, d.N, d.N, d.N, d.tmp, d.N, d.tmp, d.N, d.occ, d.tmp2, d.N, 1, 0, 0, rtk::single()));
    CK(rtk::copy_d(st, d.tmp, d.tmp2, NN));
  } else {
    CK(hipMemcpyAsync(d.tmp, pgs.data(), NN * sizeof(double), hipMemcpyHostToDevice, st));
  }
  std::vector<int> one(1, 1);
  RET(eval_h(c, d, 1, nullptr, one, d.tmp, NN, d.Hgs, true));
  CK(rtk::copy_d(st, d.vloc_gs, d.vloc, d.ng));
  CK(rtk::copy_d(st, d.rho_gs64, d.rho, d.ng));
  if (d.mlp) {
    CK(hipMemcpyAsync(d.mlp_params, c->run.mlp_params, rtk::mlp_n_params(pred_dims()) * sizeof(float),
                      hipMemcpyHostToDevice, st));
  }
  if (d.feat) CK(hipMemcpyAsync(d.mlp_mask, d.mlp_on.data(), d.T * sizeof(int), hipMemcpyHostToDevice, st));
  if (d.mixed) {
    CK(rtk::copy_d(st, d.rho_gs, d.rho, d.ng));
    CK(rtk::copy_d(st, d.S_gs, d.tmp, NN));
    if (d.N <= rtk::proj_tri_max_n())
      CK(rtk::split_bf16_kb(st, d.psi, d.psi_hi, d.psi_lo, d.N, ng));
    else
      CK(rtk::split_bf16(st, d.psi, d.psi_hi, d.psi_lo, N * ng));
    if (d.psiT_hi) CK(rtk::split_bf16_t(st, d.psi, d.psiT_hi, d.psiT_lo, (int)N, d.wld, ng));
  }
  // trajectories: P_0 = P_gs, then each slot's kick through the series
  std::vector<double> p0((long)d.T * 2 * NN, 0.0);
  if (!d.nonorth)
    for (int t = 0; t < d.T; ++t)
      for (long i = 0; i < N; ++i) p0[(long)t * 2 * NN + i * N + i] = occ[i];
  CK(hipMemcpyAsync(d.P1, p0.data(), p0.size() * sizeof(double), hipMemcpyHostToDevice, st));
  if (d.nonorth)
    for (int t = 0; t < d.T; ++t) CK(rtk::copy_d(st, d.P1 + (long)t * 2 * NN, d.tmp, NN));
  CK(rtk::copy_d(st, d.P0, d.P1, (long)d.T * 2 * NN));
  for (int t = 0; t < d.T; ++t) {
    int g = d.slot_traj[t];
    if (g < 0) continue;
    const TrajDev& tr = c->traj[g];
    if (tr.kappa == 0.0) continue;
    // delta kick: exp(-i kappa M_q) P_0 exp(+i kappa M_q), same series with Hbar = M_q, dt = kappa
    CK(rtk::copy_d(st, d.Hbar + t * NN, d.M3 + tr.axis * NN, NN));
    std::vector<int> terms, on(1, 1);
    RET(series(c, d, t, 1, nullptr, on, d.Hbar + t * NN, tr.kappa, d.P1 + t * 2 * NN, d.P0 + t * 2 * NN, terms));
  }
  {
    // pulse parameters per slot (zero amplitude where the trajectory has no field)
    std::vector<double> fp((long)d.T * 7, 0.0);
    d.field = false;
    for (int t = 0; t < d.T; ++t) {
      int g = d.slot_traj[t];
      if (g < 0) continue;
      for (int q = 0; q < 7; ++q) fp[7L * t + q] = c->traj[g].field[q];
      d.field = d.field || fp[7L * t] != 0.0;
    }
    CK(hipMemcpyAsync(d.fieldp, fp.data(), fp.size() * sizeof(double), hipMemcpyHostToDevice, st));
    CK(hipStreamSynchronize(st));
  }
  std::vector<int> all(d.T, 1);
  RET(eval_h(c, d, d.T, nullptr, all, d.P0, 2 * NN, d.H0, false));
  CK(rtk::copy_d(st, d.Hm1, d.H0, (long)d.T * NN));
  CK(rtk::copy_d(st, d.Hm2, d.H0, (long)d.T * NN));
  d.step = 0;
  RET(observe(c, d, 0));
  RET(update_features(c, d));
  CK(hipStreamSynchronize(st));  // host vectors above must outlive their copies
  return RT_OK;
}

// One lockstep time step of every trajectory of a system (Algorithm 1 time loop body).
// One time step of every system with trajectories.  The systems advance through the
// self-consistency rounds together: each round launches every live system's series
// start, waits once for all their stop flags, then launches every live system's
// Hamiltonian update and waits once for all residuals, so the host round trips per
// step do not grow with the number of molecules.
struct StepState {
  bool predicted = false;
  int n_active = 0;
  std::vector<int> m_of, terms_of, terms;
  std::vector<double> res_of;
};

rt_status step_prologue(rt_ctx* c, SysDev& d, StepState& ss) {
  hipStream_t st = c->stream;
  const rt_run& run = c->run;
  const long NN = nsq(d.N);
  const int T = d.T;
  // first guess of H(t + dt): linear extrapolation 2 H_0 - H_-1 (Algorithm 1), or the
  // quadratic one 3 H_0 - 3 H_-1 + H_-2 (error O(dt^3) instead of O(dt^2))
  if (run.predictor == RT_PRED_QUADRATIC)
    CK(rtk::lincomb3(st, d.H1, 3.0, d.H0, -3.0, d.Hm1, 1.0, d.Hm2, T * NN));
  else
    CK(rtk::lincomb(st, d.H1, 2.0, d.H0, -1.0, d.Hm1, T * NN));
  ss.predicted = false;
  if (d.mlp && d.x_valid) {
    bool any = false;
    for (int t = 0; t < T; ++t) any = any || d.mlp_on[t];
    if (any) {
      RET(predict_correction(c, d));
      ss.predicted = true;
    }
  }
  d.active_host.assign(T, 1);
  RET(push_active(c, d));
  CK(rtk::fill(st, d.tcur, 1, d.step * run.dt));  // t_j for the field terms of this step
  ss.m_of.assign(T, 0);
  ss.terms_of.assign(T, 0);
  ss.res_of.assign(T, 0.0);
  ss.n_active = T;
  return RT_OK;
}

// Hamiltonian update and its residual: one captured sequence (the host loops over
// trajectories in the full-apply mode, so the active pattern is part of the key)
rt_status launch_update(rt_ctx* c, SysDev& d) {
  const long NN = nsq(d.N);
  const int T = d.T;
  auto update = [&]() -> rt_status {
    RET(eval_h(c, d, T, d.active, d.active_host, d.P1, 2 * NN, d.Hn, false));
    {
      Timed tm(c, PH_SMALL);
      CK(rtk::max_diff_assign(c->stream, d.Hn, d.H1, NN, d.resid, T, d.active));
    }
    return enqueue_publish(c, d, d.resid, T * sizeof(unsigned long long));
  };
  std::vector<uintptr_t> key{2, (uintptr_t)T, (uintptr_t)d.P1, (uintptr_t)d.H1};
  // the captured sequence depends on the host's copy of the active flags only where
  // launches are made per active trajectory (FP64 full updates, frozen potentials);
  // elsewhere every kernel reads the device flags, so one graph serves every mask
  if (c->run.frozen_hxc || (!d.mixed && c->run.hupdate == RT_HUPDATE_FULL))
    for (int t = 0; t < T; ++t) key.push_back((uintptr_t)d.active_host[t]);
  return run_graph(c, d, key, update);
}

// after the wait for launch_update's publish: residuals, convergence, learned-guess fallback
rt_status process_update(rt_ctx* c, SysDev& d, StepState& ss, int m) {
  const rt_run& run = c->run;
  const int T = d.T;
  std::vector<unsigned long long> bits(T);
  slot_read(c, d, T * sizeof(unsigned long long), bits.data());
  bool changed = false;
  bool mask_changed = false;
  for (int t = 0; t < T; ++t) {
    if (!d.active_host[t]) continue;
    double r;
    std::memcpy(&r, &bits[t], sizeof(r));
    if (m == 1 && d.mlp) {
      if (ss.predicted && d.mlp_on[t]) {
        // fallback: the network's first residual against the median of linear first residuals
        std::vector<double> v = d.r1_linear[t];
        if (!v.empty()) {
          std::nth_element(v.begin(), v.begin() + v.size() / 2, v.end());
          if (r > 10.0 * v[v.size() / 2]) { d.mlp_on[t] = 0; mask_changed = true; }
        }
      } else {
        d.r1_linear[t].push_back(r);
      }
    }
    if (!std::isfinite(r))
      return fail(c, RT_ENOCONV, "non-finite Hamiltonian (residual " + std::to_string(r) + ") in trajectory " +
                                     std::to_string(d.slot_traj[t]));
    ss.m_of[t] = m;
    ss.terms_of[t] += ss.terms[t];
    ss.res_of[t] = r;
    if (r <= run.h_thrs) {
      d.active_host[t] = 0;
      --ss.n_active;
      changed = true;
    }
  }
  if (changed && ss.n_active > 0) RET(push_active(c, d));
  if (mask_changed) RET(upload_flags(c, d.mlp_mask, d.mlp_on));
  return RT_OK;
}

rt_status step_epilogue(rt_ctx* c, SysDev& d, StepState& ss, rt_step_stats* stats) {
  const int T = d.T;
  // H_-2 <- H_-1, H_-1 <- H_0, H_0 <- H_1, P_0 <- P_1 (all slots together)
  double* old_m2 = d.Hm2;
  d.Hm2 = d.Hm1;
  d.Hm1 = d.H0;
  d.H0 = d.H1;
  d.H1 = old_m2;
  std::swap(d.P0, d.P1);
  d.step += 1;
  if (stats) {
    for (int t = 0; t < T; ++t) {
      int g = d.slot_traj[t];
      if (g < 0) continue;
      stats[g].scf_iters = ss.m_of[t];
      stats[g].series_terms = ss.terms_of[t];
      stats[g].residual = ss.res_of[t];
    }
  }
  RET(observe(c, d, d.step));
  RET(update_features(c, d));
  return RT_OK;
}

rt_status step_all(rt_ctx* c, rt_step_stats* stats) {
  const rt_run& run = c->run;
  std::vector<SysDev*> sv;
  for (auto& d : c->sys)
    if (d.slot_traj[0] >= 0) sv.push_back(&d);  // systems without trajectories stay put
  const int n = (int)sv.size();
  // several systems run on their own streams, joined to the caller's stream at both ends
  if (n > 1) {
    CK(hipEventRecord(c->join, c->stream));
    for (SysDev* d : sv) CK(hipStreamWaitEvent(d->sst, c->join, 0));
  }
  std::vector<StepState> ss(n);
  for (int i = 0; i < n; ++i) {
    OnStream on(c, stream_of(c, *sv[i]));
    RET(step_prologue(c, *sv[i], ss[i]));
  }
  for (int m = 1; m <= run.max_scf; ++m) {
    std::vector<int> live;
    std::vector<SysDev*> lv;
    for (int i = 0; i < n; ++i)
      if (ss[i].n_active > 0) {
        live.push_back(i);
        lv.push_back(sv[i]);
      }
    if (live.empty()) break;
    std::vector<std::unique_ptr<Series>> sr(n);
    for (int i : live) {
      SysDev& d = *sv[i];
      OnStream on(c, stream_of(c, d));
      sr[i].reset(new Series(c, d, 0, d.T, d.active, d.Hbar, run.dt, d.P0, d.P1, d.H0, d.H1, d.resid, d.tcur));
      RET(sr[i]->start());
    }
    RET(wait_slots(c, lv));
    for (int i : live) {
      OnStream on(c, stream_of(c, *sv[i]));
      RET(sr[i]->complete(sv[i]->active_host, ss[i].terms));
    }
    for (int i : live) {
      OnStream on(c, stream_of(c, *sv[i]));
      RET(launch_update(c, *sv[i]));
    }
    RET(wait_slots(c, lv));
    for (int i : live) {
      OnStream on(c, stream_of(c, *sv[i]));
      RET(process_update(c, *sv[i], ss[i], m));
    }
  }
  for (int i = 0; i < n; ++i)
    if (ss[i].n_active > 0) return fail(c, RT_ENOCONV, "self-consistent Hamiltonian loop reached max_scf");
  for (int i = 0; i < n; ++i) {
    OnStream on(c, stream_of(c, *sv[i]));
    RET(step_epilogue(c, *sv[i], ss[i], stats));
  }
  if (n > 1) {
    for (SysDev* d : sv) {
      CK(hipEventRecord(d->ev, d->sst));
      CK(hipStreamWaitEvent(c->stream, d->ev, 0));
    }
  }
  return RT_OK;
}

// ---------------------------------------------------------------------------
// Dense symmetric eigensolver (Rayleigh-Ritz step of the ground-state solve,
// also exported as rt_eigh): parallel cyclic Jacobi sweeps until the
// off-diagonal Frobenius norm is below 1e-15 of the matrix norm.
// ---------------------------------------------------------------------------
struct EighWork {
  int n = 0, ld = 0;
  double *A = nullptr, *A2 = nullptr, *V = nullptr, *off = nullptr;
  int* rank = nullptr;
};

void eigh_layout(Arena& a, EighWork& w, int n) {
  w.n = n;
  w.ld = n + (n & 1);
  const long LL = (long)w.ld * w.ld;
  w.A = a.take<double>(LL);
  w.A2 = a.take<double>(LL);
  w.V = a.take<double>(LL);
  w.off = a.take<double>(3);
  w.rank = a.take<int>(w.ld);
}

constexpr int kMaxSweeps = 60;

// evals[k] ascending, vecs row k its eigenvector; *sweeps the sweeps taken.
rt_status eigh_run(rt_ctx* c, EighWork& w, const double* A, double* evals, double* vecs, int* sweeps) {
  hipStream_t st = c->stream;
  CK(rtk::jacobi_setup(st, A, w.n, w.ld, w.A, w.V));
  if (w.ld <= rtk::jacobi_small_max()) {
    // one block holds the matrix in LDS and runs every sweep
    double stat[3] = {0.0, 0.0, 0.0};
    CK(rtk::jacobi_small(st, w.A, w.V, w.ld, kMaxSweeps, w.off));
    CK(hipMemcpyAsync(stat, w.off, sizeof(stat), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    if (!std::isfinite(stat[2])) return fail(c, RT_EINVAL, "eigensolver: matrix has non-finite entries");
    if (!std::isfinite(stat[1])) return fail(c, RT_ENOCONV, "eigensolver: non-finite iterate");
    if ((int)stat[0] >= kMaxSweeps && stat[1] > 1e-26 * stat[2])
      return fail(c, RT_ENOCONV, "eigensolver: Jacobi sweeps did not converge");
    CK(rtk::jacobi_sort(st, w.A, w.V, w.n, w.ld, evals, vecs, w.rank));
    if (sweeps) *sweeps = (int)stat[0];
    return RT_OK;
  }
  double* a = w.A;
  double* b = w.A2;
  double off[2] = {0.0, 0.0};
  CK(rtk::jacobi_offdiag(st, a, w.ld, w.off));
  CK(hipMemcpyAsync(off, w.off, sizeof(off), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  const double total = off[0] + off[1];  // Frobenius norm^2, invariant under the rotations
  if (!std::isfinite(total)) return fail(c, RT_EINVAL, "eigensolver: matrix has non-finite entries");
  int sw = 0;
  double prev = off[0];
  while (off[0] > 1e-30 * total) {
    if (sw == kMaxSweeps) return fail(c, RT_ENOCONV, "eigensolver: Jacobi sweeps did not converge");
    for (int r = 0; r < w.ld - 1; ++r) {
      CK(rtk::jacobi_round(st, a, b, w.V, w.ld, r));
      std::swap(a, b);
    }
    ++sw;
    CK(rtk::jacobi_offdiag(st, a, w.ld, w.off));
    CK(hipMemcpyAsync(off, w.off, sizeof(off), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    if (!std::isfinite(off[0])) return fail(c, RT_ENOCONV, "eigensolver: non-finite iterate");
    // rounding floor: no longer shrinking once at the level of a few ulps
    if (off[0] <= 1e-26 * total && off[0] > 0.25 * prev) break;
    prev = off[0];
  }
  CK(rtk::jacobi_sort(st, a, w.V, w.n, w.ld, evals, vecs, w.rank));
  if (sweeps) *sweeps = sw;
  return RT_OK;
}

// ---------------------------------------------------------------------------
// Ground state: Chebyshev-filtered subspace iteration (Zhou, Saad, Tiago and
// Chelikowsky, J. Comput. Phys. 219, 172 (2006)) inside a Pulay-mixed density
// loop.  The system's grid operator is the one of the time step (stencil,
// V_loc, projectors); the orbital block holds nb = N + n_guard vectors.
// ---------------------------------------------------------------------------
struct GsDev {
  double* blk[3] = {nullptr, nullptr, nullptr};  // orbital blocks [nb][ng]
  double *Hs = nullptr, *vecs = nullptr, *evals = nullptr, *res = nullptr, *occ = nullptr;
  double *rho_out = nullptr, *hin = nullptr, *hres = nullptr, *Bp = nullptr, *coef = nullptr, *dpart = nullptr;
  double* rpart = nullptr;  // residual partial sums [nb][row_residual_parts()]
  unsigned long long* slot = nullptr;
  EighWork eig;
  int depth = 1;
};

void layout_gs(Arena& a, SysDev& d, GsDev& g) {
  const long ng = d.ng, nb = d.N, NN = nb * nb;
  for (auto& p : g.blk) p = a.take<double>(nb * ng);
  d.vion = a.take<double>(ng);
  d.z = a.take<double2>(ng);
  d.twx = a.take<double2>(d.nx);
  d.twy = a.take<double2>(d.ny);
  d.twz = a.take<double2>(d.nz);
  d.pos = a.take<double>(3 * std::max(1, d.n_atoms));
  d.depth = a.take<double>(std::max(1, d.n_atoms));
  d.width = a.take<double>(std::max(1, d.n_atoms));
  d.atom_off = a.take<int>(d.nl.atom_off.size() + 1);
  d.sph_idx = a.take<int>(d.nl.sph_idx.size() + 1);
  d.beta = a.take<double>(d.nl.beta.size() + 1);
  d.Dd = a.take<double>(d.nl.D.size() + 1);
  d.u_idx = a.take<int>(d.nl.u_idx.size() + 1);
  d.u_ptr = a.take<int>(d.nl.u_ptr.size() + 1);
  d.ent_pt = a.take<int>(d.nl.ent_pt.size() + 1);
  d.ent_atom = a.take<int>(d.nl.ent_atom.size() + 1);
  d.cnl = a.take<double>(nb * std::max(1, d.nl.n_proj));
  d.tmp = a.take<double>(NN);
  d.tmp2 = a.take<double>(NN);
  d.info = a.take<int>(4);
  d.red2 = a.take<double>(2 * rtk::kRedBlocks);
  d.escale = a.take<double>(2);
  d.eparts = a.take<double>(2);
  d.dscale = a.take<double>(3);
  d.dfield = a.take<double>(3);
  d.dpart = a.take<double>(d.dcorr ? 3 * rtk::kRedBlocks : 1);
  d.rho = a.take<double>(ng);
  d.vh = a.take<double>(ng);
  d.vx = a.take<double>(ng);
  d.vloc = a.take<double>(ng);
  d.part = a.take<double>(d.n_split * NN);
  g.Hs = a.take<double>(NN);
  g.vecs = a.take<double>(NN);
  g.evals = a.take<double>(nb);
  g.res = a.take<double>(nb);
  g.rpart = a.take<double>(nb * rtk::row_residual_parts());
  g.occ = a.take<double>(nb);
  g.rho_out = a.take<double>(ng);
  g.hin = a.take<double>(g.depth * ng);
  g.hres = a.take<double>(g.depth * ng);
  g.Bp = a.take<double>(64);
  g.coef = a.take<double>(8);
  g.dpart = a.take<double>(8 * 256);
  g.slot = a.take<unsigned long long>(1);
  eigh_layout(a, g.eig, (int)nb);
}

rt_status validate_gs(const rt_system* s, const rt_gs_params* p, std::string& why) {
  if (!s || !p) { why = "null system or parameters"; return RT_EINVAL; }
  RET(validate_system(*s, why));
  if (s->nonorthogonal || s->orthonormalize) { why = "the ground state takes neither nonorthogonal nor orthonormalize"; return RT_EINVAL; }
  const int N = s->n_occ + s->n_virt;
  if (p->n_guard < 2 || N + p->n_guard > 1024) { why = "n_guard >= 2 and N + n_guard <= 1024"; return RT_EINVAL; }
  if (p->degree < 1 || p->degree > 64) { why = "degree outside [1, 64]"; return RT_EINVAL; }
  if (p->max_scf < 1 || p->max_passes < 1) { why = "max_scf and max_passes must be >= 1"; return RT_EINVAL; }
  if (!(p->tol_rho > 0) || !(p->tol_res > 0)) { why = "tolerances must be positive"; return RT_EINVAL; }
  if (!(p->mix > 0 && p->mix <= 1)) { why = "mix outside (0, 1]"; return RT_EINVAL; }
  if (p->pulay_depth < 1 || p->pulay_depth > 8) { why = "pulay_depth outside [1, 8]"; return RT_EINVAL; }
  if (s->occ)
    for (int i = 0; i < N; ++i)
      if (!std::isfinite(s->occ[i])) { why = "occupations must be finite"; return RT_EINVAL; }
  return RT_OK;
}

void describe_gs(const rt_system* s, const rt_gs_params* p, SysDev& d, GsDev& g) {
  rt_run r{};
  r.precision = RT_FP64;
  std::vector<SysDev> S;
  std::vector<TrajDev> T;
  describe(s, 1, &r, S, T);
  d = std::move(S[0]);
  d.N = s->n_occ + s->n_virt + p->n_guard;  // block size: wanted pairs + guard vectors
  choose_split(d);
  g.depth = p->pulay_depth;
}

// Upper bound of the spectrum of H = T + V_loc + V_nl: the FD kinetic symbol is
// largest at the zone corner, |T| <= (1/2) h^-2 3 (|a_0| + 2 sum_k |a_k|) (the
// alternating signs of the coefficients make this exact); V_loc <= max|V_loc|;
// ||V_nl|| <= max_a sum_b sqrt(d_a g_a d_b g_b) over atoms b whose spheres share a
// grid point with a's (d: largest |D| of an atom, g: Gershgorin bound of its
// projector Gram matrix h^3 beta^T beta), a block Gershgorin bound.
double kinetic_max(const SysDev& d) {
  double s = std::fabs(d.coef[0]);
  for (int k = 1; k <= 4; ++k) s += 2.0 * std::fabs(d.coef[k]);
  return 0.5 * 3.0 * s / (d.h * d.h);
}

double nonlocal_bound(const SysDev& d) {
  const NlTables& t = d.nl;
  if (!t.rank || !t.n_atoms) return 0.0;
  const int na = t.n_atoms, R = t.rank;
  std::vector<double> dg(na, 0.0);
  for (int a = 0; a < na; ++a) {
    double dm = 0.0, gm = 0.0;
    for (int p = 0; p < R; ++p) dm = std::max(dm, std::fabs(t.D[a * R + p]));
    std::vector<double> G(R * R, 0.0);
    for (int e = t.atom_off[a]; e < t.atom_off[a + 1]; ++e)
      for (int p = 0; p < R; ++p)
        for (int q = 0; q < R; ++q) G[p * R + q] += t.beta[(long)e * R + p] * t.beta[(long)e * R + q];
    for (int p = 0; p < R; ++p) {
      double row = 0.0;
      for (int q = 0; q < R; ++q) row += std::fabs(G[p * R + q]) * d.h3;
      gm = std::max(gm, row);
    }
    dg[a] = dm * gm;
  }
  std::vector<char> adj((size_t)na * na, 0);
  for (int a = 0; a < na; ++a) adj[(size_t)a * na + a] = 1;
  for (size_t u = 0; u + 1 < t.u_ptr.size(); ++u)
    for (int e = t.u_ptr[u]; e < t.u_ptr[u + 1]; ++e)
      for (int f = t.u_ptr[u]; f < t.u_ptr[u + 1]; ++f)
        adj[(size_t)t.ent_atom[e] * na + t.ent_atom[f]] = 1;
  double nu = 0.0;
  for (int a = 0; a < na; ++a) {
    double row = 0.0;
    for (int b = 0; b < na; ++b)
      if (adj[(size_t)a * na + b]) row += std::sqrt(dg[a] * dg[b]);
    nu = std::max(nu, row);
  }
  return nu;
}

struct GsRun {
  rt_ctx* c;
  SysDev& d;
  GsDev& g;
  int N;
  int cur = 0;                       // block holding the current Ritz vectors
  double a0 = 0, acut = 0, bup = 0;  // filter: damped interval [acut, bup], scale point a0
  double static_bound = 0;           // kinetic + nonlocal part of bup
  std::vector<double> ev, res;
  long applies = 0;
  int passes = 0, eighs = 0;
  long sweeps = 0;
  GsRun(rt_ctx* c_, SysDev& d_, GsDev& g_, int N_) : c(c_), d(d_), g(g_), N(N_) {}

  rt_status apply(const double* x, double* y) {
    ++applies;
    return apply_h64(c, d, x, y, d.vloc, d.N);
  }

  // bup from the current V_loc
  rt_status bound() {
    hipStream_t st = c->stream;
    CK(rtk::fill_u64(st, g.slot, 1, 0ull));
    CK(rtk::abs_max(st, d.vloc, d.ng, g.slot));
    unsigned long long bits = 0;
    CK(hipMemcpyAsync(&bits, g.slot, 8, hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    double vmax;
    std::memcpy(&vmax, &bits, 8);
    bup = static_bound + vmax;
    bup += 1e-12 * std::fabs(bup);
    return RT_OK;
  }

  // block i <- its h^3-orthonormal basis by Cholesky QR, twice (j: scratch block)
  rt_status orth(int i, int j) {
    hipStream_t st = c->stream;
    const int nb = d.N;
    for (int pass = 0; pass < 2; ++pass) {
      double* src = g.blk[pass ? j : i];
      double* dst = g.blk[pass ? i : j];
      RET(project(c, d, src, src, nullptr, d.tmp));
      if (nb <= rtk::jacobi_small_max()) {
        CK(rtk::chol_inv_small(st, d.tmp, d.tmp2, nb, d.info + pass));
      } else {
        CK(rtk::cholesky(st, d.tmp, nb, d.info + pass));
        CK(rtk::tri_inverse_lower(st, d.tmp, d.tmp2, nb));
      }
      CK(rtk::smalltall_f64(st, nb, d.ng, d.tmp2, src, dst, 0, 2, 1, nullptr));
    }
    int info[2] = {0, 0};
    CK(hipMemcpyAsync(info, d.info, sizeof(info), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    if (info[0] || info[1]) return fail(c, RT_ENOCONV, "ground state: the orbital block lost rank");
    return RT_OK;
  }

  // Rayleigh-Ritz on the orthonormal block i: Ritz vectors and values, residual norms
  rt_status ritz(int i) {
    hipStream_t st = c->stream;
    const int nb = d.N, j = (i + 1) % 3, k = (i + 2) % 3;
    RET(apply(g.blk[i], g.blk[k]));
    RET(project(c, d, g.blk[i], g.blk[k], nullptr, g.Hs));
    int sw = 0;
    RET(eigh_run(c, g.eig, g.Hs, g.evals, g.vecs, &sw));
    sweeps += sw;
    ++eighs;
    CK(rtk::smalltall_f64(st, nb, d.ng, g.vecs, g.blk[i], g.blk[j], 0, 0, 1, nullptr));  // X
    CK(rtk::smalltall_f64(st, nb, d.ng, g.vecs, g.blk[k], g.blk[i], 0, 0, 1, nullptr));  // H X
    CK(rtk::row_residuals(st, g.blk[i], g.blk[j], g.evals, nb, d.ng, d.h3, g.res, g.rpart));
    ev.resize(nb);
    res.resize(nb);
    CK(hipMemcpyAsync(ev.data(), g.evals, nb * 8, hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(res.data(), g.res, nb * 8, hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    for (int q = 0; q < nb; ++q)
      if (!std::isfinite(ev[q]) || !std::isfinite(res[q])) return fail(c, RT_ENOCONV, "ground state: non-finite Ritz pairs");
    cur = j;
    a0 = ev[0];
    acut = ev[nb - 1];
    return RT_OK;
  }

  // Scaled Chebyshev filter of degree m on block cur (the damped interval
  // [acut, bup] maps to [-1, 1], the scale point a0 to -1/sigma_1); returns the
  // block that holds the filtered vectors.
  rt_status filter(int m, int& out) {
    if (!(bup > acut)) return fail(c, RT_ENOCONV, "ground state: Ritz value above the spectral bound");
    const long n = (long)d.N * d.ng;
    const double e = 0.5 * (bup - acut), cc = 0.5 * (bup + acut);
    double lo = a0;
    if (!(lo < acut - 1e-12 * e)) lo = acut - 0.05 * e;
    double sigma = e / (lo - cc);
    const double tau = 2.0 / sigma;
    int x = cur, y = (cur + 1) % 3, z = (cur + 2) % 3;
    RET(apply(g.blk[x], g.blk[z]));
    CK(rtk::lincomb(c->stream, g.blk[y], sigma / e, g.blk[z], -sigma * cc / e, g.blk[x], n));
    for (int k = 2; k <= m; ++k) {
      const double sn = 1.0 / (tau - sigma);
      RET(apply(g.blk[y], g.blk[z]));
      CK(rtk::lincomb3(c->stream, g.blk[x], 2.0 * sn / e, g.blk[z], -2.0 * sn * cc / e, g.blk[y], -sigma * sn,
                       g.blk[x], n));
      std::swap(x, y);
      sigma = sn;
    }
    out = y;
    return RT_OK;
  }

  rt_status pass(int m) {
    int f = 0;
    RET(filter(m, f));
    RET(orth(f, (f + 1) % 3));
    RET(ritz(f));
    ++passes;
    return RT_OK;
  }

  double wanted_res() const {
    double r = 0.0;
    for (int q = 0; q < N; ++q) r = std::max(r, res[q]);
    return r;
  }

  // filter passes at fixed V_loc until the wanted residuals are below tol
  rt_status solve(int m, double tol, int max_passes) {
    for (int p = 0; p < max_passes; ++p) {
      RET(pass(m));
      if (wanted_res() <= tol) return RT_OK;
    }
    return RT_OK;
  }

  double read_slot() {
    unsigned long long bits = 0;
    if (hipMemcpyAsync(&bits, g.slot, 8, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
      return NAN;
    double v;
    std::memcpy(&v, &bits, 8);
    return v;
  }
};

rt_status gs_run(rt_ctx* c, SysDev& d, GsDev& g, const rt_system& s, const rt_gs_params& p, double* psi_out,
                 double* eps_out, double* rho_out, rt_gs_stats* stats) {
  hipStream_t st = c->stream;
  const int N = s.n_occ + s.n_virt, nb = d.N;
  const long ng = d.ng;
  // static fields and tables
  double esc[2] = {d.h3, 0.5 * d.h3};
  CK(hipMemcpyAsync(d.escale, esc, sizeof(esc), hipMemcpyHostToDevice, st));
  RET(upload_dscale(c, d));
  if (d.n_atoms) {
    CK(hipMemcpyAsync(d.pos, s.pos, 3 * d.n_atoms * sizeof(double), hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(d.depth, s.depth, d.n_atoms * sizeof(double), hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(d.width, s.width, d.n_atoms * sizeof(double), hipMemcpyHostToDevice, st));
  }
  RET(upload(c, d.atom_off, d.nl.atom_off));
  RET(upload(c, d.sph_idx, d.nl.sph_idx));
  RET(upload(c, d.beta, d.nl.beta));
  RET(upload(c, d.Dd, d.nl.D));
  RET(upload(c, d.u_idx, d.nl.u_idx));
  RET(upload(c, d.u_ptr, d.nl.u_ptr));
  RET(upload(c, d.ent_pt, d.nl.ent_pt));
  RET(upload(c, d.ent_atom, d.nl.ent_atom));
  CK(rtk::twiddles(st, d.twx, d.nx));
  CK(rtk::twiddles(st, d.twy, d.ny));
  CK(rtk::twiddles(st, d.twz, d.nz));
  CK(rtk::vion(st, d.vion, d.nx, d.ny, d.nz, d.h, d.n_atoms, d.pos, d.depth, d.width, d.n_images));
  std::vector<double> occ(nb, 0.0);
  for (int i = 0; i < N; ++i) occ[i] = s.occ ? s.occ[i] : (i < s.n_occ ? 2.0 : 0.0);
  CK(hipMemcpyAsync(g.occ, occ.data(), nb * sizeof(double), hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(g.blk[0], s.psi0, (size_t)nb * ng * sizeof(double),
                    s.psi0_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
  {
    unsigned long long bad = 0;
    RET(count_bad(c, g.blk[0], (long)nb * ng, g.slot, bad));
    if (bad) return fail(c, RT_EINVAL, "start block has " + std::to_string(bad) + " non-finite entries");
  }
  CK(rtk::fill(st, g.Bp, 64, 0.0));

  GsRun R(c, d, g, N);
  R.static_bound = kinetic_max(d) + nonlocal_bound(d);
  const int m = p.degree;
  // start: the given block, orthonormalised, and its Ritz pairs for V_loc = V_ion
  RET(R.orth(0, 1));
  CK(rtk::copy_d(st, d.vloc, d.vion, ng));
  RET(R.bound());
  RET(R.ritz(0));
  RET(R.solve(m, std::max(1e-2, p.tol_res), p.max_passes));
  CK(rtk::occ_density(st, g.blk[R.cur], g.occ, nb, ng, d.rho));
  // density loop: V_loc[rho_in] -> filtered Ritz pairs -> rho_out, Pulay-mixed
  double err = INFINITY;
  int it = 0, count = 0;
  bool conv = false;
  for (it = 1; it <= p.max_scf; ++it) {
    RET(poisson_lda(c, d, 1, nullptr));
    RET(R.bound());
    RET(R.solve(m, std::max(p.tol_res, std::min(1e-2, 0.1 * err)), p.max_passes));
    CK(rtk::occ_density(st, g.blk[R.cur], g.occ, nb, ng, g.rho_out));
    const int sn = count % g.depth;
    double* hres = g.hres + (long)sn * ng;
    CK(rtk::lincomb(st, hres, 1.0, g.rho_out, -1.0, d.rho, ng));
    CK(rtk::copy_d(st, g.hin + (long)sn * ng, d.rho, ng));
    CK(rtk::fill_u64(st, g.slot, 1, 0ull));
    CK(rtk::abs_max(st, hres, ng, g.slot));
    err = R.read_slot();
    if (!std::isfinite(err)) return fail(c, RT_ENOCONV, "ground state: non-finite density");
    if (err < p.tol_rho) {
      conv = true;
      break;
    }
    ++count;
    const int mm = std::min(count, g.depth);
    CK(rtk::pulay_dots(st, g.hres, mm, sn, ng, g.dpart));
    CK(rtk::pulay_solve(st, g.dpart, mm, sn, g.depth, g.Bp, g.coef));
    CK(rtk::pulay_mix(st, g.hin, g.hres, g.coef, mm, p.mix, ng, d.rho));
  }
  auto report = [&](double rho_err, double res) {
    if (eps_out) std::copy(R.ev.begin(), R.ev.end(), eps_out);
    if (stats) {
      stats->scf_iters = std::min(it, p.max_scf);
      stats->filter_passes = R.passes;
      stats->h_applies = R.applies;
      stats->eigensolves = R.eighs;
      stats->jacobi_sweeps = R.sweeps;
      stats->rho_err = rho_err;
      stats->residual = res;
    }
  };
  if (!conv) {
    // the last iterate, for diagnosis or as an approximate ground state: its Ritz
    // vectors (signs fixed) and their density
    double* X = g.blk[R.cur];
    CK(rtk::fix_signs(st, X, N, ng));
    CK(hipMemcpyAsync(psi_out, X, (size_t)N * ng * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (rho_out) {
      CK(rtk::occ_density(st, X, g.occ, nb, ng, g.rho_out));
      CK(hipMemcpyAsync(rho_out, g.rho_out, ng * sizeof(double), hipMemcpyDeviceToDevice, st));
    }
    CK(hipStreamSynchronize(st));
    report(err, R.wanted_res());
    return fail(c, RT_ENOCONV, "ground state: density loop hit max_scf");
  }
  // final orbitals: eigenpairs of H[rho_in] at the converged input density
  RET(poisson_lda(c, d, 1, nullptr));
  RET(R.bound());
  RET(R.solve(m, p.tol_res, p.max_passes));
  const double res = R.wanted_res();
  if (!(res <= p.tol_res)) return fail(c, RT_ENOCONV, "ground state: eigen-residual above tol_res after max_passes");
  double* X = g.blk[R.cur];
  CK(rtk::fix_signs(st, X, N, ng));
  CK(rtk::occ_density(st, X, g.occ, nb, ng, g.rho_out));
  CK(rtk::lincomb(st, g.hres, 1.0, g.rho_out, -1.0, d.rho, ng));
  CK(rtk::fill_u64(st, g.slot, 1, 0ull));
  CK(rtk::abs_max(st, g.hres, ng, g.slot));
  const double rho_err = R.read_slot();
  CK(hipMemcpyAsync(psi_out, X, (size_t)N * ng * sizeof(double), hipMemcpyDeviceToDevice, st));
  if (rho_out) CK(hipMemcpyAsync(rho_out, g.rho_out, ng * sizeof(double), hipMemcpyDeviceToDevice, st));
  CK(hipStreamSynchronize(st));
  report(rho_err, res);
  return RT_OK;
}

// ---------------------------------------------------------------------------
// Checkpoints: every value the next step reads, per system in context order.
// Layout: header {magic, version, n_sys, hist_cap}; per system: shape and counters
// (N, T, nx, ny, nz, step, feat, mlp, mom_head, cd_cur, cv_head, n_hist, x_valid),
// mlp_on[T], per slot the fallback history (count, then doubles); then the arrays
// P_0 [T][2N^2], H_0, H_-1, H_-2 [T][N^2], the observables [T][step + 1][5], and
// with features the moment ring, coarse density and potential rings and the
// assembled feature vector.
// ---------------------------------------------------------------------------
constexpr uint32_t kCkptMagic = 0x4b435452u;  // "RTCK"
constexpr uint32_t kCkptVersion = 1;

struct CkptWriter {
  char* p;
  size_t n = 0, cap;
  bool sizing;
  void put(const void* src, size_t bytes) {
    if (!sizing && n + bytes <= cap) std::memcpy(p + n, src, bytes);
    n += bytes;
  }
  template <class V>
  void val(const V& v) { put(&v, sizeof(V)); }
};

struct CkptReader {
  const char* p;
  size_t n = 0, cap;
  bool ok = true;
  const char* take(size_t bytes) {
    if (!ok || n + bytes > cap) { ok = false; return nullptr; }
    const char* r = p + n;
    n += bytes;
    return r;
  }
  template <class V>
  V val() {
    V v{};
    if (const char* r = take(sizeof(V))) std::memcpy(&v, r, sizeof(V));
    return v;
  }
};

struct CkptArray {
  const void* dev;
  size_t bytes;
};

// device arrays of system d in checkpoint order (hist rows: step + 1 of each slot)
std::vector<CkptArray> ckpt_arrays(const rt_ctx* c, const SysDev& d) {
  const size_t NN = (size_t)d.N * d.N, T = d.T;
  std::vector<CkptArray> a{{d.P0, T * 2 * NN * 8}, {d.H0, T * NN * 8}, {d.Hm1, T * NN * 8}, {d.Hm2, T * NN * 8}};
  for (int t = 0; t < d.T; ++t) a.push_back({d.hist + (size_t)t * 5 * (c->hist_cap + 1), (size_t)5 * (d.step + 1) * 8});
  if (d.feat) {
    a.push_back({d.mom_ring, T * 72 * 4});
    a.push_back({d.cd_ring, T * 2 * 4096 * 4});
    a.push_back({d.cv_ring, T * 3 * 4096 * 8});
    a.push_back({d.xbuf, T * (size_t)kNIn * 4});
  }
  return a;
}

// Serialises (w.sizing) or writes the checkpoint; device arrays are copied with
// dev_copy(host_offset, array).
template <class F>
void ckpt_walk(const rt_ctx* c, CkptWriter& w, F&& dev_copy) {
  w.val(kCkptMagic);
  w.val(kCkptVersion);
  w.val((int32_t)c->sys.size());
  w.val((int32_t)c->hist_cap);
  for (const SysDev& d : c->sys) {
    const int32_t hdr[13] = {d.N, d.T, d.nx, d.ny, d.nz, d.step, d.feat, d.mlp, d.mom_head, d.cd_cur, d.cv_head,
                             d.n_hist, d.x_valid};
    w.put(hdr, sizeof(hdr));
    for (int t = 0; t < d.T; ++t) w.val((int32_t)d.mlp_on[t]);
    for (int t = 0; t < d.T; ++t) {
      w.val((int64_t)d.r1_linear[t].size());
      w.put(d.r1_linear[t].data(), d.r1_linear[t].size() * sizeof(double));
    }
    for (const CkptArray& a : ckpt_arrays(c, d)) {
      if (!w.sizing && w.n + a.bytes <= w.cap) dev_copy(w.n, a);
      w.n += a.bytes;
    }
  }
}

// ---------------------------------------------------------------------------
// Autotuner: each tunable launch shape of a system is timed over its candidates
// on the context's own buffers (hipEvents on the context's stream, one warm-up
// and three timed launches each) and the fastest kept.  Choices are cached in a
// text file, one line per (GPU architecture, kernel, grid, N, trajectories):
// "key value1 value2 value3"; a later context with the same key takes the cached
// value without timing.  The stencil tiling changes no arithmetic; the projection
// splits change the order of the partial sums (results within rounding).
// ---------------------------------------------------------------------------
enum { TUNE_STENCIL64 = 0, TUNE_STENCIL32 = 1, TUNE_PROJ64 = 2, TUNE_PROJ_MIXED = 3 };
const char* kTuneNames[4] = {"stencil_fp64", "stencil_fp32", "projection_fp64", "projection_bf16x3"};

std::string tune_arch() {
  int dev = 0;
  hipDeviceProp_t p;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
  std::string a = p.gcnArchName;
  return a.substr(0, a.find(':'));
}

std::string tune_key(const std::string& arch, int kernel, const SysDev& d) {
  char b[160];
  std::snprintf(b, sizeof(b), "%s|%s|%dx%dx%d|N%d|T%d", arch.c_str(), kTuneNames[kernel], d.nx, d.ny, d.nz, d.N,
                d.T);
  return b;
}

std::map<std::string, std::vector<int>> tune_cache_read(const char* path) {
  std::map<std::string, std::vector<int>> m;
  if (!path) return m;
  FILE* f = std::fopen(path, "r");
  if (!f) return m;
  char line[512];
  while (std::fgets(line, sizeof(line), f)) {
    char key[256];
    int v0 = 0, v1 = 0, v2 = 0;
    if (std::sscanf(line, "%255s %d %d %d", key, &v0, &v1, &v2) >= 3) m[key] = {v0, v1, v2};
  }
  std::fclose(f);
  return m;
}

void drop_graphs(SysDev& d) {
  for (auto& kv : d.graphs) (void)hipGraphExecDestroy(kv.second);
  d.graphs.clear();
}

// applies a launch shape (validated); the projections re-split
rt_status tune_apply(rt_ctx* c, SysDev& d, int kernel, int p1, int p2, int p3) {
  if (p3 && kernel != TUNE_STENCIL64 && kernel != TUNE_STENCIL32)
    return fail(c, RT_EINVAL, "the projections take no third launch parameter");
  switch (kernel) {
    case TUNE_STENCIL64:
    case TUNE_STENCIL32: {
      std::vector<int> ty, nz, hq;
      if (kernel == TUNE_STENCIL64) rtk::stencil_tiles<double>(d.nx, d.ny, d.nz, d.N, ty, nz);
      else rtk::stencil_tiles<float>(d.nx, d.ny, d.nz, d.N, ty, nz);
      rtk::stencil_halo_ahead(hq);
      if ((p1 && std::find(ty.begin(), ty.end(), p1) == ty.end()) || p2 < 0 || p2 > d.nz ||
          (p3 && std::find(hq.begin(), hq.end(), p3) == hq.end()))
        return fail(c, RT_EINVAL, "stencil tiling (y rows " + std::to_string(p1) + ", z chunks " +
                                      std::to_string(p2) + ", halo look-ahead " + std::to_string(p3) +
                                      ") not available on this grid");
      d.st_ty[kernel] = p1;
      d.st_nzc[kernel] = p2;
      d.st_hq[kernel] = p3;
      break;
    }
    case TUNE_PROJ64:
      if (p1 && std::find(std::begin(kGemmTargets), std::end(kGemmTargets), p1) == std::end(kGemmTargets))
        return fail(c, RT_EINVAL, "FP64 projection target must be 0, 1024, 2048 or 4096 blocks");
      d.gemm_target = p1;
      choose_split(d);
      break;
    case TUNE_PROJ_MIXED:
      if (!d.mixed || d.N > rtk::proj_tri_max_n())
        return fail(c, RT_EINVAL, "the BF16x3 triangle projection is not used by this system");
      if (p1 && std::find(std::begin(kTriSplits), std::end(kTriSplits), p1) == std::end(kTriSplits))
        return fail(c, RT_EINVAL, "BF16x3 projection splits must be 0, 85, 128, 170 or 255");
      d.tri_splits = p1;
      choose_split_tri(d);
      break;
    default:
      return fail(c, RT_EINVAL, "unknown tunable kernel");
  }
  drop_graphs(d);  // captured sequences hold the old launch shapes
  return RT_OK;
}

// average device milliseconds of one call of f (one warm-up, three timed)
template <class F>
rt_status tune_time(rt_ctx* c, F&& f, double& ms) {
  hipEvent_t a = nullptr, b = nullptr;
  CK(hipEventCreate(&a));
  CK(hipEventCreate(&b));
  rt_status st = f();
  if (st == RT_OK) {
    CK(hipEventRecord(a, c->stream));
    for (int i = 0; i < 3 && st == RT_OK; ++i) st = f();
    CK(hipEventRecord(b, c->stream));
    CK(hipEventSynchronize(b));
    float e = 0.f;
    CK(hipEventElapsedTime(&e, a, b));
    ms = e / 3.0;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return st;
}

// one launch of the tunable kernel as the time step runs it
rt_status tune_run(rt_ctx* c, SysDev& d, int kernel) {
  hipStream_t s = c->stream;
  const long NN = nsq(d.N);
  switch (kernel) {
    case TUNE_STENCIL64:
      CK(rtk::stencil<double>(s, d.psi, d.hpsi, d.vloc_gs, d.hb, d.nx, d.ny, d.nz, d.h, d.coef, d.st_ty[0],
                              d.st_nzc[0], d.st_hq[0]));
      return RT_OK;
    case TUNE_STENCIL32: {
      float* in = reinterpret_cast<float*>(d.hpsi);  // FP32 copy of hb orbitals, then the output
      CK(rtk::stencil<float>(s, in, in + (long)d.hb * d.ng, d.vloc32, d.hb, d.nx, d.ny, d.nz, d.h, d.coef, d.st_ty[1],
                             d.st_nzc[1], d.st_hq[1]));
      return RT_OK;
    }
    case TUNE_PROJ64:
      if (c->run.hupdate == RT_HUPDATE_FULL) return project(c, d, d.psi, d.hpsi, nullptr, d.Hn);
      {
        const long sp = (long)d.n_split * NN;
        CK(rtk::gemm_nt_f64(s, d.N, d.N, d.ng, d.psi, d.ng, d.psi, d.ng, d.dv, d.part, d.kps, d.n_split, 1, d.big,
                            rtk::Batch{d.T, nullptr, 0, 0, d.ng, sp}));
        CK(rtk::reduce_parts(s, d.part, d.n_split, d.N, d.N, d.h3, d.Hn, 1, d.Hgs, d.T, sp, 0, NN, nullptr));
      }
      return RT_OK;
    default:
      CK(proj_x(s, d, d.T, nullptr));
      CK(rtk::reduce_parts_f32(s, d.part32, d.n_split_x, d.N, d.h3, d.Hgs, d.Hn, d.T, nullptr, 0));
      return RT_OK;
  }
}

rt_status autotune_system(rt_ctx* c, SysDev& d, int si, const std::string& arch,
                          std::map<std::string, std::vector<int>>& cache, FILE* out, std::string& rep) {
  hipStream_t s = c->stream;
  std::vector<int> kernels{TUNE_STENCIL64, TUNE_STENCIL32};
  if (!d.mixed) kernels.push_back(TUNE_PROJ64);
  if (d.mixed && d.N <= rtk::proj_tri_max_n()) kernels.push_back(TUNE_PROJ_MIXED);
  // inputs of the timed launches: FP32 orbitals and potential, the ground-state
  // potential change (zero) as projection weights
  CK(rtk::cast_d2f(s, reinterpret_cast<float*>(d.hpsi), d.psi, (long)d.hb * d.ng));
  CK(rtk::cast_d2f(s, d.vloc32, d.vloc_gs, d.ng));
  if (!d.mixed) CK(rtk::sub_d(s, d.dv, d.vloc, d.vloc_gs, d.ng, d.T, nullptr));
  else CK(rtk::delta_f32(s, d.dv32, d.vloc, d.vloc_gs, d.ng, d.T, nullptr));
  for (int k : kernels) {
    const std::string key = tune_key(arch, k, d);
    auto it = cache.find(key);
    char line[320];
    if (it != cache.end()) {
      RET(tune_apply(c, d, k, it->second[0], it->second[1], it->second[2]));
      std::snprintf(line, sizeof(line), "system %d %s: %d %d %d (cached)\n", si, kTuneNames[k], it->second[0],
                    it->second[1], it->second[2]);
      rep += line;
      continue;
    }
    // candidates (p1, p2, p3); for the stencils the halo look-ahead is swept in a
    // second round at the best tiling of the first
    std::vector<std::array<int, 3>> cand;
    std::vector<int> hq;
    const bool stencil = k == TUNE_STENCIL64 || k == TUNE_STENCIL32;
    if (stencil) {
      std::vector<int> ty, nz;
      if (k == TUNE_STENCIL64) rtk::stencil_tiles<double>(d.nx, d.ny, d.nz, d.N, ty, nz);
      else rtk::stencil_tiles<float>(d.nx, d.ny, d.nz, d.N, ty, nz);
      rtk::stencil_halo_ahead(hq);
      cand.push_back({0, 0, 0});
      for (int a : ty)
        for (int b : nz) cand.push_back({a, b, 0});
    } else if (k == TUNE_PROJ64) {
      cand.push_back({0, 0, 0});
      for (int v : kGemmTargets) cand.push_back({v, 0, 0});
    } else {
      cand.push_back({0, 0, 0});
      for (int v : kTriSplits) cand.push_back({v, 0, 0});
    }
    double best = 1e300, t_def = 0.0;
    std::array<int, 3> pick{0, 0, 0};
    size_t n_cand = 0;
    for (int round = 0; round < (stencil ? 2 : 1); ++round) {
      if (round == 1) {
        cand.clear();
        for (int v : hq) cand.push_back({pick[0], pick[1], v});
      }
      for (auto& p : cand) {
        // a shape the kernel refuses (LDS) is skipped
        if (tune_apply(c, d, k, p[0], p[1], p[2]) != RT_OK) continue;
        double ms = 0.0;
        rt_status st = tune_time(c, [&] { return tune_run(c, d, k); }, ms);
        if (st != RT_OK) {
          if (p[2] == 0) return st;  // the tilings of the first round all launch
          (void)hipGetLastError();
          continue;
        }
        ++n_cand;
        if (p[0] == 0 && p[1] == 0 && p[2] == 0) t_def = ms;
        if (ms < best) { best = ms; pick = p; }
      }
    }
    c->err.clear();
    RET(tune_apply(c, d, k, pick[0], pick[1], pick[2]));
    cache[key] = {pick[0], pick[1], pick[2]};
    if (out) std::fprintf(out, "%s %d %d %d\n", key.c_str(), pick[0], pick[1], pick[2]);
    std::snprintf(line, sizeof(line), "system %d %s: %d %d %d, %.1f us (built-in choice %.1f us, %zu candidates)\n",
                  si, kTuneNames[k], pick[0], pick[1], pick[2], 1e3 * best, 1e3 * t_def, n_cand);
    rep += line;
  }
  return RT_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

rt_status rt_workspace_size(const rt_system* sys, int n_sys, const rt_run* run, size_t* bytes) {
  std::string why;
  if (!bytes) { g_init_error = "bytes is NULL"; return RT_EINVAL; }
  rt_status st = validate(sys, n_sys, run, why);
  if (st != RT_OK) { g_init_error = why; return st; }
  std::vector<SysDev> S;
  std::vector<TrajDev> T;
  describe(sys, n_sys, run, S, T);
  Arena a;
  layout(a, S, *run, run->n_steps_max);
  *bytes = a.used + 256;
  return RT_OK;
}

rt_status rt_init(const rt_system* sys, int n_sys, const rt_run* run, void* workspace_dev, size_t ws_bytes,
                  void* hip_stream, rt_ctx** out) {
  if (!out) { g_init_error = "out is NULL"; return RT_EINVAL; }
  *out = nullptr;
  std::string why;
  rt_status st = validate(sys, n_sys, run, why);
  if (st != RT_OK) { g_init_error = why; return st; }
  if (!workspace_dev) { g_init_error = "workspace is NULL"; return RT_EINVAL; }
  rt_ctx* c = new rt_ctx();
  c->stream = (hipStream_t)hip_stream;
  c->run = *run;
  c->run.traj_sys = nullptr;
  c->run.traj_kappa = nullptr;
  c->run.traj_axis = nullptr;
  c->hist_cap = run->n_steps_max;
  describe(sys, n_sys, run, c->sys, c->traj);
  Arena a;
  layout(a, c->sys, *run, c->hist_cap);
  size_t need = a.used + 256;
  if (ws_bytes < need) {
    g_init_error = "workspace too small: need " + std::to_string(need) + " bytes";
    delete c;
    return RT_ENOMEM;
  }
  Arena b;
  b.base = reinterpret_cast<char*>(((uintptr_t)workspace_dev + 255) & ~uintptr_t(255));
  layout(b, c->sys, *run, c->hist_cap);
  size_t words = 0;
  for (SysDev& d : c->sys) {
    d.box_off = (int)words;  // even: the 8-byte sequence word stays aligned
    words += 2 * (size_t)d.T + 4;
  }
  c->box_bytes = (64 + 4 * words + 4095) / 4096 * 4096;
  void* box = nullptr;
  if (hipHostMalloc(&box, c->box_bytes, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
      hipHostGetDevicePointer((void**)&c->box_dev, box, 0) != hipSuccess) {
    if (box) (void)hipHostFree(box);
    g_init_error = "rt_init: pinned host mailbox";
    delete c;
    return RT_ENOMEM;
  }
  c->box_host = static_cast<unsigned*>(box);
  std::memset(c->box_host, 0, c->box_bytes);
  for (SysDev& d : c->sys)
    if (rtk::fill_u64(c->stream, d.box_ctr, 1, 0ull) != hipSuccess) {
      g_init_error = "rt_init: mailbox counter";
      delete c;
      return RT_EDEVICE;
    }
  {
    int n_stepped = 0;
    for (SysDev& d : c->sys) n_stepped += d.slot_traj[0] >= 0;
    if (n_stepped > 1) {
      bool ok = hipEventCreateWithFlags(&c->join, hipEventDisableTiming) == hipSuccess;
      for (SysDev& d : c->sys) {
        if (d.slot_traj[0] < 0) continue;
        ok = ok && hipStreamCreateWithFlags(&d.sst, hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&d.ev, hipEventDisableTiming) == hipSuccess;
      }
      if (!ok) {
        g_init_error = "rt_init: system streams";
        delete c;
        return RT_EDEVICE;
      }
    }
  }
  if (run->graph_capture && hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess) {
    c->cap = nullptr;
    g_init_error = "rt_init: capture stream";
    delete c;
    return RT_EDEVICE;
  }
  for (int i = 0; i < n_sys; ++i) {
    st = init_system(c, c->sys[i], sys[i]);
    if (st != RT_OK) { g_init_error = c->err; delete c; return st; }
  }
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    g_init_error = std::string("rt_init: ") + hipGetErrorString(e);
    delete c;
    return RT_EDEVICE;
  }
  c->graphs = run->graph_capture != 0;  // the one-off kicks of init ran eagerly
  *out = c;
  return RT_OK;
}

rt_status rt_apply_h(rt_ctx* c, int si, const void* psi_dev, void* hpsi_dev, int n_orb, int dtype) {
  if (!c) return RT_EINVAL;
  if (si < 0 || si >= (int)c->sys.size()) return fail(c, RT_EINVAL, "sys_index out of range");
  if (!psi_dev || !hpsi_dev || n_orb < 0 || (dtype != 0 && dtype != 1))
    return fail(c, RT_EINVAL, "rt_apply_h arguments");
  SysDev& d = c->sys[si];
  size_t esz = dtype == 0 ? 8 : 4;
  uintptr_t p0 = (uintptr_t)psi_dev, p1 = (uintptr_t)hpsi_dev, len = (uintptr_t)n_orb * d.ng * esz;
  if (n_orb > 0 && p0 < p1 + len && p1 < p0 + len) return fail(c, RT_EINVAL, "psi and hpsi must not overlap");
  if (dtype == 1) CK(rtk::cast_d2f(c->stream, d.vloc32, d.vloc, d.ng));
  for (int o = 0; o < n_orb; o += d.N) {
    int n = std::min(d.N, n_orb - o);
    if (dtype == 0)
      RET(apply_h64(c, d, (const double*)psi_dev + (long)o * d.ng, (double*)hpsi_dev + (long)o * d.ng, d.vloc, n));
    else
      RET(apply_h32(c, d, (const float*)psi_dev + (long)o * d.ng, (float*)hpsi_dev + (long)o * d.ng, n));
  }
  return RT_OK;
}

rt_status rt_step(rt_ctx* c, int n_steps, rt_step_stats* stats) {
  if (!c) return RT_EINVAL;
  if (n_steps < 0) return fail(c, RT_EINVAL, "n_steps < 0");
  for (auto& d : c->sys)
    if (d.step + n_steps > c->hist_cap) return fail(c, RT_ESTATE, "history capacity n_steps_max exhausted");
  const int nt = (int)c->traj.size();
  for (int k = 0; k < n_steps; ++k) RET(step_all(c, stats ? stats + (long)k * nt : nullptr));
  if (c->prof) {
    CK(hipStreamSynchronize(c->stream));
    prof_collect(c);
  }
  return RT_OK;
}

rt_status rt_profile(rt_ctx* c, int enable, int reset) {
  if (!c) return RT_EINVAL;
  CK(hipStreamSynchronize(c->stream));
  prof_collect(c);
  if (reset) {
    for (int i = 0; i < PH_COUNT; ++i) { c->prof_ms[i] = 0.0; c->prof_n[i] = 0; }
  }
  c->prof = enable != 0;
  return RT_OK;
}

rt_status rt_profile_read(rt_ctx* c, int phase, double* total_ms, long* launches, const char** name) {
  if (!c) return RT_EINVAL;
  if (phase < 0 || phase >= PH_COUNT) return fail(c, RT_EINVAL, "phase out of range");
  CK(hipStreamSynchronize(c->stream));
  prof_collect(c);
  if (total_ms) *total_ms = c->prof_ms[phase];
  if (launches) *launches = c->prof_n[phase];
  if (name) *name = kPhaseNames[phase];
  return RT_OK;
}

rt_status rt_dipole(rt_ctx* c, int traj, int first_step, int count, double* mu_host, double* energy_host,
                    double* trace_host) {
  if (!c) return RT_EINVAL;
  if (traj < 0 || traj >= (int)c->traj.size()) return fail(c, RT_EINVAL, "traj out of range");
  TrajDev& t = c->traj[traj];
  SysDev& d = c->sys[t.sys];
  if (first_step < 0 || count < 0 || first_step + count > d.step + 1 || !mu_host)
    return fail(c, RT_EINVAL, "requested steps outside the recorded history");
  std::vector<double> buf(5L * count);
  const double* src = d.hist + (long)t.slot * 5L * (c->hist_cap + 1) + 5L * first_step;
  if (count) CK(hipMemcpyAsync(buf.data(), src, buf.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  CK(hipStreamSynchronize(c->stream));
  for (int i = 0; i < count; ++i) {
    for (int q = 0; q < 3; ++q) mu_host[3 * i + q] = buf[5 * i + q];
    if (energy_host) energy_host[i] = buf[5 * i + 3];
    if (trace_host) trace_host[i] = buf[5 * i + 4];
  }
  return RT_OK;
}

rt_status rt_get_matrix(rt_ctx* c, int traj, int which, double* out) {
  if (!c) return RT_EINVAL;
  if (traj < 0 || traj >= (int)c->traj.size() || !out) return fail(c, RT_EINVAL, "rt_get_matrix arguments");
  TrajDev& t = c->traj[traj];
  SysDev& d = c->sys[t.sys];
  const long NN = nsq(d.N);
  const double* src = nullptr;
  switch (which) {
    case 0: src = d.H0 + t.slot * NN; break;
    case 1: src = d.Hm1 + t.slot * NN; break;
    case 2: src = d.P0 + t.slot * 2 * NN; break;
    case 3: src = d.P0 + t.slot * 2 * NN + NN; break;
    case 4: src = d.hcore; break;
    case 5: case 6: case 7: src = d.M3 + (which - 5) * NN; break;
    case 8: src = d.Hgs; break;
    default: return fail(c, RT_EINVAL, "unknown matrix");
  }
  CK(hipMemcpyAsync(out, src, NN * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  CK(hipStreamSynchronize(c->stream));
  return RT_OK;
}

rt_status rt_set_state(rt_ctx* c, int traj, const double* p_re, const double* p_im, const double* h0,
                       const double* hm1) {
  if (!c) return RT_EINVAL;
  if (traj < 0 || traj >= (int)c->traj.size()) return fail(c, RT_EINVAL, "traj out of range");
  TrajDev& t = c->traj[traj];
  SysDev& d = c->sys[t.sys];
  const long NN = nsq(d.N);
  hipStream_t s = c->stream;
  for (const double* m : {p_re, p_im, h0, hm1})
    if (m)
      for (long e = 0; e < NN; ++e)
        if (!std::isfinite(m[e])) return fail(c, RT_EINVAL, "rt_set_state: non-finite matrix entry");
  if (p_re) CK(hipMemcpyAsync(d.P0 + t.slot * 2 * NN, p_re, NN * 8, hipMemcpyHostToDevice, s));
  if (p_im) CK(hipMemcpyAsync(d.P0 + t.slot * 2 * NN + NN, p_im, NN * 8, hipMemcpyHostToDevice, s));
  if (h0) CK(hipMemcpyAsync(d.H0 + t.slot * NN, h0, NN * 8, hipMemcpyHostToDevice, s));
  if (hm1) {
    CK(hipMemcpyAsync(d.Hm1 + t.slot * NN, hm1, NN * 8, hipMemcpyHostToDevice, s));
    CK(hipMemcpyAsync(d.Hm2 + t.slot * NN, hm1, NN * 8, hipMemcpyHostToDevice, s));
  }
  CK(hipStreamSynchronize(s));
  return RT_OK;
}

rt_status rt_autotune(rt_ctx* c, const char* cache_path) {
  if (!c) return RT_EINVAL;
  const std::string arch = tune_arch();
  auto cache = tune_cache_read(cache_path);
  FILE* out = cache_path ? std::fopen(cache_path, "a") : nullptr;
  std::string rep = "architecture " + arch + "\n";
  rt_status st = RT_OK;
  for (size_t i = 0; i < c->sys.size() && st == RT_OK; ++i) st = autotune_system(c, c->sys[i], (int)i, arch, cache, out, rep);
  if (out) std::fclose(out);
  c->tune_report = rep;
  if (st == RT_OK) CK(hipStreamSynchronize(c->stream));
  return st;
}

rt_status rt_tune_set(rt_ctx* c, int si, int kernel, int p1, int p2, int p3) {
  if (!c) return RT_EINVAL;
  if (si < 0 || si >= (int)c->sys.size()) return fail(c, RT_EINVAL, "sys_index out of range");
  return tune_apply(c, c->sys[si], kernel, p1, p2, p3);
}

rt_status rt_tune_get(rt_ctx* c, int si, int kernel, int* p1, int* p2, int* p3) {
  if (!c || !p1 || !p2 || !p3) return RT_EINVAL;
  if (si < 0 || si >= (int)c->sys.size()) return fail(c, RT_EINVAL, "sys_index out of range");
  const SysDev& d = c->sys[si];
  *p3 = 0;
  switch (kernel) {
    case TUNE_STENCIL64: case TUNE_STENCIL32:
      *p1 = d.st_ty[kernel]; *p2 = d.st_nzc[kernel]; *p3 = d.st_hq[kernel]; break;
    case TUNE_PROJ64: *p1 = d.gemm_target; *p2 = d.n_split; break;
    case TUNE_PROJ_MIXED: *p1 = d.tri_splits; *p2 = d.n_split_x; break;
    default: return fail(c, RT_EINVAL, "unknown tunable kernel");
  }
  return RT_OK;
}

const char* rt_tune_report(const rt_ctx* c) { return c ? c->tune_report.c_str() : ""; }

rt_status rt_checkpoint_size(rt_ctx* c, size_t* bytes) {
  if (!c || !bytes) return RT_EINVAL;
  CkptWriter w{nullptr, 0, 0, true};
  ckpt_walk(c, w, [](size_t, const CkptArray&) {});
  *bytes = w.n;
  return RT_OK;
}

rt_status rt_checkpoint_save(rt_ctx* c, void* host, size_t bytes) {
  if (!c || !host) return RT_EINVAL;
  size_t need = 0;
  RET(rt_checkpoint_size(c, &need));
  if (bytes < need) return fail(c, RT_ENOMEM, "rt_checkpoint_save: buffer of " + std::to_string(bytes) +
                                                   " bytes, need " + std::to_string(need));
  CkptWriter w{static_cast<char*>(host), 0, bytes, false};
  hipError_t err = hipSuccess;
  ckpt_walk(c, w, [&](size_t off, const CkptArray& a) {
    if (err == hipSuccess && a.bytes)
      err = hipMemcpyAsync(static_cast<char*>(host) + off, a.dev, a.bytes, hipMemcpyDeviceToHost, c->stream);
  });
  CK(err);
  CK(hipStreamSynchronize(c->stream));
  return RT_OK;
}

rt_status rt_checkpoint_load(rt_ctx* c, const void* host, size_t bytes) {
  if (!c || !host) return RT_EINVAL;
  // validate everything before anything is changed
  CkptReader r{static_cast<const char*>(host), 0, bytes};
  if (r.val<uint32_t>() != kCkptMagic || r.val<uint32_t>() != kCkptVersion)
    return fail(c, RT_EINVAL, "rt_checkpoint_load: not a checkpoint of this library version");
  if (r.val<int32_t>() != (int32_t)c->sys.size()) return fail(c, RT_EINVAL, "rt_checkpoint_load: system count differs");
  r.val<int32_t>();  // the saving context's history capacity (any)
  struct SysState {
    int32_t hdr[13];
    std::vector<int> mlp_on;
    std::vector<std::vector<double>> r1;
    size_t arrays_at;
  };
  std::vector<SysState> st(c->sys.size());
  for (size_t i = 0; i < c->sys.size(); ++i) {
    const SysDev& d = c->sys[i];
    SysState& x = st[i];
    const char* h = r.take(sizeof(x.hdr));
    if (!h) break;
    std::memcpy(x.hdr, h, sizeof(x.hdr));
    if (x.hdr[0] != d.N || x.hdr[1] != d.T || x.hdr[2] != d.nx || x.hdr[3] != d.ny || x.hdr[4] != d.nz ||
        x.hdr[6] != (int)d.feat || x.hdr[7] != (int)d.mlp)
      return fail(c, RT_EINVAL, "rt_checkpoint_load: system " + std::to_string(i) + " has a different shape or mode");
    if (x.hdr[5] < 0 || x.hdr[5] > c->hist_cap)
      return fail(c, RT_EINVAL, "rt_checkpoint_load: step beyond this context's history capacity");
    x.mlp_on.resize(d.T);
    for (int t = 0; t < d.T; ++t) x.mlp_on[t] = r.val<int32_t>();
    x.r1.resize(d.T);
    for (int t = 0; t < d.T; ++t) {
      const int64_t k = r.val<int64_t>();
      if (k < 0 || k > (int64_t)(1L << 30)) { r.ok = false; break; }
      const char* v = r.take((size_t)k * sizeof(double));
      if (!v) break;
      x.r1[t].resize(k);
      std::memcpy(x.r1[t].data(), v, (size_t)k * sizeof(double));
    }
    x.arrays_at = r.n;
    // arrays: sizes as this context would write them at the saved step
    SysDev probe = d;
    probe.step = x.hdr[5];
    for (const CkptArray& a : ckpt_arrays(c, probe))
      if (!r.take(a.bytes)) break;
  }
  if (!r.ok || r.n != bytes) return fail(c, RT_EINVAL, "rt_checkpoint_load: truncated or oversized checkpoint");
  for (size_t i = 0; i < c->sys.size(); ++i) {
    SysDev& d = c->sys[i];
    const SysState& x = st[i];
    d.step = x.hdr[5];
    d.mom_head = x.hdr[8];
    d.cd_cur = x.hdr[9];
    d.cv_head = x.hdr[10];
    d.n_hist = x.hdr[11];
    d.x_valid = x.hdr[12] != 0;
    d.mlp_on = x.mlp_on;
    d.r1_linear = x.r1;
    size_t off = x.arrays_at;
    for (const CkptArray& a : ckpt_arrays(c, d)) {
      if (a.bytes)
        CK(hipMemcpyAsync(const_cast<void*>(a.dev), static_cast<const char*>(host) + off, a.bytes,
                          hipMemcpyHostToDevice, c->stream));
      off += a.bytes;
    }
    if (d.feat) RET(upload_flags(c, d.mlp_mask, d.mlp_on));
  }
  CK(hipStreamSynchronize(c->stream));
  return RT_OK;
}

rt_status rt_eval_h(rt_ctx* c, int si, const double* p_re_dev, double* h_out_dev) {
  if (!c) return RT_EINVAL;
  if (si < 0 || si >= (int)c->sys.size() || !p_re_dev || !h_out_dev) return fail(c, RT_EINVAL, "rt_eval_h arguments");
  std::vector<int> one(1, 1);
  return eval_h(c, c->sys[si], 1, nullptr, one, p_re_dev, 0, h_out_dev, false);
}

rt_status rt_propagate(rt_ctx* c, int si, const double* hbar_dev, double dt, double* p_re_dev, double* p_im_dev,
                       int* terms_out) {
  if (!c) return RT_EINVAL;
  if (si < 0 || si >= (int)c->sys.size() || !hbar_dev || !p_re_dev || !p_im_dev)
    return fail(c, RT_EINVAL, "rt_propagate arguments");
  SysDev& d = c->sys[si];
  const long NN = nsq(d.N);
  hipStream_t s = c->stream;
  // slot 0's work buffers: input in Hn/Hbar-free scratch (C), output in P1; the state P0 is untouched
  double* in = d.C;
  double* outp = d.P1;
  CK(hipMemcpyAsync(in, p_re_dev, NN * 8, hipMemcpyDeviceToDevice, s));
  CK(hipMemcpyAsync(in + NN, p_im_dev, NN * 8, hipMemcpyDeviceToDevice, s));
  std::vector<int> terms, one(1, 1);
  const bool g = c->graphs;
  c->graphs = false;  // caller-owned buffers: not worth a graph per pointer set
  const rt_status st = series(c, d, 0, 1, nullptr, one, hbar_dev, dt, in, outp, terms);
  c->graphs = g;
  RET(st);
  CK(hipMemcpyAsync(p_re_dev, outp, NN * 8, hipMemcpyDeviceToDevice, s));
  CK(hipMemcpyAsync(p_im_dev, outp + NN, NN * 8, hipMemcpyDeviceToDevice, s));
  CK(hipStreamSynchronize(s));
  if (terms_out) *terms_out = terms.empty() ? 0 : terms[0];
  return RT_OK;
}

rt_status rt_get_grid(rt_ctx* c, int si, int which, double* out_host) {
  if (!c) return RT_EINVAL;
  if (si < 0 || si >= (int)c->sys.size() || !out_host) return fail(c, RT_EINVAL, "rt_get_grid arguments");
  SysDev& d = c->sys[si];
  const double* src = nullptr;
  switch (which) {
    case 0: src = d.rho; break;
    case 1: src = d.vh; break;
    case 2: src = d.vx; break;
    case 3: src = d.vion; break;
    case 4: src = d.vloc; break;
    default: return fail(c, RT_EINVAL, "unknown grid field");
  }
  CK(hipMemcpyAsync(out_host, src, d.ng * 8, hipMemcpyDeviceToHost, c->stream));
  CK(hipStreamSynchronize(c->stream));
  return RT_OK;
}

rt_status rt_eigh_workspace_size(int n, size_t* bytes) {
  if (!bytes || n < 1 || n > 4096) { g_init_error = "rt_eigh_workspace_size: n outside [1, 4096] or bytes NULL"; return RT_EINVAL; }
  Arena a;
  EighWork w;
  eigh_layout(a, w, n);
  *bytes = a.used + 256;
  return RT_OK;
}

rt_status rt_eigh(void* hip_stream, int n, const double* a_dev, double* evals_dev, double* vecs_dev,
                  void* workspace_dev, size_t ws_bytes, int* sweeps_out) {
  size_t need = 0;
  if (!a_dev || !evals_dev || !vecs_dev || !workspace_dev || rt_eigh_workspace_size(n, &need) != RT_OK) {
    g_init_error = "rt_eigh arguments";
    return RT_EINVAL;
  }
  if (ws_bytes < need) {
    g_init_error = "rt_eigh: workspace too small: need " + std::to_string(need) + " bytes";
    return RT_ENOMEM;
  }
  Arena a;
  a.base = reinterpret_cast<char*>(((uintptr_t)workspace_dev + 255) & ~uintptr_t(255));
  EighWork w;
  eigh_layout(a, w, n);
  rt_ctx c;
  c.stream = (hipStream_t)hip_stream;
  rt_status st = eigh_run(&c, w, a_dev, evals_dev, vecs_dev, sweeps_out);
  if (st != RT_OK) g_init_error = c.err;
  return st;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// rt_eigh_noalloc: the eigensolver's work matrices in one static device array
// (one copy on every GPU the library runs on, held until the process ends).
// Host code never passes the array's name to a kernel: its device address is
// taken once per device with hipGetSymbolAddress and kept in eigh_scratch_ptr.
// Nothing in it has to start at zero (every kernel writes what it later reads).
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kEighScratchBytes =
    3ull * RT_EIGH_NOALLOC_MAX_N * RT_EIGH_NOALLOC_MAX_N * sizeof(double) + 8192;
__device__ __align__(256) unsigned char scratch[kEighScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex eigh_scratch_mu;
void* eigh_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev, looked up (with dev current) on the
// first call for that device.
rt_status eigh_scratch(int dev, char** out) {
  std::lock_guard<std::mutex> lock(eigh_scratch_mu);
  if (dev < 0 || dev >= kMaxDevices) {
    g_init_error = "rt_eigh_noalloc: device index " + std::to_string(dev) + " out of range";
    return RT_EDEVICE;
  }
  if (!eigh_scratch_ptr[dev]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
    void* p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur >= 0 && cur != dev) {
      hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess || !p) {
      g_init_error = std::string("rt_eigh_noalloc: hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return RT_EDEVICE;
    }
    eigh_scratch_ptr[dev] = p;
  }
  *out = static_cast<char*>(eigh_scratch_ptr[dev]);
  return RT_OK;
}
}  // namespace

extern "C" {

rt_status rt_eigh_noalloc(void* hip_stream, int n, const double* a_dev, double* evals_dev, double* vecs_dev,
                          int* sweeps_out) {
  if (n < 1 || n > RT_EIGH_NOALLOC_MAX_N) {
    g_init_error = "rt_eigh_noalloc: n = " + std::to_string(n) + " outside [1, " +
                   std::to_string(RT_EIGH_NOALLOC_MAX_N) + "] (use rt_eigh with a workspace)";
    return RT_EINVAL;
  }
  if (!a_dev || !evals_dev || !vecs_dev) {
    g_init_error = "rt_eigh_noalloc: NULL device pointer";
    return RT_EINVAL;
  }
  int dev = -1;
  hipError_t e = hip_stream ? hipStreamGetDevice((hipStream_t)hip_stream, &dev) : hipGetDevice(&dev);
  if (e != hipSuccess) {
    g_init_error = std::string("rt_eigh_noalloc: stream device: ") + hipGetErrorString(e);
    return RT_EDEVICE;
  }
  char* base = nullptr;
  rt_status st = eigh_scratch(dev, &base);
  if (st != RT_OK) return st;
  Arena a;
  a.base = base;  // 256-byte aligned
  EighWork w;
  eigh_layout(a, w, n);
  if (a.used > kEighScratchBytes) {
    g_init_error = "rt_eigh_noalloc: scratch layout exceeds the static array";
    return RT_EINVAL;
  }
  rt_ctx c;
  c.stream = (hipStream_t)hip_stream;
  st = eigh_run(&c, w, a_dev, evals_dev, vecs_dev, sweeps_out);
  if (st != RT_OK) g_init_error = c.err;
  return st;
}

rt_status rt_ground_state_workspace_size(const rt_system* sys, const rt_gs_params* params, size_t* bytes) {
  std::string why;
  if (!bytes) { g_init_error = "bytes is NULL"; return RT_EINVAL; }
  rt_status st = validate_gs(sys, params, why);
  if (st != RT_OK) { g_init_error = why; return st; }
  SysDev d;
  GsDev g;
  describe_gs(sys, params, d, g);
  Arena a;
  layout_gs(a, d, g);
  *bytes = a.used + 256;
  return RT_OK;
}

rt_status rt_ground_state(const rt_system* sys, const rt_gs_params* params, void* workspace_dev, size_t ws_bytes,
                          void* hip_stream, double* psi_out_dev, double* eps_out_host, double* rho_out_dev,
                          rt_gs_stats* stats) {
  std::string why;
  rt_status st = validate_gs(sys, params, why);
  if (st != RT_OK) { g_init_error = why; return st; }
  if (!workspace_dev || !psi_out_dev) { g_init_error = "workspace or psi_out is NULL"; return RT_EINVAL; }
  SysDev d;
  GsDev g;
  describe_gs(sys, params, d, g);
  Arena sz;
  layout_gs(sz, d, g);
  if (ws_bytes < sz.used + 256) {
    g_init_error = "rt_ground_state: workspace too small: need " + std::to_string(sz.used + 256) + " bytes";
    return RT_ENOMEM;
  }
  Arena a;
  a.base = reinterpret_cast<char*>(((uintptr_t)workspace_dev + 255) & ~uintptr_t(255));
  layout_gs(a, d, g);
  rt_ctx c;
  c.stream = (hipStream_t)hip_stream;
  st = gs_run(&c, d, g, *sys, *params, psi_out_dev, eps_out_host, rho_out_dev, stats);
  if (st != RT_OK) g_init_error = c.err;
  return st;
}

void rt_mlp_dims(int* n_in, int* n_h, int* n_out) {
  if (n_in) *n_in = kNIn;
  if (n_h) *n_h = kNH;
  if (n_out) *n_out = kNOut;
}

int64_t rt_mlp_n_params(int n_in, int n_h, int n_out) { return rtk::mlp_n_params(rtk::MlpDims{n_in, n_h, n_out}); }

int64_t rt_mlp_work_floats(int n_in, int n_h, int n_out, int batch) {
  return rtk::mlp_work_floats(rtk::MlpDims{n_in, n_h, n_out}, batch);
}

static rt_status mlp_check(int n_in, int n_h, int n_out, int batch) {
  if (n_in < 1 || n_h < 1 || n_out < 1 || batch < 1) { g_init_error = "mlp dimensions"; return RT_EINVAL; }
  return RT_OK;
}
#define CKS(expr)                                                                          \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) { g_init_error = hipGetErrorString(e_); return RT_EDEVICE; }     \
  } while (0)

rt_status rt_mlp_forward(void* stream, int n_in, int n_h, int n_out, const float* params, const float* x, float* y,
                         int batch, float* work) {
  RET(mlp_check(n_in, n_h, n_out, batch));
  if (!params || !x || !y || !work) { g_init_error = "null buffer"; return RT_EINVAL; }
  CKS(rtk::mlp_forward((hipStream_t)stream, rtk::MlpDims{n_in, n_h, n_out}, params, x, y, batch, work, false));
  return RT_OK;
}

rt_status rt_mlp_loss_grad(void* stream, int n_in, int n_h, int n_out, const float* params, const float* x,
                           const float* target, int batch, float* grads, float* work, float* loss) {
  RET(mlp_check(n_in, n_h, n_out, batch));
  if (!params || !x || !target || !grads || !work || !loss) { g_init_error = "null buffer"; return RT_EINVAL; }
  CKS(rtk::mlp_loss_grad((hipStream_t)stream, rtk::MlpDims{n_in, n_h, n_out}, params, x, target, batch, grads, work,
                         loss));
  return RT_OK;
}

rt_status rt_mlp_adam(void* stream, float* p, const float* g, float* m, float* v, int64_t n, int t, float lr) {
  if (!p || !g || !m || !v || n < 1 || t < 1) { g_init_error = "rt_mlp_adam arguments"; return RT_EINVAL; }
  CKS(rtk::mlp_adam((hipStream_t)stream, p, g, m, v, n, t, lr));
  return RT_OK;
}

rt_status rt_mlp_colstats(void* stream, const float* x, int rows, int cols, float* mean, float* scale,
                          float floor_std) {
  if (!x || !mean || !scale || rows < 1 || cols < 1) { g_init_error = "rt_mlp_colstats arguments"; return RT_EINVAL; }
  CKS(rtk::mlp_colstats((hipStream_t)stream, x, rows, cols, mean, scale, floor_std));
  return RT_OK;
}

rt_status rt_record(rt_ctx* c, float* x_dev, float* y_dev, int capacity) {
  if (!c) return RT_EINVAL;
  if (!x_dev || !y_dev || capacity < 0) return fail(c, RT_EINVAL, "rt_record arguments");
  for (auto& d : c->sys)
    if (!d.feat) return fail(c, RT_EINVAL, "recording needs grid edges divisible by 16");
  c->rec_x = x_dev;
  c->rec_y = y_dev;
  c->rec_cap = capacity;
  c->rec_count = 0;
  return RT_OK;
}

rt_status rt_record_count(rt_ctx* c, int* rows) {
  if (!c || !rows) return RT_EINVAL;
  *rows = c->rec_count;
  return RT_OK;
}

void rt_free(rt_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  prof_collect(c);
  for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
  delete c;
}

const char* rt_last_error(const rt_ctx* c) { return c ? c->err.c_str() : g_init_error.c_str(); }

}  // extern "C"
