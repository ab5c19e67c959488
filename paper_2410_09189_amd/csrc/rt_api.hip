// Runtime behind the C ABI of rt_tddft.h: workspace layout, projector tables,
// initialisation (orthonormalisation, V_ion, H_core, dipole matrices, kicks)
// and the self-consistent time loop of Algorithm 1 driving the kernels.
#include "../../include/rt_tddft.h"
#include "kernels.h"

#include <hip/hip_runtime.h>

#include <algorithm>
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

struct SysDev {
  int nx, ny, nz, N, n_occ, n_atoms, n_images;
  long ng;
  double h, h3;
  double coef[5];
  NlTables nl;
  int n_union = 0;
  int n_split = 1, big = 0;
  long kps = 0;
  // device buffers
  double *psi, *hpsi, *vion, *rho, *vh, *vx, *vloc, *vloc_gs, *dv;
  float *psi32, *vloc32;
  double2* z;
  double2 *twx, *twy, *twz;
  double *pos, *depth, *width;
  int *atom_off, *sph_idx, *u_idx, *u_ptr, *ent_pt, *ent_atom;
  double *beta, *Dd, *cnl;
  double *hcore, *M3, *Hgs, *W, *tmp, *part, *occ;
  double *red2, *eparts, *escale, *ezero;
  int* info;
};

struct TrajDev {
  int sys, axis;
  double kappa;
  double *P0, *P1, *dP, *dPn, *C;
  double *H0, *H1, *Hm1, *Hn, *Hbar;
  double* hist;
  double* kmin;
  unsigned long long *slots, *resid;
  int* done;
  int step = 0;
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
  int hist_cap = 0;
  double* coef_dev = nullptr;
};

namespace {

#define CK(expr)                                                                    \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) return fail(c, RT_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

rt_status fail(rt_ctx* c, rt_status st, const std::string& msg) {
  if (c) c->err = msg; else g_init_error = msg;
  return st;
}

long nsq(int N) { return (long)N * N; }

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

rt_status validate(const rt_system* sys, int n_sys, const rt_run* run, std::string& why) {
  if (!sys || n_sys < 1 || !run) { why = "null system/run or n_sys < 1"; return RT_EINVAL; }
  for (int i = 0; i < n_sys; ++i) {
    const rt_system& s = sys[i];
    for (int q = 0; q < 3; ++q)
      if (s.n[q] < 8 || s.n[q] > 1024) { why = "grid edge outside [8, 1024]"; return RT_EINVAL; }
    if ((s.n[1] > 256) || (s.n[2] > 256)) { why = "y and z grid edges above 256 are not supported"; return RT_EINVAL; }
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
  }
  if (!(run->dt != 0.0) || run->n_steps_max < 0 || run->max_scf < 1 || run->max_terms < 1 ||
      !(run->h_thrs > 0) || !(run->dp_thrs > 0)) { why = "run parameters"; return RT_EINVAL; }
  if (run->precision != RT_FP64 && run->precision != RT_MIXED) { why = "precision"; return RT_EINVAL; }
  if (run->precision == RT_MIXED) { why = "mixed precision is not available in this build"; return RT_EINVAL; }
  if (run->predictor != RT_PRED_LINEAR) { why = "only the linear predictor is available in this build"; return RT_EINVAL; }
  if (run->hupdate != RT_HUPDATE_FULL && run->hupdate != RT_HUPDATE_LOCAL) { why = "hupdate"; return RT_EINVAL; }
  if (run->n_traj < 0 || (run->n_traj > 0 && (!run->traj_sys || !run->traj_kappa || !run->traj_axis))) {
    why = "trajectory arrays"; return RT_EINVAL;
  }
  for (int t = 0; t < run->n_traj; ++t) {
    if (run->traj_sys[t] < 0 || run->traj_sys[t] >= n_sys) { why = "traj_sys out of range"; return RT_EINVAL; }
    if (run->traj_axis[t] < 0 || run->traj_axis[t] > 2) { why = "traj_axis out of range"; return RT_EINVAL; }
  }
  return RT_OK;
}

void choose_split(SysDev& d) {
  d.big = d.N >= 128 ? 1 : 0;
  int tile = d.big ? 128 : 64;
  int ntm = (d.N + tile - 1) / tile;
  int tiles = ntm * (ntm + 1) / 2;
  long target = 1024;
  long ns = (target + tiles - 1) / tiles;
  long maxs = std::max(1L, d.ng / 1024);
  ns = std::min(ns, maxs);
  int bk = d.big ? 16 : 32;
  long kps = (d.ng + ns - 1) / ns;
  kps = (kps + bk - 1) / bk * bk;
  d.kps = kps;
  d.n_split = (int)((d.ng + kps - 1) / kps);
}

// Places every buffer; with a.base == nullptr only sizes.
void layout(Arena& a, std::vector<SysDev>& S, std::vector<TrajDev>& T, const rt_run& run, int hist_cap) {
  for (auto& d : S) {
    long ng = d.ng, N = d.N;
    d.psi = a.take<double>(N * ng);
    d.hpsi = a.take<double>(N * ng);
    d.vion = a.take<double>(ng);
    d.rho = a.take<double>(ng);
    d.vh = a.take<double>(ng);
    d.vx = a.take<double>(ng);
    d.vloc = a.take<double>(ng);
    d.vloc_gs = a.take<double>(ng);
    d.dv = a.take<double>(ng);
    d.vloc32 = a.take<float>(ng);
    d.psi32 = nullptr;
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
    d.cnl = a.take<double>(N * std::max(1, d.nl.n_proj));
    d.hcore = a.take<double>(N * N);
    d.M3 = a.take<double>(3 * N * N);
    d.Hgs = a.take<double>(N * N);
    d.W = a.take<double>(N * N);
    d.tmp = a.take<double>(N * N);
    d.part = a.take<double>((long)d.n_split * N * N);
    d.occ = a.take<double>(N);
    d.red2 = a.take<double>(2 * rtk::kRedBlocks);
    d.eparts = a.take<double>(2);
    d.escale = a.take<double>(2);
    d.ezero = a.take<double>(2);
    d.info = a.take<int>(4);
  }
  for (auto& t : T) {
    long N = S[t.sys].N;
    t.P0 = a.take<double>(2 * N * N);
    t.P1 = a.take<double>(2 * N * N);
    t.dP = a.take<double>(2 * N * N);
    t.dPn = a.take<double>(2 * N * N);
    t.C = a.take<double>(2 * N * N);
    t.H0 = a.take<double>(N * N);
    t.H1 = a.take<double>(N * N);
    t.Hm1 = a.take<double>(N * N);
    t.Hn = a.take<double>(N * N);
    t.Hbar = a.take<double>(N * N);
    t.hist = a.take<double>(5L * (hist_cap + 1));
    t.kmin = a.take<double>(1);
    t.slots = a.take<unsigned long long>(run.max_terms + 2);
    t.resid = a.take<unsigned long long>(1);
    t.done = a.take<int>(2);
  }
}

void describe(const rt_system* sys, int n_sys, const rt_run* run, std::vector<SysDev>& S,
              std::vector<TrajDev>& T) {
  S.resize(n_sys);
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
    choose_split(d);
  }
  T.resize(run->n_traj);
  for (int t = 0; t < run->n_traj; ++t) {
    T[t].sys = run->traj_sys[t];
    T[t].axis = run->traj_axis[t];
    T[t].kappa = run->traj_kappa[t];
  }
}

template <typename V>
rt_status upload(rt_ctx* c, void* dst, const std::vector<V>& v) {
  if (v.empty()) return RT_OK;
  CK(hipMemcpyAsync(dst, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice, c->stream));
  return RT_OK;
}

// ---------------------------------------------------------------------------
// Stages
// ---------------------------------------------------------------------------
// Symmetric projection out = alpha * A diag(w) B^T over the grid (upper tiles, mirrored).
rt_status project(rt_ctx* c, SysDev& d, const double* A, const double* B, const double* w, double* out) {
  {
    Timed tm(c, PH_PROJECT);
    CK(rtk::gemm_nt_f64(c->stream, d.N, d.N, d.ng, A, d.ng, B, d.ng, w, d.part, d.kps, d.n_split, 1, d.big));
  }
  Timed tm(c, PH_REDUCE);
  CK(rtk::reduce_parts(c->stream, d.part, d.n_split, d.N, d.N, d.h3, out, 1));
  return RT_OK;
}

// hpsi = (T + vloc + V_nl) psi for n rows (FP64).
rt_status apply_h64(rt_ctx* c, SysDev& d, const double* psi, double* hpsi, const double* vloc, int n) {
  {
    Timed tm(c, PH_STENCIL);
    CK(rtk::stencil<double>(c->stream, psi, hpsi, vloc, n, d.nx, d.ny, d.nz, d.h, d.coef));
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
    CK(rtk::stencil<float>(c->stream, psi, hpsi, d.vloc32, n, d.nx, d.ny, d.nz, d.h, d.coef));
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

// rho = sum_ij S_ij psi_i psi_j; V_H by spectral Poisson; v_x, V_loc and energies.
rt_status potentials(rt_ctx* c, SysDev& d, const double* S) {
  hipStream_t s = c->stream;
  {
    Timed tm(c, PH_DENSITY);
    CK(rtk::upper_weighted(s, S, d.W, d.N));
    CK(rtk::smalltall_f64(s, d.N, d.ng, d.W, d.psi, d.rho, 1, 1));
  }
  {
  Timed tp(c, PH_POISSON);
  CK(rtk::pack_real(s, d.z, d.rho, d.ng));
  CK(rtk::dft_axis(s, d.z, d.nx, d.ny, d.nz, 0, d.twx, 0));
  CK(rtk::dft_axis(s, d.z, d.nx, d.ny, d.nz, 1, d.twy, 0));
  CK(rtk::dft_axis(s, d.z, d.nx, d.ny, d.nz, 2, d.twz, 0));
  CK(rtk::poisson_scale(s, d.z, d.nx, d.ny, d.nz, d.h));
  CK(rtk::dft_axis(s, d.z, d.nx, d.ny, d.nz, 0, d.twx, 1));
  CK(rtk::dft_axis(s, d.z, d.nx, d.ny, d.nz, 1, d.twy, 1));
  CK(rtk::dft_axis(s, d.z, d.nx, d.ny, d.nz, 2, d.twz, 1));
  CK(rtk::real_part(s, d.vh, d.z, d.ng));
  }
  Timed tl(c, PH_LDA);
  CK(rtk::lda_vloc(s, d.rho, d.vh, d.vion, d.vx, d.vloc, d.ng, d.red2));
  CK(rtk::reduce_cols(s, d.red2, rtk::kRedBlocks, 2, d.escale, d.eparts));
  return RT_OK;
}

// H_out = H[P] for P with real part S (Algorithm 1: H_1 <- DFT(rho(P_1))).
rt_status eval_h(rt_ctx* c, SysDev& d, const double* S, double* Hout, int force_full) {
  const rt_run& r = c->run;
  if (r.frozen_hxc && !force_full) {
    CK(rtk::copy_d(c->stream, Hout, d.Hgs, nsq(d.N)));
    return RT_OK;
  }
  rt_status st = potentials(c, d, S);
  if (st != RT_OK) return st;
  if (r.hupdate == RT_HUPDATE_FULL || force_full) {
    st = apply_h64(c, d, d.psi, d.hpsi, d.vloc, d.N);
    if (st != RT_OK) return st;
    return project(c, d, d.psi, d.hpsi, nullptr, Hout);
  }
  // local update: H[P] = H_gs + h^3 Psi diag(V_loc - V_loc,gs) Psi^T
  CK(rtk::sub_d(c->stream, d.dv, d.vloc, d.vloc_gs, d.ng));
  st = project(c, d, d.psi, d.psi, d.dv, d.tmp);
  if (st != RT_OK) return st;
  CK(rtk::lincomb(c->stream, Hout, 1.0, d.Hgs, 1.0, d.tmp, nsq(d.N)));
  return RT_OK;
}

// P (stacked [S; A]) -> U P U^dagger, U = exp(-i dt Hbar), by the commutator series.
rt_status series(rt_ctx* c, TrajDev& t, SysDev& d, const double* Hbar, double dt, const double* Pin,
                 double* Pout, int* terms) {
  hipStream_t s = c->stream;
  const long n2 = 2 * nsq(d.N);
  const int max_terms = c->run.max_terms;
  const double thrs = c->run.dp_thrs;
  CK(rtk::copy_d(s, Pout, Pin, n2));
  CK(rtk::copy_d(s, t.dP, Pin, n2));
  CK(rtk::gershgorin(s, Hbar, d.N, dt, t.kmin));
  CK(rtk::fill_u64(s, t.slots, max_terms + 2, 0ULL));
  int zero2[2] = {0, 0};
  CK(hipMemcpyAsync(t.done, zero2, sizeof(zero2), hipMemcpyHostToDevice, s));
  double* dP = t.dP;
  double* dPn = t.dPn;
  int k = 1;
  const int CH = 8;
  while (true) {
    int kend = std::min(max_terms, k + CH - 1);
    for (; k <= kend; ++k) {
      {
        Timed tm(c, PH_SERIES_GEMM);
        CK(rtk::gemm_nt_f64_series(s, d.N, Hbar, dP, t.C, k, t.slots, t.kmin, thrs, t.done));
      }
      {
        Timed tm(c, PH_SERIES_UPDATE);
        CK(rtk::series_update(s, t.C, dPn, Pout, d.N, dt, k, t.slots, t.kmin, thrs, t.done));
      }
      std::swap(dP, dPn);
    }
    CK(rtk::series_finish(s, kend, t.slots, t.kmin, thrs, t.done));
    int hd[2];
    CK(hipMemcpyAsync(hd, t.done, sizeof(hd), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    if (hd[0]) {
      if (terms) *terms = hd[1];
      return RT_OK;
    }
    if (kend >= max_terms) return fail(c, RT_ENOCONV, "commutator series reached max_terms");
  }
}

rt_status observe(rt_ctx* c, TrajDev& t, SysDev& d, int row) {
  const double* Hc = c->run.frozen_hxc ? d.Hgs : d.hcore;
  const double* ep = c->run.frozen_hxc ? d.ezero : d.eparts;
  CK(rtk::observables(c->stream, t.P0, d.M3, Hc, d.N, ep, t.hist + 5L * row));
  return RT_OK;
}

rt_status init_system(rt_ctx* c, SysDev& d, const rt_system& s) {
  hipStream_t st = c->stream;
  const long N = d.N, ng = d.ng;
  CK(hipMemcpyAsync(d.psi, s.psi0, N * ng * sizeof(double),
                    s.psi0_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
  std::vector<double> occ(N);
  for (long i = 0; i < N; ++i) occ[i] = s.occ ? s.occ[i] : (i < s.n_occ ? 2.0 : 0.0);
  CK(hipMemcpyAsync(d.occ, occ.data(), N * sizeof(double), hipMemcpyHostToDevice, st));
  double esc[2] = {d.h3, 0.5 * d.h3}, ez[2] = {0.0, 0.0};
  CK(hipMemcpyAsync(d.escale, esc, sizeof(esc), hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(d.ezero, ez, sizeof(ez), hipMemcpyHostToDevice, st));
  if (d.n_atoms) {
    CK(hipMemcpyAsync(d.pos, s.pos, 3 * d.n_atoms * sizeof(double), hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(d.depth, s.depth, d.n_atoms * sizeof(double), hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(d.width, s.width, d.n_atoms * sizeof(double), hipMemcpyHostToDevice, st));
  }
  rt_status r;
  if ((r = upload(c, d.atom_off, d.nl.atom_off)) != RT_OK) return r;
  if ((r = upload(c, d.sph_idx, d.nl.sph_idx)) != RT_OK) return r;
  if ((r = upload(c, d.beta, d.nl.beta)) != RT_OK) return r;
  if ((r = upload(c, d.Dd, d.nl.D)) != RT_OK) return r;
  if ((r = upload(c, d.u_idx, d.nl.u_idx)) != RT_OK) return r;
  if ((r = upload(c, d.u_ptr, d.nl.u_ptr)) != RT_OK) return r;
  if ((r = upload(c, d.ent_pt, d.nl.ent_pt)) != RT_OK) return r;
  if ((r = upload(c, d.ent_atom, d.nl.ent_atom)) != RT_OK) return r;
  CK(rtk::twiddles(st, d.twx, d.nx));
  CK(rtk::twiddles(st, d.twy, d.ny));
  CK(rtk::twiddles(st, d.twz, d.nz));
  if (s.orthonormalize) {
    // S = h^3 Psi Psi^T = L L^T;  Psi <- L^-1 Psi
    if ((r = project(c, d, d.psi, d.psi, nullptr, d.tmp)) != RT_OK) return r;
    CK(rtk::cholesky(st, d.tmp, d.N, d.info));
    int info = 0;
    CK(hipMemcpyAsync(&info, d.info, sizeof(int), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    if (info) return fail(c, RT_EINVAL, "orbital overlap matrix is not positive definite");
    CK(rtk::tri_inverse_lower(st, d.tmp, d.W, d.N));
    CK(rtk::smalltall_f64(st, d.N, d.ng, d.W, d.psi, d.hpsi, 0, 2));
    std::swap(d.psi, d.hpsi);
  }
  CK(rtk::vion(st, d.vion, d.nx, d.ny, d.nz, d.h, d.n_atoms, d.pos, d.depth, d.width, d.n_images));
  for (int q = 0; q < 3; ++q) {
    CK(rtk::coord(st, d.dv, d.nx, d.ny, d.nz, d.h, q));
    if ((r = project(c, d, d.psi, d.psi, d.dv, d.M3 + q * N * N)) != RT_OK) return r;
  }
  if ((r = apply_h64(c, d, d.psi, d.hpsi, d.vion, d.N)) != RT_OK) return r;
  if ((r = project(c, d, d.psi, d.hpsi, nullptr, d.hcore)) != RT_OK) return r;
  // ground-state Hamiltonian H_gs = H[diag(f)] with the full apply; V_loc of that density kept
  std::vector<double> pgs(N * N, 0.0);
  for (long i = 0; i < N; ++i) pgs[i * N + i] = occ[i];
  CK(hipMemcpyAsync(d.tmp, pgs.data(), N * N * sizeof(double), hipMemcpyHostToDevice, st));
  if ((r = eval_h(c, d, d.tmp, d.Hgs, 1)) != RT_OK) return r;
  CK(rtk::copy_d(st, d.vloc_gs, d.vloc, d.ng));
  CK(hipStreamSynchronize(st));
  return RT_OK;
}

rt_status init_traj(rt_ctx* c, TrajDev& t) {
  SysDev& d = c->sys[t.sys];
  hipStream_t st = c->stream;
  const long N = d.N;
  std::vector<double> p0(2 * N * N, 0.0);
  std::vector<double> occ(N);
  CK(hipMemcpyAsync(occ.data(), d.occ, N * sizeof(double), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  for (long i = 0; i < N; ++i) p0[i * N + i] = occ[i];
  CK(hipMemcpyAsync(t.P1, p0.data(), 2 * N * N * sizeof(double), hipMemcpyHostToDevice, st));
  rt_status r;
  if (t.kappa != 0.0) {
    // delta kick: exp(-i kappa M_q) P_0 exp(+i kappa M_q), same series with Hbar = M_q, dt = kappa
    int terms = 0;
    if ((r = series(c, t, d, d.M3 + t.axis * N * N, t.kappa, t.P1, t.P0, &terms)) != RT_OK) return r;
  } else {
    CK(rtk::copy_d(st, t.P0, t.P1, 2 * N * N));
  }
  if ((r = eval_h(c, d, t.P0, t.H0, 0)) != RT_OK) return r;
  CK(rtk::copy_d(st, t.Hm1, t.H0, N * N));
  t.step = 0;
  if ((r = observe(c, t, d, 0)) != RT_OK) return r;
  CK(hipStreamSynchronize(st));  // p0 (host) must outlive its copy
  return RT_OK;
}

rt_status step_traj(rt_ctx* c, TrajDev& t, rt_step_stats* stat) {
  SysDev& d = c->sys[t.sys];
  hipStream_t st = c->stream;
  const rt_run& run = c->run;
  const long NN = nsq(d.N);
  CK(rtk::lincomb(st, t.H1, 2.0, t.H0, -1.0, t.Hm1, NN));
  int terms_total = 0;
  double res = 0.0;
  int m = 0;
  bool conv = false;
  rt_status r;
  for (m = 1; m <= run.max_scf; ++m) {
    CK(rtk::lincomb(st, t.Hbar, 0.5, t.H0, 0.5, t.H1, NN));
    int terms = 0;
    if ((r = series(c, t, d, t.Hbar, run.dt, t.P0, t.P1, &terms)) != RT_OK) return r;
    terms_total += terms;
    if ((r = eval_h(c, d, t.P1, t.Hn, 0)) != RT_OK) return r;
    CK(rtk::fill_u64(st, t.resid, 1, 0ULL));
    CK(rtk::max_abs_diff(st, t.Hn, t.H1, NN, t.resid));
    unsigned long long bits = 0;
    CK(hipMemcpyAsync(&bits, t.resid, sizeof(bits), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    std::memcpy(&res, &bits, sizeof(res));
    std::swap(t.H1, t.Hn);
    if (res <= run.h_thrs) { conv = true; break; }
  }
  if (!conv) return fail(c, RT_ENOCONV, "self-consistent Hamiltonian loop reached max_scf");
  // H_-1 <- H_0, H_0 <- H_1, P_0 <- P_1
  double* old_m1 = t.Hm1;
  t.Hm1 = t.H0;
  t.H0 = t.H1;
  t.H1 = old_m1;
  std::swap(t.P0, t.P1);
  t.step += 1;
  if (stat) {
    stat->scf_iters = m;
    stat->series_terms = terms_total;
    stat->residual = res;
  }
  return observe(c, t, d, t.step);
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
  layout(a, S, T, *run, run->n_steps_max);
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
  layout(a, c->sys, c->traj, *run, c->hist_cap);
  size_t need = a.used + 256;
  if (ws_bytes < need) {
    g_init_error = "workspace too small: need " + std::to_string(need) + " bytes";
    delete c;
    return RT_ENOMEM;
  }
  Arena b;
  b.base = reinterpret_cast<char*>(((uintptr_t)workspace_dev + 255) & ~uintptr_t(255));
  layout(b, c->sys, c->traj, *run, c->hist_cap);
  for (int i = 0; i < n_sys; ++i) {
    st = init_system(c, c->sys[i], sys[i]);
    if (st != RT_OK) { g_init_error = c->err; delete c; return st; }
  }
  for (auto& t : c->traj) {
    st = init_traj(c, t);
    if (st != RT_OK) { g_init_error = c->err; delete c; return st; }
  }
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    g_init_error = std::string("rt_init: ") + hipGetErrorString(e);
    delete c;
    return RT_EDEVICE;
  }
  *out = c;
  return RT_OK;
}

rt_status rt_apply_h(rt_ctx* c, int si, const void* psi_dev, void* hpsi_dev, int n_orb, int dtype) {
  if (!c) return RT_EINVAL;
  if (si < 0 || si >= (int)c->sys.size()) return fail(c, RT_EINVAL, "sys_index out of range");
  if (!psi_dev || !hpsi_dev || n_orb < 0 || (dtype != 0 && dtype != 1))
    return fail(c, RT_EINVAL, "rt_apply_h arguments");
  if (psi_dev == hpsi_dev) return fail(c, RT_EINVAL, "psi and hpsi must not overlap");
  SysDev& d = c->sys[si];
  size_t esz = dtype == 0 ? 8 : 4;
  uintptr_t p0 = (uintptr_t)psi_dev, p1 = (uintptr_t)hpsi_dev, len = (uintptr_t)n_orb * d.ng * esz;
  if (p0 < p1 + len && p1 < p0 + len) return fail(c, RT_EINVAL, "psi and hpsi must not overlap");
  if (dtype == 1) CK(rtk::cast_d2f(c->stream, d.vloc32, d.vloc, d.ng));
  for (int o = 0; o < n_orb; o += d.N) {
    int n = std::min(d.N, n_orb - o);
    rt_status r;
    if (dtype == 0)
      r = apply_h64(c, d, (const double*)psi_dev + (long)o * d.ng, (double*)hpsi_dev + (long)o * d.ng, d.vloc, n);
    else
      r = apply_h32(c, d, (const float*)psi_dev + (long)o * d.ng, (float*)hpsi_dev + (long)o * d.ng, n);
    if (r != RT_OK) return r;
  }
  return RT_OK;
}

rt_status rt_step(rt_ctx* c, int n_steps, rt_step_stats* stats) {
  if (!c) return RT_EINVAL;
  if (n_steps < 0) return fail(c, RT_EINVAL, "n_steps < 0");
  for (auto& t : c->traj)
    if (t.step + n_steps > c->hist_cap) return fail(c, RT_ESTATE, "history capacity n_steps_max exhausted");
  const int nt = (int)c->traj.size();
  for (int k = 0; k < n_steps; ++k) {
    for (int i = 0; i < nt; ++i) {
      rt_status r = step_traj(c, c->traj[i], stats ? stats + (long)k * nt + i : nullptr);
      if (r != RT_OK) return r;
    }
  }
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
  if (first_step < 0 || count < 0 || first_step + count > t.step + 1 || !mu_host)
    return fail(c, RT_EINVAL, "requested steps outside the recorded history");
  std::vector<double> buf(5L * count);
  if (count) {
    CK(hipMemcpyAsync(buf.data(), t.hist + 5L * first_step, buf.size() * sizeof(double),
                      hipMemcpyDeviceToHost, c->stream));
  }
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
    case 0: src = t.H0; break;
    case 1: src = t.Hm1; break;
    case 2: src = t.P0; break;
    case 3: src = t.P0 + NN; break;
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
  if (p_re) CK(hipMemcpyAsync(t.P0, p_re, NN * 8, hipMemcpyHostToDevice, s));
  if (p_im) CK(hipMemcpyAsync(t.P0 + NN, p_im, NN * 8, hipMemcpyHostToDevice, s));
  if (h0) CK(hipMemcpyAsync(t.H0, h0, NN * 8, hipMemcpyHostToDevice, s));
  if (hm1) CK(hipMemcpyAsync(t.Hm1, hm1, NN * 8, hipMemcpyHostToDevice, s));
  CK(hipStreamSynchronize(s));
  return RT_OK;
}

rt_status rt_eval_h(rt_ctx* c, int si, const double* p_re_dev, double* h_out_dev) {
  if (!c) return RT_EINVAL;
  if (si < 0 || si >= (int)c->sys.size() || !p_re_dev || !h_out_dev) return fail(c, RT_EINVAL, "rt_eval_h arguments");
  return eval_h(c, c->sys[si], p_re_dev, h_out_dev, 0);
}

rt_status rt_propagate(rt_ctx* c, int si, const double* hbar_dev, double dt, double* p_re_dev, double* p_im_dev,
                       int* terms_out) {
  if (!c) return RT_EINVAL;
  if (si < 0 || si >= (int)c->sys.size() || !hbar_dev || !p_re_dev || !p_im_dev)
    return fail(c, RT_EINVAL, "rt_propagate arguments");
  int ti = -1;
  for (int i = 0; i < (int)c->traj.size(); ++i)
    if (c->traj[i].sys == si) { ti = i; break; }
  if (ti < 0) return fail(c, RT_ESTATE, "rt_propagate needs a trajectory of this system for its work buffers");
  TrajDev& t = c->traj[ti];
  SysDev& d = c->sys[si];
  const long NN = nsq(d.N);
  hipStream_t s = c->stream;
  // work in the trajectory's P1/dP buffers, leaving its state P0 untouched
  double* in = t.C;
  CK(hipMemcpyAsync(in, p_re_dev, NN * 8, hipMemcpyDeviceToDevice, s));
  CK(hipMemcpyAsync(in + NN, p_im_dev, NN * 8, hipMemcpyDeviceToDevice, s));
  double* saved_P1 = t.P1;
  rt_status r = series(c, t, d, hbar_dev, dt, in, saved_P1, terms_out);
  if (r != RT_OK) return r;
  CK(hipMemcpyAsync(p_re_dev, saved_P1, NN * 8, hipMemcpyDeviceToDevice, s));
  CK(hipMemcpyAsync(p_im_dev, saved_P1 + NN, NN * 8, hipMemcpyDeviceToDevice, s));
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

void rt_free(rt_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  prof_collect(c);
  for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
  delete c;
}

const char* rt_last_error(const rt_ctx* c) { return c ? c->err.c_str() : g_init_error.c_str(); }

}  // extern "C"
