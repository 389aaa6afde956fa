// Host side of the dsweep library: partition, routing rules, schedules,
// factorisation driver, sweeps, flexible GMRES and FWI, behind the C ABI of
// include/dsweep.h.
#include <algorithm>
#include <complex>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "dsweep.h"
#include "kernels.hpp"
#include "nd.hpp"

using namespace dsd;

namespace {

thread_local std::string g_detail;

#define HIPCHK(expr)                                                              \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess) {                                                       \
      g_detail = std::string(#expr) + ": " + hipGetErrorString(e_);               \
      return e_ == hipErrorOutOfMemory ? DSD_ENOMEM : DSD_EHIP;                   \
    }                                                                             \
  } while (0)

#define CHK(expr)                  \
  do {                             \
    int rc_ = (expr);              \
    if (rc_ < 0) return rc_;       \
  } while (0)

// ---------------------------------------------------------------- sweep rules
// Sweep directions: Section 3 (2D order) and (Sorder3D) of Section 4.1, or
// (3D, variant 1) the other order given there, along which the L1 distance
// from the first direction never decreases.
const int ORDER2[4][3] = {{1, 1, 0}, {-1, 1, 0}, {1, -1, 0}, {-1, -1, 0}};
const int ORDER3[8][3] = {{1, 1, 1},  {-1, 1, 1},  {1, -1, 1},  {-1, -1, 1},
                          {1, 1, -1}, {-1, 1, -1}, {1, -1, -1}, {-1, -1, -1}};
const int ORDER3_L1[8][3] = {{1, 1, 1},   {-1, 1, 1},  {1, -1, 1},  {1, 1, -1},
                             {-1, -1, 1}, {-1, 1, -1}, {1, -1, -1}, {-1, -1, -1}};

const int* sweep_dir(int dim, int variant, int l) {
  return dim == 2 ? ORDER2[l] : (variant == 1 ? ORDER3_L1[l] : ORDER3[l]);
}

// Rule 3.1 (t.D > 0) / Rule 4.1 (t.D > 0 and every t_k D_k >= 0)
bool similar(int dim, const int* t, const int* D) {
  int dot = 0;
  bool comp = true;
  for (int k = 0; k < dim; ++k) {
    dot += t[k] * D[k];
    if (t[k] * D[k] < 0) comp = false;
  }
  return dim == 2 ? dot > 0 : (dot > 0 && comp);
}

// Rule 3.2 / 4.2: barred if, in a coordinate plane, the projection of t has
// exactly one zero component and the projections of the sweeps are opposite.
bool barred(int dim, const int* t, const int* D1, const int* D2) {
  const int planes3[3][2] = {{0, 1}, {0, 2}, {1, 2}};
  const int np = dim == 2 ? 1 : 3;
  for (int q = 0; q < np; ++q) {
    const int a = planes3[q][0], b = planes3[q][1];
    const int zeros = (t[a] == 0) + (t[b] == 0);
    if (zeros != 1) continue;
    if (D1[a] == -D2[a] && D1[b] == -D2[b]) return true;
  }
  return false;
}

// Sweep (>= l) that uses a transfer of direction t generated in sweep l; -1 if dropped.
int route(int dim, int variant, int l, const int* t) {
  const int L = 1 << dim;
  for (int lp = l; lp < L; ++lp)
    if (similar(dim, t, sweep_dir(dim, variant, lp)) &&
        !barred(dim, t, sweep_dir(dim, variant, l), sweep_dir(dim, variant, lp)))
      return lp;
  return -1;
}

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
  ~Buf() { if (p) (void)hipFree(p); }
  int alloc(size_t b) {
    if (p) { (void)hipFree(p); p = nullptr; bytes = 0; }
    if (b == 0) return 0;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      p = nullptr;
      g_detail = "hipMalloc of " + std::to_string(b) + " bytes failed";
      return DSD_ENOMEM;
    }
    bytes = b;
    return 0;
  }
  template <typename U> U* as() const { return reinterpret_cast<U*>(p); }
};

template <typename U>
int upload(Buf& b, const std::vector<U>& v) {
  CHK(b.alloc(std::max<size_t>(1, v.size()) * sizeof(U)));
  if (!v.empty()) HIPCHK(hipMemcpy(b.p, v.data(), v.size() * sizeof(U), hipMemcpyHostToDevice));
  return 0;
}


struct StepTab {
  int mem_off, nmem;           // members (subdomain ids) in d_members
  int job_off;                 // fwd/bwd jobs (2 per member) in d_jobs2; mid jobs at d_jobs1
  int er_off;                  // edge ranges (1 per member) in d_erange
  long long max_nloc, max_box;
  double fac_bytes_fb;         // factor bytes touched by the fwd (= bwd) launch
  double fac_bytes_mid;
  long long blk_cells_fb;      // block-cells processed by the fwd launch (for vector bytes)
  long long blk_cells_mid;
};

// Block cyclic reduction of one subdomain: the blocks still present at every
// level (original indices; the even positions are eliminated there) and the
// factor offsets of W_L = P_k A[k][left], W_R = P_k A[k][right] and of their
// transposes (the products A[j][k] P_k the kept neighbours use), per block.
struct BcrSub {
  int top = 0;                               // level where a single block remains
  int dtop = -1;                             // level solved densely (-1: none)
  int dm = 0;                                // blocks of that level
  long long dense = -1;                      // factor offset of its inverse (dm row blocks)
  std::vector<std::vector<int>> lev;
  std::vector<long long> wl, wr, wlt, wrt;   // -1: absent
};

struct BcrLaunch {
  int off, n;        // job range
  int dfwd;          // 1: level-0 coupling update (vector kernel)
  int nset;          // most matrices (operand vectors) of one job
  int cg;            // wave groups splitting the columns (from the level only)
  int rt;            // most 64-row tiles per workgroup (0: default)
  int kg;            // RHS per workgroup (0: the plan's)
  double fbytes;     // factor bytes streamed (once per launch)
  double vcells;     // vector entries read and written per right-hand side
};

}  // namespace

struct dsd_plan {
  dsd_params prm{};
  double omega = 0;
  Problem P{};
  int dim = 2, L = 4, nsteps = 0, S = 0, kmax = 1, kg = 2, max_nb = 0;
  bool c64 = true;
  bool sequential = false;      // anti-diagonal steps in order instead of DAG launch groups
  bool additive = false;        // the additive DDM (every subdomain at every step)
  std::vector<SubDesc> subs;
  std::vector<AxisPart> parts[3];
  std::vector<StepTab> steps;   // launch groups, in order
  int solver = 2;               // 1: twisted block LDL^T chains, 2: block cyclic reduction
  std::vector<BcrSub> bcr;
  std::vector<std::vector<BcrLaunch>> bcr_launch;   // per launch group
  // local-solve tables of every subdomain (dsd_local_solve and its
  // allocation-free variant): job tables addressing a subdomain's vectors from
  // offset 0 (vbase = 0, and descriptors with vec_off = 0), so one table serves
  // the plan's pools and the static scratch alike
  std::vector<std::vector<BcrLaunch>> local_launch;  // per subdomain, offsets into d_local_jobs
  int device = 0;
  void* scratch = nullptr;        // this device's allocation-free scratch (see below)
  std::vector<std::vector<int2>> groups;            // launch groups: {subdomain, sweep}
  // launch shape of a reduction level: (wide_cg, wide_rt) column groups and
  // row tiles per workgroup while >= cg_wide blocks per subdomain remain at the
  // level, (mid_cg, mid_rt) while >= cg_mid remain, else (deep_cg, deep_rt);
  // dense jobs use (dense_cg, one row tile).  Only the column groups change
  // the summation order.
  int cg_wide = 64, cg_mid = 16;
  int wide_cg = 1, wide_rt = 0, mid_cg = 4, mid_rt = 1, deep_cg = 8, deep_rt = 1, dense_cg = 8;
  int wide_kg = 0;                // RHS per workgroup on the wide levels (0: kg)
  int dense_max = 0;              // largest reduced system solved densely (0: none)
  // chain factor solved with one launch per block step (all chains of a
  // launch group together) instead of one workgroup looping over the blocks
  bool chain_steps = false;
  int chain_cg = 3, chain_rt = 0;
  Buf d_bcr_jobs;
  long long sum_nloc = 0, sum_fac = 0;

  Buf d_subs, d_m, d_gcoef[4], d_lcoef64[4], d_lcoefT[4], d_fac;
  Buf d_rpool, d_vpool, d_members, d_jobs2, d_jobs1, d_edges, d_erange;
  Buf d_part_of[3], d_axparts[3];
  Buf d_subs_local, d_local_jobs;
  // nested dissection (solver 4): shapes, device tables, per launch group jobs
  struct NdLevel {               // one level (depth below the subtree roots) of every subtree
    int off = 0, n = 0;          // node jobs (d_nd_lvl), ordered: wide both ways, wide
                                 // backward only, narrow, wide forward only
    int nf_off = 0, nf_n = 0;    // the narrow forward products (jobs)
    int nb_off = 0, nb_n = 0;    // the narrow backward products (jobs)
    // wide-mode tiles (d_nd_wide): f_S forming, forward rows, backward rows
    int fm_off = 0, fm_n = 0, wf_off = 0, wf_n = 0, wb_off = 0, wb_n = 0;
    // factor bytes and front cells of the narrow and wide, forward and backward products
    double nf_bytes = 0, nb_bytes = 0, nf_cells = 0, nb_cells = 0;
    double wf_bytes = 0, wb_bytes = 0, wf_cells = 0, wb_cells = 0;
  };
  struct NdLaunch {
    std::vector<NdLevel> levels; // level 0 = the subtree roots (levels above the fusion level)
    int fj_off = 0, fj_n = 0;    // fused subtrees (d_nd_fj)
    double fu_fbytes = 0, fu_bbytes = 0, fu_cells = 0;   // their factor bytes; front cells
    int top_off = 0, ntop = 0;   // dense-top jobs (d_nd_top)
    double top_bytes = 0, top_cells = 0;
    long long upd = 0;           // update-vector entries per RHS of the members
  };
  // Per level, over every shape of the plan: the largest narrow node (forward:
  // rows nbd, columns ns; backward: rows ns, columns nf).  A level's launch
  // shape follows from these alone, so a node's arithmetic never depends on
  // which other nodes share its launch.
  struct NdLevelMax {
    int f_rows = 0, f_cols = 0, f_nf = 0, b_rows = 0, b_cols = 0;
  };
  std::vector<NdLevelMax> nd_lvmax;
  std::vector<NdShape> nd_shapes;
  std::vector<NdShapeTab> nd_tabs;
  std::vector<int> nd_shape_of;                      // per subdomain
  std::vector<NdLaunch> nd_launch;                   // per launch group
  std::vector<NdLaunch> nd_local;                    // per subdomain (local solves)
  Buf d_nd_nodes, d_nd_cells, d_nd_maps, d_nd_umaps, d_nd_src, d_nd_usrc, d_nd_lev, d_nd_levmax,
      d_nd_levnodes;
  Buf d_nd_lvl, d_nd_top, d_upool;
  long long nd_upd_max = 0;                          // entries per RHS of the update pool
  int nd_max_nf = 0, nd_max_ntop = 0;   // largest subtree front; largest dense top
  int nd_wide = 1024;                   // fronts of at least this size run in wide mode
  int nd_max_nf_narrow = 0;             // largest front below nd_wide
  Buf d_nd_wide;                        // wide-mode tiles {job, first row}
  int nd_fuse_level = 1 << 30;          // subtree levels from here down run fused
  // pivot report: the largest max|pivot| / min|pivot| over the inversions of
  // the factorisation, and its subdomain
  double piv_ratio = 0.0;
  int piv_sub = -1;
  Buf d_nd_fj, d_nd_fb;                 // fused subtrees {first batch, batches}; batches {job, jobs}
  std::vector<int> nd_cell_of, nd_map_of;  // per node-table entry: cell and map offsets
  int nd_small = 4;    // levels whose largest node needs at most this many (row pass x
                       // column) / 64 run one node per wave
  // Krylov workspace
  Buf d_V, d_Z, d_w, d_r, d_xa, d_ba, d_part, d_h1, d_h2, d_hn, d_scal, d_idx, d_coef;
  int kr_restart = 0, kr_k = 0;
  // FWI workspace
  Buf d_res, d_adj, d_y, d_mpart, d_u;

  hipStream_t stream = nullptr;
  // timing: an event pair around every solve launch, recorded without waiting
  // (so the launches stay back to back) and read once the application is done
  bool timing = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::vector<hipEvent_t> tev;
  size_t tev_used = 0;
  double t_solve_ms = 0, t_other_ms = 0, solve_bytes = 0, solve_flops = 0;
  long long solve_launches = 0;

  // captured preconditioner applications, keyed by (f, u, nrhs)
  bool use_graph = false;
  hipStream_t cap_stream = nullptr;
  std::map<std::tuple<const void*, void*, int>, hipGraphExec_t> graphs;

  ~dsd_plan() {
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    for (hipEvent_t e : tev) (void)hipEventDestroy(e);
  }
};

// Pivot report of a set of inversions: stats (2 doubles per job, the smallest
// and largest squared pivot magnitude) start at (+inf, 0); piv_end folds them
// into the plan's largest max|pivot| / min|pivot| and its subdomain.
int piv_begin(Buf& d, size_t njobs) {
  std::vector<double> h(2 * std::max<size_t>(njobs, 1), 0.0);
  for (size_t k = 0; k < njobs; ++k) h[2 * k] = HUGE_VAL;
  return upload(d, h);
}
int piv_end(dsd_plan* pl, const Buf& d, const std::vector<int>& sub_of_job) {
  if (sub_of_job.empty()) return 0;
  std::vector<double> h(2 * sub_of_job.size());
  HIPCHK(hipMemcpyAsync(h.data(), d.p, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                        pl->stream));
  HIPCHK(hipStreamSynchronize(pl->stream));
  for (size_t k = 0; k < sub_of_job.size(); ++k) {
    if (!(h[2 * k + 1] > 0.0)) continue;
    const double r = h[2 * k] > 0.0 ? std::sqrt(h[2 * k + 1] / h[2 * k]) : HUGE_VAL;
    if (r > pl->piv_ratio) {
      pl->piv_ratio = r;
      pl->piv_sub = sub_of_job[k];
    }
  }
  return 0;
}

namespace {

size_t tsize(const dsd_plan* p) { return p->c64 ? sizeof(cpx<float>) : sizeof(cpx<double>); }

int build_partition(dsd_plan* pl) {
  const dsd_params& q = pl->prm;
  Problem& P = pl->P;
  P.dim = q.dim;
  P.pml = q.pml;
  P.d = q.overlap;
  P.h = q.h;
  P.omega = pl->omega;
  P.s0d = q.sigma0_delta > 0 ? q.sigma0_delta : 60.0;
  P.N = 1;
  for (int a = 0; a < 3; ++a) {
    P.n[a] = a < q.dim ? q.n[a] : 1;
    P.ng[a] = a < q.dim ? q.n[a] + 2 * q.pml : 1;
    P.N *= P.ng[a];
  }
  // axis partitions: array_split of the physical cells, larger parts first
  for (int a = 0; a < 3; ++a) {
    pl->parts[a].clear();
    if (a >= q.dim) {
      pl->parts[a].push_back(AxisPart{0, 1, 1, 1});
      continue;
    }
    const int n = q.n[a], Pp = q.parts[a];
    int q0 = 0;
    for (int p = 0; p < Pp; ++p) {
      const int len = n / Pp + (p < n % Pp ? 1 : 0);
      const int q1 = q0 + len;
      if (Pp > 1 && len < q.overlap) {
        g_detail = "axis " + std::to_string(a) + " part " + std::to_string(p) +
                   " owns fewer cells than the overlap";
        return DSD_EINVAL;
      }
      // an interior part must own >= 2d-2 cells, so that no cell lies in the
      // cutoff support of three parts of an axis (the assembly of u_DDM relies on it)
      if (p > 0 && p < Pp - 1 && len < 2 * q.overlap - 2) {
        g_detail = "axis " + std::to_string(a) + " part " + std::to_string(p) +
                   " owns fewer than 2*overlap-2 cells";
        return DSD_EINVAL;
      }
      AxisPart ap;
      ap.o0 = p == 0 ? 0 : q0 + q.pml;
      ap.o1 = p == Pp - 1 ? n + 2 * q.pml : q1 + q.pml;
      ap.first = p == 0;
      ap.last = p == Pp - 1;
      pl->parts[a].push_back(ap);
      q0 = q1;
    }
  }
  // subdomains (x part fastest)
  const int Px = q.parts[0], Py = q.parts[1], Pz = q.dim == 3 ? q.parts[2] : 1;
  pl->S = Px * Py * Pz;
  pl->subs.assign(pl->S, SubDesc{});
  long long coff = 0, foff = 0;
  pl->max_nb = 0;
  for (int iz = 0; iz < Pz; ++iz)
    for (int iy = 0; iy < Py; ++iy)
      for (int ix = 0; ix < Px; ++ix) {
        const int sid = (iz * Py + iy) * Px + ix;
        SubDesc& S = pl->subs[sid];
        const int pidx[3] = {ix, iy, iz};
        S.nloc = 1;
        for (int a = 0; a < 3; ++a) {
          S.part[a] = pidx[a];
          S.pt[a] = pl->parts[a][pidx[a]];
          if (a >= q.dim) {
            S.ax[a] = AxisGrid{0, 1, -1e300, 1e300, q.pml, q.pml};
            S.dims[a] = 1;
            continue;
          }
          const int n = q.n[a], Pp = q.parts[a], d = q.overlap, pm = q.pml;
          const AxisPart& ap = S.pt[a];
          const int q0 = ap.first ? 0 : ap.o0 - pm;        // physical own range
          const int q1 = ap.last ? n : ap.o1 - pm;
          AxisGrid g;
          g.g0 = ap.first ? 0 : q0 - d;
          const int g1 = ap.last ? n + 2 * pm : q1 + d + 2 * pm;
          g.n = g1 - g.g0;
          g.lo = ap.first ? 0.0 : (q0 - d) * q.h;
          g.hi = ap.last ? n * q.h : (q1 + d) * q.h;
          g.clo = ap.first ? pm : q0 - d + pm;
          g.chi = ap.last ? n + pm - 1 : q1 + d + pm - 1;
          (void)Pp;
          S.ax[a] = g;
          S.dims[a] = g.n;
          S.nloc *= g.n;
        }
        if (q.dim == 2) {
          S.nb = S.dims[0];
          S.nblk = S.dims[1];
        } else {
          S.nb = S.dims[0] * S.dims[1];
          S.nblk = S.dims[2];
        }
        S.mid = S.nblk / 2;
        S.coef_off = coff;
        S.vec_off = coff;
        S.fac_off = foff;
        coff += S.nloc;
        foff += (long long)S.nblk * S.nb * S.nb;
        pl->max_nb = std::max(pl->max_nb, S.nb);
      }
  pl->sum_nloc = coff;
  pl->sum_fac = foff;
  return 0;
}

int sub_index(const dsd_plan* pl, const int* pidx) {
  for (int a = 0; a < pl->dim; ++a)
    if (pidx[a] < 0 || pidx[a] >= pl->prm.parts[a]) return -1;
  const int Px = pl->prm.parts[0], Py = pl->prm.parts[1];
  const int z = pl->dim == 3 ? pidx[2] : 0;
  return (z * Py + pidx[1]) * Px + pidx[0];
}

void bcr_group_jobs(const dsd_plan* pl, const std::vector<int2>& mem, std::vector<BcrJob>& jobs,
                    std::vector<BcrLaunch>& out);
int bcr_check_jobs(const dsd_plan* pl, const std::vector<BcrJob>& jobs, bool local = false);
void chain_step_jobs(const dsd_plan* pl, const std::vector<int2>& mem, std::vector<BcrJob>& jobs,
                     std::vector<BcrLaunch>& out);
// jobs of one launch group (or one subdomain) with the plan's local solver
void solve_jobs(const dsd_plan* pl, const std::vector<int2>& mem, std::vector<BcrJob>& jobs,
                std::vector<BcrLaunch>& out) {
  if (pl->solver == 2) bcr_group_jobs(pl, mem, jobs, out);
  else chain_step_jobs(pl, mem, jobs, out);
}

int build_nd_jobs(dsd_plan* pl);

// Solve-job tables of the cyclic reduction (or of the chain block steps, or
// of the nested dissection) for every launch group.
int build_bcr_jobs(dsd_plan* pl) {
  pl->bcr_launch.clear();
  if (pl->solver == 4) return build_nd_jobs(pl);
  if (pl->solver != 2 && !pl->chain_steps) return 0;
  std::vector<BcrJob> bj;
  for (auto& grp : pl->groups) {
    pl->bcr_launch.emplace_back();
    solve_jobs(pl, grp, bj, pl->bcr_launch.back());
  }
  CHK(bcr_check_jobs(pl, bj));
  CHK(upload(pl->d_bcr_jobs, bj));
  return 0;
}

int build_schedule(dsd_plan* pl) {
  const int dim = pl->dim, L = pl->L;
  const dsd_params& q = pl->prm;
  // additive DDM (Algorithms 2.1 / 2.2): every subdomain at every step; step s
  // keeps its solutions in slot (s - 1) mod (dim + 1), which holds them while
  // steps s + 1 .. s + dim read them (a neighbour at L1 distance |t| reads the
  // solution of step s - |t|)
  const bool additive = pl->additive;
  const int Ls = additive ? dim + 1 : L;
  int nsteps = 1;
  for (int a = 0; a < dim; ++a) nsteps += q.parts[a] - 1;
  pl->nsteps = nsteps;
  std::vector<Edge> edges;
  // incoming transfers of every (sweep, receiver), in a fixed direction order
  std::vector<int2> edge_of((size_t)L * pl->S);
  std::vector<int> tdirs;
  for (int tz = (dim == 3 ? -1 : 0); tz <= (dim == 3 ? 1 : 0); ++tz)
    for (int ty = -1; ty <= 1; ++ty)
      for (int tx = -1; tx <= 1; ++tx) {
        if (tx == 0 && ty == 0 && tz == 0) continue;
        tdirs.push_back(tx);
        tdirs.push_back(ty);
        tdirs.push_back(tz);
      }
  const int ndir = (int)tdirs.size() / 3;
  for (int l = 0; l < Ls; ++l)
    for (int rid = 0; rid < pl->S; ++rid) {
      const SubDesc& R = pl->subs[rid];
      const int start = (int)edges.size();
      for (int di = 0; di < ndir; ++di) {
        const int* t = &tdirs[3 * di];
        int sp[3] = {R.part[0] - t[0], R.part[1] - t[1], R.part[2] - t[2]};
        const int sid = sub_index(pl, sp);
        if (sid < 0) continue;
        unsigned mask = 0;
        if (additive) {
          const int dist = std::abs(t[0]) + std::abs(t[1]) + std::abs(t[2]);
          mask = 1u << (((l - dist) % Ls + Ls) % Ls);
        } else {
          for (int lg = 0; lg <= l; ++lg)
            if (route(dim, q.sweep_order, lg, t) == l) mask |= 1u << lg;
        }
        if (!mask) continue;
        const SubDesc& Sd = pl->subs[sid];
        Edge e{};
        e.sender = sid;
        e.lmask = mask;
        for (int a = 0; a < 3; ++a) {
          e.t[a] = t[a];
          e.off[a] = R.ax[a].g0 - Sd.ax[a].g0;
          if (a >= dim || t[a] == 0) {
            e.lo[a] = 0;
            e.hi[a] = R.dims[a];
            if (a < dim && (R.ax[a].g0 != Sd.ax[a].g0 || R.dims[a] != Sd.dims[a])) {
              g_detail = "tangential grids of neighbours differ";
              return DSD_EINVAL;
            }
          } else if (t[a] > 0) {
            const int e0 = Sd.pt[a].o1 - R.ax[a].g0;   // receiver's first own cell
            e.lo[a] = e0;
            e.hi[a] = e0 + q.overlap;
          } else {
            const int e1 = Sd.pt[a].o0 - R.ax[a].g0;   // one past the receiver's last own cell
            e.lo[a] = e1 - q.overlap;
            e.hi[a] = e1;
          }
          if (e.lo[a] < 0 || e.hi[a] > R.dims[a] || e.lo[a] + e.off[a] < 0 ||
              e.hi[a] + e.off[a] > Sd.dims[a]) {
            g_detail = "transfer box outside a local grid";
            return DSD_EINVAL;
          }
        }
        edges.push_back(e);
      }
      edge_of[(size_t)l * pl->S + rid] = make_int2(start, (int)edges.size() - start);
    }
  // Launch groups.  Sequential: the anti-diagonal steps of every sweep in
  // order (Algorithms 3.1 / 4.1).  DAG: every (sweep, subdomain) solve is
  // launched at 1 + the latest launch group of the solves its transfers come
  // from; the sources and their summation order are unchanged, so both
  // schedules give identical results.
  std::vector<int> level((size_t)L * pl->S, 0);
  std::vector<std::vector<int2>> groups;
  if (additive)
    for (int st = 0; st < nsteps; ++st) {
      groups.emplace_back();
      for (int sid = 0; sid < pl->S; ++sid) groups.back().push_back(make_int2(sid, st % Ls));
    }
  for (int l = 0; l < (additive ? 0 : L); ++l) {
    const int* D = sweep_dir(dim, pl->prm.sweep_order, l);
    std::vector<std::vector<int>> steps(nsteps);
    for (int sid = 0; sid < pl->S; ++sid) {
      const SubDesc& S = pl->subs[sid];
      int st = 0;
      for (int a = 0; a < dim; ++a) st += D[a] > 0 ? S.part[a] : q.parts[a] - 1 - S.part[a];
      steps[st].push_back(sid);
    }
    for (int s = 0; s < nsteps; ++s)
      for (int sid : steps[s]) {
        int lev;
        if (pl->sequential) {
          lev = l * nsteps + s;
        } else {
          lev = 0;
          const int2 er = edge_of[(size_t)l * pl->S + sid];
          for (int e = er.x; e < er.x + er.y; ++e)
            for (int lg = 0; lg < L; ++lg)
              if (edges[e].lmask & (1u << lg))
                lev = std::max(lev, level[(size_t)lg * pl->S + edges[e].sender] + 1);
        }
        level[(size_t)l * pl->S + sid] = lev;
        if ((int)groups.size() <= lev) groups.resize(lev + 1);
        groups[lev].push_back(make_int2(sid, l));
      }
  }
  std::vector<int2> members, erange;
  std::vector<int4> jobs2, jobs1;
  pl->steps.clear();
  for (auto& grp : groups) {
    StepTab T{};
    T.mem_off = (int)members.size();
    T.nmem = (int)grp.size();
    T.job_off = (int)jobs2.size();
    T.er_off = (int)erange.size();
    for (const int2& mb : grp) {
      const SubDesc& S = pl->subs[mb.x];
      members.push_back(mb);
      jobs2.push_back(make_int4(mb.x, 0, mb.y, 0));
      jobs2.push_back(make_int4(mb.x, 1, mb.y, 0));
      jobs1.push_back(make_int4(mb.x, 0, mb.y, 0));
      const int2 er = edge_of[(size_t)mb.y * pl->S + mb.x];
      if (er.y > MAX_IN_EDGES) {
        g_detail = "internal error: more incoming transfers than the pull kernel stages";
        return DSD_EINVAL;
      }
      erange.push_back(er);
      long long box = 0;
      for (int e = er.x; e < er.x + er.y; ++e)
        box += (long long)(edges[e].hi[0] - edges[e].lo[0]) * (edges[e].hi[1] - edges[e].lo[1]) *
               (edges[e].hi[2] - edges[e].lo[2]);
      T.max_box = std::max(T.max_box, box);
      T.max_nloc = std::max(T.max_nloc, S.nloc);
      const double blk = (double)S.nb * S.nb * tsize(pl);
      T.fac_bytes_fb += (double)(S.nblk - 1) * blk;
      T.fac_bytes_mid += blk;
      T.blk_cells_fb += (long long)(S.nblk - 1) * S.nb;
      T.blk_cells_mid += S.nb;
    }
    pl->steps.push_back(T);
  }
  pl->groups = groups;
  CHK(build_bcr_jobs(pl));
  CHK(upload(pl->d_members, members));
  CHK(upload(pl->d_jobs2, jobs2));
  CHK(upload(pl->d_jobs1, jobs1));
  CHK(upload(pl->d_edges, edges));
  CHK(upload(pl->d_erange, erange));
  // part tables for the assembly of u_DDM
  for (int a = 0; a < 3; ++a) {
    std::vector<int> po(pl->P.ng[a], 0);
    for (int g = 0; g < pl->P.ng[a]; ++g)
      for (int p = 0; p < (int)pl->parts[a].size(); ++p)
        if (g >= pl->parts[a][p].o0 && g < pl->parts[a][p].o1) po[g] = p;
    CHK(upload(pl->d_part_of[a], po));
    CHK(upload(pl->d_axparts[a], pl->parts[a]));
  }
  return 0;
}

// ------------------------------------------------------ block cyclic reduction
// Level of the reduction solved densely: the first level >= 1 with at most
// dense_max blocks, unless that is the single top block.
int dense_level(const BcrSub& B, int dense_max) {
  if (dense_max < 2) return -1;
  for (int l = 1; l < B.top; ++l)
    if ((int)B.lev[l].size() <= dense_max) return l;
  return -1;
}
// last level of the reduction a subdomain's solve runs level by level
inline int etop(const BcrSub& B) { return B.dtop >= 0 ? B.dtop : B.top; }

// Level structure and factor layout: P_k = D_k^{-1} of every block at
// fac_off + k nb^2, then the W blocks of the blocks eliminated at levels >= 1
// below the dense level, then the dm row blocks (nb x dm nb) of the inverse of
// the reduced system at the dense level.
void bcr_layout(dsd_plan* pl) {
  pl->bcr.assign(pl->S, BcrSub{});
  long long foff = 0;
  for (int sid = 0; sid < pl->S; ++sid) {
    SubDesc& S = pl->subs[sid];
    BcrSub& B = pl->bcr[sid];
    const long long nb2 = (long long)S.nb * S.nb;
    std::vector<int> all(S.nblk);
    for (int k = 0; k < S.nblk; ++k) all[k] = k;
    B.lev.push_back(all);
    while (B.lev.back().size() > 1) {
      const std::vector<int>& c = B.lev.back();
      std::vector<int> nxt;
      for (size_t q = 1; q < c.size(); q += 2) nxt.push_back(c[q]);
      B.lev.push_back(nxt);
    }
    B.top = (int)B.lev.size() - 1;
    B.dtop = dense_level(B, pl->dense_max);
    B.dm = B.dtop >= 0 ? (int)B.lev[B.dtop].size() : 0;
    B.wl.assign(S.nblk, -1);
    B.wr.assign(S.nblk, -1);
    B.wlt.assign(S.nblk, -1);
    B.wrt.assign(S.nblk, -1);
    S.fac_off = foff;
    long long slot = S.nblk;
    for (int l = 1; l < etop(B); ++l) {
      const std::vector<int>& c = B.lev[l];
      for (size_t p = 0; p < c.size(); p += 2) {
        const int k = c[p];
        if (p > 0) {
          B.wl[k] = foff + slot++ * nb2;
          B.wlt[k] = foff + slot++ * nb2;
        }
        if (p + 1 < c.size()) {
          B.wr[k] = foff + slot++ * nb2;
          B.wrt[k] = foff + slot++ * nb2;
        }
      }
    }
    if (B.dtop >= 0) {
      B.dense = foff + slot * nb2;
      slot += (long long)B.dm * B.dm;
    }
    foff += slot * nb2;
  }
  pl->sum_fac = foff;
}

// Runs `fn(first, count)` over [0, n) in pieces the grid's y dimension holds.
template <typename F>
void in_chunks(int n, F fn) {
  const int cap = 65535;
  for (int i = 0; i < n; i += cap) fn(i, std::min(cap, n - i));
}

// FP64 factorisation by block cyclic reduction, subdomains in batches sized to
// the free device memory.  Level 0 has the diagonal couplings of the stencil
// (elementwise updates); the deeper levels use batched GEMMs.
int bcr_factor(dsd_plan* pl) {
  hipStream_t st = pl->stream;
  const Problem& P = pl->P;
  CHK(pl->d_fac.alloc((size_t)pl->sum_fac * tsize(pl)));
  const long long blk = (long long)pl->max_nb * pl->max_nb;
  int maxblk = 1;
  for (const SubDesc& S : pl->subs) maxblk = std::max(maxblk, S.nblk);
  const long long half = maxblk / 2 + 1;
  const long long slots = maxblk + 4 * half;             // D, E (two levels), W_L, W_R
  const long long per_sub = slots * blk;                 // complex entries per subdomain
  long long dn_max = 0;                                  // order of the largest dense system
  for (int sid = 0; sid < pl->S; ++sid)
    if (pl->bcr[sid].dtop >= 0) dn_max = std::max(dn_max, (long long)pl->bcr[sid].dm * pl->subs[sid].nb);
  const long long dn2 = dn_max * dn_max;
  size_t freeb = 0, totb = 0;
  HIPCHK(hipMemGetInfo(&freeb, &totb));
  const long long budget = std::min<long long>((long long)(freeb / 2), 48LL << 30);
  int batch = (int)std::max<long long>(1, budget / ((per_sub + dn2) * (long long)sizeof(cpx<double>)));
  batch = std::min(batch, pl->S);
  Buf work, derr, dpiv, drbuf, dj, dwork, dpivd, drbufd;
  CHK(work.alloc((size_t)batch * per_sub * sizeof(cpx<double>)));
  if (dn_max > 0) {
    CHK(dwork.alloc((size_t)batch * dn2 * sizeof(cpx<double>)));
    CHK(dpivd.alloc((size_t)batch * dn_max * sizeof(int)));
    CHK(drbufd.alloc((size_t)batch * gj_rbuf_entries((int)dn_max) * sizeof(cpx<double>)));
  }
  long long ninv = 0;
  for (const SubDesc& S : pl->subs) ninv += S.nblk + 1;
  CHK(derr.alloc((size_t)ninv * sizeof(int)));
  HIPCHK(hipMemsetAsync(derr.p, 0, (size_t)ninv * sizeof(int), st));
  Buf dpst;
  CHK(piv_begin(dpst, (size_t)ninv));
  std::vector<int> job_sub;              // subdomain of every inversion, in err_off order
  const int maxinv = std::min(batch * (int)half, 2048);   // inversions per launch
  CHK(dpiv.alloc((size_t)maxinv * pl->max_nb * sizeof(int)));
  CHK(drbuf.alloc((size_t)maxinv * gj_rbuf_entries(pl->max_nb) * sizeof(cpx<double>)));
  cpx<double>* W = work.as<cpx<double>>();
  const cpx<double>* c64d[4] = {pl->d_lcoef64[0].as<cpx<double>>(), pl->d_lcoef64[1].as<cpx<double>>(),
                                pl->d_lcoef64[2].as<cpx<double>>(), pl->d_lcoef64[3].as<cpx<double>>()};
  long long err_off = 0;
  std::vector<unsigned char> hbuf;
  // uploads a job vector into dj (the previous launches on the stream are done with it)
  auto put = [&](const void* data, size_t bytes) -> int {
    HIPCHK(hipStreamSynchronize(st));
    if (dj.bytes < bytes) CHK(dj.alloc(std::max<size_t>(bytes, 1 << 20)));
    HIPCHK(hipMemcpy(dj.p, data, bytes, hipMemcpyHostToDevice));
    return 0;
  };
  for (int s0 = 0; s0 < pl->S; s0 += batch) {
    const int s1 = std::min(pl->S, s0 + batch);
    auto slot = [&](int sid, long long k) { return ((long long)(sid - s0) * slots + k) * blk; };
    auto D = [&](int sid, int k) { return slot(sid, k); };
    auto E = [&](int sid, int which, long long e) { return slot(sid, maxblk + which * half + e); };
    auto WL = [&](int sid, long long e) { return slot(sid, maxblk + 2 * half + e); };
    auto WR = [&](int sid, long long e) { return slot(sid, maxblk + 3 * half + e); };
    const long long wend = (long long)(s1 - s0) * per_sub;   // working entries in use
    // every block a job touches must lie inside its buffer (checked before any launch)
    auto inw = [&](long long off, int nb) { return off >= 0 && off + (long long)nb * nb <= wend; };
    auto inf = [&](long long off, int nb) { return off >= 0 && off + (long long)nb * nb <= pl->sum_fac; };
    bool bad_off = false;
    {
      std::vector<BcrBlkJob> aj;
      for (int sid = s0; sid < s1; ++sid)
        for (int k = 0; k < pl->subs[sid].nblk; ++k) {
          aj.push_back(BcrBlkJob{sid, k, D(sid, k)});
          bad_off |= !inw(D(sid, k), pl->subs[sid].nb);
        }
      if (bad_off) {
        g_detail = "internal error: cyclic-reduction assembly job outside its buffer";
        return DSD_EINVAL;
      }
      CHK(put(aj.data(), aj.size() * sizeof(BcrBlkJob)));
      in_chunks((int)aj.size(), [&](int i0, int n) {
        launch_bcr_assemble(P, pl->d_subs.as<SubDesc>(), dj.as<BcrBlkJob>() + i0, n, pl->max_nb,
                            c64d[0], c64d[1], c64d[2], W, st);
      });
      HIPCHK(hipGetLastError());
    }
    int maxtop = 0;
    for (int sid = s0; sid < s1; ++sid) maxtop = std::max(maxtop, etop(pl->bcr[sid]));
    for (int l = 0; l <= maxtop; ++l) {
      std::vector<BcrInvJob> inv;
      std::vector<BcrDiagUpd> du;
      std::vector<ZGemmJob> gw, gd1, gd2, ge;
      std::vector<BcrCopyJob> cp;
      std::vector<BcrDenseJob> dns;
      std::vector<int> dns_sub;
      const int rd = l & 1, wr_ = (l + 1) & 1;
      for (int sid = s0; sid < s1; ++sid) {
        const BcrSub& B = pl->bcr[sid];
        if (l > etop(B)) continue;
        const SubDesc& S = pl->subs[sid];
        const int nb = S.nb;
        const long long nb2 = (long long)nb * nb;
        const std::vector<int>& c = B.lev[l];
        const int len = (int)c.size();
        if (l == B.dtop) {
          // the reduced system left at this level, inverted as one dense matrix
          const int first = c[0], stride = c[1] - c[0];
          for (int q = 0; q < len; ++q) bad_off |= c[q] != first + q * stride;
          const long long n = (long long)len * nb;
          const BcrDenseJob dj_{nb, len, first, stride, blk, D(sid, 0), E(sid, rd, 0),
                                (long long)(sid - s0) * dn2, B.dense};
          for (int q = 0; q < len; ++q) bad_off |= !inw(D(sid, c[q]), nb);
          for (int q = 0; q + 1 < len; ++q) bad_off |= !inw(E(sid, rd, q), nb);
          bad_off |= n > dn_max || dj_.out + n * n > (long long)batch * dn2 ||
                     B.dense < 0 || B.dense + n * n > pl->sum_fac;
          dns.push_back(dj_);
          dns_sub.push_back(sid);
          continue;
        }
        for (int p = 0; p < len; p += 2)
          inv.push_back(BcrInvJob{nb, sid, D(sid, c[p]), S.fac_off + (long long)c[p] * nb2});
        if (l == B.top) continue;
        if (l == 0) {
          for (int q = 1; q < len; q += 2) {
            const int j = c[q];
            du.push_back(BcrDiagUpd{sid, j, D(sid, j), D(sid, j - 1),
                                    j + 1 < S.nblk ? D(sid, j + 1) : -1,
                                    j + 2 < S.nblk ? E(sid, wr_, (q - 1) / 2) : -1});
          }
          continue;
        }
        for (int p = 0; p < len; p += 2) {
          const int k = c[p];
          if (p > 0) {
            gw.push_back(ZGemmJob{nb, 0, 1, 0, 1.0, D(sid, k), E(sid, rd, p - 1), WL(sid, p / 2)});
            cp.push_back(BcrCopyJob{nb, 0, WL(sid, p / 2), B.wl[k]});
            cp.push_back(BcrCopyJob{nb, 1, WL(sid, p / 2), B.wlt[k]});
          }
          if (p + 1 < len) {
            gw.push_back(ZGemmJob{nb, 0, 0, 0, 1.0, D(sid, k), E(sid, rd, p), WR(sid, p / 2)});
            cp.push_back(BcrCopyJob{nb, 0, WR(sid, p / 2), B.wr[k]});
            cp.push_back(BcrCopyJob{nb, 1, WR(sid, p / 2), B.wrt[k]});
          }
        }
        for (int q = 1; q < len; q += 2) {
          const int j = c[q];
          gd1.push_back(ZGemmJob{nb, 1, 0, 1, -1.0, E(sid, rd, q - 1), WR(sid, (q - 1) / 2), D(sid, j)});
          if (q + 1 < len)
            gd2.push_back(ZGemmJob{nb, 0, 0, 1, -1.0, E(sid, rd, q), WL(sid, (q + 1) / 2), D(sid, j)});
          if (q + 2 < len)
            ge.push_back(ZGemmJob{nb, 0, 0, 0, -1.0, E(sid, rd, q), WR(sid, (q + 1) / 2),
                                  E(sid, wr_, (q - 1) / 2)});
        }
      }
      for (const BcrInvJob& j : inv) bad_off |= !inw(j.src, j.nb) || !inf(j.dst, j.nb);
      for (const BcrDiagUpd& j : du) {
        const int nb = pl->subs[j.sub].nb;
        bad_off |= !inw(j.d, nb) || !inw(j.pl, nb) || (j.pr >= 0 && !inw(j.pr, nb)) ||
                   (j.eout >= 0 && (j.pr < 0 || !inw(j.eout, nb)));
      }
      for (const std::vector<ZGemmJob>* v : {&gw, &gd1, &gd2, &ge})
        for (const ZGemmJob& j : *v) bad_off |= !inw(j.a, j.nb) || !inw(j.b, j.nb) || !inw(j.c, j.nb);
      for (const BcrCopyJob& j : cp) bad_off |= !inw(j.src, j.nb) || !inf(j.dst, j.nb);
      if (bad_off) {
        g_detail = "internal error: cyclic-reduction factor job outside its buffer";
        return DSD_EINVAL;
      }
      if (!dns.empty()) {
        // dense top level: assemble, invert in FP64 (Gauss-Jordan), round into row blocks
        std::vector<BcrInvJob> dinv;
        for (size_t k = 0; k < dns.size(); ++k)
          dinv.push_back(BcrInvJob{dns[k].nb * dns[k].m, dns_sub[k], dns[k].out, -1});
        std::vector<unsigned char> pack(dns.size() * sizeof(BcrDenseJob) + dinv.size() * sizeof(BcrInvJob));
        memcpy(pack.data(), dns.data(), dns.size() * sizeof(BcrDenseJob));
        memcpy(pack.data() + dns.size() * sizeof(BcrDenseJob), dinv.data(), dinv.size() * sizeof(BcrInvJob));
        CHK(put(pack.data(), pack.size()));
        const BcrDenseJob* ddj = dj.as<BcrDenseJob>();
        const BcrInvJob* dij = reinterpret_cast<const BcrInvJob*>(dj.as<unsigned char>() +
                                                                   dns.size() * sizeof(BcrDenseJob));
        cpx<double>* DW = dwork.as<cpx<double>>();
        launch_bcr_dense_build(ddj, (int)dns.size(), (int)dn_max, W, DW, st);
        if (pl->c64) {
          launch_bcr_invert<float>(dij, (int)dinv.size(), (int)dn_max, DW, pl->d_fac.as<cpx<float>>(),
                                   derr.as<int>() + err_off, dpivd.as<int>(), drbufd.as<cpx<double>>(),
                                   dpst.as<double>() + 2 * err_off, st);
          launch_bcr_dense_store<float>(ddj, (int)dns.size(), (int)dn_max, DW, pl->d_fac.as<cpx<float>>(), st);
        } else {
          launch_bcr_invert<double>(dij, (int)dinv.size(), (int)dn_max, DW, pl->d_fac.as<cpx<double>>(),
                                    derr.as<int>() + err_off, dpivd.as<int>(), drbufd.as<cpx<double>>(),
                                    dpst.as<double>() + 2 * err_off, st);
          launch_bcr_dense_store<double>(ddj, (int)dns.size(), (int)dn_max, DW,
                                         pl->d_fac.as<cpx<double>>(), st);
        }
        err_off += (long long)dinv.size();
        job_sub.insert(job_sub.end(), dns_sub.begin(), dns_sub.end());
        HIPCHK(hipGetLastError());
      }
      // inversions of the eliminated blocks (FP64 in place; rounded copy into the factor)
      CHK(put(inv.data(), inv.size() * sizeof(BcrInvJob)));
      for (int i0 = 0; i0 < (int)inv.size(); i0 += maxinv) {
        const int n = std::min(maxinv, (int)inv.size() - i0);
        if (pl->c64)
          launch_bcr_invert<float>(dj.as<BcrInvJob>() + i0, n, pl->max_nb, W, pl->d_fac.as<cpx<float>>(),
                                   derr.as<int>() + err_off, dpiv.as<int>(), drbuf.as<cpx<double>>(),
                                   dpst.as<double>() + 2 * err_off, st);
        else
          launch_bcr_invert<double>(dj.as<BcrInvJob>() + i0, n, pl->max_nb, W,
                                    pl->d_fac.as<cpx<double>>(), derr.as<int>() + err_off,
                                    dpiv.as<int>(), drbuf.as<cpx<double>>(),
                                    dpst.as<double>() + 2 * err_off, st);
        for (int k = i0; k < i0 + n; ++k) job_sub.push_back(inv[k].sub);
        err_off += n;
      }
      HIPCHK(hipGetLastError());
      if (!du.empty()) {
        CHK(put(du.data(), du.size() * sizeof(BcrDiagUpd)));
        in_chunks((int)du.size(), [&](int i0, int n) {
          launch_bcr_diag_update(P, pl->d_subs.as<SubDesc>(), dj.as<BcrDiagUpd>() + i0, n,
                                 pl->max_nb, c64d[2], c64d[3], W, st);
        });
        HIPCHK(hipGetLastError());
      }
      auto gemm = [&](const std::vector<ZGemmJob>& v) -> int {
        if (v.empty()) return 0;
        CHK(put(v.data(), v.size() * sizeof(ZGemmJob)));
        launch_zgemm(dj.as<ZGemmJob>(), (int)v.size(), pl->max_nb, W, st);
        HIPCHK(hipGetLastError());
        return 0;
      };
      CHK(gemm(gw));
      if (!cp.empty()) {
        CHK(put(cp.data(), cp.size() * sizeof(BcrCopyJob)));
        in_chunks((int)cp.size(), [&](int i0, int n) {
          if (pl->c64)
            launch_bcr_copy<float>(dj.as<BcrCopyJob>() + i0, n, pl->max_nb, W, pl->d_fac.as<cpx<float>>(), st);
          else
            launch_bcr_copy<double>(dj.as<BcrCopyJob>() + i0, n, pl->max_nb, W, pl->d_fac.as<cpx<double>>(), st);
        });
        HIPCHK(hipGetLastError());
      }
      CHK(gemm(gd1));
      CHK(gemm(gd2));
      CHK(gemm(ge));
    }
  }
  std::vector<int> herr(ninv);
  HIPCHK(hipMemcpyAsync(herr.data(), derr.p, ninv * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (long long i = 0; i < ninv; ++i)
    if (herr[i]) {
      g_detail = "singular block in the cyclic reduction (inversion " + std::to_string(i) + ")";
      return DSD_EPIVOT;
    }
  return piv_end(pl, dpst, job_sub);
}

// Solve launches of one launch group (members {subdomain, sweep}): the forward
// reduction levels, then the backward substitution from the top level down.
// Local-solve tables of every subdomain, built once with the plan (the
// allocation-free local solve must not upload anything): the solve jobs of
// {subdomain, sweep 0} with vbase = 0, and descriptors with vec_off = 0 for the
// kernels that address vectors through them, so that the caller hands the
// subdomain's vector slice (plan pool or static scratch) as the pool base.
int resolve_scratch(int dev, void** out);   // the allocation-free local solve's scratch

int build_local_tables(dsd_plan* pl) {
  std::vector<SubDesc> sl = pl->subs;
  for (SubDesc& S : sl) S.vec_off = 0;
  CHK(upload(pl->d_subs_local, sl));
  pl->local_launch.assign(pl->S, {});
  if (pl->solver == 4) return 0;   // nested dissection: nd_local (build_nd_jobs)
  if (pl->solver != 2 && !pl->chain_steps) {
    // chains: per subdomain {sub, top half}, {sub, bottom half} (forward and
    // backward phases) and {sub, middle} (the middle block)
    std::vector<int4> cj;
    for (int s = 0; s < pl->S; ++s) {
      cj.push_back(make_int4(s, 0, 0, 0));
      cj.push_back(make_int4(s, 1, 0, 0));
      cj.push_back(make_int4(s, 0, 0, 0));
    }
    return upload(pl->d_local_jobs, cj);
  }
  std::vector<BcrJob> bj;
  for (int s = 0; s < pl->S; ++s) {
    const size_t first = bj.size();
    solve_jobs(pl, std::vector<int2>{make_int2(s, 0)}, bj, pl->local_launch[s]);
    for (size_t i = first; i < bj.size(); ++i) bj[i].vbase = 0;
  }
  CHK(bcr_check_jobs(pl, bj, true));
  CHK(upload(pl->d_local_jobs, bj));
  return 0;
}

void bcr_group_jobs(const dsd_plan* pl, const std::vector<int2>& mem, std::vector<BcrJob>& jobs,
                    std::vector<BcrLaunch>& out) {
  int maxtop = 0;
  for (const int2& m : mem) maxtop = std::max(maxtop, etop(pl->bcr[m.x]));
  const double ts = (double)tsize(pl);
  int maxblk = 1;
  for (const SubDesc& S : pl->subs) maxblk = std::max(maxblk, S.nblk);
  // Column groups of a level: wide levels (many blocks per subdomain) keep one
  // wave per row tile; the deep levels split the columns to shorten each job.
  // It depends on the level and the plan's thresholds only, never on the
  // launch, so every schedule sums every job in the same order.
  int cur_cg = 1, cur_rt = 0, cur_kg = 0;
  auto level_shape = [&](int lev) {
    const int per_sub = maxblk >> (lev + 1);
    cur_kg = 0;
    if (per_sub >= pl->cg_wide) { cur_cg = pl->wide_cg; cur_rt = pl->wide_rt; cur_kg = pl->wide_kg; }
    else if (per_sub >= pl->cg_mid) { cur_cg = pl->mid_cg; cur_rt = pl->mid_rt; }
    else { cur_cg = pl->deep_cg; cur_rt = pl->deep_rt; }
  };
  auto begin = [&](int dfwd) {
    return BcrLaunch{(int)jobs.size(), 0, dfwd, 1, cur_cg, cur_rt, cur_kg, 0.0, 0.0};
  };
  auto finish = [&](BcrLaunch& L) {
    L.n = (int)jobs.size() - L.off;
    if (L.n > 0) out.push_back(L);
  };
  auto add = [&](BcrLaunch& L, const int2& m, int blk, int mode, int nl, int nr, long long m0,
                 long long m1, long long m2, int nmat, int nvec, int pad = 0) {
    const SubDesc& S = pl->subs[m.x];
    jobs.push_back(BcrJob{m.x, m.y, blk, mode, nl, nr, S.nb, pad, m0, m1, m2, S.nloc,
                          S.vec_off * pl->kmax, S.coef_off});
    L.nset = std::max(L.nset, nmat);
    L.fbytes += (double)nmat * S.nb * S.nb * ts;
    L.vcells += (double)nvec * S.nb;
  };
  auto Pk = [&](const SubDesc& S, int k) { return S.fac_off + (long long)k * S.nb * S.nb; };
  for (int f = 0; f < maxtop; ++f) {
    level_shape(f);
    if (f == 0) {
      BcrLaunch L = begin(0);
      for (const int2& m : mem) {
        const SubDesc& S = pl->subs[m.x];
        if (pl->bcr[m.x].top == 0) continue;
        for (int k = 0; k < S.nblk; k += 2) add(L, m, k, BCR_PR, -1, -1, Pk(S, k), 0, 0, 1, 2);
      }
      finish(L);
      BcrLaunch Ld = begin(1);
      for (const int2& m : mem) {
        const SubDesc& S = pl->subs[m.x];
        if (pl->bcr[m.x].top == 0) continue;
        for (int k = 1; k < S.nblk; k += 2)
          add(Ld, m, k, BCR_DFWD, k - 1, k + 1 < S.nblk ? k + 1 : -1, 0, 0, 0, 0, 4);
      }
      finish(Ld);
      continue;
    }
    BcrLaunch L = begin(0);
    for (const int2& m : mem) {
      const BcrSub& B = pl->bcr[m.x];
      if (f >= etop(B)) continue;
      const std::vector<int>& c = B.lev[f];
      const int len = (int)c.size();
      for (int q = 1; q < len; q += 2) {
        const bool hr = q + 1 < len;
        add(L, m, c[q], BCR_KEPT, c[q - 1], hr ? c[q + 1] : -1, B.wrt[c[q - 1]],
            hr ? B.wlt[c[q + 1]] : 0, 0, 1 + (int)hr, 3 + (int)hr);
      }
    }
    finish(L);
  }
  for (int b = maxtop; b >= 0; --b) {
    // dense top levels: one job per block row of the inverse, in a launch of
    // their own (one row tile per workgroup)
    cur_cg = pl->dense_cg;
    cur_rt = 1;
    cur_kg = 0;
    BcrLaunch Ld = begin(0);
    for (const int2& m : mem) {
      const BcrSub& B = pl->bcr[m.x];
      const SubDesc& S = pl->subs[m.x];
      if (b != B.dtop) continue;
      const std::vector<int>& c = B.lev[b];
      const int len = (int)c.size();
      const long long rows = (long long)S.nb * len * S.nb;   // one row block: nb x (len nb)
      for (int q = 0; q < len; ++q)
        add(Ld, m, c[q], BCR_DENSE, c[0], c[1] - c[0], B.dense + q * rows, 0, 0, len, len + 1, len);
    }
    finish(Ld);
    level_shape(b);
    BcrLaunch L = begin(0);
    for (const int2& m : mem) {
      const BcrSub& B = pl->bcr[m.x];
      const SubDesc& S = pl->subs[m.x];
      if (b > etop(B) || b == B.dtop) continue;
      const std::vector<int>& c = B.lev[b];
      const int len = (int)c.size();
      if (b == B.top) {
        add(L, m, c[0], BCR_PR, -1, -1, Pk(S, c[0]), 0, 0, 1, 2);
        continue;
      }
      for (int p = 0; p < len; p += 2) {
        const int k = c[p];
        const bool hl = p > 0, hr = p + 1 < len;
        const int nl = hl ? c[p - 1] : -1, nr = hr ? c[p + 1] : -1;
        if (b == 0)
          add(L, m, k, BCR_BWD0, nl, nr, Pk(S, k), 0, 0, 1, 2 + (int)hl + (int)hr);
        else
          add(L, m, k, BCR_BWD, nl, nr, Pk(S, k), hl ? B.wl[k] : 0, hr ? B.wr[k] : 0,
              1 + (int)hl + (int)hr, 2 + (int)hl + (int)hr);
      }
    }
    finish(L);
  }
}

// Block steps of the twisted block LDL^T chains, every chain of the launch
// group in one launch per step (B_k the stored inverse Schur blocks):
//   forward  w_k = B_k (r_k - c_{k-1} w_{k-1})  (top, k < m)
//            w_k = B_k (r_k - c_k w_{k+1})      (bottom, k > m)
//   middle   x_m = B_m (r_m - c_{m-1} w_{m-1} - c_m w_{m+1})
//   backward x_k = w_k - B_k (c_k x_{k+1})      (top)
//            x_k = w_k - B_k (c_{k-1} x_{k-1})  (bottom)
// w and x share the solution pool; a step reads only blocks a previous
// launch wrote.
void chain_step_jobs(const dsd_plan* pl, const std::vector<int2>& mem, std::vector<BcrJob>& jobs,
                     std::vector<BcrLaunch>& out) {
  const double ts = (double)tsize(pl);
  int T = 0;
  for (const int2& m : mem) {
    const SubDesc& S = pl->subs[m.x];
    T = std::max(T, std::max(S.mid, S.nblk - 1 - S.mid));
  }
  auto begin = [&]() {
    return BcrLaunch{(int)jobs.size(), 0, 0, 1, pl->chain_cg, pl->chain_rt, 0, 0.0, 0.0};
  };
  auto finish = [&](BcrLaunch& L) {
    L.n = (int)jobs.size() - L.off;
    if (L.n > 0) out.push_back(L);
  };
  auto add = [&](BcrLaunch& L, const int2& m, int blk, int mode, int nl, int nr) {
    const SubDesc& S = pl->subs[m.x];
    jobs.push_back(BcrJob{m.x, m.y, blk, mode, nl, nr, S.nb, 0,
                          S.fac_off + (long long)blk * S.nb * S.nb, 0, 0, S.nloc,
                          S.vec_off * pl->kmax, S.coef_off});
    const int nvec = 2 + (int)(nl >= 0) + (int)(nr >= 0) + (mode == BCR_CHB ? 1 : 0);
    L.fbytes += (double)S.nb * S.nb * ts;
    L.vcells += (double)nvec * S.nb;
  };
  for (int t = 0; t < T; ++t) {
    BcrLaunch L = begin();
    for (const int2& m : mem) {
      const SubDesc& S = pl->subs[m.x];
      if (t < S.mid) add(L, m, t, BCR_BWD0, t > 0 ? t - 1 : -1, -1);
      const int k = S.nblk - 1 - t;
      if (k > S.mid) add(L, m, k, BCR_BWD0, -1, k + 1 < S.nblk ? k + 1 : -1);
    }
    finish(L);
  }
  BcrLaunch Lm = begin();
  for (const int2& m : mem) {
    const SubDesc& S = pl->subs[m.x];
    add(Lm, m, S.mid, BCR_BWD0, S.mid > 0 ? S.mid - 1 : -1, S.mid + 1 < S.nblk ? S.mid + 1 : -1);
  }
  finish(Lm);
  for (int s = 1; s <= T; ++s) {
    BcrLaunch L = begin();
    for (const int2& m : mem) {
      const SubDesc& S = pl->subs[m.x];
      if (S.mid - s >= 0) add(L, m, S.mid - s, BCR_CHB, -1, S.mid - s + 1);
      if (S.mid + s < S.nblk) add(L, m, S.mid + s, BCR_CHB, S.mid + s - 1, -1);
    }
    finish(L);
  }
}

// Host check of a solve-job table against the factor and the subdomain grids.
int bcr_check_jobs(const dsd_plan* pl, const std::vector<BcrJob>& jobs, bool local) {
  for (const BcrJob& J : jobs) {
    bool ok = J.sub >= 0 && J.sub < pl->S && J.l >= 0 && J.l < pl->L;
    if (ok) {
      const SubDesc& S = pl->subs[J.sub];
      const long long nb2 = (long long)S.nb * S.nb;
      if (J.nb != S.nb || J.nloc != S.nloc || J.vbase != (local ? 0 : S.vec_off * pl->kmax) ||
          J.cbase != S.coef_off)
        ok = false;
      auto blk_ok = [&](int b) { return b >= 0 && b < S.nblk; };
      auto mat_ok = [&](long long o) { return o >= 0 && o + nb2 <= pl->sum_fac; };
      ok = ok && blk_ok(J.blk) && (J.nl == -1 || blk_ok(J.nl)) && (J.nr == -1 || blk_ok(J.nr));
      const bool hl = J.nl >= 0, hr = J.nr >= 0;
      switch (J.mode) {
        case BCR_PR: ok = ok && mat_ok(J.m0); break;
        case BCR_KEPT: ok = ok && hl && mat_ok(J.m0) && (!hr || mat_ok(J.m1)); break;
        case BCR_BWD0:
        case BCR_DFWD:
          ok = ok && (!hl || J.blk >= 1) && (!hr || J.blk + 1 < S.nblk) &&
               (J.mode == BCR_DFWD || mat_ok(J.m0));
          break;
        case BCR_BWD: ok = ok && mat_ok(J.m0) && (!hl || mat_ok(J.m1)) && (!hr || mat_ok(J.m2)); break;
        case BCR_CHB:
          ok = ok && mat_ok(J.m0) && (hl != hr) && (!hl || J.blk >= 1) && (!hr || J.blk + 1 < S.nblk);
          break;
        case BCR_DENSE: {
          // blocks nl + q nr, q < pad, of one reduction level; matrix nb x (pad nb)
          const int m = J.pad;
          ok = ok && m >= 2 && hl && J.nr >= 1 && (long long)J.nl + (long long)(m - 1) * J.nr < S.nblk &&
               (J.blk - J.nl) % J.nr == 0 && J.blk >= J.nl && (J.blk - J.nl) / J.nr < m &&
               J.m0 >= 0 && J.m0 + (long long)m * nb2 <= pl->sum_fac;
          break;
        }
        default: ok = false;
      }
    }
    if (!ok) {
      g_detail = "internal error: cyclic-reduction solve job out of range";
      return DSD_EINVAL;
    }
  }
  return 0;
}

int device_lds();

// ------------------------------------------- nested dissection (local solver 4)
// Whether a node's forward (rows = boundary) or backward (rows = separator)
// product runs in wide mode: a front of at least nd_wide cells, or more rows
// than the LDS-front kernels cover (eight 64-row tiles).
bool nd_wide_node(const dsd_plan* pl, int ns, int nbd, bool fwd) {
  return ns + nbd >= pl->nd_wide || (fwd ? nbd : ns) > 512;
}

// Analysis of every distinct local grid shape, the factor layout (per
// subdomain: the nodes' L and K blocks, then P_top) and the device tables.
int nd_setup(dsd_plan* pl) {
  const dsd_params& q = pl->prm;
  const int leaf = q.nd_leaf > 0 ? q.nd_leaf : 128;
  const int ntop_max = q.nd_top_cells > 0 ? q.nd_top_cells : 1200;
  std::map<std::tuple<int, int, int>, int> shape_id;
  pl->nd_shapes.clear();
  pl->nd_shape_of.assign(pl->S, 0);
  for (int s = 0; s < pl->S; ++s) {
    const SubDesc& S = pl->subs[s];
    const auto key = std::make_tuple(S.dims[0], S.dims[1], S.dims[2]);
    auto it = shape_id.find(key);
    if (it == shape_id.end()) {
      it = shape_id.emplace(key, (int)pl->nd_shapes.size()).first;
      pl->nd_shapes.push_back(nd_analyse(pl->dim, S.dims, leaf, ntop_max));
    }
    pl->nd_shape_of[s] = it->second;
  }
  std::vector<NdNodeDev> nodes;
  std::vector<int> cells, maps, umaps, src, usrc, lev, levmax, levnodes;
  pl->nd_tabs.assign(pl->nd_shapes.size(), NdShapeTab{});
  pl->nd_max_nf = pl->nd_max_ntop = pl->nd_max_nf_narrow = 0;
  pl->nd_lvmax.clear();
  pl->nd_wide = q.nd_wide > 0 ? q.nd_wide : 1024;
  pl->nd_small = q.nd_wave_steps > 0 ? q.nd_wave_steps : 4;
  // fusion level: the shallowest subtree level from which every node below
  // (in every shape) has a front of at most nd_fuse cells
  {
    const int fuse_nf = std::min(ND_FUSE_CAP, q.nd_fuse > 0 ? q.nd_fuse : 128);
    std::vector<int> mx;
    for (const NdShape& sh : pl->nd_shapes)
      for (const NdNode& n : sh.nodes) {
        if (n.top) continue;
        if ((int)mx.size() <= n.level) mx.resize(n.level + 1, 0);
        mx[n.level] = std::max(mx[n.level], (int)(n.sep.size() + n.bnd.size()));
      }
    pl->nd_fuse_level = 1 << 30;
    for (int l = (int)mx.size() - 1; l >= 0 && mx[l] <= fuse_nf; --l) pl->nd_fuse_level = l;
  }
  for (size_t k = 0; k < pl->nd_shapes.size(); ++k) {
    const NdShape& sh = pl->nd_shapes[k];
    if (!nd_append_tables(sh, pl->nd_tabs[k], nodes, cells, maps, umaps, src, usrc, lev,
                          levmax, levnodes)) {
      g_detail = "internal error: nested-dissection tables inconsistent";
      return DSD_EINVAL;
    }
    pl->nd_max_nf = std::max(pl->nd_max_nf, sh.max_nf);
    for (const NdNode& n : sh.nodes) {
      if (n.top) continue;
      const int ns = (int)n.sep.size(), nbd = (int)n.bnd.size(), nf = ns + nbd;
      if (nf < pl->nd_wide) pl->nd_max_nf_narrow = std::max(pl->nd_max_nf_narrow, nf);
      if (n.level >= pl->nd_fuse_level) continue;
      if ((int)pl->nd_lvmax.size() <= n.level) pl->nd_lvmax.resize(n.level + 1);
      dsd_plan::NdLevelMax& M = pl->nd_lvmax[n.level];
      if (!nd_wide_node(pl, ns, nbd, true)) {
        M.f_rows = std::max(M.f_rows, nbd);
        M.f_cols = std::max(M.f_cols, ns);
        M.f_nf = std::max(M.f_nf, nf);
      }
      if (!nd_wide_node(pl, ns, nbd, false)) {
        // a leaf's backward product runs over its separator only
        const bool leaf = n.child[0] < 0 && n.child[1] < 0;
        M.b_rows = std::max(M.b_rows, ns);
        M.b_cols = std::max(M.b_cols, leaf ? ns : nf);
      }
    }
    pl->nd_max_ntop = std::max(pl->nd_max_ntop, sh.ntop());
  }
  // the inversions run the split Gauss-Jordan form, whose panel kernel keeps
  // one column of the matrix in LDS
  int max_inv = pl->nd_max_ntop;
  for (const NdShape& sh : pl->nd_shapes) max_inv = std::max(max_inv, sh.max_ns);
  if ((size_t)(max_inv + 32) * sizeof(cpx<double>) > (size_t)device_lds()) {
    g_detail = "nested dissection: a separator or dense top of " + std::to_string(max_inv) +
               " cells exceeds the inversion kernel's LDS (lower nd_top_cells or use more "
               "subdomains)";
    return DSD_EINVAL;
  }
  long long foff = 0;
  for (int s = 0; s < pl->S; ++s) {
    pl->subs[s].fac_off = foff;
    foff += pl->nd_shapes[pl->nd_shape_of[s]].fac_entries;
  }
  pl->sum_fac = foff;
  pl->nd_cell_of.resize(nodes.size());
  pl->nd_map_of.resize(nodes.size());
  for (size_t i = 0; i < nodes.size(); ++i) {
    pl->nd_cell_of[i] = nodes[i].cell;
    pl->nd_map_of[i] = nodes[i].map;
  }
  CHK(upload(pl->d_nd_nodes, nodes));
  CHK(upload(pl->d_nd_cells, cells));
  CHK(upload(pl->d_nd_maps, maps));
  CHK(upload(pl->d_nd_umaps, umaps));
  CHK(upload(pl->d_nd_src, src));
  CHK(upload(pl->d_nd_usrc, usrc));
  CHK(upload(pl->d_nd_lev, lev));
  CHK(upload(pl->d_nd_levmax, levmax));
  CHK(upload(pl->d_nd_levnodes, levnodes));
  return 0;
}

// Solve jobs of a set of members {subdomain, sweep slot}: every node of every
// member's subtrees, grouped by level (depth below its subtree root), and
// every member's dense top.  Update vectors of member i start at the sum of
// the earlier members' (entries x kmax).  With `local` the vectors are
// addressed from offset 0 (vbase = 0) and kmax is the call's right-hand-side
// count (passed at launch), so ubase is in entries per RHS.
void nd_group_jobs(const dsd_plan* pl, const std::vector<int2>& mem, bool local,
                   std::vector<NdLvlJob>& lj, std::vector<NdTopJob>& tj, std::vector<int2>& wt,
                   std::vector<int2>& fj, std::vector<int2>& fb, dsd_plan::NdLaunch& L) {
  const double ts = (double)tsize(pl);
  L = dsd_plan::NdLaunch{};
  L.top_off = (int)tj.size();
  L.fj_off = (int)fj.size();
  int nlev = 0;
  for (const int2& m : mem) nlev = std::max(nlev, pl->nd_shapes[pl->nd_shape_of[m.x]].nlev);
  nlev = std::min(nlev, pl->nd_fuse_level);
  std::vector<std::vector<NdLvlJob>> per(nlev);
  std::vector<NdTopJob> tops;
  L.levels.assign(nlev, dsd_plan::NdLevel{});
  long long ubase = 0;
  for (const int2& m : mem) {
    const SubDesc& S = pl->subs[m.x];
    const int k = pl->nd_shape_of[m.x];
    const NdShape& sh = pl->nd_shapes[k];
    const NdShapeTab& tb = pl->nd_tabs[k];
    const long long vb = local ? 0 : S.vec_off * pl->kmax;
    const long long ub = local ? ubase : ubase * pl->kmax;
    auto job_of = [&](size_t i) {
      const NdNode& n = sh.nodes[i];
      NdLvlJob J{};
      J.ns = (int)n.sep.size();
      J.nbd = (int)n.bnd.size();
      J.cell = pl->nd_cell_of[tb.node0 + i];
      J.umap = pl->nd_map_of[tb.node0 + i];
      J.l = m.y;
      J.nloc = S.nloc;
      J.fac = S.fac_off + n.fac;
      J.upd = n.upd;
      J.vbase = vb;
      J.ubase = ub;
      J.leaf = n.child[0] < 0 && n.child[1] < 0;
      for (int a = 0; a < 3; ++a) {
        J.lo[a] = n.lo[a];
        J.hi[a] = n.hi[a];
        J.dims[a] = S.dims[a];
      }
      J.coef = S.coef_off;
      return J;
    };
    // fused subtrees: the nodes below the fusion level, by their ancestor at
    // it; per ancestor, level by level from the deepest, in batches whose
    // fronts fit ND_FUSE_CAP positions
    std::map<int, std::vector<std::vector<int>>> fuse;   // ancestor -> nodes per level
    for (size_t i = 0; i < sh.nodes.size(); ++i) {
      const NdNode& n = sh.nodes[i];
      if (n.top || n.level < pl->nd_fuse_level) continue;
      int a = (int)i;
      while (sh.nodes[a].level > pl->nd_fuse_level) a = sh.nodes[a].parent;
      std::vector<std::vector<int>>& lv = fuse[a];
      const int d = n.level - pl->nd_fuse_level;
      if ((int)lv.size() <= d) lv.resize(d + 1);
      lv[d].push_back((int)i);
    }
    for (auto& kv : fuse) {
      const int b0 = (int)fb.size();
      for (int d = (int)kv.second.size() - 1; d >= 0; --d) {
        int used = ND_FUSE_CAP;
        for (int i : kv.second[d]) {
          NdLvlJob J = job_of((size_t)i);
          const int nf = J.ns + J.nbd;
          if (used + nf > ND_FUSE_CAP) {
            fb.push_back(make_int2((int)lj.size(), 0));
            used = 0;
          }
          J.pad = used;
          used += nf;
          lj.push_back(J);
          ++fb.back().y;
          L.fu_fbytes += (double)J.nbd * J.ns * ts;
          L.fu_bbytes += (double)J.ns * nf * ts;
          L.fu_cells += (double)nf;
        }
      }
      fj.push_back(make_int2(b0, (int)fb.size() - b0));
    }
    for (size_t i = 0; i < sh.nodes.size(); ++i) {
      const NdNode& n = sh.nodes[i];
      if (n.top || n.level >= pl->nd_fuse_level) continue;
      per[n.level].push_back(job_of(i));
    }
    if (sh.ntop() > 0) {
      NdTopJob T{};
      T.ntop = sh.ntop();
      T.dim2 = 2 * pl->dim;
      T.cell = tb.top_cell;
      T.usrc = tb.top_usrc;
      T.nloc = S.nloc;
      T.fac = S.fac_off + sh.top_fac;
      T.vbase = vb;
      T.ubase = ub;
      T.l = m.y;
      tops.push_back(T);
    }
    ubase += sh.upd_entries;
  }
  // Per level: jobs ordered wide both ways, wide backward only, narrow, wide
  // forward only (each class by decreasing front), so that the narrow forward
  // and the narrow backward products are contiguous ranges.
  auto cat = [&](const NdLvlJob& J) {
    const bool wf = nd_wide_node(pl, J.ns, J.nbd, true), wb = nd_wide_node(pl, J.ns, J.nbd, false);
    return wf && wb ? 0 : wb ? 1 : !wf ? 2 : 3;
  };
  for (int l = 0; l < nlev; ++l) {
    std::vector<NdLvlJob>& v = per[l];
    std::stable_sort(v.begin(), v.end(), [&](const NdLvlJob& a, const NdLvlJob& b) {
      const int ca = cat(a), cb = cat(b);
      if (ca != cb) return ca < cb;
      return a.ns + a.nbd > b.ns + b.nbd;
    });
    dsd_plan::NdLevel& V = L.levels[l];
    V.off = (int)lj.size();
    V.n = (int)v.size();
    int c[5] = {0, 0, 0, 0, 0};
    for (const NdLvlJob& J : v) ++c[cat(J) + 1];
    for (int k = 1; k < 5; ++k) c[k] += c[k - 1];
    V.nf_off = V.off + c[1];
    V.nf_n = c[3] - c[1];
    V.nb_off = V.off + c[2];
    V.nb_n = c[4] - c[2];
    // wide-mode tiles: 256 separator positions (forming f_S), ND_WROWS rows
    auto add_tiles = [&](bool fwd, bool form, int& off, int& cnt) {
      off = (int)wt.size();
      for (size_t j = 0; j < v.size(); ++j) {
        const NdLvlJob& J = v[j];
        if (!nd_wide_node(pl, J.ns, J.nbd, fwd)) continue;
        const int rows = form ? J.ns : fwd ? J.nbd : J.ns;
        const int step = form ? 256 : ND_WROWS;
        for (int r0 = 0; r0 < rows; r0 += step) wt.push_back(make_int2(V.off + (int)j, r0));
      }
      cnt = (int)wt.size() - off;
    };
    add_tiles(true, true, V.fm_off, V.fm_n);
    add_tiles(true, false, V.wf_off, V.wf_n);
    add_tiles(false, false, V.wb_off, V.wb_n);
    for (const NdLvlJob& J : v) {
      const bool wb = nd_wide_node(pl, J.ns, J.nbd, false);
      const double fb = (double)J.nbd * J.ns * ts,
                   bb = (double)J.ns * (J.leaf && !wb ? J.ns : J.ns + J.nbd) * ts;
      const double fc = (double)(J.ns + J.nbd);
      if (nd_wide_node(pl, J.ns, J.nbd, true)) { V.wf_bytes += fb; V.wf_cells += fc; }
      else { V.nf_bytes += fb; V.nf_cells += fc; }
      if (wb) { V.wb_bytes += bb; V.wb_cells += fc; }
      else { V.nb_bytes += bb; V.nb_cells += fc; }
    }
    lj.insert(lj.end(), v.begin(), v.end());
  }
  for (const NdTopJob& T : tops) {
    L.top_bytes += (double)T.ntop * T.ntop * ts;
    L.top_cells += (double)T.ntop;
  }
  tj.insert(tj.end(), tops.begin(), tops.end());
  L.fj_n = (int)fj.size() - L.fj_off;
  L.ntop = (int)tops.size();
  L.upd = ubase;
}

// Job tables of every launch group and of every subdomain's local solve.
int build_nd_jobs(dsd_plan* pl) {
  std::vector<NdLvlJob> sj;
  std::vector<NdTopJob> tj;
  std::vector<int2> wt, fj, fb;
  pl->nd_launch.assign(pl->groups.size(), dsd_plan::NdLaunch{});
  pl->nd_upd_max = 0;
  for (size_t g = 0; g < pl->groups.size(); ++g) {
    nd_group_jobs(pl, pl->groups[g], false, sj, tj, wt, fj, fb, pl->nd_launch[g]);
    pl->nd_upd_max = std::max(pl->nd_upd_max, pl->nd_launch[g].upd);
  }
  pl->nd_local.assign(pl->S, dsd_plan::NdLaunch{});
  for (int s = 0; s < pl->S; ++s) {
    nd_group_jobs(pl, std::vector<int2>{make_int2(s, 0)}, true, sj, tj, wt, fj, fb, pl->nd_local[s]);
    pl->nd_upd_max = std::max(pl->nd_upd_max, pl->nd_local[s].upd);
  }
  CHK(upload(pl->d_nd_lvl, sj));
  CHK(upload(pl->d_nd_top, tj));
  if (wt.empty()) wt.push_back(make_int2(0, 0));
  CHK(upload(pl->d_nd_wide, wt));
  if (fj.empty()) fj.push_back(make_int2(0, 0));
  if (fb.empty()) fb.push_back(make_int2(0, 0));
  CHK(upload(pl->d_nd_fj, fj));
  CHK(upload(pl->d_nd_fb, fb));
  return 0;
}

// Factorisation, bottom-up by depth over all subdomains of a chunk (FP64
// fronts): assemble every front (original couplings of its separator plus the
// children's update matrices), invert F_SS (Gauss-Jordan, partial pivoting),
// L = F_BS P and the update F_BB -= L F_SB, and round L and K = [P | L^T] into
// the factors; then assemble the dense top from the subtree roots' updates,
// invert it and round it into the factors.
int nd_factor(dsd_plan* pl) {
  hipStream_t st = pl->stream;
  CHK(pl->d_fac.alloc((size_t)pl->sum_fac * tsize(pl)));
  const cpx<double>* cf[4] = {pl->d_lcoef64[0].as<cpx<double>>(), pl->d_lcoef64[1].as<cpx<double>>(),
                              pl->d_lcoef64[2].as<cpx<double>>(), pl->d_lcoef64[3].as<cpx<double>>()};
  // FP64 work per subdomain.  A depth's fronts are assembled from the next
  // depth's and are dead once their parents are, so the fronts of even and of
  // odd depths share two regions; then the top matrix and the largest depth's
  // S (ns x ns) and L (nbd x ns) blocks.
  int maxdepth = 0;
  for (const NdShape& sh : pl->nd_shapes)
    for (const NdNode& n : sh.nodes) maxdepth = std::max(maxdepth, n.depth);
  auto depth_entries = [&](int s, std::vector<long long>& e, std::vector<long long>& sl) {
    e.assign(maxdepth + 2, 0);
    sl.assign(maxdepth + 2, 0);
    for (const NdNode& n : pl->nd_shapes[pl->nd_shape_of[s]].nodes) {
      if (n.top) continue;
      const long long ns = (long long)n.sep.size(), nf = ns + (long long)n.bnd.size();
      e[n.depth] += nf * nf;
      sl[n.depth] += ns * nf;
    }
  };
  std::vector<long long> fneed(pl->S, 0);
  {
    std::vector<long long> e, sl;
    for (int s = 0; s < pl->S; ++s) {
      depth_entries(s, e, sl);
      long long m2 = 0, ms = 0;
      for (int d = 0; d <= maxdepth; ++d) {
        m2 = std::max(m2, e[d] + e[d + 1]);
        ms = std::max(ms, sl[d]);
      }
      const long long nt = pl->nd_shapes[pl->nd_shape_of[s]].ntop();
      fneed[s] = m2 + nt * nt + ms;
    }
  }
  size_t fr = 0, tot = 0;
  HIPCHK(hipMemGetInfo(&fr, &tot));
  const double budget = 0.4 * (double)fr / sizeof(cpx<double>);
  int s0 = 0;
  while (s0 < pl->S) {
    // chunk [s0, s1)
    int s1 = s0;
    double need = 0;
    while (s1 < pl->S && s1 - s0 < 255 && (s1 == s0 || need + (double)fneed[s1] < budget)) {
      need += (double)fneed[s1];
      ++s1;
    }
    // front offsets: depth d in region d % 2
    std::vector<long long> E(maxdepth + 2, 0), SL(maxdepth + 2, 0);
    {
      std::vector<long long> e, sl;
      for (int s = s0; s < s1; ++s) {
        depth_entries(s, e, sl);
        for (int d = 0; d <= maxdepth; ++d) {
          E[d] += e[d];
          SL[d] += sl[d];
        }
      }
    }
    long long half[2] = {0, 0}, lvl_max = 0;
    for (int d = 0; d <= maxdepth; ++d) {
      half[d & 1] = std::max(half[d & 1], E[d]);
      lvl_max = std::max(lvl_max, SL[d]);
    }
    std::vector<long long> cur(maxdepth + 1);
    for (int d = 0; d <= maxdepth; ++d) cur[d] = (d & 1) ? half[0] : 0;
    std::vector<long long> fo;          // per (sub in chunk, node of its shape); -1 for top nodes
    std::vector<int> fo_base(s1 - s0);
    std::vector<long long> toff(s1 - s0);
    for (int s = s0; s < s1; ++s) {
      const NdShape& sh = pl->nd_shapes[pl->nd_shape_of[s]];
      fo_base[s - s0] = (int)fo.size();
      for (const NdNode& n : sh.nodes) {
        if (n.top) {
          fo.push_back(-1);
          continue;
        }
        fo.push_back(cur[n.depth]);
        cur[n.depth] += (long long)(n.sep.size() + n.bnd.size()) * (n.sep.size() + n.bnd.size());
      }
    }
    long long w = half[0] + half[1];
    for (int s = s0; s < s1; ++s) {
      const NdShape& sh = pl->nd_shapes[pl->nd_shape_of[s]];
      toff[s - s0] = w;
      w += (long long)sh.ntop() * sh.ntop();
    }
    const long long sl_base = w;
    w += lvl_max;
    Buf work, dfo, derr, dpiv, drbuf, dj1, dj2, dj3, dj4;
    CHK(work.alloc((size_t)w * sizeof(cpx<double>)));
    CHK(upload(dfo, fo));
    cpx<double>* W = work.as<cpx<double>>();
    const NdNodeDev* dn = pl->d_nd_nodes.as<NdNodeDev>();
    for (int d = maxdepth; d >= 0; --d) {
      std::vector<NdFrontJob> fj;
      std::vector<NdCopyJob> cj, sj;
      std::vector<BcrInvJob> ij;
      std::vector<NdGemmJob> g1, g2;
      int max_nf = 0, max_ns = 0, max_nbd = 0;
      long long so = sl_base;
      for (int s = s0; s < s1; ++s) {
        const int k = pl->nd_shape_of[s];
        const NdShape& sh = pl->nd_shapes[k];
        const SubDesc& S = pl->subs[s];
        for (size_t i = 0; i < sh.nodes.size(); ++i) {
          const NdNode& n = sh.nodes[i];
          if (n.top || n.depth != d) continue;
          const int ns = (int)n.sep.size(), nbd = (int)n.bnd.size(), nf = ns + nbd;
          max_nf = std::max(max_nf, nf);
          max_ns = std::max(max_ns, ns);
          max_nbd = std::max(max_nbd, nbd);
          const long long F = fo[fo_base[s - s0] + i];
          NdFrontJob J{};
          J.node = pl->nd_tabs[k].node0 + (int)i;
          for (int a = 0; a < 3; ++a) J.dims[a] = S.dims[a];
          J.coef = S.coef_off;
          J.F = F;
          J.F0 = n.child[0] >= 0 ? fo[fo_base[s - s0] + n.child[0]] : -1;
          J.F1 = n.child[1] >= 0 ? fo[fo_base[s - s0] + n.child[1]] : -1;
          fj.push_back(J);
          const long long Sb = so, Lb = so + (long long)ns * ns;
          so += (long long)ns * nf;
          cj.push_back(NdCopyJob{ns, ns, nf, ns, 0, 0, F, Sb});
          ij.push_back(BcrInvJob{ns, s, Sb, -1});
          g1.push_back(NdGemmJob{nbd, ns, ns, nf, ns, nbd, 0, 0, 1.0, F + ns, Sb, Lb});
          g2.push_back(NdGemmJob{nbd, nbd, ns, nbd, nf, nf, 1, 0, -1.0, Lb,
                                 F + (long long)ns * nf, F + ns + (long long)ns * nf});
          const long long fb = S.fac_off + n.fac;
          sj.push_back(NdCopyJob{nbd, ns, nbd, nbd, 0, 1, Lb, fb});
          sj.push_back(NdCopyJob{ns, ns, ns, ns, 0, 1, Sb, fb + (long long)nbd * ns});
          sj.push_back(NdCopyJob{ns, nbd, nbd, ns, 1, 1, Lb, fb + (long long)nbd * ns + (long long)ns * ns});
        }
      }
      if (fj.empty()) continue;
      const int nj = (int)fj.size();
      CHK(upload(dj1, fj));
      launch_nd_front(dj1.as<NdFrontJob>(), nj, max_nf, dn, pl->d_nd_cells.as<int>(),
                      pl->d_nd_maps.as<int>(), cf[0], cf[1], cf[2], cf[3], W, st);
      CHK(upload(dj2, cj));
      if (pl->c64) launch_nd_copy<float>(dj2.as<NdCopyJob>(), nj, max_ns, max_ns, W, pl->d_fac.as<cpx<float>>(), st);
      else launch_nd_copy<double>(dj2.as<NdCopyJob>(), nj, max_ns, max_ns, W, pl->d_fac.as<cpx<double>>(), st);
      CHK(upload(dj3, ij));
      CHK(derr.alloc((size_t)nj * sizeof(int)));
      HIPCHK(hipMemsetAsync(derr.p, 0, (size_t)nj * sizeof(int), st));
      Buf dpst;
      CHK(piv_begin(dpst, (size_t)nj));
      // inversions in launches of at most 255 (the split form serves large orders)
      const int step = 255;
      CHK(dpiv.alloc((size_t)std::min(nj, step) * max_ns * sizeof(int)));
      CHK(drbuf.alloc((size_t)std::min(nj, step) * gj_rbuf_entries(max_ns) * sizeof(cpx<double>)));
      for (int j0 = 0; j0 < nj; j0 += step) {
        const int n = std::min(step, nj - j0);
        if (pl->c64)
          launch_bcr_invert<float>(dj3.as<BcrInvJob>() + j0, n, max_ns, W, pl->d_fac.as<cpx<float>>(),
                                   derr.as<int>() + j0, dpiv.as<int>(), drbuf.as<cpx<double>>(),
                                   dpst.as<double>() + 2 * j0, st);
        else
          launch_bcr_invert<double>(dj3.as<BcrInvJob>() + j0, n, max_ns, W, pl->d_fac.as<cpx<double>>(),
                                    derr.as<int>() + j0, dpiv.as<int>(), drbuf.as<cpx<double>>(),
                                    dpst.as<double>() + 2 * j0, st);
      }
      HIPCHK(hipGetLastError());
      CHK(upload(dj4, g1));
      launch_nd_gemm(dj4.as<NdGemmJob>(), nj, max_nbd, max_ns, W, st);
      Buf dg2;
      CHK(upload(dg2, g2));
      launch_nd_gemm(dg2.as<NdGemmJob>(), nj, max_nbd, max_nbd, W, st);
      Buf ds;
      CHK(upload(ds, sj));
      const int mr = std::max(max_nbd, max_ns), mc = std::max(max_nbd, max_ns);
      if (pl->c64) launch_nd_copy<float>(ds.as<NdCopyJob>(), (int)sj.size(), mr, mc, W, pl->d_fac.as<cpx<float>>(), st);
      else launch_nd_copy<double>(ds.as<NdCopyJob>(), (int)sj.size(), mr, mc, W, pl->d_fac.as<cpx<double>>(), st);
      HIPCHK(hipGetLastError());
      std::vector<int> herr(nj);
      HIPCHK(hipMemcpyAsync(herr.data(), derr.p, nj * sizeof(int), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      for (int j = 0; j < nj; ++j)
        if (herr[j]) {
          g_detail = "singular separator block in a nested-dissection front (depth " +
                     std::to_string(d) + ", subdomain " + std::to_string(ij[j].sub) + ")";
          return DSD_EPIVOT;
        }
      {
        std::vector<int> js(nj);
        for (int j = 0; j < nj; ++j) js[j] = ij[j].sub;
        CHK(piv_end(pl, dpst, js));
      }
    }
    // dense tops of the chunk
    std::vector<NdTopAsmJob> tj;
    std::vector<BcrInvJob> ti;
    std::vector<NdCopyJob> tc;
    int max_top = 0;
    for (int s = s0; s < s1; ++s) {
      const int k = pl->nd_shape_of[s];
      const NdShape& sh = pl->nd_shapes[k];
      const int nt = sh.ntop();
      if (nt == 0) continue;
      const SubDesc& S = pl->subs[s];
      NdTopAsmJob J{};
      J.ntop = nt;
      J.dim2 = 2 * pl->dim;
      J.cell = pl->nd_tabs[k].top_cell;
      J.src = pl->nd_tabs[k].top_src;
      for (int a = 0; a < 3; ++a) J.dims[a] = S.dims[a];
      J.fo = fo_base[s - s0];
      J.node0 = pl->nd_tabs[k].node0;
      J.coef = S.coef_off;
      J.T = toff[s - s0];
      tj.push_back(J);
      ti.push_back(BcrInvJob{nt, s, toff[s - s0], -1});
      tc.push_back(NdCopyJob{nt, nt, nt, nt, 0, 1, toff[s - s0], S.fac_off + sh.top_fac});
      max_top = std::max(max_top, nt);
    }
    if (!tj.empty()) {
      const int nj = (int)tj.size();
      CHK(upload(dj1, tj));
      launch_nd_top_asm(dj1.as<NdTopAsmJob>(), nj, max_top, dn, pl->d_nd_cells.as<int>(),
                        pl->d_nd_src.as<int>(), dfo.as<long long>(), cf[0], cf[1], cf[2], cf[3], W,
                        st);
      CHK(upload(dj3, ti));
      CHK(derr.alloc((size_t)nj * sizeof(int)));
      HIPCHK(hipMemsetAsync(derr.p, 0, (size_t)nj * sizeof(int), st));
      Buf dpst;
      CHK(piv_begin(dpst, (size_t)nj));
      CHK(dpiv.alloc((size_t)nj * max_top * sizeof(int)));
      CHK(drbuf.alloc((size_t)nj * gj_rbuf_entries(max_top) * sizeof(cpx<double>)));
      if (pl->c64)
        launch_bcr_invert<float>(dj3.as<BcrInvJob>(), nj, max_top, W, pl->d_fac.as<cpx<float>>(),
                                 derr.as<int>(), dpiv.as<int>(), drbuf.as<cpx<double>>(),
                                 dpst.as<double>(), st);
      else
        launch_bcr_invert<double>(dj3.as<BcrInvJob>(), nj, max_top, W, pl->d_fac.as<cpx<double>>(),
                                  derr.as<int>(), dpiv.as<int>(), drbuf.as<cpx<double>>(),
                                  dpst.as<double>(), st);
      CHK(upload(dj2, tc));
      if (pl->c64) launch_nd_copy<float>(dj2.as<NdCopyJob>(), nj, max_top, max_top, W, pl->d_fac.as<cpx<float>>(), st);
      else launch_nd_copy<double>(dj2.as<NdCopyJob>(), nj, max_top, max_top, W, pl->d_fac.as<cpx<double>>(), st);
      HIPCHK(hipGetLastError());
      std::vector<int> herr(nj);
      HIPCHK(hipMemcpyAsync(herr.data(), derr.p, nj * sizeof(int), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      for (int j = 0; j < nj; ++j)
        if (herr[j]) {
          g_detail = "singular dense top in a nested-dissection factorisation (subdomain " +
                     std::to_string(ti[j].sub) + ")";
          return DSD_EPIVOT;
        }
      {
        std::vector<int> js(nj);
        for (int j = 0; j < nj; ++j) js[j] = ti[j].sub;
        CHK(piv_end(pl, dpst, js));
      }
    }
    HIPCHK(hipStreamSynchronize(st));
    s0 = s1;
  }
  return 0;
}

int assemble_and_factor(dsd_plan* pl, const double* m_dev) {
  hipStream_t st = pl->stream;
  const Problem& P = pl->P;
  long long nphys = (long long)P.n[0] * P.n[1] * P.n[2];
  CHK(pl->d_m.alloc(nphys * sizeof(double)));
  HIPCHK(hipMemcpyAsync(pl->d_m.p, m_dev, nphys * sizeof(double), hipMemcpyDeviceToDevice, st));
  // grids: 0 = global, 1.. = subdomains
  std::vector<AxisGrid> grids;
  std::vector<long long> offs;
  for (int a = 0; a < 3; ++a) {
    if (a < pl->dim)
      grids.push_back(AxisGrid{0, P.ng[a], 0.0, P.n[a] * P.h, P.pml, P.n[a] + P.pml - 1});
    else
      grids.push_back(AxisGrid{0, 1, -1e300, 1e300, P.pml, P.pml});
  }
  offs.push_back(0);
  long long maxc = P.N;
  for (const SubDesc& S : pl->subs) {
    for (int a = 0; a < 3; ++a) grids.push_back(S.ax[a]);
    offs.push_back(S.coef_off);
    maxc = std::max(maxc, S.nloc);
  }
  Buf dg, doff;
  CHK(upload(dg, grids));
  CHK(upload(doff, offs));
  for (int i = 0; i < 4; ++i) {
    CHK(pl->d_gcoef[i].alloc(P.N * sizeof(cpx<double>)));
    CHK(pl->d_lcoef64[i].alloc(pl->sum_nloc * sizeof(cpx<double>)));
    CHK(pl->d_lcoefT[i].alloc(pl->sum_nloc * tsize(pl)));
  }
  // global grid
  launch_assemble(P, dg.as<AxisGrid>(), doff.as<long long>(), 1, P.N, pl->d_m.as<double>(),
                  pl->d_gcoef[0].as<cpx<double>>(), pl->d_gcoef[1].as<cpx<double>>(),
                  pl->d_gcoef[2].as<cpx<double>>(), pl->d_gcoef[3].as<cpx<double>>(), st);
  HIPCHK(hipGetLastError());
  // subdomain grids
  launch_assemble(P, dg.as<AxisGrid>() + 3, doff.as<long long>() + 1, pl->S, maxc,
                  pl->d_m.as<double>(), pl->d_lcoef64[0].as<cpx<double>>(),
                  pl->d_lcoef64[1].as<cpx<double>>(), pl->d_lcoef64[2].as<cpx<double>>(),
                  pl->d_lcoef64[3].as<cpx<double>>(), st);
  HIPCHK(hipGetLastError());
  for (int i = 0; i < 4; ++i) {
    if (pl->c64)
      launch_convert<float>(pl->d_lcoef64[i].as<cpx<double>>(), pl->d_lcoefT[i].as<cpx<float>>(),
                            pl->sum_nloc, st);
    else
      launch_convert<double>(pl->d_lcoef64[i].as<cpx<double>>(),
                             pl->d_lcoefT[i].as<cpx<double>>(), pl->sum_nloc, st);
  }
  HIPCHK(hipGetLastError());

  if (pl->solver == 4) return nd_factor(pl);
  if (pl->solver == 2) return bcr_factor(pl);
  // ---- factorisation: chains of Schur complements towards the middle block
  CHK(pl->d_fac.alloc((size_t)pl->sum_fac * tsize(pl)));
  const long long blk = (long long)pl->max_nb * pl->max_nb;
  Buf scratch, derr, dpiv, djobs;
  CHK(scratch.alloc((size_t)pl->S * 4 * blk * sizeof(cpx<double>)));
  auto slot = [&](int sid, int half, int parity) {
    return ((long long)sid * 4 + half * 2 + parity) * blk;
  };
  int maxlen = 0;
  for (const SubDesc& S : pl->subs) maxlen = std::max(maxlen, std::max(S.mid, S.nblk - 1 - S.mid));
  std::vector<FactorJob> all;
  std::vector<int> job_off(maxlen + 2, 0);
  for (int t = 0; t < maxlen; ++t) {
    job_off[t] = (int)all.size();
    for (int sid = 0; sid < pl->S; ++sid) {
      const SubDesc& S = pl->subs[sid];
      if (t < S.mid) {
        FactorJob J{};
        J.sub = sid;
        J.k = t;
        J.cp_blk = t > 0 ? t - 1 : -1;
        J.cq_blk = -1;
        J.prev = slot(sid, 0, (t + 1) & 1);
        J.prev2 = 0;
        J.cur = slot(sid, 0, t & 1);
        all.push_back(J);
      }
      if (t < S.nblk - 1 - S.mid) {
        FactorJob J{};
        J.sub = sid;
        J.k = S.nblk - 1 - t;
        J.cp_blk = t > 0 ? J.k : -1;
        J.cq_blk = -1;
        J.prev = slot(sid, 1, (t + 1) & 1);
        J.prev2 = 0;
        J.cur = slot(sid, 1, t & 1);
        all.push_back(J);
      }
    }
  }
  job_off[maxlen] = (int)all.size();
  for (int sid = 0; sid < pl->S; ++sid) {
    const SubDesc& S = pl->subs[sid];
    FactorJob J{};
    J.sub = sid;
    J.k = S.mid;
    J.cp_blk = S.mid > 0 ? S.mid - 1 : -1;
    J.prev = slot(sid, 0, (S.mid - 1) & 1);
    const int nbot = S.nblk - 1 - S.mid;
    J.cq_blk = nbot > 0 ? S.mid : -1;
    J.prev2 = slot(sid, 1, (nbot - 1) & 1);
    J.cur = slot(sid, 0, S.mid & 1);
    all.push_back(J);
  }
  job_off[maxlen + 1] = (int)all.size();
  CHK(upload(djobs, all));
  CHK(derr.alloc(all.size() * sizeof(int)));
  HIPCHK(hipMemsetAsync(derr.p, 0, all.size() * sizeof(int), st));
  Buf dpst;
  CHK(piv_begin(dpst, all.size()));
  int maxjobs = 0;
  for (int t = 0; t <= maxlen; ++t) maxjobs = std::max(maxjobs, job_off[t + 1] - job_off[t]);
  CHK(dpiv.alloc((size_t)maxjobs * pl->max_nb * sizeof(int)));
  Buf drbuf;
  CHK(drbuf.alloc((size_t)maxjobs * gj_rbuf_entries(pl->max_nb) * sizeof(cpx<double>)));
  for (int t = 0; t <= maxlen; ++t) {
    const int j0 = job_off[t], nj = job_off[t + 1] - j0;
    const FactorJob* jp = djobs.as<FactorJob>() + j0;
    launch_schur(P, pl->d_subs.as<SubDesc>(), jp, nj, pl->max_nb,
                 pl->d_lcoef64[0].as<cpx<double>>(), pl->d_lcoef64[1].as<cpx<double>>(),
                 pl->d_lcoef64[2].as<cpx<double>>(), pl->d_lcoef64[3].as<cpx<double>>(),
                 scratch.as<cpx<double>>(), st);
    if (pl->c64)
      launch_invert<float>(pl->d_subs.as<SubDesc>(), jp, nj, pl->max_nb,
                           scratch.as<cpx<double>>(), pl->d_fac.as<cpx<float>>(),
                           derr.as<int>() + j0, dpiv.as<int>(), drbuf.as<cpx<double>>(),
                           dpst.as<double>() + 2 * j0, st);
    else
      launch_invert<double>(pl->d_subs.as<SubDesc>(), jp, nj, pl->max_nb,
                            scratch.as<cpx<double>>(), pl->d_fac.as<cpx<double>>(),
                            derr.as<int>() + j0, dpiv.as<int>(), drbuf.as<cpx<double>>(),
                            dpst.as<double>() + 2 * j0, st);
    HIPCHK(hipGetLastError());
  }
  std::vector<int> herr(all.size());
  HIPCHK(hipMemcpyAsync(herr.data(), derr.p, all.size() * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int v : herr)
    if (v) {
      g_detail = "singular Schur block in subdomain " + std::to_string(v - 1);
      return DSD_EPIVOT;
    }
  std::vector<int> js(all.size());
  for (size_t k = 0; k < all.size(); ++k) js[k] = all[k].sub;
  return piv_end(pl, dpst, js);
}

int ensure_pools(dsd_plan* pl) {
  if (pl->d_rpool.p) return 0;
  CHK(pl->d_rpool.alloc((size_t)pl->L * pl->sum_nloc * pl->kmax * tsize(pl)));
  CHK(pl->d_vpool.alloc((size_t)pl->L * pl->sum_nloc * pl->kmax * tsize(pl)));
  if (pl->solver == 4) CHK(pl->d_upool.alloc((size_t)pl->nd_upd_max * pl->kmax * tsize(pl)));
  return 0;
}

// Solve-launch timing (timing mode only): mark the start, then the end with
// the launch's algorithmic bytes; flush reads the pairs after one wait.
void time_begin(dsd_plan* pl) {
  if (!pl->timing) return;
  while (pl->tev.size() < pl->tev_used + 2) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) { pl->timing = false; return; }
    pl->tev.push_back(e);
  }
  (void)hipEventRecord(pl->tev[pl->tev_used], pl->stream);
}
void time_end(dsd_plan* pl, double bytes, double flops) {
  if (!pl->timing) return;
  (void)hipEventRecord(pl->tev[pl->tev_used + 1], pl->stream);
  pl->tev_used += 2;
  pl->solve_launches += 1;
  pl->solve_bytes += bytes;
  pl->solve_flops += flops;
}
void time_flush(dsd_plan* pl) {
  if (pl->tev_used == 0) return;
  (void)hipEventSynchronize(pl->tev[pl->tev_used - 1]);
  for (size_t i = 0; i < pl->tev_used; i += 2) {
    float ms = 0;
    (void)hipEventElapsedTime(&ms, pl->tev[i], pl->tev[i + 1]);
    pl->t_solve_ms += ms;
  }
  pl->tev_used = 0;
}

int device_lds();

// Shape of a level launch (rows x cols: the level's largest matrix): one
// node per wave when its (row, RHS) passes times its columns are at most
// `small` x 64 and eight fronts fit the LDS (tt = 0); else one node per
// workgroup of tt 64-row tiles x cg column groups (about 24 columns or more
// per group, at most eight waves).
void nd_shape(int rows, int cols, int kg, int max_nf, size_t ts, int small, int& tt, int& cg) {
  const int rpp = 64 / std::max(1, kg);
  const int passes = (rows + rpp - 1) / rpp;
  if ((long long)passes * cols <= (long long)small * 64 &&
      (size_t)8 * max_nf * kg * ts <= (size_t)device_lds()) {
    tt = 0;
    cg = 1;
    return;
  }
  tt = std::max(1, std::min(8, (rows + 63) / 64));
  cg = std::max(1, std::min(8 / tt, (cols + 23) / 24));
  // the column groups' partial sums must fit next to the front
  while (cg > 1 && ((size_t)max_nf * kg + (size_t)(cg - 1) * tt * 64 * kg) * ts > (size_t)device_lds())
    --cg;
}

// The nested-dissection solves of one launch (a launch group's members or
// one subdomain): the forward levels from the deepest to the subtree roots,
// the dense tops, the backward levels.  Timed launches carry their factor
// bytes plus their vectors (the fronts read and the rows written per RHS) and
// 8 flops per factor entry and RHS.
template <typename T>
void nd_phase(dsd_plan* pl, const dsd_plan::NdLaunch& L, cpx<T>* R, cpx<T>* X, cpx<T>* U,
              long long pool_stride, int nrhs, int kmax, bool timed) {
  hipStream_t st = pl->stream;
  const NdLvlJob* lj = pl->d_nd_lvl.as<NdLvlJob>();
  const NdTopJob* tj = pl->d_nd_top.as<NdTopJob>() + L.top_off;
  const cpx<T>* fac = pl->d_fac.as<cpx<T>>();
  const size_t tsz = sizeof(cpx<T>);
  const double ts = (double)tsz;
  const int* cells = pl->d_nd_cells.as<int>();
  // One level, forward (rows = boundary, columns = separator) or backward
  // (rows = separator, columns = front): the wide nodes' tiles, then the
  // narrow nodes in one launch of the level's plan-wide shape.
  const int2* wt = pl->d_nd_wide.as<int2>();
  auto level = [&](int l, const dsd_plan::NdLevel& V, bool fwd) {
    if (fwd && V.fm_n > 0)
      launch_nd_form<T>(lj, wt + V.fm_off, V.fm_n, cells, pl->d_nd_umaps.as<int>(), R, U, pool_stride,
                        nrhs, kmax, st);
    const int wn = fwd ? V.wf_n : V.wb_n;
    if (wn > 0) {
      if (timed) time_begin(pl);
      if (fwd)
        launch_nd_wide_fwd<T>(lj, wt + V.wf_off, wn, cells, pl->d_nd_umaps.as<int>(), fac, R, U,
                              pool_stride, nrhs, kmax, st);
      else
        launch_nd_wide_bwd<T>(lj, wt + V.wb_off, wn, cells, fac, R, X, pool_stride, nrhs, st);
      const double b = fwd ? V.wf_bytes : V.wb_bytes, c = fwd ? V.wf_cells : V.wb_cells;
      if (timed) time_end(pl, b + 2.0 * c * nrhs * ts, b / ts * nrhs * 8.0);
    }
    const int n = fwd ? V.nf_n : V.nb_n;
    if (n == 0) return;
    const dsd_plan::NdLevelMax& M = pl->nd_lvmax[l];
    int tt, cg;
    if (timed) time_begin(pl);
    if (fwd) {
      nd_shape(M.f_rows, M.f_cols, pl->kg, M.f_nf, tsz, pl->nd_small, tt, cg);
      launch_nd_lvl_fwd<T>(pl->kg, tt, cg, lj + V.nf_off, n, cells, pl->d_nd_umaps.as<int>(), fac, R,
                           U, pool_stride, nrhs, kmax, M.f_nf, st);
    } else {
      nd_shape(M.b_rows, M.b_cols, pl->kg, M.b_cols, tsz, pl->nd_small, tt, cg);
      const cpx<T>* coef[3] = {pl->d_lcoefT[1].as<cpx<T>>(), pl->d_lcoefT[2].as<cpx<T>>(),
                               pl->d_lcoefT[3].as<cpx<T>>()};
      launch_nd_lvl_bwd<T>(pl->kg, tt, cg, lj + V.nb_off, n, cells, fac, R, X, pool_stride, nrhs,
                           M.b_cols, coef, st);
    }
    const double b = fwd ? V.nf_bytes : V.nb_bytes, c = fwd ? V.nf_cells : V.nb_cells;
    if (timed) time_end(pl, b + 2.0 * c * nrhs * ts, b / ts * nrhs * 8.0);
  };
  const int nlev = (int)L.levels.size();
  auto fused = [&](bool fwd) {
    if (L.fj_n == 0) return;
    if (timed) time_begin(pl);
    launch_nd_fused<T>(fwd, pl->kg, pl->d_nd_fj.as<int2>() + L.fj_off, L.fj_n, pl->d_nd_fb.as<int2>(),
                       lj, cells, pl->d_nd_umaps.as<int>(), fac, R, U, X, pool_stride, nrhs, kmax, st);
    const double b = fwd ? L.fu_fbytes : L.fu_bbytes;
    if (timed) time_end(pl, b + 2.0 * L.fu_cells * nrhs * ts, b / ts * nrhs * 8.0);
  };
  fused(true);
  for (int l = nlev - 1; l >= 0; --l) level(l, L.levels[l], true);
  // dense tops: the RHS group of the plan's largest top
  if (L.ntop > 0) {
    if (timed) time_begin(pl);
    launch_nd_top<T>(nd_top_kg(tsz, pl->nd_max_ntop, pl->kg), tj, L.ntop, cells,
                     pl->d_nd_usrc.as<int>(), fac, R, U, X, pool_stride, nrhs, kmax, pl->nd_max_ntop,
                     st);
    if (timed) time_end(pl, L.top_bytes + 2.0 * L.top_cells * nrhs * ts, L.top_bytes / ts * nrhs * 8.0);
  }
  for (int l = 0; l < nlev; ++l) level(l, L.levels[l], false);
  fused(false);
}

template <typename T>
void chain_phase(dsd_plan* pl, int phase, const int4* jobs, int njobs, int nrhs, double fbytes,
                 long long blk_cells) {
  hipStream_t st = pl->stream;
  time_begin(pl);
  launch_chain<T>(pl->kg, phase, pl->d_subs.as<SubDesc>(), jobs, njobs, nrhs, pl->kmax,
                  pl->max_nb, pl->d_fac.as<cpx<T>>(), pl->d_lcoefT[pl->dim == 2 ? 2 : 3].as<cpx<T>>(),
                  pl->d_rpool.as<cpx<T>>(), pl->d_vpool.as<cpx<T>>(), pl->sum_nloc * pl->kmax, st);
  // factor blocks once per launch plus the vectors read and written per RHS;
  // 8 real flops per complex factor entry and right-hand side
  time_end(pl, fbytes + (double)blk_cells * nrhs * 2.0 * sizeof(cpx<T>),
           fbytes / sizeof(cpx<T>) * nrhs * 8.0);
}

template <typename T>
void bcr_phase(dsd_plan* pl, const BcrJob* jobs, const BcrLaunch& L, int nrhs) {
  hipStream_t st = pl->stream;
  const long long ps = pl->sum_nloc * pl->kmax;
  const cpx<T>* cpl = pl->d_lcoefT[pl->dim == 2 ? 2 : 3].as<cpx<T>>();
  cpx<T>* rpool = pl->d_rpool.as<cpx<T>>();
  cpx<T>* vpool = pl->d_vpool.as<cpx<T>>();
  if (L.dfwd) {
    launch_bcr_dfwd<T>(pl->d_subs.as<SubDesc>(), jobs + L.off, L.n, nrhs, pl->kmax, pl->max_nb, cpl,
                       rpool, vpool, ps, st);
    return;
  }
  time_begin(pl);
  launch_bcr_solve<T>(L.kg > 0 ? L.kg : pl->kg, pl->d_subs.as<SubDesc>(), jobs + L.off, L.n, L.nset, L.cg, L.rt, nrhs,
                      pl->kmax, pl->max_nb, pl->d_fac.as<cpx<T>>(), cpl, rpool, vpool, ps, st);
  time_end(pl, L.fbytes + L.vcells * nrhs * (double)sizeof(cpx<T>),
           L.fbytes / sizeof(cpx<T>) * nrhs * 8.0);
}

template <typename T>
int sweep_apply_t(dsd_plan* pl, const cpx<double>* f, cpx<double>* u, int nrhs) {
  CHK(ensure_pools(pl));
  hipStream_t st = pl->stream;
  const Problem& P = pl->P;
  const long long pool_stride = pl->sum_nloc * pl->kmax;
  cpx<T>* rpool = pl->d_rpool.as<cpx<T>>();
  cpx<T>* vpool = pl->d_vpool.as<cpx<T>>();
  PartTables pt;
  for (int a = 0; a < 3; ++a) {
    pt.part_of[a] = pl->d_part_of[a].as<int>();
    pt.parts[a] = pl->d_axparts[a].as<AxisPart>();
    pt.P[a] = (int)pl->parts[a].size();
  }
  // additive DDM: the solution slots of steps before the first start at zero
  // (their transfers are read before any step has written them)
  const int Ls = pl->additive ? pl->dim + 1 : pl->L;
  if (pl->additive) {
    launch_zero<T>(vpool, (long long)Ls * pool_stride, st);
  } else {
    // every (sweep, subdomain) solve has a right-hand-side slot of its own, so
    // all of them are initialised up front in one launch (f in the first
    // sweep's slots, 0 elsewhere) and each launch group only adds its transfers
    long long nmem = 0, max_nloc = 0;
    for (const StepTab& t : pl->steps) {
      nmem += t.nmem;
      max_nloc = std::max(max_nloc, t.max_nloc);
    }
    launch_init_rhs<T>(P, pl->d_subs.as<SubDesc>(), pl->d_members.as<int2>(), (int)nmem, max_nloc,
                       nrhs, pl->kmax, f, rpool, pool_stride, 0, st);
  }
  for (size_t gi = 0; gi < pl->steps.size(); ++gi) {
    const StepTab& st_ = pl->steps[gi];
    if (st_.nmem == 0) continue;
    const int2* mem = pl->d_members.as<int2>() + st_.mem_off;
    if (pl->additive)   // the slots rotate: each step starts from f (step 1) or 0
      launch_init_rhs<T>(P, pl->d_subs.as<SubDesc>(), mem, st_.nmem, st_.max_nloc, nrhs, pl->kmax,
                         f, rpool, pool_stride, gi == 0 ? 0 : -1, st);
    launch_pull<T>(P, pl->d_subs.as<SubDesc>(), mem, st_.nmem, pl->d_edges.as<Edge>(),
                   pl->d_erange.as<int2>() + st_.er_off, st_.max_box, nrhs, pl->kmax, vpool,
                   pool_stride, pl->d_lcoefT[0].as<cpx<T>>(), pl->d_lcoefT[1].as<cpx<T>>(),
                   pl->d_lcoefT[2].as<cpx<T>>(), pl->d_lcoefT[3].as<cpx<T>>(), rpool, st);
    if (pl->solver == 4) {
      nd_phase<T>(pl, pl->nd_launch[gi], rpool, vpool, pl->d_upool.as<cpx<T>>(), pool_stride, nrhs,
                  pl->kmax, true);
    } else if (pl->solver == 2 || pl->chain_steps) {
      for (const BcrLaunch& L : pl->bcr_launch[gi]) bcr_phase<T>(pl, pl->d_bcr_jobs.as<BcrJob>(), L, nrhs);
    } else {
      const int4* j2 = pl->d_jobs2.as<int4>() + st_.job_off;
      const int4* j1 = pl->d_jobs1.as<int4>() + st_.mem_off;
      chain_phase<T>(pl, 0, j2, 2 * st_.nmem, nrhs, st_.fac_bytes_fb, st_.blk_cells_fb);
      chain_phase<T>(pl, 1, j1, st_.nmem, nrhs, st_.fac_bytes_mid, st_.blk_cells_mid);
      chain_phase<T>(pl, 2, j2, 2 * st_.nmem, nrhs, st_.fac_bytes_fb, st_.blk_cells_fb);
    }
    if (pl->additive)   // u_DDM += sum_sub beta_0 u^s (step gi's slot)
      launch_assemble_u<T>(P, pl->d_subs.as<SubDesc>(), pt, (int)(gi % Ls), 1, gi > 0 ? 1 : 0,
                           nrhs, pl->kmax, vpool, pool_stride, u, st);
  }
  if (!pl->additive)
    launch_assemble_u<T>(P, pl->d_subs.as<SubDesc>(), pt, 0, pl->L, 0, nrhs, pl->kmax, vpool,
                         pool_stride, u, st);
  HIPCHK(hipGetLastError());
  time_flush(pl);
  return 0;
}

int sweep_apply_eager(dsd_plan* pl, const cpx<double>* f, cpx<double>* u, int nrhs) {
  return pl->c64 ? sweep_apply_t<float>(pl, f, u, nrhs) : sweep_apply_t<double>(pl, f, u, nrhs);
}

// One application as a HIP graph: captured once per (f, u, nrhs) on a private
// stream of default priority, replayed on the plan's stream.  The capture holds
// kernels only (no memset nodes).  Timing mode runs eagerly.
int sweep_apply_any(dsd_plan* pl, const cpx<double>* f, cpx<double>* u, int nrhs) {
  if (!pl->use_graph || pl->timing) return sweep_apply_eager(pl, f, u, nrhs);
  CHK(ensure_pools(pl));
  const auto key = std::make_tuple((const void*)f, (void*)u, nrhs);
  auto it = pl->graphs.find(key);
  if (it == pl->graphs.end()) {
    if (!pl->cap_stream) HIPCHK(hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking));
    const hipStream_t caller = pl->stream;
    pl->stream = pl->cap_stream;
    hipError_t e = hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal);
    int rc = e == hipSuccess ? sweep_apply_eager(pl, f, u, nrhs) : DSD_EHIP;
    hipGraph_t g = nullptr;
    const hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(pl->cap_stream, &g) : e;
    pl->stream = caller;
    if (rc == 0 && e2 != hipSuccess) {
      g_detail = std::string("graph capture: ") + hipGetErrorString(e2);
      rc = DSD_EHIP;
    }
    hipGraphExec_t ex = nullptr;
    if (rc == 0 && hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
      g_detail = "graph instantiation failed";
      rc = DSD_EHIP;
    }
    if (g) (void)hipGraphDestroy(g);
    if (rc != 0) return rc;
    it = pl->graphs.emplace(key, ex).first;
  }
  HIPCHK(hipGraphLaunch(it->second, pl->stream));
  return 0;
}

// ---------------------------------------------------------------- FGMRES (FP64)
// Krylov workspace for batches of up to kb right-hand sides.
int ensure_krylov(dsd_plan* pl, int restart, int kb) {
  if (pl->kr_restart >= restart && pl->kr_k >= kb && pl->d_V.p) return 0;
  const size_t vec = (size_t)kb * pl->P.N * sizeof(cpx<double>);
  CHK(pl->d_V.alloc((size_t)(restart + 1) * vec));
  CHK(pl->d_Z.alloc((size_t)restart * vec));
  CHK(pl->d_w.alloc(vec));
  CHK(pl->d_r.alloc(vec));
  CHK(pl->d_xa.alloc(vec));
  CHK(pl->d_ba.alloc(vec));
  const int nblk = 256;
  CHK(pl->d_part.alloc((size_t)(restart + 1) * kb * nblk * sizeof(cpx<double>)));
  CHK(pl->d_h1.alloc((size_t)(restart + 1) * kb * sizeof(cpx<double>)));
  CHK(pl->d_h2.alloc((size_t)(restart + 1) * kb * sizeof(cpx<double>)));
  CHK(pl->d_hn.alloc((size_t)kb * sizeof(cpx<double>)));
  CHK(pl->d_scal.alloc((size_t)kb * sizeof(double)));
  CHK(pl->d_idx.alloc((size_t)kb * sizeof(int)));
  CHK(pl->d_coef.alloc((size_t)(restart + 1) * kb * sizeof(cpx<double>)));
  pl->kr_restart = restart;
  pl->kr_k = kb;
  return 0;
}

// Right-hand sides one FGMRES batch can hold: the FP64 Krylov vectors
// (restart + 1 basis, restart preconditioned, 4 work) of every RHS must fit in
// the free device memory (plus what the current workspace would release).
int krylov_batch(dsd_plan* pl, int restart, int nrhs) {
  if (pl->d_V.p && pl->kr_restart >= restart && pl->kr_k >= nrhs) return nrhs;
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) return nrhs;
  const Buf* held[] = {&pl->d_V, &pl->d_Z, &pl->d_w, &pl->d_r, &pl->d_xa, &pl->d_ba};
  double have = (double)fr;
  for (const Buf* b : held) have += (double)b->bytes;
  const double per = (double)(2 * restart + 5) * pl->P.N * sizeof(cpx<double>);
  const long long kb = (long long)(0.85 * have / per);
  return (int)std::max(0LL, std::min<long long>(kb, nrhs));
}

typedef std::complex<double> zc;

// Flexible GMRES, right-preconditioned by one sweep application per step,
// batched over the RHS that are still active; classical Gram-Schmidt applied
// twice; restarts from the current iterate with the true FP64 residual.
int gmres_batch(dsd_plan* pl, const cpx<double>* b, cpx<double>* x, int nrhs, double tol,
                int maxit, int restart, int* iters_host, double* relres_host) {
  hipStream_t st = pl->stream;
  const long long N = pl->P.N;
  if (nrhs <= 0) return 0;
  const int nblk = 256;
  cpx<double>* V = pl->d_V.as<cpx<double>>();
  cpx<double>* Z = pl->d_Z.as<cpx<double>>();
  cpx<double>* w = pl->d_w.as<cpx<double>>();
  cpx<double>* r = pl->d_r.as<cpx<double>>();
  cpx<double>* xa = pl->d_xa.as<cpx<double>>();
  cpx<double>* ba = pl->d_ba.as<cpx<double>>();
  cpx<double>* part = pl->d_part.as<cpx<double>>();
  cpx<double>* h1 = pl->d_h1.as<cpx<double>>();
  cpx<double>* h2 = pl->d_h2.as<cpx<double>>();
  cpx<double>* hn = pl->d_hn.as<cpx<double>>();
  double* scal = pl->d_scal.as<double>();
  int* idx = pl->d_idx.as<int>();
  cpx<double>* coef = pl->d_coef.as<cpx<double>>();

  std::vector<cpx<double>> hb(nrhs);
  launch_mdot(b, 1, b, nrhs, N, part, nblk, h1, st);
  HIPCHK(hipMemcpyAsync(hb.data(), h1, nrhs * sizeof(cpx<double>), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemsetAsync(x, 0, (size_t)nrhs * N * sizeof(cpx<double>), st));
  HIPCHK(hipStreamSynchronize(st));
  std::vector<double> bn(nrhs), rel(nrhs, 1.0);
  std::vector<int> it(nrhs, 0);
  std::vector<char> done(nrhs, 0);
  for (int i = 0; i < nrhs; ++i) {
    bn[i] = std::sqrt(hb[i].re);
    if (!std::isfinite(bn[i])) { g_detail = "non-finite right-hand side"; return DSD_ENOTFINITE; }
    if (bn[i] == 0) { done[i] = 1; rel[i] = 0; }
  }
  bool first = true;
  std::vector<int> act, pend;
  std::vector<cpx<double>> hh1, hh2, hhn;
  std::vector<double> hscal;
  while (true) {
    // true residual of every RHS not yet converged
    pend.clear();
    for (int i = 0; i < nrhs; ++i)
      if (!done[i]) pend.push_back(i);
    if (pend.empty()) break;
    const int np = (int)pend.size();
    HIPCHK(hipMemcpyAsync(idx, pend.data(), np * sizeof(int), hipMemcpyHostToDevice, st));
    launch_gather_rhs(b, idx, ba, np, N, st);
    if (first) {
      HIPCHK(hipMemcpyAsync(r, ba, (size_t)np * N * sizeof(cpx<double>), hipMemcpyDeviceToDevice, st));
    } else {
      launch_gather_rhs(x, idx, xa, np, N, st);
      launch_apply_op(pl->P, pl->d_gcoef[0].as<cpx<double>>(), pl->d_gcoef[1].as<cpx<double>>(),
                      pl->d_gcoef[2].as<cpx<double>>(), pl->d_gcoef[3].as<cpx<double>>(), xa, w,
                      np, st);
      launch_sub(ba, w, r, (long long)np * N, st);
    }
    launch_mdot(r, 1, r, np, N, part, nblk, hn, st);
    hhn.resize(np);
    HIPCHK(hipMemcpyAsync(hhn.data(), hn, np * sizeof(cpx<double>), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    act.clear();
    for (int k = 0; k < np; ++k) {
      const int i = pend[k];
      const double beta = std::sqrt(hhn[k].re);
      if (!std::isfinite(beta)) { g_detail = "non-finite residual"; return DSD_ENOTFINITE; }
      rel[i] = beta / bn[i];
      if (rel[i] <= tol || it[i] >= maxit) done[i] = 1;
      else act.push_back(i);
    }
    first = false;
    if (act.empty()) break;
    if ((int)act.size() != np) continue;   // recompute with the reduced set
    const int na = np;
    // V_0 = r / beta
    hscal.resize(na);
    std::vector<double> beta0(na);
    for (int k = 0; k < na; ++k) {
      beta0[k] = std::sqrt(hhn[k].re);
      hscal[k] = 1.0 / beta0[k];
    }
    HIPCHK(hipMemcpyAsync(scal, hscal.data(), na * sizeof(double), hipMemcpyHostToDevice, st));
    launch_scale(r, scal, V, na, N, st);
    const long long vs = (long long)na * N;
    std::vector<std::vector<zc>> H(na, std::vector<zc>((size_t)(restart + 1) * restart));
    std::vector<std::vector<zc>> cs(na, std::vector<zc>(restart)), sn(na, std::vector<zc>(restart));
    std::vector<std::vector<zc>> g(na, std::vector<zc>(restart + 1));
    std::vector<int> js(na, -1);
    for (int k = 0; k < na; ++k) g[k][0] = beta0[k];
    int jmax = 0;
    std::vector<int> live, dead;
    for (int j = 0; j < restart; ++j) {
      live.clear();
      dead.clear();
      for (int k = 0; k < na; ++k) (js[k] < 0 ? live : dead).push_back(k);
      if (live.empty()) break;
      if (dead.empty()) {
        CHK(sweep_apply_any(pl, V + j * vs, Z + j * vs, na));
      } else {
        // only the right-hand sides still iterating are swept (gathered into
        // the residual and right-hand-side work rows, free inside a cycle);
        // the others' rows of Z_j are zero, so every later row stays finite
        const int nl = (int)live.size(), nd = (int)dead.size();
        HIPCHK(hipMemcpyAsync(idx, live.data(), nl * sizeof(int), hipMemcpyHostToDevice, st));
        launch_gather_rhs(V + j * vs, idx, r, nl, N, st);
        CHK(sweep_apply_any(pl, r, ba, nl));
        launch_scatter_rhs(ba, idx, Z + j * vs, nl, N, st);
        HIPCHK(hipMemcpyAsync(idx, dead.data(), nd * sizeof(int), hipMemcpyHostToDevice, st));
        launch_zero_rhs(Z + j * vs, idx, nd, N, st);
      }
      launch_apply_op(pl->P, pl->d_gcoef[0].as<cpx<double>>(), pl->d_gcoef[1].as<cpx<double>>(),
                      pl->d_gcoef[2].as<cpx<double>>(), pl->d_gcoef[3].as<cpx<double>>(),
                      Z + j * vs, w, na, st);
      launch_mdot(V, j + 1, w, na, N, part, nblk, h1, st);
      launch_maxpy(V, j + 1, h1, -1.0, w, na, N, st);
      launch_mdot(V, j + 1, w, na, N, part, nblk, h2, st);
      launch_maxpy(V, j + 1, h2, -1.0, w, na, N, st);
      launch_mdot(w, 1, w, na, N, part, nblk, hn, st);
      hh1.resize((size_t)(j + 1) * na);
      hh2.resize((size_t)(j + 1) * na);
      hhn.resize(na);
      HIPCHK(hipMemcpyAsync(hh1.data(), h1, hh1.size() * sizeof(cpx<double>), hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(hh2.data(), h2, hh2.size() * sizeof(cpx<double>), hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(hhn.data(), hn, na * sizeof(cpx<double>), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      for (int k = 0; k < na; ++k) {
        const double hnorm = std::sqrt(hhn[k].re);
        if (!std::isfinite(hnorm)) { g_detail = "non-finite Arnoldi norm"; return DSD_ENOTFINITE; }
        hscal[k] = hnorm > 1e-300 && js[k] < 0 ? 1.0 / hnorm : 0.0;
      }
      HIPCHK(hipMemcpyAsync(scal, hscal.data(), na * sizeof(double), hipMemcpyHostToDevice, st));
      launch_scale(w, scal, V + (j + 1) * vs, na, N, st);
      HIPCHK(hipGetLastError());
      jmax = j + 1;
      for (int k = 0; k < na; ++k) {
        if (js[k] >= 0) continue;
        const int i = act[k];
        zc* Hk = H[k].data();
        auto Hij = [&](int a, int c) -> zc& { return Hk[(size_t)a * restart + c]; };
        for (int a = 0; a <= j; ++a) {
          const size_t o = (size_t)a * na + k;
          Hij(a, j) = zc(hh1[o].re + hh2[o].re, hh1[o].im + hh2[o].im);
        }
        Hij(j + 1, j) = std::sqrt(hhn[k].re);
        // complex Givens rotations G = [[conj(c), conj(s)], [-s, c]]
        for (int a = 0; a < j; ++a) {
          const zc t0 = std::conj(cs[k][a]) * Hij(a, j) + std::conj(sn[k][a]) * Hij(a + 1, j);
          Hij(a + 1, j) = -sn[k][a] * Hij(a, j) + cs[k][a] * Hij(a + 1, j);
          Hij(a, j) = t0;
        }
        const zc av = Hij(j, j), cv = Hij(j + 1, j);
        const double rho = std::sqrt(std::norm(av) + std::norm(cv));
        cs[k][j] = rho > 0 ? av / rho : zc(1.0);
        sn[k][j] = rho > 0 ? cv / rho : zc(0.0);
        Hij(j, j) = rho;
        Hij(j + 1, j) = 0.0;
        g[k][j + 1] = -sn[k][j] * g[k][j];
        g[k][j] = std::conj(cs[k][j]) * g[k][j];
        it[i] += 1;
        const double est = std::abs(g[k][j + 1]) / bn[i];
        if (est <= tol || it[i] >= maxit || j == restart - 1) js[k] = j + 1;
      }
    }
    // y = H^{-1} g per RHS, x += Z y
    std::vector<cpx<double>> hc((size_t)jmax * na, mk(0.0, 0.0));
    for (int k = 0; k < na; ++k) {
      const int m = js[k] < 0 ? jmax : js[k];
      std::vector<zc> y(m);
      const zc* Hk = H[k].data();
      for (int a = m - 1; a >= 0; --a) {
        zc s = g[k][a];
        for (int c = a + 1; c < m; ++c) s -= Hk[(size_t)a * restart + c] * y[c];
        y[a] = s / Hk[(size_t)a * restart + a];
      }
      for (int a = 0; a < m; ++a) hc[(size_t)a * na + k] = mk(y[a].real(), y[a].imag());
    }
    HIPCHK(hipMemcpyAsync(coef, hc.data(), hc.size() * sizeof(cpx<double>), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(idx, act.data(), na * sizeof(int), hipMemcpyHostToDevice, st));
    launch_gather_rhs(x, idx, xa, na, N, st);
    launch_maxpy(Z, jmax, coef, 1.0, xa, na, N, st);
    launch_scatter_rhs(xa, idx, x, na, N, st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
  }
  bool ok = true;
  for (int i = 0; i < nrhs; ++i) {
    if (iters_host) iters_host[i] = it[i];
    if (relres_host) relres_host[i] = rel[i];
    ok = ok && rel[i] <= tol;
  }
  return ok ? DSD_OK : DSD_NOT_CONVERGED;
}

// Flexible GMRES over any number of right-hand sides (<= max_rhs), in batches
// whose Krylov vectors fit the device memory.
int gmres_core(dsd_plan* pl, const cpx<double>* b, cpx<double>* x, int nrhs, double tol,
               int maxit, int restart, int* iters_host, double* relres_host) {
  if (nrhs <= 0) return 0;
  if (nrhs > pl->kmax || maxit <= 0 || !(tol > 0)) {
    g_detail = "gmres: nrhs must be <= max_rhs, maxit > 0 and tol > 0";
    return DSD_EINVAL;
  }
  if (restart <= 0) restart = 30;
  restart = std::min(restart, maxit);
  CHK(ensure_pools(pl));                 // the sweeps' pools first, then the Krylov batch
  int kb = krylov_batch(pl, restart, nrhs);
  while (true) {
    if (kb < 1) {
      g_detail = "gmres: the Krylov vectors of one right-hand side do not fit in device memory";
      return DSD_ENOMEM;
    }
    const int rc = ensure_krylov(pl, restart, kb);
    if (rc == 0) break;
    if (rc != DSD_ENOMEM) return rc;
    // the free-memory estimate was optimistic: release and try half as many
    Buf* kr[] = {&pl->d_V, &pl->d_Z, &pl->d_w, &pl->d_r, &pl->d_xa, &pl->d_ba};
    for (Buf* b : kr) (void)b->alloc(0);
    pl->kr_restart = pl->kr_k = 0;
    kb /= 2;
  }
  const long long N = pl->P.N;
  int worst = 0;
  for (int r0 = 0; r0 < nrhs; r0 += kb) {
    const int n = std::min(kb, nrhs - r0);
    const int rc = gmres_batch(pl, b + (long long)r0 * N, x + (long long)r0 * N, n, tol, maxit,
                               restart, iters_host ? iters_host + r0 : nullptr,
                               relres_host ? relres_host + r0 : nullptr);
    if (rc < 0) return rc;
    worst = std::max(worst, rc);
  }
  return worst;
}

// Receiver indices are read by kernels: check them on the host first.
int check_receivers(const dsd_plan* pl, const long long* rec_dev, int nrec) {
  std::vector<long long> rec(nrec);
  HIPCHK(hipMemcpy(rec.data(), rec_dev, nrec * sizeof(long long), hipMemcpyDeviceToHost));
  for (long long r : rec)
    if (r < 0 || r >= pl->P.N) {
      g_detail = "receiver index outside the global grid";
      return DSD_EINVAL;
    }
  return 0;
}

int device_lds() {
  int dev = 0, lds = 65536;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
      lds = v;
  }
  return lds;
}

// Largest reduced system (in blocks) the cyclic reduction solves densely: the
// requested bound (default 8), lowered until the dense solve launch fits the
// LDS at the widest RHS group the plan may use, its order m nb <= 2048, and
// its inversion fits the LDS.
int dense_blocks(const dsd_plan* pl, int req) {
  if (req < 0) return 0;
  int m = req > 0 ? req : 8;
  const int lds = device_lds();
  const int kgcap = pl->c64 ? bcr_kg<float>(pl->max_nb, 16) : bcr_kg<double>(pl->max_nb, 16);
  auto need = [&](int mm) {
    return pl->c64 ? bcr_launch_lds_bytes<float>(pl->max_nb, kgcap, mm, 12, 1)
                   : bcr_launch_lds_bytes<double>(pl->max_nb, kgcap, mm, 12, 1);
  };
  while (m >= 2 && (need(m) > (size_t)lds || (long long)m * pl->max_nb > 2048 ||
                    gj_lds_bytes(m * pl->max_nb) > (size_t)lds))
    --m;
  return m >= 2 ? m : 0;
}

int choose_kg(const dsd_plan* pl, int want) {
  const int lds = device_lds();
  if (pl->solver == 4)
    return pl->c64 ? nd_kg<float>(std::max(1, pl->nd_max_nf_narrow), want, (size_t)lds)
                   : nd_kg<double>(std::max(1, pl->nd_max_nf_narrow), want, (size_t)lds);
  if (pl->chain_steps) {
    int kg = pl->c64 ? bcr_kg<float>(pl->max_nb, want) : bcr_kg<double>(pl->max_nb, want);
    auto need = [&](int k) {
      return pl->c64 ? bcr_launch_lds_bytes<float>(pl->max_nb, k, 1, pl->chain_cg, pl->chain_rt)
                     : bcr_launch_lds_bytes<double>(pl->max_nb, k, 1, pl->chain_cg, pl->chain_rt);
    };
    while (kg > 1 && need(kg) > (size_t)lds) kg >>= 1;
    return need(kg) > (size_t)lds ? 0 : kg;
  }
  if (pl->solver == 2) {
    int kg = pl->c64 ? bcr_kg<float>(pl->max_nb, want) : bcr_kg<double>(pl->max_nb, want);
    auto need = [&](int k) {
      return pl->c64 ? bcr_lds_bytes<float>(pl->max_nb, k, 3) : bcr_lds_bytes<double>(pl->max_nb, k, 3);
    };
    while (kg > 1 && need(kg) > (size_t)lds) kg >>= 1;
    return need(kg) > (size_t)lds ? 0 : kg;
  }
  int kg = 4;
  if (!pl->c64 && pl->max_nb > 192) kg = 2;   // register budget of the 4-tile c128 kernel
  while (kg > want && kg > 1) kg >>= 1;
  auto need = [&](int k) {
    return pl->c64 ? chain_lds_bytes<float>(pl->max_nb, k) : chain_lds_bytes<double>(pl->max_nb, k);
  };
  while (kg > 1 && need(kg) > (size_t)lds) kg >>= 1;
  if (need(kg) > (size_t)lds) return 0;
  return kg;
}

}  // namespace

// ============================================================================ C ABI
namespace {

// One subdomain's local solve on R (right-hand sides; the reduction overwrites
// them) and X (solution), both [nrhs][N_loc] in the plan precision from offset
// 0, with the plan's local-solve tables.  Nothing is allocated or uploaded;
// the launches are timed (timing mode) only when `timed`.
template <typename T>
void local_solve_launches(dsd_plan* pl, int sub, cpx<T>* R, cpx<T>* X, cpx<T>* U, int nrhs,
                          bool timed) {
  hipStream_t st = pl->stream;
  if (pl->solver == 4) {   // update vectors: entries x nrhs from U
    nd_phase<T>(pl, pl->nd_local[sub], R, X, U, 0, nrhs, nrhs, timed);
    return;
  }
  const SubDesc* dsub = pl->d_subs_local.as<SubDesc>();
  const cpx<T>* cpl = pl->d_lcoefT[pl->dim == 2 ? 2 : 3].as<cpx<T>>();
  const cpx<T>* fac = pl->d_fac.as<cpx<T>>();
  if (pl->solver == 2 || pl->chain_steps) {
    const BcrJob* jobs = pl->d_local_jobs.as<BcrJob>();
    for (const BcrLaunch& L : pl->local_launch[sub]) {
      if (L.dfwd) {
        launch_bcr_dfwd<T>(dsub, jobs + L.off, L.n, nrhs, pl->kmax, pl->max_nb, cpl, R, X, 0, st);
        continue;
      }
      if (timed) time_begin(pl);
      launch_bcr_solve<T>(L.kg > 0 ? L.kg : pl->kg, dsub, jobs + L.off, L.n, L.nset, L.cg, L.rt,
                          nrhs, pl->kmax, pl->max_nb, fac, cpl, R, X, 0, st);
      if (timed)
        time_end(pl, L.fbytes + L.vcells * nrhs * (double)sizeof(cpx<T>),
                 L.fbytes / sizeof(cpx<T>) * nrhs * 8.0);
    }
    return;
  }
  // chains: phase 0 and 2 run the two halves {sub, 0}, {sub, 1}; phase 1 the middle block
  const int4* jobs = pl->d_local_jobs.as<int4>() + 3 * (long long)sub;
  for (int ph = 0; ph < 3; ++ph) {
    if (timed) time_begin(pl);
    launch_chain<T>(pl->kg, ph, dsub, jobs + (ph == 1 ? 2 : 0), ph == 1 ? 1 : 2, nrhs, pl->kmax,
                    pl->max_nb, fac, cpl, R, X, 0, st);
    if (timed) time_end(pl, 0, 0);
  }
}

template <typename T>
void local_solve_any(dsd_plan* pl, int sub, const double* r_dev, double* u_dev, int nrhs,
                     cpx<T>* R, cpx<T>* X, cpx<T>* U, bool timed) {
  const SubDesc& S = pl->subs[sub];
  launch_pack_local<T>((const cpx<double>*)r_dev, R, S.nloc, nrhs, pl->kmax, pl->stream);
  local_solve_launches<T>(pl, sub, R, X, U, nrhs, timed);
  launch_unpack_local<T>(X, (cpx<double>*)u_dev, S.nloc, nrhs, pl->kmax, pl->stream);
}

}  // namespace

// ------------------------------------------------- allocation-free local solve
// Working memory of dsd_local_solve_noalloc: the packed right-hand sides and
// solutions of one call in the plan precision.  Every GPU the library runs on
// holds its own copy of this array until the process ends; host code never
// uses the array's name (a host-side stand-in), only the device address that
// hipGetSymbolAddress returns for the current device, resolved once per device
// when the first plan is created on it.
static __device__ __align__(256) unsigned char scratch[DSD_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch (resolved once per device).
int resolve_scratch(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) {
    g_detail = "device index beyond the scratch table";
    return DSD_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      g_detail = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return DSD_EHIP;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return 0;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
}  // namespace

extern "C" {

int dsd_plan_create(const dsd_params* params, double omega, const double* m_dev, void* stream,
                    dsd_plan** out) {
  g_detail.clear();
  if (!params || !out || !m_dev) { g_detail = "null argument"; return DSD_EINVAL; }
  *out = nullptr;
  const dsd_params& q = *params;
  if ((q.dim != 2 && q.dim != 3) || q.overlap < 3 || q.pml < 0 || !(q.h > 0) || !(omega > 0) ||
      (q.precision != DSD_C64 && q.precision != DSD_C128) || q.local_solver < 0 ||
      q.local_solver > 4 || q.schedule < 0 || q.schedule > 2 || q.dense_top < -1 ||
      q.dense_top > 64 || q.sweep_order < 0 || q.sweep_order > 1 ||
      (q.sweep_order == 1 && q.dim != 3) || q.nd_leaf < 0 || q.nd_top_cells < 0 ||
      q.nd_top_cells > 9000 || q.nd_wide < 0 || q.nd_wave_steps < 0 || q.nd_fuse < 0) {
    g_detail = "dim must be 2 or 3, overlap >= 3, pml >= 0, h > 0, omega > 0, precision C64|C128, "
               "local_solver 0..4, schedule 0..2, dense_top -1..64, sweep_order 0..1 (1: 3D only), "
               "nd_leaf >= 0, nd_top_cells 0..9000, nd_wide >= 0, nd_wave_steps >= 0, nd_fuse >= 0";
    return DSD_EINVAL;
  }
  for (int a = 0; a < q.dim; ++a)
    if (q.n[a] < 1 || q.parts[a] < 1 || q.parts[a] > q.n[a]) {
      g_detail = "bad grid or partition size";
      return DSD_EINVAL;
    }
  dsd_plan* pl = new dsd_plan();
  pl->prm = q;
  pl->omega = omega;
  pl->dim = q.dim;
  pl->L = 1 << q.dim;
  pl->c64 = q.precision == DSD_C64;
  pl->kmax = std::max(1, q.max_rhs);
  pl->stream = (hipStream_t)stream;
  int rc = build_partition(pl);
  pl->sequential = q.schedule == 1;
  pl->additive = q.schedule == 2;
  if (rc == 0) {
    // local solver: nested dissection in 3D; in 2D block cyclic reduction
    // unless its factor (about three times the chain factor) would take more
    // than 45% of the device memory, then the chains (one launch per block
    // step for blocks of 512 cells or more).  In 2D the subdomains span many
    // wavelengths and nested dissection eliminates closed boxes of physical
    // medium first, whose Dirichlet problems can sit near resonance
    // (ill-conditioned separator blocks); the reduction and the chains
    // eliminate slabs that reach the PML.
    std::vector<long long> toff(pl->S);
    for (int i = 0; i < pl->S; ++i) toff[i] = pl->subs[i].fac_off;
    const long long tsum = pl->sum_fac;
    pl->solver = q.local_solver == 1 || q.local_solver == 3 ? 1
               : q.local_solver == 2 || (q.local_solver == 0 && q.dim == 2) ? 2 : 4;
    if (pl->solver == 4) rc = nd_setup(pl);
    if (pl->solver == 2) {
      pl->dense_max = dense_blocks(pl, q.dense_top);
      bcr_layout(pl);
      size_t fr = 0, tot = 0;
      if (q.local_solver == 0 && hipMemGetInfo(&fr, &tot) == hipSuccess &&
          (double)pl->sum_fac * tsize(pl) > 0.45 * (double)tot) {
        pl->solver = 1;
        for (int i = 0; i < pl->S; ++i) pl->subs[i].fac_off = toff[i];
        pl->sum_fac = tsum;
      }
    }
    pl->chain_steps = pl->solver == 1 &&
                      (q.local_solver == 3 || (q.local_solver == 0 && pl->max_nb >= 512));
  }
  if (rc == 0) {
    const int kdef = pl->solver == 4 ? 8 : ((pl->solver == 2 || pl->chain_steps) ? (pl->c64 ? 8 : 4) : 2);
    pl->kg = choose_kg(pl, q.rhs_per_group > 0 ? q.rhs_per_group : kdef);
    if (pl->kg == 0) {
      g_detail = "subdomain blocks too large for the solve kernel's LDS";
      rc = DSD_EINVAL;
    }
    if (rc == 0 && pl->solver == 4 &&
        nd_top_lds_need(tsize(pl), pl->nd_max_ntop) > (size_t)device_lds()) {
      g_detail = "nested dissection: dense top too large for the top kernel's LDS";
      rc = DSD_EINVAL;
    }
    if (rc == 0 && pl->solver != 4 && gj_lds_bytes(pl->max_nb) > (size_t)device_lds()) {
      g_detail = "subdomain blocks too large for the inversion kernel's LDS";
      rc = DSD_EINVAL;
    }
  }
  if (rc == 0) rc = upload(pl->d_subs, pl->subs);
  if (rc == 0) rc = assemble_and_factor(pl, m_dev);
  if (rc == 0) rc = build_schedule(pl);
  if (rc == 0) rc = build_local_tables(pl);
  if (rc == 0 && hipGetDevice(&pl->device) != hipSuccess) {
    g_detail = "hipGetDevice failed";
    rc = DSD_EHIP;
  }
  if (rc == 0) rc = resolve_scratch(pl->device, &pl->scratch);
  if (rc == 0 && (hipEventCreate(&pl->ev0) != hipSuccess || hipEventCreate(&pl->ev1) != hipSuccess)) {
    g_detail = "hipEventCreate failed";
    rc = DSD_EHIP;
  }
  if (rc != 0) {
    delete pl;
    return rc;
  }
  *out = pl;
  return DSD_OK;
}

void dsd_destroy(dsd_plan* plan) {
  if (plan) {
    (void)hipDeviceSynchronize();
    delete plan;
  }
}

int dsd_plan_info(const dsd_plan* pl, long long* n_global, int* n_subdomains,
                  long long* factor_bytes, long long* workspace_bytes) {
  if (!pl) return DSD_EINVAL;
  if (n_global) *n_global = pl->P.N;
  if (n_subdomains) *n_subdomains = pl->S;
  if (factor_bytes) *factor_bytes = (long long)(pl->sum_fac * tsize(pl));
  if (workspace_bytes) {
    long long w = 0;
    const Buf* bs[] = {&pl->d_rpool, &pl->d_vpool, &pl->d_V, &pl->d_Z, &pl->d_w, &pl->d_r,
                       &pl->d_xa, &pl->d_ba, &pl->d_lcoef64[0], &pl->d_lcoef64[1],
                       &pl->d_lcoef64[2], &pl->d_lcoef64[3], &pl->d_gcoef[0], &pl->d_gcoef[1],
                       &pl->d_gcoef[2], &pl->d_gcoef[3]};
    for (const Buf* b : bs) w += (long long)b->bytes;
    *workspace_bytes = w;
  }
  return DSD_OK;
}

int dsd_plan_pivots(const dsd_plan* pl, double* ratio, int* subdomain) {
  if (!pl) return DSD_EINVAL;
  if (ratio) *ratio = pl->piv_ratio;
  if (subdomain) *subdomain = pl->piv_sub;
  return DSD_OK;
}

int dsd_plan_local_solver(const dsd_plan* pl) {
  return pl ? (pl->chain_steps ? 3 : pl->solver) : DSD_EINVAL;
}

int dsd_set_graph(dsd_plan* pl, int on) {
  if (!pl) return DSD_EINVAL;
  pl->use_graph = on != 0;
  return DSD_OK;
}

int dsd_autotune(dsd_plan* pl, int nrhs, int reps, int* kg_host, int* cg_wide_host,
                 int* cg_mid_host, double* ms_host, void* stream) {
  g_detail.clear();
  if (!pl || nrhs <= 0 || nrhs > pl->kmax || reps <= 0) {
    g_detail = "autotune: bad plan, nrhs (1..max_rhs) or reps";
    return DSD_EINVAL;
  }
  pl->stream = (hipStream_t)stream;
  hipStream_t st = pl->stream;
  const bool was_timing = pl->timing;
  pl->timing = false;
  for (auto& kv : pl->graphs) (void)hipGraphExecDestroy(kv.second);   // tables change
  pl->graphs.clear();
  CHK(ensure_pools(pl));
  Buf f, u;
  const size_t vb = (size_t)nrhs * pl->P.N * sizeof(cpx<double>);
  CHK(f.alloc(vb));
  CHK(u.alloc(vb));
  HIPCHK(hipMemsetAsync(f.p, 0, vb, st));
  // candidates: RHS per workgroup, and the column-group thresholds (2D and 3D
  // block counts differ by an order of magnitude, so the thresholds scale)
  std::vector<int> kgs;
  for (int k : {2, 4, 8, 16}) {
    const int kk = choose_kg(pl, k);
    if (kk > 0 && std::find(kgs.begin(), kgs.end(), kk) == kgs.end()) kgs.push_back(kk);
  }
  // shape policies: {cg_wide, cg_mid, wide_cg, wide_rt, mid_cg, mid_rt, deep_cg, deep_rt, dense_cg}
  const int inf = 1 << 30;
  const int pols[][9] = {
      {32, 8, 1, 0, 4, 1, 8, 1, 8},   {32, 8, 1, 0, 2, 0, 4, 0, 8},   {32, 8, 1, 0, 4, 1, 12, 1, 12},
      {64, 16, 1, 0, 4, 1, 8, 1, 8},  {16, 4, 1, 0, 4, 1, 8, 1, 8},   {32, 8, 2, 0, 4, 1, 8, 1, 8},
      {64, 8, 1, 0, 4, 1, 12, 1, 12}, {32, 8, 1, 0, 2, 1, 8, 1, 4},   {inf, inf, 1, 0, 1, 0, 1, 0, 8}};
  auto get = [&](int* v) {
    const int t[12] = {pl->cg_wide, pl->cg_mid,  pl->wide_cg,  pl->wide_rt, pl->mid_cg,   pl->mid_rt,
                       pl->deep_cg, pl->deep_rt, pl->dense_cg, pl->wide_kg, pl->chain_cg, pl->chain_rt};
    for (int i = 0; i < 12; ++i) v[i] = t[i];
  };
  auto set = [&](const int* v) {
    pl->cg_wide = v[0]; pl->cg_mid = v[1]; pl->wide_cg = v[2]; pl->wide_rt = v[3]; pl->mid_cg = v[4];
    pl->mid_rt = v[5]; pl->deep_cg = v[6]; pl->deep_rt = v[7]; pl->dense_cg = v[8]; pl->wide_kg = v[9];
    pl->chain_cg = v[10]; pl->chain_rt = v[11];
  };
  const int best0_kg = pl->kg;
  int best0[12], bpol[12];
  get(best0);
  get(bpol);
  double best = 1e300;
  int bkg = best0_kg;
  hipEvent_t a = nullptr, b = nullptr;
  HIPCHK(hipEventCreate(&a));
  HIPCHK(hipEventCreate(&b));
  int rc = 0;
  // one candidate: time `reps` applications after one untimed one
  const int lds_dev = device_lds();
  auto trial = [&](int kg, const int* v) -> int {
    if (pl->chain_steps) {   // the chain-step launch must fit the LDS at this shape
      const size_t need = pl->c64 ? bcr_launch_lds_bytes<float>(pl->max_nb, kg, 1, v[10], v[11])
                                  : bcr_launch_lds_bytes<double>(pl->max_nb, kg, 1, v[10], v[11]);
      if (need > (size_t)lds_dev) return 0;
    }
    pl->kg = kg;
    set(v);
    CHK(build_bcr_jobs(pl));
    CHK(sweep_apply_eager(pl, f.as<cpx<double>>(), u.as<cpx<double>>(), nrhs));
    (void)hipEventRecord(a, st);
    for (int r = 0; r < reps; ++r) CHK(sweep_apply_eager(pl, f.as<cpx<double>>(), u.as<cpx<double>>(), nrhs));
    (void)hipEventRecord(b, st);
    if (hipEventSynchronize(b) != hipSuccess) return DSD_EHIP;
    float ms = 0;
    (void)hipEventElapsedTime(&ms, a, b);
    if (ms / reps < best) {
      best = ms / reps;
      bkg = kg;
      for (int i = 0; i < 12; ++i) bpol[i] = v[i];
    }
    return 0;
  };
  // coordinate search: the RHS group width under the current policy, then the
  // level-shape policies at that width, then a wider RHS group on the wide
  // levels (each wide job then streams its matrices once for all of them)
  for (int kg : kgs)
    if ((rc = trial(kg, best0)) != 0) break;
  if (rc == 0 && pl->solver == 2) {
    const int kg1 = bkg;
    for (const auto& pol : pols) {
      int v[12];
      for (int i = 0; i < 9; ++i) v[i] = pol[i];
      v[9] = 0;
      v[10] = best0[10];
      v[11] = best0[11];
      if ((rc = trial(kg1, v)) != 0) break;
    }
    if (rc == 0 && !kgs.empty() && kgs.back() > kg1) {
      int v[12];
      for (int i = 0; i < 12; ++i) v[i] = bpol[i];
      v[9] = kgs.back();
      rc = trial(kg1, v);
    }
  }
  if (rc == 0 && pl->chain_steps) {
    // chain steps: (column groups, row tiles per workgroup) at the best width
    const int shapes[][2] = {{3, 0}, {2, 0}, {1, 0}, {4, 1}, {8, 1}, {12, 1}};
    for (int kg : kgs)
      for (const auto& sh : shapes) {
        int v[12];
        for (int i = 0; i < 12; ++i) v[i] = bpol[i];
        v[10] = sh[0];
        v[11] = sh[1];
        if ((rc = trial(kg, v)) != 0) break;
      }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  pl->kg = rc == 0 ? bkg : best0_kg;
  set(rc == 0 ? bpol : best0);
  const int rc2 = build_bcr_jobs(pl);
  pl->timing = was_timing;
  if (rc != 0) return rc;
  if (rc2 != 0) return rc2;
  if (kg_host) *kg_host = pl->kg;
  if (cg_wide_host) *cg_wide_host = pl->cg_wide;
  if (cg_mid_host) *cg_mid_host = pl->cg_mid;
  if (ms_host) *ms_host = best;
  HIPCHK(hipStreamSynchronize(st));
  return DSD_OK;
}

int dsd_get_solve_shape(const dsd_plan* pl, int* v) {
  if (!pl || !v) return DSD_EINVAL;
  const int t[13] = {pl->kg,      pl->cg_wide, pl->cg_mid,   pl->wide_cg, pl->wide_rt,
                     pl->mid_cg,  pl->mid_rt,  pl->deep_cg,  pl->deep_rt, pl->dense_cg,
                     pl->wide_kg, pl->chain_cg, pl->chain_rt};
  for (int i = 0; i < 13; ++i) v[i] = t[i];
  return DSD_OK;
}

int dsd_set_solve_shape(dsd_plan* pl, const int* v) {
  g_detail.clear();
  if (!pl || !v) { g_detail = "null argument"; return DSD_EINVAL; }
  auto shape_ok = [](int cg, int rt) { return (rt == 0 && cg >= 1 && cg <= 4) || (rt == 1 && cg >= 1 && cg <= 12); };
  const int c0 = pl->chain_cg, r0 = pl->chain_rt;
  pl->chain_cg = v[11];
  pl->chain_rt = v[12];
  const int kg = shape_ok(v[11], v[12]) ? choose_kg(pl, v[0]) : 0;
  const bool wkg_ok = v[10] == 0 || (v[10] >= 1 && choose_kg(pl, v[10]) == v[10]);
  pl->chain_cg = c0;
  pl->chain_rt = r0;
  if (v[0] < 1 || kg != v[0] || v[1] < 1 || v[2] < 1 || !shape_ok(v[3], v[4]) || !shape_ok(v[5], v[6]) ||
      !shape_ok(v[7], v[8]) || v[9] < 1 || v[9] > 12 || !wkg_ok || !shape_ok(v[11], v[12])) {
    g_detail = "solve shape: RHS per workgroup the plan supports, thresholds >= 1, (cg, rt) with rt 0 "
               "and cg 1..4 or rt 1 and cg 1..12, dense cg 1..12, wide-level RHS per workgroup 0 or supported";
    return DSD_EINVAL;
  }
  pl->kg = v[0];
  pl->cg_wide = v[1]; pl->cg_mid = v[2]; pl->wide_cg = v[3]; pl->wide_rt = v[4];
  pl->mid_cg = v[5]; pl->mid_rt = v[6]; pl->deep_cg = v[7]; pl->deep_rt = v[8]; pl->dense_cg = v[9];
  pl->wide_kg = v[10];
  pl->chain_cg = v[11];
  pl->chain_rt = v[12];
  for (auto& kv : pl->graphs) (void)hipGraphExecDestroy(kv.second);   // tables change
  pl->graphs.clear();
  return build_bcr_jobs(pl);
}

int dsd_subdomain_grid(const dsd_plan* pl, int sub, int* dims, int* g0) {
  if (!pl || sub < 0 || sub >= pl->S) return DSD_EINVAL;
  for (int a = 0; a < 3; ++a) {
    if (dims) dims[a] = pl->subs[sub].dims[a];
    if (g0) g0[a] = pl->subs[sub].ax[a].g0;
  }
  return DSD_OK;
}

int dsd_local_solve(dsd_plan* pl, int sub, const double* r_dev, double* u_dev, int nrhs,
                    void* stream) {
  g_detail.clear();
  if (!pl || sub < 0 || sub >= pl->S || nrhs <= 0 || nrhs > pl->kmax || !r_dev || !u_dev) {
    g_detail = "local_solve: bad subdomain, nrhs or pointer";
    return DSD_EINVAL;
  }
  pl->stream = (hipStream_t)stream;
  CHK(ensure_pools(pl));
  const long long off = pl->subs[sub].vec_off * pl->kmax;
  if (pl->c64)
    local_solve_any<float>(pl, sub, r_dev, u_dev, nrhs, pl->d_rpool.as<cpx<float>>() + off,
                           pl->d_vpool.as<cpx<float>>() + off, pl->d_upool.as<cpx<float>>(), true);
  else
    local_solve_any<double>(pl, sub, r_dev, u_dev, nrhs, pl->d_rpool.as<cpx<double>>() + off,
                            pl->d_vpool.as<cpx<double>>() + off, pl->d_upool.as<cpx<double>>(),
                            true);
  HIPCHK(hipGetLastError());
  time_flush(pl);
  HIPCHK(hipStreamSynchronize(pl->stream));
  return DSD_OK;
}

int dsd_local_solve_noalloc(dsd_plan* pl, int sub, const double* r_dev, double* u_dev,
                            int nrhs, void* stream) {
  g_detail.clear();
  if (!pl || sub < 0 || sub >= pl->S || nrhs <= 0 || nrhs > pl->kmax || !r_dev || !u_dev) {
    g_detail = "local_solve_noalloc: bad subdomain, nrhs or pointer";
    return DSD_EINVAL;
  }
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev != pl->device || !pl->scratch) {
    g_detail = "local_solve_noalloc: the current device is not the plan's device";
    return DSD_EINVAL;
  }
  const size_t part = align256((size_t)pl->subs[sub].nloc * nrhs * tsize(pl));
  const size_t upart = pl->solver == 4 ? align256((size_t)pl->nd_local[sub].upd * nrhs * tsize(pl)) : 0;
  if (2 * part + upart > (size_t)DSD_NOALLOC_SCRATCH_BYTES) {
    g_detail = "local_solve_noalloc: the call's working values (" +
               std::to_string(2 * part + upart) + " bytes) exceed the static scratch of " +
               std::to_string((long long)DSD_NOALLOC_SCRATCH_BYTES) + " bytes";
    return DSD_EINVAL;
  }
  pl->stream = (hipStream_t)stream;
  unsigned char* base = static_cast<unsigned char*>(pl->scratch);
  if (pl->c64)
    local_solve_any<float>(pl, sub, r_dev, u_dev, nrhs, reinterpret_cast<cpx<float>*>(base),
                           reinterpret_cast<cpx<float>*>(base + part),
                           reinterpret_cast<cpx<float>*>(base + 2 * part), false);
  else
    local_solve_any<double>(pl, sub, r_dev, u_dev, nrhs, reinterpret_cast<cpx<double>*>(base),
                            reinterpret_cast<cpx<double>*>(base + part),
                            reinterpret_cast<cpx<double>*>(base + 2 * part), false);
  HIPCHK(hipGetLastError());
  return DSD_OK;
}

int dsd_sweep_apply(dsd_plan* pl, const double* f_dev, double* u_dev, int nrhs, void* stream) {
  g_detail.clear();
  if (!pl || !f_dev || !u_dev || nrhs <= 0 || nrhs > pl->kmax) {
    g_detail = "sweep_apply: bad pointer or nrhs (must be 1..max_rhs)";
    return DSD_EINVAL;
  }
  pl->stream = (hipStream_t)stream;
  return sweep_apply_any(pl, (const cpx<double>*)f_dev, (cpx<double>*)u_dev, nrhs);
}

int dsd_apply_operator(dsd_plan* pl, const double* x_dev, double* y_dev, int nrhs, void* stream) {
  g_detail.clear();
  if (!pl || !x_dev || !y_dev || nrhs <= 0 || x_dev == y_dev) {
    g_detail = "apply_operator: bad pointer or nrhs";
    return DSD_EINVAL;
  }
  pl->stream = (hipStream_t)stream;
  launch_apply_op(pl->P, pl->d_gcoef[0].as<cpx<double>>(), pl->d_gcoef[1].as<cpx<double>>(),
                  pl->d_gcoef[2].as<cpx<double>>(), pl->d_gcoef[3].as<cpx<double>>(),
                  (const cpx<double>*)x_dev, (cpx<double>*)y_dev, nrhs, pl->stream);
  HIPCHK(hipGetLastError());
  return DSD_OK;
}

int dsd_gmres_solve(dsd_plan* pl, const double* b_dev, double* x_dev, int nrhs, double tol,
                    int maxit, int restart, int* iters_host, double* relres_host, void* stream) {
  g_detail.clear();
  if (!pl || !b_dev || !x_dev || b_dev == x_dev) { g_detail = "gmres: bad pointer"; return DSD_EINVAL; }
  pl->stream = (hipStream_t)stream;
  return gmres_core(pl, (const cpx<double>*)b_dev, (cpx<double>*)x_dev, nrhs, tol, maxit, restart,
                    iters_host, relres_host);
}

// The diagonal sweeps as a stand-alone iterative solver (Section 5.2 uses them
// so for the three-layer residual-decay test): x_0 = 0 and
//   x_{k+1} = x_k + DDM(f - M x_k),
// with the true FP64 residual after every sweep application.
int dsd_ddm_iterate(dsd_plan* pl, const double* f_dev, double* x_dev, int nrhs, int iters,
                    double* relres_hist_host, void* stream) {
  g_detail.clear();
  if (!pl || !f_dev || !x_dev || f_dev == x_dev || !relres_hist_host || nrhs <= 0 ||
      nrhs > pl->kmax || iters < 0) {
    g_detail = "ddm_iterate: bad pointer, nrhs (1..max_rhs) or iters (>= 0)";
    return DSD_EINVAL;
  }
  pl->stream = (hipStream_t)stream;
  hipStream_t st = pl->stream;
  CHK(ensure_pools(pl));
  CHK(ensure_krylov(pl, 1, nrhs));
  const long long N = pl->P.N;
  const int nblk = 256;
  const cpx<double>* f = (const cpx<double>*)f_dev;
  cpx<double>* x = (cpx<double>*)x_dev;
  cpx<double>* r = pl->d_r.as<cpx<double>>();
  cpx<double>* z = pl->d_Z.as<cpx<double>>();
  cpx<double>* w = pl->d_w.as<cpx<double>>();
  cpx<double>* part = pl->d_part.as<cpx<double>>();
  cpx<double>* hn = pl->d_hn.as<cpx<double>>();
  cpx<double>* ones = pl->d_coef.as<cpx<double>>();
  std::vector<cpx<double>> h(nrhs, mk(1.0, 0.0));
  HIPCHK(hipMemcpyAsync(ones, h.data(), nrhs * sizeof(cpx<double>), hipMemcpyHostToDevice, st));
  auto norms = [&](const cpx<double>* v, std::vector<double>& out) -> int {
    launch_mdot(v, 1, v, nrhs, N, part, nblk, hn, st);
    HIPCHK(hipMemcpyAsync(h.data(), hn, nrhs * sizeof(cpx<double>), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    out.resize(nrhs);
    for (int i = 0; i < nrhs; ++i) out[i] = std::sqrt(h[i].re);
    return 0;
  };
  std::vector<double> fn, rn;
  CHK(norms(f, fn));
  for (int i = 0; i < nrhs; ++i) {
    if (!std::isfinite(fn[i])) { g_detail = "non-finite right-hand side"; return DSD_ENOTFINITE; }
    relres_hist_host[i] = fn[i] > 0 ? 1.0 : 0.0;
  }
  HIPCHK(hipMemsetAsync(x, 0, (size_t)nrhs * N * sizeof(cpx<double>), st));
  HIPCHK(hipMemcpyAsync(r, f, (size_t)nrhs * N * sizeof(cpx<double>), hipMemcpyDeviceToDevice, st));
  for (int k = 1; k <= iters; ++k) {
    CHK(sweep_apply_any(pl, r, z, nrhs));
    launch_maxpy(z, 1, ones, 1.0, x, nrhs, N, st);
    launch_apply_op(pl->P, pl->d_gcoef[0].as<cpx<double>>(), pl->d_gcoef[1].as<cpx<double>>(),
                    pl->d_gcoef[2].as<cpx<double>>(), pl->d_gcoef[3].as<cpx<double>>(), x, w,
                    nrhs, st);
    launch_sub(f, w, r, (long long)nrhs * N, st);
    HIPCHK(hipGetLastError());
    CHK(norms(r, rn));
    for (int i = 0; i < nrhs; ++i) {
      if (!std::isfinite(rn[i])) { g_detail = "non-finite residual"; return DSD_ENOTFINITE; }
      relres_hist_host[(long long)k * nrhs + i] = fn[i] > 0 ? rn[i] / fn[i] : 0.0;
    }
  }
  return DSD_OK;
}

int dsd_adjoint_solve(dsd_plan* pl, const double* b_dev, double* x_dev, int nrhs, double tol,
                      int maxit, int restart, int* iters_host, double* relres_host,
                      void* stream) {
  g_detail.clear();
  if (!pl || !b_dev || !x_dev || b_dev == x_dev || nrhs <= 0 || nrhs > pl->kmax) {
    g_detail = "adjoint: bad pointer or nrhs";
    return DSD_EINVAL;
  }
  pl->stream = (hipStream_t)stream;
  const long long n = (long long)nrhs * pl->P.N;
  CHK(pl->d_y.bytes >= (size_t)n * sizeof(cpx<double>) ? 0 : pl->d_y.alloc((size_t)pl->kmax * pl->P.N * sizeof(cpx<double>)));
  cpx<double>* tmp = pl->d_y.as<cpx<double>>();
  launch_conj((const cpx<double>*)b_dev, tmp, n, pl->stream);
  int rc = gmres_core(pl, tmp, (cpx<double>*)x_dev, nrhs, tol, maxit, restart, iters_host,
                      relres_host);
  if (rc < 0) return rc;
  launch_conj((const cpx<double>*)x_dev, (cpx<double>*)x_dev, n, pl->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(pl->stream));
  return rc;
}

int dsd_fwi_forward(dsd_plan* pl, const double* f_dev, int nsrc, const long long* rec_dev,
                    int nrec, double tol, int maxit, double* d_dev, void* stream) {
  g_detail.clear();
  if (!pl || !f_dev || !rec_dev || !d_dev || nsrc <= 0 || nsrc > pl->kmax || nrec <= 0) {
    g_detail = "fwi_forward: bad pointer, nsrc (<= max_rhs) or nrec";
    return DSD_EINVAL;
  }
  pl->stream = (hipStream_t)stream;
  CHK(check_receivers(pl, rec_dev, nrec));
  const size_t vec = (size_t)pl->kmax * pl->P.N * sizeof(cpx<double>);
  if (pl->d_u.bytes < vec) CHK(pl->d_u.alloc(vec));
  int rc = gmres_core(pl, (const cpx<double>*)f_dev, pl->d_u.as<cpx<double>>(), nsrc, tol, maxit,
                      0, nullptr, nullptr);
  if (rc < 0) return rc;
  launch_sample(pl->d_u.as<cpx<double>>(), nsrc, pl->P.N, rec_dev, nrec, (cpx<double>*)d_dev,
                pl->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(pl->stream));
  return rc;
}

int dsd_fwi_gradient(dsd_plan* pl, const double* f_dev, int nsrc, const long long* rec_dev,
                     int nrec, const double* dobs_dev, double tol, int maxit, double* grad_dev,
                     double* misfit_host, double* u_dev, void* stream) {
  g_detail.clear();
  if (!pl || !f_dev || !rec_dev || !dobs_dev || !grad_dev || nsrc <= 0 || nsrc > pl->kmax ||
      nrec <= 0) {
    g_detail = "fwi_gradient: bad pointer, nsrc (<= max_rhs) or nrec";
    return DSD_EINVAL;
  }
  pl->stream = (hipStream_t)stream;
  CHK(check_receivers(pl, rec_dev, nrec));
  hipStream_t st = pl->stream;
  const long long N = pl->P.N;
  const size_t vec = (size_t)pl->kmax * N * sizeof(cpx<double>);
  if (pl->d_u.bytes < vec) CHK(pl->d_u.alloc(vec));
  if (pl->d_adj.bytes < vec) CHK(pl->d_adj.alloc(vec));
  if (pl->d_y.bytes < vec) CHK(pl->d_y.alloc(vec));
  CHK(pl->d_res.alloc((size_t)nsrc * nrec * sizeof(cpx<double>)));
  CHK(pl->d_mpart.alloc((size_t)nsrc * sizeof(double)));
  cpx<double>* u = u_dev ? (cpx<double>*)u_dev : pl->d_u.as<cpx<double>>();
  int rc1 = gmres_core(pl, (const cpx<double>*)f_dev, u, nsrc, tol, maxit, 0, nullptr, nullptr);
  if (rc1 < 0) return rc1;
  HIPCHK(hipMemsetAsync(pl->d_adj.p, 0, (size_t)nsrc * N * sizeof(cpx<double>), st));
  launch_fwi_residual(u, nsrc, N, rec_dev, nrec, (const cpx<double>*)dobs_dev,
                      pl->d_res.as<cpx<double>>(), pl->d_adj.as<cpx<double>>(),
                      pl->d_mpart.as<double>(), st);
  std::vector<double> mp(nsrc);
  HIPCHK(hipMemcpyAsync(mp.data(), pl->d_mpart.p, nsrc * sizeof(double), hipMemcpyDeviceToHost, st));
  int rc2 = gmres_core(pl, pl->d_adj.as<cpx<double>>(), pl->d_y.as<cpx<double>>(), nsrc, tol,
                       maxit, 0, nullptr, nullptr);
  if (rc2 < 0) return rc2;
  launch_fwi_gradient(pl->P, u, pl->d_y.as<cpx<double>>(), nsrc, grad_dev, st);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  double J = 0;
  for (double v : mp) J += v;
  if (misfit_host) *misfit_host = J;
  return (rc1 == DSD_NOT_CONVERGED || rc2 == DSD_NOT_CONVERGED) ? DSD_NOT_CONVERGED : DSD_OK;
}

const char* dsd_strerror(int code) {
  switch (code) {
    case DSD_OK: return "success";
    case DSD_NOT_CONVERGED: return "tolerance not reached within maxit";
    case DSD_EINVAL: return "invalid argument";
    case DSD_ENOMEM: return "out of device memory";
    case DSD_EHIP: return "HIP runtime error";
    case DSD_EPIVOT: return "singular block in a subdomain factorisation";
    case DSD_ENOTFINITE: return "non-finite value in a norm";
    default: return "unknown error";
  }
}

const char* dsd_last_error_detail(void) { return g_detail.c_str(); }

int dsd_timing_enable(dsd_plan* pl, int on) {
  if (!pl) return DSD_EINVAL;
  time_flush(pl);
  pl->timing = on != 0;
  pl->t_solve_ms = pl->t_other_ms = pl->solve_bytes = pl->solve_flops = 0;
  pl->solve_launches = 0;
  return DSD_OK;
}

int dsd_timing_read(dsd_plan* pl, double* solve_ms, long long* solve_launches,
                    double* solve_bytes, double* other_ms) {
  if (!pl) return DSD_EINVAL;
  time_flush(pl);
  if (solve_ms) *solve_ms = pl->t_solve_ms;
  if (solve_launches) *solve_launches = pl->solve_launches;
  if (solve_bytes) *solve_bytes = pl->solve_bytes;
  if (other_ms) *other_ms = pl->t_other_ms;
  return DSD_OK;
}

int dsd_timing_flops(dsd_plan* pl, double* solve_flops) {
  if (!pl || !solve_flops) return DSD_EINVAL;
  time_flush(pl);
  *solve_flops = pl->solve_flops;
  return DSD_OK;
}

}  // extern "C"
