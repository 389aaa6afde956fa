// Nested-dissection (multifrontal) local solver: symbolic analysis of a local
// grid shape (host), factorisation kernels (FP64) and the subtree / dense-top
// solve kernels (plan precision).  The layout of the tables is described in
// nd.hpp.
#include <algorithm>
#include <type_traits>
#include <vector>

#include "nd.hpp"

namespace dsd {

static inline unsigned nd_cdiv(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

// ============================================================================
// Analysis (host)
// ============================================================================
namespace {

struct NdBuilder {
  int dim;
  int dims[3];
  int leaf_max;
  std::vector<NdNode>* nodes;

  int index(int x, int y, int z) const { return x + dims[0] * (y + dims[1] * z); }

  void box(const int* lo, const int* hi, std::vector<int>& out) const {
    for (int z = lo[2]; z < hi[2]; ++z)
      for (int y = lo[1]; y < hi[1]; ++y)
        for (int x = lo[0]; x < hi[0]; ++x) out.push_back(index(x, y, z));
  }

  // Node of box [lo, hi) and (recursively, first) its children; returns its id.
  int build(const int* lo, const int* hi, int depth) {
    int ext[3], a = 0;
    long long vol = 1;
    for (int k = 0; k < 3; ++k) {
      ext[k] = hi[k] - lo[k];
      vol *= ext[k];
    }
    for (int k = 1; k < dim; ++k)
      if (ext[k] > ext[a]) a = k;
    NdNode n;
    for (int k = 0; k < 3; ++k) {
      n.lo[k] = lo[k];
      n.hi[k] = hi[k];
    }
    n.depth = depth;
    if (vol <= leaf_max || ext[a] < 3) {
      box(lo, hi, n.sep);
    } else {
      const int mid = lo[a] + ext[a] / 2;
      int h1[3] = {hi[0], hi[1], hi[2]}, l2[3] = {lo[0], lo[1], lo[2]};
      h1[a] = mid;
      l2[a] = mid + 1;
      n.child[0] = build(lo, h1, depth + 1);
      n.child[1] = build(l2, hi, depth + 1);
      int sl[3] = {lo[0], lo[1], lo[2]}, sh[3] = {hi[0], hi[1], hi[2]};
      sl[a] = mid;
      sh[a] = mid + 1;
      box(sl, sh, n.sep);
    }
    // boundary: the cells just outside every face of the box
    for (int k = 0; k < dim; ++k)
      for (int side = 0; side < 2; ++side) {
        const int c = side == 0 ? lo[k] - 1 : hi[k];
        if (c < 0 || c >= dims[k]) continue;
        int fl[3] = {lo[0], lo[1], lo[2]}, fh[3] = {hi[0], hi[1], hi[2]};
        fl[k] = c;
        fh[k] = c + 1;
        box(fl, fh, n.bnd);
      }
    std::sort(n.bnd.begin(), n.bnd.end());
    nodes->push_back(std::move(n));
    const int id = (int)nodes->size() - 1;
    for (int c : (*nodes)[id].child)
      if (c >= 0) (*nodes)[c].parent = id;
    return id;
  }
};

}  // namespace

NdShape nd_analyse(int dim, const int* dims, int leaf_max, int ntop_max) {
  NdShape S;
  S.dim = dim;
  for (int k = 0; k < 3; ++k) S.dims[k] = k < dim ? dims[k] : 1;
  NdBuilder b{dim, {S.dims[0], S.dims[1], S.dims[2]}, std::max(1, leaf_max), &S.nodes};
  const int lo[3] = {0, 0, 0};
  b.build(lo, S.dims, 0);
  // dense top: the deepest depth whose separators (with all above) fit ntop_max
  int maxd = 0;
  for (const NdNode& n : S.nodes) maxd = std::max(maxd, n.depth);
  std::vector<long long> at(maxd + 1, 0);
  for (const NdNode& n : S.nodes) at[n.depth] += (long long)n.sep.size();
  long long cum = 0;
  S.dtop = 0;
  for (int d = 0; d <= maxd; ++d) {
    if (cum + at[d] > ntop_max) break;
    cum += at[d];
    S.dtop = d + 1;
  }
  const int N = (int)S.nodes.size();
  for (int i = 0; i < N; ++i) {
    NdNode& n = S.nodes[i];
    n.top = n.depth < S.dtop;
    if (n.top) S.top_cells.insert(S.top_cells.end(), n.sep.begin(), n.sep.end());
  }
  for (int i = 0; i < N; ++i) {
    NdNode& n = S.nodes[i];
    if (!n.top && (n.parent < 0 || S.nodes[n.parent].top)) {
      n.subtree = (int)S.roots.size();
      n.level = 0;
      S.roots.push_back(i);
    }
  }
  // parents come after their children in postorder: walk backwards
  for (int i = N - 1; i >= 0; --i) {
    NdNode& n = S.nodes[i];
    if (n.top) continue;
    if (n.subtree < 0) {
      n.subtree = S.nodes[n.parent].subtree;
      n.level = S.nodes[n.parent].level + 1;
    }
    S.nlev = std::max(S.nlev, n.level + 1);
  }
  long long fo = 0, uo = 0;
  for (NdNode& n : S.nodes) {
    if (n.top) continue;
    const long long ns = (long long)n.sep.size(), nb = (long long)n.bnd.size();
    n.fac = fo;
    fo += nb * ns + ns * (ns + nb);
    n.upd = uo;
    uo += nb;
    S.max_ns = std::max(S.max_ns, (int)ns);
    S.max_nbd = std::max(S.max_nbd, (int)nb);
    S.max_nf = std::max(S.max_nf, (int)(ns + nb));
  }
  S.top_fac = fo;
  S.fac_entries = fo + (long long)S.ntop() * S.ntop();
  S.upd_entries = uo;
  return S;
}

constexpr int ND_TW = 8;    // waves per dense-top workgroup

bool nd_append_tables(const NdShape& S, NdShapeTab& tab, std::vector<NdNodeDev>& nodes,
                      std::vector<int>& cells, std::vector<int>& maps, std::vector<int>& umaps,
                      std::vector<int>& src, std::vector<int>& usrc, std::vector<int>& lev,
                      std::vector<int>& levmax, std::vector<int>& levnodes) {
  const int dim2 = 2 * S.dim;
  const int N = (int)S.nodes.size();
  const long long ncell = (long long)S.dims[0] * S.dims[1] * S.dims[2];
  tab.node0 = (int)nodes.size();
  std::vector<int> pos(ncell, -1);
  for (int i = 0; i < N; ++i) {
    const NdNode& n = S.nodes[i];
    NdNodeDev d{};
    d.ns = (int)n.sep.size();
    d.nbd = (int)n.bnd.size();
    d.cell = (int)cells.size();
    cells.insert(cells.end(), n.sep.begin(), n.sep.end());
    cells.insert(cells.end(), n.bnd.begin(), n.bnd.end());
    d.map = (int)maps.size();
    d.ch0 = n.child[0] >= 0 && !n.top ? tab.node0 + n.child[0] : -1;
    d.ch1 = n.child[1] >= 0 && !n.top ? tab.node0 + n.child[1] : -1;
    d.fac = n.fac;
    d.upd = n.upd;
    const int nf = d.ns + d.nbd;
    maps.insert(maps.end(), (size_t)2 * nf, -1);
    umaps.insert(umaps.end(), (size_t)2 * nf, -1);
    if (!n.top) {
      // front position of every cell of this node's front
      for (int p = 0; p < nf; ++p) pos[p < d.ns ? n.sep[p] : n.bnd[p - d.ns]] = p;
      for (int c = 0; c < 2; ++c) {
        if (n.child[c] < 0) continue;
        const std::vector<int>& cb = S.nodes[n.child[c]].bnd;
        for (int i2 = 0; i2 < (int)cb.size(); ++i2) {
          const int p = pos[cb[i2]];
          if (p < 0) return false;   // a child's boundary must lie in the parent's front
          maps[d.map + 2 * p + c] = i2;
          umaps[d.map + 2 * p + c] = (int)(S.nodes[n.child[c]].upd + i2);
        }
      }
      for (int p = 0; p < nf; ++p) pos[p < d.ns ? n.sep[p] : n.bnd[p - d.ns]] = -1;
    }
    nodes.push_back(d);
  }
  // top cells and the subtree-root updates that land on each of them
  tab.top_cell = (int)cells.size();
  cells.insert(cells.end(), S.top_cells.begin(), S.top_cells.end());
  tab.top_src = (int)src.size();
  const int ntop = S.ntop();
  src.insert(src.end(), (size_t)ntop * dim2 * 2, -1);
  for (int p = 0; p < ntop; ++p) pos[S.top_cells[p]] = p;
  for (int r : S.roots) {
    const std::vector<int>& rb = S.nodes[r].bnd;
    for (int i = 0; i < (int)rb.size(); ++i) {
      const int p = pos[rb[i]];
      if (p < 0) return false;       // a subtree root's boundary must lie in the top
      int k = 0;
      while (k < dim2 && src[tab.top_src + (p * dim2 + k) * 2] >= 0) ++k;
      if (k == dim2) return false;
      src[tab.top_src + (p * dim2 + k) * 2] = r;
      src[tab.top_src + (p * dim2 + k) * 2 + 1] = i;
    }
  }
  tab.top_usrc = (int)usrc.size();
  for (int p = 0; p < ntop; ++p)
    for (int k = 0; k < dim2; ++k) {
      const int r = src[tab.top_src + (p * dim2 + k) * 2];
      usrc.push_back(r < 0 ? -1 : (int)(S.nodes[r].upd + src[tab.top_src + (p * dim2 + k) * 2 + 1]));
    }
  // level lists of every subtree and the largest front of each level
  tab.lev0.clear();
  tab.nlev.clear();
  for (size_t s = 0; s < S.roots.size(); ++s) {
    int nl = 0;
    for (const NdNode& n : S.nodes)
      if (n.subtree == (int)s) nl = std::max(nl, n.level + 1);
    tab.lev0.push_back((int)lev.size());
    tab.nlev.push_back(nl);
    for (int l = 0; l < nl; ++l) {
      lev.push_back((int)levnodes.size());
      int mx = 0;
      for (int i = 0; i < N; ++i)
        if (S.nodes[i].subtree == (int)s && S.nodes[i].level == l) {
          levnodes.push_back(tab.node0 + i);
          mx = std::max(mx, (int)(S.nodes[i].sep.size() + S.nodes[i].bnd.size()));
        }
      levmax.push_back(mx);
    }
    lev.push_back((int)levnodes.size());
    levmax.push_back(0);
  }
  return true;
}

// ============================================================================
// Solve kernels
// ============================================================================
// Lanes take (row, right-hand side) pairs: 64 / KG rows of one node per pass,
// so the small separators of the deep levels still fill the wave; gathers
// take one front position per lane (index loads once, then KG data loads).

// Load through a global-address-space pointer: a pointer selected between two
// arrays would otherwise be generic and compile to flat loads, whose wait
// also covers every other load in flight.
template <typename T>
__device__ __forceinline__ cpx<T> nd_gload(const cpx<T>* p) {
  const __attribute__((address_space(1))) T* g = (const __attribute__((address_space(1))) T*)p;
  return mk(g[0], g[1]);
}

// Select between two complex values by component: a conditional between two
// complex lvalues selects an address, which keeps the arrays in memory
// (scratch, or flat loads when one side is in LDS).
template <typename T>
__device__ __forceinline__ cpx<T> nd_sel(bool c, cpx<T> a, cpx<T> b) {
  return mk(c ? a.re : b.re, c ? a.im : b.im);
}

__device__ __forceinline__ void nd_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// XCD-aware order (grid a multiple of 8): consecutive tasks share an L2.
__device__ __forceinline__ int nd_task(int b, int total) {
  const int per = total >> 3;
  return (b & 7) * per + (b >> 3);
}

// XCD-aware order of the level and wide kernels (grid 8 ceil(groups / 8) G): node
// groups dealt round-robin to the eight XCDs, a contiguous share per XCD would
// give some XCDs the larger nodes of a level (jobs are sorted by size); the G
// RHS groups of a node run on one XCD one after another and share its matrix
// through that XCD's L2.
__device__ __forceinline__ int nd_task_rr(int b, int G) {
  const int x = b & 7, k = b >> 3;
  return (x + 8 * (k / G)) * G + k % G;
}
static unsigned nd_grid_rr(long long groups, int G) { return (unsigned)(8 * ((groups + 7) / 8) * G); }

// Dot products of the node kernels: acc -= (or +=) sum_j A[j * lda] y[j * KG],
// the matrix column loads issued eight at a time and one batch ahead of the
// FMAs that use them (so a row's loads are in flight together).
template <typename T, int KG, bool SUB>
__device__ __forceinline__ void nd_dot(cpx<T>& acc, const cpx<T>* __restrict__ A, long long lda,
                                       const cpx<T>* y, int n) {
  typedef cpx<T> C;
  constexpr int B = 8;
  C a[B], b[B];
  auto load = [&](C (&buf)[B], int j0) {
#pragma unroll
    for (int u = 0; u < B; ++u) buf[u] = A[(long long)min(j0 + u, n - 1) * lda];
  };
  auto use = [&](const C (&buf)[B], int j0) {
#pragma unroll
    for (int u = 0; u < B; ++u) {
      if (j0 + u >= n) break;
      const C m = buf[u], v = y[(j0 + u) * KG];
      if (SUB) {
        acc.re = fma(-m.re, v.re, acc.re);
        acc.re = fma(m.im, v.im, acc.re);
        acc.im = fma(-m.re, v.im, acc.im);
        acc.im = fma(-m.im, v.re, acc.im);
      } else {
        fma_acc(acc, m, v);
      }
    }
  };
  if (n <= 0) return;
  load(a, 0);
  for (int j0 = 0; j0 < n; j0 += 2 * B) {
    if (j0 + B < n) load(b, j0 + B);
    use(a, j0);
    if (j0 + B < n) {
      if (j0 + 2 * B < n) load(a, j0 + 2 * B);
      use(b, j0 + B);
    }
  }
}

// Lanes over rows: acc[q] -= (or +=) sum_{j in [c0, c1)} A[j * lda] y[j * KG + q]
// for all KG right-hand sides; the column loads (64 consecutive rows, one
// load per column) issued eight at a time, one batch ahead of their FMAs.
// The first batch (nd_rows_first, c1 > c0) can be issued early by the caller,
// so that it travels with the loads of the front gather.
template <typename T>
__device__ __forceinline__ void nd_rows_first(cpx<T> (&a)[8], const cpx<T>* __restrict__ A,
                                              long long lda, int c0, int c1) {
  const int n = c1 - c0;
#pragma unroll
  for (int u = 0; u < 8; ++u) a[u] = A[(long long)(c0 + min(u, n - 1)) * lda];
}

template <typename T, int KG, bool SUB>
__device__ __forceinline__ void nd_dot_rows_pre(cpx<T> (&acc)[KG], cpx<T> (&a)[8],
                                                const cpx<T>* __restrict__ A, long long lda,
                                                const cpx<T>* y, int c0, int c1) {
  typedef cpx<T> C;
  constexpr int B = 8;
  C b[B];
  const int n = c1 - c0;
  if (n <= 0) return;
  auto load = [&](C (&buf)[B], int j0) {
#pragma unroll
    for (int u = 0; u < B; ++u) buf[u] = A[(long long)(c0 + min(j0 + u, n - 1)) * lda];
  };
  auto use = [&](const C (&buf)[B], int j0) {
#pragma unroll
    for (int u = 0; u < B; ++u) {
      if (j0 + u >= n) break;
      const C m = buf[u];
      const C* yj = y + (c0 + j0 + u) * KG;
#pragma unroll
      for (int q = 0; q < KG; ++q) {
        const C v = yj[q];
        if (SUB) {
          acc[q].re = fma(-m.re, v.re, acc[q].re);
          acc[q].re = fma(m.im, v.im, acc[q].re);
          acc[q].im = fma(-m.re, v.im, acc[q].im);
          acc[q].im = fma(-m.im, v.re, acc[q].im);
        } else {
          fma_acc(acc[q], m, v);
        }
      }
    }
  };
  for (int j0 = 0; j0 < n; j0 += 2 * B) {
    if (j0 + B < n) load(b, j0 + B);
    use(a, j0);
    if (j0 + B < n) {
      if (j0 + 2 * B < n) load(a, j0 + 2 * B);
      use(b, j0 + B);
    }
  }
}

template <typename T, int KG, bool SUB>
__device__ __forceinline__ void nd_dot_rows(cpx<T> (&acc)[KG], const cpx<T>* __restrict__ A,
                                            long long lda, const cpx<T>* y, int c0, int c1) {
  if (c1 <= c0) return;
  cpx<T> a[8];
  nd_rows_first(a, A, lda, c0, c1);
  nd_dot_rows_pre<T, KG, SUB>(acc, a, A, lda, y, c0, c1);
}

// ---- complex64 on the FP32 matrix cores (v_mfma_f32_16x16x4f32): a wave
// computes a 64-row tile (four 16-row blocks) against KG = 8 JB right-hand
// sides.  Lane l holds A[16 rb + l % 16][k = l / 16] of a 4-column chunk and
// B[k][n = l % 16] with n = 2 q + (re/im): Re(A) against [Re y_q, Im y_q] and
// Im(A) against [-Im y_q, Re y_q] give [Re (A y)_q, Im (A y)_q].  Output
// acc[rb][jb][r] = row 16 rb + 4 (l / 16) + r, column n = l % 16 of block jb.
typedef float nd_mf4 __attribute__((ext_vector_type(4)));
// The LDS-front kernels (one node per workgroup, and the dense top) take the
// matrix cores from this RHS group up; with fewer right-hand sides per group
// the FP32 vector FMAs were measured faster there.
constexpr int ND_MFMA_KG = 8;

// The right-hand sides y sit in LDS at entry y_off of the dynamic LDS.  All
// loads are issued at clamped (valid) addresses and masked afterwards: a
// conditional load `c ? p[i] : 0` becomes a load from a selected address, a
// generic pointer, which compiles to flat loads; those wait for every global
// load in flight and break the pipelining of the matrix loads.
// CH 4-column chunks per batch of loads: 4 where few waves share a compute unit
// (loads in flight), 2 in the level kernels (registers: more waves).
template <int JB, int CH = 4>
__device__ __forceinline__ void nd_mfma_rows(nd_mf4 (&acc)[4][JB], const cpx<float>* __restrict__ A,
                                             long long lda, int nrows, long long y_off,
                                             int c0, int c1, int lane) {
  typedef cpx<float> C;
  extern __shared__ unsigned char smem_raw[];
  const C* y = reinterpret_cast<const C*>(smem_raw) + y_off;
  constexpr int KG = 8 * JB;
  const int lr = lane & 15, lk = lane >> 4, n = lane & 15, qn = n >> 1;
  const bool im = n & 1;
  const C zero = mk(0.0f, 0.0f);
  C a[CH][4], b[CH][4];
  auto load = [&](C (&buf)[CH][4], int j0) {
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int col = j0 + 4 * c + lk;
      const bool cv = col < c1;
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        const int row = 16 * rb + lr;
        const C v = A[(long long)min(col, c1 - 1) * lda + min(row, nrows - 1)];
        buf[c][rb] = (cv && row < nrows) ? v : zero;
      }
    }
  };
  auto use = [&](const C (&buf)[CH][4], int j0) {
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      if (j0 + 4 * c >= c1) break;            // wave-uniform
      const int col = j0 + 4 * c + lk;
      float bre[JB], bim[JB];
#pragma unroll
      for (int jb = 0; jb < JB; ++jb) {
        const C y0 = y[min(col, c1 - 1) * KG + jb * 8 + qn];
        const C yv = col < c1 ? y0 : zero;
        bre[jb] = im ? yv.im : yv.re;
        bim[jb] = im ? yv.re : -yv.im;
      }
#pragma unroll
      for (int jb = 0; jb < JB; ++jb)
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
          acc[rb][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(buf[c][rb].re, bre[jb], acc[rb][jb], 0, 0, 0);
          acc[rb][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(buf[c][rb].im, bim[jb], acc[rb][jb], 0, 0, 0);
        }
    }
  };
  if (c1 <= c0) return;
  constexpr int STEP = 4 * CH;
  load(a, c0);
  for (int j0 = c0; j0 < c1; j0 += 2 * STEP) {
    if (j0 + STEP < c1) load(b, j0 + STEP);
    use(a, j0);
    if (j0 + STEP < c1) {
      if (j0 + 2 * STEP < c1) load(a, j0 + 2 * STEP);
      use(b, j0 + STEP);
    }
  }
}

// The complex outputs of a wave's MFMA tile: the (re, im) halves of a value sit
// in neighbouring lanes; they meet through the wave's LDS staging area (64 x KG
// complex, at float st_off of the dynamic LDS) and come back as row `lane`,
// all KG right-hand sides.
template <int JB>
__device__ __forceinline__ void nd_mfma_out(const nd_mf4 (&acc)[4][JB], long long st_off, int lane,
                                            cpx<float> (&out)[8 * JB]) {
  constexpr int KG = 8 * JB;
  extern __shared__ unsigned char smem_raw[];
  float* st = reinterpret_cast<float*>(smem_raw) + st_off;
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int jb = 0; jb < JB; ++jb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rl = 16 * rb + 4 * (lane >> 4) + r;
        const int nn = jb * 16 + (lane & 15);
        st[((nn >> 1) * 64 + rl) * 2 + (nn & 1)] = acc[rb][jb][r];
      }
  nd_wave_sync();
#pragma unroll
  for (int q = 0; q < KG; ++q) out[q] = mk(st[(q * 64 + lane) * 2], st[(q * 64 + lane) * 2 + 1]);
}

// One level of the forward pass: one workgroup per (node, group of KG
// right-hand sides); front = (r on S, 0 on B) + children's updates (built by
// all waves, one front position per thread), f_S back into R, then the
// waves share the row passes of u_B = front_B - L f_S.
// With npw > 1 every wave of the workgroup runs a node of its own (the small
// nodes of the deep levels: fewer, fuller workgroups) and only waits for itself.
template <typename T, int KG>
__global__ __launch_bounds__(512) void k_nd_lvl_fwd(
    const NdLvlJob* __restrict__ jobs, int njobs, int G, int npw, int region, int TT, int CG,
    const int* __restrict__ cells, const int* __restrict__ umaps, const cpx<T>* __restrict__ fac,
    cpx<T>* __restrict__ rpool, cpx<T>* __restrict__ upool, long long pool_stride, int nrhs,
    int kmax) {
  typedef cpx<T> C;
  constexpr int RPP = 64 / KG;
  const int Lg = nd_task_rr(blockIdx.x, G);
  const int grp = Lg / G, g = Lg - (Lg / G) * G;
  int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63;
  int w = __builtin_amdgcn_readfirstlane(tid >> 6), W = nt >> 6;
  extern __shared__ unsigned char smem_raw[];
  C* fr = reinterpret_cast<C*>(smem_raw);
  int job = grp;
  if (npw > 1) {              // one node per wave: the wave is the workgroup
    job = grp * npw + w;
    fr += (long long)w * region;
    tid = lane;
    nt = 64;
    w = 0;
    W = 1;
  }
  if (job >= njobs) return;
  const NdLvlJob J = jobs[job];
  C* __restrict__ R = rpool + (long long)J.l * pool_stride + J.vbase;
  C* __restrict__ U = upool + J.ubase;
  const long long nloc = J.nloc;
  const C zero = mk((T)0, (T)0);
  const int q0 = g * KG, nq = min(KG, nrhs - q0);
  const int ns = J.ns, nbd = J.nbd, nf = ns + nbd;
  // lanes over rows (vector FMAs): wave w takes row tile w % TT and column
  // group w / TT; its first batch of matrix columns is issued before the
  // front gather, so that the two travel together
  constexpr bool VEC = !(std::is_same<T, float>::value && KG % 8 == 0 && KG >= ND_MFMA_KG);
  const int t = w % TT, cgi = w / TT;
  const int cw = (ns + CG - 1) / CG;
  const int c0 = min(ns, cgi * cw), c1 = min(ns, c0 + cw);
  // (complex128 keeps its registers for occupancy and loads after the gather)
  constexpr bool PRE = VEC && sizeof(T) == 4;
  C pre[8];
  if (PRE && npw == 1 && t * 64 < nbd && c1 > c0)
    nd_rows_first(pre, fac + J.fac + min(t * 64 + lane, nbd - 1), nbd, c0, c1);
  {
    const int* fc = cells + J.cell;
    const int* um = umaps + J.umap;
    // Lanes over positions: the separator's R entries (RHS q at q * nloc, so
    // neighbouring cells share cache lines), 0 on the boundary; every load at
    // a valid address and selected afterwards, so they go out together.
    for (int p = tid; p < nf; p += nt) {
      // (a boundary position reads its separator's last cell, selected out:
      // the boundary's own cells would pull extra cache lines)
      const C* Rc = R + (long long)q0 * nloc + fc[min(p, ns - 1)];
      C r[KG];
#pragma unroll
      for (int q = 0; q < KG; ++q) r[q] = Rc[(long long)min(q, nq - 1) * nloc];
#pragma unroll
      for (int q = 0; q < KG; ++q) fr[p * KG + q] = nd_sel(p < ns && q < nq, r[q], zero);
    }
    if (!J.leaf) {
      if (npw > 1) nd_wave_sync();
      else __syncthreads();
      // Lanes over (position, RHS) pairs, RHS fastest: a child's update entry
      // holds the KG right-hand sides of a position contiguously, read whole
      // by KG neighbouring lanes; the sum goes back to R on the separator.
      // Four pairs per thread per pass, every load at a valid address (an
      // absent child reads the position's R entry) so that all go out together.
      constexpr int PP = sizeof(T) == 4 ? 4 : 2;
      const int cell0 = fc[0];
      for (int e0 = tid; e0 < nf * KG; e0 += PP * nt) {
        int i0[PP], i1[PP], cl[PP];
#pragma unroll
        for (int k = 0; k < PP; ++k) {
          const int e = min(e0 + k * nt, nf * KG - 1), p = e / KG;
          i0[k] = um[2 * p];
          i1[k] = um[2 * p + 1];
          cl[k] = fc[p];
        }
        C a[PP], b[PP];
#pragma unroll
        for (int k = 0; k < PP; ++k) {
          const int e = min(e0 + k * nt, nf * KG - 1), q = e - (e / KG) * KG;
          // an absent child reads the other child's entry, or with neither
          // the separator's first cell (one shared line): no extra lines
          const C* rq = R + (long long)(q0 + min(q, nq - 1)) * nloc + cell0;
          const C* u0 = i0[k] >= 0 ? U + (long long)i0[k] * kmax + q0 + q : nullptr;
          const C* u1 = i1[k] >= 0 ? U + (long long)i1[k] * kmax + q0 + q : nullptr;
          a[k] = nd_gload(u0 ? u0 : u1 ? u1 : rq);
          b[k] = nd_gload(u1 ? u1 : u0 ? u0 : rq);
        }
#pragma unroll
        for (int k = 0; k < PP; ++k) {
          const int e = e0 + k * nt;
          const int p = e / KG, q = e - (e / KG) * KG;
          if (e < nf * KG && q < nq && (i0[k] >= 0 || i1[k] >= 0)) {
            C v = fr[e];
            v = i0[k] >= 0 ? v + a[k] : v;
            v = i1[k] >= 0 ? v + b[k] : v;
            fr[e] = v;
            if (p < ns) R[(long long)(q0 + q) * nloc + cl[k]] = v;
          }
        }
      }
    }
  }
  if (npw > 1) nd_wave_sync();
  else __syncthreads();
  const C* __restrict__ L = fac + J.fac;
  if (npw > 1) {
    // (row, right-hand side) lanes: 64 / KG rows per pass
    const int qq = lane % KG, rr = lane / KG;
    for (int i0 = 0; i0 < nbd; i0 += RPP) {
      const int i = i0 + rr;
      if (i >= nbd) continue;
      C acc = fr[(ns + i) * KG + qq];
      nd_dot<T, KG, true>(acc, L + i, nbd, fr + qq, ns);
      if (qq < nq) U[(J.upd + i) * kmax + q0 + qq] = acc;
    }
    return;
  }
  (void)W;
  const int i = t * 64 + lane;
  const bool live = i < nbd;
  if constexpr (std::is_same<T, float>::value && KG % 8 == 0 && KG >= ND_MFMA_KG) {
    constexpr int JB = KG / 8;
    nd_mf4 macc[4][JB];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int jb = 0; jb < JB; ++jb) macc[rb][jb] = nd_mf4{0.f, 0.f, 0.f, 0.f};
    if (t * 64 < nbd) nd_mfma_rows<JB, 2>(macc, L + t * 64, nbd, nbd - t * 64, 0, c0, c1, lane);
    float* pf = reinterpret_cast<float*>(smem_raw) + 2LL * region;
    if (CG > 1) {
      if (cgi > 0) {
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
          for (int jb = 0; jb < JB; ++jb)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              pf[((((cgi - 1) * TT + t) * 4 + rb) * JB * 4 + jb * 4 + r) * 64 + lane] = macc[rb][jb][r];
      }
      __syncthreads();
      if (cgi > 0) return;
      for (int o = 1; o < CG; ++o)
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
          for (int jb = 0; jb < JB; ++jb)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              macc[rb][jb][r] += pf[((((o - 1) * TT + t) * 4 + rb) * JB * 4 + jb * 4 + r) * 64 + lane];
    }
    C out[KG];
    nd_mfma_out<JB>(macc, 2LL * region + (long long)t * 64 * KG * 2, lane, out);
    if (live) {
#pragma unroll
      for (int q = 0; q < KG; ++q)
        if (q < nq) U[(J.upd + i) * kmax + q0 + q] = fr[(ns + i) * KG + q] - out[q];
    }
    return;
  }
  C acc[KG];
  const int ri = live ? ns + i : 0;    // LDS read at a valid position, selected after
#pragma unroll
  for (int q = 0; q < KG; ++q) {
    const C f = fr[ri * KG + q];
    acc[q] = nd_sel(cgi == 0 && live, f, zero);
  }
  if (live) {
    if constexpr (PRE) nd_dot_rows_pre<T, KG, true>(acc, pre, L + i, nbd, fr, c0, c1);
    else nd_dot_rows<T, KG, true>(acc, L + i, nbd, fr, c0, c1);
  }
  C* part = fr + region;
  if (CG > 1) {
    if (cgi > 0) {
#pragma unroll
      for (int q = 0; q < KG; ++q) part[(((cgi - 1) * TT + t) * KG + q) * 64 + lane] = acc[q];
    }
    __syncthreads();
    if (cgi > 0) return;
    for (int o = 1; o < CG; ++o)
#pragma unroll
      for (int q = 0; q < KG; ++q) acc[q] = acc[q] + part[(((o - 1) * TT + t) * KG + q) * 64 + lane];
  }
  if (live) {
#pragma unroll
    for (int q = 0; q < KG; ++q)
      if (q < nq) U[(J.upd + i) * kmax + q0 + q] = acc[q];
  }
}

// One level of the backward pass: x_S = K [f_S; -x_B] with K = [P | L^T]
// (ns x nf), f_S from R, x_B from X (ancestors, or the dense top).  For a
// leaf L^T x_B = P A_SB x_B with A_SB the operator's face couplings of the
// box, so the front is v = f_S - A_SB x_B (ns entries) and x_S = P v.
template <typename T, int KG>
__global__ __launch_bounds__(512) void k_nd_lvl_bwd(
    const NdLvlJob* __restrict__ jobs, int njobs, int G, int npw, int region, int TT, int CG,
    const int* __restrict__ cells, const cpx<T>* __restrict__ fac, const cpx<T>* __restrict__ rpool,
    cpx<T>* __restrict__ xpool, long long pool_stride, int nrhs, const cpx<T>* __restrict__ cx,
    const cpx<T>* __restrict__ cy, const cpx<T>* __restrict__ cz) {
  typedef cpx<T> C;
  constexpr int RPP = 64 / KG;
  const int Lg = nd_task_rr(blockIdx.x, G);
  const int grp = Lg / G, g = Lg - (Lg / G) * G;
  int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63;
  int w = __builtin_amdgcn_readfirstlane(tid >> 6), W = nt >> 6;
  extern __shared__ unsigned char smem_raw[];
  C* v = reinterpret_cast<C*>(smem_raw);
  int job = grp;
  if (npw > 1) {
    job = grp * npw + w;
    v += (long long)w * region;
    tid = lane;
    nt = 64;
    w = 0;
    W = 1;
  }
  if (job >= njobs) return;
  const NdLvlJob J = jobs[job];
  const C* __restrict__ R = rpool + (long long)J.l * pool_stride + J.vbase;
  C* __restrict__ X = xpool + (long long)J.l * pool_stride + J.vbase;
  const long long nloc = J.nloc;
  const C zero = mk((T)0, (T)0);
  const int q0 = g * KG, nq = min(KG, nrhs - q0);
  const int ns = J.ns, nbd = J.nbd, nf = ns + nbd;
  const int* fc = cells + J.cell;
  const int ncol = J.leaf ? ns : nf;
  constexpr bool VEC = !(std::is_same<T, float>::value && KG % 8 == 0 && KG >= ND_MFMA_KG);
  const int t = w % TT, cgi = w / TT;
  const int cw = (ncol + CG - 1) / CG;
  const int c0 = min(ncol, cgi * cw), c1 = min(ncol, c0 + cw);
  constexpr bool PRE = VEC && sizeof(T) == 4;
  C pre[8];
  if (PRE && npw == 1 && t * 64 < ns && c1 > c0)
    nd_rows_first(pre, fac + J.fac + (long long)nbd * ns + min(t * 64 + lane, ns - 1), ns, c0, c1);
  for (int p = tid; p < ncol; p += nt) {
    const bool own = p < ns;
    const int cell = fc[p];
    // loads at valid addresses, selected afterwards (see the forward gather)
    const C* xs = (own ? R : X) + (long long)q0 * nloc + cell;
    C x[KG];
#pragma unroll
    for (int q = 0; q < KG; ++q) x[q] = nd_gload(xs + (long long)min(q, nq - 1) * nloc);
#pragma unroll
    for (int q = 0; q < KG; ++q) x[q] = nd_sel(q < nq, nd_sel(own, x[q], -x[q]), zero);
    if (J.leaf) {
      // the box's faces, in a fixed order: -x, +x, -y, +y, -z, +z (one at a
      // time: the kernel's registers are set by its largest live set)
      const int nx = J.dims[0], ny = J.dims[1], nz = J.dims[2], nxy = nx * ny;
      const int px = cell % nx, py = (cell / nx) % ny, pz = cell / nxy;
      const int na = nz > 1 ? 3 : 2;
      // complex128: one face at a time (registers); complex64: both faces of
      // an axis, their loads going out together
      constexpr bool PAIR = sizeof(T) == 4;
#pragma unroll 1
      for (int a = 0; a < na; ++a) {
        const int pa = a == 0 ? px : a == 1 ? py : pz;
        const int ea = a == 0 ? nx : a == 1 ? ny : nz;
        const int sa = a == 0 ? 1 : a == 1 ? nx : nxy;
        const int la = a == 0 ? J.lo[0] : a == 1 ? J.lo[1] : J.lo[2];
        const int ha = a == 0 ? J.hi[0] : a == 1 ? J.hi[1] : J.hi[2];
        const C* __restrict__ ca = (a == 0 ? cx : a == 1 ? cy : cz) + J.coef;
        const bool f0 = pa == la && la > 0, f1 = pa == ha - 1 && ha < ea;
        const int n0 = f0 ? cell - sa : cell, n1 = f1 ? cell + sa : cell;
        const C c0v = nd_gload(ca + n0), c1v = nd_gload(ca + cell);
        // off the face: the cell's own R entries (already read above), not
        // X's, so that no extra cache lines are pulled
        const C* rs = R + (long long)q0 * nloc + cell;
        const C* x0 = f0 ? X + (long long)q0 * nloc + n0 : rs;
        const C* x1 = f1 ? X + (long long)q0 * nloc + n1 : rs;
        if constexpr (PAIR) {
          C y0[KG], y1[KG];
#pragma unroll
          for (int q = 0; q < KG; ++q) {
            y0[q] = nd_gload(x0 + (long long)min(q, nq - 1) * nloc);
            y1[q] = nd_gload(x1 + (long long)min(q, nq - 1) * nloc);
          }
#pragma unroll
          for (int q = 0; q < KG; ++q) {
            x[q] = f0 && q < nq ? x[q] - c0v * y0[q] : x[q];
            x[q] = f1 && q < nq ? x[q] - c1v * y1[q] : x[q];
          }
        } else {
#pragma unroll 1
          for (int side = 0; side < 2; ++side) {
            const C* xs_ = side == 0 ? x0 : x1;
            const C cv = side == 0 ? c0v : c1v;
            const bool f = side == 0 ? f0 : f1;
            C y[KG];
#pragma unroll
            for (int q = 0; q < KG; ++q) y[q] = nd_gload(xs_ + (long long)min(q, nq - 1) * nloc);
#pragma unroll
            for (int q = 0; q < KG; ++q) x[q] = f && q < nq ? x[q] - cv * y[q] : x[q];
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < KG; ++q) v[p * KG + q] = x[q];
  }
  if (npw > 1) nd_wave_sync();
  else __syncthreads();
  const C* __restrict__ K = fac + J.fac + (long long)nbd * ns;
  if (npw > 1) {
    const int qq = lane % KG, rr = lane / KG;
    for (int i0 = 0; i0 < ns; i0 += RPP) {
      const int i = i0 + rr;
      if (i >= ns) continue;
      C acc = zero;
      nd_dot<T, KG, false>(acc, K + i, ns, v + qq, ncol);
      if (qq < nq) X[(long long)(q0 + qq) * nloc + fc[i]] = acc;
    }
    return;
  }
  (void)W;
  const int i = t * 64 + lane;
  const bool live = i < ns;
  if constexpr (std::is_same<T, float>::value && KG % 8 == 0 && KG >= ND_MFMA_KG) {
    constexpr int JB = KG / 8;
    nd_mf4 macc[4][JB];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int jb = 0; jb < JB; ++jb) macc[rb][jb] = nd_mf4{0.f, 0.f, 0.f, 0.f};
    if (t * 64 < ns) nd_mfma_rows<JB, 2>(macc, K + t * 64, ns, ns - t * 64, 0, c0, c1, lane);
    float* pf = reinterpret_cast<float*>(smem_raw) + 2LL * region;
    if (CG > 1) {
      if (cgi > 0) {
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
          for (int jb = 0; jb < JB; ++jb)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              pf[((((cgi - 1) * TT + t) * 4 + rb) * JB * 4 + jb * 4 + r) * 64 + lane] = macc[rb][jb][r];
      }
      __syncthreads();
      if (cgi > 0) return;
      for (int o = 1; o < CG; ++o)
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
          for (int jb = 0; jb < JB; ++jb)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              macc[rb][jb][r] += pf[((((o - 1) * TT + t) * 4 + rb) * JB * 4 + jb * 4 + r) * 64 + lane];
    }
    C out[KG];
    nd_mfma_out<JB>(macc, 2LL * region + (long long)t * 64 * KG * 2, lane, out);
    if (live) {
      const int cell = fc[i];
#pragma unroll
      for (int q = 0; q < KG; ++q)
        if (q < nq) X[(long long)(q0 + q) * nloc + cell] = out[q];
    }
    return;
  }
  C acc[KG];
#pragma unroll
  for (int q = 0; q < KG; ++q) acc[q] = zero;
  if (live) {
    if constexpr (PRE) nd_dot_rows_pre<T, KG, false>(acc, pre, K + i, ns, v, c0, c1);
    else nd_dot_rows<T, KG, false>(acc, K + i, ns, v, c0, c1);
  }
  C* part = v + region;
  if (CG > 1) {
    if (cgi > 0) {
#pragma unroll
      for (int q = 0; q < KG; ++q) part[(((cgi - 1) * TT + t) * KG + q) * 64 + lane] = acc[q];
    }
    __syncthreads();
    if (cgi > 0) return;
    for (int o = 1; o < CG; ++o)
#pragma unroll
      for (int q = 0; q < KG; ++q) acc[q] = acc[q] + part[(((o - 1) * TT + t) * KG + q) * 64 + lane];
  }
  if (live) {
    const int cell = fc[i];
#pragma unroll
    for (int q = 0; q < KG; ++q)
      if (q < nq) X[(long long)(q0 + q) * nloc + cell] = acc[q];
  }
}

// Dense top: rows [64 tile, 64 tile + 64) of x_top = P_top g, g = r_top plus
// the subtree roots' updates; the waves split the columns (each gathers its
// own columns of g into LDS, one column per lane) and meet in LDS for the
// sum, in wave order.
template <typename T, int KG>
__global__ __launch_bounds__(64 * ND_TW) void k_nd_top(
    const NdTopJob* __restrict__ jobs, int njobs, int G, int ntiles, const int* __restrict__ cells,
    const int* __restrict__ usrc, const cpx<T>* __restrict__ fac, const cpx<T>* __restrict__ rpool,
    const cpx<T>* __restrict__ upool, cpx<T>* __restrict__ xpool, long long pool_stride, int nrhs,
    int kmax, int cwmax) {
  typedef cpx<T> C;
  const int Lg = nd_task(blockIdx.x, gridDim.x);
  const int per = G * ntiles;
  const int job = Lg / per;
  if (job >= njobs) return;
  const int rem = Lg - job * per;
  const int g = rem / ntiles, tile = rem - (rem / ntiles) * ntiles;
  const NdTopJob J = jobs[job];
  const int ntop = J.ntop;
  if (tile * 64 >= ntop) return;
  const C* __restrict__ R = rpool + (long long)J.l * pool_stride + J.vbase;
  C* __restrict__ X = xpool + (long long)J.l * pool_stride + J.vbase;
  const C* __restrict__ U = upool + J.ubase;
  const C* __restrict__ P = fac + J.fac;
  const int* tc = cells + J.cell;
  const int* us = usrc + J.usrc;
  const long long nloc = J.nloc;
  extern __shared__ unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const C zero = mk((T)0, (T)0);
  const int q0 = g * KG, nq = min(KG, nrhs - q0);
  const int cw = (ntop + ND_TW - 1) / ND_TW;
  const int c0 = min(ntop, w * cw), c1 = min(ntop, c0 + cw);
  C* gl = lds + (long long)w * cwmax * KG;
  // lanes over columns: r_top (RHS q at q * nloc: neighbouring cells share
  // cache lines), loads at valid addresses and selected afterwards
  for (int j = c0 + lane; j < c1; j += 64) {
    const C* Rc = R + (long long)q0 * nloc + tc[j];
    C v[KG];
#pragma unroll
    for (int q = 0; q < KG; ++q) v[q] = Rc[(long long)min(q, nq - 1) * nloc];
#pragma unroll
    for (int q = 0; q < KG; ++q) gl[(j - c0) * KG + q] = nd_sel(q < nq, v[q], zero);
  }
  nd_wave_sync();
  // lanes over (column, RHS) pairs, RHS fastest: a subtree root's update entry
  // holds the KG right-hand sides contiguously, read whole by KG lanes
  // (two pairs per lane per pass in complex64, one in complex128 for
  // registers; every load at a valid address, an absent update reading the
  // column's R entry, so that all go out together)
  constexpr int HH = sizeof(T) == 4 ? 2 : 1;
  const int ne = (c1 - c0) * KG, d2 = J.dim2;
  for (int e0 = lane; e0 < ne; e0 += 64 * HH) {
    int o[HH][6], cl[HH];
#pragma unroll
    for (int h = 0; h < HH; ++h) {
      const int e = min(e0 + 64 * h, ne - 1), j = c0 + e / KG;
      cl[h] = tc[j];
#pragma unroll
      for (int k = 0; k < 6; ++k) o[h][k] = k < d2 ? us[j * d2 + min(k, d2 - 1)] : -1;
    }
    C u[HH][6];
#pragma unroll
    for (int h = 0; h < HH; ++h) {
      const int e = min(e0 + 64 * h, ne - 1), q = e - (e / KG) * KG;
      const C* rq = R + (long long)(q0 + min(q, nq - 1)) * nloc + cl[h];
#pragma unroll
      for (int k = 0; k < 6; ++k)
        if (k < d2) u[h][k] = nd_gload(o[h][k] >= 0 ? U + (long long)o[h][k] * kmax + q0 + q : rq);
    }
#pragma unroll
    for (int h = 0; h < HH; ++h) {
      const int e = e0 + 64 * h;
      const int q = e - (e / KG) * KG;
      if (e < ne && q < nq) {
        C v = gl[e];
#pragma unroll
        for (int k = 0; k < 6; ++k)
          if (k < d2) v = o[h][k] >= 0 ? v + u[h][k] : v;
        gl[e] = v;
      }
    }
  }
  nd_wave_sync();
  const int i = tile * 64 + lane;
  if constexpr (std::is_same<T, float>::value && KG % 8 == 0) {
    constexpr int JB = KG / 8;
    nd_mf4 macc[4][JB];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int jb = 0; jb < JB; ++jb) macc[rb][jb] = nd_mf4{0.f, 0.f, 0.f, 0.f};
    // gl holds this wave's columns c0..c1 from its start: shift y so that y[col] = gl[col - c0]
    nd_mfma_rows<JB>(macc, P + tile * 64 + (long long)c0 * ntop, ntop, ntop - tile * 64,
                     (long long)w * cwmax * KG, 0, c1 - c0, lane);
    float* pf = reinterpret_cast<float*>(smem_raw) + 2LL * ND_TW * cwmax * KG;
    if (w > 0) {
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int jb = 0; jb < JB; ++jb)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            pf[(((w - 1) * 4 + rb) * JB * 4 + jb * 4 + r) * 64 + lane] = macc[rb][jb][r];
    }
    __syncthreads();
    if (w > 0) return;
    for (int o = 1; o < ND_TW; ++o)
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int jb = 0; jb < JB; ++jb)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            macc[rb][jb][r] += pf[(((o - 1) * 4 + rb) * JB * 4 + jb * 4 + r) * 64 + lane];
    C out[KG];
    nd_mfma_out<JB>(macc, 2LL * ND_TW * cwmax * KG, lane, out);
    if (i < ntop) {
      const int cell = tc[i];
#pragma unroll
      for (int q = 0; q < KG; ++q)
        if (q < nq) X[(long long)(q0 + q) * nloc + cell] = out[q];
    }
    return;
  }
  C acc[KG];
#pragma unroll
  for (int q = 0; q < KG; ++q) acc[q] = zero;
  if (i < ntop) {
    // column loads eight at a time, one batch ahead of the FMAs that use them
    constexpr int B = 8;
    C a[B], b[B];
    const C* __restrict__ Pi = P + i;
    const int n = c1 - c0;
    auto load = [&](C (&buf)[B], int j0) {
#pragma unroll
      for (int u = 0; u < B; ++u) buf[u] = Pi[(long long)(c0 + min(j0 + u, n - 1)) * ntop];
    };
    auto use = [&](const C (&buf)[B], int j0) {
#pragma unroll
      for (int u = 0; u < B; ++u) {
        if (j0 + u >= n) break;
#pragma unroll
        for (int q = 0; q < KG; ++q) fma_acc(acc[q], buf[u], gl[(j0 + u) * KG + q]);
      }
    };
    if (n > 0) {
      load(a, 0);
      for (int j0 = 0; j0 < n; j0 += 2 * B) {
        if (j0 + B < n) load(b, j0 + B);
        use(a, j0);
        if (j0 + B < n) {
          if (j0 + 2 * B < n) load(a, j0 + 2 * B);
          use(b, j0 + B);
        }
      }
    }
  }
  C* part = lds + (long long)ND_TW * cwmax * KG;
  if (w > 0) {
#pragma unroll
    for (int q = 0; q < KG; ++q) part[((w - 1) * KG + q) * 64 + lane] = acc[q];
  }
  __syncthreads();
  if (w == 0 && i < ntop) {
    for (int o = 1; o < ND_TW; ++o)
#pragma unroll
      for (int q = 0; q < KG; ++q) acc[q] = acc[q] + part[((o - 1) * KG + q) * 64 + lane];
    const int cell = tc[i];
#pragma unroll
    for (int q = 0; q < KG; ++q)
      if (q < nq) X[(long long)(q0 + q) * nloc + cell] = acc[q];
  }
}

// ---- wide mode: nodes whose front is too large for the LDS (or with more
// than 512 rows) run their products as tiled matrix products over every
// right-hand side of a group of KG (up to 32) at once, so that each factor
// entry is read once per solve.  A workgroup of eight waves takes ND_WROWS =
// 128 rows of one node: ND_WRT = 2 64-row tiles x ND_WCQ = 4 column quarters
// (more workgroups than 256-row tiles would give, so the few large nodes of a
// launch still reach every compute unit; two waves per SIMD).  Each quarter
// streams its columns through LDS in chunks of ND_WCK (the vector entries of
// the chunk for all KG right-hand sides, double-buffered), and the quarters
// meet in LDS: quarters 1..3 add their partial sums to quarter 0's in that
// order, so every row sums its columns the same way whatever else the launch
// holds.  The forward pass first forms f_S (k_nd_form)
// and ends with u_B = (children's updates on B) - L f_S; the backward pass is
// x_S = K [f_S; -x_B].  Tiles are {job, first row} entries of a table.
constexpr int ND_WCK = 64;
constexpr int ND_WRT = 2, ND_WCQ = 4;   // row tiles x column quarters of a workgroup

// f_S = r_S + children's updates on S, into R: one thread per (position, RHS)
template <typename T>
__global__ __launch_bounds__(256) void k_nd_form(const NdLvlJob* __restrict__ jobs,
                                                 const int2* __restrict__ tiles, int ntiles,
                                                 const int* __restrict__ cells,
                                                 const int* __restrict__ umaps,
                                                 cpx<T>* __restrict__ rpool,
                                                 const cpx<T>* __restrict__ upool,
                                                 long long pool_stride, int nrhs, int kmax) {
  // tiles in launch order: consecutive workgroups go to different XCDs, so the
  // tiles of the large and the small nodes spread over all of them
  const int tix = blockIdx.x;
  if (tix >= ntiles) return;
  const int2 t = tiles[tix];
  const NdLvlJob J = jobs[t.x];
  cpx<T>* __restrict__ R = rpool + (long long)J.l * pool_stride + J.vbase;
  const cpx<T>* __restrict__ U = upool + J.ubase;
  const int* fc = cells + J.cell;
  const int* um = umaps + J.umap;
  const int span = min(256, J.ns - t.y);
  for (int e = threadIdx.x; e < span * nrhs; e += 256) {
    const int p = t.y + e / nrhs, q = e - (e / nrhs) * nrhs;
    const int i0 = um[2 * p], i1 = um[2 * p + 1];
    cpx<T>* r = R + (long long)q * J.nloc + fc[p];
    cpx<T> v = *r;
    if (i0 >= 0) v = v + U[(long long)i0 * kmax + q];
    if (i1 >= 0) v = v + U[(long long)i1 * kmax + q];
    *r = v;
  }
}

// Stage the vector entries of columns [c0, c0 + n) for right-hand sides
// [q0, q0 + nq) into buf[c * KG + q] (zero beyond n or nq), by the threads of
// one column quarter: column c < ns from R (f_S), column c >= ns from -X
// (boundary, backward pass only).
template <typename T, int KG>
__device__ __forceinline__ void nd_wide_stage(cpx<T>* buf, const int* fc, int ns, int c0, int n,
                                              int q0, int nq, const cpx<T>* R, const cpx<T>* X,
                                              long long nloc) {
  constexpr int GT = ND_WRT * 64;
  for (int e = threadIdx.x % GT; e < ND_WCK * KG; e += GT) {
    const int c = e / KG, q = e - (e / KG) * KG;
    cpx<T> v = mk((T)0, (T)0);
    if (c < n && q < nq) {
      const int col = c0 + c;
      const long long o = (long long)(q0 + q) * nloc + fc[col];
      v = col < ns ? R[o] : -X[o];
    }
    buf[e] = v;
  }
}

// The same staging in two halves: load issues the loads of this thread's
// entries into registers (at clamped addresses, masked afterwards), store
// writes them to LDS -- so a chunk's loads are in flight while the previous
// chunk is multiplied.
template <typename T, int KG>
struct NdWideStager {
  static constexpr int GT = ND_WRT * 64;            // threads of one column quarter
  static constexpr int PER = ND_WCK * KG / GT;
  cpx<T> v[PER];
  __device__ __forceinline__ void load(const int* fc, int ns, int c0, int n, int q0, int nq,
                                       const cpx<T>* R, const cpx<T>* X, long long nloc) {
    const int tid = threadIdx.x % GT;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + GT * u, c = e / KG, q = e - (e / KG) * KG;
      const int col = c0 + min(c, n - 1);
      const bool own = col < ns;
      const cpx<T>* src = own ? R : X;
      const cpx<T> x = src[(long long)(q0 + min(q, nq - 1)) * nloc + fc[col]];
      const cpx<T> y = own ? x : -x;
      v[u] = (c < n && q < nq) ? y : mk((T)0, (T)0);
    }
  }
  __device__ __forceinline__ void store(cpx<T>* buf) const {
    const int tid = threadIdx.x % GT;
#pragma unroll
    for (int u = 0; u < PER; ++u) buf[tid + GT * u] = v[u];
  }
};

// out (row `lane` of this wave's 64-row tile) = A[tile rows, 0:ncol] y, A
// column-major (lda, already offset to the tile), the columns of this wave's
// quarter staged chunk by chunk; complex64 on the FP32 matrix cores,
// complex128 with vector FMAs.  out is valid in quarter 0's waves (w <
// ND_WRT) only.  LDS (entries from the base): staging [0, ND_WCQ 2 ND_WCK KG)
// (quarter h at 2 h ND_WCK KG), reused for the other quarters' partial sums;
// the MFMA output staging after it (ND_WRT x 64 x KG).
template <typename T, int KG>
__device__ __forceinline__ void nd_wide_product(const cpx<T>* __restrict__ A, long long lda,
                                                int nrows_tile, int ncol, int ns, const int* fc,
                                                int q0, int nq, const cpx<T>* R, const cpx<T>* X,
                                                long long nloc, cpx<T>* lds, cpx<T> (&out)[KG]) {
  typedef cpx<T> C;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int h = w / ND_WRT, t = w % ND_WRT;
  const int part = ((ncol + ND_WCQ - 1) / ND_WCQ + 3) / 4 * 4;   // a multiple of the MFMA column step
  const int cb = min(ncol, h * part), ce = min(ncol, cb + part);
  const int nown = (ce - cb + ND_WCK - 1) / ND_WCK;
  const int nch = (min(ncol, part) + ND_WCK - 1) / ND_WCK;   // quarter 0's chunks (>= any other's)
  const long long hb = (long long)h * 2 * ND_WCK * KG;        // this quarter's staging
  constexpr long long STG = (long long)ND_WCQ * 2 * ND_WCK * KG;
  C* buf0 = lds + hb;
  C* buf1 = buf0 + ND_WCK * KG;
  if (nown > 0) nd_wide_stage<T, KG>(buf0, fc, ns, cb, min(ND_WCK, ce - cb), q0, nq, R, X, nloc);
  __syncthreads();
  if constexpr (std::is_same<T, float>::value && KG % 8 == 0) {
    constexpr int JB = KG / 8;
    nd_mf4 macc[4][JB];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int jb = 0; jb < JB; ++jb) macc[rb][jb] = nd_mf4{0.f, 0.f, 0.f, 0.f};
    // lds is the base of the dynamic LDS: this quarter's buffer k & 1 starts at
    // entry hb + (k & 1) ND_WCK KG.  The next chunk's vector loads are issued
    // before this chunk's products and written to LDS after them.
    NdWideStager<T, KG> stg;
    for (int k = 0; k < nch; ++k) {
      C* nxt = (k & 1) ? buf0 : buf1;
      const int c0 = cb + k * ND_WCK, cn = min(ND_WCK, ce - c0);
      if (k + 1 < nown) stg.load(fc, ns, c0 + ND_WCK, min(ND_WCK, ce - c0 - ND_WCK), q0, nq, R, X, nloc);
      if (k < nown && nrows_tile > 0)
        nd_mfma_rows<JB>(macc, A + (long long)c0 * lda, lda, nrows_tile,
                         hb + ((k & 1) ? ND_WCK * KG : 0), 0, cn, lane);
      if (k + 1 < nown) stg.store(nxt);
      __syncthreads();
    }
    // the staging area is free: the other quarters' partial sums go there
    float* pf = reinterpret_cast<float*>(lds);
    constexpr int PW = 16 * JB * 64;                          // floats per wave
    if (h > 0) {
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int jb = 0; jb < JB; ++jb)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            pf[((h - 1) * ND_WRT + t) * PW + ((rb * JB + jb) * 4 + r) * 64 + lane] = macc[rb][jb][r];
    }
    __syncthreads();
    if (h > 0) return;
    for (int o = 1; o < ND_WCQ; ++o)
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int jb = 0; jb < JB; ++jb)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            macc[rb][jb][r] += pf[((o - 1) * ND_WRT + t) * PW + ((rb * JB + jb) * 4 + r) * 64 + lane];
    nd_mfma_out<JB>(macc, 2 * STG + (long long)t * 64 * KG * 2, lane, out);
  } else {
#pragma unroll
    for (int q = 0; q < KG; ++q) out[q] = mk((T)0, (T)0);
    for (int k = 0; k < nch; ++k) {
      C* cur = (k & 1) ? buf1 : buf0;
      C* nxt = (k & 1) ? buf0 : buf1;
      const int c0 = cb + k * ND_WCK, cn = min(ND_WCK, ce - c0);
      if (k + 1 < nown)
        nd_wide_stage<T, KG>(nxt, fc, ns, c0 + ND_WCK, min(ND_WCK, ce - c0 - ND_WCK), q0, nq, R,
                             X, nloc);
      if (k < nown && lane < nrows_tile)
        nd_dot_rows<T, KG, false>(out, A + (long long)c0 * lda + lane, lda, cur, 0, cn);
      __syncthreads();
    }
    C* part_s = lds;
    if (h > 0) {
#pragma unroll
      for (int q = 0; q < KG; ++q) part_s[(((h - 1) * ND_WRT + t) * KG + q) * 64 + lane] = out[q];
    }
    __syncthreads();
    if (h > 0) return;
    for (int o = 1; o < ND_WCQ; ++o)
#pragma unroll
      for (int q = 0; q < KG; ++q) out[q] = out[q] + part_s[(((o - 1) * ND_WRT + t) * KG + q) * 64 + lane];
  }
}

template <typename T>
constexpr size_t nd_wide_lds_entries(int kg) {
  // the quarters' staging chunks (reused for the partial sums of quarters 1..3),
  // then the MFMA output staging (ND_WRT waves x 64 x KG)
  return (size_t)std::max(ND_WCQ * 2 * ND_WCK * kg, (ND_WCQ - 1) * ND_WRT * 64 * kg) +
         (size_t)ND_WRT * 64 * kg;
}

// u_B = (children's updates on B) - L f_S for rows [t.y, t.y + ND_WROWS) of node t.x
template <typename T, int KG>
__global__ __launch_bounds__(512) void k_nd_wide_fwd(
    const NdLvlJob* __restrict__ jobs, const int2* __restrict__ tiles, int ntiles, int G,
    const int* __restrict__ cells, const int* __restrict__ umaps, const cpx<T>* __restrict__ fac,
    const cpx<T>* __restrict__ rpool, cpx<T>* __restrict__ upool, long long pool_stride,
    int nrhs, int kmax) {
  typedef cpx<T> C;
  // tiles dealt round-robin to the XCDs (the tiles of large and small nodes
  // spread over all of them), a tile's RHS groups on one XCD
  const int Lg = nd_task_rr(blockIdx.x, G);
  const int tix = Lg / G, g = Lg - (Lg / G) * G;
  if (tix >= ntiles) return;
  const int2 t = tiles[tix];
  const NdLvlJob J = jobs[t.x];
  const C* __restrict__ R = rpool + (long long)J.l * pool_stride + J.vbase;
  C* __restrict__ U = upool + J.ubase;
  const int ns = J.ns, nbd = J.nbd;
  const int q0 = g * KG, nq = min(KG, nrhs - q0);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r0 = t.y + 64 * (w % ND_WRT);
  extern __shared__ unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  C out[KG];
  nd_wide_product<T, KG>(fac + J.fac + r0, nbd, max(0, min(64, nbd - r0)), ns, ns, cells + J.cell,
                         q0, nq, R, R, J.nloc, lds, out);
  const int i = r0 + lane;
  if (w < ND_WRT && i < nbd) {            // column quarter 0 holds the sums
    const int p = ns + i;
    const int i0 = umaps[J.umap + 2 * p], i1 = umaps[J.umap + 2 * p + 1];
#pragma unroll
    for (int q = 0; q < KG; ++q) {
      if (q < nq) {
        C v = mk((T)0, (T)0);
        if (i0 >= 0) v = v + U[(long long)i0 * kmax + q0 + q];
        if (i1 >= 0) v = v + U[(long long)i1 * kmax + q0 + q];
        U[(J.upd + i) * kmax + q0 + q] = v - out[q];
      }
    }
  }
}

// x_S = K [f_S; -x_B] for rows [t.y, t.y + ND_WROWS) of node t.x
template <typename T, int KG>
__global__ __launch_bounds__(512) void k_nd_wide_bwd(
    const NdLvlJob* __restrict__ jobs, const int2* __restrict__ tiles, int ntiles, int G,
    const int* __restrict__ cells, const cpx<T>* __restrict__ fac, const cpx<T>* __restrict__ rpool,
    cpx<T>* __restrict__ xpool, long long pool_stride, int nrhs) {
  typedef cpx<T> C;
  const int Lg = nd_task_rr(blockIdx.x, G);   // as in the forward kernel
  const int tix = Lg / G, g = Lg - (Lg / G) * G;
  if (tix >= ntiles) return;
  const int2 t = tiles[tix];
  const NdLvlJob J = jobs[t.x];
  const C* __restrict__ R = rpool + (long long)J.l * pool_stride + J.vbase;
  C* __restrict__ X = xpool + (long long)J.l * pool_stride + J.vbase;
  const int ns = J.ns, nf = J.ns + J.nbd;
  const int q0 = g * KG, nq = min(KG, nrhs - q0);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r0 = t.y + 64 * (w % ND_WRT);
  extern __shared__ unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  C out[KG];
  nd_wide_product<T, KG>(fac + J.fac + (long long)J.nbd * ns + r0, ns, max(0, min(64, ns - r0)), nf,
                         ns, cells + J.cell, q0, nq, R, X, J.nloc, lds, out);
  const int i = r0 + lane;
  if (w < ND_WRT && i < ns) {             // column quarter 0 holds the sums
    const int cell = cells[J.cell + i];
#pragma unroll
    for (int q = 0; q < KG; ++q)
      if (q < nq) X[(long long)(q0 + q) * J.nloc + cell] = out[q];
  }
}

// ---- fused bottom levels: the small nodes below the fusion level run one
// workgroup per (subtree, RHS group), level by level inside the workgroup
// (workgroup barriers instead of launches).  The subtree's nodes come in
// batches of one level whose fronts fit the LDS together (job.pad = the
// node's front offset in the batch): the waves gather the batch's fronts
// (a node per wave, lanes over front positions), then share its row passes
// (64 / KG rows x KG right-hand sides per pass, as in the one-node-per-wave
// kernels, so the arithmetic of a node is the same in either).  The forward
// pass runs the batches deepest level first, the backward pass in reverse.
template <typename T, int KG>
__global__ __launch_bounds__(512) void k_nd_fused_fwd(
    const int2* __restrict__ fjobs, int nfj, int G, const int2* __restrict__ batches,
    const NdLvlJob* __restrict__ jobs, const int* __restrict__ cells, const int* __restrict__ umaps,
    const cpx<T>* __restrict__ fac, cpx<T>* __restrict__ rpool, cpx<T>* __restrict__ upool,
    long long pool_stride, int nrhs, int kmax) {
  typedef cpx<T> C;
  constexpr int RPP = 64 / KG;
  const int Lg = nd_task(blockIdx.x, gridDim.x);
  const int fj = Lg / G, g = Lg - (Lg / G) * G;
  if (fj >= nfj) return;
  const int2 F = fjobs[fj];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int qq = lane % KG, rr = lane / KG;
  const int q0 = g * KG, nq = min(KG, nrhs - q0);
  const C zero = mk((T)0, (T)0);
  extern __shared__ unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  for (int b = F.x; b < F.x + F.y; ++b) {
    const int2 B = batches[b];
    for (int k = w; k < B.y; k += 8) {
      const NdLvlJob J = jobs[B.x + k];
      C* __restrict__ R = rpool + (long long)J.l * pool_stride + J.vbase;
      const C* __restrict__ U = upool + J.ubase;
      const int* fc = cells + J.cell;
      const int* um = umaps + J.umap;
      C* fr = lds + (long long)J.pad * KG;
      const int ns = J.ns, nf = J.ns + J.nbd;
      for (int p = lane; p < nf; p += 64) {
        const int i0 = um[2 * p], i1 = um[2 * p + 1];
        const bool own = p < ns;
        const int cell = own ? fc[p] : 0;
        const C* U0 = U + (long long)i0 * kmax + q0;
        const C* U1 = U + (long long)i1 * kmax + q0;
        C* Rc = R + (long long)q0 * J.nloc + cell;
#pragma unroll
        for (int q = 0; q < KG; ++q) {
          C v = zero;
          if (q < nq) {
            if (own) v = Rc[(long long)q * J.nloc];
            if (i0 >= 0) v = v + U0[q];
            if (i1 >= 0) v = v + U1[q];
            if (own && (i0 >= 0 || i1 >= 0)) Rc[(long long)q * J.nloc] = v;
          }
          fr[p * KG + q] = v;
        }
      }
    }
    __syncthreads();
    int item = 0;
    for (int k = 0; k < B.y; ++k) {
      const NdLvlJob J = jobs[B.x + k];
      const int np = (J.nbd + RPP - 1) / RPP;
      const C* fr = lds + (long long)J.pad * KG;
      const C* __restrict__ Lf = fac + J.fac;
      C* __restrict__ U = upool + J.ubase;
      for (int p = (w - item % 8 + 8) % 8; p < np; p += 8) {
        const int i = p * RPP + rr;
        if (i >= J.nbd) continue;
        C acc = fr[(J.ns + i) * KG + qq];
        nd_dot<T, KG, true>(acc, Lf + i, J.nbd, fr + qq, J.ns);
        if (qq < nq) U[(J.upd + i) * kmax + q0 + qq] = acc;
      }
      item += np;
    }
    __syncthreads();
  }
}

template <typename T, int KG>
__global__ __launch_bounds__(512) void k_nd_fused_bwd(
    const int2* __restrict__ fjobs, int nfj, int G, const int2* __restrict__ batches,
    const NdLvlJob* __restrict__ jobs, const int* __restrict__ cells, const cpx<T>* __restrict__ fac,
    const cpx<T>* __restrict__ rpool, cpx<T>* __restrict__ xpool, long long pool_stride, int nrhs) {
  typedef cpx<T> C;
  constexpr int RPP = 64 / KG;
  const int Lg = nd_task(blockIdx.x, gridDim.x);
  const int fj = Lg / G, g = Lg - (Lg / G) * G;
  if (fj >= nfj) return;
  const int2 F = fjobs[fj];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int qq = lane % KG, rr = lane / KG;
  const int q0 = g * KG, nq = min(KG, nrhs - q0);
  const C zero = mk((T)0, (T)0);
  extern __shared__ unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  for (int b = F.x + F.y - 1; b >= F.x; --b) {
    const int2 B = batches[b];
    for (int k = w; k < B.y; k += 8) {
      const NdLvlJob J = jobs[B.x + k];
      const C* __restrict__ R = rpool + (long long)J.l * pool_stride + J.vbase;
      const C* __restrict__ X = xpool + (long long)J.l * pool_stride + J.vbase;
      const int* fc = cells + J.cell;
      C* v = lds + (long long)J.pad * KG;
      const int ns = J.ns, nf = J.ns + J.nbd;
      for (int p = lane; p < nf; p += 64) {
        const bool own = p < ns;
        const long long c = (long long)q0 * J.nloc + fc[p];
#pragma unroll
        for (int q = 0; q < KG; ++q) {
          C x = zero;
          if (q < nq) x = own ? R[c + (long long)q * J.nloc] : -X[c + (long long)q * J.nloc];
          v[p * KG + q] = x;
        }
      }
    }
    __syncthreads();
    int item = 0;
    for (int k = 0; k < B.y; ++k) {
      const NdLvlJob J = jobs[B.x + k];
      const int np = (J.ns + RPP - 1) / RPP;
      const C* v = lds + (long long)J.pad * KG;
      const C* __restrict__ K = fac + J.fac + (long long)J.nbd * J.ns;
      C* __restrict__ X = xpool + (long long)J.l * pool_stride + J.vbase;
      const int* fc = cells + J.cell;
      for (int p = (w - item % 8 + 8) % 8; p < np; p += 8) {
        const int i = p * RPP + rr;
        if (i >= J.ns) continue;
        C acc = zero;
        nd_dot<T, KG, false>(acc, K + i, J.ns, v + qq, J.ns + J.nbd);
        if (qq < nq) X[(long long)(q0 + qq) * J.nloc + fc[i]] = acc;
      }
      item += np;
    }
    __syncthreads();
  }
}

template <typename T>
size_t nd_lvl_lds_bytes(int max_nf, int kg) {
  return (size_t)std::max(1, max_nf) * kg * sizeof(cpx<T>);
}

static size_t nd_top_lds_bytes(size_t ts, int max_ntop, int kg) {
  const int cw = (max_ntop + ND_TW - 1) / ND_TW;
  return ((size_t)ND_TW * cw + (size_t)(ND_TW - 1) * 64) * kg * ts;
}

template <typename T>
int nd_kg(int max_nf, int kg, size_t lds_cap) {
  int k = 16;
  while (k > kg && k > 1) k >>= 1;
  while (k > 1 && nd_lvl_lds_bytes<T>(max_nf, k) > lds_cap) k >>= 1;
  return nd_lvl_lds_bytes<T>(max_nf, k) <= lds_cap ? k : 0;
}

static unsigned nd_grid(long long tasks) { return (unsigned)(((tasks + 7) / 8) * 8); }

// shape: tt <= 0: one node per wave, eight nodes per workgroup; else one node
// per workgroup of tt row tiles x cg column groups of waves.
template <typename T, int KG>
static void launch_lvl_fwd_k(int tt, int cg, const NdLvlJob* jobs, int njobs, const int* cells,
                             const int* umaps, const cpx<T>* fac, cpx<T>* rpool, cpx<T>* upool,
                             long long ps, int nrhs, int kmax, int max_nf, hipStream_t s) {
  const int G = (nrhs + KG - 1) / KG;
  const int npw = tt <= 0 ? 8 : 1, wv = tt <= 0 ? 8 : tt * cg;
  const int region = std::max(1, max_nf) * KG;
  const long long groups = (njobs + npw - 1) / npw;
  const size_t lds = tt <= 0 ? (size_t)npw * region
                             : (size_t)region + (size_t)std::max(cg - 1, 1) * tt * 64 * KG;
  hipLaunchKernelGGL((k_nd_lvl_fwd<T, KG>), dim3(nd_grid_rr(groups, G)), dim3(64 * wv),
                     lds * sizeof(cpx<T>), s, jobs, njobs, G, npw, region, std::max(1, tt),
                     std::max(1, cg), cells, umaps, fac, rpool, upool, ps, nrhs, kmax);
}

template <typename T>
void launch_nd_lvl_fwd(int kg, int tt, int cg, const NdLvlJob* jobs, int njobs, const int* cells,
                       const int* umaps, const cpx<T>* fac, cpx<T>* rpool, cpx<T>* upool,
                       long long pool_stride, int nrhs, int kmax, int max_nf, hipStream_t s) {
  if (njobs <= 0 || nrhs <= 0) return;
#define ND_FWD(K) launch_lvl_fwd_k<T, K>(tt, cg, jobs, njobs, cells, umaps, fac, rpool, upool, \
                                         pool_stride, nrhs, kmax, max_nf, s)
  switch (kg) {
    case 16: ND_FWD(16); break;
    case 8: ND_FWD(8); break;
    case 4: ND_FWD(4); break;
    case 2: ND_FWD(2); break;
    default: ND_FWD(1); break;
  }
#undef ND_FWD
}

template <typename T, int KG>
static void launch_lvl_bwd_k(int tt, int cg, const NdLvlJob* jobs, int njobs, const int* cells,
                             const cpx<T>* fac, const cpx<T>* rpool, cpx<T>* xpool, long long ps,
                             int nrhs, int max_nf, const cpx<T>* const* coef, hipStream_t s) {
  const int G = (nrhs + KG - 1) / KG;
  const int npw = tt <= 0 ? 8 : 1, wv = tt <= 0 ? 8 : tt * cg;
  const int region = std::max(1, max_nf) * KG;
  const long long groups = (njobs + npw - 1) / npw;
  const size_t lds = tt <= 0 ? (size_t)npw * region
                             : (size_t)region + (size_t)std::max(cg - 1, 1) * tt * 64 * KG;
  hipLaunchKernelGGL((k_nd_lvl_bwd<T, KG>), dim3(nd_grid_rr(groups, G)), dim3(64 * wv),
                     lds * sizeof(cpx<T>), s, jobs, njobs, G, npw, region, std::max(1, tt),
                     std::max(1, cg), cells, fac, rpool, xpool, ps, nrhs, coef[0], coef[1], coef[2]);
}

template <typename T>
void launch_nd_lvl_bwd(int kg, int tt, int cg, const NdLvlJob* jobs, int njobs, const int* cells,
                       const cpx<T>* fac, const cpx<T>* rpool, cpx<T>* xpool,
                       long long pool_stride, int nrhs, int max_nf, const cpx<T>* const* coef,
                       hipStream_t s) {
  if (njobs <= 0 || nrhs <= 0) return;
#define ND_BWD(K) launch_lvl_bwd_k<T, K>(tt, cg, jobs, njobs, cells, fac, rpool, xpool, pool_stride, \
                                         nrhs, max_nf, coef, s)
  switch (kg) {
    case 16: ND_BWD(16); break;
    case 8: ND_BWD(8); break;
    case 4: ND_BWD(4); break;
    case 2: ND_BWD(2); break;
    default: ND_BWD(1); break;
  }
#undef ND_BWD
}

template <typename T, int KG>
static void launch_top_k(const NdTopJob* jobs, int njobs, const int* cells, const int* usrc,
                         const cpx<T>* fac, const cpx<T>* rpool, const cpx<T>* upool,
                         cpx<T>* xpool, long long ps, int nrhs, int kmax, int max_ntop,
                         hipStream_t s) {
  const int G = (nrhs + KG - 1) / KG;
  const int ntiles = (max_ntop + 63) / 64;
  const int cwmax = (max_ntop + ND_TW - 1) / ND_TW;
  hipLaunchKernelGGL((k_nd_top<T, KG>), dim3(nd_grid((long long)njobs * G * ntiles)),
                     dim3(64 * ND_TW), nd_top_lds_bytes(sizeof(cpx<T>), max_ntop, KG), s, jobs,
                     njobs, G, ntiles, cells, usrc, fac, rpool, upool, xpool, ps, nrhs, kmax,
                     cwmax);
}

template <typename T>
void launch_nd_top(int kg, const NdTopJob* jobs, int njobs, const int* cells, const int* usrc,
                   const cpx<T>* fac, const cpx<T>* rpool, const cpx<T>* upool, cpx<T>* xpool,
                   long long pool_stride, int nrhs, int kmax, int max_ntop, hipStream_t s) {
  if (njobs <= 0 || nrhs <= 0 || max_ntop <= 0) return;
  const int k = kg;
#define ND_TOP(K) launch_top_k<T, K>(jobs, njobs, cells, usrc, fac, rpool, upool, xpool, \
                                     pool_stride, nrhs, kmax, max_ntop, s)
  switch (k) {
    case 16: ND_TOP(16); break;
    case 8: ND_TOP(8); break;
    case 4: ND_TOP(4); break;
    case 2: ND_TOP(2); break;
    default: ND_TOP(1); break;
  }
#undef ND_TOP
}

// ---- wide-mode launchers
template <typename T>
void launch_nd_form(const NdLvlJob* jobs, const int2* tiles, int ntiles, const int* cells,
                    const int* umaps, cpx<T>* rpool, const cpx<T>* upool, long long pool_stride,
                    int nrhs, int kmax, hipStream_t s) {
  if (ntiles <= 0 || nrhs <= 0) return;
  hipLaunchKernelGGL(k_nd_form<T>, dim3(nd_grid(ntiles)), dim3(256), 0, s, jobs, tiles, ntiles,
                     cells, umaps, rpool, upool, pool_stride, nrhs, kmax);
}

int nd_wide_kg(size_t ts, int nrhs) {
  if (ts > sizeof(cpx<float>)) return 8;
  return nrhs <= 8 ? 8 : nrhs <= 16 ? 16 : 32;
}

template <typename T, int KG>
static void launch_wide_fwd_k(const NdLvlJob* jobs, const int2* tiles, int ntiles, const int* cells,
                              const int* umaps, const cpx<T>* fac, const cpx<T>* rpool,
                              cpx<T>* upool, long long ps, int nrhs, int kmax, hipStream_t s) {
  const int G = (nrhs + KG - 1) / KG;
  hipLaunchKernelGGL((k_nd_wide_fwd<T, KG>), dim3(nd_grid_rr(ntiles, G)), dim3(512),
                     nd_wide_lds_entries<T>(KG) * sizeof(cpx<T>), s, jobs, tiles, ntiles, G, cells,
                     umaps, fac, rpool, upool, ps, nrhs, kmax);
}

template <typename T, int KG>
static void launch_wide_bwd_k(const NdLvlJob* jobs, const int2* tiles, int ntiles, const int* cells,
                              const cpx<T>* fac, const cpx<T>* rpool, cpx<T>* xpool, long long ps,
                              int nrhs, hipStream_t s) {
  const int G = (nrhs + KG - 1) / KG;
  hipLaunchKernelGGL((k_nd_wide_bwd<T, KG>), dim3(nd_grid_rr(ntiles, G)), dim3(512),
                     nd_wide_lds_entries<T>(KG) * sizeof(cpx<T>), s, jobs, tiles, ntiles, G, cells,
                     fac, rpool, xpool, ps, nrhs);
}

template <typename T>
void launch_nd_wide_fwd(const NdLvlJob* jobs, const int2* tiles, int ntiles, const int* cells,
                        const int* umaps, const cpx<T>* fac, const cpx<T>* rpool, cpx<T>* upool,
                        long long pool_stride, int nrhs, int kmax, hipStream_t s) {
  if (ntiles <= 0 || nrhs <= 0) return;
  switch (nd_wide_kg(sizeof(cpx<T>), nrhs)) {
    case 32: launch_wide_fwd_k<T, 32>(jobs, tiles, ntiles, cells, umaps, fac, rpool, upool, pool_stride, nrhs, kmax, s); break;
    case 16: launch_wide_fwd_k<T, 16>(jobs, tiles, ntiles, cells, umaps, fac, rpool, upool, pool_stride, nrhs, kmax, s); break;
    default: launch_wide_fwd_k<T, 8>(jobs, tiles, ntiles, cells, umaps, fac, rpool, upool, pool_stride, nrhs, kmax, s); break;
  }
}

template <typename T>
void launch_nd_wide_bwd(const NdLvlJob* jobs, const int2* tiles, int ntiles, const int* cells,
                        const cpx<T>* fac, const cpx<T>* rpool, cpx<T>* xpool, long long pool_stride,
                        int nrhs, hipStream_t s) {
  if (ntiles <= 0 || nrhs <= 0) return;
  switch (nd_wide_kg(sizeof(cpx<T>), nrhs)) {
    case 32: launch_wide_bwd_k<T, 32>(jobs, tiles, ntiles, cells, fac, rpool, xpool, pool_stride, nrhs, s); break;
    case 16: launch_wide_bwd_k<T, 16>(jobs, tiles, ntiles, cells, fac, rpool, xpool, pool_stride, nrhs, s); break;
    default: launch_wide_bwd_k<T, 8>(jobs, tiles, ntiles, cells, fac, rpool, xpool, pool_stride, nrhs, s); break;
  }
}

// ---- fused bottom levels: launchers
template <typename T, int KG>
static void launch_fused_k(bool fwd, const int2* fjobs, int nfj, const int2* batches,
                           const NdLvlJob* jobs, const int* cells, const int* umaps,
                           const cpx<T>* fac, cpx<T>* rpool, cpx<T>* upool, cpx<T>* xpool,
                           long long ps, int nrhs, int kmax, hipStream_t s) {
  const int G = (nrhs + KG - 1) / KG;
  const size_t lds = (size_t)ND_FUSE_CAP * KG * sizeof(cpx<T>);
  if (fwd)
    hipLaunchKernelGGL((k_nd_fused_fwd<T, KG>), dim3(nd_grid((long long)nfj * G)), dim3(512), lds, s,
                       fjobs, nfj, G, batches, jobs, cells, umaps, fac, rpool, upool, ps, nrhs, kmax);
  else
    hipLaunchKernelGGL((k_nd_fused_bwd<T, KG>), dim3(nd_grid((long long)nfj * G)), dim3(512), lds, s,
                       fjobs, nfj, G, batches, jobs, cells, fac, rpool, xpool, ps, nrhs);
}

template <typename T>
void launch_nd_fused(bool fwd, int kg, const int2* fjobs, int nfj, const int2* batches,
                     const NdLvlJob* jobs, const int* cells, const int* umaps, const cpx<T>* fac,
                     cpx<T>* rpool, cpx<T>* upool, cpx<T>* xpool, long long pool_stride, int nrhs,
                     int kmax, hipStream_t s) {
  if (nfj <= 0 || nrhs <= 0) return;
#define ND_FUSED(K) launch_fused_k<T, K>(fwd, fjobs, nfj, batches, jobs, cells, umaps, fac, rpool, \
                                         upool, xpool, pool_stride, nrhs, kmax, s)
  switch (kg) {
    case 16: ND_FUSED(16); break;
    case 8: ND_FUSED(8); break;
    case 4: ND_FUSED(4); break;
    case 2: ND_FUSED(2); break;
    default: ND_FUSED(1); break;
  }
#undef ND_FUSED
}

// LDS needed by the dense top for a given RHS group (1 if even that does not fit)
size_t nd_top_lds_need(size_t ts, int max_ntop) { return nd_top_lds_bytes(ts, max_ntop, 1); }

// The largest RHS group (a power of two <= kg) whose gathered columns fit the LDS
int nd_top_kg(size_t ts, int ntop, int kg) {
  int k = 16;
  while (k > kg && k > 1) k >>= 1;
  while (k > 1 && nd_top_lds_bytes(ts, ntop, k) > 160 * 1024) k >>= 1;
  return k;
}

// ============================================================================
// Factorisation kernels (FP64)
// ============================================================================
// Entry (ci, cj) of the J-scaled local operator: the diagonal, or the face
// coupling stored at the lower-indexed cell of a neighbour pair.
__device__ inline cpx<double> nd_coef(int ci, int cj, const int* dims, long long coef,
                                      const cpx<double>* diag, const cpx<double>* cx,
                                      const cpx<double>* cy, const cpx<double>* cz) {
  if (ci == cj) return diag[coef + ci];
  const int lo = min(ci, cj), d = max(ci, cj) - lo;
  const int nx = dims[0], ny = dims[1];
  if (d == 1 && lo % nx != nx - 1) return cx[coef + lo];
  if (d == nx && (lo / nx) % ny != ny - 1) return cy[coef + lo];
  if (d == nx * ny) return cz[coef + lo];
  return mk(0.0, 0.0);
}

__global__ __launch_bounds__(256) void k_nd_front(const NdFrontJob* __restrict__ jobs,
                                                  const NdNodeDev* __restrict__ nodes,
                                                  const int* __restrict__ cells,
                                                  const int* __restrict__ maps,
                                                  const cpx<double>* diag, const cpx<double>* cx,
                                                  const cpx<double>* cy, const cpx<double>* cz,
                                                  cpx<double>* W) {
  const NdFrontJob J = jobs[blockIdx.y];
  const NdNodeDev N = nodes[J.node];
  const int nf = N.ns + N.nbd;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)nf * nf) return;
  const int p = (int)(e % nf), q = (int)(e / nf);
  const int* fc = cells + N.cell;
  cpx<double> v = mk(0.0, 0.0);
  if (p < N.ns || q < N.ns) v = nd_coef(fc[p], fc[q], J.dims, J.coef, diag, cx, cy, cz);
  const int* mp = maps + N.map;
  if (N.ch0 >= 0) {
    const int i = mp[2 * p], j = mp[2 * q];
    if (i >= 0 && j >= 0) {
      const NdNodeDev C0 = nodes[N.ch0];
      const int f0 = C0.ns + C0.nbd;
      v = v + W[J.F0 + (C0.ns + i) + (long long)(C0.ns + j) * f0];
    }
  }
  if (N.ch1 >= 0) {
    const int i = mp[2 * p + 1], j = mp[2 * q + 1];
    if (i >= 0 && j >= 0) {
      const NdNodeDev C1 = nodes[N.ch1];
      const int f1 = C1.ns + C1.nbd;
      v = v + W[J.F1 + (C1.ns + i) + (long long)(C1.ns + j) * f1];
    }
  }
  W[J.F + p + (long long)q * nf] = v;
}

void launch_nd_front(const NdFrontJob* jobs, int njobs, int max_nf, const NdNodeDev* nodes,
                     const int* cells, const int* maps, const cpx<double>* diag,
                     const cpx<double>* cx, const cpx<double>* cy, const cpx<double>* cz,
                     cpx<double>* work, hipStream_t s) {
  if (njobs <= 0) return;
  hipLaunchKernelGGL(k_nd_front, dim3(nd_cdiv((long long)max_nf * max_nf, 256), njobs), dim3(256),
                     0, s, jobs, nodes, cells, maps, diag, cx, cy, cz, work);
}

__global__ __launch_bounds__(256) void k_nd_top_asm(const NdTopAsmJob* __restrict__ jobs,
                                                    const NdNodeDev* __restrict__ nodes,
                                                    const int* __restrict__ cells,
                                                    const int* __restrict__ srcs,
                                                    const long long* __restrict__ fo,
                                                    const cpx<double>* diag, const cpx<double>* cx,
                                                    const cpx<double>* cy, const cpx<double>* cz,
                                                    cpx<double>* W) {
  const NdTopAsmJob J = jobs[blockIdx.y];
  const int n = J.ntop;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)n * n) return;
  const int p = (int)(e % n), q = (int)(e / n);
  const int* tc = cells + J.cell;
  const int* sr = srcs + J.src;
  cpx<double> v = nd_coef(tc[p], tc[q], J.dims, J.coef, diag, cx, cy, cz);
  // update matrices of the subtree roots whose boundaries hold both cells
  for (int a = 0; a < J.dim2; ++a) {
    const int rp = sr[(p * J.dim2 + a) * 2];
    if (rp < 0) break;
    for (int b = 0; b < J.dim2; ++b) {
      const int rq = sr[(q * J.dim2 + b) * 2];
      if (rq < 0) break;
      if (rq != rp) continue;
      const NdNodeDev N = nodes[J.node0 + rp];
      const int nf = N.ns + N.nbd;
      const int i = sr[(p * J.dim2 + a) * 2 + 1], j = sr[(q * J.dim2 + b) * 2 + 1];
      v = v + W[fo[J.fo + rp] + (N.ns + i) + (long long)(N.ns + j) * nf];
    }
  }
  W[J.T + p + (long long)q * n] = v;
}

void launch_nd_top_asm(const NdTopAsmJob* jobs, int njobs, int max_ntop, const NdNodeDev* nodes,
                       const int* cells, const int* src, const long long* fo,
                       const cpx<double>* diag, const cpx<double>* cx, const cpx<double>* cy,
                       const cpx<double>* cz, cpx<double>* work, hipStream_t s) {
  if (njobs <= 0 || max_ntop <= 0) return;
  hipLaunchKernelGGL(k_nd_top_asm, dim3(nd_cdiv((long long)max_ntop * max_ntop, 256), njobs),
                     dim3(256), 0, s, jobs, nodes, cells, src, fo, diag, cx, cy, cz, work);
}

template <typename T>
__global__ __launch_bounds__(256) void k_nd_copy(const NdCopyJob* __restrict__ jobs, cpx<double>* W,
                                                 cpx<T>* fac) {
  const NdCopyJob J = jobs[blockIdx.y];
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)J.rows * J.cols) return;
  const int i = (int)(e % J.rows), j = (int)(e / J.rows);
  const long long s = J.trans ? J.src + j + (long long)i * J.ld_src : J.src + i + (long long)j * J.ld_src;
  const long long d = J.dst + i + (long long)j * J.ld_dst;
  if (J.to_fac) fac[d] = cvt<T>(W[s]);
  else W[d] = W[s];
}

template <typename T>
void launch_nd_copy(const NdCopyJob* jobs, int njobs, int max_rows, int max_cols,
                    cpx<double>* work, cpx<T>* fac, hipStream_t s) {
  if (njobs <= 0) return;
  hipLaunchKernelGGL(k_nd_copy<T>, dim3(nd_cdiv((long long)max_rows * max_cols, 256), njobs),
                     dim3(256), 0, s, jobs, work, fac);
}

// C = beta C + alpha A B (FP64 complex, column-major with leading dimensions)
// on the FP64 matrix cores (v_mfma_f64_16x16x4f64): a 64 x 64 output tile per
// 256-thread workgroup, K staged through LDS in panels of 16; wave w owns the
// 32 x 32 quarter at (32 (w % 2), 32 (w / 2)) as 2 x 2 blocks of 16 x 16.
// Operand lanes: A[row l % 16][k l / 16], B[k l / 16][col l % 16]; output j of
// lane l is row 4 j + l / 16, column l % 16 of the block.
typedef double nd_f64x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_nd_gemm(const NdGemmJob* __restrict__ jobs,
                                                 cpx<double>* W) {
  const NdGemmJob J = jobs[blockIdx.z];
  const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  if (i0 >= J.m || j0 >= J.n) return;
  __shared__ cpx<double> As[16][65];   // [k][row]
  __shared__ cpx<double> Bs[16][65];   // [k][col]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = (w & 1) * 32, wc = (w >> 1) * 32, l16 = lane & 15, l4 = lane >> 4;
  const cpx<double>* __restrict__ A = W + J.a;
  const cpx<double>* __restrict__ B = W + J.b;
  nd_f64x4 cr[2][2], ci[2][2];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      cr[rb][cb] = nd_f64x4{0.0, 0.0, 0.0, 0.0};
      ci[rb][cb] = nd_f64x4{0.0, 0.0, 0.0, 0.0};
    }
  for (int k0 = 0; k0 < J.k; k0 += 16) {
    for (int e = tid; e < 1024; e += 256) {
      const int mm = e & 63, ka = e >> 6;
      const int r = i0 + mm, ka0 = k0 + ka;
      As[ka][mm] = (r < J.m && ka0 < J.k) ? A[r + (long long)ka0 * J.lda] : mk(0.0, 0.0);
      const int kb = e & 15, nn = e >> 4;
      const int cc = j0 + nn, kb0 = k0 + kb;
      Bs[kb][nn] = (cc < J.n && kb0 < J.k) ? B[kb0 + (long long)cc * J.ldb] : mk(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      cpx<double> av[2], bv[2];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) av[rb] = As[kk + l4][wr + 16 * rb + l16];
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) bv[cb] = Bs[kk + l4][wc + 16 * cb + l16];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
          cr[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[rb].re, bv[cb].re, cr[rb][cb], 0, 0, 0);
          cr[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[rb].im, bv[cb].im, cr[rb][cb], 0, 0, 0);
          ci[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[rb].re, bv[cb].im, ci[rb][cb], 0, 0, 0);
          ci[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[rb].im, bv[cb].re, ci[rb][cb], 0, 0, 0);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = i0 + wr + 16 * rb + 4 * j + l4, cc = j0 + wc + 16 * cb + l16;
        if (r < J.m && cc < J.n) {
          const long long o = J.c + r + (long long)cc * J.ldc;
          const cpx<double> v = mk(J.alpha * cr[rb][cb][j], J.alpha * ci[rb][cb][j]);
          W[o] = J.beta ? W[o] + v : v;
        }
      }
}

void launch_nd_gemm(const NdGemmJob* jobs, int njobs, int max_m, int max_n, cpx<double>* work,
                    hipStream_t s) {
  if (njobs <= 0 || max_m <= 0 || max_n <= 0) return;
  hipLaunchKernelGGL(k_nd_gemm, dim3(nd_cdiv(max_m, 64), nd_cdiv(max_n, 64), njobs), dim3(256), 0,
                     s, jobs, work);
}

#define ND_INST(T)                                                                              \
  template void launch_nd_lvl_fwd<T>(int, int, int, const NdLvlJob*, int, const int*,           \
                                     const int*, const cpx<T>*, cpx<T>*, cpx<T>*, long long, int, \
                                     int, int, hipStream_t);                                     \
  template void launch_nd_lvl_bwd<T>(int, int, int, const NdLvlJob*, int, const int*,           \
                                     const cpx<T>*, const cpx<T>*, cpx<T>*, long long, int, int,  \
                                     const cpx<T>* const*, hipStream_t);                         \
  template void launch_nd_top<T>(int, const NdTopJob*, int, const int*, const int*,              \
                                 const cpx<T>*, const cpx<T>*, const cpx<T>*, cpx<T>*, long long, \
                                 int, int, int, hipStream_t);                                    \
  template void launch_nd_form<T>(const NdLvlJob*, const int2*, int, const int*, const int*,      \
                                 cpx<T>*, const cpx<T>*, long long, int, int, hipStream_t);      \
  template void launch_nd_wide_fwd<T>(const NdLvlJob*, const int2*, int, const int*, const int*,  \
                                      const cpx<T>*, const cpx<T>*, cpx<T>*, long long, int, int, \
                                      hipStream_t);                                               \
  template void launch_nd_wide_bwd<T>(const NdLvlJob*, const int2*, int, const int*,              \
                                      const cpx<T>*, const cpx<T>*, cpx<T>*, long long, int,      \
                                      hipStream_t);                                               \
  template void launch_nd_fused<T>(bool, int, const int2*, int, const int2*, const NdLvlJob*,     \
                                   const int*, const int*, const cpx<T>*, cpx<T>*, cpx<T>*,       \
                                   cpx<T>*, long long, int, int, hipStream_t);                    \
  template size_t nd_lvl_lds_bytes<T>(int, int);                                                 \
  template int nd_kg<T>(int, int, size_t);                                                       \
  template void launch_nd_copy<T>(const NdCopyJob*, int, int, int, cpx<double>*, cpx<T>*,       \
                                  hipStream_t);

ND_INST(float)
ND_INST(double)

}  // namespace dsd
