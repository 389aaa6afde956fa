// Nested-dissection (multifrontal) local solver: symbolic analysis of a local
// grid shape (host), the device tables the kernels read, and the launchers.
// Internal header: not part of the C ABI.
//
// A subdomain operator (5/7-point stencil on a box of cells) is ordered by
// recursive bisection: a node is a box; unless it is small (a leaf, whose
// separator is the whole box) its separator is the plane of cells in the
// middle of its longest axis and its two children are the halves on either
// side.  The front of a node is its separator S followed by its boundary B,
// the cells outside the box that touch it through the stencil (all of them
// belong to ancestors' separators).  Eliminating the subtree below a node
// leaves a dense Schur complement F on S u B, and with P = F_SS^{-1}:
//   forward (leaves to root):  f_S = r_S + (children's updates on S)
//                              u_B = (children's updates on B) - L f_S,  L = F_BS P
//   backward (root to leaves): x_S = P f_S - L^T x_B   (F symmetric: L^T = P F_SB)
// The nodes above a chosen depth form the dense top: the Schur complement on
// all of their separator cells is inverted once (P_top) and applied as one
// dense product.  The remaining subtrees are independent: one workgroup runs
// a whole subtree, level by level, for a group of right-hand sides.
#pragma once
#include "common.hpp"

#ifndef __HIPCC_RTC__
#include <vector>
#endif

namespace dsd {

struct NdNodeDev;

// ---- host: analysis of one local grid shape -------------------------------
struct NdNode {
  int lo[3], hi[3];          // box [lo, hi) per axis
  int depth = 0;
  int parent = -1, child[2] = {-1, -1};
  std::vector<int> sep;      // local cell indices (x fastest), ascending
  std::vector<int> bnd;      // ascending
  bool top = false;          // separator belongs to the dense top
  int subtree = -1;          // subtree (root order) of a non-top node
  int level = 0;             // depth below its subtree root
  long long fac = 0;         // factor offset (entries) within the subdomain: L (nbd x ns), K (ns x nf)
  long long upd = 0;         // update-vector offset (entries per right-hand side)
};

struct NdShape {
  int dim = 2, dims[3] = {1, 1, 1};
  int dtop = 0;                    // nodes of depth < dtop are in the dense top
  std::vector<NdNode> nodes;       // postorder (children before parents)
  std::vector<int> top_cells;      // the dense top's cells, in order
  std::vector<int> roots;          // subtree roots (node ids)
  int nlev = 0;                    // most levels of a subtree
  long long top_fac = 0;           // offset of P_top (ntop x ntop, column-major)
  long long fac_entries = 0;       // factor entries of one subdomain
  long long upd_entries = 0;       // update-vector entries per right-hand side
  int max_ns = 0, max_nbd = 0, max_nf = 0;
  int ntop() const { return (int)top_cells.size(); }
};

// leaf_max: largest box (cells) kept whole; ntop_max: largest dense top.
NdShape nd_analyse(int dim, const int* dims, int leaf_max, int ntop_max);

// Where one shape's entries start in the device tables, and its subtrees'
// level-pointer ranges.
struct NdShapeTab {
  int node0 = 0;             // first node in the node table
  int top_cell = 0;          // top cells in the cell table
  int top_src = 0;           // top update sources (2 dim pairs per top cell)
  int top_usrc = 0;          // the same as update-vector entries (2 dim per top cell)
  std::vector<int> lev0;     // per subtree: first entry in the level-pointer table
  std::vector<int> nlev;     // per subtree: levels
};
// Append one shape to the device tables (node, cell, gather-map, top-source,
// level-pointer, level-size and level-node tables).  False if the analysis is
// inconsistent (a boundary outside its parent's front or the top).
bool nd_append_tables(const NdShape& S, NdShapeTab& tab, std::vector<NdNodeDev>& nodes,
                      std::vector<int>& cells, std::vector<int>& maps, std::vector<int>& umaps,
                      std::vector<int>& src, std::vector<int>& usrc, std::vector<int>& lev,
                      std::vector<int>& levmax, std::vector<int>& levnodes);

// ---- device tables ---------------------------------------------------------
// Node table entry (shared by every subdomain of one shape).  The front's
// cells are cells[cell .. cell + ns + nbd): separator, then boundary.  The
// front gather map holds, per front position, the position in child 0's and
// child 1's boundary that contributes to it (-1: none).
struct NdNodeDev {
  int ns, nbd;
  int cell;                  // offset of the front's cells in the cell table
  int map;                   // offset of the gather map (2 ints per front position); the
                             // update-map table (umaps) has the same layout, holding the
                             // update entries (child upd + position) instead
  int ch0, ch1;              // children (node-table indices; -1 none)
  long long fac;             // factor offset within the subdomain: L (nbd x ns), then K (ns x nf)
  long long upd;             // update-vector offset within the member (entries)
};

// One node of one member in a level launch, with everything its kernels
// need (no further descriptor loads): sizes, the front's cells, the update
// entries its front gathers from (umap: 2 per front position, entries
// relative to the member's base, -1 none), its factor and update offsets.
struct NdLvlJob {
  int ns, nbd;
  int cell, umap;            // offsets in the cell table and the update-map table
  int l;                     // sweep slot
  int pad;
  long long nloc;            // local cells
  long long fac;             // factor offset of the node (L, then K)
  long long upd;             // update-vector entry of the node (within the member)
  long long vbase;           // vector-pool offset of the subdomain slice
  long long ubase;           // update-vector base of this member (entries x kmax)
  // Leaves (no children): the separator is the whole box [lo, hi) of the local
  // grid and its couplings to the boundary are the operator's own face
  // couplings, so the backward product forms f_S - A_SB x_B from the
  // coefficients and multiplies it by P alone (the first ns columns of K).
  int leaf;
  int lo[3], hi[3], dims[3];
  long long coef;            // first cell of the subdomain in the coefficient arrays
};

// Dense top of one subdomain solve.  usrc holds, per top cell, dim2
// update-vector entries (relative to the member's base; -1: none) of the
// subtree-root updates that land on it.
struct NdTopJob {
  int ntop, dim2;
  int cell, usrc;            // offsets of the top cells and of their update entries
  long long nloc, fac, vbase, ubase;
  int l;                     // sweep slot
  int pad;
};

// Factorisation (FP64) jobs.
struct NdFrontJob {          // assemble the front of one node of one subdomain
  int node;                  // node-table index
  int dims[3];               // local grid
  long long coef;            // subdomain coefficient base
  long long F, F0, F1;       // FP64 front offsets: this node, child 0, child 1 (-1 none)
};
struct NdTopAsmJob {         // assemble the dense top of one subdomain
  int ntop, dim2;
  int cell, src;             // top cells; update sources
  int dims[3];
  int fo;                    // offset of the subdomain's per-node front offsets in fo[]
  int node0;                 // the shape's first node in the node table
  int pad;
  long long coef;
  long long T;               // FP64 top matrix offset
};
struct NdCopyJob {           // dst(i, j) = src(i, j) or src(j, i): FP64 work -> work or factors
  int rows, cols;            // of the destination block
  int ld_src, ld_dst;
  int trans;                 // 1: dst(i, j) = src(j, i)
  int to_fac;                // 1: destination is the factor array (rounded to T)
  long long src, dst;
};
struct NdGemmJob {           // C = beta C + alpha A B  (FP64 complex, column-major, leading dims)
  int m, n, k;
  int lda, ldb, ldc;
  int beta, pad;
  double alpha;
  long long a, b, c;
};

// One level of the forward / backward passes: one workgroup of `waves` waves
// per (node, RHS group); max_nf = the largest front of the launch.
// Shape (tt, cg): tt <= 0 runs one node per wave, eight per workgroup, lanes
// over (row, RHS) pairs (the small nodes of the deep levels); otherwise one
// node per workgroup of tt 64-row tiles x cg column groups of waves, lanes
// over rows and the column groups summed in LDS (the large nodes).
template <typename T>
void launch_nd_lvl_fwd(int kg, int tt, int cg, const NdLvlJob* jobs, int njobs, const int* cells,
                       const int* umaps, const cpx<T>* fac, cpx<T>* rpool, cpx<T>* upool,
                       long long pool_stride, int nrhs, int kmax, int max_nf, hipStream_t s);
template <typename T>
void launch_nd_lvl_bwd(int kg, int tt, int cg, const NdLvlJob* jobs, int njobs, const int* cells,
                       const cpx<T>* fac, const cpx<T>* rpool, cpx<T>* xpool,
                       long long pool_stride, int nrhs, int max_nf, const cpx<T>* const* coef,
                       hipStream_t s);
// dense top: x_top = P_top (r_top + gathered updates); kg = the RHS group
// (nd_top_kg of the launch's largest top)
template <typename T>
void launch_nd_top(int kg, const NdTopJob* jobs, int njobs, const int* cells, const int* usrc,
                   const cpx<T>* fac, const cpx<T>* rpool, const cpx<T>* upool, cpx<T>* xpool,
                   long long pool_stride, int nrhs, int kmax, int max_ntop, hipStream_t s);
// Wide mode (fronts too large for the LDS, or more than 512 rows): tiles are
// {node job, first of ND_WROWS rows (or of 256 separator positions for the
// form step)}.
// Forward: launch_nd_form (f_S = r_S + children's updates, into R), then
// launch_nd_wide_fwd (u_B); backward: launch_nd_wide_bwd (x_S).  Every
// right-hand side of a group of nd_wide_kg(ts, nrhs) in one pass.
template <typename T>
void launch_nd_form(const NdLvlJob* jobs, const int2* tiles, int ntiles, const int* cells,
                    const int* umaps, cpx<T>* rpool, const cpx<T>* upool, long long pool_stride,
                    int nrhs, int kmax, hipStream_t s);
template <typename T>
void launch_nd_wide_fwd(const NdLvlJob* jobs, const int2* tiles, int ntiles, const int* cells,
                        const int* umaps, const cpx<T>* fac, const cpx<T>* rpool, cpx<T>* upool,
                        long long pool_stride, int nrhs, int kmax, hipStream_t s);
template <typename T>
void launch_nd_wide_bwd(const NdLvlJob* jobs, const int2* tiles, int ntiles, const int* cells,
                        const cpx<T>* fac, const cpx<T>* rpool, cpx<T>* xpool, long long pool_stride,
                        int nrhs, hipStream_t s);
int nd_wide_kg(size_t ts, int nrhs);
// Fused bottom levels: one workgroup per (subtree below the fusion level, RHS
// group); fjobs[i] = {first batch, batches}; a batch = {first job, jobs} of one
// level whose fronts total at most ND_FUSE_CAP positions (job.pad = the node's
// front offset in the batch).  Forward: batches in order; backward: reversed.
constexpr int ND_FUSE_CAP = 512;
constexpr int ND_WROWS = 128;      // rows of a wide-mode tile
template <typename T>
void launch_nd_fused(bool fwd, int kg, const int2* fjobs, int nfj, const int2* batches,
                     const NdLvlJob* jobs, const int* cells, const int* umaps, const cpx<T>* fac,
                     cpx<T>* rpool, cpx<T>* upool, cpx<T>* xpool, long long pool_stride, int nrhs,
                     int kmax, hipStream_t s);
// LDS the dense top needs with one right-hand side per workgroup
size_t nd_top_lds_need(size_t ts, int max_ntop);
// RHS group of a dense top of ntop cells (a power of two <= kg that fits the LDS)
int nd_top_kg(size_t ts, int ntop, int kg);
// LDS of a level launch (max_nf front entries per RHS), and the RHS per workgroup that fit
template <typename T>
size_t nd_lvl_lds_bytes(int max_nf, int kg);
template <typename T>
int nd_kg(int max_nf, int kg, size_t lds_cap);

// factorisation
void launch_nd_front(const NdFrontJob* jobs, int njobs, int max_nf, const NdNodeDev* nodes,
                     const int* cells, const int* maps, const cpx<double>* diag,
                     const cpx<double>* cx, const cpx<double>* cy, const cpx<double>* cz,
                     cpx<double>* work, hipStream_t s);
void launch_nd_top_asm(const NdTopAsmJob* jobs, int njobs, int max_ntop, const NdNodeDev* nodes,
                       const int* cells, const int* src, const long long* fo,
                       const cpx<double>* diag, const cpx<double>* cx, const cpx<double>* cy,
                       const cpx<double>* cz, cpx<double>* work, hipStream_t s);
template <typename T>
void launch_nd_copy(const NdCopyJob* jobs, int njobs, int max_rows, int max_cols,
                    cpx<double>* work, cpx<T>* fac, hipStream_t s);
void launch_nd_gemm(const NdGemmJob* jobs, int njobs, int max_m, int max_n, cpx<double>* work,
                    hipStream_t s);

}  // namespace dsd
