// Launchers of the dsweep kernels (internal; called by the plan in plan.hip).
#pragma once
#include "common.hpp"

namespace dsd {

// Tables describing the partition for the pull-style FP64 assembly.
struct PartTables {
  const int* part_of[3];        // [ng_a] own part of every global array index
  const AxisPart* parts[3];     // [P_a] parts of each axis
  int P[3];                     // parts per axis
};

// ---- a1: coefficient assembly (FP64) for a list of grids
void launch_assemble(const Problem& P, const AxisGrid* d_grids, const long long* d_offs, int ngrids,
                     long long max_cells, const double* d_m, cpx<double>* diag, cpx<double>* cx,
                     cpx<double>* cy, cpx<double>* cz, hipStream_t s);

template <typename T>
void launch_convert(const cpx<double>* src, cpx<T>* dst, long long n, hipStream_t s);

// ---- a2: factorisation
// A factorisation job forms S = A_k - C_p Binv_p C_p (- C_q Binv_q C_q) in FP64
// scratch and inverts it in place (Gauss-Jordan, partial pivoting), then rounds
// it into the factor slot.
struct FactorJob {
  int sub;
  int k;            // block being factored
  int cp_blk;       // block index whose coupling array couples to the previous block (-1: none)
  int cq_blk;       // second neighbour (middle block only; -1: none)
  long long prev;   // scratch offset (doubles-complex) of the FP64 inverse of the previous block
  long long prev2;  // second neighbour's inverse (middle block)
  long long cur;    // scratch offset of this block's working matrix
};
void launch_schur(const Problem& P, const SubDesc* d_subs, const FactorJob* d_jobs, int njobs,
                  int max_nb, const cpx<double>* diag, const cpx<double>* cx,
                  const cpx<double>* cy, const cpx<double>* cz, cpx<double>* scratch,
                  hipStream_t s);
// Inversions (blocked Gauss-Jordan, FP64): d_piv holds max_nb ints and d_rbuf
// gj_rbuf_entries(max_nb) complex entries per job of the launch; d_pst (may be
// null) 2 doubles per job, updated to the smallest and largest squared pivot
// magnitude (initialise to +inf and 0).
template <typename T>
void launch_invert(const SubDesc* d_subs, const FactorJob* d_jobs, int njobs, int max_nb,
                   cpx<double>* scratch, cpx<T>* fac, int* d_err, int* d_piv, cpx<double>* d_rbuf,
                   double* d_pst, hipStream_t s);
size_t gj_rbuf_entries(int max_n);
size_t gj_lds_bytes(int max_n);   // dynamic LDS of an inversion launch

// ---- a3: subdomain solves (block-tridiagonal chains); phase 0 fwd, 1 mid, 2 bwd.
// A job is {subdomain, half (0 top / 1 bottom), sweep, unused}; the right-hand
// side and the solution of sweep l live at pool offset l * pool_stride.
template <typename T>
void launch_chain(int kg, int phase, const SubDesc* d_subs, const int4* d_jobs, int njobs,
                  int nrhs, int kmax, int max_nb, const cpx<T>* fac, const cpx<T>* cpl,
                  const cpx<T>* rpool, cpx<T>* vpool, long long pool_stride, hipStream_t s);
template <typename T>
size_t chain_lds_bytes(int max_nb, int kg);

// ---- a2/a3 (block cyclic reduction form).  Every level eliminates the
// even-position blocks of the remaining block-tridiagonal system.
// Factorisation jobs operate on FP64 working blocks (column-major nb x nb,
// offsets in complex entries into one working array).
struct BcrBlkJob {        // D := A_k (assembly of a diagonal block)
  int sub, k;
  long long dst;
};
struct BcrInvJob {        // invert src in place (FP64); round the inverse into fac[dst] (dst >= 0)
  int nb;
  int sub;                // subdomain (pivot report)
  long long src, dst;
};
struct BcrDiagUpd {       // level 0: D_j -= c_{j-1} P_{j-1} c_{j-1} + c_j P_{j+1} c_j;
  int sub, j;             //          E_out = -c_j P_{j+1} c_{j+1}
  long long d, pl, pr, eout;   // working offsets (-1: absent)
};
struct BcrCopyJob {       // fac[dst] = (T) work[src] or its transpose
  int nb, trans;
  long long src, dst;
};
void launch_bcr_assemble(const Problem& P, const SubDesc* d_subs, const BcrBlkJob* d_jobs, int njobs,
                         int max_nb, const cpx<double>* diag, const cpx<double>* cx,
                         const cpx<double>* cy, cpx<double>* work, hipStream_t s);
template <typename T>
void launch_bcr_invert(const BcrInvJob* d_jobs, int njobs, int max_nb, cpx<double>* work,
                       cpx<T>* fac, int* d_err, int* d_piv, cpx<double>* d_rbuf, double* d_pst,
                       hipStream_t s);
void launch_bcr_diag_update(const Problem& P, const SubDesc* d_subs, const BcrDiagUpd* d_jobs,
                            int njobs, int max_nb, const cpx<double>* cy, const cpx<double>* cz,
                            cpx<double>* work, hipStream_t s);
template <typename T>
void launch_bcr_copy(const BcrCopyJob* d_jobs, int njobs, int max_nb, const cpx<double>* work,
                     cpx<T>* fac, hipStream_t s);

// Solve jobs of the block cyclic reduction: one block of one subdomain in
// pool slot l.  R = reduced right-hand sides, X = solution (both in the pools).
enum {
  BCR_PR = 0,     // X_blk = M0 R_blk                                   (level-0 z; top level)
  BCR_KEPT = 1,   // R_blk = R_blk - M0 R_nl - M1 R_nr                  (forward, level >= 1)
  BCR_BWD0 = 2,   // X_blk = M0 (R_blk - c_{blk-1} X_nl - c_blk X_nr)   (backward, level 0)
  BCR_BWD = 3,    // X_blk = M0 R_blk - M1 X_nl - M2 X_nr               (backward, level >= 1)
  BCR_DFWD = 4,   // R_blk = R_blk - c_{blk-1} X_nl - c_blk X_nr        (forward, level 0)
  BCR_DENSE = 5,  // X_blk = M0 [R_b0; R_b1; ...; R_b(m-1)] with b_q = nl + q nr, m = pad:
                  // one nb x (m nb) row block of the inverse of a small reduced system
  BCR_CHB = 6     // X_blk = X_blk - M0 (c_{blk-1} X_nl)  or  X_blk - M0 (c_blk X_nr):
                  // a backward step of the block LDL^T chains (one neighbour)
};
struct BcrJob {
  int sub, l, blk, mode;
  int nl, nr, nb, pad;        // neighbour blocks (-1: none); block size of the subdomain
  long long m0, m1, m2;       // factor element offsets of the matrices
  long long nloc, vbase, cbase;   // subdomain cells, vector-pool and coefficient offsets
};
// nset: most operand vectors a job of the launch uses (LDS is sized for it);
// cg: wave groups splitting the columns of every job (1 to 12); rt: most
// 64-row tiles per workgroup (0: up to 4).
template <typename T>
void launch_bcr_solve(int kg, const SubDesc* d_subs, const BcrJob* d_jobs, int njobs, int nset,
                      int cg, int rt, int nrhs, int kmax, int max_nb, const cpx<T>* fac,
                      const cpx<T>* cpl, cpx<T>* rpool, cpx<T>* vpool, long long pool_stride,
                      hipStream_t s);
template <typename T>
void launch_bcr_dfwd(const SubDesc* d_subs, const BcrJob* d_jobs, int njobs, int nrhs, int kmax,
                     int max_nb, const cpx<T>* cpl, cpx<T>* rpool, const cpx<T>* vpool,
                     long long pool_stride, hipStream_t s);
// RHS per workgroup the solve kernel uses for a requested kg (register budget).
template <typename T>
int bcr_kg(int max_nb, int kg);
template <typename T>
size_t bcr_lds_bytes(int max_nb, int kg, int nset);
// LDS of one launch of the given shape (the check the plan makes before it
// accepts a dense top level).
template <typename T>
size_t bcr_launch_lds_bytes(int max_nb, int kg, int nset, int cg, int rt);

// Dense top level of the reduction: the m-block reduced system of one
// subdomain, assembled column-major (n = m nb) from its diagonal blocks
// D_q = work[dbase + (first + q stride) slot] and couplings
// E_q = work[ebase + q slot] (block (q, q+1) = E_q, block (q+1, q) = E_q^T).
struct BcrDenseJob {
  int nb, m, first, stride;
  long long slot, dbase, ebase;   // working offsets (complex entries)
  long long out;                  // dense matrix offset in the dense work array
  long long fac;                  // factor offset of the m row blocks (nb x n each)
};
void launch_bcr_dense_build(const BcrDenseJob* d_jobs, int njobs, int max_n,
                            const cpx<double>* work, cpx<double>* dense, hipStream_t s);
// fac[J.fac + i nb n + c nb + r] = (T) dense[J.out + c n + i nb + r]
template <typename T>
void launch_bcr_dense_store(const BcrDenseJob* d_jobs, int njobs, int max_n,
                            const cpx<double>* dense, cpx<T>* fac, hipStream_t s);

// Batched FP64 complex GEMM on working blocks: C = beta C + alpha op(A) op(B),
// nb x nb column-major; op transposes when ta / tb is set; beta is 0 or 1.
struct ZGemmJob {
  int nb, ta, tb, beta;
  double alpha;
  long long a, b, c;
};
void launch_zgemm(const ZGemmJob* d_jobs, int njobs, int max_nb, cpx<double>* work, hipStream_t s);

// ---- a4: local right-hand sides and source transfer (pull)
// members are {subdomain, sweep}; the first sweep's right-hand side is f on own cells
template <typename T>
void launch_init_rhs(const Problem& P, const SubDesc* d_subs, const int2* d_members, int nmem,
                     long long max_nloc, int nrhs, int kmax, const cpx<double>* f, cpx<T>* rpool,
                     long long pool_stride, int src_slot, hipStream_t s);
template <typename T>
void launch_pull(const Problem& P, const SubDesc* d_subs, const int2* d_members, int nmem,
                 const Edge* d_edges, const int2* d_edge_range, long long max_box_cells,
                 int nrhs, int kmax, const cpx<T>* vpool, long long pool_stride,
                 const cpx<T>* diag, const cpx<T>* cx, const cpx<T>* cy, const cpx<T>* cz,
                 cpx<T>* rpool, hipStream_t s);

// ---- a5: u_DDM = sum_sub beta_0 sum_l v_sub^l (FP64, pull over global cells)
template <typename T>
void launch_assemble_u(const Problem& P, const SubDesc* d_subs, const PartTables& pt, int slot0,
                       int nslots, int accumulate, int nrhs, int kmax, const cpx<T>* vpool,
                       long long pool_stride, cpx<double>* u, hipStream_t s);
// p[0, n) = 0 (a kernel, so that graph captures hold no memset node)
template <typename T>
void launch_zero(cpx<T>* p, long long n, hipStream_t s);

// local solve entry point helpers: complex128 <-> plan precision on one subdomain
template <typename T>
void launch_pack_local(const cpx<double>* src, cpx<T>* dst, long long nloc, int nrhs, int kmax,
                       hipStream_t s);
template <typename T>
void launch_unpack_local(const cpx<T>* src, cpx<double>* dst, long long nloc, int nrhs, int kmax,
                         hipStream_t s);

// ---- a7: FP64 global operator
void launch_apply_op(const Problem& P, const cpx<double>* diag, const cpx<double>* cx,
                     const cpx<double>* cy, const cpx<double>* cz, const cpx<double>* x,
                     cpx<double>* y, int nrhs, hipStream_t s);

// ---- a8: FP64 Krylov vector kernels
// out[i][r] = sum_c conj(V[i][r][c]) w[r][c] for i < nv; V rows are [nrhs][N] blocks of
// a basis laid out [nv_total][nrhs][N]; partial sums go to `part` ([nv][nrhs][nblk]).
void launch_mdot(const cpx<double>* V, int nv, const cpx<double>* w, int nrhs, long long N,
                 cpx<double>* part, int nblk, cpx<double>* out, hipStream_t s);
// w[r] += sign * sum_{i<nv} coef[i][r] V[i][r]
void launch_maxpy(const cpx<double>* V, int nv, const cpx<double>* coef, double sign,
                  cpx<double>* w, int nrhs, long long N, hipStream_t s);
// dst[r] = src[r] * scal[r] (scal real, per RHS)
void launch_scale(const cpx<double>* src, const double* scal, cpx<double>* dst, int nrhs,
                  long long N, hipStream_t s);
// y = a - b
void launch_sub(const cpx<double>* a, const cpx<double>* b, cpx<double>* y, long long n,
                hipStream_t s);
void launch_conj(const cpx<double>* a, cpx<double>* y, long long n, hipStream_t s);
// dst[idx[r]] = 0 for r < nsel (rows of N entries)
void launch_zero_rhs(cpx<double>* dst, const int* idx, int nsel, long long N, hipStream_t s);
// gather / scatter RHS subsets: dst[r] = src[idx[r]] (and the reverse)
void launch_gather_rhs(const cpx<double>* src, const int* idx, cpx<double>* dst, int nsel,
                       long long N, hipStream_t s);
void launch_scatter_rhs(const cpx<double>* src, const int* idx, cpx<double>* dst, int nsel,
                        long long N, hipStream_t s);

// ---- a9: FWI
void launch_fwi_residual(const cpx<double>* u, int nsrc, long long N, const long long* rec,
                         int nrec, const cpx<double>* dobs, cpx<double>* res,
                         cpx<double>* adj_rhs, double* misfit_part, hipStream_t s);
void launch_fwi_gradient(const Problem& P, const cpx<double>* u, const cpx<double>* y, int nsrc,
                         double* grad, hipStream_t s);
void launch_sample(const cpx<double>* u, int nsrc, long long N, const long long* rec, int nrec,
                   cpx<double>* d, hipStream_t s);

}  // namespace dsd
