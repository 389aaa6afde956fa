// dsweep kernels for gfx950.
//
// Conventions: cells are indexed x fastest; a subdomain's local vectors for a
// batch of RHS are [rhs][cell] blocks of length nloc inside pools laid out by
// SubDesc::vec_off (times the plan's max RHS); complex values are interleaved.
#include "kernels.hpp"

#include <type_traits>

namespace dsd {

static inline unsigned cdiv_u(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

// ============================================================================
// a1: J-scaled coefficients of the 5/7-point PML operator on a list of grids.
// Face coefficient along axis a: prod_{b != a} s_b(centre) / s_a(face) / h^2;
// diagonal: minus the six (four) face coefficients plus omega^2 m prod_b s_b.
// ============================================================================
__global__ void k_assemble(Problem P, const AxisGrid* grids, const long long* offs, int ngrids,
                           const double* m, cpx<double>* diag, cpx<double>* cx,
                           cpx<double>* cy, cpx<double>* cz) {
  const int gi = blockIdx.y;
  const AxisGrid* ax = grids + 3 * gi;
  const long long ncell = (long long)ax[0].n * ax[1].n * ax[2].n;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  const int ix = (int)(c % ax[0].n);
  const long long r = c / ax[0].n;
  const int iy = (int)(r % ax[1].n);
  const int iz = (int)(r / ax[1].n);
  const int gx = ax[0].g0 + ix, gy = ax[1].g0 + iy, gz = ax[2].g0 + iz;
  const double h = P.h;
  const double inv_h2 = 1.0 / (h * h);
  auto s_at = [&](int a, double xphys) { return stretch(xphys, ax[a].lo, ax[a].hi, P); };
  const cpx<double> one = mk(1.0, 0.0);
  cpx<double> sxc = s_at(0, (gx - P.pml + 0.5) * h), sxl = s_at(0, (gx - P.pml) * h),
              sxh = s_at(0, (gx - P.pml + 1.0) * h);
  cpx<double> syc = s_at(1, (gy - P.pml + 0.5) * h), syl = s_at(1, (gy - P.pml) * h),
              syh = s_at(1, (gy - P.pml + 1.0) * h);
  cpx<double> szc = one, szl = one, szh = one;
  if (P.dim == 3) {
    szc = s_at(2, (gz - P.pml + 0.5) * h);
    szl = s_at(2, (gz - P.pml) * h);
    szh = s_at(2, (gz - P.pml + 1.0) * h);
  }
  // medium: clamp to the grid's undamped box, then to the physical cells
  auto clampi = [](int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); };
  const int px = clampi(gx, ax[0].clo, ax[0].chi) - P.pml;
  const int py = clampi(gy, ax[1].clo, ax[1].chi) - P.pml;
  const int pz = P.dim == 3 ? clampi(gz, ax[2].clo, ax[2].chi) - P.pml : 0;
  const double mm = m[((long long)pz * P.n[1] + py) * P.n[0] + px];

  const cpx<double> oyz = syc * szc, oxz = sxc * szc, oxy = sxc * syc;
  const cpx<double> axh = inv_h2 * cdiv(oyz, sxh), axl = inv_h2 * cdiv(oyz, sxl);
  const cpx<double> ayh = inv_h2 * cdiv(oxz, syh), ayl = inv_h2 * cdiv(oxz, syl);
  cpx<double> dg = -(axh + axl + ayh + ayl);
  cpx<double> azh = mk(0.0, 0.0);
  if (P.dim == 3) {
    azh = inv_h2 * cdiv(oxy, szh);
    const cpx<double> azl = inv_h2 * cdiv(oxy, szl);
    dg = dg - (azh + azl);
  }
  dg = dg + (P.omega * P.omega * mm) * (oxy * szc);
  const long long o = offs[gi] + c;
  diag[o] = dg;
  cx[o] = axh;
  cy[o] = ayh;
  cz[o] = azh;
}

void launch_assemble(const Problem& P, const AxisGrid* d_grids, const long long* d_offs, int ngrids,
                     long long max_cells, const double* d_m, cpx<double>* diag, cpx<double>* cx,
                     cpx<double>* cy, cpx<double>* cz, hipStream_t s) {
  dim3 grid(cdiv_u(max_cells, 256), ngrids);
  hipLaunchKernelGGL(k_assemble, grid, dim3(256), 0, s, P, d_grids, d_offs, ngrids, d_m, diag, cx,
                     cy, cz);
}

template <typename T>
__global__ void k_convert(const cpx<double>* src, cpx<T>* dst, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = cvt<T>(src[i]);
}
template <typename T>
void launch_convert(const cpx<double>* src, cpx<T>* dst, long long n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_convert<T>, dim3(cdiv_u(n, 256)), dim3(256), 0, s, src, dst, n);
}

// ============================================================================
// a2: factorisation.  Local operator in natural order is block tridiagonal
// with blocks A_k (one x-line in 2D, one xy-plane in 3D) and diagonal
// couplings C_k (the +y / +z face coefficients of block k).  Two chains of
// Schur complements run towards the middle block:
//   top    S_k = A_k - C_{k-1} S_{k-1}^{-1} C_{k-1}
//   bottom T_k = A_k - C_k T_{k+1}^{-1} C_k
//   middle M   = A_m - C_{m-1} S_{m-1}^{-1} C_{m-1} - C_m T_{m+1}^{-1} C_m
// formed and inverted in FP64, stored (rounded) in the plan precision.
// ============================================================================
__device__ inline cpx<double> block_entry(const SubDesc& S, int dim, int k, int i, int j,
                                          const cpx<double>* diag, const cpx<double>* cx,
                                          const cpx<double>* cy) {
  const long long base = S.coef_off + (long long)k * S.nb;
  if (i == j) return diag[base + i];
  if (dim == 2) {
    if (j == i + 1) return cx[base + i];
    if (i == j + 1) return cx[base + j];
    return mk(0.0, 0.0);
  }
  const int nx = S.dims[0];
  if (j == i + 1 && (i % nx) != nx - 1) return cx[base + i];
  if (i == j + 1 && (j % nx) != nx - 1) return cx[base + j];
  if (j == i + nx) return cy[base + i];
  if (i == j + nx) return cy[base + j];
  return mk(0.0, 0.0);
}

__global__ void k_schur(Problem P, const SubDesc* subs, const FactorJob* jobs,
                        const cpx<double>* diag, const cpx<double>* cx, const cpx<double>* cy,
                        const cpx<double>* cz, cpx<double>* scratch) {
  const FactorJob J = jobs[blockIdx.y];
  const SubDesc S = subs[J.sub];
  const int nb = S.nb;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)nb * nb) return;
  const int j = (int)(e / nb), i = (int)(e - (long long)j * nb);  // column-major
  const cpx<double>* cpl = P.dim == 2 ? cy : cz;
  cpx<double> v = block_entry(S, P.dim, J.k, i, j, diag, cx, cy);
  if (J.cp_blk >= 0) {
    const long long cb = S.coef_off + (long long)J.cp_blk * nb;
    v = v - (cpl[cb + i] * scratch[J.prev + e]) * cpl[cb + j];
  }
  if (J.cq_blk >= 0) {
    const long long cb = S.coef_off + (long long)J.cq_blk * nb;
    v = v - (cpl[cb + i] * scratch[J.prev2 + e]) * cpl[cb + j];
  }
  scratch[J.cur + e] = v;
}

void launch_schur(const Problem& P, const SubDesc* d_subs, const FactorJob* d_jobs, int njobs,
                  int max_nb, const cpx<double>* diag, const cpx<double>* cx,
                  const cpx<double>* cy, const cpx<double>* cz, cpx<double>* scratch,
                  hipStream_t s) {
  if (njobs <= 0) return;
  dim3 grid(cdiv_u((long long)max_nb * max_nb, 256), njobs);
  hipLaunchKernelGGL(k_schur, grid, dim3(256), 0, s, P, d_subs, d_jobs, diag, cx, cy, cz,
                     scratch);
}

// In-place inversion of the FP64 column-major n x n matrix a by blocked
// Gauss-Jordan elimination with partial (row) pivoting, one 1024-thread
// workgroup per matrix.  Panels of GJ_B columns are eliminated column by column
// (row interchanges applied to whole rows, rank-1 updates to the panel only);
// the rest of the matrix then takes the panel's transformation at once,
//   A[i, c] = [i not a pivot row of the panel] A[i, c] + sum_k P[i, k] R[k, c],
// with P the transformed panel and R the panel's pivot rows (copied to R
// first), as 64 x 64 tiled products on the FP64 matrix cores with operands
// staged in LDS.  The row interchanges are undone as column interchanges at
// the end.  LDS: tcol (max_n entries) and rowj (GJ_B), then the product tiles.
// Returns nonzero (in thread 0) for a zero pivot.
typedef double gj_f64x4 __attribute__((ext_vector_type(4)));
constexpr int GJ_B = 32;              // panel width
constexpr int GJ_TI = 64, GJ_TC = 64; // product tile: rows x columns

// One panel [j0, j1) of the elimination: its columns one by one (pivot search
// over rows >= j, whole-row interchange, rank-1 update of the panel columns),
// then, unless the panel is the whole matrix, R = the panel's pivot rows.
// 1024 threads; returns nonzero (in thread 0) for a zero pivot.
__device__ __forceinline__ int gj_panel(cpx<double>* a, const int n, const int j0, int* piv,
                                        cpx<double>* R, cpx<double>* tcol, cpx<double>* rowj,
                                        double* pst) {
  __shared__ double red_v[16];
  __shared__ int red_i[16];
  __shared__ int s_p;
  const int tid = threadIdx.x, bs = blockDim.x;
  const int lane = tid & 63, wid = tid >> 6, nw = bs >> 6;
  const int j1 = min(n, j0 + GJ_B), bw = j1 - j0;
  int bad = 0;
  for (int j = j0; j < j1; ++j) {
    // pivot: largest |a_ij| for i >= j (ties: smallest i)
    double bv = -1.0;
    int bi = n;
    for (int i = j + tid; i < n; i += bs) {
      const double v = abs2(a[(long long)j * n + i]);
      if (v > bv) { bv = v; bi = i; }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_down(bv, o, 64);
      const int oi = __shfl_down(bi, o, 64);
      if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
    }
    if (lane == 0) { red_v[wid] = bv; red_i[wid] = bi; }
    __syncthreads();
    if (tid == 0) {
      double v = red_v[0];
      int p = red_i[0];
      for (int w = 1; w < nw; ++w)
        if (red_v[w] > v || (red_v[w] == v && red_i[w] < p)) { v = red_v[w]; p = red_i[w]; }
      if (!(v > 0.0)) { bad = 1; p = j; }
      s_p = p;
      piv[j] = p;
      if (pst) {                    // smallest and largest squared pivot magnitude
        pst[0] = fmin(pst[0], v);
        pst[1] = fmax(pst[1], v);
      }
    }
    __syncthreads();
    const int p = s_p;
    if (p != j) {
      for (int c = tid; c < n; c += bs) {
        const cpx<double> t0 = a[(long long)c * n + j];
        a[(long long)c * n + j] = a[(long long)c * n + p];
        a[(long long)c * n + p] = t0;
      }
    }
    __syncthreads();
    for (int i = tid; i < n; i += bs) tcol[i] = a[(long long)j * n + i];
    __syncthreads();
    const cpx<double> pv = tcol[j];
    const cpx<double> pinv = (abs2(pv) > 0.0) ? cdiv(mk(1.0, 0.0), pv) : mk(0.0, 0.0);
    for (int c = j0 + tid; c < j1; c += bs)
      rowj[c - j0] = (c == j) ? pinv : a[(long long)c * n + j] * pinv;
    __syncthreads();
    // rank-1 update of the panel columns, one column per wave
    for (int c = j0 + wid; c < j1; c += nw) {
      cpx<double>* col = a + (long long)c * n;
      const cpx<double> rj = rowj[c - j0];
      for (int i0 = lane; i0 < n; i0 += 256) {
        cpx<double> v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = i0 + 64 * u;
          v[u] = i < n ? col[i] : mk(0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = i0 + 64 * u;
          if (i < n) {
            if (i == j) col[i] = rj;
            else if (c == j) col[i] = -(tcol[i] * pinv);
            else col[i] = v[u] - tcol[i] * rj;
          }
        }
      }
    }
    __syncthreads();
  }
  if (j1 >= n && j0 == 0) return bad;   // a single panel covers the matrix
  // R[c][k] = pivot row j0 + k at column c (all columns; panel ones unused)
  for (long long e = tid; e < (long long)bw * n; e += bs) {
    const int c = (int)(e / bw), k = (int)(e - (long long)c * bw);
    R[(long long)c * GJ_B + k] = a[(long long)c * n + j0 + k];
  }
  __syncthreads();
  return bad;
}

// One 64 x 64 tile (rows i0.., columns c0..) of the update of every column
// outside the panel, A = [not pivot row] A + P R, on the FP64 matrix cores
// (1024 threads).  Wave w owns the 16 x 16 block at rows 16 (w % 4), columns
// 16 (w / 4) of the tile; v_mfma_f64_16x16x4f64 takes A as lane l =
// (row l % 16, k l / 16), B as (k l / 16, column l % 16), and returns lane l,
// item j = (row 4 j + l / 16, column l % 16).  A complex product is four real
// ones: Re += Re P Re R - Im P Im R, Im += Re P Im R + Im P Re R.
__device__ __forceinline__ void gj_tile(cpx<double>* a, const int n, const int j0, const int j1,
                                        const cpx<double>* R, cpx<double>* Pt, cpx<double>* Rt,
                                        const int i0, const int c0) {
  const int tid = threadIdx.x, bs = blockDim.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int bw = j1 - j0;
  const int sr = (wid & 3) * 16, sc = (wid >> 2) * 16;
  const int l16 = lane & 15, l4 = lane >> 4;
  for (int e = tid; e < GJ_B * GJ_TI; e += bs) {
    const int k = e / GJ_TI, rr = e - k * GJ_TI;
    Pt[e] = (k < bw && i0 + rr < n) ? a[(long long)(j0 + k) * n + i0 + rr] : mk(0.0, 0.0);
  }
  for (int e = tid; e < GJ_B * GJ_TC; e += bs) {
    const int cc = e / GJ_B, k = e - cc * GJ_B;
    Rt[cc * (GJ_B + 1) + k] = (k < bw && c0 + cc < n) ? R[(long long)(c0 + cc) * GJ_B + k] : mk(0.0, 0.0);
  }
  __syncthreads();
  const int c = c0 + sc + l16;                       // this lane's output column
  const bool ccol = c < n && (c < j0 || c >= j1);
  const int ib = i0 + sr + l4;                       // this lane's rows: ib + 4 j
  gj_f64x4 cr, ci;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int i = ib + 4 * j;
    const bool ld = ccol && i < n && (i < j0 || i >= j1);
    const cpx<double> v = ld ? a[(long long)c * n + i] : mk(0.0, 0.0);
    cr[j] = v.re;
    ci[j] = v.im;
  }
  for (int kk = 0; kk < bw; kk += 4) {
    const cpx<double> pa = Pt[(kk + l4) * GJ_TI + sr + l16];
    const cpx<double> rb = Rt[(sc + l16) * (GJ_B + 1) + kk + l4];
    cr = __builtin_amdgcn_mfma_f64_16x16x4f64(pa.re, rb.re, cr, 0, 0, 0);
    ci = __builtin_amdgcn_mfma_f64_16x16x4f64(pa.re, rb.im, ci, 0, 0, 0);
    cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-pa.im, rb.im, cr, 0, 0, 0);
    ci = __builtin_amdgcn_mfma_f64_16x16x4f64(pa.im, rb.re, ci, 0, 0, 0);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int i = ib + 4 * j;
    if (ccol && i < n) a[(long long)c * n + i] = mk(cr[j], ci[j]);
  }
  __syncthreads();
}

// The row interchanges undone as column interchanges, in reverse order.
__device__ __forceinline__ void gj_unpermute(cpx<double>* a, const int n, const int* piv) {
  const int tid = threadIdx.x, bs = blockDim.x;
  for (int j = n - 1; j >= 0; --j) {
    const int p = piv[j];
    if (p != j) {
      for (int i = tid; i < n; i += bs) {
        const cpx<double> t0 = a[(long long)j * n + i];
        a[(long long)j * n + i] = a[(long long)p * n + i];
        a[(long long)p * n + i] = t0;
      }
    }
    __syncthreads();
  }
}

__device__ __forceinline__ int gj_blocked(cpx<double>* a, const int n, int* piv, cpx<double>* R,
                                          unsigned char* smem, const int max_n, double* pst) {
  cpx<double>* tcol = reinterpret_cast<cpx<double>*>(smem);
  cpx<double>* rowj = tcol + max_n;        // [GJ_B]
  cpx<double>* Pt = rowj + GJ_B;            // [GJ_B][GJ_TI]
  cpx<double>* Rt = Pt + GJ_B * GJ_TI;      // [GJ_TC][GJ_B + 1]
  int bad = 0;
  for (int j0 = 0; j0 < n; j0 += GJ_B) {
    const int j1 = min(n, j0 + GJ_B);
    bad |= gj_panel(a, n, j0, piv, R, tcol, rowj, pst);
    if (j1 >= n && j0 == 0) continue;
    const int nti = (n + GJ_TI - 1) / GJ_TI, ntc = (n + GJ_TC - 1) / GJ_TC;
    for (int tile = 0; tile < nti * ntc; ++tile) {
      const int i0 = (tile % nti) * GJ_TI, c0 = (tile / nti) * GJ_TC;
      if (c0 >= j0 && c0 + GJ_TC <= j1) continue;       // tile inside the panel (uniform)
      gj_tile(a, n, j0, j1, R, Pt, Rt, i0, c0);
    }
  }
  gj_unpermute(a, n, piv);
  return bad;
}

size_t gj_lds_bytes(int max_n) {
  return ((size_t)max_n + GJ_B + (size_t)GJ_B * GJ_TI + (size_t)GJ_TC * (GJ_B + 1)) * sizeof(cpx<double>);
}

// Split form for launches with few large matrices (the fused kernel would leave
// most compute units idle): per panel, one launch eliminates the panel of every
// matrix (one workgroup each) and one launch updates all tiles of all matrices
// (one workgroup per tile); a last launch undoes the interchanges and writes the
// inverse.  Every element goes through the same operations in the same order as
// in the fused kernel, so both forms give identical results.
struct GjView {
  cpx<double>* a;
  long long out;   // factor offset of the rounded inverse (-1: none)
  int n;
  int errval;      // written to err[job] for a zero pivot
};
__device__ inline GjView gj_view(const BcrInvJob* jobs, const SubDesc*, cpx<double>* base, int i) {
  const BcrInvJob J = jobs[i];
  return GjView{base + J.src, J.dst, J.nb, 1};
}
__device__ inline GjView gj_view(const FactorJob* jobs, const SubDesc* subs, cpx<double>* base,
                                 int i) {
  const FactorJob J = jobs[i];
  const SubDesc& S = subs[J.sub];
  return GjView{base + J.cur, S.fac_off + (long long)J.k * S.nb * S.nb, S.nb, J.sub + 1};
}

template <typename JOB>
__global__ __launch_bounds__(1024) void k_gj_panel(const JOB* jobs, const SubDesc* subs,
                                                   cpx<double>* base, int* pivbuf,
                                                   cpx<double>* rbuf, int* err, double* pstat,
                                                   int j0, int max_n) {
  const GjView V = gj_view(jobs, subs, base, blockIdx.x);
  if (j0 >= V.n) return;
  extern __shared__ unsigned char smem_raw[];
  cpx<double>* tcol = reinterpret_cast<cpx<double>*>(smem_raw);
  const int bad = gj_panel(V.a, V.n, j0, pivbuf + (long long)blockIdx.x * max_n,
                           rbuf + (long long)blockIdx.x * GJ_B * max_n, tcol, tcol + max_n,
                           pstat ? pstat + 2 * blockIdx.x : nullptr);
  if (threadIdx.x == 0 && bad) err[blockIdx.x] = V.errval;
}

template <typename JOB>
__global__ __launch_bounds__(1024) void k_gj_update(const JOB* jobs, const SubDesc* subs,
                                                    cpx<double>* base, const cpx<double>* rbuf,
                                                    int j0, int max_n) {
  const GjView V = gj_view(jobs, subs, base, blockIdx.y);
  const int n = V.n, j1 = min(n, j0 + GJ_B);
  if (j0 >= n || (j1 >= n && j0 == 0)) return;
  const int nti = (n + GJ_TI - 1) / GJ_TI, ntc = (n + GJ_TC - 1) / GJ_TC;
  const int tile = blockIdx.x;
  if (tile >= nti * ntc) return;
  const int i0 = (tile % nti) * GJ_TI, c0 = (tile / nti) * GJ_TC;
  if (c0 >= j0 && c0 + GJ_TC <= j1) return;
  extern __shared__ unsigned char smem_raw[];
  cpx<double>* Pt = reinterpret_cast<cpx<double>*>(smem_raw);
  gj_tile(V.a, n, j0, j1, rbuf + (long long)blockIdx.y * GJ_B * max_n, Pt, Pt + GJ_B * GJ_TI, i0, c0);
}

template <typename T, typename JOB>
__global__ __launch_bounds__(1024) void k_gj_finish(const JOB* jobs, const SubDesc* subs,
                                                    cpx<double>* base, const int* pivbuf,
                                                    cpx<T>* fac, int max_n) {
  const GjView V = gj_view(jobs, subs, base, blockIdx.x);
  gj_unpermute(V.a, V.n, pivbuf + (long long)blockIdx.x * max_n);
  if (V.out >= 0) {
    const long long ne = (long long)V.n * V.n;
    for (long long e = threadIdx.x; e < ne; e += blockDim.x) fac[V.out + e] = cvt<T>(V.a[e]);
  }
}

// The split form pays when the launch has fewer matrices than compute units
// and each matrix has many tiles.
static inline bool gj_use_split(int njobs, int max_n) { return njobs < 256 && max_n > 256; }

template <typename T, typename JOB>
static void launch_gj_split(const JOB* d_jobs, const SubDesc* d_subs, int njobs, int max_n,
                            cpx<double>* base, cpx<T>* fac, int* d_err, int* d_piv,
                            cpx<double>* d_rbuf, double* d_pst, hipStream_t s) {
  const int nt = (max_n + GJ_TI - 1) / GJ_TI;
  const size_t lds_panel = ((size_t)max_n + GJ_B) * sizeof(cpx<double>);
  const size_t lds_tile = ((size_t)GJ_B * GJ_TI + (size_t)GJ_TC * (GJ_B + 1)) * sizeof(cpx<double>);
  for (int j0 = 0; j0 < max_n; j0 += GJ_B) {
    hipLaunchKernelGGL(k_gj_panel<JOB>, dim3(njobs), dim3(1024), lds_panel, s, d_jobs, d_subs, base,
                       d_piv, d_rbuf, d_err, d_pst, j0, max_n);
    hipLaunchKernelGGL(k_gj_update<JOB>, dim3(nt * nt, njobs), dim3(1024), lds_tile, s, d_jobs,
                       d_subs, base, d_rbuf, j0, max_n);
  }
  hipLaunchKernelGGL((k_gj_finish<T, JOB>), dim3(njobs), dim3(1024), 0, s, d_jobs, d_subs, base,
                     d_piv, fac, max_n);
}

// Inversion of the Schur block at scratch[cur] (one workgroup per job); the
// inverse is then rounded into the factor slot of block k.
template <typename T>
__global__ __launch_bounds__(1024) void k_invert(const SubDesc* subs, const FactorJob* jobs,
                                                 cpx<double>* scratch, cpx<T>* fac, int* err,
                                                 int* pivbuf, cpx<double>* rbuf, double* pstat,
                                                 int max_nb) {
  const FactorJob J = jobs[blockIdx.x];
  const SubDesc S = subs[J.sub];
  const int nb = S.nb;
  cpx<double>* a = scratch + J.cur;
  extern __shared__ unsigned char smem_raw[];
  const int bad = gj_blocked(a, nb, pivbuf + (long long)blockIdx.x * max_nb,
                             rbuf + (long long)blockIdx.x * GJ_B * max_nb, smem_raw, max_nb,
                             pstat ? pstat + 2 * blockIdx.x : nullptr);
  cpx<T>* out = fac + S.fac_off + (long long)J.k * nb * nb;
  const long long ne = (long long)nb * nb;
  for (long long e = threadIdx.x; e < ne; e += blockDim.x) out[e] = cvt<T>(a[e]);
  if (threadIdx.x == 0 && bad) err[blockIdx.x] = J.sub + 1;
}

size_t gj_rbuf_entries(int max_n) { return (size_t)GJ_B * max_n; }

template <typename T>
void launch_invert(const SubDesc* d_subs, const FactorJob* d_jobs, int njobs, int max_nb,
                   cpx<double>* scratch, cpx<T>* fac, int* d_err, int* d_piv, cpx<double>* d_rbuf,
                   double* d_pst, hipStream_t s) {
  if (njobs <= 0) return;
  if (gj_use_split(njobs, max_nb)) {
    launch_gj_split<T, FactorJob>(d_jobs, d_subs, njobs, max_nb, scratch, fac, d_err, d_piv, d_rbuf,
                                  d_pst, s);
    return;
  }
  hipLaunchKernelGGL(k_invert<T>, dim3(njobs), dim3(1024), gj_lds_bytes(max_nb), s, d_subs, d_jobs,
                     scratch, fac, d_err, d_piv, d_rbuf, d_pst, max_nb);
}

// ============================================================================
// a3: subdomain solves.  With B_k the stored inverse Schur blocks and c_k the
// coupling of blocks k and k+1:
//   forward top    y_k = r_k - c_{k-1} w_{k-1},  w_k = B_k y_k        (k < m)
//   forward bottom y_k = r_k - c_k w_{k+1},      w_k = B_k y_k        (k > m)
//   middle         x_m = B_m (r_m - c_{m-1} w_{m-1} - c_m w_{m+1})
//   backward top    x_k = w_k - B_k (c_k x_{k+1})                      (k < m)
//   backward bottom x_k = w_k - B_k (c_{k-1} x_{k-1})                  (k > m)
// One workgroup (8 waves) runs one chain (subdomain, half, sweep) for KG
// right-hand sides.  A block step is a dense (nb x nb) x (nb x KG) product:
// the eight waves split the columns of B_k (each lane owns rows lane + 64 t
// of a 256-row chunk, loads are coalesced 64-element column segments issued
// eight columns deep), partial sums meet in LDS.  Workgroups of one chain
// (different RHS groups) are placed on one XCD so that B_k is shared in L2.
// ============================================================================
constexpr int CH_WAVES = 8;
constexpr int CH_THREADS = 64 * CH_WAVES;
constexpr int CH_ROUND_BYTES = 96;   // bytes of B per lane and row tile in one round

template <typename T> struct vec2;
template <> struct vec2<float> { typedef float2 type; };
template <> struct vec2<double> { typedef double2 type; };

// Block index processed at step t of a chain phase.
__device__ __forceinline__ int chain_block(int phase, int half, int t, int nblk, int mid) {
  if (phase == 0) return half == 0 ? t : nblk - 1 - t;
  if (phase == 1) return mid;
  return half == 0 ? mid - 1 - t : mid + 1 + t;
}

// Workgroup barrier that orders LDS only: waits for this wave's LDS operations
// and meets the other waves, leaving global loads (prefetches) and stores in
// flight.  Used where the data exchanged between waves lives in LDS and no
// global location is written and then read inside the kernel.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

template <typename T, int KG, int RT>
__global__ __launch_bounds__(CH_THREADS) void k_chain(int phase, const SubDesc* __restrict__ subs,
                                                      const int4* __restrict__ jobs, int njobs,
                                                      int G, int nrhs, int kmax,
                                                      const cpx<T>* __restrict__ fac,
                                                      const cpx<T>* __restrict__ cpl,
                                                      const cpx<T>* __restrict__ rpool,
                                                      cpx<T>* __restrict__ vpool,
                                                      long long pool_stride) {
  typedef typename vec2<T>::type V2;
  constexpr int U = CH_ROUND_BYTES / (int)sizeof(V2);   // columns per round
  constexpr int ROWS = 64 * RT;                          // rows per chunk
  const int total = gridDim.x;
  const int per = total >> 3;
  const int b = blockIdx.x;
  const int Lg = (b & 7) * per + (b >> 3);
  const int job = Lg / G, g = Lg - (Lg / G) * G;
  if (job >= njobs) return;
  const int4 jb = jobs[job];
  const SubDesc S = subs[jb.x];
  const int half = jb.y;
  const int nb = S.nb, nblk = S.nblk, mid = S.mid;
  const long long nloc = S.nloc, nb2 = (long long)nb * nb;
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* yin = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* prev = yin + (long long)nb * KG;
  cpx<T>* red = prev + (long long)nb * KG;              // [CH_WAVES][KG][ROWS]
  const cpx<T>* __restrict__ R = rpool + (long long)jb.z * pool_stride + S.vec_off * kmax;
  cpx<T>* __restrict__ X = vpool + (long long)jb.z * pool_stride + S.vec_off * kmax;
  const cpx<T>* __restrict__ C = cpl + S.coef_off;
  const V2* __restrict__ Bv = reinterpret_cast<const V2*>(fac + S.fac_off);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const cpx<T> zero = mk((T)0, (T)0);
  const int nsteps = phase == 1 ? 1 : (half == 0 ? mid : nblk - 1 - mid);
  if (nsteps <= 0) return;
  const int cw = (nb + CH_WAVES - 1) / CH_WAVES;
  const int j0 = w * cw;
  const int j1 = min(nb, j0 + cw);
  const int nr = (cw + U - 1) / U;                       // rounds per chunk (same for all waves)
  const int nchunk = (nb + ROWS - 1) / ROWS;
  const int per_step = nchunk * nr;                      // rounds per block step
  const int total_rounds = nsteps * per_step;

  // Issue the loads of round `gr` (a position in the whole chain's column stream).
  auto issue = [&](V2 (&buf)[U][RT], int gr) {
    const int t = gr / per_step, rem = gr - t * per_step;
    const int ch = rem / nr, rd = rem - ch * nr;
    const int k = chain_block(phase, half, t, nblk, mid);
    const V2* __restrict__ Bk = Bv + k * nb2;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int jc = j0 + rd * U + u;
      jc = jc < j1 ? jc : (j1 > j0 ? j1 - 1 : 0);
#pragma unroll
      for (int tt = 0; tt < RT; ++tt) {
        int row = ch * ROWS + tt * 64 + lane;
        row = row < nb ? row : nb - 1;
        buf[u][tt] = Bk[(long long)jc * nb + row];
      }
    }
  };

  V2 cur[U][RT], nxt[U][RT];
  issue(cur, 0);
  int gr = 0;
  for (int t = 0; t < nsteps; ++t) {
    const int k = chain_block(phase, half, t, nblk, mid);
    // ---- right-hand side of this block step into yin
    for (int idx = tid; idx < nb * KG; idx += CH_THREADS) {
      const int q = idx / nb, i = idx - q * nb;
      const int rq = g * KG + q;
      cpx<T> y = zero;
      if (phase == 0) {
        y = rq < nrhs ? R[(long long)rq * nloc + (long long)k * nb + i] : zero;
        if (t > 0) {
          const cpx<T> c = half == 0 ? C[(long long)(k - 1) * nb + i] : C[(long long)k * nb + i];
          y = y - c * prev[q * nb + i];
        }
      } else if (phase == 1) {
        if (rq < nrhs) {
          const long long ro = (long long)rq * nloc;
          y = R[ro + (long long)k * nb + i];
          if (k > 0) y = y - C[(long long)(k - 1) * nb + i] * X[ro + (long long)(k - 1) * nb + i];
          if (k < nblk - 1) y = y - C[(long long)k * nb + i] * X[ro + (long long)(k + 1) * nb + i];
        }
      } else {
        const int kn = half == 0 ? k + 1 : k - 1;
        const int cb = half == 0 ? k : k - 1;
        cpx<T> xn;
        if (t == 0) xn = rq < nrhs ? X[(long long)rq * nloc + (long long)kn * nb + i] : zero;
        else xn = prev[q * nb + i];
        y = C[(long long)cb * nb + i] * xn;
      }
      yin[q * nb + i] = y;
    }
    lds_barrier();
    for (int ch = 0; ch < nchunk; ++ch) {
      T ar[RT][KG], ai[RT][KG];
#pragma unroll
      for (int tt = 0; tt < RT; ++tt)
#pragma unroll
        for (int q = 0; q < KG; ++q) { ar[tt][q] = (T)0; ai[tt][q] = (T)0; }
      for (int rd = 0; rd < nr; ++rd, ++gr) {
        if (gr + 1 < total_rounds) issue(nxt, gr + 1);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int j = j0 + rd * U + u;
          const bool ok = j < j1;
          const int jc = ok ? j : 0;
#pragma unroll
          for (int q = 0; q < KG; ++q) {
            const cpx<T> y = yin[q * nb + jc];
            const T yr = ok ? y.re : (T)0, yi = ok ? y.im : (T)0;
#pragma unroll
            for (int tt = 0; tt < RT; ++tt) {
              ar[tt][q] = fma(cur[u][tt].x, yr, ar[tt][q]);
              ar[tt][q] = fma(-cur[u][tt].y, yi, ar[tt][q]);
              ai[tt][q] = fma(cur[u][tt].x, yi, ai[tt][q]);
              ai[tt][q] = fma(cur[u][tt].y, yr, ai[tt][q]);
            }
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int tt = 0; tt < RT; ++tt) cur[u][tt] = nxt[u][tt];
      }
#pragma unroll
      for (int tt = 0; tt < RT; ++tt)
#pragma unroll
        for (int q = 0; q < KG; ++q)
          red[(w * KG + q) * ROWS + tt * 64 + lane] = mk(ar[tt][q], ai[tt][q]);
      lds_barrier();
      for (int o = tid; o < KG * ROWS; o += CH_THREADS) {
        const int q = o / ROWS, il = o - q * ROWS, i = ch * ROWS + il;
        if (i >= nb) continue;
        cpx<T> out = zero;
#pragma unroll
        for (int ww = 0; ww < CH_WAVES; ++ww) out = out + red[(ww * KG + q) * ROWS + il];
        const int rq = g * KG + q;
        const long long oo = (long long)rq * nloc + (long long)k * nb + i;
        if (phase == 2) out = (rq < nrhs ? X[oo] : zero) - out;
        prev[q * nb + i] = out;
        if (rq < nrhs) X[oo] = out;
      }
      lds_barrier();
    }
  }
}

// Complex64 variant on the matrix cores.  v_mfma_f32_4x4x1f32 computes 16
// independent 4x4 outer products: lane 4b+i supplies A[b][i], lane 4b+j
// supplies B[b][j] and holds D[b][i][j] in accumulator register i.  Here the
// 16 blocks are 16 groups of 4 rows of a 64-row tile (A = one factor element
// per lane: Re in one product, Im in the other) and the 4 columns of a block
// are (Re, Im) of two right-hand sides, so
//   D += Re(B) (x) [yr0, yi0, yr1, yi1] + Im(B) (x) [-yi0, yr0, -yi1, yr1]
// accumulates the complex product without waste.
typedef float mf4 __attribute__((ext_vector_type(4)));

template <int KG, int RT>
__global__ __launch_bounds__(CH_THREADS) void k_chain_mfma(int phase, const SubDesc* __restrict__ subs,
                                                           const int4* __restrict__ jobs, int njobs,
                                                           int G, int nrhs, int kmax,
                                                           const cpx<float>* __restrict__ fac,
                                                           const cpx<float>* __restrict__ cpl,
                                                           const cpx<float>* __restrict__ rpool,
                                                           cpx<float>* __restrict__ vpool,
                                                           long long pool_stride) {
  typedef float2 V2;
  typedef cpx<float> C;
  constexpr int U = CH_ROUND_BYTES / (int)sizeof(V2);   // columns per round (12)
  constexpr int NG = KG / 2;                             // RHS pairs
  constexpr int ROWS = 64 * RT;
  constexpr int PF = (KG * 256 + CH_THREADS - 1) / CH_THREADS;   // vector elements per thread
  const int total = gridDim.x;
  const int per = total >> 3;
  const int b = blockIdx.x;
  const int Lg = (b & 7) * per + (b >> 3);
  const int job = Lg / G, g = Lg - (Lg / G) * G;
  if (job >= njobs) return;
  const int4 jb = jobs[job];
  const SubDesc S = subs[jb.x];
  const int half = jb.y;
  const int nb = S.nb, nblk = S.nblk, mid = S.mid;
  const long long nloc = S.nloc, nb2 = (long long)nb * nb;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int cw = (nb + CH_WAVES - 1) / CH_WAVES;
  int nr = (cw + U - 1) / U;
  nr += nr & 1;                                          // even: chunks start in buffer A
  const int ncol = CH_WAVES * nr * U;                    // padded column count of the operands
  extern __shared__ unsigned char smem_raw[];
  V2* yop = reinterpret_cast<V2*>(smem_raw);            // [NG][ncol][4] MFMA B-operand pairs
  C* prev = reinterpret_cast<C*>(yop + (long long)NG * ncol * 4);   // [KG][nb]
  float* redf = reinterpret_cast<float*>(prev + (long long)KG * nb); // [W][RT][NG][4][64]
  const C* __restrict__ R = rpool + (long long)jb.z * pool_stride + S.vec_off * kmax;
  C* __restrict__ X = vpool + (long long)jb.z * pool_stride + S.vec_off * kmax;
  const C* __restrict__ Cp = cpl + S.coef_off;
  const V2* __restrict__ Bv = reinterpret_cast<const V2*>(fac + S.fac_off);
  const C zero = mk(0.f, 0.f);
  const int nsteps = phase == 1 ? 1 : (half == 0 ? mid : nblk - 1 - mid);
  if (nsteps <= 0) return;
  const int j0 = w * cw;
  const int j1 = min(nb, j0 + cw);
  const int nchunk = (nb + ROWS - 1) / ROWS;

  // Operand slots: wave w owns slots [w * nr * U, (w + 1) * nr * U); slot
  // w * nr * U + l holds column j0 + l for l < cw (and j0 + l < nb).  The
  // other slots stay zero, so padded rounds add nothing.
  const int nru = nr * U;
  for (int idx = tid; idx < NG * ncol * 4; idx += CH_THREADS) yop[idx] = make_float2(0.f, 0.f);
  __syncthreads();

  // column stream position of the next issue: (step, chunk, round)
  int is_t = 0, is_ch = 0, is_rd = 0;
  auto issue = [&](V2 (&buf)[U][RT]) {
    if (is_t < nsteps) {
      const int k = chain_block(phase, half, is_t, nblk, mid);
      const V2* __restrict__ Bk = Bv + k * nb2;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        int jc = j0 + is_rd * U + u;
        jc = jc < j1 ? jc : (j1 > j0 ? j1 - 1 : 0);
        const V2* __restrict__ col = Bk + (long long)jc * nb;
#pragma unroll
        for (int tt = 0; tt < RT; ++tt) {
          int row = is_ch * ROWS + tt * 64 + lane;
          row = row < nb ? row : nb - 1;
          buf[u][tt] = col[row];
        }
      }
    }
    if (++is_rd == nr) { is_rd = 0; if (++is_ch == nchunk) { is_ch = 0; ++is_t; } }
  };
  auto compute = [&](const V2 (&buf)[U][RT], int rd, mf4 (&acc)[RT][NG]) {
    const int sb0 = w * nru + rd * U;
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int ng = 0; ng < NG; ++ng) {
        const V2 y = yop[((long long)ng * ncol + sb0 + u) * 4 + (lane & 3)];
#pragma unroll
        for (int tt = 0; tt < RT; ++tt) {
          acc[tt][ng] = __builtin_amdgcn_mfma_f32_4x4x1f32(buf[u][tt].x, y.x, acc[tt][ng], 0, 0, 0);
          acc[tt][ng] = __builtin_amdgcn_mfma_f32_4x4x1f32(buf[u][tt].y, y.y, acc[tt][ng], 0, 0, 0);
        }
      }
    }
  };
  // Store the block step's input y(q, i) as MFMA operands: slot 2(q&1) holds
  // (Re y, -Im y), slot 2(q&1)+1 holds (Im y, Re y).
  auto put_y = [&](int q, int i, C y) {
    const int slot = (i / cw) * nru + (i - (i / cw) * cw);
    V2* o = yop + ((long long)(q >> 1) * ncol + slot) * 4 + 2 * (q & 1);
    o[0] = make_float2(y.re, -y.im);
    o[1] = make_float2(y.im, y.re);
  };

  // prefetched inputs of the next step's right-hand side (phases 0 and 2)
  C pre_r[PF], pre_c[PF];
  auto prefetch_rhs = [&](int t) {
    const int k = chain_block(phase, half, t, nblk, mid);
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      const int idx = tid + p * CH_THREADS;
      pre_r[p] = zero;
      pre_c[p] = zero;
      if (idx < nb * KG && t < nsteps) {
        const int q = idx / nb, i = idx - q * nb;
        const int rq = g * KG + q;
        if (phase == 0) {
          if (rq < nrhs) pre_r[p] = R[(long long)rq * nloc + (long long)k * nb + i];
          if (t > 0) pre_c[p] = half == 0 ? Cp[(long long)(k - 1) * nb + i] : Cp[(long long)k * nb + i];
        } else if (phase == 2) {
          pre_c[p] = Cp[(long long)(half == 0 ? k : k - 1) * nb + i];
          if (t == 0) {
            const int kn = half == 0 ? k + 1 : k - 1;
            pre_r[p] = rq < nrhs ? X[(long long)rq * nloc + (long long)kn * nb + i] : zero;
          }
        }
      }
    }
  };

  V2 bufA[U][RT], bufB[U][RT];
  issue(bufA);
  if (phase != 1) prefetch_rhs(0);
  for (int t = 0; t < nsteps; ++t) {
    const int k = chain_block(phase, half, t, nblk, mid);
    // ---- right-hand side of this block step as MFMA operands
    if (phase == 1) {
      for (int idx = tid; idx < nb * KG; idx += CH_THREADS) {
        const int q = idx / nb, i = idx - q * nb;
        const int rq = g * KG + q;
        C y = zero;
        if (rq < nrhs) {
          const long long ro = (long long)rq * nloc;
          y = R[ro + (long long)k * nb + i];
          if (k > 0) y = y - Cp[(long long)(k - 1) * nb + i] * X[ro + (long long)(k - 1) * nb + i];
          if (k < nblk - 1) y = y - Cp[(long long)k * nb + i] * X[ro + (long long)(k + 1) * nb + i];
        }
        put_y(q, i, y);
      }
    } else {
#pragma unroll
      for (int p = 0; p < PF; ++p) {
        const int idx = tid + p * CH_THREADS;
        if (idx < nb * KG) {
          const int q = idx / nb, i = idx - q * nb;
          C y;
          if (phase == 0) y = t > 0 ? pre_r[p] - pre_c[p] * prev[q * nb + i] : pre_r[p];
          else y = pre_c[p] * (t == 0 ? pre_r[p] : prev[q * nb + i]);
          put_y(q, i, y);
        }
      }
      // blocks wider than the prefetch covers (nb > 256): the rest directly
      for (int idx = PF * CH_THREADS + tid; idx < nb * KG; idx += CH_THREADS) {
        const int q = idx / nb, i = idx - q * nb;
        const int rq = g * KG + q;
        C y = zero;
        if (phase == 0) {
          const C r = rq < nrhs ? R[(long long)rq * nloc + (long long)k * nb + i] : zero;
          if (t > 0) {
            const C c = half == 0 ? Cp[(long long)(k - 1) * nb + i] : Cp[(long long)k * nb + i];
            y = r - c * prev[q * nb + i];
          } else {
            y = r;
          }
        } else {
          const C c = Cp[(long long)(half == 0 ? k : k - 1) * nb + i];
          C xin;
          if (t == 0) {
            const int kn = half == 0 ? k + 1 : k - 1;
            xin = rq < nrhs ? X[(long long)rq * nloc + (long long)kn * nb + i] : zero;
          } else {
            xin = prev[q * nb + i];
          }
          y = c * xin;
        }
        put_y(q, i, y);
      }
    }
    lds_barrier();
    if (phase != 1 && t + 1 < nsteps) prefetch_rhs(t + 1);
    for (int ch = 0; ch < nchunk; ++ch) {
      // w_k of the outputs this thread will write (backward phase)
      C pre_x[PF];
#pragma unroll
      for (int p = 0; p < PF; ++p) {
        pre_x[p] = zero;
        const int o = tid + p * CH_THREADS;
        if (phase == 2 && o < KG * ROWS) {
          const int q = o / ROWS, i = ch * ROWS + (o - q * ROWS);
          const int rq = g * KG + q;
          if (i < nb && rq < nrhs) pre_x[p] = X[(long long)rq * nloc + (long long)k * nb + i];
        }
      }
      mf4 acc[RT][NG];
#pragma unroll
      for (int tt = 0; tt < RT; ++tt)
#pragma unroll
        for (int ng = 0; ng < NG; ++ng) acc[tt][ng] = mf4{0.f, 0.f, 0.f, 0.f};
      for (int rd = 0; rd < nr; rd += 2) {
        issue(bufB);
        compute(bufA, rd, acc);
        issue(bufA);
        compute(bufB, rd + 1, acc);
      }
      // D[b][i][jj] of lane 4b+jj, register i  ->  redf[w][tt][ng][i][lane]
#pragma unroll
      for (int tt = 0; tt < RT; ++tt)
#pragma unroll
        for (int ng = 0; ng < NG; ++ng)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            redf[((((long long)w * RT + tt) * NG + ng) * 4 + i) * 64 + lane] = acc[tt][ng][i];
      lds_barrier();
#pragma unroll
      for (int p = 0; p < PF; ++p) {
        const int o = tid + p * CH_THREADS;
        if (o >= KG * ROWS) continue;
        const int q = o / ROWS, il = o - q * ROWS, i = ch * ROWS + il;
        if (i >= nb) continue;
        const int tt = il >> 6, r64 = il & 63;
        const int src = 4 * (r64 >> 2) + 2 * (q & 1);   // lane holding (row, q, Re); Im is next
        const int ii = r64 & 3, ng = q >> 1;
        C out = zero;
#pragma unroll
        for (int ww = 0; ww < CH_WAVES; ++ww) {
          const float* rb = redf + ((((long long)ww * RT + tt) * NG + ng) * 4 + ii) * 64 + src;
          out.re += rb[0];
          out.im += rb[1];
        }
        const int rq = g * KG + q;
        if (phase == 2) out = pre_x[p] - out;
        prev[q * nb + i] = out;
        if (rq < nrhs) X[(long long)rq * nloc + (long long)k * nb + i] = out;
      }
      lds_barrier();
    }
  }
}

template <typename T>
size_t chain_lds_bytes(int max_nb, int kg) {
  const int rows = max_nb <= 192 ? 192 : 256;
  if (std::is_same<T, float>::value && kg >= 2) {
    const int U = CH_ROUND_BYTES / 8;
    const int cw = (max_nb + CH_WAVES - 1) / CH_WAVES;
    int nr = (cw + U - 1) / U;
    nr += nr & 1;
    const size_t ncol = (size_t)CH_WAVES * nr * U;
    return (size_t)(kg / 2) * ncol * 4 * sizeof(float2) + (size_t)kg * max_nb * sizeof(cpx<float>) +
           (size_t)CH_WAVES * rows * (kg / 2) * 4 * sizeof(float);
  }
  return (size_t)(2 * max_nb + CH_WAVES * rows) * kg * sizeof(cpx<T>);
}

template <typename T, int KG, int RT>
static void launch_chain_kg(int phase, const SubDesc* d_subs, const int4* d_jobs, int njobs,
                            int nrhs, int kmax, int max_nb, const cpx<T>* fac, const cpx<T>* cpl,
                            const cpx<T>* rpool, cpx<T>* vpool, long long pool_stride,
                            hipStream_t s) {
  const int G = (nrhs + KG - 1) / KG;
  long long total = (long long)njobs * G;
  total = (total + 7) / 8 * 8;
  if constexpr (std::is_same<T, float>::value && KG >= 2) {
    hipLaunchKernelGGL((k_chain_mfma<KG, RT>), dim3((unsigned)total), dim3(CH_THREADS),
                       chain_lds_bytes<T>(max_nb, KG), s, phase, d_subs, d_jobs, njobs, G, nrhs,
                       kmax, fac, cpl, rpool, vpool, pool_stride);
  } else {
    hipLaunchKernelGGL((k_chain<T, KG, RT>), dim3((unsigned)total), dim3(CH_THREADS),
                       chain_lds_bytes<T>(max_nb, KG), s, phase, d_subs, d_jobs, njobs, G, nrhs,
                       kmax, fac, cpl, rpool, vpool, pool_stride);
  }
}

template <typename T, int RT>
static void launch_chain_rt(int kg, int phase, const SubDesc* d_subs, const int4* d_jobs,
                            int njobs, int nrhs, int kmax, int max_nb, const cpx<T>* fac,
                            const cpx<T>* cpl, const cpx<T>* rpool, cpx<T>* vpool,
                            long long pool_stride, hipStream_t s) {
  switch (kg) {
    case 1: launch_chain_kg<T, 1, RT>(phase, d_subs, d_jobs, njobs, nrhs, kmax, max_nb, fac, cpl, rpool, vpool, pool_stride, s); break;
    case 2: launch_chain_kg<T, 2, RT>(phase, d_subs, d_jobs, njobs, nrhs, kmax, max_nb, fac, cpl, rpool, vpool, pool_stride, s); break;
    default: launch_chain_kg<T, 4, RT>(phase, d_subs, d_jobs, njobs, nrhs, kmax, max_nb, fac, cpl, rpool, vpool, pool_stride, s); break;
  }
}

template <typename T>
void launch_chain(int kg, int phase, const SubDesc* d_subs, const int4* d_jobs, int njobs,
                  int nrhs, int kmax, int max_nb, const cpx<T>* fac, const cpx<T>* cpl,
                  const cpx<T>* rpool, cpx<T>* vpool, long long pool_stride, hipStream_t s) {
  if (njobs <= 0 || nrhs <= 0) return;
  if (max_nb <= 192)
    launch_chain_rt<T, 3>(kg, phase, d_subs, d_jobs, njobs, nrhs, kmax, max_nb, fac, cpl, rpool, vpool, pool_stride, s);
  else
    launch_chain_rt<T, 4>(kg, phase, d_subs, d_jobs, njobs, nrhs, kmax, max_nb, fac, cpl, rpool, vpool, pool_stride, s);
}

// ============================================================================
// a2/a3, block cyclic reduction.  The local operator is block tridiagonal
// (blocks A_k, couplings C_k = diag(c_k) between blocks k and k+1).  Level
// by level the even-position blocks of the remaining system are eliminated:
//   P_i = D_i^{-1};  D'_j = D_j - E_{j-1}^T P_{j-1} E_{j-1} - E_j P_{j+1} E_j^T;
//   E'_j = -E_j P_{j+1} E_{j+1}   (coupling of the kept neighbours j, j+2).
// Forward solve: z_i = P_i r_i, r'_j = r_j - E_{j-1}^T z_{j-1} - E_j z_{j+1};
// backward: x_i = z_i - P_i (E_{i-1}^T x_{i-1} + E_i x_{i+1}).  Every level is
// a batch of independent dense block products.
// ============================================================================
__global__ void k_bcr_assemble(Problem P, const SubDesc* subs, const BcrBlkJob* jobs,
                               const cpx<double>* diag, const cpx<double>* cx,
                               const cpx<double>* cy, cpx<double>* work) {
  const BcrBlkJob J = jobs[blockIdx.y];
  const SubDesc S = subs[J.sub];
  const int nb = S.nb;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)nb * nb) return;
  const int j = (int)(e / nb), i = (int)(e - (long long)j * nb);
  work[J.dst + e] = block_entry(S, P.dim, J.k, i, j, diag, cx, cy);
}

void launch_bcr_assemble(const Problem& P, const SubDesc* d_subs, const BcrBlkJob* d_jobs, int njobs,
                         int max_nb, const cpx<double>* diag, const cpx<double>* cx,
                         const cpx<double>* cy, cpx<double>* work, hipStream_t s) {
  if (njobs <= 0) return;
  hipLaunchKernelGGL(k_bcr_assemble, dim3(cdiv_u((long long)max_nb * max_nb, 256), njobs),
                     dim3(256), 0, s, P, d_subs, d_jobs, diag, cx, cy, work);
}

// Inversion in place (blocked Gauss-Jordan), one workgroup per job; the
// inverse is rounded into fac[dst] when dst >= 0.
template <typename T>
__global__ __launch_bounds__(1024) void k_bcr_invert(const BcrInvJob* jobs, cpx<double>* work,
                                                     cpx<T>* fac, int* err, int* pivbuf,
                                                     cpx<double>* rbuf, double* pstat, int max_nb) {
  const BcrInvJob J = jobs[blockIdx.x];
  const int nb = J.nb;
  cpx<double>* a = work + J.src;
  extern __shared__ unsigned char smem_raw[];
  const int bad = gj_blocked(a, nb, pivbuf + (long long)blockIdx.x * max_nb,
                             rbuf + (long long)blockIdx.x * GJ_B * max_nb, smem_raw, max_nb,
                             pstat ? pstat + 2 * blockIdx.x : nullptr);
  if (J.dst >= 0) {
    const long long ne = (long long)nb * nb;
    for (long long e = threadIdx.x; e < ne; e += blockDim.x) fac[J.dst + e] = cvt<T>(a[e]);
  }
  if (threadIdx.x == 0 && bad) err[blockIdx.x] = 1;
}

template <typename T>
void launch_bcr_invert(const BcrInvJob* d_jobs, int njobs, int max_nb, cpx<double>* work,
                       cpx<T>* fac, int* d_err, int* d_piv, cpx<double>* d_rbuf, double* d_pst,
                       hipStream_t s) {
  if (njobs <= 0) return;
  if (gj_use_split(njobs, max_nb)) {
    launch_gj_split<T, BcrInvJob>(d_jobs, nullptr, njobs, max_nb, work, fac, d_err, d_piv, d_rbuf,
                                  d_pst, s);
    return;
  }
  hipLaunchKernelGGL(k_bcr_invert<T>, dim3(njobs), dim3(1024), gj_lds_bytes(max_nb), s, d_jobs,
                     work, fac, d_err, d_piv, d_rbuf, d_pst, max_nb);
}

__global__ void k_bcr_diag_update(Problem P, const SubDesc* subs, const BcrDiagUpd* jobs,
                                  const cpx<double>* cy, const cpx<double>* cz,
                                  cpx<double>* work) {
  const BcrDiagUpd J = jobs[blockIdx.y];
  const SubDesc S = subs[J.sub];
  const int nb = S.nb;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)nb * nb) return;
  const int col = (int)(e / nb), i = (int)(e - (long long)col * nb);
  const cpx<double>* c = (P.dim == 2 ? cy : cz) + S.coef_off;
  const long long j = J.j;
  if (J.d >= 0) {
    cpx<double> v = work[J.d + e];
    if (J.pl >= 0) {
      const cpx<double> cl_i = c[(j - 1) * nb + i], cl_c = c[(j - 1) * nb + col];
      v = v - (cl_i * work[J.pl + e]) * cl_c;
    }
    if (J.pr >= 0) {
      const cpx<double> cr_i = c[j * nb + i], cr_c = c[j * nb + col];
      v = v - (cr_i * work[J.pr + e]) * cr_c;
    }
    work[J.d + e] = v;
  }
  if (J.eout >= 0)
    work[J.eout + e] = -((c[j * nb + i] * work[J.pr + e]) * c[(j + 1) * nb + col]);
}

void launch_bcr_diag_update(const Problem& P, const SubDesc* d_subs, const BcrDiagUpd* d_jobs,
                            int njobs, int max_nb, const cpx<double>* cy, const cpx<double>* cz,
                            cpx<double>* work, hipStream_t s) {
  if (njobs <= 0) return;
  hipLaunchKernelGGL(k_bcr_diag_update, dim3(cdiv_u((long long)max_nb * max_nb, 256), njobs),
                     dim3(256), 0, s, P, d_subs, d_jobs, cy, cz, work);
}

template <typename T>
__global__ void k_bcr_copy(const BcrCopyJob* jobs, const cpx<double>* work, cpx<T>* fac) {
  const BcrCopyJob J = jobs[blockIdx.y];
  const int nb = J.nb;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)nb * nb) return;
  const int col = (int)(e / nb), i = (int)(e - (long long)col * nb);
  const long long se = J.trans ? (long long)i * nb + col : e;
  fac[J.dst + e] = cvt<T>(work[J.src + se]);
}

template <typename T>
void launch_bcr_copy(const BcrCopyJob* d_jobs, int njobs, int max_nb, const cpx<double>* work,
                     cpx<T>* fac, hipStream_t s) {
  if (njobs <= 0) return;
  hipLaunchKernelGGL(k_bcr_copy<T>, dim3(cdiv_u((long long)max_nb * max_nb, 256), njobs),
                     dim3(256), 0, s, d_jobs, work, fac);
}

// Batched FP64 complex GEMM for the reduction levels: 32x32 output tile per
// 256-thread workgroup, the K dimension staged through LDS in panels of 16.
__global__ __launch_bounds__(256) void k_zgemm(const ZGemmJob* jobs, cpx<double>* W) {
  const ZGemmJob J = jobs[blockIdx.x];
  const int nb = J.nb;
  const int tm = blockIdx.y * 32, tn = blockIdx.z * 32;
  if (tm >= nb || tn >= nb) return;
  __shared__ cpx<double> As[16][33];   // [k][m]
  __shared__ cpx<double> Bs[16][33];   // [k][n]
  const cpx<double>* __restrict__ A = W + J.a;
  const cpx<double>* __restrict__ B = W + J.b;
  cpx<double>* C = W + J.c;
  // FP64 matrix cores: wave w owns the 16 x 16 block at (16 (w % 2), 16 (w / 2))
  // of the 32 x 32 tile (lane layout as in the Gauss-Jordan update)
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int sr = (w & 1) * 16, sc = (w >> 1) * 16, l16 = lane & 15, l4 = lane >> 4;
  gj_f64x4 cr = {0.0, 0.0, 0.0, 0.0}, ci = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < nb; k0 += 16) {
    for (int e = tid; e < 512; e += 256) {
      int mm, kk;
      if (J.ta) { kk = e & 15; mm = e >> 4; } else { mm = e & 31; kk = e >> 5; }
      const int m = tm + mm, k = k0 + kk;
      cpx<double> v = mk(0.0, 0.0);
      if (m < nb && k < nb) v = J.ta ? A[(long long)m * nb + k] : A[(long long)k * nb + m];
      As[kk][mm] = v;
      int nn;
      if (J.tb) { nn = e & 31; kk = e >> 5; } else { kk = e & 15; nn = e >> 4; }
      const int n = tn + nn, k2 = k0 + kk;
      cpx<double> u = mk(0.0, 0.0);
      if (n < nb && k2 < nb) u = J.tb ? B[(long long)k2 * nb + n] : B[(long long)n * nb + k2];
      Bs[kk][nn] = u;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      const cpx<double> av = As[kk + l4][sr + l16];
      const cpx<double> bv = Bs[kk + l4][sc + l16];
      cr = __builtin_amdgcn_mfma_f64_16x16x4f64(av.re, bv.re, cr, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f64_16x16x4f64(av.re, bv.im, ci, 0, 0, 0);
      cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-av.im, bv.im, cr, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f64_16x16x4f64(av.im, bv.re, ci, 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int m = tm + sr + 4 * j + l4, n = tn + sc + l16;
    if (m < nb && n < nb) {
      const long long o = (long long)n * nb + m;
      const cpx<double> v = mk(J.alpha * cr[j], J.alpha * ci[j]);
      C[o] = J.beta ? C[o] + v : v;
    }
  }
}

void launch_zgemm(const ZGemmJob* d_jobs, int njobs, int max_nb, cpx<double>* work, hipStream_t s) {
  if (njobs <= 0) return;
  const unsigned t = (unsigned)((max_nb + 31) / 32);
  hipLaunchKernelGGL(k_zgemm, dim3(njobs, t, t), dim3(256), 0, s, d_jobs, work);
}

// ---- solve jobs ------------------------------------------------------------
// A task is (job, RHS group of KG, row group).  Its workgroup has RT x CG
// waves: wave (rt, cg) owns the 64-row tile rt and the columns
// [cg cw, (cg+1) cw) of each of the (up to three) matrices of the job,
//   out = sum_m M_m v_m   (+ R_blk for BCR_KEPT),
// and the CG partial sums of a tile meet in LDS (CG = 1 on the wide levels;
// more column groups shorten the per-task latency chain of the small, deep
// reduction levels).  A dense job has one nb x (m nb) matrix: a row block of
// the inverse of the small reduced system left at the top of the reduction,
// applied to the m right-hand-side blocks of that system.  The operand vectors
// v_m are staged in LDS as [column][KG] complex values; the first round of
// matrix loads is issued before the staging, and every round keeps the next
// one in flight.  CG is set per reduction level by the caller.
//
// complex64 with KG = 8 or 16 runs on v_mfma_f32_16x16x4f32 (A: lane l holds
// row l%16, column l/16 of a 16x4 tile; B: lane l holds k = l/16, output
// column l%16; D: lane l, register r holds row 4(l/16)+r, column l%16).  A
// is Re(M) or Im(M) of a 16-row x 4-column tile; the 16 output columns are
// (Re, Im) of 8 right-hand sides, with B = [Re y, Im y] against Re(M) and
// [-Im y, Re y] against Im(M).  The four 16-row blocks of a wave keep four
// independent accumulator chains.  Otherwise vector FMAs, one row per lane.
constexpr int BCR_ROUND_BYTES = 192;        // matrix bytes per lane in one round
constexpr int BCR_STAGE = 4;                // operand loads a thread keeps in flight
constexpr int BCR_MAXW = 12;                // waves per workgroup
constexpr int BCR_MAXRT = 4;                // 64-row tiles per workgroup

template <typename T, int KG>
struct BcrTraits {
  static constexpr bool MF = std::is_same<T, float>::value && KG >= 8;
  static constexpr int JB = MF ? KG / 8 : 1;            // 16-column output blocks
  static constexpr int PW = MF ? 4 * 4 * JB : 2 * KG;   // partial-sum words per lane
};

template <typename T, int KG>
__global__ __launch_bounds__(64 * BCR_MAXW) void k_bcr(const SubDesc* __restrict__ subs,
                                                       const BcrJob* __restrict__ jobs, int njobs,
                                                       int G, int nrg, int RT, int CG, int nrhs,
                                                       int kmax, const cpx<T>* __restrict__ fac,
                                                       const cpx<T>* __restrict__ cpl,
                                                       cpx<T>* __restrict__ rpool,
                                                       cpx<T>* __restrict__ vpool,
                                                       long long pool_stride, int lds_rg) {
  typedef typename vec2<T>::type V2;
  typedef cpx<T> C;
  typedef BcrTraits<T, KG> TR;
  constexpr bool MF = TR::MF;
  constexpr int JB = TR::JB;
  constexpr int U = BCR_ROUND_BYTES / (int)sizeof(V2);   // loads per lane per round
  constexpr int UG = U / 4;                              // MF: 4-column groups per round
  typedef float mf4v __attribute__((ext_vector_type(4)));
  const int total = gridDim.x;
  const int per = total >> 3;
  const int bid = blockIdx.x;
  const int Lg = (bid & 7) * per + (bid >> 3);   // XCD-aware: a job's tasks share an L2
  const int tpj = G * nrg;
  const int job = Lg / tpj;
  if (job >= njobs) return;
  const int rem = Lg - job * tpj;
  const int g = rem / nrg, rg = rem - (rem / nrg) * nrg;
  const BcrJob J = jobs[job];
  const int nb = J.nb;
  const int ncol = J.mode == BCR_DENSE ? J.pad * nb : nb;   // columns of every matrix
  const long long nloc = J.nloc;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int rt = w % RT, cg = w / RT;
  const int row0 = (rg * RT + rt) * 64;
  // CG wave groups split the columns (CG depends on the job's reduction level
  // only, so a job's summation order is the same in every schedule)
  int cw = (ncol + CG - 1) / CG;
  cw = (cw + 3) & ~3;
  const int c0 = min(ncol, cg * cw);
  const int c1 = min(ncol, c0 + cw);
  const bool wave_live = row0 < nb && c0 < c1;
  const C zero = mk((T)0, (T)0);
  C* __restrict__ X = vpool + (long long)J.l * pool_stride + J.vbase;
  C* __restrict__ R = rpool + (long long)J.l * pool_stride + J.vbase;
  const C* __restrict__ Cp = cpl + J.cbase;
  const V2* __restrict__ Fv = reinterpret_cast<const V2*>(fac);
  const int mode = J.mode, blk = J.blk;
  const bool hl = J.nl >= 0, hr = J.nr >= 0;
  int nm;
  long long mo0, mo1 = 0, mo2 = 0;
  if (mode == BCR_KEPT) {
    nm = (int)hl + (int)hr;
    mo0 = hl ? J.m0 : J.m1;
    mo1 = J.m1;
  } else if (mode == BCR_BWD) {
    nm = 1 + (int)hl + (int)hr;
    mo0 = J.m0;
    mo1 = hl ? J.m1 : J.m2;
    mo2 = J.m2;
  } else {
    nm = 1;
    mo0 = J.m0;
  }
  const long long d01 = mo1 - mo0, d12 = mo2 - mo1;
  // rounds per matrix: MF covers 4 columns x 16 rows per load, else 1 column x 64 rows
  const int cpr = MF ? 4 * UG : U;                       // columns per round
  const int nr = (c1 - c0 + cpr - 1) / cpr;
  const int total_rounds = nm * nr;
  // per-lane load base: MF lane l reads row 16 rb + l%16 of column 4 g + l/16
  int lrow, lcol;
  if (MF) { lrow = row0 + (lane & 15); lcol = lane >> 4; }
  else { lrow = row0 + lane; lcol = 0; }
  auto issue = [&](V2 (&buf)[U], int gr) {
    const int m = gr / nr, rd = gr - (gr / nr) * nr;
    const V2* __restrict__ Mv = Fv + mo0 + (m >= 1 ? d01 : 0) + (m >= 2 ? d12 : 0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int col, rw;
      if (MF) {
        col = c0 + rd * cpr + 4 * (u / 4) + lcol;
        rw = lrow + 16 * (u & 3);
      } else {
        col = c0 + rd * cpr + u;
        rw = lrow;
      }
      col = col < c1 ? col : c1 - 1;
      rw = rw < nb ? rw : nb - 1;
      buf[u] = Mv[(unsigned)(col * nb + rw)];
    }
  };
  V2 bufA[U], bufB[U];
  if (wave_live) issue(bufA, 0);

  // ---- operands: set m at ops + m * nb4 * KG, [column][KG]; loads batched
  // (a dense job has one set of ncol columns)
  extern __shared__ unsigned char smem_raw[];
  C* ops = reinterpret_cast<C*>(smem_raw);
  const int nb4 = (nb + 3) & ~3;                    // operand columns, zero beyond nb
  const long long ss = (long long)nb4 * KG;
  const int wcn = (ncol + 3) & ~3;
  const int nel = wcn * KG;
  for (int base = 0; base < nel; base += BCR_STAGE * (int)blockDim.x) {
    C va[BCR_STAGE], vb[BCR_STAGE], vc[BCR_STAGE];
#pragma unroll
    for (int k = 0; k < BCR_STAGE; ++k) {
      const int idx = base + k * (int)blockDim.x + tid;
      const int q = idx / wcn, i = idx - q * wcn;
      const int rq = g * KG + q;
      const bool live = idx < nel && rq < nrhs && i < ncol;
      const long long ro = (long long)rq * nloc;
      va[k] = vb[k] = vc[k] = zero;
      if (live) {
        if (mode == BCR_DENSE) {
          const int bq = i / nb;
          va[k] = R[ro + (long long)(J.nl + bq * J.nr) * nb + (i - bq * nb)];
        } else if (mode == BCR_KEPT) {
          if (hl) va[k] = R[ro + (long long)J.nl * nb + i];
          if (hr) vb[k] = R[ro + (long long)J.nr * nb + i];
        } else {
          if (mode != BCR_CHB) va[k] = R[ro + (long long)blk * nb + i];
          if (mode == BCR_BWD || mode == BCR_BWD0 || mode == BCR_CHB) {
            if (hl) vb[k] = X[ro + (long long)J.nl * nb + i];
            if (hr) vc[k] = X[ro + (long long)J.nr * nb + i];
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < BCR_STAGE; ++k) {
      const int idx = base + k * (int)blockDim.x + tid;
      if (idx >= nel) break;
      const int q = idx / wcn, i = idx - q * wcn;
      C* o = ops + (long long)i * KG + q;
      if (mode == BCR_KEPT) {
        if (hl) o[0] = -va[k];
        if (hr) o[hl ? ss : 0] = -vb[k];
      } else if (mode == BCR_BWD) {
        o[0] = va[k];
        if (hl) o[ss] = -vb[k];
        if (hr) o[hl ? 2 * ss : ss] = -vc[k];
      } else if (mode == BCR_BWD0) {
        C y = va[k];
        if (i < nb) {
          if (hl) y = y - Cp[(long long)(blk - 1) * nb + i] * vb[k];
          if (hr) y = y - Cp[(long long)blk * nb + i] * vc[k];
        }
        o[0] = y;
      } else if (mode == BCR_CHB) {
        C y = zero;
        if (i < nb) {
          if (hl) y = y - Cp[(long long)(blk - 1) * nb + i] * vb[k];
          if (hr) y = y - Cp[(long long)blk * nb + i] * vc[k];
        }
        o[0] = y;
      } else {
        o[0] = va[k];
      }
    }
  }
  __syncthreads();

  mf4v acc[4][JB];
  T ar[KG], ai[KG];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int jb = 0; jb < JB; ++jb) acc[rb][jb] = mf4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int q = 0; q < KG; ++q) { ar[q] = (T)0; ai[q] = (T)0; }
  const int jsel = lane & 15;                 // MF: output column of this lane
  auto compute = [&](const V2 (&buf)[U], int gr) {
    const int m = gr / nr, rd = gr - (gr / nr) * nr;
    const C* __restrict__ op = ops + m * ss;
    const int cbase = c0 + rd * cpr;
    if constexpr (MF) {
#pragma unroll
      for (int ug = 0; ug < UG; ++ug) {
        if (cbase + 4 * ug >= c1) break;        // wave-uniform; operands are zero past nb
        const int col = cbase + 4 * ug + lcol;  // this lane's k
        float bre[JB], bim[JB];
#pragma unroll
        for (int jb = 0; jb < JB; ++jb) {
          const int j = jb * 16 + jsel;
          const C y = op[col * KG + (j >> 1)];
          const bool im = j & 1;
          bre[jb] = im ? y.im : y.re;
          bim[jb] = im ? y.re : -y.im;
        }
#pragma unroll
        for (int jb = 0; jb < JB; ++jb) {
#pragma unroll
          for (int rb = 0; rb < 4; ++rb)
            acc[rb][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32((float)buf[4 * ug + rb].x, bre[jb], acc[rb][jb], 0, 0, 0);
#pragma unroll
          for (int rb = 0; rb < 4; ++rb)
            acc[rb][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32((float)buf[4 * ug + rb].y, bim[jb], acc[rb][jb], 0, 0, 0);
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int col = cbase + u;
        if (col >= c1) break;                    // wave-uniform
#pragma unroll
        for (int q = 0; q < KG; ++q) {
          const C y = op[col * KG + q];
          ar[q] = fma(buf[u].x, y.re, ar[q]);
          ar[q] = fma(-buf[u].y, y.im, ar[q]);
          ai[q] = fma(buf[u].x, y.im, ai[q]);
          ai[q] = fma(buf[u].y, y.re, ai[q]);
        }
      }
    }
  };
  if (wave_live) {
    // ping-pong: one buffer is computed while the other one's loads are in flight
    for (int gr = 0; gr < total_rounds; gr += 2) {
      const bool two = gr + 1 < total_rounds;
      if (two) issue(bufB, gr + 1);
      compute(bufA, gr);
      if (two) {
        if (gr + 2 < total_rounds) issue(bufA, gr + 2);
        compute(bufB, gr + 1);
      }
    }
  }
  // ---- column-group partial sums meet in LDS (in the operand area, once
  // every wave is done with the operands)
  if (CG > 1) {
    __syncthreads();
    float* part = reinterpret_cast<float*>(smem_raw);
    constexpr int PW = TR::PW;
    if (cg > 0) {
      if constexpr (MF) {
        float* pw = part + (long long)((cg - 1) * RT + rt) * PW * 64;
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
          for (int jb = 0; jb < JB; ++jb)
#pragma unroll
            for (int r = 0; r < 4; ++r) pw[((rb * JB + jb) * 4 + r) * 64 + lane] = acc[rb][jb][r];
      } else {
        T* pt = reinterpret_cast<T*>(part) + (long long)((cg - 1) * RT + rt) * PW * 64;
#pragma unroll
        for (int q = 0; q < KG; ++q) {
          pt[(2 * q) * 64 + lane] = ar[q];
          pt[(2 * q + 1) * 64 + lane] = ai[q];
        }
      }
    }
    __syncthreads();
    if (cg == 0) {
      for (int o = 1; o < CG; ++o) {
        if constexpr (MF) {
          const float* pw = part + (long long)((o - 1) * RT + rt) * PW * 64;
#pragma unroll
          for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int jb = 0; jb < JB; ++jb)
#pragma unroll
              for (int r = 0; r < 4; ++r) acc[rb][jb][r] += pw[((rb * JB + jb) * 4 + r) * 64 + lane];
        } else {
          const T* pt = reinterpret_cast<const T*>(part) + (long long)((o - 1) * RT + rt) * PW * 64;
#pragma unroll
          for (int q = 0; q < KG; ++q) {
            ar[q] += pt[(2 * q) * 64 + lane];
            ai[q] += pt[(2 * q + 1) * 64 + lane];
          }
        }
      }
    }
  }
  const int orow = row0 + lane;
  if constexpr (MF) {
    // regroup rows through LDS: with one column group each wave has a region of
    // its own after the operands (no wait for the other waves); otherwise the
    // operand area, free once every wave is done
    float* st;
    if (CG == 1) {
      st = reinterpret_cast<float*>(smem_raw + lds_rg) + (long long)rt * 64 * KG * 2;
    } else {
      __syncthreads();
      st = reinterpret_cast<float*>(smem_raw) + (long long)rt * 64 * KG * 2;
    }
    if (cg == 0) {
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int jb = 0; jb < JB; ++jb)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int rl = 16 * rb + 4 * (lane >> 4) + r;
            const int j = jb * 16 + (lane & 15);
            st[((long long)(j >> 1) * 64 + rl) * 2 + (j & 1)] = acc[rb][jb][r];
          }
    }
    if (CG == 1) {
      // the wave reads back only what it wrote; LDS operations of a wave are
      // performed in order
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
      __syncthreads();
    }
    if (cg == 0) {
#pragma unroll
      for (int q = 0; q < KG; ++q) {
        ar[q] = st[((long long)q * 64 + lane) * 2];
        ai[q] = st[((long long)q * 64 + lane) * 2 + 1];
      }
    }
  }
  if (cg == 0 && orow < nb) {
#pragma unroll
    for (int q = 0; q < KG; ++q) {
      const int rq = g * KG + q;
      if (rq < nrhs) {
        const long long oo = (long long)rq * nloc + (long long)blk * nb + orow;
        const C out = mk(ar[q], ai[q]);
        if (mode == BCR_KEPT) R[oo] = R[oo] + out;
        else if (mode == BCR_CHB) X[oo] = X[oo] + out;
        else X[oo] = out;
      }
    }
  }
}

template <typename T>
__global__ void k_bcr_dfwd(const SubDesc* __restrict__ subs, const BcrJob* __restrict__ jobs,
                           int nrhs, int kmax, const cpx<T>* __restrict__ cpl,
                           cpx<T>* __restrict__ rpool, const cpx<T>* __restrict__ vpool,
                           long long pool_stride) {
  const BcrJob J = jobs[blockIdx.y];
  const SubDesc S = subs[J.sub];
  const int nb = S.nb;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)nb * nrhs) return;
  const int q = (int)(e / nb), i = (int)(e - (long long)q * nb);
  const cpx<T>* X = vpool + (long long)J.l * pool_stride + S.vec_off * kmax + (long long)q * S.nloc;
  cpx<T>* R = rpool + (long long)J.l * pool_stride + S.vec_off * kmax + (long long)q * S.nloc;
  const cpx<T>* Cp = cpl + S.coef_off;
  cpx<T> y = R[(long long)J.blk * nb + i];
  if (J.nl >= 0) y = y - Cp[(long long)(J.blk - 1) * nb + i] * X[(long long)J.nl * nb + i];
  if (J.nr >= 0) y = y - Cp[(long long)J.blk * nb + i] * X[(long long)J.nr * nb + i];
  R[(long long)J.blk * nb + i] = y;
}

template <typename T>
void launch_bcr_dfwd(const SubDesc* d_subs, const BcrJob* d_jobs, int njobs, int nrhs, int kmax,
                     int max_nb, const cpx<T>* cpl, cpx<T>* rpool, const cpx<T>* vpool,
                     long long pool_stride, hipStream_t s) {
  if (njobs <= 0 || nrhs <= 0) return;
  hipLaunchKernelGGL(k_bcr_dfwd<T>, dim3(cdiv_u((long long)max_nb * nrhs, 256), njobs), dim3(256),
                     0, s, d_subs, d_jobs, nrhs, kmax, cpl, rpool, vpool, pool_stride);
}

template <typename T>
int bcr_kg(int max_nb, int kg) {
  (void)max_nb;
  const int cap = std::is_same<T, float>::value ? 16 : 8;
  int k = 1;
  while (k * 2 <= kg && k * 2 <= cap) k *= 2;
  return k;
}

// Waves of a solve workgroup: RT 64-row tiles (a block's rows in row groups
// of at most rt tiles) times CG column groups.
static inline void bcr_shape(int max_nb, int cg, int rt, int& RT, int& CG, int& nrg) {
  const int tiles = (max_nb + 63) / 64;
  const int rmax = rt >= 1 && rt < BCR_MAXRT ? rt : BCR_MAXRT;
  RT = tiles < rmax ? tiles : rmax;
  nrg = (tiles + RT - 1) / RT;
  CG = cg < 1 ? 1 : cg;
  while (CG > 1 && RT * CG > BCR_MAXW) --CG;
}

// LDS of a launch: the operand sets, reused for the MF row regrouping and the
// column-group partial sums once every wave is done with the operands.
// Operand area of a launch (bytes, rounded); with MF and one column group the
// row-regrouping regions of the row tiles follow it.
template <typename T>
static size_t bcr_ops_area(int max_nb, int kg, int nset) {
  const size_t ops = (size_t)nset * ((max_nb + 3) & ~3) * kg * sizeof(cpx<T>);
  return (ops + 255) / 256 * 256;
}

template <typename T>
size_t bcr_launch_lds_bytes(int max_nb, int kg, int nset, int cg, int rt) {
  int RT, CG, nrg;
  bcr_shape(max_nb, cg, rt, RT, CG, nrg);
  const size_t ops = bcr_ops_area<T>(max_nb, kg, nset);
  const size_t stage = (size_t)RT * 64 * kg * sizeof(cpx<T>);
  const bool mf = std::is_same<T, float>::value && kg >= 8;
  if (mf && CG == 1) return ops + (stage + 255) / 256 * 256;
  const size_t per_lane = mf ? (size_t)16 * (kg / 8) * sizeof(float) : 2 * (size_t)kg * sizeof(T);
  const size_t part = CG > 1 ? (size_t)(CG - 1) * RT * 64 * per_lane : 0;
  size_t b = ops > stage ? ops : stage;
  b = b > part ? b : part;
  return (b + 255) / 256 * 256;
}

// Largest LDS a launch of the level-by-level shapes can ask for (CG up to 4
// at the default row tiles, up to 12 at one row tile).
template <typename T>
size_t bcr_lds_bytes(int max_nb, int kg, int nset) {
  size_t b = 0;
  for (int cg = 1; cg <= 12; ++cg)
    for (int rt : {0, 1}) {
      if (rt == 0 && cg > 4) continue;
      const size_t v = bcr_launch_lds_bytes<T>(max_nb, kg, nset, cg, rt);
      b = v > b ? v : b;
    }
  return b;
}

template <typename T, int KG>
static void launch_bcr_k(const SubDesc* d_subs, const BcrJob* d_jobs, int njobs, int nset, int cg,
                         int rt, int nrhs, int kmax, int max_nb, const cpx<T>* fac,
                         const cpx<T>* cpl, cpx<T>* rpool, cpx<T>* vpool, long long pool_stride,
                         hipStream_t s) {
  const int G = (nrhs + KG - 1) / KG;
  int RT, CG, nrg;
  bcr_shape(max_nb, cg, rt, RT, CG, nrg);
  long long total = (long long)njobs * G * nrg;
  total = (total + 7) / 8 * 8;
  const size_t lds = bcr_launch_lds_bytes<T>(max_nb, KG, nset, cg, rt);
  hipLaunchKernelGGL((k_bcr<T, KG>), dim3((unsigned)total), dim3(64 * RT * CG), lds, s, d_subs,
                     d_jobs, njobs, G, nrg, RT, CG, nrhs, kmax, fac, cpl, rpool, vpool,
                     pool_stride, (int)bcr_ops_area<T>(max_nb, KG, nset));
}

template <typename T>
void launch_bcr_solve(int kg, const SubDesc* d_subs, const BcrJob* d_jobs, int njobs, int nset,
                      int cg, int rt, int nrhs, int kmax, int max_nb, const cpx<T>* fac,
                      const cpx<T>* cpl, cpx<T>* rpool, cpx<T>* vpool, long long pool_stride,
                      hipStream_t s) {
  if (njobs <= 0 || nrhs <= 0) return;
#define DSD_BCR_K(K) \
  launch_bcr_k<T, K>(d_subs, d_jobs, njobs, nset, cg, rt, nrhs, kmax, max_nb, fac, cpl, rpool, vpool, pool_stride, s)
  switch (bcr_kg<T>(max_nb, kg)) {
    case 1: DSD_BCR_K(1); break;
    case 2: DSD_BCR_K(2); break;
    case 4: DSD_BCR_K(4); break;
    case 8: DSD_BCR_K(8); break;
    default:
      if constexpr (std::is_same<T, float>::value) DSD_BCR_K(16);
      break;
  }
#undef DSD_BCR_K
}

// Dense top level: assemble the reduced block-tridiagonal system of one
// subdomain as a column-major n x n matrix (n = m nb).
__global__ void k_bcr_dense_build(const BcrDenseJob* jobs, const cpx<double>* work,
                                  cpx<double>* dense) {
  const BcrDenseJob J = jobs[blockIdx.y];
  const int nb = J.nb;
  const long long n = (long long)J.m * nb;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const long long C = e / n, R = e - C * n;
  const int qc = (int)(C / nb), qr = (int)(R / nb);
  const int c = (int)(C - (long long)qc * nb), r = (int)(R - (long long)qr * nb);
  cpx<double> v = mk(0.0, 0.0);
  if (qr == qc)
    v = work[J.dbase + (long long)(J.first + qr * J.stride) * J.slot + (long long)c * nb + r];
  else if (qc == qr + 1)
    v = work[J.ebase + (long long)qr * J.slot + (long long)c * nb + r];
  else if (qr == qc + 1)
    v = work[J.ebase + (long long)qc * J.slot + (long long)r * nb + c];
  dense[J.out + e] = v;
}

void launch_bcr_dense_build(const BcrDenseJob* d_jobs, int njobs, int max_n,
                            const cpx<double>* work, cpx<double>* dense, hipStream_t s) {
  if (njobs <= 0) return;
  hipLaunchKernelGGL(k_bcr_dense_build, dim3(cdiv_u((long long)max_n * max_n, 256), njobs),
                     dim3(256), 0, s, d_jobs, work, dense);
}

// Rounds the inverse into the factor as m row blocks, each nb x n column-major.
template <typename T>
__global__ void k_bcr_dense_store(const BcrDenseJob* jobs, const cpx<double>* dense, cpx<T>* fac) {
  const BcrDenseJob J = jobs[blockIdx.y];
  const int nb = J.nb;
  const long long n = (long long)J.m * nb;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const long long C = e / n, R = e - C * n;
  const long long i = R / nb, r = R - i * nb;
  fac[J.fac + i * nb * n + C * nb + r] = cvt<T>(dense[J.out + e]);
}

template <typename T>
void launch_bcr_dense_store(const BcrDenseJob* d_jobs, int njobs, int max_n,
                            const cpx<double>* dense, cpx<T>* fac, hipStream_t s) {
  if (njobs <= 0) return;
  hipLaunchKernelGGL(k_bcr_dense_store<T>, dim3(cdiv_u((long long)max_n * max_n, 256), njobs),
                     dim3(256), 0, s, d_jobs, dense, fac);
}

// ============================================================================
// a4: local right-hand sides.  init: r = f on own cells for the members in
// slot src_slot (the first sweep; the first step of the additive DDM), 0
// otherwise.  pull: every receiver cell sums, in a fixed edge order, the
// transferred sources Psi_t(v) = -M_sender(beta_t v) of the edges whose box
// holds it; each cell is written by exactly one thread (no atomics).
// ============================================================================
template <typename T>
__global__ __launch_bounds__(256) void k_init_rhs(Problem P, const SubDesc* subs, const int2* members, int nrhs, int kmax,
                           const cpx<double>* f, cpx<T>* rpool, long long pool_stride,
                           int src_slot) {
  const int2 mb = members[blockIdx.y];
  const SubDesc& S = subs[mb.x];
  const int nloc = (int)S.nloc;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nloc) return;
  cpx<T>* R = rpool + (long long)mb.y * pool_stride + S.vec_off * kmax + c;
  long long gf = -1;
  if (mb.y == src_slot) {   // the slot that takes f on the subdomain's own cells
    const int nx = S.dims[0], ny = S.dims[1];
    const int ix = c % nx, q = c / nx;
    const int iy = q % ny, iz = q / ny;
    const int g0 = S.ax[0].g0 + ix, g1 = S.ax[1].g0 + iy, g2 = S.ax[2].g0 + iz;
    bool own = g0 >= S.pt[0].o0 && g0 < S.pt[0].o1 && g1 >= S.pt[1].o0 && g1 < S.pt[1].o1;
    if (P.dim == 3) own = own && g2 >= S.pt[2].o0 && g2 < S.pt[2].o1;
    if (own) gf = ((long long)g2 * P.ng[1] + g1) * P.ng[0] + g0;
  }
  for (int r = 0; r < nrhs; ++r)
    R[(long long)r * nloc] = gf >= 0 ? cvt<T>(f[(long long)r * P.N + gf]) : mk((T)0, (T)0);
}

template <typename T>
void launch_init_rhs(const Problem& P, const SubDesc* d_subs, const int2* d_members, int nmem,
                     long long max_nloc, int nrhs, int kmax, const cpx<double>* f, cpx<T>* rpool,
                     long long pool_stride, int src_slot, hipStream_t s) {
  if (nmem <= 0 || nrhs <= 0) return;
  dim3 grid(cdiv_u(max_nloc, 256), nmem);
  hipLaunchKernelGGL(k_init_rhs<T>, grid, dim3(256), 0, s, P, d_subs, d_members, nrhs, kmax, f,
                     rpool, pool_stride, src_slot);
}

template <typename T>
__device__ inline bool in_box(const Edge& e, const int c[3]) {
  return c[0] >= e.lo[0] && c[0] < e.hi[0] && c[1] >= e.lo[1] && c[1] < e.hi[1] &&
         c[2] >= e.lo[2] && c[2] < e.hi[2];
}

// Source transfer into receiver cell c (receiver-local coordinates) for a
// group of up to PR right-hand sides starting at r0: for every incoming edge
// whose box holds c, g = -M (beta_t v) evaluated with the sender's stencil and
// the sender solutions of the sweeps in the edge's mask (Section 2.2).  The
// stencil weights (coefficient times cutoff) are formed once per edge and
// group; every load of a sweep's solutions is independent of the others (a
// stencil point off the grid or outside the cutoff reads the centre cell and
// is dropped), so they are all in flight together.
template <typename T>
constexpr int pull_r() { return sizeof(T) == 4 ? 4 : 2; }   // RHS per thread

template <typename T, int NST>
__global__ __launch_bounds__(256) void k_pull(Problem P, const SubDesc* subs, const int2* members, const Edge* edges,
                       const int2* erange, int nrhs, int kmax, const cpx<T>* vpool,
                       long long pool_stride, const cpx<T>* diag, const cpx<T>* cx,
                       const cpx<T>* cy, const cpx<T>* cz, cpx<T>* rpool) {
  const int2 mb = members[blockIdx.z];
  const int2 er = erange[blockIdx.z];
  constexpr int PULL_R = pull_r<T>();
  const int r0 = blockIdx.y * PULL_R;
  if (r0 >= nrhs || er.y <= 0) return;   // uniform over the workgroup
  // the member's edges and their senders' descriptors, staged in LDS
  __shared__ Edge E[MAX_IN_EDGES];
  __shared__ SubDesc SS[MAX_IN_EDGES];
  const int ne = er.y;
  {
    constexpr int EW = (int)(sizeof(Edge) / sizeof(int)), SW = (int)(sizeof(SubDesc) / sizeof(int));
    const int* src = reinterpret_cast<const int*>(edges + er.x);
    for (int i = threadIdx.x; i < ne * EW; i += blockDim.x) reinterpret_cast<int*>(E)[i] = src[i];
    __syncthreads();
    for (int i = threadIdx.x; i < ne * SW; i += blockDim.x) {
      const int e = i / SW, w_ = i - e * SW;
      reinterpret_cast<int*>(&SS[e])[w_] = reinterpret_cast<const int*>(subs + E[e].sender)[w_];
    }
    __syncthreads();
  }
  int f = blockIdx.x * blockDim.x + threadIdx.x;
  int eidx = -1;
  for (int e = 0; e < ne; ++e) {
    const int vol = (E[e].hi[0] - E[e].lo[0]) * (E[e].hi[1] - E[e].lo[1]) * (E[e].hi[2] - E[e].lo[2]);
    if (f < vol) { eidx = e; break; }
    f -= vol;
  }
  if (eidx < 0) return;
  const Edge& e0 = E[eidx];
  const int bx = e0.hi[0] - e0.lo[0], by = e0.hi[1] - e0.lo[1];
  int c[3];
  c[0] = e0.lo[0] + f % bx;
  const int q = f / bx;
  c[1] = e0.lo[1] + q % by;
  c[2] = e0.lo[2] + q / by;
  for (int e = 0; e < eidx; ++e)
    if (in_box<T>(E[e], c)) return;          // an earlier box owns this cell
  cpx<T> acc[PULL_R];
#pragma unroll
  for (int k = 0; k < PULL_R; ++k) acc[k] = mk((T)0, (T)0);
  for (int e = eidx; e < ne; ++e) {
    const Edge& ed = E[e];
    if (!in_box<T>(ed, c)) continue;
    const SubDesc& Sd = SS[e];
    const int dm0 = Sd.dims[0], dm1 = Sd.dims[1], dm2 = Sd.dims[2];
    const int cs0 = c[0] + ed.off[0], cs1 = c[1] + ed.off[1], cs2 = c[2] + ed.off[2];
    const long long co = Sd.coef_off + ((long long)cs2 * dm1 + cs1) * dm0 + cs0;
    const long long plane = (long long)dm0 * dm1;
    const long long cc = ((long long)cs2 * dm1 + cs1) * dm0 + cs0;
    // stencil point st: 0 centre, 1/2 +-x, 3/4 +-y, 5/6 +-z
    cpx<T> w[NST];
    long long cell[NST];
    bool live[NST];
#pragma unroll
    for (int st = 0; st < NST; ++st) {
      int p0 = cs0, p1 = cs1, p2 = cs2;
      bool ok = true;
      long long ca = co;
      const cpx<T>* arr = diag;
      if (st == 1) { ok = ok && cs0 + 1 < dm0; p0 += 1; arr = cx; }
      else if (st == 2) { ok = ok && cs0 > 0; p0 -= 1; arr = cx; ca = co - 1; }
      else if (st == 3) { ok = ok && cs1 + 1 < dm1; p1 += 1; arr = cy; }
      else if (st == 4) { ok = ok && cs1 > 0; p1 -= 1; arr = cy; ca = co - dm0; }
      else if (st == 5) { ok = ok && cs2 + 1 < dm2; p2 += 1; arr = cz; }
      else if (st == 6) { ok = ok && cs2 > 0; p2 -= 1; arr = cz; ca = co - plane; }
      double beta = 0.0;
      if (ok) {
        beta = cutoff(Sd.pt[0], ed.t[0], Sd.ax[0].g0 + p0, P.d) *
               cutoff(Sd.pt[1], ed.t[1], Sd.ax[1].g0 + p1, P.d);
        if (NST == 7) beta *= cutoff(Sd.pt[2], ed.t[2], Sd.ax[2].g0 + p2, P.d);
      }
      live[st] = ok && beta != 0.0;
      const cpx<T> a = arr[live[st] ? ca : co];
      w[st] = (T)beta * a;
      cell[st] = live[st] ? ((long long)p2 * dm1 + p1) * dm0 + p0 : cc;
    }
    // v[k][st] = sum over the masked sweeps of the sender solution at the point
    cpx<T> v[PULL_R][NST];
#pragma unroll
    for (int k = 0; k < PULL_R; ++k)
#pragma unroll
      for (int st = 0; st < NST; ++st) v[k][st] = mk((T)0, (T)0);
    const cpx<T>* V = vpool + Sd.vec_off * kmax;
    for (int l = 0; l < 8; ++l) {
      if (!(ed.lmask & (1u << l))) continue;   // uniform over the edge's box
      const cpx<T>* Vl = V + l * pool_stride;
#pragma unroll
      for (int k = 0; k < PULL_R; ++k) {
        const int r = min(r0 + k, nrhs - 1);
#pragma unroll
        for (int st = 0; st < NST; ++st) v[k][st] = v[k][st] + Vl[(long long)r * Sd.nloc + cell[st]];
      }
    }
#pragma unroll
    for (int k = 0; k < PULL_R; ++k)
#pragma unroll
      for (int st = 0; st < NST; ++st)
        if (live[st]) acc[k] = acc[k] + w[st] * v[k][st];
  }
  const SubDesc& R = subs[mb.x];
  const long long cell = ((long long)c[2] * R.dims[1] + c[1]) * R.dims[0] + c[0];
  cpx<T>* out = rpool + (long long)mb.y * pool_stride + R.vec_off * kmax + cell;
#pragma unroll
  for (int k = 0; k < PULL_R; ++k) {
    const int r = r0 + k;
    if (r < nrhs) out[(long long)r * R.nloc] = out[(long long)r * R.nloc] - acc[k];
  }
}

template <typename T>
void launch_pull(const Problem& P, const SubDesc* d_subs, const int2* d_members, int nmem,
                 const Edge* d_edges, const int2* d_edge_range, long long max_box_cells,
                 int nrhs, int kmax, const cpx<T>* vpool, long long pool_stride,
                 const cpx<T>* diag, const cpx<T>* cx, const cpx<T>* cy, const cpx<T>* cz,
                 cpx<T>* rpool, hipStream_t s) {
  if (nmem <= 0 || nrhs <= 0 || max_box_cells <= 0) return;
  constexpr int PR = pull_r<T>();
  dim3 grid(cdiv_u(max_box_cells, 256), (nrhs + PR - 1) / PR, nmem);
  if (P.dim == 3)
    hipLaunchKernelGGL((k_pull<T, 7>), grid, dim3(256), 0, s, P, d_subs, d_members, d_edges,
                       d_edge_range, nrhs, kmax, vpool, pool_stride, diag, cx, cy, cz, rpool);
  else
    hipLaunchKernelGGL((k_pull<T, 5>), grid, dim3(256), 0, s, P, d_subs, d_members, d_edges,
                       d_edge_range, nrhs, kmax, vpool, pool_stride, diag, cx, cy, cz, rpool);
}

// ============================================================================
// a5: u_DDM = sum_sub beta_{0;sub} sum_l v_sub^l over the slots l in
// [slot0, slot0 + nslots), FP64, pulled per global cell from the (at most two
// per axis) subdomains whose cutoff support covers it; written, or added to u
// (accumulate: the additive DDM adds every step's solutions).
// ============================================================================
template <typename T>
__global__ __launch_bounds__(256) void k_assemble_u(Problem P, const SubDesc* subs, PartTables pt,
                                                    int slot0, int nslots, int accumulate,
                                                    int nrhs, int kmax,
                                                    const cpx<T>* __restrict__ vpool,
                                                    long long pool_stride,
                                                    cpx<double>* __restrict__ u) {
  const int gflat = blockIdx.x * blockDim.x + threadIdx.x;
  if (gflat >= (int)P.N) return;
  int g[3];
  g[0] = gflat % P.ng[0];
  const int q = gflat / P.ng[0];
  g[1] = q % P.ng[1];
  g[2] = q / P.ng[1];
  // a cell lies in the cutoff support of at most two parts per axis (parts own
  // at least d cells), so at most 2^dim subdomains contribute
  int cand[3][2], ncand[3];
  double wgt[3][2];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cand[a][0] = cand[a][1] = 0;
    wgt[a][0] = wgt[a][1] = 0.0;
    ncand[a] = 0;
    if (a >= P.dim) { wgt[a][0] = 1.0; ncand[a] = 1; continue; }
    const int p = pt.part_of[a][g[a]];
#pragma unroll
    for (int dp = -1; dp <= 1; ++dp) {
      const int pp = p + dp;
      if (pp < 0 || pp >= pt.P[a]) continue;
      const AxisPart ap = pt.parts[a][pp];
      const double w = cutoff(ap, -1, g[a], P.d) * cutoff(ap, 1, g[a], P.d);
      if (w != 0.0 && ncand[a] < 2) {
        if (ncand[a] == 0) { cand[a][0] = pp; wgt[a][0] = w; }
        else { cand[a][1] = pp; wgt[a][1] = w; }
        ++ncand[a];
      }
    }
  }
  long long base[8];
  long long nl[8];
  double wc[8];
  int nc = 0;
#pragma unroll
  for (int iz = 0; iz < 2; ++iz)
#pragma unroll
    for (int iy = 0; iy < 2; ++iy)
#pragma unroll
      for (int ix = 0; ix < 2; ++ix) {
        const int k = (iz * 2 + iy) * 2 + ix;
        base[k] = 0; nl[k] = 0; wc[k] = 0.0;
        if (ix < ncand[0] && iy < ncand[1] && iz < ncand[2]) {
          const int sub = (cand[2][iz] * pt.P[1] + cand[1][iy]) * pt.P[0] + cand[0][ix];
          const SubDesc& S = subs[sub];
          const int lx = g[0] - S.ax[0].g0, ly = g[1] - S.ax[1].g0, lz = g[2] - S.ax[2].g0;
          base[k] = S.vec_off * kmax + ((long long)lz * S.dims[1] + ly) * S.dims[0] + lx;
          nl[k] = S.nloc;
          wc[k] = wgt[0][ix] * wgt[1][iy] * wgt[2][iz];
          ++nc;
        }
      }
  for (int r = 0; r < nrhs; ++r) {
    cpx<double> acc = mk(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (wc[k] == 0.0) continue;
      const long long o = base[k] + (long long)r * nl[k];
      cpx<double> v = mk(0.0, 0.0);
      for (int l = slot0; l < slot0 + nslots; ++l) v = v + cvt<double>(vpool[l * pool_stride + o]);
      acc = acc + wc[k] * v;
    }
    const long long uo = (long long)r * P.N + gflat;
    u[uo] = accumulate ? u[uo] + acc : acc;
  }
  (void)nc;
}

template <typename T>
void launch_assemble_u(const Problem& P, const SubDesc* d_subs, const PartTables& pt, int slot0,
                       int nslots, int accumulate, int nrhs, int kmax, const cpx<T>* vpool,
                       long long pool_stride, cpx<double>* u, hipStream_t s) {
  hipLaunchKernelGGL(k_assemble_u<T>, dim3(cdiv_u(P.N, 256)), dim3(256), 0, s, P, d_subs, pt,
                     slot0, nslots, accumulate, nrhs, kmax, vpool, pool_stride, u);
}

template <typename T>
__global__ void k_zero(cpx<T>* p, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = mk((T)0, (T)0);
}
template <typename T>
void launch_zero(cpx<T>* p, long long n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_zero<T>, dim3(cdiv_u(n, 256)), dim3(256), 0, s, p, n);
}

template <typename T>
__global__ void k_pack_local(const cpx<double>* src, cpx<T>* dst, long long nloc, int nrhs) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nloc * nrhs) dst[i] = cvt<T>(src[i]);
}
template <typename T>
__global__ void k_unpack_local(const cpx<T>* src, cpx<double>* dst, long long nloc, int nrhs) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nloc * nrhs) dst[i] = cvt<double>(src[i]);
}
template <typename T>
void launch_pack_local(const cpx<double>* src, cpx<T>* dst, long long nloc, int nrhs, int kmax,
                       hipStream_t s) {
  (void)kmax;
  hipLaunchKernelGGL(k_pack_local<T>, dim3(cdiv_u(nloc * nrhs, 256)), dim3(256), 0, s, src, dst,
                     nloc, nrhs);
}
template <typename T>
void launch_unpack_local(const cpx<T>* src, cpx<double>* dst, long long nloc, int nrhs, int kmax,
                         hipStream_t s) {
  (void)kmax;
  hipLaunchKernelGGL(k_unpack_local<T>, dim3(cdiv_u(nloc * nrhs, 256)), dim3(256), 0, s, src,
                     dst, nloc, nrhs);
}

// ============================================================================
// a7: y = M x, FP64 global 5/7-point operator (coefficients per cell).
// ============================================================================
__global__ void k_apply_op(Problem P, const cpx<double>* diag, const cpx<double>* cx,
                           const cpx<double>* cy, const cpx<double>* cz, const cpx<double>* x,
                           cpx<double>* y, int nrhs) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P.N) return;
  const int ix = (int)(c % P.ng[0]);
  const long long q = c / P.ng[0];
  const int iy = (int)(q % P.ng[1]);
  const int iz = (int)(q / P.ng[1]);
  const long long sy = P.ng[0], sz = (long long)P.ng[0] * P.ng[1];
  const cpx<double> d = diag[c];
  const cpx<double> xp = ix + 1 < P.ng[0] ? cx[c] : mk(0.0, 0.0);
  const cpx<double> xm = ix > 0 ? cx[c - 1] : mk(0.0, 0.0);
  const cpx<double> yp = iy + 1 < P.ng[1] ? cy[c] : mk(0.0, 0.0);
  const cpx<double> ym = iy > 0 ? cy[c - sy] : mk(0.0, 0.0);
  cpx<double> zp = mk(0.0, 0.0), zm = mk(0.0, 0.0);
  if (P.dim == 3) {
    zp = iz + 1 < P.ng[2] ? cz[c] : mk(0.0, 0.0);
    zm = iz > 0 ? cz[c - sz] : mk(0.0, 0.0);
  }
  for (int r = 0; r < nrhs; ++r) {
    const cpx<double>* xr = x + (long long)r * P.N;
    cpx<double> acc = d * xr[c];
    if (ix + 1 < P.ng[0]) acc = acc + xp * xr[c + 1];
    if (ix > 0) acc = acc + xm * xr[c - 1];
    if (iy + 1 < P.ng[1]) acc = acc + yp * xr[c + sy];
    if (iy > 0) acc = acc + ym * xr[c - sy];
    if (P.dim == 3) {
      if (iz + 1 < P.ng[2]) acc = acc + zp * xr[c + sz];
      if (iz > 0) acc = acc + zm * xr[c - sz];
    }
    y[(long long)r * P.N + c] = acc;
  }
}

void launch_apply_op(const Problem& P, const cpx<double>* diag, const cpx<double>* cx,
                     const cpx<double>* cy, const cpx<double>* cz, const cpx<double>* x,
                     cpx<double>* y, int nrhs, hipStream_t s) {
  if (nrhs <= 0) return;
  hipLaunchKernelGGL(k_apply_op, dim3(cdiv_u(P.N, 256)), dim3(256), 0, s, P, diag, cx, cy, cz, x,
                     y, nrhs);
}

// ============================================================================
// a8: FP64 Krylov kernels (batched over RHS).  Reductions are two-stage with a
// fixed summation order, so results are reproducible run to run.
// ============================================================================
__device__ inline cpx<double> block_sum(cpx<double> v, cpx<double>* sh) {
  for (int o = 32; o > 0; o >>= 1) {
    v.re += __shfl_down(v.re, o, 64);
    v.im += __shfl_down(v.im, o, 64);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  cpx<double> t = mk(0.0, 0.0);
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t = t + sh[w];
  __syncthreads();
  return t;
}

// part[(i * nrhs + r) * nblk + b]
__global__ __launch_bounds__(256) void k_mdot(const cpx<double>* V, int nv, const cpx<double>* w,
                                              int nrhs, long long N, cpx<double>* part,
                                              int nblk) {
  __shared__ cpx<double> sh[4];
  const int r = blockIdx.y;
  const int b = blockIdx.x;
  const cpx<double>* wr = w + (long long)r * N;
  // eight basis vectors per pass over w (one pass for the first eight Arnoldi steps)
  for (int i0 = 0; i0 < nv; i0 += 8) {
    cpx<double> acc[8];
    for (int t = 0; t < 8; ++t) acc[t] = mk(0.0, 0.0);
    for (long long c = (long long)b * blockDim.x + threadIdx.x; c < N;
         c += (long long)nblk * blockDim.x) {
      const cpx<double> wv = wr[c];
#pragma unroll
      for (int t = 0; t < 8; ++t)
        if (i0 + t < nv) fma_acc(acc[t], conj(V[((long long)(i0 + t) * nrhs + r) * N + c]), wv);
    }
    for (int t = 0; t < 8 && i0 + t < nv; ++t) {
      cpx<double> s = block_sum(acc[t], sh);
      if (threadIdx.x == 0) part[((long long)(i0 + t) * nrhs + r) * nblk + b] = s;
    }
  }
}

__global__ void k_mdot_final(const cpx<double>* part, int nv, int nrhs, int nblk,
                             cpx<double>* out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nv * nrhs) return;
  cpx<double> s = mk(0.0, 0.0);
  for (int b = 0; b < nblk; ++b) s = s + part[(long long)idx * nblk + b];
  out[idx] = s;
}

void launch_mdot(const cpx<double>* V, int nv, const cpx<double>* w, int nrhs, long long N,
                 cpx<double>* part, int nblk, cpx<double>* out, hipStream_t s) {
  if (nv <= 0 || nrhs <= 0) return;
  hipLaunchKernelGGL(k_mdot, dim3(nblk, nrhs), dim3(256), 0, s, V, nv, w, nrhs, N, part, nblk);
  hipLaunchKernelGGL(k_mdot_final, dim3(cdiv_u((long long)nv * nrhs, 256)), dim3(256), 0, s, part,
                     nv, nrhs, nblk, out);
}

__global__ void k_maxpy(const cpx<double>* V, int nv, const cpx<double>* coef, double sign,
                        cpx<double>* w, int nrhs, long long N) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (c >= N) return;
  cpx<double> acc = mk(0.0, 0.0);
  for (int i = 0; i < nv; ++i) fma_acc(acc, coef[i * nrhs + r], V[((long long)i * nrhs + r) * N + c]);
  const long long o = (long long)r * N + c;
  w[o] = w[o] + sign * acc;
}

void launch_maxpy(const cpx<double>* V, int nv, const cpx<double>* coef, double sign,
                  cpx<double>* w, int nrhs, long long N, hipStream_t s) {
  if (nv <= 0 || nrhs <= 0) return;
  hipLaunchKernelGGL(k_maxpy, dim3(cdiv_u(N, 256), nrhs), dim3(256), 0, s, V, nv, coef, sign, w,
                     nrhs, N);
}

__global__ void k_scale(const cpx<double>* src, const double* scal, cpx<double>* dst, int nrhs,
                        long long N) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (c >= N) return;
  const long long o = (long long)r * N + c;
  dst[o] = scal[r] * src[o];
}
void launch_scale(const cpx<double>* src, const double* scal, cpx<double>* dst, int nrhs,
                  long long N, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(cdiv_u(N, 256), nrhs), dim3(256), 0, s, src, scal, dst, nrhs, N);
}

__global__ void k_sub(const cpx<double>* a, const cpx<double>* b, cpx<double>* y, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a[i] - b[i];
}
void launch_sub(const cpx<double>* a, const cpx<double>* b, cpx<double>* y, long long n,
                hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_sub, dim3(cdiv_u(n, 256)), dim3(256), 0, s, a, b, y, n);
}
__global__ void k_conj(const cpx<double>* a, cpx<double>* y, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = conj(a[i]);
}
void launch_conj(const cpx<double>* a, cpx<double>* y, long long n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_conj, dim3(cdiv_u(n, 256)), dim3(256), 0, s, a, y, n);
}
__global__ void k_gather_rhs(const cpx<double>* src, const int* idx, cpx<double>* dst,
                             long long N) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (c < N) dst[(long long)r * N + c] = src[(long long)idx[r] * N + c];
}
__global__ void k_scatter_rhs(const cpx<double>* src, const int* idx, cpx<double>* dst,
                              long long N) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (c < N) dst[(long long)idx[r] * N + c] = src[(long long)r * N + c];
}
__global__ void k_zero_rhs(cpx<double>* dst, const int* idx, long long N) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < N) dst[(long long)idx[blockIdx.y] * N + c] = mk(0.0, 0.0);
}
void launch_zero_rhs(cpx<double>* dst, const int* idx, int nsel, long long N, hipStream_t s) {
  if (nsel <= 0) return;
  hipLaunchKernelGGL(k_zero_rhs, dim3(cdiv_u(N, 256), nsel), dim3(256), 0, s, dst, idx, N);
}
void launch_gather_rhs(const cpx<double>* src, const int* idx, cpx<double>* dst, int nsel,
                       long long N, hipStream_t s) {
  if (nsel > 0)
    hipLaunchKernelGGL(k_gather_rhs, dim3(cdiv_u(N, 256), nsel), dim3(256), 0, s, src, idx, dst, N);
}
void launch_scatter_rhs(const cpx<double>* src, const int* idx, cpx<double>* dst, int nsel,
                        long long N, hipStream_t s) {
  if (nsel > 0)
    hipLaunchKernelGGL(k_scatter_rhs, dim3(cdiv_u(N, 256), nsel), dim3(256), 0, s, src, idx, dst,
                       N);
}

// ============================================================================
// a9: FWI.  res = P u - d at the receivers; adjoint source conj(P^T res)
// (summed per cell in receiver order by one thread per source); misfit
// partials per source; gradient -omega^2 Re(J sum_s y_s u_s) with
// y_s = M^{-1} conj(P^T res_s) (so lam_s = conj(y_s)), transposed through
// the clamp extension onto the physical cells.
// ============================================================================
__global__ void k_fwi_residual(const cpx<double>* u, int nsrc, long long N, const long long* rec,
                               int nrec, const cpx<double>* dobs, cpx<double>* res,
                               cpx<double>* adj, double* mpart) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsrc) return;
  double acc = 0.0;
  for (int k = 0; k < nrec; ++k) {
    const cpx<double> rv = u[(long long)s * N + rec[k]] - dobs[(long long)s * nrec + k];
    res[(long long)s * nrec + k] = rv;
    acc += abs2(rv);
  }
  for (int k = 0; k < nrec; ++k) {
    const long long o = (long long)s * N + rec[k];
    adj[o] = adj[o] + conj(res[(long long)s * nrec + k]);
  }
  mpart[s] = 0.5 * acc;
}
void launch_fwi_residual(const cpx<double>* u, int nsrc, long long N, const long long* rec,
                         int nrec, const cpx<double>* dobs, cpx<double>* res,
                         cpx<double>* adj_rhs, double* misfit_part, hipStream_t s) {
  hipLaunchKernelGGL(k_fwi_residual, dim3(cdiv_u(nsrc, 64)), dim3(64), 0, s, u, nsrc, N, rec, nrec,
                     dobs, res, adj_rhs, misfit_part);
}

__global__ void k_fwi_gradient(Problem P, const cpx<double>* u, const cpx<double>* y, int nsrc,
                               double* grad) {
  const long long pflat = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nphys = (long long)P.n[0] * P.n[1] * (P.dim == 3 ? P.n[2] : 1);
  if (pflat >= nphys) return;
  int p[3];
  p[0] = (int)(pflat % P.n[0]);
  const long long q = pflat / P.n[0];
  p[1] = (int)(q % P.n[1]);
  p[2] = (int)(q / P.n[1]);
  int lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    if (a >= P.dim) { lo[a] = 0; hi[a] = 0; continue; }
    lo[a] = p[a] == 0 ? 0 : p[a] + P.pml;
    hi[a] = p[a] == P.n[a] - 1 ? P.ng[a] - 1 : p[a] + P.pml;
  }
  double acc = 0.0;
  for (int gz = lo[2]; gz <= hi[2]; ++gz)
    for (int gy = lo[1]; gy <= hi[1]; ++gy)
      for (int gx = lo[0]; gx <= hi[0]; ++gx) {
        const long long c = ((long long)gz * P.ng[1] + gy) * P.ng[0] + gx;
        const double h = P.h;
        const double xs[3] = {(gx - P.pml + 0.5) * h, (gy - P.pml + 0.5) * h,
                              (gz - P.pml + 0.5) * h};
        cpx<double> J = mk(1.0, 0.0);
        for (int a = 0; a < P.dim; ++a) J = J * stretch(xs[a], 0.0, P.n[a] * h, P);
        cpx<double> sum = mk(0.0, 0.0);
        for (int s = 0; s < nsrc; ++s)
          fma_acc(sum, y[(long long)s * P.N + c], u[(long long)s * P.N + c]);
        acc += (J * sum).re;
      }
  grad[pflat] = -P.omega * P.omega * acc;
}
void launch_fwi_gradient(const Problem& P, const cpx<double>* u, const cpx<double>* y, int nsrc,
                         double* grad, hipStream_t s) {
  const long long nphys = (long long)P.n[0] * P.n[1] * (P.dim == 3 ? P.n[2] : 1);
  hipLaunchKernelGGL(k_fwi_gradient, dim3(cdiv_u(nphys, 256)), dim3(256), 0, s, P, u, y, nsrc,
                     grad);
}

__global__ void k_sample(const cpx<double>* u, int nsrc, long long N, const long long* rec,
                         int nrec, cpx<double>* d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsrc * nrec) return;
  const int s = i / nrec, k = i - s * nrec;
  d[i] = u[(long long)s * N + rec[k]];
}
void launch_sample(const cpx<double>* u, int nsrc, long long N, const long long* rec, int nrec,
                   cpx<double>* d, hipStream_t s) {
  hipLaunchKernelGGL(k_sample, dim3(cdiv_u((long long)nsrc * nrec, 256)), dim3(256), 0, s, u, nsrc,
                     N, rec, nrec, d);
}

// ---- explicit instantiations
#define DSD_INST(T)                                                                              \
  template void launch_convert<T>(const cpx<double>*, cpx<T>*, long long, hipStream_t);          \
  template void launch_invert<T>(const SubDesc*, const FactorJob*, int, int, cpx<double>*,      \
                                 cpx<T>*, int*, int*, cpx<double>*, double*, hipStream_t);       \
  template void launch_chain<T>(int, int, const SubDesc*, const int4*, int, int, int, int,      \
                                const cpx<T>*, const cpx<T>*, const cpx<T>*, cpx<T>*, long long, \
                                hipStream_t);                                                    \
  template size_t chain_lds_bytes<T>(int, int);                                                 \
  template void launch_init_rhs<T>(const Problem&, const SubDesc*, const int2*, int, long long, \
                                   int, int, const cpx<double>*, cpx<T>*, long long, int,        \
                                   hipStream_t);                                                 \
  template void launch_zero<T>(cpx<T>*, long long, hipStream_t);                                \
  template void launch_pull<T>(const Problem&, const SubDesc*, const int2*, int, const Edge*,   \
                               const int2*, long long, int, int, const cpx<T>*, long long,       \
                               const cpx<T>*, const cpx<T>*, const cpx<T>*, const cpx<T>*,       \
                               cpx<T>*, hipStream_t);                                            \
  template void launch_assemble_u<T>(const Problem&, const SubDesc*, const PartTables&, int,    \
                                     int, int, int, int, const cpx<T>*, long long, cpx<double>*, \
                                     hipStream_t);                                               \
  template void launch_bcr_invert<T>(const BcrInvJob*, int, int, cpx<double>*, cpx<T>*, int*,  \
                                     int*, cpx<double>*, double*, hipStream_t);                  \
  template void launch_bcr_copy<T>(const BcrCopyJob*, int, int, const cpx<double>*, cpx<T>*,    \
                                   hipStream_t);                                                 \
  template void launch_bcr_solve<T>(int, const SubDesc*, const BcrJob*, int, int, int, int, int,\
                                    int, int, const cpx<T>*, const cpx<T>*, cpx<T>*, cpx<T>*,    \
                                    long long, hipStream_t);                                     \
  template size_t bcr_launch_lds_bytes<T>(int, int, int, int, int);                             \
  template void launch_bcr_dense_store<T>(const BcrDenseJob*, int, int, const cpx<double>*,     \
                                          cpx<T>*, hipStream_t);                                 \
  template void launch_bcr_dfwd<T>(const SubDesc*, const BcrJob*, int, int, int, int,           \
                                   const cpx<T>*, cpx<T>*, const cpx<T>*, long long,            \
                                   hipStream_t);                                                 \
  template int bcr_kg<T>(int, int);                                                             \
  template size_t bcr_lds_bytes<T>(int, int, int);                                              \
  template void launch_pack_local<T>(const cpx<double>*, cpx<T>*, long long, int, int,          \
                                     hipStream_t);                                               \
  template void launch_unpack_local<T>(const cpx<T>*, cpx<double>*, long long, int, int,        \
                                       hipStream_t);
DSD_INST(float)
DSD_INST(double)

}  // namespace dsd
