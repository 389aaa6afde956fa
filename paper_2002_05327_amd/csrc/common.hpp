// Shared device-side types for the dsweep library (complex arithmetic, grid and
// subdomain descriptors).  Internal header: not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace dsd {

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T re, im;
};

template <typename T>
__host__ __device__ inline cpx<T> mk(T r, T i) { cpx<T> z; z.re = r; z.im = i; return z; }
template <typename T>
__host__ __device__ inline cpx<T> operator+(cpx<T> a, cpx<T> b) { return mk(a.re + b.re, a.im + b.im); }
template <typename T>
__host__ __device__ inline cpx<T> operator-(cpx<T> a, cpx<T> b) { return mk(a.re - b.re, a.im - b.im); }
template <typename T>
__host__ __device__ inline cpx<T> operator*(cpx<T> a, cpx<T> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T>
__host__ __device__ inline cpx<T> operator*(T s, cpx<T> b) { return mk(s * b.re, s * b.im); }
template <typename T>
__host__ __device__ inline cpx<T> operator-(cpx<T> a) { return mk(-a.re, -a.im); }
template <typename T>
__host__ __device__ inline cpx<T> conj(cpx<T> a) { return mk(a.re, -a.im); }
template <typename T>
__host__ __device__ inline T abs2(cpx<T> a) { return a.re * a.re + a.im * a.im; }
// acc += a * b
template <typename T>
__host__ __device__ inline void fma_acc(cpx<T>& acc, cpx<T> a, cpx<T> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}
// a / b (Smith's algorithm, avoids overflow of |b|^2)
template <typename T>
__host__ __device__ inline cpx<T> cdiv(cpx<T> a, cpx<T> b) {
  if (fabs(b.re) >= fabs(b.im)) {
    T r = b.im / b.re, den = b.re + b.im * r;
    return mk((a.re + a.im * r) / den, (a.im - a.re * r) / den);
  } else {
    T r = b.re / b.im, den = b.re * r + b.im;
    return mk((a.re * r + a.im) / den, (a.im * r - a.re) / den);
  }
}
template <typename D, typename S>
__host__ __device__ inline cpx<D> cvt(cpx<S> a) { return mk((D)a.re, (D)a.im); }

// One axis of a grid (global or local), in global array indices.
// Array index g is physical cell g - pml, centre (g - pml + 1/2) h.
struct AxisGrid {
  int g0;       // first cell
  int n;        // cells
  double lo;    // physical coordinate of the low-side PML inner face
  double hi;    // ... high side
  int clo;      // medium clamp range (global array indices, inclusive)
  int chi;
};

// Part p of an axis partition.
struct AxisPart {
  int o0, o1;   // own range, global array indices [o0, o1)
  int first;    // 1 if p == 0 (no low-side neighbour)
  int last;     // 1 if p == P-1
};

struct Problem {
  int dim;
  int n[3];       // physical cells
  int ng[3];      // global cells per axis (n + 2 pml); 1 for unused axes
  long long N;    // global cells
  int pml;
  int d;          // overlap
  double h, omega, s0d;  // cell size, angular frequency, sigma0 * W
};

// A subdomain: local grid, factor layout and vector offsets.
struct SubDesc {
  AxisGrid ax[3];
  AxisPart pt[3];     // own range and neighbour flags per axis
  int part[3];
  int dims[3];        // local cells per axis (1 for unused)
  long long nloc;     // local cells
  long long coef_off; // first cell in the coefficient arrays
  long long fac_off;  // first complex entry in the factor array
  long long vec_off;  // first cell in the local vector pools (times max_rhs)
  int nb;             // block size (cells of one x-line in 2D, one xy-plane in 3D)
  int nblk;           // number of blocks (y cells in 2D, z cells in 3D)
  int mid;            // block where the two elimination chains meet
};

// Most incoming transfers of one receiver in one sweep (26 directions in 3D).
constexpr int MAX_IN_EDGES = 32;

// One incoming transfer of a receiver in one sweep (pull model).
struct Edge {
  int sender;
  int t[3];
  unsigned lmask;     // sweeps whose sender solutions feed this transfer
  int lo[3], hi[3];   // box in receiver-local coordinates [lo, hi)
  int off[3];         // sender-local = receiver-local + off
};

// quintic smoothstep cutoff: 1 for t <= 0, 0 for t >= 1
__host__ __device__ inline double bhat(double t) {
  t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
  return 1.0 - t * t * t * (10.0 - 15.0 * t + 6.0 * t * t);
}

// beta^{(a)}_{comp} of a part at global array index g (index-form cutoff)
__host__ __device__ inline double cutoff(const AxisPart& p, int comp, int g, int d) {
  if (comp == 0) return 1.0;
  if (comp > 0) {
    if (p.last) return 1.0;
    return bhat((double)(g - p.o1) / (double)(d - 1));
  }
  if (p.first) return 1.0;
  return bhat((double)(p.o0 - 1 - g) / (double)(d - 1));
}

// complex stretch s = 1 + i sigma/omega at physical coordinate x
__host__ __device__ inline cpx<double> stretch(double x, double lo, double hi, const Problem& P) {
  if (P.pml == 0) return mk(1.0, 0.0);
  double W = P.pml * P.h;
  double t = lo - x;
  double t2 = x - hi;
  t = t > t2 ? t : t2;
  t = t > 0.0 ? t : 0.0;
  double sigma = (P.s0d / W) * (t / W) * (t / W);
  return mk(1.0, sigma / P.omega);
}

}  // namespace dsd
