// Device helpers shared by the HIP translation units of libadl: vector
// loads and stores with (row start, column) addressing, the boundary rule for
// row indices, and the fixed-order grid reduction with a last-block ticket
// (used by the one-pass kernels: Gershgorin bound, field statistics).
#pragma once

#include "internal.h"

#include <cmath>

namespace adl {

enum { MODE_ZERO = 0, MODE_EDGE = 1 };

template <typename T, int VEC>
__device__ __forceinline__ void load_c(const T* __restrict__ a, long off, double (&c)[VEC]) {
  if constexpr (VEC == 1) {
    c[0] = (double)a[off];
  } else if constexpr (sizeof(T) == 8) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 v = *reinterpret_cast<const d2*>(a + off);
    c[0] = v.x;
    c[1] = v.y;
  } else {
    typedef float f2 __attribute__((ext_vector_type(2)));
    const f2 v = *reinterpret_cast<const f2*>(a + off);
    c[0] = (double)v.x;
    c[1] = (double)v.y;
  }
}

template <typename T, int VEC>
__device__ __forceinline__ void store_c(T* __restrict__ a, long off, const double (&c)[VEC]) {
  if constexpr (VEC == 1) {
    a[off] = (T)c[0];
  } else if constexpr (sizeof(T) == 8) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    d2 v;
    v.x = c[0];
    v.y = c[1];
    *reinterpret_cast<d2*>(a + off) = v;
  } else {
    typedef float f2 __attribute__((ext_vector_type(2)));
    f2 v;
    v.x = (float)c[0];
    v.y = (float)c[1];
    *reinterpret_cast<f2*>(a + off) = v;
  }
}

// Element addressing as (row start, column): the row start is wave-uniform
// (kept in SGPRs), the column part a 32-bit byte offset, which is the
// global load/store form with a scalar base and a 32-bit vector offset; no
// 64-bit address is held in VGPRs.
template <typename T>
__device__ __forceinline__ const T* at_col(const T* rowp, int col) {
  return reinterpret_cast<const T*>(reinterpret_cast<const char*>(rowp) + (unsigned)(col * (int)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ T* at_col(T* rowp, int col) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(rowp) + (unsigned)(col * (int)sizeof(T)));
}
template <typename T, int VEC>
__device__ __forceinline__ void ldr(const T* rowp, int col, double (&c)[VEC]) {
  load_c<T, VEC>(at_col(rowp, col), 0, c);
}
template <typename T>
__device__ __forceinline__ double ld1(const T* rowp, int col) {
  return (double)*at_col(rowp, col);
}
template <typename T, int VEC>
__device__ __forceinline__ void str(T* rowp, int col, const double (&c)[VEC]) {
  store_c<T, VEC>(at_col(rowp, col), 0, c);
}

// Forms for vectors that one launch reads or writes exactly once (p_k in,
// y and p out), with the non-temporal hint when NT is set: on working sets
// beyond the caches their lines then go first, so the rows that
// neighbouring waves re-read stay in L2.  (A template parameter, not a
// runtime flag: the compiler merges the two forms of a runtime branch and
// drops the hint.)
template <bool NT, typename T, int VEC>
__device__ __forceinline__ void ldr_s(const T* rowp, int col, double (&c)[VEC]) {
  const T* a = at_col(rowp, col);
  if constexpr (!NT) {
    load_c<T, VEC>(a, 0, c);
  } else if constexpr (VEC == 1) {
    c[0] = (double)__builtin_nontemporal_load(a);
  } else if constexpr (sizeof(T) == 8) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 v = __builtin_nontemporal_load(reinterpret_cast<const d2*>(a));
    c[0] = v.x;
    c[1] = v.y;
  } else {
    typedef float f2 __attribute__((ext_vector_type(2)));
    const f2 v = __builtin_nontemporal_load(reinterpret_cast<const f2*>(a));
    c[0] = (double)v.x;
    c[1] = (double)v.y;
  }
}
template <bool NT, typename T, int VEC>
__device__ __forceinline__ void str_s(T* rowp, int col, const double (&c)[VEC]) {
  T* a = at_col(rowp, col);
  if constexpr (!NT) {
    store_c<T, VEC>(a, 0, c);
  } else if constexpr (VEC == 1) {
    __builtin_nontemporal_store((T)c[0], a);
  } else if constexpr (sizeof(T) == 8) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    d2 v;
    v.x = c[0];
    v.y = c[1];
    __builtin_nontemporal_store(v, reinterpret_cast<d2*>(a));
  } else {
    typedef float f2 __attribute__((ext_vector_type(2)));
    f2 v;
    v.x = (float)c[0];
    v.y = (float)c[1];
    __builtin_nontemporal_store(v, reinterpret_cast<f2*>(a));
  }
}

// Row index after the boundary rule; zero = the whole row is a zero ghost row.
__device__ __forceinline__ int map_row(int r, int ny, int bc, int mode, bool& zero) {
  zero = false;
  if (r >= 0 && r < ny) return r;
  if (bc == BC_PERIODIC) return r < 0 ? r + ny : r - ny;
  if (mode == MODE_EDGE) return r < 0 ? 0 : ny - 1;
  zero = true;
  return 0;
}

template <int VEC>
struct RowN {
  double c[VEC];
  double l, r;
  __device__ __forceinline__ double at(int v) const { return c[v]; }
  __device__ __forceinline__ double west(int v) const { return v == 0 ? l : c[v - 1]; }
  __device__ __forceinline__ double east(int v) const { return v == VEC - 1 ? r : c[v + 1]; }
};

template <int VEC>
struct RowC {
  double c[VEC];
};

__device__ __forceinline__ double nanmax(double a, double b) {
  // max that propagates NaN
  return (a != a || b != b) ? (a + b) : (a > b ? a : b);
}

// Block partials -> last block sums them in fixed order -> fin(totals).
// Sums for the first NS values, NaN-propagating max for the rest.  nb blocks
// take part (block b writes partial b), counted on ctl->ticket; a launch may
// hold several such reductions, each with its own partials and ticket.
template <int NA, int NS, class Fin>
__device__ __forceinline__ void grid_reduce(double (&acc)[NA], double* partials, Ctl* ctl, int nb, int b, Fin fin) {
  __shared__ double sh[NA * 16];
  __shared__ int last;
  // block reduce: sums for k < NS, max for k >= NS
#pragma unroll
  for (int k = 0; k < NA; ++k) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double t = __shfl_xor(acc[k], o);
      acc[k] = (k < NS) ? acc[k] + t : nanmax(acc[k], t);
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NA; ++k) sh[wave * NA + k] = acc[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NA; ++k) {
      double s = sh[k];
      for (int w = 1; w < nw; ++w) s = (k < NS) ? s + sh[w * NA + k] : nanmax(s, sh[w * NA + k]);
      partials[(long)k * nb + b] = s;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned int t = atomicAdd(&ctl->ticket, 1u);
    last = (t == (unsigned)(nb - 1));
  }
  __syncthreads();
  if (!last) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  double tot[NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) {
    double s = (k < NS) ? 0.0 : 0.0;
    bool any = false;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
      const double v = __builtin_nontemporal_load(&partials[(long)k * nb + i]);
      if (k < NS) s += v;
      else s = any ? nanmax(s, v) : v;
      any = true;
    }
    tot[k] = s;
  }
#pragma unroll
  for (int k = 0; k < NA; ++k) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double t = __shfl_xor(tot[k], o);
      tot[k] = (k < NS) ? tot[k] + t : nanmax(tot[k], t);
    }
  }
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NA; ++k) sh[wave * NA + k] = tot[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NA; ++k) {
      double s = sh[k];
      for (int w = 1; w < nw; ++w) s = (k < NS) ? s + sh[w * NA + k] : nanmax(s, sh[w * NA + k]);
      tot[k] = s;
    }
    fin(tot);
    ctl->ticket = 0u;
  }
}

// the same over the whole grid
template <int NA, int NS, class Fin>
__device__ __forceinline__ void grid_reduce(double (&acc)[NA], double* partials, Ctl* ctl, Fin fin) {
  grid_reduce<NA, NS>(acc, partials, ctl, (int)gridDim.x, (int)blockIdx.x, fin);
}



}  // namespace adl
