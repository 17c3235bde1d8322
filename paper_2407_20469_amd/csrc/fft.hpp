// Batched 2D FFTs for gfx950: self-sorting (Stockham) radix-4 passes with a
// final radix-2 pass when log2 L is odd, one sequence set resident in LDS per
// workgroup.  A 2D transform is a row pass and a column pass; each pass loads
// its lines from HBM once (column panels of NSEQ adjacent columns so that every
// row segment is a contiguous 64-128 B read), runs all stages in LDS and
// stores once.  Element-wise work of the method (log, masks, exp, |.|^2,
// scaling, zero embedding) is fused into the load / between-transform / store
// hooks of the pass so no intermediate array is materialised.
//
// Stage s with radix R and current sub-transform length NS maps butterfly j to
// inputs j + r L/R, multiplies input r by w^{(j mod NS) r L/(NS R)}, and writes
// output r to (j / NS) NS R + (j mod NS) + r NS.
#pragma once

#include <type_traits>

#include "common.hpp"

namespace apic {

template <bool INV, class C>
__device__ __forceinline__ void bfly4(C &a0, C &a1, C &a2, C &a3) {
  const C s02 = cadd(a0, a2), d02 = csub(a0, a2), s13 = cadd(a1, a3), d13 = csub(a1, a3);
  C jd;  // forward: -j * d13, inverse: +j * d13
  if (INV) {
    jd.x = -d13.y;
    jd.y = d13.x;
  } else {
    jd.x = d13.y;
    jd.y = -d13.x;
  }
  a0 = cadd(s02, s13);
  a2 = csub(s02, s13);
  a1 = cadd(d02, jd);
  a3 = csub(d02, jd);
}

// Element (seq, pos) lives at buf[seq * SS + pos * PS].  SF: consecutive
// threads take consecutive sequences (column panels) instead of consecutive
// butterflies of one sequence (rows).
template <class C, int L, int NSEQ, int NT, bool INV, bool SF, int SS, int PS, int R, int NS>
__device__ __forceinline__ void fft_stage(C *buf, const C *__restrict__ tw) {
  constexpr int NBSEQ = L / R;
  constexpr int NB = NSEQ * NBSEQ;
  constexpr int BPT = (NB + NT - 1) / NT;
  C v[BPT][R];
  const int tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < BPT; ++k) {
    const int b = tid + k * NT;
    if (NB % NT == 0 || b < NB) {
      const int seq = SF ? b % NSEQ : b / NBSEQ;
      const int jj = SF ? b / NSEQ : b % NBSEQ;
#pragma unroll
      for (int r = 0; r < R; ++r) v[k][r] = buf[seq * SS + (jj + r * NBSEQ) * PS];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < BPT; ++k) {
    const int b = tid + k * NT;
    if (NB % NT == 0 || b < NB) {
      const int seq = SF ? b % NSEQ : b / NBSEQ;
      const int jj = SF ? b / NSEQ : b % NBSEQ;
      const int jm = jj & (NS - 1);
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          C w = tw[jm * r * (L / (NS * R))];
          if (INV) w.y = -w.y;
          v[k][r] = cmul(v[k][r], w);
        }
      }
      if constexpr (R == 4) {
        bfly4<INV>(v[k][0], v[k][1], v[k][2], v[k][3]);
      } else {
        const C t0 = v[k][0];
        v[k][0] = cadd(t0, v[k][1]);
        v[k][1] = csub(t0, v[k][1]);
      }
      const int base = (jj / NS) * NS * R + jm;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[seq * SS + (base + r * NS) * PS] = v[k][r];
    }
  }
  __syncthreads();
}

// All stages of an L-point transform of NSEQ sequences held in LDS.  The
// caller must synchronise after filling `buf`; results are visible on return.
template <class C, int L, int NSEQ, int NT, bool INV, bool SF, int SS, int PS, int NS = 1>
__device__ __forceinline__ void lds_fft(C *buf) {
  if constexpr (NS < L) {
    constexpr int R = ((L / NS) % 4 == 0) ? 4 : 2;
    fft_stage<C, L, NSEQ, NT, INV, SF, SS, PS, R, NS>(buf, tw_table<C>(L));
    lds_fft<C, L, NSEQ, NT, INV, SF, SS, PS, NS * R>(buf);
  }
}

constexpr int kFftThreads = 256;

template <class C, int L> struct RowShape {
  static constexpr int ROWS = (4 * kFftThreads) / L;  // rows per workgroup
};
template <class C, int L> struct ColShape {
  // Column panel width: up to 16 columns, at most 2048 elements (8 per
  // thread; 32 KiB of complex128), at least 4 columns (64 B of complex128
  // per row).  Small panels leave LDS for several workgroups per CU, which
  // hides the strided HBM reads better than wider rows would.
  static constexpr int NSEQ = (2048 / L >= 16) ? 16 : (2048 / L >= 8) ? 8 : 4;
};
// The alternative panel the batch autotuner may pick per geometry class:
// twice as wide (longer contiguous row segments, fewer workgroups) while the
// panel stays within 64 KiB of LDS and 16 columns, else half as wide (more
// workgroups per CU).  A column's transform is the same either way, so the
// results are identical; only the memory access pattern changes.
template <class C, int L> struct ColShapeAlt {
  static constexpr int N0 = ColShape<C, L>::NSEQ;
  static constexpr int NSEQ =
      (2 * N0 <= 16 && 2 * N0 * L * (int)sizeof(C) <= 65536) ? 2 * N0 : (N0 >= 8 ? N0 / 2 : N0);
};

// Row pass: workgroup = ROWS consecutive rows of one 2D array.  Op provides
//   static constexpr bool INV1, TWO, INV2;
//   C load(int arr, int y, int x); void mid(int arr, int y, int x, C &v);
//   void store(int arr, int y, int x, C v);
//   int rows() (rows transformed per array) and int row_of(int r) (the array
//   row of the r-th transformed row, for passes that skip all-zero rows).
template <class C, int L, class Op>
__global__ __launch_bounds__(kFftThreads) void k_rows(Op op) {
  constexpr int ROWS = RowShape<C, L>::ROWS;
  __shared__ C buf[ROWS * L];
  const int groups = op.rows() / ROWS;
  const int arr = blockIdx.x / groups;
  const int rbase = (blockIdx.x % groups) * ROWS;
  for (int e = threadIdx.x; e < ROWS * L; e += kFftThreads) {
    const int rr = e / L, x = e % L;
    buf[e] = op.load(arr, op.row_of(rbase + rr), x);
  }
  __syncthreads();
  lds_fft<C, L, ROWS, kFftThreads, Op::INV1, false, L, 1>(buf);
  if constexpr (Op::TWO) {
    for (int e = threadIdx.x; e < ROWS * L; e += kFftThreads) {
      const int rr = e / L, x = e % L;
      op.mid(arr, op.row_of(rbase + rr), x, buf[e]);
    }
    __syncthreads();
    lds_fft<C, L, ROWS, kFftThreads, Op::INV2, false, L, 1>(buf);
  }
  for (int e = threadIdx.x; e < ROWS * L; e += kFftThreads) {
    const int rr = e / L, x = e % L;
    op.store(arr, op.row_of(rbase + rr), x, buf[e]);
  }
}

// An op of a two-transform column pass may read one float per element for its
// between-transform hook (SIDE = true: side() and mid_side()); the column pass
// issues those reads with its loads, so they are not a dependent wait between
// the two transforms.
template <class Op, class = void> struct SideOf {
  static constexpr bool value = false;
};
template <class Op> struct SideOf<Op, std::void_t<decltype(Op::SIDE)>> {
  static constexpr bool value = Op::SIDE;
};

// Column pass: workgroup = NSEQ adjacent columns of one 2D array (all L rows).
template <class C, int L, class Op, int NSEQ = ColShape<C, L>::NSEQ>
__global__ __launch_bounds__(kFftThreads) void k_cols(Op op) {
  __shared__ C buf[L * NSEQ];
  constexpr int groups = L / NSEQ;
  constexpr bool kSide = SideOf<Op>::value;
  constexpr int PER = (L * NSEQ) / kFftThreads;  // elements per thread
  static_assert(PER * kFftThreads == L * NSEQ, "whole elements per thread");
  const int bid = xcd_remap(blockIdx.x, gridDim.x);  // neighbouring panels on one XCD
  const int arr = bid / groups;
  const int x0 = (bid % groups) * NSEQ;
  float side[kSide ? PER : 1];
  if constexpr (kSide) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = threadIdx.x + i * kFftThreads;
      const int y = e / NSEQ, c = e % NSEQ;
      buf[e] = op.load(arr, y, x0 + c);
      side[i] = op.side(arr, y, x0 + c);
    }
  } else {
    for (int e = threadIdx.x; e < L * NSEQ; e += kFftThreads) {
      const int y = e / NSEQ, c = e % NSEQ;
      buf[e] = op.load(arr, y, x0 + c);
    }
  }
  __syncthreads();
  lds_fft<C, L, NSEQ, kFftThreads, Op::INV1, true, 1, NSEQ>(buf);
  if constexpr (Op::TWO) {
    if constexpr (kSide) {
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int e = threadIdx.x + i * kFftThreads;
        const int y = e / NSEQ, c = e % NSEQ;
        op.mid_side(arr, y, x0 + c, buf[e], side[i]);
      }
    } else {
      for (int e = threadIdx.x; e < L * NSEQ; e += kFftThreads) {
        const int y = e / NSEQ, c = e % NSEQ;
        op.mid(arr, y, x0 + c, buf[e]);
      }
    }
    __syncthreads();
    lds_fft<C, L, NSEQ, kFftThreads, Op::INV2, true, 1, NSEQ>(buf);
  }
  for (int e = threadIdx.x; e < L * NSEQ; e += kFftThreads) {
    const int y = e / NSEQ, c = e % NSEQ;
    op.store(arr, y, x0 + c, buf[e]);
  }
}

template <class C, int L> inline int row_blocks(int arrays, int rows) {
  return arrays * (rows / RowShape<C, L>::ROWS);
}
template <class C, int L, int NSEQ = ColShape<C, L>::NSEQ> inline int col_blocks(int arrays) {
  return arrays * (L / NSEQ);
}

// Plain batched transform of contiguous L x L arrays (library utility).
template <class C, int L, bool INV> struct OpPlainRows {
  static constexpr bool INV1 = INV, TWO = false, INV2 = false;
  const C *in;
  C *out;
  __device__ int rows() const { return L; }
  __device__ int row_of(int r) const { return r; }
  __device__ C load(int a, int y, int x) const { return in[((int64_t)a * L + y) * L + x]; }
  __device__ void mid(int, int, int, C &) const {}
  __device__ void store(int a, int y, int x, C v) const { out[((int64_t)a * L + y) * L + x] = v; }
};
template <class C, int L, bool INV> struct OpPlainCols {
  static constexpr bool INV1 = INV, TWO = false, INV2 = false;
  C *io;
  __device__ C load(int a, int y, int x) const { return io[((int64_t)a * L + y) * L + x]; }
  __device__ void mid(int, int, int, C &) const {}
  __device__ void store(int a, int y, int x, C v) const { io[((int64_t)a * L + y) * L + x] = v; }
};

}  // namespace apic
