// Binary-tree blocked QR of a tall matrix (Sec. 3.3, Eq. 1-4).
//
// One batched blocked-Householder engine serves every level:
//   * leaves (Eq. 1): each row block of Y, in the working precision T;
//   * tree nodes (Eq. 2-3): the stacked pair [R_a; R_b] of child R factors,
//     always in float64;
//   * Q formation (Eq. 4): Q = blockdiag(leaf Q) (tree Q) [I; 0] is built top
//     down: every node maps its d x d block M to Q_node [M; 0], whose halves are
//     the children's blocks, and every leaf writes its rows Q_leaf [M_leaf; 0].
// A panel of NB columns is factored by one 512-thread workgroup per matrix
// (rows in registers, one block reduction per reflector), producing LAPACK
// style reflectors (beta = -sign(alpha) |x|, tau = 0 when the part below the
// diagonal is zero) and the compact-WY factor T with H_1 ... H_NB = I - V T V^T.
// Inner panels are applied only inside an outer panel of 64 columns; the
// trailing columns and the Q formation take one rank-64 update
// B -= V (T' (V^T B)) per outer panel on the matrix cores.
#include <vector>

#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace lr {

constexpr int kUpdThreads = 256;
constexpr int kUpdCols = 64;
constexpr int kNarrowCols = 8;  // float columns per workgroup of a narrow update over few matrices

// Column block and matrix of this workgroup for the update kernels (grid:
// column blocks x matrices). Workgroups go to the 8 XCDs round robin by their
// linear id, so the launch order would spread the column blocks of one matrix
// over every XCD and fetch its reflector panel V into every L2. Here each
// XCD takes whole matrices: its k-th workgroup is column block k mod nx of
// matrix xcd + 8 (k / nx). A bijection when the matrix count is a multiple of
// 8; otherwise the launch order is kept.
constexpr int kXcds = 8;
__device__ __forceinline__ void xcd_block(int& cbx, int& b) {
  const int nx = (int)gridDim.x, ny = (int)gridDim.y;
  if (ny % kXcds != 0) {
    cbx = (int)blockIdx.x;
    b = (int)blockIdx.y;
    return;
  }
  const int lin = (int)blockIdx.x + nx * (int)blockIdx.y;
  const int k = lin / kXcds;
  cbx = k % nx;
  b = lin % kXcds + kXcds * (k / nx);
}

// Sum of NV values (NV a power of two <= 16) over the TPB-thread block; every
// thread gets the totals. Inside each 16-lane row a transpose reduction halves
// the vector at every DPP exchange (partners: half-row mirror, xor 8, xor 2,
// xor 1), so after log2(NV) exchanges each lane holds the row sum of one value
// and the remaining exchanges finish the row; the 4 row sums of every wave go
// through LDS and NV threads add them in a fixed order (two barriers).
template <typename T, int NV>
__device__ __forceinline__ T row_exchange(T x, int stage) {
  // stage 0: half-row mirror (l <-> 7 - l within each 8), 1: xor 8, 2: xor 2, 3: xor 1
  if (stage == 0) return dpp_move<0x141>(x);
  if (stage == 1) return dpp_move<0x128>(x);
  if (stage == 2) return dpp_move<0x4E>(x);
  return dpp_move<0xB1>(x);
}

template <typename T, int NV, int TPB>
__device__ __forceinline__ void block_sum_vec(T (&v)[NV], int nvalid, T* red, T* res) {
  static_assert(NV == 1 || NV == 2 || NV == 4 || NV == 8 || NV == 16, "NV must be a power of two <= 16");
  constexpr int NW = TPB / 64;
  constexpr int LOG = NV == 1 ? 0 : NV == 2 ? 1 : NV == 4 ? 2 : NV == 8 ? 3 : 4;
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  // lane bit that decides which half is kept at each transpose stage
  const int kbit[4] = {(lane >> 2) & 1, (lane >> 3) & 1, (lane >> 1) & 1, lane & 1};
  int idx = 0;
  static_for<0, LOG>([&](auto ss) {
    constexpr int S = decltype(ss)::value;
    constexpr int H = NV >> (S + 1);  // half length at this stage
    const bool hi = kbit[S] != 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const T mine = hi ? v[H + i] : v[i];
      const T other = hi ? v[i] : v[H + i];
      v[i] = mine + row_exchange<T, NV>(other, S);
    }
    idx += hi ? H : 0;
  });
  // remaining exchanges: plain sums of the single kept value
  if constexpr (NV == 1) {
    // order xor 1, xor 2, mirror, xor 8 (mirror pairs whole quads once the quads agree)
    v[0] += row_exchange<T, NV>(v[0], 3);
    v[0] += row_exchange<T, NV>(v[0], 2);
    v[0] += row_exchange<T, NV>(v[0], 0);
    v[0] += row_exchange<T, NV>(v[0], 1);
  } else {
    static_for<LOG, 4>([&](auto ss) {
      constexpr int S = decltype(ss)::value;
      v[0] += row_exchange<T, NV>(v[0], S);
    });
  }
  // lanes whose unused bits are zero write their row's sum of value idx
  const int row = lane >> 4;
  bool writer = true;
#pragma unroll
  for (int st = LOG; st < 4; ++st) writer = writer && (kbit[st] == 0);
  if (writer) red[(w * 4 + row) * NV + idx] = v[0];
  __syncthreads();
  if ((int)threadIdx.x < nvalid) {
    T sum = 0;
#pragma unroll
    for (int k = 0; k < NW * 4; ++k) sum += red[k * NV + threadIdx.x];
    res[threadIdx.x] = sum;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = (i < nvalid) ? res[i] : (T)0;
}

// Rows a panel touches. Plain mode: rows p0 .. m-1. Tree mode (tree_d = d > 0,
// the matrix is a stacked pair [R_a; R_b] of upper triangles): reflectors of
// columns < p0 + NB can only be nonzero in the top rows p0 .. p0+NB-1 and the
// bottom rows d .. d+p0+NB-1 (R_a's lower rows and R_b's rows below the panel
// are still exact zeros there), so only those rows are visited.
struct RowMap {
  int p0, ntop, nact, d;
  __device__ __forceinline__ int row(int ci) const { return ci < ntop ? p0 + ci : d + (ci - ntop); }
};

template <int NB>
__device__ __forceinline__ RowMap make_rowmap(int m, int p0, int tree_d) {
  RowMap rm;
  rm.p0 = p0;
  rm.d = tree_d;
  if (tree_d > 0) {
    rm.ntop = min(NB, tree_d - p0);
    const int nbot = min(p0 + NB, tree_d);
    rm.nact = rm.ntop + nbot;
  } else {
    rm.ntop = m - p0;
    rm.nact = m - p0;
  }
  return rm;
}

// Row r of the compact-WY T of one panel: T[r][c] = 0 for c < r, tau_r on the
// diagonal, -tau_c sum_{q=r}^{c-1} T[r][q] y_c[q] right of it, where
// y_c[q] = v_q^T v_c. Register array indices are compile-time constants.
template <typename T, int NB>
__device__ __forceinline__ void row_t_build(T (&row)[NB], int r, int nbw, const T* s_tau, const T* s_y) {
  static_for<0, NB>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    if (c < nbw) {
      if (c == r) {
        row[c] = s_tau[c];
      } else if (c > r) {
        T acc = 0;
#pragma unroll
        for (int q = 0; q < c; ++q)
          if (q >= r) acc += row[q] * s_y[c * NB + q];
        row[c] = -s_tau[c] * acc;
      }
    }
  });
}

// Factor columns [p0, p0 + nbw) of every matrix in the batch.
template <typename T, int RPT, int NB, int TPB>
__global__ __launch_bounds__(TPB) void panel_factor_kernel(T* __restrict__ A, int64_t bstride, int m_full,
                                                                     int m_last, int nbatch, int ld, int p0, int nbw,
                                                                     int tree_d, T* __restrict__ tau_all,
                                                                     int64_t tau_bstride, T* __restrict__ tmat,
                                                                     int64_t t_bstride) {
  __shared__ T red[(TPB / 64) * 4 * NB];
  __shared__ T res[NB];
  __shared__ T s_alpha[NB];
  __shared__ T s_tau[NB];
  __shared__ T s_y[NB * NB];  // s_y[c * NB + c1] = (V^T v_c)[c1], c1 < c
  __shared__ T s_t[NB * NB];

  const int b = blockIdx.x;
  const int m = (b == nbatch - 1) ? m_last : m_full;
  T* M = A + (int64_t)b * bstride;
  const RowMap rm = make_rowmap<NB>(m, p0, tree_d);
  const int rows = rm.nact;
  const int t = threadIdx.x;

  // a full-width panel whose rows start on 16-byte boundaries moves as
  // 16-byte vectors (NB * sizeof(T) / 16 per row) instead of NB scalars
  constexpr int kVecs = NB * (int)sizeof(T) / 16;
  const bool vec = kVecs > 0 && nbw == NB && ((int64_t)ld * sizeof(T)) % 16 == 0 &&
                   (reinterpret_cast<uintptr_t>(M + p0) % 16) == 0;
  T a[RPT][NB];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int lr = t + k * TPB;
    const int64_t roff = (lr < rows) ? (int64_t)rm.row(lr) * ld + p0 : 0;
    if (vec) {
#pragma unroll
      for (int q = 0; q < kVecs; ++q) {
        uint4 v = {0u, 0u, 0u, 0u};
        if (lr < rows) v = reinterpret_cast<const uint4*>(M + roff)[q];
        __builtin_memcpy(&a[k][q * (16 / sizeof(T))], &v, 16);
      }
    } else {
#pragma unroll
      for (int c = 0; c < NB; ++c) a[k][c] = (lr < rows && c < nbw) ? M[roff + c] : (T)0;
    }
  }

  // Expanded at compile time so every register-array index is a constant.
  // Columns c >= nbw are zero: their reflector is the identity (tau = 0) and
  // changes nothing, so all NB columns are processed.
  static_for<0, NB>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    // sigma = |x below the diagonal|^2 ; alpha = diagonal entry (compact row c)
    T part[1] = {0};
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int lr = t + k * TPB;
      if (lr > c && lr < rows) part[0] += a[k][c] * a[k][c];
    }
    if (t == c) s_alpha[c] = a[0][c];
    block_sum_vec<T, 1, TPB>(part, 1, red, res);
    const T sigma = part[0];
    const T alpha = s_alpha[c];
    T tau, beta, scal;
    if (sigma == (T)0) {
      tau = 0;
      beta = alpha;
      scal = 0;
    } else {
      const T nrm = sqrt(alpha * alpha + sigma);
      beta = alpha >= (T)0 ? -nrm : nrm;
      tau = (beta - alpha) / beta;
      scal = (T)1 / (alpha - beta);
    }
    T vk[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int lr = t + k * TPB;
      if (lr > c && lr < rows) {
        a[k][c] *= scal;
        vk[k] = a[k][c];
      } else {
        vk[k] = (lr == c) ? (T)1 : (T)0;
      }
      if (lr == c) a[k][c] = beta;
    }
    // w[c'] = v^T x_{c'} for c' > c ; y[c1] = v_{c1}^T v for c1 < c
    // (i > c: a[k][i] is x_i(lr); i < c: a[k][i] is the stored reflector entry
    // v_i(lr) for lr > i, so both sums are v^T a[:, i]). Rows above c and
    // rows past the panel have vk = 0 and add exact zeros, so no row mask.
    T wv[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) wv[i] = 0;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
#pragma unroll
      for (int i = 0; i < NB; ++i)
        if (i != c) wv[i] += vk[k] * a[k][i];
    }
    block_sum_vec<T, NB, TPB>(wv, nbw, red, res);
    if (t == 0) {
      s_tau[c] = tau;
#pragma unroll
      for (int i = 0; i < NB; ++i)
        if (i < c) s_y[c * NB + i] = wv[i];
    }
    // columns past nbw are zero with wv = 0 there, rows above c have vk = 0:
    // both updates subtract exact zeros, so neither is masked
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
#pragma unroll
      for (int i = 0; i < NB; ++i)
        if (i > c) a[k][i] -= tau * wv[i] * vk[k];
    }
  });
  __syncthreads();

  // write the panel back (R on/above the diagonal, V below)
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int lr = t + k * TPB;
    if (lr < rows) {
      const int64_t roff = (int64_t)rm.row(lr) * ld + p0;
      if (vec) {
#pragma unroll
        for (int q = 0; q < kVecs; ++q) {
          uint4 v;
          __builtin_memcpy(&v, &a[k][q * (16 / sizeof(T))], 16);
          reinterpret_cast<uint4*>(M + roff)[q] = v;
        }
      } else {
#pragma unroll
        for (int c = 0; c < NB; ++c)
          if (c < nbw) M[roff + c] = a[k][c];
      }
    }
  }
  // T (upper triangular): T[c][c] = tau_c, T[0:c, c] = -tau_c T[0:c, 0:c] y_c.
  // Row r of T depends only on row r (T[r][c] = -tau_c sum_{q=r}^{c-1}
  // T[r][q] y_c[q]), so thread r < nbw builds its row left to right in
  // registers, with no barrier.
  for (int i = t; i < NB * NB; i += TPB) s_t[i] = 0;
  __syncthreads();
  if (t < nbw) {
    T row[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) row[c] = 0;
    row_t_build<T, NB>(row, t, nbw, s_tau, s_y);
#pragma unroll
    for (int c = 0; c < NB; ++c) s_t[t * NB + c] = row[c];
  }
  __syncthreads();
  for (int i = t; i < NB * NB; i += TPB) tmat[(int64_t)b * t_bstride + i] = s_t[i];
  if (t < nbw) tau_all[(int64_t)b * tau_bstride + p0 + t] = s_tau[t];
}

// B[rows, cols] <- (I - V T' V^T) B[rows, cols], T' = T^T (TRANS) or T, over the
// rows of the panel's row map. V occupies columns [p0, p0 + NB) of Vmat (unit
// diagonal, zeros above). A 256-thread workgroup owns UC (16 or 64) columns; each thread
// owns 16 bytes of consecutive columns (CPT = 4 floats or 2 doubles) so every
// load keeps a full 16-byte request in flight; row groups are combined by
// cross-lane shuffles and the 4 wave partials in LDS. Every thread reads the
// V rows of its own rows directly, so the row loops have no barriers.

template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  using type = float4;
  static constexpr int n = 4;
};
template <>
struct Vec16<double> {
  using type = double2;
  static constexpr int n = 2;
};

template <typename T, int NB, bool TRANS, int UC>
__global__ __launch_bounds__(kUpdThreads) void panel_apply_kernel(const T* Vmat, int64_t vstride, T* Bmat,
                                                                  int64_t bstride, int m_full, int m_last,
                                                                  int nbatch, int ld, int p0, int nbw, int tree_d,
                                                                  int col_begin, int col_end,
                                                                  const T* __restrict__ tmat, int64_t t_bstride) {
  using VT = typename Vec16<T>::type;
  constexpr int CPT = Vec16<T>::n;         // columns per thread
  constexpr int TPR = UC / CPT;      // threads per row
  constexpr int RG = kUpdThreads / TPR;    // row groups
  constexpr int RGW = 64 / TPR;            // row groups per wave
  __shared__ T red[4][NB][UC];
  __shared__ T wsh[NB][UC];
  __shared__ T Ts[NB * NB];

  int cbx, b;
  xcd_block(cbx, b);
  const int m = (b == nbatch - 1) ? m_last : m_full;
  const T* V = Vmat + (int64_t)b * vstride;
  T* B = Bmat + (int64_t)b * bstride;
  const RowMap rm = make_rowmap<NB>(m, p0, tree_d);
  const int nact = rm.nact;
  const int t = threadIdx.x;
  const int w = t >> 6;
  const int lane = t & 63;
  const int tc = t % TPR;
  const int rg = t / TPR;
  const int cbase = col_begin + cbx * UC;
  const int col0 = cbase + tc * CPT;
  // vector access needs every column of the vector present and 16-byte alignment
  const bool vec_ok = (col0 + CPT <= col_end) && (((int64_t)ld * sizeof(T)) % 16 == 0) && (col0 % CPT == 0);

  if (t < NB * NB) Ts[t] = tmat[(int64_t)b * t_bstride + t];

  // V row ci (panel columns 0..NB-1) with the unit-lower mask; whole rows
  // are read with 16-byte loads when aligned
  const bool vvec = (((int64_t)ld * sizeof(T)) % 16 == 0) && (p0 % CPT == 0) &&
                    (reinterpret_cast<uintptr_t>(V) % 16 == 0) && (NB % CPT == 0) && (nbw == NB);
  auto vrow = [&](int ci, T (&v)[NB]) {
    const T* src = V + (int64_t)rm.row(ci) * ld + p0;
    if (vvec) {  // a full panel: the whole row segment lies inside the row
#pragma unroll
      for (int q = 0; q < NB / CPT; ++q) {
        const VT x = *reinterpret_cast<const VT*>(src + q * CPT);
        __builtin_memcpy(&v[q * CPT], &x, sizeof(VT));
      }
    } else {
#pragma unroll
      for (int i = 0; i < NB; ++i) v[i] = (i < nbw) ? src[i] : (T)0;
    }
    if (ci < NB) {
#pragma unroll
      for (int i = 0; i < NB; ++i) v[i] = (i >= nbw) ? (T)0 : (ci > i ? v[i] : (ci == i ? (T)1 : (T)0));
    }
  };
  auto load_row = [&](int ci, T (&x)[CPT]) {
    const T* src = B + (int64_t)rm.row(ci) * ld + col0;
    if (vec_ok) {
      const VT v = *reinterpret_cast<const VT*>(src);
      __builtin_memcpy(&x[0], &v, sizeof(VT));
    } else {
#pragma unroll
      for (int q = 0; q < CPT; ++q) x[q] = (col0 + q < col_end) ? src[q] : (T)0;
    }
  };

  T acc[NB][CPT];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int q = 0; q < CPT; ++q) acc[i][q] = 0;
  // no LDS staging: each thread reads the V rows it needs (shared by the TPR
  // threads of a row through the caches), so the row loop has no barriers
#pragma unroll 4
  for (int ci = rg; ci < nact; ci += RG) {
    T v[NB], x[CPT];
    vrow(ci, v);
    load_row(ci, x);
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int q = 0; q < CPT; ++q) acc[i][q] += v[i] * x[q];
  }
  // combine the row groups of each wave (lanes tc, tc + TPR, ...), then the waves
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      T v = acc[i][q];
#pragma unroll
      for (int off = TPR; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
      acc[i][q] = v;
    }
  if (lane < TPR) {
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int q = 0; q < CPT; ++q) red[w][i][tc * CPT + q] = acc[i][q];
  }
  __syncthreads();
  if (t < UC) {
    T wv[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) wv[i] = red[0][i][t] + red[1][i][t] + red[2][i][t] + red[3][i][t];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      T sum = 0;
      if (TRANS) {
        // (T^T w)_i = sum_{k <= i} T[k][i] w_k
#pragma unroll
        for (int k = 0; k < NB; ++k)
          if (k <= i) sum += Ts[k * NB + i] * wv[k];
      } else {
        // (T w)_i = sum_{k >= i} T[i][k] w_k
#pragma unroll
        for (int k = 0; k < NB; ++k)
          if (k >= i) sum += Ts[i * NB + k] * wv[k];
      }
      wsh[i][t] = sum;
    }
  }
  __syncthreads();
  T wl[NB][CPT];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int q = 0; q < CPT; ++q) wl[i][q] = wsh[i][tc * CPT + q];
#pragma unroll 4
  for (int ci = rg; ci < nact; ci += RG) {
    T v[NB], x[CPT];
    vrow(ci, v);
    load_row(ci, x);
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int q = 0; q < CPT; ++q) x[q] -= v[i] * wl[i][q];
    T* dst = B + (int64_t)rm.row(ci) * ld + col0;
    if (vec_ok) {
      VT vv;
      __builtin_memcpy(&vv, &x[0], sizeof(VT));
      *reinterpret_cast<VT*>(dst) = vv;
    } else {
#pragma unroll
      for (int q = 0; q < CPT; ++q)
        if (col0 + q < col_end) dst[q] = x[q];
    }
  }
}

// ---------------------------------------------------------------- outer panels
//
// Two-level blocking: inner panels of NB columns (above) are factored and
// applied only inside an outer panel of kOuter = 64 columns; the outer panel's
// reflectors are then combined into one compact-WY factor T_big (64 x 64,
// block_t_kernel, from the inner T's and the Gram matrix V^T V) and applied to
// the trailing columns, or to the block being turned into Q, by
// block_apply_kernel: W = V^T B, W' = T' W, B -= V W', with both products on
// the matrix cores (16x16x4 in float or double). One 256-thread workgroup owns
// 64 columns of B of one matrix; its 4 waves split the rows.
constexpr int kOuter = 64;
constexpr int kBlkThreads = 256;
// The Gram matrix V^T V of an outer panel of a few tall blocks is summed by
// up to kGramSplits workgroups per block over row ranges (partials added in
// order by block_t_kernel); one workgroup per block would leave most CUs idle.
constexpr int kGramSplits = 4;
constexpr int kRowSplits = 4;  // row shares of a narrow trailing update
__host__ __device__ inline int gram_splits(int nbatch, int tree_d) {
  return (tree_d == 0 && nbatch <= 64) ? kGramSplits : 1;
}

template <typename T>
struct BlkMfma;
template <>
struct BlkMfma<float> {
  using Acc = f32x4_t;
  __device__ __forceinline__ static Acc step(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct BlkMfma<double> {
  using Acc = f64x4_t;
  __device__ __forceinline__ static Acc step(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// x[0..3] = src[0..3] for the columns c0 .. c0+3 that are < cend (others 0).
template <typename T>
__device__ __forceinline__ void load4(const T* src, int c0, int cend, bool vec, T (&x)[4]) {
  if (vec && c0 + 4 <= cend) {
    if constexpr (sizeof(T) == 4) {
      const float4 v = *reinterpret_cast<const float4*>(src);
      x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
    } else {
      const double2 u = *reinterpret_cast<const double2*>(src);
      const double2 v = *reinterpret_cast<const double2*>(src + 2);
      x[0] = u.x; x[1] = u.y; x[2] = v.x; x[3] = v.y;
    }
  } else {
#pragma unroll
    for (int t = 0; t < 4; ++t) x[t] = (c0 + t < cend) ? src[t] : (T)0;
  }
}

// MODE 0: B <- (I - V T^T V^T) B   (factorisation, Q^T B)
// MODE 1: B <- (I - V T V^T) B     (Q formation, Q B)
// MODE 2: gout = V^T V             (Gram matrix of the outer panel)
// V = columns [P0, P0 + W) of Vmat with unit diagonal and zeros above, over the
// rows of the outer panel's row map; B columns [col_begin, col_end).
// MODE 0/1 over row shares (phase 1 and 2, rsplit shares per column block,
// gridDim.x = column blocks x rsplit): phase 1 writes the share's partial
// V^T B to wpart, phase 2 applies the summed W to the share's rows.
template <typename T, int MODE>
__global__ __launch_bounds__(kBlkThreads) __attribute__((amdgpu_waves_per_eu(1, 2))) void block_apply_kernel(const T* Vmat, int64_t vstride, T* Bmat,
                                                                  int64_t bstride, int m_full, int m_last,
                                                                  int nbatch, int ld, int P0, int W, int tree_d,
                                                                  int col_begin, int col_end,
                                                                  const T* __restrict__ tbig, T* __restrict__ gout,
                                                                  int phase, int rsplit, T* __restrict__ wpart) {
  using M = BlkMfma<T>;
  using Acc = typename M::Acc;
  __shared__ T Ws[kOuter][kOuter + 1];
  __shared__ T Ts[kOuter][kOuter + 1];

  int cbx, b;
  xcd_block(cbx, b);
  const int m = (b == nbatch - 1) ? m_last : m_full;
  const T* V = Vmat + (int64_t)b * vstride;
  T* B = Bmat + (int64_t)b * bstride;
  const RowMap rm = make_rowmap<kOuter>(m, P0, tree_d);
  const int nact = rm.nact;
  const int t = threadIdx.x;
  const int w = t >> 6;
  const int lane = t & 63;
  const int l15 = lane & 15;
  const int lg = lane >> 4;
  const bool shared_rows = MODE != 2 && phase != 0;
  const int ncb_real = shared_rows ? (int)gridDim.x / rsplit : (int)gridDim.x;
  const int cbk = shared_rows ? cbx % ncb_real : cbx;
  const int cb0 = (MODE == 2) ? P0 : col_begin + cbk * kOuter;
  const int cend = (MODE == 2) ? P0 + W : col_end;
  const bool vec_ld = ((int64_t)ld * sizeof(T)) % 16 == 0;
  const bool vec_v = vec_ld && (reinterpret_cast<uintptr_t>(V) % 16 == 0) && (P0 % 4 == 0);
  const bool vec_b = vec_ld && (reinterpret_cast<uintptr_t>(B) % 16 == 0) && (cb0 % 4 == 0);

  // 4 consecutive panel columns 4q .. 4q+3 of compact row ci, masked to the
  // unit lower trapezoid (zero for ci >= nact)
  auto vrow4 = [&](int ci, int q, T (&x)[4]) {
    if (ci >= nact) {
#pragma unroll
      for (int e = 0; e < 4; ++e) x[e] = 0;
      return;
    }
    load4<T>(V + (int64_t)rm.row(ci) * ld + P0 + 4 * q, P0 + 4 * q, P0 + W, vec_v, x);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = 4 * q + e;
      x[e] = (ci > i) ? x[e] : (ci == i ? (T)1 : (T)0);
    }
  };

  // Interior rows (compact index >= kOuter, below every reflector's unit
  // diagonal, and < nact) of a full-width block take unmasked 16-byte loads;
  // the first kOuter rows and the ragged end take the masked path.
  const bool fast = vec_v && vec_b && (W == kOuter) && (cb0 + kOuter <= cend);
  const int nint = nact & ~15;  // rows [kOuter, nint) are interior
  auto vrow4_fast = [&](int ci, int q, T (&x)[4]) {
    const T* src = V + (int64_t)rm.row(ci) * ld + P0 + 4 * q;
    if constexpr (sizeof(T) == 4) {
      const float4 v = *reinterpret_cast<const float4*>(src);
      x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
    } else {
      const double2 u = *reinterpret_cast<const double2*>(src);
      const double2 v = *reinterpret_cast<const double2*>(src + 2);
      x[0] = u.x; x[1] = u.y; x[2] = v.x; x[3] = v.y;
    }
  };
  auto brow4_fast = [&](int ci, int q, T (&x)[4]) {
    const T* src = B + (int64_t)rm.row(ci) * ld + cb0 + 4 * q;
    if constexpr (sizeof(T) == 4) {
      const float4 v = *reinterpret_cast<const float4*>(src);
      x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
    } else {
      const double2 u = *reinterpret_cast<const double2*>(src);
      const double2 v = *reinterpret_cast<const double2*>(src + 2);
      x[0] = u.x; x[1] = u.y; x[2] = v.x; x[3] = v.y;
    }
  };

  // Row shares (Gram mode, or phase 1/2): share split of nsplit takes the
  // head rows (if first), interior rows [ilo, ihi) in 64-row units, and the
  // tail (if last); a panel off the fast path is done by the first alone.
  const int nsplit = (MODE == 2) ? (int)gridDim.x : (shared_rows ? rsplit : 1);
  const int split = (MODE == 2) ? cbx : (shared_rows ? cbx / ncb_real : 0);
  int ilo = kOuter, ihi = nint;
  if (nsplit > 1) {
    const int span = nint > kOuter ? nint - kOuter : 0;
    const int per = ((span + 63) / 64 + nsplit - 1) / nsplit;
    ilo = kOuter + min(split * per * 64, span);
    ihi = kOuter + min((split + 1) * per * 64, span);
  }
  T* wshare = shared_rows ? wpart + (((int64_t)split * ncb_real + cbk) * nbatch + b) * kOuter * kOuter : nullptr;

  if (MODE != 2 && phase == 2) {
    // the summed W of every share of this column block
    for (int e = t; e < kOuter * kOuter; e += kBlkThreads) {
      T sum = 0;
      for (int q = 0; q < nsplit; ++q) sum += wpart[(((int64_t)q * ncb_real + cbk) * nbatch + b) * kOuter * kOuter + e];
      Ws[e / kOuter][e % kOuter] = sum;
    }
    __syncthreads();
  } else {
  // ---- pass 1: W = V^T B (tile (ti, tj) entry (r, c) is W[4r + ti][4c + tj])
  Acc acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[a][c][e] = 0;
  auto quad_masked = [&](int r0) {
    const int ci = r0 + lg;
    T va[4], vb[4];
    vrow4(ci, l15, va);
    if (MODE == 2) {
#pragma unroll
      for (int e = 0; e < 4; ++e) vb[e] = va[e];
    } else if (ci < nact) {
      load4<T>(B + (int64_t)rm.row(ci) * ld + cb0 + 4 * l15, cb0 + 4 * l15, cend, vec_b, vb);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) vb[e] = 0;
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[a][c] = M::step(va[a], vb[c], acc[a][c]);
  };
  int r0 = 4 * w;
  const int head_end = fast ? kOuter : nact;
  if (split == 0)
    for (; r0 < head_end && r0 < nact; r0 += 16) quad_masked(r0);
  if (fast) {
    if (nsplit > 1) r0 = ilo + 4 * w;
    // four row quads per trip; the next trip's loads are issued before this
    // trip's products (two register sets, trips in pairs). Rows of a trip past
    // the interior are clamped to the last interior quad and multiply nothing.
    // trip k reads rows r0 + 64 k .. r0 + 64 k + 51, all below ihi
    const int ntrip = (ihi - r0 >= 52) ? (ihi - r0 - 52) / 64 + 1 : 0;
    auto load_trip = [&](int k, T (&va)[4][4], T (&vb)[4][4]) {
      const int rb = r0 + 64 * (k < ntrip ? k : ntrip - 1);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        vrow4_fast(rb + 16 * u + lg, l15, va[u]);
        if (MODE != 2) brow4_fast(rb + 16 * u + lg, l15, vb[u]);
      }
    };
    auto mma_trip = [&](const T (&va)[4][4], const T (&vb)[4][4]) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[a][c] = M::step(va[u][a], MODE == 2 ? va[u][c] : vb[u][c], acc[a][c]);
    };
    if (ntrip > 0) {
      T va0[4][4], vb0[4][4], va1[4][4], vb1[4][4];
      load_trip(0, va0, vb0);
      int k = 0;
      for (; k + 1 < ntrip; k += 2) {
        load_trip(k + 1, va1, vb1);
        mma_trip(va0, vb0);
        load_trip(k + 2, va0, vb0);
        mma_trip(va1, vb1);
      }
      if (k < ntrip) mma_trip(va0, vb0);
      r0 += 64 * ntrip;
    }
    for (; r0 < ihi; r0 += 16) quad_masked(r0);
    if (split == nsplit - 1)
      for (; r0 < nact; r0 += 16) quad_masked(r0);
  }
  // combine the 4 waves' partial sums in LDS, one wave after the other
  for (int ww = 0; ww < 4; ++ww) {
    if (w == ww) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int i = 4 * acc_row<Acc>(lg, e) + a;
            const int j = 4 * l15 + c;
            Ws[i][j] = (ww == 0) ? acc[a][c][e] : Ws[i][j] + acc[a][c][e];
          }
    }
    __syncthreads();
  }
  if (MODE == 2) {
    T* g = gout + ((int64_t)split * nbatch + b) * kOuter * kOuter;
    for (int e = t; e < kOuter * kOuter; e += kBlkThreads) g[e] = Ws[e / kOuter][e % kOuter];
    return;
  }
  if (phase == 1) {
    for (int e = t; e < kOuter * kOuter; e += kBlkThreads) wshare[e] = Ws[e / kOuter][e % kOuter];
    return;
  }
  }  // pass 1

  // ---- W' = T' W (T' = T^T for MODE 0, T for MODE 1); T is upper triangular
  const T* tb = tbig + (int64_t)b * kOuter * kOuter;
  for (int e = t; e < kOuter * kOuter; e += kBlkThreads) Ts[e / kOuter][e % kOuter] = tb[e];
  __syncthreads();
  T wp[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = t + q * kBlkThreads;
    const int i = e / kOuter, j = e % kOuter;
    T sum = 0;
    if (MODE == 0) {
      for (int k = 0; k <= i; ++k) sum += Ts[k][i] * Ws[k][j];
    } else {
      for (int k = i; k < kOuter; ++k) sum += Ts[i][k] * Ws[k][j];
    }
    wp[q] = sum;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = t + q * kBlkThreads;
    Ws[e / kOuter][e % kOuter] = wp[q];
  }
  __syncthreads();

  // ---- pass 2: B -= V W'. Step (q, u) uses panel columns k = 16q + 4lg + u;
  // output tile tc covers B columns cb0 + 16 tc .. + 15.
  T wb[4][4][4];  // [q][u][tc] = W'[16q + 4lg + u][16 tc + l15]
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int tc = 0; tc < 4; ++tc) wb[q][u][tc] = Ws[16 * q + 4 * lg + u][16 * tc + l15];
  auto chunk = [&](int c0, auto fast_tag) {
    constexpr bool FAST = decltype(fast_tag)::value;
    T va[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      T x[4];
      if constexpr (FAST) {
        vrow4_fast(c0 + l15, 4 * q + lg, x);
      } else {
        vrow4(c0 + l15, 4 * q + lg, x);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) va[q][u] = x[u];
    }
    // the B entries this lane updates, requested before the products
    T bold[4][4];
    if constexpr (FAST) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const T* src = B + (int64_t)rm.row(c0 + acc_row<Acc>(lg, e)) * ld + cb0 + l15;
#pragma unroll
        for (int tc = 0; tc < 4; ++tc) bold[e][tc] = src[16 * tc];
      }
    }
    Acc out[4];
#pragma unroll
    for (int tc = 0; tc < 4; ++tc)
#pragma unroll
      for (int e = 0; e < 4; ++e) out[tc][e] = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int tc = 0; tc < 4; ++tc) out[tc] = M::step(va[q][u], wb[q][u][tc], out[tc]);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int ci = c0 + acc_row<Acc>(lg, e);
      if (FAST) {
        T* dst = B + (int64_t)rm.row(ci) * ld + cb0 + l15;
#pragma unroll
        for (int tc = 0; tc < 4; ++tc) dst[16 * tc] = bold[e][tc] - out[tc][e];
      } else if (ci < nact) {
        T* dst = B + (int64_t)rm.row(ci) * ld + cb0 + l15;
#pragma unroll
        for (int tc = 0; tc < 4; ++tc)
          if (cb0 + 16 * tc + l15 < cend) dst[16 * tc] -= out[tc][e];
      }
    }
  };
  int c0 = 16 * w;
  if (split == 0)
    for (; c0 < (fast ? kOuter : nact) && c0 < nact; c0 += 64) chunk(c0, std::false_type{});
  if (fast) {
    if (nsplit > 1) c0 = ilo + 16 * w;
    // interior chunks: the next chunk's V rows and B entries are loaded before
    // this chunk's products (two register sets, chunks in pairs; the load past
    // the last chunk re-reads it and is unused)
    const int nch = (ihi - c0 >= 16) ? (ihi - c0 - 16) / 64 + 1 : 0;
    auto load_chunk = [&](int k, T (&va)[4][4], T (&bo)[4][4]) {
      const int cc = c0 + 64 * (k < nch ? k : nch - 1);
#pragma unroll
      for (int q = 0; q < 4; ++q) vrow4_fast(cc + l15, 4 * q + lg, va[q]);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const T* src = B + (int64_t)rm.row(cc + acc_row<Acc>(lg, e)) * ld + cb0 + l15;
#pragma unroll
        for (int tc = 0; tc < 4; ++tc) bo[e][tc] = src[16 * tc];
      }
    };
    auto run_chunk = [&](int k, const T (&va)[4][4], const T (&bo)[4][4]) {
      const int cc = c0 + 64 * k;
      Acc out[4];
#pragma unroll
      for (int tc = 0; tc < 4; ++tc)
#pragma unroll
        for (int e = 0; e < 4; ++e) out[tc][e] = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int tc = 0; tc < 4; ++tc) out[tc] = M::step(va[q][u], wb[q][u][tc], out[tc]);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        T* dst = B + (int64_t)rm.row(cc + acc_row<Acc>(lg, e)) * ld + cb0 + l15;
#pragma unroll
        for (int tc = 0; tc < 4; ++tc) dst[16 * tc] = bo[e][tc] - out[tc][e];
      }
    };
    if (nch > 0) {
      T va0[4][4], bo0[4][4], va1[4][4], bo1[4][4];
      load_chunk(0, va0, bo0);
      int k = 0;
      for (; k + 1 < nch; k += 2) {
        load_chunk(k + 1, va1, bo1);
        run_chunk(k, va0, bo0);
        load_chunk(k + 2, va0, bo0);
        run_chunk(k + 1, va1, bo1);
      }
      if (k < nch) run_chunk(k, va0, bo0);
      c0 += 64 * nch;
    }
    for (; c0 < ihi; c0 += 64) chunk(c0, std::false_type{});
    if (split == nsplit - 1)
      for (; c0 < nact; c0 += 64) chunk(c0, std::false_type{});
  }
}

// T_big (kOuter x kOuter, upper triangular) of the outer panel [P0, P0 + W)
// from the inner factors T_k (nb x nb, at tm + (P0/nb + k) nb^2) and the Gram
// matrix G = V^T V: merging block k into the leading blocks 0..k-1 sets
//   T_big[0:k nb, k nb : k nb + nb] = -T_big[0:k nb, 0:k nb] G[0:k nb, k-th block] T_k.
// Entries outside the W x W block are zero.
template <typename T>
__global__ __launch_bounds__(kBlkThreads) void block_t_kernel(const T* __restrict__ tm, int64_t t_bstride, int nb,
                                                              int P0, int W, const T* __restrict__ gram,
                                                              int nsplit, int nbatch, T* __restrict__ tbig) {
  __shared__ T Tb[kOuter][kOuter + 1];
  __shared__ T G[kOuter][kOuter + 1];
  __shared__ T X[kOuter][kOuter + 1];
  const int b = blockIdx.x;
  const int t = threadIdx.x;
  for (int e = t; e < kOuter * kOuter; e += kBlkThreads) {
    const int i = e / kOuter, j = e % kOuter;
    T gs = gram[(int64_t)b * kOuter * kOuter + e];
    for (int q = 1; q < nsplit; ++q) gs += gram[((int64_t)q * nbatch + b) * kOuter * kOuter + e];
    G[i][j] = gs;
    T v = 0;
    if (i < W && j < W && i / nb == j / nb && i <= j) {
      const int k = i / nb;
      v = tm[(int64_t)b * t_bstride + (int64_t)(P0 / nb + k) * nb * nb + (i - k * nb) * nb + (j - k * nb)];
    }
    Tb[i][j] = v;
  }
  __syncthreads();
  const int K = (W + nb - 1) / nb;
  for (int k = 1; k < K; ++k) {
    const int r = k * nb;                // rows of the leading part
    const int nbk = min(nb, W - r);      // width of block k
    // X = Tb[0:r, 0:r] G[0:r, r:r+nbk]
    for (int e = t; e < r * nbk; e += kBlkThreads) {
      const int i = e / nbk, j = e % nbk;
      T sum = 0;
      for (int q = i; q < r; ++q) sum += Tb[i][q] * G[q][r + j];
      X[i][j] = sum;
    }
    __syncthreads();
    // Tb[0:r, r:r+nbk] = -X T_k
    for (int e = t; e < r * nbk; e += kBlkThreads) {
      const int i = e / nbk, j = e % nbk;
      T sum = 0;
      for (int q = 0; q <= j; ++q) sum += X[i][q] * Tb[r + q][r + j];
      Tb[i][r + j] = -sum;
    }
    __syncthreads();
  }
  T* out = tbig + (int64_t)b * kOuter * kOuter;
  for (int e = t; e < kOuter * kOuter; e += kBlkThreads) out[e] = Tb[e / kOuter][e % kOuter];
}

// Rdst[b] = upper triangle of the top d x d block of src[b] (as double, zeros below).
template <typename T>
__global__ void extract_r_kernel(const T* __restrict__ src, int64_t sstride, int ld, int d,
                                 double* __restrict__ dst, int nbatch) {
  const int b = blockIdx.y;
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)d * d) return;
  const int i = (int)(idx / d), j = (int)(idx % d);
  dst[(int64_t)b * d * d + idx] = (j >= i) ? (double)src[(int64_t)b * sstride + (int64_t)i * ld + j] : 0.0;
}

// Bdst[b] (rows x d, ld d) = [M[b] (d x d, double); 0].
template <typename T>
__global__ void init_qblock_kernel(const double* __restrict__ M, T* __restrict__ dst, int64_t dstride, int m_full,
                                   int m_last, int nbatch, int d) {
  const int b = blockIdx.y;
  const int m = (b == nbatch - 1) ? m_last : m_full;
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * d) return;
  const int i = (int)(idx / d);
  dst[(int64_t)b * dstride + idx] = (i < d) ? (T)M[(int64_t)b * d * d + idx] : (T)0;
}

// Final R with diag >= 0 and the root block M = diag(sign).
__global__ void finalize_r_kernel(const double* __restrict__ Rroot, double* __restrict__ R,
                                  double* __restrict__ Mroot, int d) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)d * d) return;
  const int i = (int)(idx / d), j = (int)(idx % d);
  const double sg = Rroot[(int64_t)i * d + i] < 0.0 ? -1.0 : 1.0;
  R[idx] = (j >= i) ? sg * Rroot[idx] : 0.0;
  const double sj = Rroot[(int64_t)j * d + j] < 0.0 ? -1.0 : 1.0;
  Mroot[idx] = (i == j) ? sj : 0.0;
}

template <typename T>
__global__ void copy_kernel(const T* __restrict__ src, T* __restrict__ dst, int64_t count) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx < count) dst[idx] = src[idx];
}

// ------------------------------------------------------------------ host side

// Panels are factored by kFactorThreads threads holding RPT rows each.
constexpr int kFactorThreads = 512;

static int pick_rpt(int m) {
  int r = 1;
  while (r * kFactorThreads < m) r *= 2;
  return r;
}

// Panel width: keep the register panel at <= 64 32-bit words per thread, so
// panel, reduction vector and temporaries fit the 256 VGPRs a 512-thread
// workgroup allows without spilling.
template <typename T>
static int pick_nb(int rpt) {
  const int words = rpt * (int)(sizeof(T) / 4);
  if (words <= 4) return 16;
  if (words <= 8) return 8;
  return 4;
}

struct QrShape {
  int m_full, m_last, nbatch, d, nb, npanels, tree_d;
};

// tree = true: every matrix is a stacked pair of d x d upper triangles.
template <typename T>
static QrShape qr_shape(int m_full, int m_last, int nbatch, int d, bool tree = false) {
  QrShape s;
  s.m_full = m_full;
  s.m_last = m_last;
  s.nbatch = nbatch;
  s.d = d;
  s.tree_d = tree ? d : 0;
  s.nb = pick_nb<T>(pick_rpt(m_full > m_last ? m_full : m_last));
  s.npanels = (d + s.nb - 1) / s.nb;
  return s;
}

template <typename T, int RPT, int NB>
static hipError_t launch_panel_factor_rn(hipStream_t st, T* A, int64_t bstride, const QrShape& s, int p0, int nbw,
                                         T* tau, T* tm) {
  hipLaunchKernelGGL((panel_factor_kernel<T, RPT, NB, kFactorThreads>), dim3(s.nbatch), dim3(kFactorThreads), 0, st,
                     A, bstride, s.m_full, s.m_last, s.nbatch, s.d, p0, nbw, s.tree_d, tau, (int64_t)s.d, tm,
                     (int64_t)s.npanels * NB * NB);
  return hipGetLastError();
}

template <typename T, int NB, int TPB>
static hipError_t launch_panel_factor_small(hipStream_t st, T* A, int64_t bstride, const QrShape& s, int p0, int nbw,
                                            T* tau, T* tm) {
  hipLaunchKernelGGL((panel_factor_kernel<T, 1, NB, TPB>), dim3(s.nbatch), dim3(TPB), 0, st, A, bstride, s.m_full,
                     s.m_last, s.nbatch, s.d, p0, nbw, s.tree_d, tau, (int64_t)s.d, tm, (int64_t)s.npanels * NB * NB);
  return hipGetLastError();
}

template <typename T, int NB>
static hipError_t launch_panel_factor_nb(hipStream_t st, int rpt, T* A, int64_t bstride, const QrShape& s, int p0,
                                         int nbw, T* tau, T* tm) {
  // Tree panels touch NB top rows and p0 + NB bottom rows (see RowMap): the
  // smallest workgroup holding one of them per thread does the panel, so the
  // early panels pay for fewer waves at every barrier.
  if constexpr (std::is_same<T, double>::value) {
    if (s.tree_d > 0) {
      const int nact = (NB < s.tree_d - p0 ? NB : s.tree_d - p0) + (p0 + NB < s.tree_d ? p0 + NB : s.tree_d);
      if (nact <= 64) return launch_panel_factor_small<T, NB, 64>(st, A, bstride, s, p0, nbw, tau, tm);
      if (nact <= 128) return launch_panel_factor_small<T, NB, 128>(st, A, bstride, s, p0, nbw, tau, tm);
      if (nact <= 256) return launch_panel_factor_small<T, NB, 256>(st, A, bstride, s, p0, nbw, tau, tm);
      if (nact <= kFactorThreads) rpt = 1;
    }
  }
  switch (rpt) {
    case 1: return launch_panel_factor_rn<T, 1, NB>(st, A, bstride, s, p0, nbw, tau, tm);
    case 2: return launch_panel_factor_rn<T, 2, NB>(st, A, bstride, s, p0, nbw, tau, tm);
    case 4: return launch_panel_factor_rn<T, 4, NB>(st, A, bstride, s, p0, nbw, tau, tm);
    case 8: return launch_panel_factor_rn<T, 8, NB>(st, A, bstride, s, p0, nbw, tau, tm);
    default: return launch_panel_factor_rn<T, 16, NB>(st, A, bstride, s, p0, nbw, tau, tm);
  }
}

// Narrow updates (at most 64 columns, the inner panels inside an outer panel)
// take 16-column workgroups, so a batch of a few matrices still fills the chip;
// float updates that would get at most one 16-column workgroup per CU take
// 8-column ones (C3 leaves: TSQR 27.7 -> 27.0 ms; 4 columns measured 27.6).
template <typename T, int NB, bool TRANS>
static hipError_t launch_apply_nb(hipStream_t st, const T* V, int64_t vstride, T* B, int64_t bstride,
                                  const QrShape& s, int p0, int nbw, int c0, int c1, const T* tm) {
  if (c1 <= c0) return hipSuccess;
  const int64_t tbs = (int64_t)s.npanels * NB * NB;
  if constexpr (sizeof(T) == 4 && TRANS) {
    if (c1 - c0 <= 64 && s.nbatch * ((c1 - c0 + 15) / 16) <= 256) {
      // few workgroups at 16 columns (one per CU or fewer): narrower
      // workgroups put more row streams in flight
      const int ncb = (c1 - c0 + kNarrowCols - 1) / kNarrowCols;
      hipLaunchKernelGGL((panel_apply_kernel<T, NB, TRANS, kNarrowCols>), dim3(ncb, s.nbatch), dim3(kUpdThreads), 0,
                         st, V, vstride, B, bstride, s.m_full, s.m_last, s.nbatch, s.d, p0, nbw, s.tree_d, c0, c1, tm,
                         tbs);
      return hipGetLastError();
    }
  }
  if (c1 - c0 <= 64) {
    const int ncb = (c1 - c0 + 15) / 16;
    hipLaunchKernelGGL((panel_apply_kernel<T, NB, TRANS, 16>), dim3(ncb, s.nbatch), dim3(kUpdThreads), 0, st, V,
                       vstride, B, bstride, s.m_full, s.m_last, s.nbatch, s.d, p0, nbw, s.tree_d, c0, c1, tm, tbs);
  } else {
    const int ncb = (c1 - c0 + kUpdCols - 1) / kUpdCols;
    hipLaunchKernelGGL((panel_apply_kernel<T, NB, TRANS, kUpdCols>), dim3(ncb, s.nbatch), dim3(kUpdThreads), 0, st,
                       V, vstride, B, bstride, s.m_full, s.m_last, s.nbatch, s.d, p0, nbw, s.tree_d, c0, c1, tm, tbs);
  }
  return hipGetLastError();
}

template <typename T, bool TRANS>
static hipError_t launch_apply(hipStream_t st, int nb, const T* V, int64_t vstride, T* B, int64_t bstride,
                               const QrShape& s, int p0, int nbw, int c0, int c1, const T* tm) {
  if (nb == 16) return launch_apply_nb<T, 16, TRANS>(st, V, vstride, B, bstride, s, p0, nbw, c0, c1, tm);
  if (nb == 8) return launch_apply_nb<T, 8, TRANS>(st, V, vstride, B, bstride, s, p0, nbw, c0, c1, tm);
  return launch_apply_nb<T, 4, TRANS>(st, V, vstride, B, bstride, s, p0, nbw, c0, c1, tm);
}

#define LR_TRY(x)                          \
  do {                                     \
    hipError_t e__ = (x);                  \
    if (e__ != hipSuccess) return e__;     \
  } while (0)

template <typename T, int MODE>
static hipError_t launch_block_apply(hipStream_t st, const T* V, int64_t vstride, T* B, int64_t bstride,
                                     const QrShape& s, int P0, int W, int c0, int c1, const T* tbig, T* gout,
                                     int phase = 0, int rsplit = 1, T* wpart = nullptr) {
  int ncb = (MODE == 2) ? gram_splits(s.nbatch, s.tree_d) : (c1 - c0 + kOuter - 1) / kOuter;
  if (ncb <= 0) return hipSuccess;
  if (MODE != 2 && phase != 0) ncb *= rsplit;
  hipLaunchKernelGGL((block_apply_kernel<T, MODE>), dim3(ncb, s.nbatch), dim3(kBlkThreads), 0, st, V, vstride, B,
                     bstride, s.m_full, s.m_last, s.nbatch, s.d, P0, W, s.tree_d, c0, c1, tbig, gout, phase, rsplit,
                     wpart);
  return hipGetLastError();
}

// Number of outer panels and the T_big / Gram storage they need per matrix.
static int n_outer(int d) { return (d + kOuter - 1) / kOuter; }

// Batched Householder QR in place: A[b] (m_b x d, ld d) -> R (upper) + V (below).
// Inner panels are factored and applied inside each outer panel; the outer
// panel's T_big (kept in tbig for the Q formation) then updates the trailing
// columns in one pass.
//
// With wpart (kRowSplits x 256 W blocks), a trailing update of so few column
// blocks that they would leave CUs idle runs over kRowSplits row shares: one
// launch for the shares' partial W = V^T B, one for the update with their sum.
template <typename T>
static hipError_t batched_qr(hipStream_t st, T* A, int64_t bstride, const QrShape& s, T* tau, T* tm, T* tbig,
                             T* gram, T* wpart = nullptr) {
  const int rpt = pick_rpt(s.m_full > s.m_last ? s.m_full : s.m_last);
  const int64_t t_bstride = (int64_t)s.npanels * s.nb * s.nb;
  for (int o = 0; o < n_outer(s.d); ++o) {
    const int P0 = o * kOuter;
    const int W = (s.d - P0) < kOuter ? (s.d - P0) : kOuter;
    for (int p0 = P0; p0 < P0 + W; p0 += s.nb) {
      const int nbw = (s.d - p0) < s.nb ? (s.d - p0) : s.nb;
      T* tmp = tm + (int64_t)(p0 / s.nb) * s.nb * s.nb;
      if (s.nb == 16) {
        LR_TRY((launch_panel_factor_nb<T, 16>(st, rpt, A, bstride, s, p0, nbw, tau, tmp)));
      } else if (s.nb == 8) {
        LR_TRY((launch_panel_factor_nb<T, 8>(st, rpt, A, bstride, s, p0, nbw, tau, tmp)));
      } else {
        LR_TRY((launch_panel_factor_nb<T, 4>(st, rpt, A, bstride, s, p0, nbw, tau, tmp)));
      }
      LR_TRY((launch_apply<T, true>(st, s.nb, A, bstride, A, bstride, s, p0, nbw, p0 + nbw, P0 + W, tmp)));
    }
    T* tb = tbig + (int64_t)o * s.nbatch * kOuter * kOuter;
    LR_TRY((launch_block_apply<T, 2>(st, A, bstride, A, bstride, s, P0, W, 0, 0, nullptr, gram)));
    hipLaunchKernelGGL(block_t_kernel<T>, dim3(s.nbatch), dim3(kBlkThreads), 0, st, tm, t_bstride, s.nb, P0, W, gram,
                       gram_splits(s.nbatch, s.tree_d), s.nbatch, tb);
    LR_TRY(hipGetLastError());
    const int ncb = (s.d - (P0 + W) + kOuter - 1) / kOuter;
    if (wpart != nullptr && s.tree_d == 0 && ncb > 0 && ncb * s.nbatch <= 256) {
      LR_TRY((launch_block_apply<T, 0>(st, A, bstride, A, bstride, s, P0, W, P0 + W, s.d, tb, nullptr, 1, kRowSplits,
                                       wpart)));
      LR_TRY((launch_block_apply<T, 0>(st, A, bstride, A, bstride, s, P0, W, P0 + W, s.d, tb, nullptr, 2, kRowSplits,
                                       wpart)));
    } else {
      LR_TRY((launch_block_apply<T, 0>(st, A, bstride, A, bstride, s, P0, W, P0 + W, s.d, tb, nullptr)));
    }
  }
  return hipSuccess;
}

// B[b] <- Q[b] B[b] with Q[b] from batched_qr (outer panels last to first).
template <typename T>
static hipError_t batched_apply_q(hipStream_t st, const T* V, int64_t vstride, T* B, int64_t bstride,
                                  const QrShape& s, const T* tbig) {
  for (int o = n_outer(s.d) - 1; o >= 0; --o) {
    const int P0 = o * kOuter;
    const int W = (s.d - P0) < kOuter ? (s.d - P0) : kOuter;
    LR_TRY((launch_block_apply<T, 1>(st, V, vstride, B, bstride, s, P0, W, 0, s.d,
                                     tbig + (int64_t)o * s.nbatch * kOuter * kOuter, nullptr)));
  }
  return hipSuccess;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

template <typename T>
static hipError_t launch_copy(hipStream_t st, const T* src, T* dst, int64_t count) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy_kernel<T>, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, src, dst, count);
  return hipGetLastError();
}

// The binary tree over b R factors (Eq. 2-3) and the push of the d x d blocks
// back down it (Eq. 4): workspace offsets per level.
struct TreePlan {
  std::vector<int> count;  // R factors per level (level 0 = the tree's leaves)
  std::vector<int> pairs;  // nodes per tree level
  std::vector<size_t> off_r, off_m, off_node, off_ntau, off_nt, off_ntbig, off_ngram;
  size_t end;
};

static TreePlan make_tree_plan(int nleaf, int d, size_t off) {
  TreePlan p;
  int c = nleaf;
  p.count.push_back(c);
  while (c > 1) {
    p.pairs.push_back(c / 2);
    c = (c + 1) / 2;
    p.count.push_back(c);
  }
  const size_t dd = (size_t)d * d * sizeof(double);
  const size_t blk = (size_t)kOuter * kOuter;
  for (size_t l = 0; l < p.count.size(); ++l) {
    p.off_r.push_back(off);
    off = align256(off + (size_t)p.count[l] * dd);
    p.off_m.push_back(off);
    off = align256(off + (size_t)p.count[l] * dd);
  }
  for (size_t l = 0; l < p.pairs.size(); ++l) {
    QrShape ns = qr_shape<double>(2 * d, 2 * d, p.pairs[l], d, true);
    p.off_node.push_back(off);
    off = align256(off + (size_t)p.pairs[l] * 2 * dd);
    p.off_ntau.push_back(off);
    off = align256(off + (size_t)p.pairs[l] * d * sizeof(double));
    p.off_nt.push_back(off);
    off = align256(off + (size_t)p.pairs[l] * ns.npanels * ns.nb * ns.nb * sizeof(double));
    p.off_ntbig.push_back(off);
    off = align256(off + (size_t)n_outer(d) * p.pairs[l] * blk * sizeof(double));
    p.off_ngram.push_back(off);
    off = align256(off + (size_t)p.pairs[l] * blk * sizeof(double));
  }
  p.end = off;
  return p;
}

// Reduces the count[0] R factors at off_r[0] to R (diag >= 0) and, with
// want_q, leaves the d x d block of Q's tree factor for every tree leaf at
// off_m[0].
static hipError_t tree_run(hipStream_t st, const TreePlan& p, int d, char* base, double* R, bool want_q) {
  const int64_t dd = (int64_t)d * d;
  const unsigned ddblocks = (unsigned)((dd + 255) / 256);
  const int levels = (int)p.pairs.size();
  for (int l = 0; l < levels; ++l) {
    const int np = p.pairs[l];
    double* rin = reinterpret_cast<double*>(base + p.off_r[l]);
    double* rout = reinterpret_cast<double*>(base + p.off_r[l + 1]);
    double* node = reinterpret_cast<double*>(base + p.off_node[l]);
    double* ntau = reinterpret_cast<double*>(base + p.off_ntau[l]);
    double* nt = reinterpret_cast<double*>(base + p.off_nt[l]);
    double* ntbig = reinterpret_cast<double*>(base + p.off_ntbig[l]);
    double* ngram = reinterpret_cast<double*>(base + p.off_ngram[l]);
    const QrShape ns = qr_shape<double>(2 * d, 2 * d, np, d, true);
    LR_TRY(launch_copy<double>(st, rin, node, (int64_t)np * 2 * dd));  // pairs are adjacent in rin
    LR_TRY(batched_qr<double>(st, node, 2 * dd, ns, ntau, nt, ntbig, ngram));
    hipLaunchKernelGGL(extract_r_kernel<double>, dim3(ddblocks, np), dim3(256), 0, st, node, 2 * dd, d, d, rout, np);
    LR_TRY(hipGetLastError());
    if (p.count[l] % 2 == 1)
      LR_TRY(launch_copy<double>(st, rin + (int64_t)(p.count[l] - 1) * dd, rout + (int64_t)np * dd, dd));
  }
  // Root: R with diag >= 0, and the root block of Q's tree factor.
  double* rroot = reinterpret_cast<double*>(base + p.off_r[levels]);
  double* mroot = reinterpret_cast<double*>(base + p.off_m[levels]);
  hipLaunchKernelGGL(finalize_r_kernel, dim3(ddblocks), dim3(256), 0, st, rroot, R, mroot, d);
  LR_TRY(hipGetLastError());
  if (!want_q) return hipSuccess;
  // Eq. (4): push the d x d blocks down the tree.
  for (int l = levels - 1; l >= 0; --l) {
    const int np = p.pairs[l];
    double* mup = reinterpret_cast<double*>(base + p.off_m[l + 1]);
    double* mdn = reinterpret_cast<double*>(base + p.off_m[l]);
    double* node = reinterpret_cast<double*>(base + p.off_node[l]);
    double* ntbig = reinterpret_cast<double*>(base + p.off_ntbig[l]);
    const QrShape ns = qr_shape<double>(2 * d, 2 * d, np, d, true);
    // [M_up[k]; 0] into the pair slot (2k, 2k+1) of this level
    const unsigned b2 = (unsigned)((2 * dd + 255) / 256);
    hipLaunchKernelGGL(init_qblock_kernel<double>, dim3(b2, np), dim3(256), 0, st, mup, mdn, 2 * dd, 2 * d, 2 * d,
                       np, d);
    LR_TRY(hipGetLastError());
    LR_TRY(batched_apply_q<double>(st, node, 2 * dd, mdn, 2 * dd, ns, ntbig));
    if (p.count[l] % 2 == 1)
      LR_TRY(launch_copy<double>(st, mup + (int64_t)np * dd, mdn + (int64_t)(p.count[l] - 1) * dd, dd));
  }
  return hipSuccess;
}

struct TsqrPlan {
  int64_t n;
  int d, leaf_rows, nleaf, m_last;
  size_t off_work, off_tau, off_t, off_tbig, off_gram, off_wpart;
  TreePlan tree;
  size_t total;
};

template <typename T>
static TsqrPlan make_plan(int64_t n, int d, int leaf_rows) {
  TsqrPlan p;
  p.n = n;
  p.d = d;
  p.leaf_rows = leaf_rows;
  p.nleaf = (int)((n + leaf_rows - 1) / leaf_rows);
  p.m_last = (int)(n - (int64_t)(p.nleaf - 1) * leaf_rows);
  QrShape ls = qr_shape<T>(leaf_rows, p.m_last, p.nleaf, d);
  size_t off = 0;
  p.off_work = off;
  off = align256(off + (size_t)n * d * sizeof(T));
  p.off_tau = off;
  off = align256(off + (size_t)p.nleaf * d * sizeof(T));
  p.off_t = off;
  off = align256(off + (size_t)p.nleaf * ls.npanels * ls.nb * ls.nb * sizeof(T));
  const size_t blk = (size_t)kOuter * kOuter;
  p.off_tbig = off;
  off = align256(off + (size_t)n_outer(d) * p.nleaf * blk * sizeof(T));
  p.off_gram = off;
  off = align256(off + (size_t)kGramSplits * p.nleaf * blk * sizeof(T));
  p.off_wpart = off;
  off = align256(off + (size_t)kRowSplits * 256 * blk * sizeof(T));
  p.tree = make_tree_plan(p.nleaf, d, off);
  p.total = p.tree.end;
  return p;
}

size_t tsqr_workspace(int64_t n, int d, int leaf_rows, bool f64) {
  return f64 ? make_plan<double>(n, d, leaf_rows).total : make_plan<float>(n, d, leaf_rows).total;
}

template <typename T>
hipError_t tsqr_run(hipStream_t st, int64_t n, int d, int leaf_rows, const T* Y, T* Q, double* R, void* ws) {
  const TsqrPlan p = make_plan<T>(n, d, leaf_rows);
  char* base = static_cast<char*>(ws);
  T* work = reinterpret_cast<T*>(base + p.off_work);
  T* tau = reinterpret_cast<T*>(base + p.off_tau);
  T* tm = reinterpret_cast<T*>(base + p.off_t);
  T* tbig = reinterpret_cast<T*>(base + p.off_tbig);
  T* gram = reinterpret_cast<T*>(base + p.off_gram);
  const QrShape ls = qr_shape<T>(leaf_rows, p.m_last, p.nleaf, d);
  const int64_t lstride = (int64_t)leaf_rows * d;
  const int64_t dd = (int64_t)d * d;
  const unsigned ddblocks = (unsigned)((dd + 255) / 256);

  // Eq. (1): leaf QRs on a working copy of Y.
  LR_TRY(launch_copy<T>(st, Y, work, n * d));
  LR_TRY(batched_qr<T>(st, work, lstride, ls, tau, tm, tbig, gram, reinterpret_cast<T*>(base + p.off_wpart)));
  double* r0 = reinterpret_cast<double*>(base + p.tree.off_r[0]);
  hipLaunchKernelGGL(extract_r_kernel<T>, dim3(ddblocks, p.nleaf), dim3(256), 0, st, work, lstride, d, d, r0,
                     p.nleaf);
  LR_TRY(hipGetLastError());
  // Eq. (2)-(4) over the leaf R factors; without Q only R is wanted
  LR_TRY(tree_run(st, p.tree, d, base, R, Q != nullptr));
  if (Q == nullptr) return hipSuccess;

  // Leaves: Q rows = Q_leaf [M_leaf; 0].
  double* m0 = reinterpret_cast<double*>(base + p.tree.off_m[0]);
  const unsigned lb = (unsigned)(((int64_t)leaf_rows * d + 255) / 256);
  hipLaunchKernelGGL(init_qblock_kernel<T>, dim3(lb, p.nleaf), dim3(256), 0, st, m0, Q, lstride, leaf_rows,
                     p.m_last, p.nleaf, d);
  LR_TRY(hipGetLastError());
  LR_TRY(batched_apply_q<T>(st, work, lstride, Q, lstride, ls, tbig));
  return hipSuccess;
}

// ------------------------------------------------------------------ sequential groups (Eq. 5)
//
// Leaves are taken in groups of g consecutive blocks. Inside a group the QR
// runs in sequence: the first block's QR, then for t = 1 .. g-1 the QR of the
// previous R stacked on block t, [R_{t-1}; K_t] ((d + L) x d), in the working
// precision. Every group runs its step t at once (one batched QR per step), the
// groups' last R factors go through the binary tree of Eq. (2)-(4), and Q is
// pushed back: Q_t [M_t; 0] gives the rows of block t (bottom L rows) and the
// block M_{t-1} for the step before (top d rows). g = 1 is the binary tree
// alone; g = the number of blocks is the fully sequential scheme.

// dst[b] = [upper(top d x d of prev[b]); Y rows of block (b g + t)] ((d + L) x d).
template <typename T>
__global__ void stack_step_kernel(const T* __restrict__ prev, int64_t pstride, const T* __restrict__ Y, int64_t L,
                                  int g, int t, int d, T* __restrict__ dst, int64_t dstride) {
  const int b = blockIdx.y;
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t rows = d + L;
  if (idx >= rows * d) return;
  const int64_t i = idx / d;
  const int j = (int)(idx % d);
  T v;
  if (i < d)
    v = (j >= i) ? prev[(int64_t)b * pstride + i * d + j] : (T)0;
  else
    v = Y[(((int64_t)b * g + t) * L + (i - d)) * d + j];
  dst[(int64_t)b * dstride + idx] = v;
}

// M[b] (double, d x d) = top d x d block of src[b]; rows of block (b g + t) of
// Q = the bottom L rows of src[b].
template <typename T>
__global__ void split_step_kernel(const T* __restrict__ src, int64_t sstride, int64_t L, int g, int t, int d,
                                  double* __restrict__ M, T* __restrict__ Q) {
  const int b = blockIdx.y;
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (d + L) * d) return;
  const int64_t i = idx / d;
  const int j = (int)(idx % d);
  const T v = src[(int64_t)b * sstride + idx];
  if (i < d)
    M[(int64_t)b * d * d + idx] = (double)v;
  else
    Q[(((int64_t)b * g + t) * L + (i - d)) * d + j] = v;
}

struct DominoPlan {
  int d, L, nleaf, g, groups;
  size_t off_work, off_tau, off_t, off_tbig0, off_gram, off_mstep, off_qb;
  std::vector<size_t> off_step, off_stbig;  // steps t = 1 .. g-1
  TreePlan tree;
  size_t total;
};

template <typename T>
static DominoPlan make_domino_plan(int64_t n, int d, int L, int g) {
  DominoPlan p;
  p.d = d;
  p.L = L;
  p.nleaf = (int)(n / L);
  p.g = g;
  p.groups = p.nleaf / g;
  const QrShape s0 = qr_shape<T>(L, L, p.groups, d);
  const QrShape s1 = qr_shape<T>(d + L, d + L, p.groups, d);
  const int tsz = s0.npanels * s0.nb * s0.nb > s1.npanels * s1.nb * s1.nb ? s0.npanels * s0.nb * s0.nb
                                                                          : s1.npanels * s1.nb * s1.nb;
  const size_t blk = (size_t)kOuter * kOuter;
  const size_t tbig_bytes = (size_t)n_outer(d) * p.groups * blk * sizeof(T);
  size_t off = 0;
  p.off_work = off;
  off = align256(off + (size_t)n * d * sizeof(T));
  p.off_tau = off;
  off = align256(off + (size_t)p.groups * d * sizeof(T));
  p.off_t = off;
  off = align256(off + (size_t)p.groups * tsz * sizeof(T));
  p.off_gram = off;
  off = align256(off + (size_t)kGramSplits * p.groups * blk * sizeof(T));
  p.off_tbig0 = off;
  off = align256(off + tbig_bytes);
  for (int t = 1; t < g; ++t) {
    p.off_step.push_back(off);
    off = align256(off + (size_t)p.groups * (d + L) * d * sizeof(T));
    p.off_stbig.push_back(off);
    off = align256(off + tbig_bytes);
  }
  p.off_mstep = off;
  off = align256(off + (size_t)p.groups * d * d * sizeof(double));
  p.off_qb = off;
  off = align256(off + (size_t)p.groups * (d + L) * d * sizeof(T));
  p.tree = make_tree_plan(p.groups, d, off);
  p.total = p.tree.end;
  return p;
}

size_t tsqr_domino_workspace(int64_t n, int d, int leaf_rows, int group, bool f64) {
  return f64 ? make_domino_plan<double>(n, d, leaf_rows, group).total
             : make_domino_plan<float>(n, d, leaf_rows, group).total;
}

template <typename T>
hipError_t tsqr_domino_run(hipStream_t st, int64_t n, int d, int L, int g, const T* Y, T* Q, double* R, void* ws) {
  const DominoPlan p = make_domino_plan<T>(n, d, L, g);
  char* base = static_cast<char*>(ws);
  T* work = reinterpret_cast<T*>(base + p.off_work);
  T* tau = reinterpret_cast<T*>(base + p.off_tau);
  T* tm = reinterpret_cast<T*>(base + p.off_t);
  T* gram = reinterpret_cast<T*>(base + p.off_gram);
  T* tbig0 = reinterpret_cast<T*>(base + p.off_tbig0);
  const int G = p.groups;
  const int64_t dd = (int64_t)d * d;
  const int64_t gstride = (int64_t)g * L * d;  // first block of each group in work / Y / Q
  const int64_t sstride = (int64_t)(d + L) * d;
  const QrShape s0 = qr_shape<T>(L, L, G, d);
  const QrShape s1 = qr_shape<T>(d + L, d + L, G, d);
  const unsigned ddblocks = (unsigned)((dd + 255) / 256);
  const unsigned sblocks = (unsigned)((sstride + 255) / 256);

  // step 0: the first block of every group
  LR_TRY(launch_copy<T>(st, Y, work, n * d));
  LR_TRY(batched_qr<T>(st, work, gstride, s0, tau, tm, tbig0, gram));
  // steps 1 .. g-1: [R_{t-1}; K_t]
  const T* prev = work;
  int64_t pstride = gstride;
  for (int t = 1; t < g; ++t) {
    T* S = reinterpret_cast<T*>(base + p.off_step[t - 1]);
    T* tb = reinterpret_cast<T*>(base + p.off_stbig[t - 1]);
    hipLaunchKernelGGL(stack_step_kernel<T>, dim3(sblocks, G), dim3(256), 0, st, prev, pstride, Y, (int64_t)L, g, t,
                       d, S, sstride);
    LR_TRY(hipGetLastError());
    LR_TRY(batched_qr<T>(st, S, sstride, s1, tau, tm, tb, gram));
    prev = S;
    pstride = sstride;
  }
  double* r0 = reinterpret_cast<double*>(base + p.tree.off_r[0]);
  hipLaunchKernelGGL(extract_r_kernel<T>, dim3(ddblocks, G), dim3(256), 0, st, prev, pstride, d, d, r0, G);
  LR_TRY(hipGetLastError());
  LR_TRY(tree_run(st, p.tree, d, base, R, Q != nullptr));
  if (Q == nullptr) return hipSuccess;

  // Q back down every group, starting from the tree's block for the group
  double* mcur = reinterpret_cast<double*>(base + p.tree.off_m[0]);
  double* mnext = reinterpret_cast<double*>(base + p.off_mstep);
  T* qb = reinterpret_cast<T*>(base + p.off_qb);
  for (int t = g - 1; t >= 1; --t) {
    const T* S = reinterpret_cast<const T*>(base + p.off_step[t - 1]);
    const T* tb = reinterpret_cast<const T*>(base + p.off_stbig[t - 1]);
    hipLaunchKernelGGL(init_qblock_kernel<T>, dim3(sblocks, G), dim3(256), 0, st, mcur, qb, sstride, d + L, d + L, G,
                       d);
    LR_TRY(hipGetLastError());
    LR_TRY(batched_apply_q<T>(st, S, sstride, qb, sstride, s1, tb));
    hipLaunchKernelGGL(split_step_kernel<T>, dim3(sblocks, G), dim3(256), 0, st, qb, sstride, (int64_t)L, g, t, d,
                       mnext, Q);
    LR_TRY(hipGetLastError());
    double* tmp = mcur;
    mcur = mnext;
    mnext = tmp;
  }
  // the first block of every group: Q rows = Q_0 [M_0; 0]
  const unsigned lb = (unsigned)(((int64_t)L * d + 255) / 256);
  hipLaunchKernelGGL(init_qblock_kernel<T>, dim3(lb, G), dim3(256), 0, st, mcur, Q, gstride, L, L, G, d);
  LR_TRY(hipGetLastError());
  LR_TRY(batched_apply_q<T>(st, work, gstride, Q, gstride, s0, tbig0));
  return hipSuccess;
}

template hipError_t tsqr_domino_run<float>(hipStream_t, int64_t, int, int, int, const float*, float*, double*, void*);
template hipError_t tsqr_domino_run<double>(hipStream_t, int64_t, int, int, int, const double*, double*, double*,
                                            void*);
template hipError_t tsqr_run<float>(hipStream_t, int64_t, int, int, const float*, float*, double*, void*);
template hipError_t tsqr_run<double>(hipStream_t, int64_t, int, int, const double*, double*, double*, void*);

}  // namespace lr
