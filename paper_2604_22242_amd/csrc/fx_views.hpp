// Strided views: submatrix, transpose and diagonal leaves (Sec. 3 builds
// the element access of a transposed matrix by swapping row and column in
// the index; Sec. 4 uses the centre submatrix with half the rows and
// columns, and diagonals).
//
//   Sub<T>    element (r, c) = p[off + r + c * ld]      (submatrix)
//   Trans<T>  element (r, c) = p[off + c + r * ld]      (transposed matrix)
//   Diag<T>   element (r, 0) = p[off + r * stride]      (diagonal, a vector)
//
// t(E) moves a transpose down to the leaves at compile time:
// (B + C).t() is B.t() + C.t(), and a double transpose cancels.
//
// Evaluation.  A diagonal is a vector, so expressions over diagonals run
// through the linear skeletons.  Expressions with Sub or Trans leaves run
// through k_ew2d: one block per output tile ((16 * N) x 64 with transposed
// leaves, (64 * N) x 16 without), each thread a vector of N consecutive rows
// in four columns.  Dense and submatrix leaves
// are read straight from HBM (16-byte vectors when every view is aligned);
// a transposed leaf's source tile is first staged in LDS by the whole block
// with coalesced reads along the source's columns (column pitch 16 * N + 1
// elements, so the strided LDS writes do not conflict), and the threads
// then read their transposed vectors from LDS.
#pragma once

#include "fx_kernels.hpp"

namespace fx {

// ---- view leaves -------------------------------------------------------------

template <class T> struct Sub : expr_tag {
  using storage = T;
  using ct = ct_t<T>;
  const T* p;
  int64_t off, ld, n_rows, n_cols;
  __device__ __forceinline__ ct at(int64_t i) const {  // linear access (not on the fast path)
    const int64_t r = i % n_rows, c = i / n_rows;
    return static_cast<ct>(p[off + r + c * ld]);
  }
  template <int N, bool NT>
  __device__ __forceinline__ lanes<ct, N> at_vec(int64_t i) const {
    lanes<ct, N> x;
#pragma unroll
    for (int j = 0; j < N; ++j) x.v[j] = at(i + j);
    return x;
  }
  void collect(leaf_info& li) const {
    if (!p && n_rows * n_cols > 0) li.any_null = true;
    li.add_shape(n_rows, n_cols);
  }
  static constexpr int kLeaves = 0;  // not de-duplicated
  template <int OFF, int N, bool NT, class R>
  __device__ __forceinline__ void gather(R*, const uint8_t*, int64_t) const {}
  template <int OFF, int N, bool NT, class R>
  __device__ __forceinline__ lanes<ct, N> at_regs(const R*, int64_t i) const {
    return at_vec<N, NT>(i);
  }
  void leaf_ids(leaf_id*, int&) const {}
};

template <class T> struct Trans : expr_tag {
  using storage = T;
  using ct = ct_t<T>;
  const T* p;
  int64_t off, ld, n_rows, n_cols;
  __device__ __forceinline__ ct at(int64_t i) const {  // linear access (not on the fast path)
    const int64_t r = i % n_rows, c = i / n_rows;
    return static_cast<ct>(p[off + c + r * ld]);
  }
  template <int N, bool NT>
  __device__ __forceinline__ lanes<ct, N> at_vec(int64_t i) const {
    lanes<ct, N> x;
#pragma unroll
    for (int j = 0; j < N; ++j) x.v[j] = at(i + j);
    return x;
  }
  void collect(leaf_info& li) const {
    if (!p && n_rows * n_cols > 0) li.any_null = true;
    li.add_shape(n_rows, n_cols);
  }
  static constexpr int kLeaves = 0;
  template <int OFF, int N, bool NT, class R>
  __device__ __forceinline__ void gather(R*, const uint8_t*, int64_t) const {}
  template <int OFF, int N, bool NT, class R>
  __device__ __forceinline__ lanes<ct, N> at_regs(const R*, int64_t i) const {
    return at_vec<N, NT>(i);
  }
  void leaf_ids(leaf_id*, int&) const {}
};

template <class T> struct Diag : expr_tag {
  using storage = T;
  using ct = ct_t<T>;
  const T* p;
  int64_t off, stride, n_rows;
  static constexpr int64_t n_cols = 1;
  __device__ __forceinline__ ct at(int64_t i) const {
    return static_cast<ct>(p[off + i * stride]);
  }
  template <int N, bool NT>
  __device__ __forceinline__ lanes<ct, N> at_vec(int64_t i) const {
    lanes<ct, N> x;
#pragma unroll
    for (int j = 0; j < N; ++j) x.v[j] = at(i + j);
    return x;
  }
  void collect(leaf_info& li) const {
    if (!p && n_rows > 0) li.any_null = true;
    li.add_shape(n_rows, 1);
  }
  static constexpr int kLeaves = 0;
  template <int OFF, int N, bool NT, class R>
  __device__ __forceinline__ void gather(R*, const uint8_t*, int64_t) const {}
  template <int OFF, int N, bool NT, class R>
  __device__ __forceinline__ lanes<ct, N> at_regs(const R*, int64_t i) const {
    return at_vec<N, NT>(i);
  }
  void leaf_ids(leaf_id*, int&) const {}
};

// ---- front end ----------------------------------------------------------------

// submat(X, r0, c0, rows, cols): rows x cols block of X from (r0, c0).
template <class T> inline Sub<T> submat(const Leaf<T>& x, int64_t r0, int64_t c0, int64_t rows,
                                        int64_t cols) {
  Sub<T> s;
  s.p = x.p;
  s.off = r0 + c0 * x.n_rows;
  s.ld = x.n_rows;
  s.n_rows = rows;
  s.n_cols = cols;
  return s;
}
// diag(X, k): diagonal k of X (k > 0 above the main diagonal) as a column.
template <class T> inline Diag<T> diag(const Leaf<T>& x, int64_t k) {
  Diag<T> d;
  d.p = x.p;
  d.off = (k < 0 ? -k : 0) + (k > 0 ? k : 0) * x.n_rows;
  d.stride = x.n_rows + 1;
  d.n_rows = std::max<int64_t>(0, k >= 0 ? std::min(x.n_rows, x.n_cols - k)
                                         : std::min(x.n_rows + k, x.n_cols));
  return d;
}

// Is a leaf range inside its matrix?  (Host check for submat / diag.)
template <class T> inline bool view_inside(const Leaf<T>& x, int64_t r0, int64_t c0,
                                           int64_t rows, int64_t cols) {
  return r0 >= 0 && c0 >= 0 && rows >= 0 && cols >= 0 && r0 + rows <= x.n_rows &&
         c0 + cols <= x.n_cols;
}

template <class T> inline Trans<T> t(const Leaf<T>& x) {
  Trans<T> r;
  r.p = x.p;
  r.off = 0;
  r.ld = x.n_rows;
  r.n_rows = x.n_cols;
  r.n_cols = x.n_rows;
  return r;
}
template <class T> inline Trans<T> t(const Sub<T>& x) {
  Trans<T> r;
  r.p = x.p;
  r.off = x.off;
  r.ld = x.ld;
  r.n_rows = x.n_cols;
  r.n_cols = x.n_rows;
  return r;
}
template <class T> inline Sub<T> t(const Trans<T>& x) {
  Sub<T> r;
  r.p = x.p;
  r.off = x.off;
  r.ld = x.ld;
  r.n_rows = x.n_cols;
  r.n_cols = x.n_rows;
  return r;
}
template <class Op, class A> inline auto t(const Unary<Op, A>& u) {
  auto a = t(u.a);
  return Unary<Op, decltype(a)>{{}, a};
}
template <class Op, class A, class B> inline auto t(const Binary<Op, A, B>& b) {
  auto x = t(b.a);
  auto y = t(b.b);
  return Binary<Op, decltype(x), decltype(y)>{{}, x, y};
}
template <class Op, class A, bool LEFT> inline auto t(const Scalar<Op, A, LEFT>& s) {
  auto a = t(s.a);
  Scalar<Op, decltype(a), LEFT> r{{}, a, s.k};
  r.aux = s.aux;
  r.mode = s.mode;
  return r;
}
template <class To, class A> inline auto t(const Convert<To, A>& cv) {
  auto a = t(cv.a);
  return Convert<To, decltype(a)>{{}, a};
}
template <class T> inline auto t(const dmat<T>& m) { return t(m.expr()); }

// ---- traits -------------------------------------------------------------------

// Number of transposed leaves (each gets an LDS tile), and whether the
// expression needs the 2-D skeleton.
template <class E> struct trans_count { static constexpr int value = 0; };
template <class T> struct trans_count<Trans<T>> { static constexpr int value = 1; };
template <class Op, class A> struct trans_count<Unary<Op, A>> : trans_count<A> {};
template <class Op, class A, bool L> struct trans_count<Scalar<Op, A, L>> : trans_count<A> {};
template <class To, class A> struct trans_count<Convert<To, A>> : trans_count<A> {};
template <class Op, class A, class B> struct trans_count<Binary<Op, A, B>> {
  static constexpr int value = trans_count<A>::value + trans_count<B>::value;
};

template <class E> struct needs_2d { static constexpr bool value = false; };
template <class T> struct needs_2d<Sub<T>> { static constexpr bool value = true; };
template <class T> struct needs_2d<Trans<T>> { static constexpr bool value = true; };
template <class Op, class A> struct needs_2d<Unary<Op, A>> : needs_2d<A> {};
template <class Op, class A, bool L> struct needs_2d<Scalar<Op, A, L>> : needs_2d<A> {};
template <class To, class A> struct needs_2d<Convert<To, A>> : needs_2d<A> {};
template <class Op, class A, class B> struct needs_2d<Binary<Op, A, B>> {
  static constexpr bool value = needs_2d<A>::value || needs_2d<B>::value;
};

// ---- 2-D evaluation -------------------------------------------------------------

constexpr int kTileCols = 64;
constexpr int kTileThreads = 256;
template <int N> constexpr int kTileRows = 16 * N;
template <int N> constexpr int kTilePitch = 16 * N + 1;
template <int N> constexpr int kTileBuf = kTileCols * kTilePitch<N>;

// The tile being computed; NL is the vector width the LDS tiles were laid
// out for (a scalar read inside a vector tile keeps that layout).
template <class C, int NL> struct tile_ctx {
  C* lds;
  int64_t r0, c0;
};

// at2<TOFF, N>(e, r, c, x): rows r..r+N-1 of column c.  TOFF numbers the
// transposed leaves depth-first (their LDS tiles).
template <int TOFF, int N, class T, int NL>
__device__ __forceinline__ lanes<ct_t<T>, N> at2(const Leaf<T>& e, int64_t r, int64_t c,
                                                 const tile_ctx<ct_t<T>, NL>&) {
  if constexpr (N > 1) return load_lanes<N, kNT>(e.p, r + c * e.n_rows);
  lanes<ct_t<T>, N> v;
  v.v[0] = static_cast<ct_t<T>>(e.p[r + c * e.n_rows]);
  return v;
}
template <int TOFF, int N, class T, int NL>
__device__ __forceinline__ lanes<ct_t<T>, N> at2(const Sub<T>& e, int64_t r, int64_t c,
                                                 const tile_ctx<ct_t<T>, NL>&) {
  if constexpr (N > 1) return load_lanes<N, kNT>(e.p, e.off + r + c * e.ld);
  lanes<ct_t<T>, N> v;
  v.v[0] = static_cast<ct_t<T>>(e.p[e.off + r + c * e.ld]);
  return v;
}
template <int TOFF, int N, class T, int NL>
__device__ __forceinline__ lanes<ct_t<T>, N> at2(const Trans<T>&, int64_t r, int64_t c,
                                                 const tile_ctx<ct_t<T>, NL>& x) {
  const ct_t<T>* buf = x.lds + TOFF * kTileBuf<NL> + (c - x.c0) * kTilePitch<NL> + (r - x.r0);
  lanes<ct_t<T>, N> v;
#pragma unroll
  for (int j = 0; j < N; ++j) v.v[j] = buf[j];
  return v;
}
template <int TOFF, int N, class T, int NL>
__device__ __forceinline__ lanes<ct_t<T>, N> at2(const Diag<T>& e, int64_t r, int64_t,
                                                 const tile_ctx<ct_t<T>, NL>&) {
  return e.template at_vec<N, kNT>(r);
}
template <int TOFF, int N, class Op, class A, int NL>
__device__ __forceinline__ lanes<typename A::ct, N> at2(const Unary<Op, A>& e, int64_t r, int64_t c,
                                                        const tile_ctx<typename A::ct, NL>& x) {
  lanes<typename A::ct, N> v = at2<TOFF, N>(e.a, r, c, x);
#pragma unroll
  for (int j = 0; j < N; ++j) v.v[j] = Op::apply(v.v[j]);
  return v;
}
template <int TOFF, int N, class Op, class A, bool L, int NL>
__device__ __forceinline__ lanes<typename A::ct, N> at2(const Scalar<Op, A, L>& e, int64_t r,
                                                        int64_t c,
                                                        const tile_ctx<typename A::ct, NL>& x) {
  lanes<typename A::ct, N> v = at2<TOFF, N>(e.a, r, c, x);
#pragma unroll
  for (int j = 0; j < N; ++j) v.v[j] = e.apply1(v.v[j]);
  return v;
}
template <int TOFF, int N, class Op, class A, class B, int NL>
__device__ __forceinline__ lanes<typename A::ct, N> at2(const Binary<Op, A, B>& e, int64_t r,
                                                        int64_t c,
                                                        const tile_ctx<typename A::ct, NL>& x) {
  lanes<typename A::ct, N> u = at2<TOFF, N>(e.a, r, c, x);
  lanes<typename A::ct, N> w = at2<TOFF + trans_count<A>::value, N>(e.b, r, c, x);
#pragma unroll
  for (int j = 0; j < N; ++j) u.v[j] = Op::apply(u.v[j], w.v[j]);
  return u;
}
template <int TOFF, int N, class To, class A, int NL>
__device__ __forceinline__ lanes<To, N> at2(const Convert<To, A>& e, int64_t r, int64_t c,
                                            const tile_ctx<To, NL>& x) {
  static_assert(trans_count<A>::value == 0, "a transposed leaf below conv_to is not staged");
  const tile_ctx<typename A::ct, NL> none{nullptr, x.r0, x.c0};
  lanes<typename A::ct, N> v = at2<0, N>(e.a, r, c, none);
  lanes<To, N> o;
#pragma unroll
  for (int j = 0; j < N; ++j) o.v[j] = static_cast<To>(v.v[j]);
  return o;
}

// stage<TOFF, N>: every transposed leaf loads its source tile into LDS.
template <int TOFF, int N, class E>
__device__ __forceinline__ void stage(const E&, const tile_ctx<typename E::ct, N>&, int64_t, int64_t) {}
template <int TOFF, int N, class T>
__device__ __forceinline__ void stage(const Trans<T>& e, const tile_ctx<ct_t<T>, N>& x, int64_t rows,
                                      int64_t cols) {
  ct_t<T>* buf = x.lds + TOFF * kTileBuf<N>;
  constexpr int TR = kTileRows<N>;
  // idx -> (view columns cl..cl+N-1, view row rl); consecutive threads take
  // consecutive view columns = consecutive source rows (coalesced); with
  // N > 1 the host has checked that these N source elements form one
  // aligned vector inside the source column
  constexpr int CV = kTileCols / N;  // vectors per view row of the tile
  for (int idx = threadIdx.x; idx < TR * CV; idx += kTileThreads) {
    const int cl = (idx % CV) * N, rl = idx / CV;
    const int64_t r = x.r0 + rl, c = x.c0 + cl;
    if (r >= rows || c >= cols) continue;
    if constexpr (N > 1) {
      const lanes<ct_t<T>, N> v = load_lanes<N, kNT>(e.p, e.off + c + r * e.ld);
#pragma unroll
      for (int j = 0; j < N; ++j) buf[(cl + j) * kTilePitch<N> + rl] = v.v[j];
    } else {
      buf[cl * kTilePitch<N> + rl] = static_cast<ct_t<T>>(e.p[e.off + c + r * e.ld]);
    }
  }
}
template <int TOFF, int N, class Op, class A>
__device__ __forceinline__ void stage(const Unary<Op, A>& e, const tile_ctx<typename A::ct, N>& x,
                                      int64_t rows, int64_t cols) {
  stage<TOFF, N>(e.a, x, rows, cols);
}
template <int TOFF, int N, class Op, class A, bool L>
__device__ __forceinline__ void stage(const Scalar<Op, A, L>& e, const tile_ctx<typename A::ct, N>& x,
                                      int64_t rows, int64_t cols) {
  stage<TOFF, N>(e.a, x, rows, cols);
}
template <int TOFF, int N, class Op, class A, class B>
__device__ __forceinline__ void stage(const Binary<Op, A, B>& e, const tile_ctx<typename A::ct, N>& x,
                                      int64_t rows, int64_t cols) {
  stage<TOFF, N>(e.a, x, rows, cols);
  stage<TOFF + trans_count<A>::value, N>(e.b, x, rows, cols);
}

// Workgroups are dispatched to the eight XCDs round-robin by block id, and
// each XCD has its own L2.  Where a leading dimension is not a multiple of
// the 128-byte line (10000 floats = 40000 B), vertically adjacent tiles
// share the line their column runs straddle; under the plain order those two
// tiles run on different XCDs and both fetch it from HBM (12% more reads for
// submatrices, 25% with transposes).  xcd_order() gives each XCD a
// contiguous run of tiles instead (a bijection on [0, G)), so the second
// fetch of a shared line is an L2 hit.
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_order(uint32_t b, uint32_t G) {
  const uint32_t per = G / kXcds, extra = G % kXcds;
  const uint32_t xcd = b % kXcds, k = b / kXcds;
  return xcd * per + (xcd < extra ? xcd : extra) + k;
}

// Z (dense rows x cols) = E over a grid of tiles, numbered down the tile
// columns (tile t: tile row t % tile_rows, tile column t / tile_rows) and
// taken in xcd_order.  (Launching the partner tiles (I, J) and (J, I) side
// by side, to find a transposed operand's tile in the last-level cache,
// measured slower on the 10k x 10k expressions.)
// Tile geometry: with transposed leaves the tile is (16 N) x 64 (square for
// FP32, the LDS staging tile); without them it is (64 N) x 16, so that each
// column of every leaf is read in 1 KB-or-longer contiguous runs (square
// tiles read only 256 B per column of a submatrix, measured slower).
template <int KT> constexpr int kRowVecs = KT > 0 ? 16 : 64;        // thread rows per tile
template <int KT> constexpr int kColsPerTile = KT > 0 ? kTileCols : 16;

template <class E, class T, int N, bool NTS>
__global__ __launch_bounds__(kTileThreads) void k_ew2d(E e, T* __restrict__ z, int64_t rows,
                                                      int64_t cols, uint32_t tile_rows) {
  using C = typename E::ct;
  constexpr int KT = trans_count<E>::value;
  constexpr int RV = kRowVecs<KT>, CG = kTileThreads / RV, TC = kColsPerTile<KT>;
  __shared__ C lds[KT > 0 ? KT * kTileBuf<N> : 1];
  const uint32_t t = xcd_order(blockIdx.x, gridDim.x);
  const tile_ctx<C, N> x{lds, (int64_t)(t % tile_rows) * RV * N, (int64_t)(t / tile_rows) * TC};
  if constexpr (KT > 0) {
    static_assert(RV * N == kTileRows<N> && TC == kTileCols, "staging tile geometry");
    stage<0, N>(e, x, rows, cols);
    __syncthreads();
  }
  const int rv = threadIdx.x % RV, cg = threadIdx.x / RV;
  const int64_t r = x.r0 + rv * N;
#pragma unroll
  for (int q = 0; q < TC / CG; ++q) {
    const int64_t c = x.c0 + cg + CG * q;
    if (c >= cols || r >= rows) continue;
    if (r + N <= rows) {
      store_lanes<N, NTS>(z, r + c * rows, at2<0, N>(e, r, c, x));
    } else {
      for (int j = 0; r + j < rows; ++j) z[r + j + c * rows] = static_cast<T>(at2<0, 1>(e, r + j, c, x).v[0]);
    }
  }
}

// ---- paired tiles: a matrix read both directly and transposed ----------------
//
// When an expression over square matrices names a matrix both directly and
// transposed (expr1: X and X.t()), output tiles (I, J) and (J, I) need the same
// two tiles of it.  One block then computes both output tiles: it stages tiles
// (I, J) and (J, I) of every distinct matrix in LDS once (natural layout,
// column pitch 65) and every leaf reads from there, the direct ones at
// [c][r] of their own tile, the transposed ones at [r][c] of the partner
// tile.  Each matrix is read from HBM once.  FP32 (64 x 64 square tiles),
// whole matrices only, at most kPairMats distinct ones.
constexpr int kPairMats = 2;
constexpr int kPairT = 64;            // tile side
constexpr int kPairPitch = kPairT + 1;
constexpr int kPairBuf = kPairT * kPairPitch;

template <class E> struct pairable { static constexpr bool value = false; };
template <class T> struct pairable<Leaf<T>> { static constexpr bool value = true; };
template <class T> struct pairable<Trans<T>> { static constexpr bool value = true; };
template <class Op, class A> struct pairable<Unary<Op, A>> : pairable<A> {};
template <class Op, class A, bool L> struct pairable<Scalar<Op, A, L>> : pairable<A> {};
template <class Op, class A, class B> struct pairable<Binary<Op, A, B>> {
  static constexpr bool value = pairable<A>::value && pairable<B>::value;
};
template <class E> struct pair_leaves { static constexpr int value = 0; };
template <class T> struct pair_leaves<Leaf<T>> { static constexpr int value = 1; };
template <class T> struct pair_leaves<Trans<T>> { static constexpr int value = 1; };
template <class Op, class A> struct pair_leaves<Unary<Op, A>> : pair_leaves<A> {};
template <class Op, class A, bool L> struct pair_leaves<Scalar<Op, A, L>> : pair_leaves<A> {};
template <class Op, class A, class B> struct pair_leaves<Binary<Op, A, B>> {
  static constexpr int value = pair_leaves<A>::value + pair_leaves<B>::value;
};
constexpr int kPairMaxLeaves = 16;

struct pair_tab {
  uint8_t mid[kPairMaxLeaves];  // leaf (depth-first) -> distinct matrix
  const float* mat[kPairMats];  // distinct matrices
  int32_t n_mats;
};

struct pair_ctx {
  const float* lds;
  const uint8_t* mid;
  int64_t r0, c0;
  int swap;  // 0: output tile (I, J), 1: its partner (J, I)
};

// region 2m holds tile (I, J) of matrix m, region 2m + 1 tile (J, I)
template <int LOFF, class T>
__device__ __forceinline__ lanes<float, 4> at2p(const Leaf<T>&, int64_t r, int64_t c,
                                                const pair_ctx& x) {
  const float* b = x.lds + (2 * x.mid[LOFF] + x.swap) * kPairBuf + (c - x.c0) * kPairPitch + (r - x.r0);
  lanes<float, 4> v;
#pragma unroll
  for (int j = 0; j < 4; ++j) v.v[j] = b[j];
  return v;
}
template <int LOFF, class T>
__device__ __forceinline__ lanes<float, 4> at2p(const Trans<T>&, int64_t r, int64_t c,
                                                const pair_ctx& x) {
  const float* b = x.lds + (2 * x.mid[LOFF] + 1 - x.swap) * kPairBuf + (r - x.r0) * kPairPitch + (c - x.c0);
  lanes<float, 4> v;
#pragma unroll
  for (int j = 0; j < 4; ++j) v.v[j] = b[j * kPairPitch];
  return v;
}
template <int LOFF, class Op, class A>
__device__ __forceinline__ lanes<float, 4> at2p(const Unary<Op, A>& e, int64_t r, int64_t c,
                                                const pair_ctx& x) {
  lanes<float, 4> v = at2p<LOFF>(e.a, r, c, x);
#pragma unroll
  for (int j = 0; j < 4; ++j) v.v[j] = Op::apply(v.v[j]);
  return v;
}
template <int LOFF, class Op, class A, bool L>
__device__ __forceinline__ lanes<float, 4> at2p(const Scalar<Op, A, L>& e, int64_t r, int64_t c,
                                                const pair_ctx& x) {
  lanes<float, 4> v = at2p<LOFF>(e.a, r, c, x);
#pragma unroll
  for (int j = 0; j < 4; ++j) v.v[j] = e.apply1(v.v[j]);
  return v;
}
template <int LOFF, class Op, class A, class B>
__device__ __forceinline__ lanes<float, 4> at2p(const Binary<Op, A, B>& e, int64_t r, int64_t c,
                                                const pair_ctx& x) {
  lanes<float, 4> u = at2p<LOFF>(e.a, r, c, x);
  lanes<float, 4> w = at2p<LOFF + pair_leaves<A>::value>(e.b, r, c, x);
#pragma unroll
  for (int j = 0; j < 4; ++j) u.v[j] = Op::apply(u.v[j], w.v[j]);
  return u;
}

// One block per tile pair I <= J (p enumerates them column by column); n x n
// FP32 result, n a multiple of 4.
template <class E, bool NTS>
__global__ __launch_bounds__(kTileThreads) void k_ew2d_pair(E e, pair_tab tab, float* __restrict__ z,
                                                           int64_t n) {
  __shared__ float lds[2 * kPairMats * kPairBuf];
  const int64_t p = xcd_order(blockIdx.x, gridDim.x);
  int64_t J = (int64_t)((::sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
  while (J * (J + 1) / 2 > p) --J;
  while ((J + 1) * (J + 2) / 2 <= p) ++J;
  const int64_t I = p - J * (J + 1) / 2;
  // stage tiles (I, J) and (J, I) of every matrix: 16-byte loads down the
  // columns (64 rows = 16 vectors per column); each thread issues all its
  // loads before the first LDS write
  constexpr int PER = kPairT * (kPairT / 4) / kTileThreads;  // vectors per thread per tile
  lanes<float, 4> v[kPairMats][2][PER];
#pragma unroll
  for (int m = 0; m < kPairMats; ++m)
#pragma unroll
    for (int w = 0; w < 2; ++w)
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int idx = threadIdx.x + k * kTileThreads;
        const int64_t r = (w ? J : I) * kPairT + (idx % (kPairT / 4)) * 4;
        const int64_t c = (w ? I : J) * kPairT + idx / (kPairT / 4);
        if (m < tab.n_mats && r < n && c < n) v[m][w][k] = load_lanes<4, kNT>(tab.mat[m], r + c * n);
      }
#pragma unroll
  for (int m = 0; m < kPairMats; ++m)
#pragma unroll
    for (int w = 0; w < 2; ++w)
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int idx = threadIdx.x + k * kTileThreads;
        const int rl = (idx % (kPairT / 4)) * 4, cl = idx / (kPairT / 4);
        float* buf = lds + (2 * m + w) * kPairBuf + cl * kPairPitch + rl;
        if (m < tab.n_mats)
#pragma unroll
          for (int j = 0; j < 4; ++j) buf[j] = v[m][w][k].v[j];
      }
  __syncthreads();
  const int rv = threadIdx.x % 16, cg = threadIdx.x / 16;
  for (int s = 0; s < (I == J ? 1 : 2); ++s) {
    const pair_ctx x{lds, tab.mid, (s ? J : I) * kPairT, (s ? I : J) * kPairT, s};
    const int64_t r = x.r0 + rv * 4;
#pragma unroll
    for (int q = 0; q < kPairT / 16; ++q) {
      const int64_t c = x.c0 + cg + 16 * q;
      if (c < n && r < n) store_lanes<4, NTS>(z, r + c * n, at2p<0>(e, r, c, x));
    }
  }
}

// Host: the leaves (depth-first) of a pairable expression.
template <class T> inline void pair_leaf_list(const Leaf<T>& e, const void** p, int64_t* off,
                                              int64_t* ld, bool* tr, int& k) {
  p[k] = e.p; off[k] = 0; ld[k] = e.n_rows; tr[k] = false; ++k;
}
template <class T> inline void pair_leaf_list(const Trans<T>& e, const void** p, int64_t* off,
                                              int64_t* ld, bool* tr, int& k) {
  p[k] = e.p; off[k] = e.off; ld[k] = e.ld; tr[k] = true; ++k;
}
template <class Op, class A> inline void pair_leaf_list(const Unary<Op, A>& e, const void** p,
                                                        int64_t* off, int64_t* ld, bool* tr, int& k) {
  pair_leaf_list(e.a, p, off, ld, tr, k);
}
template <class Op, class A, bool L> inline void pair_leaf_list(const Scalar<Op, A, L>& e,
                                                                const void** p, int64_t* off,
                                                                int64_t* ld, bool* tr, int& k) {
  pair_leaf_list(e.a, p, off, ld, tr, k);
}
template <class Op, class A, class B> inline void pair_leaf_list(const Binary<Op, A, B>& e,
                                                                 const void** p, int64_t* off,
                                                                 int64_t* ld, bool* tr, int& k) {
  pair_leaf_list(e.a, p, off, ld, tr, k);
  pair_leaf_list(e.b, p, off, ld, tr, k);
}

// Build the pair table if the paired kernel applies: n x n FP32 result,
// every leaf a whole n x n matrix, at most kPairMats distinct ones, one of
// them read both ways, 16-byte aligned.
template <class E> inline bool pair_plan(const E& e, int64_t n, const float* z, pair_tab* tab) {
  constexpr int L = pair_leaves<E>::value;
  if (L > kPairMaxLeaves || n % 4 || reinterpret_cast<uintptr_t>(z) % 16) return false;
  const void* p[kPairMaxLeaves];
  int64_t off[kPairMaxLeaves], ld[kPairMaxLeaves];
  bool tr[kPairMaxLeaves];
  int k = 0;
  pair_leaf_list(e, p, off, ld, tr, k);
  bool dir[kPairMats] = {false, false}, trn[kPairMats] = {false, false};
  tab->n_mats = 0;
  for (int i = 0; i < L; ++i) {
    if (off[i] != 0 || ld[i] != n || reinterpret_cast<uintptr_t>(p[i]) % 16) return false;
    int m = 0;
    while (m < tab->n_mats && tab->mat[m] != p[i]) ++m;
    if (m == tab->n_mats) {
      if (m == kPairMats) return false;
      tab->mat[m] = static_cast<const float*>(p[i]);
      ++tab->n_mats;
    }
    tab->mid[i] = (uint8_t)m;
    (tr[i] ? trn : dir)[m] = true;
  }
  for (int m = 0; m < tab->n_mats; ++m)
    if (dir[m] && trn[m]) return true;
  return false;
}

// Host: may every dense / submatrix leaf and the output be read N at a time?
template <class T> inline bool vec_ok(const Leaf<T>& e, int N) {
  return (reinterpret_cast<uintptr_t>(e.p) % (N * sizeof(T))) == 0 && e.n_rows % N == 0;
}
template <class T> inline bool vec_ok(const Sub<T>& e, int N) {
  return (reinterpret_cast<uintptr_t>(e.p + e.off) % (N * sizeof(T))) == 0 && e.ld % N == 0;
}
template <class T> inline bool vec_ok(const Trans<T>& e, int N) {  // staged N source rows at a time
  return (reinterpret_cast<uintptr_t>(e.p + e.off) % (N * sizeof(T))) == 0 && e.ld % N == 0 &&
         e.n_cols % N == 0;
}
template <class T> inline bool vec_ok(const Diag<T>&, int) { return true; }
template <class Op, class A> inline bool vec_ok(const Unary<Op, A>& e, int N) { return vec_ok(e.a, N); }
template <class Op, class A, bool L> inline bool vec_ok(const Scalar<Op, A, L>& e, int N) {
  return vec_ok(e.a, N);
}
template <class To, class A> inline bool vec_ok(const Convert<To, A>& e, int N) { return vec_ok(e.a, N); }
template <class Op, class A, class B> inline bool vec_ok(const Binary<Op, A, B>& e, int N) {
  return vec_ok(e.a, N) && vec_ok(e.b, N);
}

// Z = E for an expression with submatrix or transposed leaves.
template <class E, class T>
int eval_views(T* z, const E& e, hipStream_t st) {
  int64_t rows, cols;
  if (int rc = check_expr(e, &rows, &cols)) return rc;
  if (rows * cols == 0) return FX_OK;
  if (!z) return fail(FX_E_ARG, "NULL output pointer");
  constexpr int NV = 16 / (int)sizeof(T) > 0 ? 16 / (int)sizeof(T) : 1;
  const bool vec = vec_ok(e, NV) && rows % NV == 0 &&
                   reinterpret_cast<uintptr_t>(z) % 16 == 0;
  constexpr int KT = trans_count<E>::value;
  const bool nts = kNTS || (uint64_t)rows * (uint64_t)cols * sizeof(T) > kStreamStoresAbove;
  if constexpr (KT > 0 && pairable<E>::value && std::is_same_v<T, float> &&
                std::is_same_v<typename E::ct, float>) {
    pair_tab tab;
    if (rows == cols && pair_plan(e, rows, z, &tab)) {
      const int64_t t = ceil_div(rows, (int64_t)kPairT);
      if (nts)
        hipLaunchKernelGGL((k_ew2d_pair<E, true>), dim3((unsigned)(t * (t + 1) / 2)),
                           dim3(kTileThreads), 0, st, e, tab, z, rows);
      else
        hipLaunchKernelGGL((k_ew2d_pair<E, false>), dim3((unsigned)(t * (t + 1) / 2)),
                           dim3(kTileThreads), 0, st, e, tab, z, rows);
      return hip_check(hipGetLastError(), "k_ew2d_pair launch");
    }
  }
  const int64_t tc = ceil_div(cols, kColsPerTile<KT>);
  const int64_t tr = ceil_div(rows, (int64_t)kRowVecs<KT> * (vec ? NV : 1));
  if (tr * tc > 0x7fffffff)
    return fail(FX_E_UNSUPPORTED, "%lld x %lld exceeds the tile grid", (long long)rows, (long long)cols);
  const dim3 grid((unsigned)(tr * tc)), block(kTileThreads);
  if (vec && nts)
    hipLaunchKernelGGL((k_ew2d<E, T, NV, true>), grid, block, 0, st, e, z, rows, cols, (uint32_t)tr);
  else if (vec)
    hipLaunchKernelGGL((k_ew2d<E, T, NV, false>), grid, block, 0, st, e, z, rows, cols, (uint32_t)tr);
  else
    hipLaunchKernelGGL((k_ew2d<E, T, 1, false>), grid, block, 0, st, e, z, rows, cols, (uint32_t)tr);
  return hip_check(hipGetLastError(), "k_ew2d launch");
}

}  // namespace fx
