// Register-resident mixed-radix FFT passes for CDNA4 (gfx950, wave64).
//
// A workgroup owns a 2-D tile of complex values (a plane of the FFT box, or a
// bundle of pencils).  A 1-D transform of length L along one tile axis is done
// in two radix passes (L = R0 * R1, radices 3..16) in the autosort
// (Stockham) form: pass s with radix R and span P (product of the radices
// already done) takes butterfly i, k = i mod P, reads x[i + r L/R], multiplies
// by the twiddle w_{PR}^{r k}, does a radix-R DFT in registers, and writes
// y[(i - k) R + k + r P].  After the last pass the output is in natural order.
//
// Values live in registers across a pass; between passes they are exchanged
// through LDS (rows padded by one element to spread banks).  The first pass
// of a transform can read straight from HBM and the last can write straight
// to HBM, so a whole 2-D transform costs one HBM read and one HBM write.
//
// Lane mapping: for a transform along the contiguous tile axis ("row") the
// lanes walk the butterfly index first, for the strided axis ("column") they
// walk the batch (column) index first; both keep HBM accesses coalesced.
//
// Twiddle factors: compile-time constants inside the radix DFTs are computed
// by a constexpr sine/cosine of an exact rational multiple of 2 pi (octant
// reduction in integers, Taylor series on [0, pi/4]); the inter-pass factors
// come from a per-length table built on the host by the same function in
// FP64 (rounded once to FP32 for the FP32 path).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fockx {

// ---------------------------------------------------------------------------
// complex helpers
// ---------------------------------------------------------------------------
template <typename T> struct cx_of;
template <> struct cx_of<float> { using type = float2; };
template <> struct cx_of<double> { using type = double2; };
template <typename T> using cx = typename cx_of<T>::type;

// Load and store marked non-temporal, for the pair buffer: each pass writes
// a tile's pairs in full or reads each of them once, so its lines need not
// stay in the caches, which then keep the orbital planes the passes re-read.
template <typename T> __device__ __forceinline__ cx<T> load_stream(const cx<T>* p) {
  using V = T __attribute__((ext_vector_type(2)));
  const V x = __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
  cx<T> r;
  r.x = x.x;
  r.y = x.y;
  return r;
}
template <typename T> __device__ __forceinline__ void store_stream(cx<T>* p, cx<T> v) {
  using V = T __attribute__((ext_vector_type(2)));
  V x = {v.x, v.y};
  __builtin_nontemporal_store(x, reinterpret_cast<V*>(p));
}

template <typename T> __host__ __device__ __forceinline__ cx<T> mk(T x, T y) {
  cx<T> r;
  r.x = x;
  r.y = y;
  return r;
}
template <typename T> __device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T> __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
template <typename T> __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return mk<T>(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
template <typename T> __device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
// multiply by DIR * i  (DIR = +1 or -1)
template <int DIR, typename T> __device__ __forceinline__ cx<T> rot_i(cx<T> v) {
  return DIR > 0 ? mk<T>(-v.y, v.x) : mk<T>(v.y, -v.x);
}

// ---------------------------------------------------------------------------
// constexpr cos / sin of 2 pi num / den
// ---------------------------------------------------------------------------
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double taylor_sin(double x) {
  double term = x, sum = x;
  for (int k = 1; k < 16; ++k) {
    term *= -x * x / double((2 * k) * (2 * k + 1));
    sum += term;
  }
  return sum;
}
constexpr double taylor_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 16; ++k) {
    term *= -x * x / double((2 * k - 1) * (2 * k));
    sum += term;
  }
  return sum;
}
struct CosSin {
  double c, s;
};
// cos and sin of 2 pi num / den.  The angle is reduced to a quadrant with
// integer arithmetic, then to [0, pi/4] by the complement identity.
__host__ __device__ constexpr CosSin cossin_2pi(long num, long den) {
  num %= den;
  if (num < 0) num += den;
  const long quad = (4 * num) / den;
  const long rem = 4 * num - quad * den;  // angle inside the quadrant = rem/den * pi/2
  double c = 0.0, s = 0.0;
  if (2 * rem <= den) {
    const double x = double(rem) / double(den) * (kPi / 2);
    c = taylor_cos(x);
    s = taylor_sin(x);
  } else {
    const double x = double(den - rem) / double(den) * (kPi / 2);
    c = taylor_sin(x);
    s = taylor_cos(x);
  }
  switch (quad) {
    case 0: return CosSin{c, s};
    case 1: return CosSin{-s, c};
    case 2: return CosSin{-c, -s};
    default: return CosSin{s, -c};
  }
}

// v * exp(DIR * 2 pi i E / R), E a compile-time integer
template <int E, int R, int DIR, typename T> __device__ __forceinline__ cx<T> twc(cx<T> v) {
  constexpr int e = (((DIR * E) % R) + R) % R;
  if constexpr (e == 0) {
    return v;
  } else if constexpr ((4 * e) % R == 0) {
    constexpr int q = 4 * e / R;  // 1: i, 2: -1, 3: -i
    if constexpr (q == 1) return mk<T>(-v.y, v.x);
    else if constexpr (q == 2) return mk<T>(-v.x, -v.y);
    else return mk<T>(v.y, -v.x);
  } else if constexpr ((8 * e) % R == 0) {
    constexpr T h = T(0.70710678118654752440084436210484904);
    constexpr int o = 8 * e / R;  // odd: 1,3,5,7 -> (1+i)/sqrt2 * i^((o-1)/2)
    const cx<T> w = mk<T>((v.x - v.y) * h, (v.x + v.y) * h);
    if constexpr (o == 1) return w;
    else if constexpr (o == 3) return mk<T>(-w.y, w.x);
    else if constexpr (o == 5) return mk<T>(-w.x, -w.y);
    else return mk<T>(w.y, -w.x);
  } else {
    constexpr CosSin cs = cossin_2pi(e, R);
    constexpr T c = T(cs.c), s = T(cs.s);
    return mk<T>(v.x * c - v.y * s, v.x * s + v.y * c);
  }
}

// ---------------------------------------------------------------------------
// radix-R DFT in registers: x[t] <- sum_s x[s] exp(DIR 2 pi i s t / R)
// ---------------------------------------------------------------------------
template <int R> constexpr int radix_split() {
  return (R == 8 || R == 12 || R == 16) ? 4 : (R == 9 ? 3 : (R == 6 ? 2 : 0));
}

template <int R, int DIR, typename T> __device__ __forceinline__ void dft(cx<T>* x);

template <int R, int DIR, typename T, int A, int B>
__device__ __forceinline__ void dft_composite(cx<T>* x) {
  // x[m1 B + m2]: B transforms of size A over m1, twiddle w_R^{m2 k1}, then A of size B over m2.
  cx<T> y[R];
#pragma unroll
  for (int m2 = 0; m2 < B; ++m2) {
    cx<T> a[A];
#pragma unroll
    for (int m1 = 0; m1 < A; ++m1) a[m1] = x[m1 * B + m2];
    dft<A, DIR, T>(a);
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) y[m2 * A + k1] = a[k1];
  }
  // twiddles with compile-time exponents m2 * k1
  [&]<int... I>(std::integer_sequence<int, I...>) {
    ((y[I] = twc<(I / A) * (I % A), R, DIR, T>(y[I])), ...);
  }(std::make_integer_sequence<int, R>{});
#pragma unroll
  for (int k1 = 0; k1 < A; ++k1) {
    cx<T> b[B];
#pragma unroll
    for (int m2 = 0; m2 < B; ++m2) b[m2] = y[m2 * A + k1];
    dft<B, DIR, T>(b);
#pragma unroll
    for (int k2 = 0; k2 < B; ++k2) x[k1 + A * k2] = b[k2];
  }
}

template <int R, int DIR, typename T> __device__ __forceinline__ void dft(cx<T>* x) {
  if constexpr (R == 1) {
    return;
  } else if constexpr (R == 2) {
    const cx<T> a = x[0], b = x[1];
    x[0] = cadd<T>(a, b);
    x[1] = csub<T>(a, b);
  } else if constexpr (R == 3) {
    constexpr T s3 = T(0.86602540378443864676372317075293618);
    const cx<T> t1 = cadd<T>(x[1], x[2]);
    const cx<T> t2 = mk<T>(x[0].x - T(0.5) * t1.x, x[0].y - T(0.5) * t1.y);
    const cx<T> d = csub<T>(x[1], x[2]);
    const cx<T> t3 = rot_i<DIR, T>(mk<T>(s3 * d.x, s3 * d.y));
    x[0] = cadd<T>(x[0], t1);
    x[1] = cadd<T>(t2, t3);
    x[2] = csub<T>(t2, t3);
  } else if constexpr (R == 4) {
    const cx<T> s02 = cadd<T>(x[0], x[2]), d02 = csub<T>(x[0], x[2]);
    const cx<T> s13 = cadd<T>(x[1], x[3]), d13 = rot_i<DIR, T>(csub<T>(x[1], x[3]));
    x[0] = cadd<T>(s02, s13);
    x[2] = csub<T>(s02, s13);
    x[1] = cadd<T>(d02, d13);
    x[3] = csub<T>(d02, d13);
  } else {
    constexpr int A = radix_split<R>();
    static_assert(A > 0 && R % A == 0, "unsupported radix");
    dft_composite<R, DIR, T, A, R / A>(x);
  }
}

// ---------------------------------------------------------------------------
// One autosort pass over a tile held by W threads.
//   L      transform length, R radix, P span (product of earlier radices)
//   BATCH  number of transforms in the tile
//   ROW    true: transform along the contiguous axis: element (b, x) is at
//          tile row b, column x; false: along the strided axis: element
//          (b, x) is at row x, column b
//   LB     lanes walk the batch index b first (default for a column pass,
//          whose lanes then walk the tile's columns); otherwise the
//          butterfly index i (default for a row pass, whose lanes then walk
//          the row).  Either keeps HBM accesses coalesced in the default; a
//          row pass that only touches LDS may walk the batch (rows) instead,
//          which spreads an exchange's lanes over rows, hence banks.
//   SL     row stride of the tile in LDS (padded; in elements)
// Thread t owns butterflies beta = t + s W, s < NS.  W is a multiple of the
// lane-fastest extent (BATCH if LB, else NI), so (b, i) are affine in s and
// every element position is base(t) + constant: the per-element offsets
// fold into instruction immediates.
// ---------------------------------------------------------------------------
template <int L_, int R_, int P_, int BATCH_, bool ROW_, int W_, bool LB_ = !ROW_> struct Pass {
  static constexpr int L = L_, R = R_, P = P_, BATCH = BATCH_, W = W_;
  static constexpr bool ROW = ROW_, LB = LB_;
  static constexpr int NI = L / R;           // butterflies per transform
  static constexpr int NBF = BATCH * NI;     // butterflies in the tile
  static constexpr int NS = (NBF + W - 1) / W;
  static constexpr bool EXACT = (NBF % W) == 0;
  static constexpr int NV = NS * R;          // register values per thread
  static constexpr int FAST = LB ? BATCH : NI;
  static_assert(L % R == 0 && L % (P * R) == 0, "bad pass");
  static_assert(P == 1 || P == NI, "two-pass factorisations only");
  static_assert(W % FAST == 0, "block size must be a multiple of the lane-fastest extent");
  static constexpr int STEP = W / FAST;      // per-slot increment of the slow index

  struct Lane {
    int b0, i0;   // slot-0 batch index and butterfly index
    int tlim;     // last slot active iff t < tlim
  };
  __device__ static __forceinline__ Lane lane(int t) {
    Lane l;
    if constexpr (LB) {
      l.b0 = t % BATCH;
      l.i0 = t / BATCH;
    } else {
      l.i0 = t % NI;
      l.b0 = t / NI;
    }
    l.tlim = NBF - (NS - 1) * W;
    return l;
  }
  __device__ static __forceinline__ int b_of(const Lane& l, int s) { return LB ? l.b0 : l.b0 + s * STEP; }
  __device__ static __forceinline__ int i_of(const Lane& l, int s) { return LB ? l.i0 + s * STEP : l.i0; }
  __device__ static __forceinline__ bool active(const Lane& l, int t, int s) {
    return EXACT || s < NS - 1 || t < l.tlim;
  }
  __device__ static __forceinline__ int in_x(int i, int r) { return i + r * NI; }
  // P == 1: k = 0;  P == NI (last pass of two): i < P so k = i
  __device__ static __forceinline__ int out_x(int i, int r) { return P == 1 ? i * R + r : i + r * P; }
  // (b, x) -> (row, col) of the tile
  __device__ static __forceinline__ int row_of(int b, int x) { return ROW ? b : x; }
  __device__ static __forceinline__ int col_of(int b, int x) { return ROW ? x : b; }
};

// Factorisation L = R0 * R1 used for each supported length.
template <int L> struct Factor;
template <> struct Factor<24> { static constexpr int R0 = 8, R1 = 3; };
template <> struct Factor<48> { static constexpr int R0 = 8, R1 = 6; };
template <> struct Factor<64> { static constexpr int R0 = 8, R1 = 8; };
template <> struct Factor<72> { static constexpr int R0 = 8, R1 = 9; };
template <> struct Factor<96> { static constexpr int R0 = 8, R1 = 12; };
template <> struct Factor<128> { static constexpr int R0 = 8, R1 = 16; };

// The two passes of a length-L transform over a tile (radices FR0 then FR1),
// with the default lane order (P0, P1) and, for a row transform, with the
// lanes walking the rows (P0b, P1b: for a pass that reads and writes only LDS).
template <int L, int BATCH, bool ROW, int W, int FR0 = Factor<L>::R0, int FR1 = Factor<L>::R1> struct Axis {
  static_assert(FR0 * FR1 == L, "bad factorisation");
  using P0 = Pass<L, FR0, 1, BATCH, ROW, W>;
  using P1 = Pass<L, FR1, FR0, BATCH, ROW, W>;
  static constexpr bool LB_OK = W % BATCH == 0;  // the batch can be the lane-fastest index
  using P0b = Pass<L, FR0, 1, BATCH, ROW, W, LB_OK>;
  using P1b = Pass<L, FR1, FR0, BATCH, ROW, W, LB_OK>;
  static constexpr int NV = P0::NV > P1::NV ? P0::NV : P1::NV;
};

// f(e, row, col) for every input (for_inputs) / output (for_outputs) value
// e of this thread in pass PS.
template <class PS, class F> __device__ __forceinline__ void for_inputs(int t, F&& f) {
  const typename PS::Lane l = PS::lane(t);
#pragma unroll
  for (int s = 0; s < PS::NS; ++s) {
    if (!PS::active(l, t, s)) continue;
    const int b = PS::b_of(l, s), i = PS::i_of(l, s);
#pragma unroll
    for (int r = 0; r < PS::R; ++r) {
      const int x = PS::in_x(i, r);
      f(s * PS::R + r, PS::row_of(b, x), PS::col_of(b, x));
    }
  }
}
template <class PS, class F> __device__ __forceinline__ void for_outputs(int t, F&& f) {
  const typename PS::Lane l = PS::lane(t);
#pragma unroll
  for (int s = 0; s < PS::NS; ++s) {
    if (!PS::active(l, t, s)) continue;
    const int b = PS::b_of(l, s), i = PS::i_of(l, s);
#pragma unroll
    for (int r = 0; r < PS::R; ++r) {
      const int x = PS::out_x(i, r);
      f(s * PS::R + r, PS::row_of(b, x), PS::col_of(b, x));
    }
  }
}

// Twiddle multiply + radix DFT for every butterfly this thread owns.
// tw[m] = exp(-2 pi i m / L); DIR = -1 forward, +1 backward.
template <class PS, int DIR, typename T>
__device__ __forceinline__ void pass_compute(cx<T>* v, const cx<T>* tw, int t) {
  const typename PS::Lane l = PS::lane(t);
#pragma unroll
  for (int s = 0; s < PS::NS; ++s) {
    if constexpr (PS::P > 1) {
      const int k = PS::i_of(l, s);  // k = i for the last pass of two
#pragma unroll
      for (int r = 1; r < PS::R; ++r) {
        cx<T> w = tw[r * k];
        if constexpr (DIR > 0) w.y = -w.y;
        v[s * PS::R + r] = cmul<T>(v[s * PS::R + r], w);
      }
    }
    dft<PS::R, DIR, T>(&v[s * PS::R]);
  }
}

// LDS tile of ROWS x COLS values for one exchange.  The layout is chosen per
// exchange kind, since each exchange writes and reads its tile between two
// barriers and owes nothing to the layout of the previous one.
//   XK_PLAIN  pencil tiles and the compact plane tiles: row stride COLS + 1.
//   XK_RR     row pass to row pass: one spare element after every 8 columns
//             (column c at c + c / 8) and a row stride from a per-width
//             table.  The first pass of a row transform writes column 8i + r
//             from lane i, a stride of 8 elements that lands many lanes in
//             one bank; padded, lane i writes element 9i + r.
//   XK_RC, XK_CR, XK_CC  exchanges with a column pass on either side: plain
//             rows (a column pass walks consecutive columns, which padding
//             every 8 would wrap into the banks of the first ones) with a
//             per-width row stride.
// Every element address stays an affine function of the lane, so the
// per-element offsets fold into instruction immediates.  The strides come
// from a model of every exchange instruction's lane addresses, served 128 or
// 256 bytes per cycle over banks of 4 bytes, for 8- and 16-byte elements; the
// largest stays within the padded tile, so the LDS footprint is unchanged.
enum XKind { XK_PLAIN = 0, XK_RR = 1, XK_RC = 2, XK_CR = 3, XK_CC = 4 };

constexpr int tile_stride(int cols, int kind) {
  switch (kind) {
    case XK_RR:
      return cols + cols / 8 + (cols == 128 ? 8 : cols == 72 ? 7 : cols == 48 ? 2 : 0);
    case XK_RC:
      return cols == 128 ? 136 : cols == 96 ? 104 : cols == 64 ? 72 : cols == 48 ? 56 : cols;
    case XK_CR:
      return cols == 128 ? 144 : cols == 96 ? 108 : cols == 72 ? 73 : cols == 64 ? 72 : cols == 48 ? 54
                                                                                 : cols == 24 ? 27 : cols + 1;
    case XK_CC:
      return cols;
    default:
      return cols + 1;
  }
}

template <int COLS, int KIND = XK_PLAIN> struct Tile {
  static_assert(KIND != XK_RR || COLS % 8 == 0, "padding every 8 columns");
  static constexpr int SL = tile_stride(COLS, KIND);
  __device__ static __forceinline__ int at(int row, int col) {
    if constexpr (KIND == XK_RR)
      return row * SL + col + (col >> 3);
    else
      return row * SL + col;
  }
  static constexpr int slots(int rows) { return rows * SL; }
};

// Exchange kind between pass A and pass B; PAD = false keeps XK_PLAIN.
template <class PA, class PB, bool PAD> constexpr int exchange_kind() {
  if constexpr (!PAD) return XK_PLAIN;
  else if constexpr (PA::ROW && PB::ROW) return XK_RR;
  else if constexpr (PA::ROW) return XK_RC;
  else if constexpr (PB::ROW) return XK_CR;
  else return XK_CC;
}

// Elements of LDS a plane tile of ROWS x COLS needs over all its exchanges.
template <int COLS, bool PAD> constexpr int plane_slots(int rows) {
  if constexpr (!PAD) {
    return Tile<COLS>::slots(rows);
  } else {
    int m = Tile<COLS, XK_RR>::slots(rows);
    m = Tile<COLS, XK_RC>::slots(rows) > m ? Tile<COLS, XK_RC>::slots(rows) : m;
    m = Tile<COLS, XK_CR>::slots(rows) > m ? Tile<COLS, XK_CR>::slots(rows) : m;
    m = Tile<COLS, XK_CC>::slots(rows) > m ? Tile<COLS, XK_CC>::slots(rows) : m;
    return m;
  }
}

// Move the outputs of pass A (in registers) to the inputs of pass B through
// an LDS tile of COLS columns.  SPLIT exchanges real and imaginary parts in
// two rounds so that an FP64 tile needs only 8 bytes of LDS per element.
template <class PA, class PB, int COLS, bool SPLIT, typename T, bool PAD = false>
__device__ __forceinline__ void exchange(cx<T>* v, void* smem, int t) {
  using TL = Tile<COLS, exchange_kind<PA, PB, PAD>()>;
  if constexpr (!SPLIT) {
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
    for_outputs<PA>(t, [&](int e, int row, int col) { buf[TL::at(row, col)] = v[e]; });
    __syncthreads();
    for_inputs<PB>(t, [&](int e, int row, int col) { v[e] = buf[TL::at(row, col)]; });
    __syncthreads();
  } else {
    T* buf = reinterpret_cast<T*>(smem);
    T tmp[PB::NV];
    for_outputs<PA>(t, [&](int e, int row, int col) { buf[TL::at(row, col)] = v[e].x; });
    __syncthreads();
    for_inputs<PB>(t, [&](int e, int row, int col) { tmp[e] = buf[TL::at(row, col)]; });
    __syncthreads();
    for_outputs<PA>(t, [&](int e, int row, int col) { buf[TL::at(row, col)] = v[e].y; });
    __syncthreads();
    for_inputs<PB>(t, [&](int e, int row, int col) { v[e] = mk<T>(tmp[e], buf[TL::at(row, col)]); });
    __syncthreads();
  }
}

}  // namespace fockx
