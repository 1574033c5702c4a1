// Workgroup-wide power-of-two FFT held in registers, exchanged through LDS.
//
// A workgroup of NT = B / R threads transforms B points; thread `tid` holds
// the R points with index tid + NT * m (m = 0..R-1) in registers, both before
// and after the transform.  Every array indexed by frequency (spectra,
// running sums, phase factors) can therefore stay in the registers of the
// thread that owns those frequencies for the whole long step.
//
// The passes follow the Stockham autosort formulation: pass s with radix r
// and span p (product of the earlier radices) reads x[i + q B / r] for
// butterfly i (q = 0..r-1), multiplies by w^(q k), k = i mod p,
// w = exp(SIGN 2 pi i / (p r)), takes an r-point DFT and writes
// y[(i - k) r + k + q p].  The first pass reads registers, the last pass
// writes registers (its output index set is again tid + NT m), the passes in
// between exchange through LDS.  Results come out in natural order.
//
// SIGN = +1 is the transform with kernel exp(+i omega t) (the paper's F),
// SIGN = -1 its unnormalised inverse.
#pragma once

#include "cx.hpp"

namespace mpa {

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }

// LDS slot of element j of a transform's exchange buffer: a permutation of
// j inside aligned groups, so that the lanes the LDS serves together (16
// lanes of 8-byte FP32 elements, 8 lanes of 16-byte FP64 elements, over 32
// banks of 4 bytes) meet distinct banks both in the contiguous reads and in
// the strided writes of the passes, for B = 512 .. 4096.  FP32:
// j ^ h(t), t = j >> 4, with h's bits (t0, t0 ^ t1, t1 ^ t2, t2): its low
// bits separate the stride-8, -4 and -2 writes of a radix-8, -4 or -2 first
// pass, its high bits the 64-, 32- and 16-element runs of the pass after it.
// FP64: j ^ ((j >> 3) & 7).  (A pad slot every 8 elements, the simpler
// layout, leaves a 2-way conflict in most FP32 accesses of 16 lanes.)
template <typename T>
__device__ __forceinline__ int lds_slot(int j) {
    if constexpr (sizeof(T) == 4) {
        const int t = j >> 4;
        const int h = (t & 1) | ((t ^ (t << 1)) & 6) | ((t << 1) & 8);
        return j ^ h;
    } else {
        return j ^ ((j >> 3) & 7);
    }
}

template <int B>
constexpr int lds_elems() { return B + B / 8; }

// ---- small DFTs in registers (output in natural order, in place) ----------

template <int SIGN, typename T>
__device__ __forceinline__ void dft2(cx<T>& a, cx<T>& b) {
    cx<T> t = a;
    a = t + b;
    b = t - b;
}

template <int SIGN, typename T>
__device__ __forceinline__ void dft4(cx<T>& x0, cx<T>& x1, cx<T>& x2, cx<T>& x3) {
    cx<T> t0 = x0 + x2, t1 = x0 - x2, t2 = x1 + x3, t3 = rot<SIGN>(x1 - x3);
    x0 = t0 + t2;
    x2 = t0 - t2;
    x1 = t1 + t3;
    x3 = t1 - t3;
}

// 8-point DFT as two 4-point DFTs of the even and odd samples:
// X_k = E_k + w^k O_k, X_{k+4} = E_k - w^k O_k, w = exp(SIGN 2 pi i / 8).
template <int SIGN, typename T>
__device__ __forceinline__ void dft8(cx<T> (&x)[8]) {
    const T h = T(0.70710678118654752440084436210484903928);
    dft4<SIGN>(x[0], x[2], x[4], x[6]);
    dft4<SIGN>(x[1], x[3], x[5], x[7]);
    // twiddle the odd half: O_1 *= w, O_2 *= w^2 = SIGN i, O_3 *= w^3
    // w O_1 = h (O_1 + SIGN i O_1) and w^3 O_3 = h (-O_3 + SIGN i O_3): the sums
    // are exact up to one rounding, the factor h is applied inside an
    // explicit fused multiply-add with E_k
    cx<T> o1 = x[3], o2 = x[5], o3 = x[7];
    const T s = T(SIGN);
    const cx<T> t1 = {o1.re - s * o1.im, o1.im + s * o1.re};
    const cx<T> t3 = {-o3.re - s * o3.im, -o3.im + s * o3.re};
    o2 = rot<SIGN>(o2);
    cx<T> e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6], o0 = x[1];
    x[0] = e0 + o0;
    x[4] = e0 - o0;
    x[1] = {fma(t1.re, h, e1.re), fma(t1.im, h, e1.im)};
    x[5] = {fma(-t1.re, h, e1.re), fma(-t1.im, h, e1.im)};
    x[2] = e2 + o2;
    x[6] = e2 - o2;
    x[3] = {fma(t3.re, h, e3.re), fma(t3.im, h, e3.im)};
    x[7] = {fma(-t3.re, h, e3.re), fma(-t3.im, h, e3.im)};
}

template <int SIGN, int r, typename T>
__device__ __forceinline__ void dft(cx<T> (&x)[r]) {
    if constexpr (r == 2) {
        dft2<SIGN>(x[0], x[1]);
    } else if constexpr (r == 4) {
        dft4<SIGN>(x[0], x[1], x[2], x[3]);
    } else {
        static_assert(r == 8, "radix");
        dft8<SIGN>(x);
    }
}

// ---- one Stockham pass ------------------------------------------------------

template <typename T, int B, int R, int r, int p, int SIGN, bool FROM_LDS, bool TO_LDS, bool COLD>
__device__ __forceinline__ void fft_pass(cx<T> (&v)[R], cx<T>* lds,
                                         const cx<T>* __restrict__ tw, int tid) {
    constexpr int NT = B / R;
    constexpr int NB = R / r;   // butterflies per thread in this pass
    if constexpr (FROM_LDS) {
        __syncthreads();        // the previous pass's writes are visible
#pragma unroll
        for (int m = 0; m < R; ++m) v[m] = lds[lds_slot<T>(tid + NT * m)];
        __syncthreads();        // every read done before this pass overwrites
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int i = tid + u * NT;
        int k = i & (p - 1);
        if constexpr (COLD) asm volatile("" : "+v"(k));   // twiddles loaded here, not kept live
        cx<T> x[r];
#pragma unroll
        for (int q = 0; q < r; ++q) x[q] = v[u + q * NB];
        if constexpr (p > 1) {
            constexpr int stride = B / (p * r);
#pragma unroll
            for (int q = 1; q < r; ++q) {
                cx<T> w = tw[q * k * stride];   // exp(+2 pi i q k / (p r))
                if constexpr (SIGN < 0) w.im = -w.im;
                x[q] = cmul(x[q], w);
            }
        }
        dft<SIGN, r>(x);
        if constexpr (TO_LDS) {
            const int base = (i - k) * r + k;
#pragma unroll
            for (int q = 0; q < r; ++q) lds[lds_slot<T>(base + q * p)] = x[q];
        } else {
#pragma unroll
            for (int q = 0; q < r; ++q) v[u + q * NB] = x[q];
        }
    }
}

// Radix of the pass whose span is P: the first pass takes the remainder
// 2^(log2 B mod 3) when B is not a power of 8, every other pass is radix 8.
template <int B, int P>
constexpr int pass_radix() {
    if constexpr (P == 1) {
        constexpr int rem = ilog2(B) % 3;
        return rem == 0 ? 8 : (1 << rem);
    } else {
        return 8;
    }
}

template <typename T, int B, int R, int SIGN, int P, bool COLD>
__device__ __forceinline__ void fft_from(cx<T> (&v)[R], cx<T>* lds,
                                         const cx<T>* __restrict__ tw, int tid) {
    constexpr int r = pass_radix<B, P>();
    constexpr bool first = (P == 1);
    constexpr bool last = (P * r == B);
    static_assert(R % r == 0, "points per thread must be a multiple of every radix");
    fft_pass<T, B, R, r, P, SIGN, !first, !last, COLD>(v, lds, tw, tid);
    if constexpr (!last) fft_from<T, B, R, SIGN, P * r, COLD>(v, lds, tw, tid);
}

// ---- double-buffered variant ---------------------------------------------------
// Passes alternate between two LDS buffers: pass s writes buf[s % 2] and pass
// s + 1 reads it after one barrier.  The barrier after the reads is not
// needed, since the next write goes to the other buffer, whose last readers
// passed the barrier before this read.  A call ends having read
// buf[(E - 1) % 2] (E exchanges); the caller's next call must start writing
// the other buffer, so for odd E the two pointers are swapped on return.
template <typename T, int B, int R, int r, int p, int SIGN, bool FROM_LDS, bool TO_LDS, bool COLD>
__device__ __forceinline__ void fft_pass_db(cx<T> (&v)[R], const cx<T>* lds_in, cx<T>* lds_out,
                                            const cx<T>* __restrict__ tw, int tid) {
    constexpr int NT = B / R;
    constexpr int NB = R / r;
    if constexpr (FROM_LDS) {
        __syncthreads();        // the previous pass's writes are visible
#pragma unroll
        for (int m = 0; m < R; ++m) v[m] = lds_in[lds_slot<T>(tid + NT * m)];
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int i = tid + u * NT;
        int k = i & (p - 1);
        if constexpr (COLD) asm volatile("" : "+v"(k));   // twiddles loaded here, not kept live
        cx<T> x[r];
#pragma unroll
        for (int q = 0; q < r; ++q) x[q] = v[u + q * NB];
        if constexpr (p > 1) {
            constexpr int stride = B / (p * r);
#pragma unroll
            for (int q = 1; q < r; ++q) {
                cx<T> w = tw[q * k * stride];
                if constexpr (SIGN < 0) w.im = -w.im;
                x[q] = cmul(x[q], w);
            }
        }
        dft<SIGN, r>(x);
        if constexpr (TO_LDS) {
            const int base = (i - k) * r + k;
#pragma unroll
            for (int q = 0; q < r; ++q) lds_out[lds_slot<T>(base + q * p)] = x[q];
        } else {
#pragma unroll
            for (int q = 0; q < r; ++q) v[u + q * NB] = x[q];
        }
    }
}

template <typename T, int B, int R, int SIGN, int P, int S, bool COLD>
__device__ __forceinline__ void fft_from_db(cx<T> (&v)[R], cx<T>* buf0, cx<T>* buf1,
                                            const cx<T>* __restrict__ tw, int tid) {
    constexpr int r = pass_radix<B, P>();
    constexpr bool first = (P == 1);
    constexpr bool last = (P * r == B);
    // pass S reads buf[(S - 1) % 2] and writes buf[S % 2]
    cx<T>* in = (S % 2) ? buf0 : buf1;
    cx<T>* out = (S % 2) ? buf1 : buf0;
    fft_pass_db<T, B, R, r, P, SIGN, !first, !last, COLD>(v, in, out, tw, tid);
    if constexpr (!last) fft_from_db<T, B, R, SIGN, P * r, S + 1, COLD>(v, buf0, buf1, tw, tid);
}

template <int B, int P>
constexpr int exchanges() {
    constexpr int r = pass_radix<B, P>();
    if constexpr (P * r == B) return 0;
    else return 1 + exchanges<B, P * r>();
}

// B-point transform through two LDS buffers (each lds_elems<B>() elements);
// see fft_pass_db.  Every LDS access made before the call must have passed
// a barrier if it touched either buffer.  COLD as for block_fft.
template <typename T, int B, int R, int SIGN, bool COLD = false>
__device__ __forceinline__ void block_fft_db(cx<T> (&v)[R], cx<T>*& buf0, cx<T>*& buf1,
                                             const cx<T>* __restrict__ tw, int tid) {
    static_assert((B & (B - 1)) == 0 && B >= 64, "power-of-two block");
    fft_from_db<T, B, R, SIGN, 1, 0, COLD>(v, buf0, buf1, tw, tid);
    if constexpr (exchanges<B, 1>() % 2 == 1) {
        cx<T>* t = buf0;
        buf0 = buf1;
        buf1 = t;
    }
}

// ---- variant with the twiddles formed from one load per pass ------------------
// For transforms outside the node loop (the FP64 carry transforms).  Passes
// after the first are radix 8 with one butterfly per thread, which needs
// w^k, w^{2k}, ..., w^{7k} (w = exp(2 pi i / (8 p))): each pass loads w^k
// alone and forms the other six by complex products (w^2 = w w, w^3 = w^2 w,
// w^4 = w^2 w^2, w^5 = w^4 w, w^6 = w^4 w^2, w^7 = w^4 w^3; at most four
// roundings deep, a few units in the last place): seven table loads per
// pass, gathered through the vector memory path, cost more than the six
// products.  TW_AHEAD: the twiddles of every pass are formed when the call
// begins (their latency paid once); TW_PASS: at the start of each pass
// (fewer registers); either way they do not stay in registers after the
// call, and the arithmetic is the same.  TW_TABLE: read from a table in LDS
// (fill_twiddle_table), the B-point table's own values, as block_fft uses
// them, for transforms inside a loop whose registers cannot hold them.
// DBUF selects the exchange of block_fft_db (two buffers) or of block_fft
// (one).
enum TwiddleSource { TW_AHEAD = 0, TW_PASS = 1, TW_TABLE = 2 };

constexpr int first_radix(int B) { return ilog2(B) % 3 == 0 ? 8 : (1 << (ilog2(B) % 3)); }

constexpr int n_passes(int B) {
    int n = 0;
    for (int p = 1; p < B; p *= (n == 0 ? first_radix(B) : 8), ++n) {
    }
    return n;
}

// span of pass s (s = 0: the first)
constexpr int pass_span(int B, int s) { return s == 0 ? 1 : first_radix(B) * (1 << (3 * (s - 1))); }

// w^{q k}, q = 1..7, of pass S (S >= 1) for this thread
template <typename T, int B, int S>
__device__ __forceinline__ void pass_twiddles(cx<T> (&w)[7], const cx<T>* __restrict__ tw, int tid) {
    constexpr int p = pass_span(B, S);
    constexpr int stride = B / (p * 8);
    const int k = tid & (p - 1);
    const cx<T> w1 = tw[k * stride];
    const cx<T> w2 = cmul(w1, w1);
    const cx<T> w3 = cmul(w2, w1);
    const cx<T> w4 = cmul(w2, w2);
    w[0] = w1;
    w[1] = w2;
    w[2] = w3;
    w[3] = w4;
    w[4] = cmul(w4, w1);
    w[5] = cmul(w4, w2);
    w[6] = cmul(w4, w3);
}

// LDS twiddle table of the radix-8 passes: pass s >= 1 (span p) holds
// w^{q k} = tw[q k B / (8 p)] for q = 1..7, k < p at tl_offset(B, s) +
// (q - 1) p + k, so that the lanes of a pass, whose k are consecutive, read
// consecutive entries.
constexpr int tl_offset(int B, int s) {
    int o = 0;
    for (int t = 1; t < s; ++t) o += 7 * pass_span(B, t);
    return o;
}

constexpr int tl_elems(int B) { return tl_offset(B, n_passes(B)); }

// Fills the table from the B-point table `tw`, `nthreads` threads striding
// over it; the caller puts a barrier between this and the first transform.
template <typename T, int B>
__device__ __forceinline__ void fill_twiddle_table(cx<T>* tl, const cx<T>* __restrict__ tw, int tid, int nthreads) {
    constexpr int NP = n_passes(B);
    for (int e = tid; e < tl_elems(B); e += nthreads) {
        int s = 1;
        while (s + 1 < NP && e >= tl_offset(B, s + 1)) ++s;
        const int p = pass_span(B, s);
        const int r = e - tl_offset(B, s);
        const int q = r / p + 1, k = r - (q - 1) * p;
        tl[e] = tw[q * k * (B / (8 * p))];
    }
}

template <typename T, int B, int S, int NP>
__device__ __forceinline__ void all_twiddles(cx<T> (&w)[NP - 1][7], const cx<T>* __restrict__ tw, int tid) {
    if constexpr (S < NP) {
        pass_twiddles<T, B, S>(w[S - 1], tw, tid);
        all_twiddles<T, B, S + 1, NP>(w, tw, tid);
    }
}

template <typename T, int B, int R, int SIGN, int S, int NP, bool DBUF, int TWS>
__device__ __forceinline__ void passes_warm(cx<T> (&v)[R], cx<T>* buf0, cx<T>* buf1, const cx<T> (&wall)[NP - 1][7],
                                            const cx<T>* __restrict__ tw, const cx<T>* tl, int tid) {
    constexpr int NT = B / R;
    constexpr int p = pass_span(B, S);
    constexpr int r = S == 0 ? first_radix(B) : 8;
    constexpr int NB = R / r;
    constexpr bool first = (S == 0), last = (S == NP - 1);
    // exchange buffers: alternating (DBUF, pass S reads buf[(S - 1) % 2] and
    // writes buf[S % 2]) or one
    cx<T>* in = DBUF ? ((S % 2) ? buf0 : buf1) : buf0;
    cx<T>* out = DBUF ? ((S % 2) ? buf1 : buf0) : buf0;
    if constexpr (!first) {
        __syncthreads();
#pragma unroll
        for (int m = 0; m < R; ++m) v[m] = in[lds_slot<T>(tid + NT * m)];
        if constexpr (!DBUF) __syncthreads();
    }
    cx<T> wp[7];
    if constexpr (!first) {
        if constexpr (TWS == TW_AHEAD) {
#pragma unroll
            for (int q = 0; q < 7; ++q) wp[q] = wall[S - 1][q];
        } else if constexpr (TWS == TW_PASS) {
            int t = tid;
            asm volatile("" : "+v"(t));      // formed here, not earlier
            pass_twiddles<T, B, S>(wp, tw, t);
        } else {
            int k = tid & (p - 1);
            asm volatile("" : "+v"(k));      // read here, not hoisted out of the caller's loops
#pragma unroll
            for (int q = 0; q < 7; ++q) wp[q] = tl[tl_offset(B, S) + q * p + k];
        }
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int i = tid + u * NT;
        const int k = i & (p - 1);
        cx<T> x[r];
#pragma unroll
        for (int q = 0; q < r; ++q) x[q] = v[u + q * NB];
        if constexpr (!first) {
#pragma unroll
            for (int q = 1; q < r; ++q) {
                cx<T> t = wp[q - 1];
                if constexpr (SIGN < 0) t.im = -t.im;
                x[q] = cmul(x[q], t);
            }
        }
        dft<SIGN, r>(x);
        if constexpr (!last) {
            const int base = (i - k) * r + k;
#pragma unroll
            for (int q = 0; q < r; ++q) out[lds_slot<T>(base + q * p)] = x[q];
        } else {
#pragma unroll
            for (int q = 0; q < r; ++q) v[u + q * NB] = x[q];
        }
    }
    if constexpr (!last) passes_warm<T, B, R, SIGN, S + 1, NP, DBUF, TWS>(v, buf0, buf1, wall, tw, tl, tid);
}

// B-point transform as block_fft (DBUF = false: buf1 unused) or block_fft_db
// (DBUF: buf0 and buf1 swapped on return when the exchange count is odd),
// with the twiddles from the source TWS (above; `tl` for TW_TABLE).
template <typename T, int B, int R, int SIGN, bool DBUF, int TWS>
__device__ __forceinline__ void block_fft_warm(cx<T> (&v)[R], cx<T>*& buf0, cx<T>*& buf1,
                                               const cx<T>* __restrict__ tw, int tid, const cx<T>* tl = nullptr) {
    static_assert((B & (B - 1)) == 0 && B >= 64 && R == 8, "power-of-two block, 8 points per thread");
    constexpr int NP = n_passes(B);
    static_assert(NP >= 2, "at least two passes");
    cx<T> w[NP - 1][7];
    if constexpr (TWS == TW_AHEAD) {
        int t = tid;
        asm volatile("" : "+v"(t));      // formed inside this call
        all_twiddles<T, B, 1, NP>(w, tw, t);
    }
    passes_warm<T, B, R, SIGN, 0, NP, DBUF, TWS>(v, buf0, buf1, w, tw, tl, tid);
    if constexpr (DBUF && (NP - 1) % 2 == 1) {
        cx<T>* s = buf0;
        buf0 = buf1;
        buf1 = s;
    }
}

// B-point transform of the workgroup's registers (see the file comment).
// `tw` holds exp(+2 pi i j / B), j = 0..B-1.  Must be called by every
// thread of the workgroup (it contains barriers).  COLD: the twiddle index
// is hidden from the optimiser, so the twiddles are loaded inside each pass
// instead of being kept in registers across the caller's code; for
// transforms outside the hot loop, whose twiddles would otherwise hold
// registers for the whole kernel.
template <typename T, int B, int R, int SIGN, bool COLD = false>
__device__ __forceinline__ void block_fft(cx<T> (&v)[R], cx<T>* lds,
                                          const cx<T>* __restrict__ tw, int tid) {
    static_assert((B & (B - 1)) == 0 && B >= 64, "power-of-two block");
    fft_from<T, B, R, SIGN, 1, COLD>(v, lds, tw, tid);
}

}  // namespace mpa
