// pd_fft.hpp -- register/LDS FFT engine for gfx950 (wave64).
//
// One line of N = 2^p complex points (8 <= N <= 1024) is transformed by
// T = N/8 threads, each holding 8 points in registers: thread j holds the
// points j + T*q, q = 0..7, both on entry and on exit (natural order).  The
// transform is a Stockham auto-sort FFT (radix 8 stages plus at most one
// radix 2 or 4 stage); data moves between stages through a per-line LDS
// region, and the first and last stages work straight from registers, so a
// caller can load from HBM, transform, multiply point-wise and transform back
// without extra LDS traffic.  Twiddles come from a table of
// exp(-2 pi i e / N), e in [0, N), computed on the host in long double.
//
// Unnormalised transforms: SIGN = -1 computes X_k = sum_n x_n e^{-2 pi i nk/N}
// (the DFT of Eq. 54 with 0-based indices), SIGN = +1 the same sum with
// e^{+2 pi i nk/N} (Eq. 53 without the 1/N factor).
#pragma once

#include <hip/hip_runtime.h>

namespace pdk {

// LDS position of FFT point i: one padding slot after every 8 points, so the
// stride-8 and stride-64 access patterns of the Stockham stages spread over
// the LDS banks instead of piling onto a few.  A line of N points therefore
// occupies fft_lds_len(N) complex slots.
__host__ __device__ __forceinline__ int fft_pad(int i) { return i + (i >> 3); }
__host__ __device__ constexpr int fft_lds_len(int N) { return N + N / 8; }
// LDS slots of a staged twiddle table of length N (plain layout).
__host__ __device__ constexpr int tw_lds_len(int N) { return N; }

template <class T>
struct __align__(2 * sizeof(T)) cx {
    T r, i;
};

// LDS-typed view of a pointer into dynamic shared memory: index arithmetic
// on it stays 32-bit (a generic pointer would force 64-bit address math).
// The address space only exists in the device compilation pass; the host
// pass (which never runs this code) sees a plain pointer.
#if defined(__HIP_DEVICE_COMPILE__)
template <class T>
using lds_ptr = __attribute__((address_space(3))) T*;
#else
template <class T>
using lds_ptr = T*;
#endif
template <class T>
__device__ __forceinline__ lds_ptr<T> as_lds(T* p) { return (lds_ptr<T>)p; }
template <class T>
__device__ __forceinline__ lds_ptr<const T> as_lds(const T* p) { return (lds_ptr<const T>)p; }

template <class T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.r + b.r, a.i + b.i}; }
template <class T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.r - b.r, a.i - b.i}; }
template <class T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
template <class T>
__device__ __forceinline__ cx<T> cconj(cx<T> a) { return {a.r, -a.i}; }
template <class T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.r * s, a.i * s}; }
// a * (i^p) for p = 0..3
template <class T>
__device__ __forceinline__ cx<T> mul_ipow(cx<T> a, int p) {
    switch (p & 3) {
        case 0: return a;
        case 1: return {-a.i, a.r};
        case 2: return {-a.r, -a.i};
        default: return {a.i, -a.r};
    }
}

// a * (SIGN * i)
template <int SIGN, class T>
__device__ __forceinline__ cx<T> mul_si(cx<T> a) {
    if constexpr (SIGN < 0) return {a.i, -a.r};
    else return {-a.i, a.r};
}

template <int SIGN, class T>
__device__ __forceinline__ void dft2(cx<T>& a, cx<T>& b) {
    cx<T> t = a - b;
    a = a + b;
    b = t;
}

template <int SIGN, class T>
__device__ __forceinline__ void dft4(cx<T>& c0, cx<T>& c1, cx<T>& c2, cx<T>& c3) {
    cx<T> t0 = c0 + c2, t1 = c0 - c2, t2 = c1 + c3, t3 = mul_si<SIGN>(c1 - c3);
    c0 = t0 + t2;
    c2 = t0 - t2;
    c1 = t1 + t3;
    c3 = t1 - t3;
}

// 8-point DFT in place: radix-2 split into two 4-point DFTs.
template <int SIGN, class T>
__device__ __forceinline__ void dft8(cx<T>* x) {
    const T h = T(0.70710678118654752440084436210484904);
    cx<T> a0 = x[0] + x[4], a1 = x[1] + x[5], a2 = x[2] + x[6], a3 = x[3] + x[7];
    cx<T> b0 = x[0] - x[4], b1 = x[1] - x[5], b2 = x[2] - x[6], b3 = x[3] - x[7];
    // b_k *= e^{SIGN i pi k/4}
    const T s = T(SIGN);
    b1 = {h * (b1.r - s * b1.i), h * (b1.i + s * b1.r)};
    b2 = mul_si<SIGN>(b2);
    b3 = {-h * (b3.r + s * b3.i), h * (s * b3.r - b3.i)};
    dft4<SIGN>(a0, a1, a2, a3);
    dft4<SIGN>(b0, b1, b2, b3);
    x[0] = a0; x[2] = a1; x[4] = a2; x[6] = a3;
    x[1] = b0; x[3] = b1; x[5] = b2; x[7] = b3;
}

template <int SIGN, class T>
__device__ __forceinline__ cx<T> twiddle(lds_ptr<const cx<T>> tw, int e) {
    cx<T> w = tw[e];
    if constexpr (SIGN > 0) w.i = -w.i;
    return w;
}

// First Stockham stage (sub-transform size 1, so no twiddles) of radix R on
// the 8 register points of thread j, for lines of N >= 16 points (so it is
// never the last stage).  Butterfly b = j + T*s (s < 8/R) reads the points
// b + r*N/R, held in register q = s + r*(8/R), and writes its outputs to
// points b*R + r in LDS.
template <int R, int SIGN, class T>
__device__ __forceinline__ void fft_first(const cx<T> (&v)[8], int j, int lgT, lds_ptr<cx<T>> lds) {
    constexpr int S = 8 / R;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        cx<T> x[R];
#pragma unroll
        for (int r = 0; r < R; ++r) x[r] = v[s + r * S];
        if constexpr (R == 8) dft8<SIGN>(x);
        else if constexpr (R == 4) dft4<SIGN>(x[0], x[1], x[2], x[3]);
        else dft2<SIGN>(x[0], x[1]);
        const int base = (j + (s << lgT)) * R;
#pragma unroll
        for (int r = 0; r < R; ++r) lds[fft_pad(base + r)] = x[r];
    }
}

// Radix-8 Stockham stage with sub-transform size Ns = 2^lgNs: thread j
// (= butterfly j) reads points j + r*N/8 (register r), multiplies by the
// twiddles W_{8Ns}^{r k}, k = j mod Ns (table index r*k*N/(8Ns)), and
// writes point ((j >> lgNs) << (lgNs+3)) | k  +  r*Ns.  Only shifts, masks
// and adds for the index math.
template <int SIGN, class T>
__device__ __forceinline__ void fft_r8(cx<T> (&v)[8], int j, int lgN, int lgNs, lds_ptr<const cx<T>> tw,
                                       int lgtws, lds_ptr<cx<T>> lds, bool last, int twmul) {
    const int k = j & ((1 << lgNs) - 1);
    const int e1 = (k << (lgN - lgNs - 3 + lgtws)) * twmul;
    int e = e1;
#pragma unroll
    for (int r = 1; r < 8; ++r) {
        v[r] = cmul(v[r], twiddle<SIGN>(tw, e));
        e += e1;
    }
    dft8<SIGN>(v);
    if (!last) {
        const int base = ((j >> lgNs) << (lgNs + 3)) | k;
#pragma unroll
        for (int r = 0; r < 8; ++r) lds[fft_pad(base + (r << lgNs))] = v[r];
    }
}

// Full line transform of N = 2^lgN points (8 <= N <= 2048).  Every thread of
// the block must call this (it contains block-wide barriers), with the same
// N.  lds points at this thread's line (fft_lds_len(N) complex slots).  The
// twiddle exp(-2 pi i e/N) is tw[(e << lgtws) * twmul] (a table of a multiple
// length: 2^lgtws * twmul times N; the table normally sits in LDS, see
// stage_twiddles).
template <int SIGN, class T>
__device__ __forceinline__ void fft_line(cx<T> (&v)[8], int j, int lgN, const cx<T>* __restrict__ tw_g, int lgtws,
                                         cx<T>* lds_g, int twmul = 1) {
    lds_ptr<const cx<T>> tw = as_lds(tw_g);
    lds_ptr<cx<T>> lds = as_lds(lds_g);
    __syncthreads();  // the caller may still be reading this LDS region
    if (lgN == 3) {   // a single 8-point transform in registers
        dft8<SIGN>(v);
        return;
    }
    const int lgT = lgN - 3;
    const int nst = (lgN + 2) / 3;      // first stage + radix-8 stages
    const int r0 = lgN - 3 * (nst - 1);  // log2 of the first radix: 1, 2 or 3
    if (r0 == 3) fft_first<8, SIGN>(v, j, lgT, lds);
    else if (r0 == 2) fft_first<4, SIGN>(v, j, lgT, lds);
    else fft_first<2, SIGN>(v, j, lgT, lds);
    int lgNs = r0;
    for (int st = 1; st < nst; ++st) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = lds[fft_pad(j + (q << lgT))];
        __syncthreads();
        fft_r8<SIGN>(v, j, lgN, lgNs, tw, lgtws, lds, st == nst - 1, twmul);
        lgNs += 3;
    }
}

// Copy the length-N twiddle table (global, at twb + N) into LDS; the caller's
// first fft_line barrier orders it before any use.
template <class T>
__device__ __forceinline__ void stage_twiddles(cx<T>* dst, const cx<T>* __restrict__ twb, int N) {
    for (int e = threadIdx.x; e < N; e += blockDim.x) dst[e] = twb[N + e];
}
// The same for a table that starts at src.
template <class T>
__device__ __forceinline__ void stage_table(cx<T>* dst, const cx<T>* __restrict__ src, int N) {
    for (int e = threadIdx.x; e < N; e += blockDim.x) dst[e] = src[e];
}

// Mixed-radix line of Nc = R * M complex points (R = 3, 5 or 9; M = 2^lgM >=
// 8): one radix-R step and R power-of-two transforms of M points
// (Cooley-Tukey with n = n2 + M n1, k = k1 + R k2, n1, k1 < R; n2, k2 < M).
// The line's Nc/8 threads form R groups of M/8: thread t = s (M/8) + j works
// on sub-line s and holds the points j + (M/8) q, q < 8, of it.
//   forward  y_s[n2] = W^{s n2} sum_n1 x[n2 + M n1] W_R^{s n1}  (W = e^{-2 pi i/Nc},
//            W_R = W^M), then the M-point transform of y_s gives X[s + R k2],
//            k2 = j + (M/8) q;
//   inverse  the M-point inverse transform of X[s + R k2] over k2 gives z_s[n2],
//            z_s[n2] W^{-s n2} goes through LDS, and
//            x[n2 + M s] = sum_k1 (z_k1[n2] W^{-k1 n2}) W_R^{-k1 s}.
// Twiddles: W^e = tw[2e], tw the table of length n1 = 2 Nc in LDS (every
// index used is below n1); the M-point transforms take W_M^e = W^{R e} from
// the same table; the R factors W_R^{s n1} of a thread are read once.  lds
// points at the line (fft_lds_len(Nc) complex slots).  Every thread of the
// block calls these (block-wide barriers); the caller fences its own LDS
// uses before and after.  RC > 0 and LGM > 0 fix R and lgM at compile time.
template <int RC, int LGM, class T, class In>
__device__ __forceinline__ void fft_mixed_fwd(cx<T> (&v)[8], int t, int Rr, int lgMr, In in, const cx<T>* tw_g,
                                              cx<T>* lds_g) {
    const int R = RC > 0 ? RC : Rr, lgM = LGM > 0 ? LGM : lgMr;
    const int M = 1 << lgM, Tq = M >> 3;
    const int s = t >> (lgM - 3), j = t & (Tq - 1);
    lds_ptr<const cx<T>> tw = as_lds(tw_g);
    constexpr int RMAX = RC > 0 ? RC : 9;
    cx<T> wr[RMAX];
#pragma unroll
    for (int r = 0; r < RMAX; ++r)
        if (r < R) wr[r] = tw[(2 * M * ((s * r) % R))];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int n2 = j + Tq * q;
        cx<T> acc = in(n2);
#pragma unroll
        for (int r = 1; r < RMAX; ++r)
            if (r < R) acc = acc + cmul(in(n2 + M * r), wr[r]);
        v[q] = cmul(acc, tw[2 * s * n2]);
    }
    fft_line<-1>(v, j, lgM, tw_g, 1, lds_g + s * fft_lds_len(M), R);
}

template <int RC, int LGM, class T>
__device__ __forceinline__ void fft_mixed_inv(cx<T> (&v)[8], int t, int Rr, int lgMr, const cx<T>* tw_g,
                                              cx<T>* lds_g) {
    const int R = RC > 0 ? RC : Rr, lgM = LGM > 0 ? LGM : lgMr;
    const int M = 1 << lgM, Tq = M >> 3;
    const int s = t >> (lgM - 3), j = t & (Tq - 1);
    fft_line<1>(v, j, lgM, tw_g, 1, lds_g + s * fft_lds_len(M), R);
    lds_ptr<const cx<T>> tw = as_lds(tw_g);
    lds_ptr<cx<T>> z = as_lds(lds_g);
    constexpr int RMAX = RC > 0 ? RC : 9;
    cx<T> wr[RMAX];
#pragma unroll
    for (int r = 0; r < RMAX; ++r)
        if (r < R) wr[r] = cconj(tw[(2 * M * ((s * r) % R))]);
    // z_s at the sub-line's own slots (pitch fft_lds_len(M), so that the
    // groups of threads of different s meet different banks)
    const int zp = fft_lds_len(M);
    __syncthreads();   // every sub-line transform is done with its LDS
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int n2 = j + Tq * q;
        z[s * zp + n2] = cmul(v[q], cconj(tw[2 * s * n2]));
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int n2 = j + Tq * q;
        cx<T> acc = z[n2];
#pragma unroll
        for (int r = 1; r < RMAX; ++r)
            if (r < R) acc = acc + cmul(z[r * zp + n2], wr[r]);
        v[q] = acc;
    }
}

}  // namespace pdk
