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

template <class T>
struct __align__(2 * sizeof(T)) cx {
    T r, i;
};

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
__device__ __forceinline__ cx<T> twiddle(const cx<T>* __restrict__ tw, int e) {
    cx<T> w = tw[e];
    if constexpr (SIGN > 0) w.i = -w.i;
    return w;
}

// One Stockham stage of radix R on the 8 register points of thread j.
// Butterfly b = j + T*s (s < 8/R) reads the points b + r*N/R, which sit in
// register q = s + r*(8/R); its outputs go to (b/Ns)*Ns*R + (b%Ns) + r*Ns.
template <int R, int SIGN, class T>
__device__ __forceinline__ void fft_stage(cx<T> (&v)[8], int j, int Tn, int N, int Ns,
                                          const cx<T>* __restrict__ tw, cx<T>* lds, int ls,
                                          bool last) {
    constexpr int S = 8 / R;
    const int wstep = N / (Ns * R);
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int b = j + Tn * s;
        const int k = b % Ns;
        cx<T> x[R];
#pragma unroll
        for (int r = 0; r < R; ++r) x[r] = v[s + r * S];
        if (Ns > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) x[r] = cmul(x[r], twiddle<SIGN>(tw, (r * k * wstep) & (N - 1)));
        }
        if constexpr (R == 8) dft8<SIGN>(x);
        else if constexpr (R == 4) dft4<SIGN>(x[0], x[1], x[2], x[3]);
        else dft2<SIGN>(x[0], x[1]);
        if (last) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[s + r * S] = x[r];
        } else {
            const int base = (b / Ns) * Ns * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) lds[(base + r * Ns) * ls] = x[r];
        }
    }
}

// Full line transform.  Every thread of the block must call this (it
// contains block-wide barriers), with the same N.  lds points at this
// thread's line, ls is the LDS distance between consecutive points.
template <int SIGN, class T>
__device__ __forceinline__ void fft_line(cx<T> (&v)[8], int j, int N, const cx<T>* __restrict__ tw,
                                         cx<T>* lds, int ls) {
    const int Tn = N >> 3;
    int log2n = 31 - __clz(N);
    int n8 = log2n / 3;
    int rem = log2n - 3 * n8;
    int nst = n8 + (rem ? 1 : 0);
    int Ns = 1;
    __syncthreads();  // the caller may still be reading this LDS region
    for (int st = 0; st < nst; ++st) {
        const bool last = (st == nst - 1);
        const int R = (st < n8) ? 8 : (1 << rem);
        if (R == 8) fft_stage<8, SIGN>(v, j, Tn, N, Ns, tw, lds, ls, last);
        else if (R == 4) fft_stage<4, SIGN>(v, j, Tn, N, Ns, tw, lds, ls, last);
        else fft_stage<2, SIGN>(v, j, Tn, N, Ns, tw, lds, ls, last);
        Ns *= R;
        if (!last) {
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = lds[(j + Tn * q) * ls];
            __syncthreads();
        }
    }
}

}  // namespace pdk
