// pd_passes.hpp -- the HBM passes of one FCBM convolution chain on gfx950.
//
// Spectral data layout (complex T, x-spectrum index kx in [0, n1/2]):
//   SA  "row spectra"   [field][z < b3][kx < h1][y < P2]  (y contiguous, only
//                       body rows y < b2 are meaningful)
//   SB  "plane spectra" [field][z < b3][kx < h1][ky < n2] (3D only)
//   SC  "output planes" [field][z < b3][kx < h1][ky < n2] (3D only)
// Only body rows/planes are ever transformed or stored: the padding of the
// periodic box (Sec. 4.2.2) is known to be zero on the way in and is not
// needed on the way out, so each pass is pruned to the body extent.
//
// Passes (2D uses 1, 3, 5; 3D uses all five):
//   1 k_xfwd    real rows of the body -> generator -> r2c FFT along x (length
//               n1 via an n1/2 complex FFT) -> transposed store into SA
//   2 k_lines   contiguous complex FFT along y (3D forward: SA -> SB)
//   3 k_lmul    2D last axis: FFT along y, spectral multiply, inverse FFT
//   4 k_zcol    3D last axis: z columns (strided, coalesced across ky),
//               FFT, spectral multiply, inverse FFT, body planes only
//   5 k_xinv    transposed load from SA, c2r along x, epilogue per node
// The spectral multiply evaluates the kernel spectra from partial spectra
// ("taps") along the last axis:
//   M_c(k) = i^P_c * sum_{t=0}^{m} B_c[t](k_prefix) trig_c(2 pi k_last t / n_last)
// with trig = cos (component even in the last axis) or sin (odd).
#pragma once

#include "pd_ops.hpp"

namespace pdk {

struct Geo {
    int dim;
    int n1, n2, n3;     // FFT grid
    int b1, b2, b3;     // body box
    int h1, Nc, P2;     // n1/2+1, n1/2, row pitch of SA (>= b2)
    long nb;            // body nodes
    long saf;           // field stride of SA: b3*h1*P2
    long sbf;           // field stride of SB/SC: b3*h1*n2
};

// Block-wide deterministic FP64 reduction of NR values; thread 0 writes the
// block result to out[0..NR).
template <int NR>
__device__ __forceinline__ void block_reduce_store(double (&red)[NR], double* out, double* sm) {
    if constexpr (NR > 0) {
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            double x = red[r];
            for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
            red[r] = x;
        }
        __syncthreads();
        if (lane == 0)
            for (int r = 0; r < NR; ++r) sm[wid * NR + r] = red[r];
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int r = 0; r < NR; ++r) {
                double s = 0;
                for (int w = 0; w < nw; ++w) s += sm[w * NR + r];
                out[r] = s;
            }
        }
    }
}

// ----------------------------------------------------------------------------
// Pass 1: generator + r2c along x + transposed store.
// grid (ceil(b2/Lt), b3), block Tc*Lt, Tc = Nc/8; dynamic LDS Lt*(Nc+2) complex.
template <class T, class G>
__global__ void __launch_bounds__(1024) k_xfwd(Geo g, G gen, cx<T>* __restrict__ SA,
                                               const cx<T>* __restrict__ twb) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    constexpr int NF = G::NIN;
    const int Nc = g.Nc, Tc = Nc >> 3;
    const int nthr = blockDim.x;
    const int Lt = nthr / Tc;
    const int tid = threadIdx.x, j = tid % Tc, l = tid / Tc;
    const int z = blockIdx.y;
    const int y0 = blockIdx.x * Lt;
    const int y = y0 + l;
    const bool rowok = y < g.b2;
    const int pitch = Nc + 2;
    cx<T> v[NF][8];
    const long rbase = ((long)z * g.b2 + y) * g.b1;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int x0 = 2 * (j + Tc * q);
        T a[NF], b[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) { a[f] = T(0); b[f] = T(0); }
        if (rowok) {
            if (x0 < g.b1) gen.gen(rbase + x0, a);
            if (x0 + 1 < g.b1) gen.gen(rbase + x0 + 1, b);
        }
#pragma unroll
        for (int f = 0; f < NF; ++f) v[f][q] = {a[f], b[f]};
    }
    const cx<T>* twN = twb + Nc;
    const cx<T>* twn1 = twb + g.n1;
    cx<T>* row = lds + l * pitch;
    const int ll = tid % Lt, kk = tid / Lt, kstep = nthr / Lt;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        fft_line<-1>(v[f], j, Nc, twN, row, 1);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 8; ++q) row[j + Tc * q] = v[f][q];
        __syncthreads();
        cx<T> X[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int k = j + Tc * q;
            cx<T> A = row[k];
            cx<T> B = cconj(row[(Nc - k) & (Nc - 1)]);
            cx<T> E = cscale(A + B, T(0.5));
            cx<T> Dm = A - B;
            cx<T> O = {T(0.5) * Dm.i, T(-0.5) * Dm.r};
            X[q] = E + cmul(twn1[k], O);
        }
        cx<T> Xn = {T(0), T(0)};
        if (j == 0) {
            cx<T> A = row[0];
            Xn = {A.r - A.i, T(0)};
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 8; ++q) row[j + Tc * q] = X[q];
        if (j == 0) row[Nc] = Xn;
        __syncthreads();
        if (y0 + ll < g.b2) {
            cx<T>* dst = SA + f * g.saf + (long)z * g.h1 * g.P2 + y0 + ll;
            for (int kx = kk; kx < g.h1; kx += kstep) dst[(long)kx * g.P2] = lds[ll * pitch + kx];
        }
    }
}

// ----------------------------------------------------------------------------
// Pass 2: plain contiguous line FFTs (one field line per line slot).
// Line li reads in[li*in_pitch + p] for p < in_len (zero beyond) and writes
// out[li*out_pitch + p] for p < out_len.  block Lw*(N/8), LDS Lw*(N+1).
template <class T, int SIGN>
__global__ void __launch_bounds__(1024) k_lines(int N, long nlines, const cx<T>* __restrict__ in,
                                                long in_pitch, int in_len, cx<T>* __restrict__ out,
                                                long out_pitch, int out_len,
                                                const cx<T>* __restrict__ twb) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    const int Tn = N >> 3;
    const int Lw = blockDim.x / Tn;
    const int tid = threadIdx.x, j = tid % Tn, l = tid / Tn;
    const long li = (long)blockIdx.x * Lw + l;
    const bool ok = li < nlines;
    cx<T> v[8];
    const cx<T>* src = in + li * in_pitch;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int p = j + Tn * q;
        v[q] = (ok && p < in_len) ? src[p] : cx<T>{T(0), T(0)};
    }
    fft_line<SIGN>(v, j, N, twb + N, lds + l * (N + 1), 1);
    if (ok) {
        cx<T>* dst = out + li * out_pitch;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int p = j + Tn * q;
            if (p < out_len) dst[p] = v[q];
        }
    }
}

// Evaluate the kernel multipliers of components [C0, C0+NC) at last-axis
// wavenumber k from taps B[c*ntap + t] (already for this line) and apply.
template <class T, class M, int NIN, int NOUT>
__device__ __forceinline__ void spectral_mul(const M& mul, const T* __restrict__ B, int ntap,
                                             uint32_t oddmask, int k, int n_last,
                                             const cx<T>* __restrict__ twl, cx<T> (&vin)[NIN][8],
                                             cx<T> (&vout)[NOUT][8], int q) {
    T K[M::NC > 0 ? M::NC : 1];
#pragma unroll
    for (int c = 0; c < M::NC; ++c) K[c] = B[c * ntap];
    for (int t = 1; t < ntap; ++t) {
        cx<T> w = twl[(k * t) & (n_last - 1)];
        const T cs = w.r, sn = -w.i;
#pragma unroll
        for (int c = 0; c < M::NC; ++c)
            K[c] += B[c * ntap + t] * (((oddmask >> (M::C0 + c)) & 1u) ? sn : cs);
    }
    cx<T> a[NIN], o[NOUT];
#pragma unroll
    for (int f = 0; f < NIN; ++f) a[f] = vin[f][q];
    mul.mul(K, k, a, o);
#pragma unroll
    for (int f = 0; f < NOUT; ++f) vout[f][q] = o[f];
}

// ----------------------------------------------------------------------------
// Pass 3 (2D): lines along y for each kx: FFT, multiply, inverse FFT.
// In place on SA (a block owns whole kx lines of every field).
// block Lw*(n2/8), LDS Lw*(n2+1) complex.
template <class T, class M>
__global__ void __launch_bounds__(1024) k_lmul(Geo g, M mul, cx<T>* SA, const T* __restrict__ taps,
                                               int ntap, uint32_t oddmask,
                                               const cx<T>* __restrict__ twb) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    constexpr int NI = M::NIN, NO = M::NOUT;
    const int N = g.n2, Tn = N >> 3;
    const int Lw = blockDim.x / Tn;
    const int tid = threadIdx.x, j = tid % Tn, l = tid / Tn;
    const int kx = blockIdx.x * Lw + l;
    const bool ok = kx < g.h1;
    const int kxc = ok ? kx : 0;
    cx<T> vin[NI][8];
#pragma unroll
    for (int f = 0; f < NI; ++f) {
        const cx<T>* src = SA + f * g.saf + (long)kxc * g.P2;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int p = j + Tn * q;
            vin[f][q] = (ok && p < g.b2) ? src[p] : cx<T>{T(0), T(0)};
        }
    }
    const cx<T>* tw = twb + N;
    cx<T>* line = lds + l * (N + 1);
#pragma unroll
    for (int f = 0; f < NI; ++f) fft_line<-1>(vin[f], j, N, tw, line, 1);
    // taps of this kx for the components in use
    T Bt[(M::NC > 0 ? M::NC : 1) * 9];
    const int NP = g.h1;
    for (int c = 0; c < M::NC; ++c)
        for (int t = 0; t < ntap; ++t) Bt[c * ntap + t] = taps[((long)(M::C0 + c) * ntap + t) * NP + kxc];
    cx<T> vout[NO][8];
#pragma unroll
    for (int q = 0; q < 8; ++q) spectral_mul<T, M, NI, NO>(mul, Bt, ntap, oddmask, j + Tn * q, N, tw, vin, vout, q);
#pragma unroll
    for (int o = 0; o < NO; ++o) {
        fft_line<1>(vout[o], j, N, tw, line, 1);
        if (ok) {
            cx<T>* dst = SA + o * g.saf + (long)kx * g.P2;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int p = j + Tn * q;
                if (p < g.b2) dst[p] = vout[o][q];
            }
        }
    }
}

// ----------------------------------------------------------------------------
// Pass 4 (3D): z columns of a tile of Lc consecutive ky at fixed kx:
// FFT along z (body planes in), multiply, inverse FFT (body planes out).
// grid (n2/Lc, h1), block Lc*(n3/8), threads ky-fastest for coalescing.
// LDS: n3*Lc complex (point-major) + taps Lc*NC*ntap.
template <class T, class M>
__global__ void __launch_bounds__(1024) k_zcol(Geo g, M mul, const cx<T>* __restrict__ SB,
                                               cx<T>* __restrict__ SC, const T* __restrict__ taps,
                                               int ntap, uint32_t oddmask,
                                               const cx<T>* __restrict__ twb) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    constexpr int NI = M::NIN, NO = M::NOUT;
    const int N = g.n3, Tn = N >> 3;
    const int Lc = blockDim.x / Tn;
    const int tid = threadIdx.x, l = tid % Lc, j = tid / Lc;
    const int kx = blockIdx.y;
    const int ky = blockIdx.x * Lc + l;
    T* tl = reinterpret_cast<T*>(lds + (long)N * Lc);
    const long NP = (long)g.h1 * g.n2;
    for (int e = tid; e < Lc * M::NC * ntap; e += blockDim.x) {
        const int ll = e % Lc, ct = e / Lc;  // ct = c*ntap + t
        const int c = ct / ntap, t = ct % ntap;
        tl[ll * (M::NC * ntap) + ct] = taps[((long)(M::C0 + c) * ntap + t) * NP + (long)kx * g.n2 + blockIdx.x * Lc + ll];
    }
    const long plane = (long)g.h1 * g.n2;
    const long col = (long)kx * g.n2 + ky;
    cx<T> vin[NI][8];
#pragma unroll
    for (int f = 0; f < NI; ++f) {
        const cx<T>* src = SB + f * g.sbf + col;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int p = j + Tn * q;
            vin[f][q] = (p < g.b3) ? src[p * plane] : cx<T>{T(0), T(0)};
        }
    }
    const cx<T>* tw = twb + N;
#pragma unroll
    for (int f = 0; f < NI; ++f) fft_line<-1>(vin[f], j, N, tw, lds + l, Lc);
    const T* Bt = tl + l * (M::NC * ntap);
    cx<T> vout[NO][8];
#pragma unroll
    for (int q = 0; q < 8; ++q) spectral_mul<T, M, NI, NO>(mul, Bt, ntap, oddmask, j + Tn * q, N, tw, vin, vout, q);
#pragma unroll
    for (int o = 0; o < NO; ++o) {
        fft_line<1>(vout[o], j, N, tw, lds + l, Lc);
        cx<T>* dst = SC + o * g.sbf + col;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int p = j + Tn * q;
            if (p < g.b3) dst[p * plane] = vout[o][q];
        }
    }
}

// ----------------------------------------------------------------------------
// Pass 5: transposed load of body rows from SA, c2r along x, epilogue.
// grid (ceil(b2/Lt), b3), block Tc*Lt; LDS Lt*(Nc+2) complex + reduction.
// partials: per block NRED doubles at (blockIdx.y*gridDim.x + blockIdx.x)*NRED.
template <class T, class F>
__global__ void __launch_bounds__(1024) k_xinv(Geo g, F fin, const cx<T>* __restrict__ SA,
                                               double* __restrict__ partials,
                                               const cx<T>* __restrict__ twb) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    constexpr int NO = F::NOUT;
    const int Nc = g.Nc, Tc = Nc >> 3;
    const int nthr = blockDim.x;
    const int Lt = nthr / Tc;
    const int tid = threadIdx.x, j = tid % Tc, l = tid / Tc;
    const int z = blockIdx.y;
    const int y0 = blockIdx.x * Lt;
    const int y = y0 + l;
    const int pitch = Nc + 2;
    cx<T>* row = lds + l * pitch;
    const cx<T>* twN = twb + Nc;
    const cx<T>* twn1 = twb + g.n1;
    const int ll = tid % Lt, kk = tid / Lt, kstep = nthr / Lt;
    T val[NO][16];
#pragma unroll
    for (int o = 0; o < NO; ++o) {
        __syncthreads();
        {
            const bool okr = (y0 + ll) < g.b2;
            const cx<T>* src = SA + o * g.saf + (long)z * g.h1 * g.P2 + y0 + ll;
            for (int kx = kk; kx < g.h1; kx += kstep)
                lds[ll * pitch + kx] = okr ? src[(long)kx * g.P2] : cx<T>{T(0), T(0)};
        }
        __syncthreads();
        cx<T> v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int k = j + Tc * q;
            cx<T> A = row[k];
            cx<T> B = cconj(row[Nc - k]);
            cx<T> w = cconj(twn1[k]);
            cx<T> Dm = cmul(w, A - B);
            v[q] = (A + B) + cx<T>{-Dm.i, Dm.r};
        }
        fft_line<1>(v, j, Nc, twN, row, 1);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            val[o][2 * q] = v[q].r;
            val[o][2 * q + 1] = v[q].i;
        }
    }
    double red[F::NRED > 0 ? F::NRED : 1];
#pragma unroll
    for (int r = 0; r < (F::NRED > 0 ? F::NRED : 1); ++r) red[r] = 0.0;
    if (y < g.b2) {
        const long rbase = ((long)z * g.b2 + y) * g.b1;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int x = 2 * (j + Tc * q) + e;
                if (x < g.b1) {
                    T vv[NO];
#pragma unroll
                    for (int o = 0; o < NO; ++o) vv[o] = val[o][2 * q + e];
                    fin.fin(rbase + x, vv, red);
                }
            }
        }
    }
    if constexpr (F::NRED > 0) {
        __syncthreads();
        double* sm = reinterpret_cast<double*>(smem_raw);
        block_reduce_store<F::NRED>(red, partials + ((long)blockIdx.y * gridDim.x + blockIdx.x) * F::NRED, sm);
    }
}

// Deterministic final sum of per-block partials: out[r] = sum_b part[b*NR + r]
// (one block, fixed order tree).
__global__ void k_reduce_final(const double* __restrict__ part, long nblk, int NR, double* __restrict__ out);

}  // namespace pdk
