// pd_passes.hpp -- the HBM passes of one FCBM convolution chain on gfx950.
//
// Spectral data layout (complex T, x-spectrum index kx in [0, n1/2]):
//   SA  "row spectra"   [field][z < b3][kx < h1][y < P2]  (y contiguous, only
//                       body rows y < b2 are meaningful)
//   SB  "column spectra" [field][kx < h1][ky < n2][z < Pz] (3D only, z
//                       contiguous, only body planes z < b3 are meaningful)
// Only body rows/planes are ever transformed or stored: the padding of the
// periodic box (Sec. 4.2.2) is known to be zero on the way in and is not
// needed on the way out, so each pass is pruned to the body extent.
//
// Passes (2D: xfwd, lastmul, xinv; 3D: xfwd, ytf, lastmul, yti, xinv):
//   k_xfwd     real rows of the body -> generator -> r2c FFT along x (length
//              n1 via an n1/2 complex FFT) -> transposed store into SA
//   k_ytf      3D: FFT along y of SA rows, transposed store into SB
//   k_lastmul  contiguous lines along the last axis: FFT, spectral multiply,
//              inverse FFT, body points only (SA in 2D, SB in 3D, in place)
//   k_yti      3D: transposed load from SB, inverse FFT along y into SA
//   k_xinv     transposed load from SA, c2r along x, epilogue per node
// Every pass reads and writes contiguous runs: the two transposes sit in
// the x and y passes, so the multiply pass works on contiguous lines.
// The spectral multiply evaluates the kernel spectra from partial spectra
// ("taps") along the last axis:
//   M_c(k) = i^P_c * sum_{t=0}^{m} B_c[t](k_prefix) trig_c(2 pi k_last t / n_last)
// with trig = cos (component even in the last axis) or sin (odd).
#pragma once

#include <type_traits>

#include "pd_ops.hpp"

namespace pdk {

// LDS pitch (complex slots) of a row holding an Nc-point FFT line plus the
// Nyquist value; odd, so column-wise (transposed) accesses are conflict-free.
__host__ __device__ constexpr int row_pitch(int Nc) { return (fft_lds_len(Nc) + 2) | 1; }
// LDS pitch of an N-point line used by the y and last-axis passes.
__host__ __device__ constexpr int line_pitch(int N) { return (fft_lds_len(N) + 1) | 1; }

// Rows per block of the x passes: 16 in FP32 and 8 in FP64 (runs of 128 B in
// the transposed spectra accesses).
template <class T>
__host__ __device__ constexpr int xrows() { return sizeof(T) == 4 ? 16 : 8; }
// Rows per block of the mixed-radix x passes: 8, which ran the 256^3 step on
// 384- and 320-point x grids faster than 16 or 4 rows.
template <class T>
__host__ __device__ constexpr int xrows_mixed() { return 8; }

// Body nodes whose loads the x passes issue together (see k_xfwd): four,
// and two in the FP64 c2r pass (the epilogues' loads of four FP64 nodes do
// not fit in the registers of two waves per SIMD).
template <class T>
__host__ __device__ constexpr int node_group() { return sizeof(T) == 4 ? 4 : 2; }

// Node flags (body | interior << 1) of node i for a generator or epilogue:
// from its node context where it has one.
template <class G, class = void>
struct has_ctx : std::false_type {};
template <class G>
struct has_ctx<G, std::void_t<decltype(std::declval<G>().c.chiB)>> : std::true_type {};
template <class G>
__device__ __forceinline__ uint8_t node_flags(const G& g, Nd i) {
    if constexpr (has_ctx<G>::value) return ldf(g.c.chiB, i);
    else return g.flags(i);
}

struct Geo {
    int dim;
    int n1, n2, n3;     // FFT grid
    int b1, b2, b3;     // body box
    int h1, Nc, P2;     // n1/2+1, n1/2, row pitch of SA (>= b2)
    int rad, lgM;       // Nc = rad * 2^lgM: rad = 1 (power of two) or 3, 5, 9 (mixed radix)
    int twn1;           // offset (complex entries) of the length-n1 table in the twiddle buffer
    long nb;            // body nodes
    long saf;           // field stride of SA: b3*h1*P2
    long sbf;           // b3*h1*n2 (spectral points of the body planes)
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

// Line length of the x passes: LG > 0 fixes Nc = 2^LG at compile time, LG = 0
// takes a power of two from g, LG = -1 the mixed-radix Nc = rad 2^lgM of g,
// and LG = mix_lg(R, lgM) < -1 fixes a mixed-radix Nc = R 2^lgM at compile
// time.
__host__ __device__ constexpr int mix_lg(int R, int lgM) { return -(16 * R + lgM); }
template <int LG>
__host__ __device__ constexpr int mix_R() { return LG < -1 ? (-LG) / 16 : 0; }
template <int LG>
__host__ __device__ constexpr int mix_lgM() { return LG < -1 ? (-LG) % 16 : 0; }
template <int LG>
__device__ __forceinline__ int x_len(const Geo& g) {
    if constexpr (LG > 0) return 1 << LG;
    else if constexpr (LG < -1) return mix_R<LG>() << mix_lgM<LG>();
    else return g.Nc;
}
template <int LG>
__device__ __forceinline__ int x_lg(const Geo& g) {
    if constexpr (LG > 0) return LG;
    else if constexpr (LG < -1) return mix_lgM<LG>();
    else if constexpr (LG == 0) return 31 - __clz(g.Nc);
    else return g.lgM;
}
// Body-node slots per thread of the x passes (the block's run of Lt rows of
// b1 nodes over its Lt Nc / 8 threads): 8 for the compile-time powers of two
// (b1 <= Nc), 11, 13, 15 for the compile-time mixed lengths of a 256-node
// body (b1 <= x_rn Nc / 8), 16 otherwise (b1 < 2 Nc).
template <int LG>
__host__ __device__ constexpr int x_rn() {
    if constexpr (LG > 0) return 8;
    else if constexpr (LG < -1) return mix_R<LG>() == 3 ? 11 : (mix_R<LG>() == 5 ? 13 : 15);
    else return 16;
}
// Rows per block an x-pass epilogue asks for on the power-of-two lengths
// (F::XROWS; 0: xrows).
template <class F, class = void>
struct fin_xrows : std::integral_constant<int, 0> {};
template <class F>
struct fin_xrows<F, std::void_t<decltype(F::XROWS)>> : std::integral_constant<int, F::XROWS> {};

// Threads of an x-pass block: fixed for the compile-time lengths (R rows, or
// xrows, of Nc / 8 threads), else the launch's block size.
template <class T, int LG, int R = 0>
__host__ __device__ constexpr int x_block_fixed() {
    if constexpr (LG > 0) return ((1 << LG) / 8) * (R > 0 ? R : xrows<T>());
    else if constexpr (LG < -1) return ((mix_R<LG>() << mix_lgM<LG>()) / 8) * xrows_mixed<T>();
    else return 0;
}

// r2c along x of NF real fields held in the flat node mapping (thread tid
// holds nodes tid + nthr r of the block's run, r < RN) and transposed store
// into SA (field f at SA + f*saf).  The twiddles of length n1 must be staged
// in LDS after the Lt row buffers; every LDS use is fenced here.
template <class T, int NF, int RN, int LG>
__device__ __forceinline__ void r2c_store(const Geo& g, const T (&gv)[NF][RN], cx<T>* __restrict__ SA, cx<T>* lds,
                                          int nthr, int nval, int z, int y0) {
    const int Nc = x_len<LG>(g), lgNc = x_lg<LG>(g), Tc = Nc >> 3, Lt = nthr / Tc;
    const int tid = threadIdx.x, j = tid % Tc, l = tid / Tc;
    const bool rowok = y0 + l < g.b2;
    const int pitch = row_pitch(Nc);
    cx<T>* twn1 = lds + Lt * pitch;
    cx<T>* row = lds + l * pitch;
    lds_ptr<cx<T>> rowv = as_lds(row);
    lds_ptr<cx<T>> ldsv = as_lds(lds);
    lds_ptr<const cx<T>> twv = as_lds(twn1);
    lds_ptr<T> flat = as_lds(reinterpret_cast<T*>(lds));
    const int ll = tid % Lt, kk = tid / Lt;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        __syncthreads();  // the row buffers are free again
#pragma unroll
        for (int r = 0; r < RN; ++r) {
            const int e = tid + nthr * r;
            if (e < nval) flat[e] = gv[f][r];
        }
        __syncthreads();
        cx<T> v[8];
        // packed pair (2n, 2n + 1) of the row's real samples
        auto pair = [&](int n) -> cx<T> {
            const int x0 = 2 * n;
            const T a = (rowok && x0 < g.b1) ? flat[l * g.b1 + x0] : T(0);
            const T b = (rowok && x0 + 1 < g.b1) ? flat[l * g.b1 + x0 + 1] : T(0);
            return cx<T>{a, b};
        };
        if constexpr (LG >= 0) {
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = pair(j + Tc * q);
            fft_line<-1>(v, j, lgNc, twn1, 1, row);
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 8; ++q) rowv[j + Tc * q] = v[q];
        } else {
            fft_mixed_fwd<mix_R<LG>(), mix_lgM<LG>(), T>(v, j, g.rad, lgNc, pair, twn1, row);
            __syncthreads();
            const int Tq = 1 << (lgNc - 3), s = j >> (lgNc - 3), jj = j & (Tq - 1);
            const int R = LG < -1 ? mix_R<LG>() : g.rad;
#pragma unroll
            for (int q = 0; q < 8; ++q) rowv[s + R * (jj + Tq * q)] = v[q];
        }
        __syncthreads();
        cx<T> X[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int k = j + Tc * q;
            cx<T> A = rowv[k];
            cx<T> B = cconj(rowv[k ? Nc - k : 0]);
            cx<T> E = cscale(A + B, T(0.5));
            cx<T> Dm = A - B;
            cx<T> O = {T(0.5) * Dm.i, T(-0.5) * Dm.r};
            X[q] = E + cmul(twv[k], O);
        }
        cx<T> Xn = {T(0), T(0)};
        if (j == 0) {
            cx<T> A = rowv[0];
            Xn = {A.r - A.i, T(0)};
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 8; ++q) rowv[j + Tc * q] = X[q];
        if (j == 0) rowv[Nc] = Xn;
        __syncthreads();
        // kk < Tc: the columns kk + Tc*i (i < 8) cover [0, Nc); kk == 0 adds Nyquist
        if (y0 + ll < g.b2) {
            cx<T>* dst = SA + f * g.saf + (long)z * g.h1 * g.P2 + y0 + ll;
#pragma unroll
            for (int i = 0; i < 8; ++i) dst[(long)(kk + Tc * i) * g.P2] = ldsv[ll * pitch + kk + Tc * i];
            if (kk == 0) dst[(long)Nc * g.P2] = ldsv[ll * pitch + Nc];
        }
    }
}


// ----------------------------------------------------------------------------
// Pass 1: generator + r2c along x + transposed store.
// grid (ceil(b2/Lt), b3), block Tc*Lt, Tc = Nc/8; dynamic LDS Lt*(Nc+2) complex.
// LG > 0 fixes Nc = 2^LG at compile time (the runtime g.Nc must match).
template <class T, class G, int LG>
__global__ void __launch_bounds__(512) k_xfwd(Geo g, G gen, cx<T>* __restrict__ SA,
                                               const cx<T>* __restrict__ twb) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    constexpr int NF = G::NIN, NG = 4;
    const int Nc = x_len<LG>(g), Tc = Nc >> 3;
    const int nthr = x_block_fixed<T, LG>() > 0 ? x_block_fixed<T, LG>() : (int)blockDim.x;
    const int Lt = nthr / Tc;
    const int tid = threadIdx.x;
    const int z = blockIdx.y;
    const int y0 = blockIdx.x * Lt;
    // The block's rows y0 .. y0+Lt-1 are consecutive in node order, so its
    // body nodes form one run [nbase, nbase + nval).  The generator runs over
    // that run with consecutive threads on consecutive nodes (coalesced
    // loads and stores); its values reach the FFT layout (thread j holds the
    // x pairs 2(j + Tc q), +1) through a flat [Lt][b1] staging area that
    // overlays the row buffers.  Nodes per thread: Lt*b1/nthr = 8 b1/Nc,
    // at most 8 when b1 <= Nc (required for LG > 0), else at most 16.
    constexpr int RN = x_rn<LG>();
    const long nbase = ((long)z * g.b2 + y0) * g.b1;
    const int nval = min(Lt, g.b2 - y0) * g.b1;
    T gv[NF][RN];
    // Node slots in groups of NG: all loads of a group are issued
    // before its first store (a store may alias any later load, so a
    // read-modify-write generator would otherwise wait out one memory latency
    // per slot).  A full block takes a branch-free path.
    auto run_gen = [&](auto full) {
        uint8_t cbv[RN];
#pragma unroll
        for (int r = 0; r < RN; ++r) {
            const int e = tid + nthr * r;
            cbv[r] = (decltype(full)::value || e < nval) ? node_flags(gen, Nd{nbase, (uint32_t)e}) : uint8_t(0);
        }
#pragma unroll
        for (int r0 = 0; r0 < RN; r0 += NG) {
            typename G::Ld ld[NG];
#pragma unroll
            for (int q = 0; q < NG; ++q) {
                if (r0 + q >= RN) break;   // the last group of an RN that NG does not divide
                const int e = tid + nthr * (r0 + q);
                if (decltype(full)::value || e < nval) ld[q] = gen.load(Nd{nbase, (uint32_t)e}, cbv[r0 + q]);
            }
#pragma unroll
            for (int q = 0; q < NG; ++q) {
                if (r0 + q >= RN) break;
                const int e = tid + nthr * (r0 + q);
                T a[NF];
#pragma unroll
                for (int f = 0; f < NF; ++f) a[f] = T(0);
                if (decltype(full)::value || e < nval) gen.gen(Nd{nbase, (uint32_t)e}, ld[q], a);
#pragma unroll
                for (int f = 0; f < NF; ++f) gv[f][r0 + q] = a[f];
            }
        }
    };
    if (nval == RN * nthr) run_gen(std::true_type{});
    else run_gen(std::false_type{});
    // twiddles of length n1 in LDS after the rows; W_Nc^e = W_n1^(2e)
    stage_table(lds + Lt * row_pitch(Nc), twb + g.twn1, g.n1);
    r2c_store<T, NF, RN, LG>(g, gv, SA, lds, nthr, nval, z, y0);
}

// Output O of the spectral multiply for the 8 wavenumbers of thread j along
// the last axis (k = j + Tn*q): evaluate the kernel multipliers of the
// components output O needs from the taps B[c*ntap + t] of this line, then
// combine the transformed inputs.
template <int O, class T, class M, int NIN>
__device__ __forceinline__ void spectral_out(const M& mul, const T* __restrict__ B_g, int ntap, uint32_t oddmask,
                                             int j, int Tn, int n_last, const cx<T>* __restrict__ twl_g,
                                             const cx<T> (&vin)[NIN][8], cx<T> (&w)[8]) {
    constexpr uint32_t need = M::template need<O>();
    const uint32_t odd = M::RT_ODD ? oddmask : M::ODD;
    lds_ptr<const T> B = as_lds(B_g);
    lds_ptr<const cx<T>> twl = as_lds(twl_g);
    // this line's taps of the components output O needs, once per line
    T Bt[M::NC > 0 ? M::NC : 1][9];
#pragma unroll
    for (int c = 0; c < M::NC; ++c)
        if ((need >> c) & 1u) {
#pragma unroll
            for (int t = 0; t < 9; ++t) Bt[c][t] = (t < ntap) ? B[c * ntap + t] : T(0);
        }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int k = j + Tn * q;
        T K[M::NC > 0 ? M::NC : 1];
#pragma unroll
        for (int c = 0; c < M::NC; ++c)
            if ((need >> c) & 1u) K[c] = Bt[c][0];
        // taps t = 1 .. ntap-1 (ntap <= 9), unrolled with a guard
#pragma unroll
        for (int t = 1; t < 9; ++t) {
            if (t < ntap) {
                cx<T> tw = twl[(k * t) & (n_last - 1)];
                const T cs = tw.r, sn = -tw.i;
#pragma unroll
                for (int c = 0; c < M::NC; ++c)
                    if ((need >> c) & 1u) K[c] += Bt[c][t] * (((odd >> (M::C0 + c)) & 1u) ? sn : cs);
            }
        }
        cx<T> a[NIN];
#pragma unroll
        for (int f = 0; f < NIN; ++f) a[f] = vin[f][q];
        w[q] = mul.template one<O>(K, a);
    }
}

// Multipliers that form all outputs of a wavenumber at once (mul.all).
template <class M, class = void>
struct has_all_out : std::false_type {};
template <class M>
struct has_all_out<M, std::void_t<decltype(&M::all)>> : std::true_type {};

// All outputs for the 8 wavenumbers of thread j: every kernel component
// evaluated once per wavenumber, then mul.all.
template <class T, class M, int NIN, int NOUT>
__device__ __forceinline__ void spectral_all(const M& mul, const T* __restrict__ B_g, int ntap, uint32_t oddmask,
                                             int j, int Tn, int n_last, const cx<T>* __restrict__ twl_g,
                                             const cx<T> (&vin)[NIN][8], cx<T> (&w)[NOUT][8]) {
    // (w may be vin: each wavenumber's inputs are copied before its outputs
    // are written)
    const uint32_t odd = M::RT_ODD ? oddmask : M::ODD;
    lds_ptr<const T> B = as_lds(B_g);
    lds_ptr<const cx<T>> twl = as_lds(twl_g);
    T Bt[M::NC][9];
#pragma unroll
    for (int c = 0; c < M::NC; ++c)
#pragma unroll
        for (int t = 0; t < 9; ++t) Bt[c][t] = (t < ntap) ? B[c * ntap + t] : T(0);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int k = j + Tn * q;
        T K[M::NC];
#pragma unroll
        for (int c = 0; c < M::NC; ++c) K[c] = Bt[c][0];
#pragma unroll
        for (int t = 1; t < 9; ++t) {
            if (t < ntap) {
                cx<T> tw = twl[(k * t) & (n_last - 1)];
                const T cs = tw.r, sn = -tw.i;
#pragma unroll
                for (int c = 0; c < M::NC; ++c) K[c] += Bt[c][t] * (((odd >> (M::C0 + c)) & 1u) ? sn : cs);
            }
        }
        cx<T> a[NIN], o[NOUT];
#pragma unroll
        for (int f = 0; f < NIN; ++f) a[f] = vin[f][q];
        mul.all(K, a, o);
#pragma unroll
        for (int f = 0; f < NOUT; ++f) w[f][q] = o[f];
    }
}

// Compile-time loop over the outputs: multiply, inverse FFT, store.
template <int O, int NO>
struct OutLoop {
    template <class F>
    __device__ __forceinline__ static void run(F&& f) {
        f(std::integral_constant<int, O>{});
        OutLoop<O + 1, NO>::run(f);
    }
};
template <int NO>
struct OutLoop<NO, NO> {
    template <class F>
    __device__ __forceinline__ static void run(F&&) {}
};

// ----------------------------------------------------------------------------
// Last-axis pass: contiguous lines along the last axis (y in 2D, z in 3D).
// Line li (0 <= li < nlines) of field f starts at base + f*fstride + li*pitch
// and holds len body points (zero-padded to the FFT length N).  The line is
// also the taps prefix index: kx in 2D, kx*n2 + ky in 3D.  FFT, spectral
// multiply, inverse FFT, body points stored back in place (a block owns
// whole lines of every field).
struct Lines {
    long nlines, pitch, fstride;
    int len, N;
    int out_off;   // outputs go to fields out_off .. out_off + NOUT - 1
};

// block Lw*(N/8), LDS Lw*(N+1) complex + taps Lw*NC*ntap.
template <class T, class M>
__global__ void __launch_bounds__(256) k_lastmul(Lines ln, M mul, cx<T>* S, const T* __restrict__ taps,
                                                 int ntap, int nct, uint32_t oddmask, const cx<T>* __restrict__ twb) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    constexpr int NI = M::NIN, NO = M::NOUT;
    const int N = ln.N, Tn = N >> 3, lgN = 31 - __clz(N);
    const int Lw = blockDim.x / Tn;
    const int tid = threadIdx.x, j = tid % Tn, l = tid / Tn;
    const long li = (long)blockIdx.x * Lw + l;
    const bool ok = li < ln.nlines;
    const long lic = ok ? li : 0;
    // twiddles after the FFT area, then the taps of this block's lines [l][c][t]
    cx<T>* tw = lds + (long)Lw * line_pitch(N);
    stage_twiddles(tw, twb, N);
    T* tl = reinterpret_cast<T*>(tw + tw_lds_len(N));
    for (int e = tid; e < Lw * M::NC * ntap; e += blockDim.x) {
        const int ll = e / (M::NC * ntap), ct = e % (M::NC * ntap);
        const long kk = min((long)blockIdx.x * Lw + ll, ln.nlines - 1);
        tl[e] = taps[(kk * nct + M::C0) * ntap + ct];
    }
    cx<T> vin[NI][8];
#pragma unroll
    for (int f = 0; f < NI; ++f) {
        const cx<T>* src = S + f * ln.fstride + lic * ln.pitch;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int p = j + Tn * q;
            vin[f][q] = (ok && p < ln.len) ? src[p] : cx<T>{T(0), T(0)};
        }
    }
    cx<T>* line = lds + l * line_pitch(N);
#pragma unroll
    for (int f = 0; f < NI; ++f) fft_line<-1>(vin[f], j, lgN, tw, 0, line);
    const T* Bt = tl + l * (M::NC * ntap);
    if constexpr (has_all_out<M>::value && NI == NO) {
        // one symbol evaluation per wavenumber for all outputs, written over
        // the inputs of that wavenumber (a separate output array next to the
        // inputs spilled in FP64)
        spectral_all<T, M, NI, NO>(mul, Bt, ntap, oddmask, j, Tn, N, tw, vin, vin);
        OutLoop<0, NO>::run([&](auto Oc) {
            constexpr int O = decltype(Oc)::value;
            fft_line<1>(vin[O], j, lgN, tw, 0, line);
            if (ok) {
                cx<T>* dst = S + (ln.out_off + O) * ln.fstride + li * ln.pitch;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int p = j + Tn * q;
                    if (p < ln.len) dst[p] = vin[O][q];
                }
            }
        });
    } else {
        OutLoop<0, NO>::run([&](auto Oc) {
            constexpr int O = decltype(Oc)::value;
            cx<T> w[8];
            spectral_out<O, T, M, NI>(mul, Bt, ntap, oddmask, j, Tn, N, tw, vin, w);
            fft_line<1>(w, j, lgN, tw, 0, line);
            if (ok) {
                cx<T>* dst = S + (ln.out_off + O) * ln.fstride + li * ln.pitch;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int p = j + Tn * q;
                    if (p < ln.len) dst[p] = w[q];
                }
            }
        });
    }
}

// ----------------------------------------------------------------------------
// Specialised last-axis pass: N = 2^LG points per line (compile time),
// exactly NT taps per component, and lines of at least 512 points so that a
// line fills whole wavefronts (N/8 >= 64 threads).  Then
//  * every address of the FFT stages is a compile-time offset from a
//    per-thread base;
//  * a wavefront works on one line only, so the line's taps are
//    wave-uniform and are read with scalar loads straight from the tap table
//    (layout [line][component][tap]), kept in scalar registers;
//  * the trig factors of the taps for the 8 wavenumbers k = j + (N/8) q of
//    thread j follow from those of j by eighth-turn rotations
//    (2 pi (N/8) q t / N = pi q t / 4), so each tap costs one table read per
//    line and no per-wavenumber lookups;
//  * for at most three outputs, all outputs are formed in one sweep over the
//    wavenumbers (each kernel component evaluated once) and the input
//    spectra die before the inverse transforms.
template <class T, int NT>
struct TapTrig {
    // per tap t >= 1: cos, sin of phi_t = 2 pi j t / N and (cos -+ sin)/sqrt2
    T c[NT], s[NT], a[NT], b[NT];
    // cos / sin of phi_t + pi m / 4, m = (q t) mod 8
    template <int M8>
    __device__ __forceinline__ T cosr(int t) const {
        if constexpr (M8 == 0) return c[t];
        else if constexpr (M8 == 1) return a[t];
        else if constexpr (M8 == 2) return -s[t];
        else if constexpr (M8 == 3) return -b[t];
        else if constexpr (M8 == 4) return -c[t];
        else if constexpr (M8 == 5) return -a[t];
        else if constexpr (M8 == 6) return s[t];
        else return b[t];
    }
    template <int M8>
    __device__ __forceinline__ T sinr(int t) const {
        if constexpr (M8 == 0) return s[t];
        else if constexpr (M8 == 1) return b[t];
        else if constexpr (M8 == 2) return c[t];
        else if constexpr (M8 == 3) return a[t];
        else if constexpr (M8 == 4) return -s[t];
        else if constexpr (M8 == 5) return -b[t];
        else if constexpr (M8 == 6) return -c[t];
        else return -a[t];
    }
};

// Kernel components at wavenumber k = j + (N/8) Q from the line's taps.
template <int Q, int T0, int NT, class T, class M>
struct TapSum {
    __device__ __forceinline__ static void run(const T* __restrict__ Bl, const TapTrig<T, NT>& tr, T* K) {
        if constexpr (T0 < NT) {
            constexpr int M8 = (Q * T0) & 7;
            const T cs = tr.template cosr<M8>(T0), sn = tr.template sinr<M8>(T0);
#pragma unroll
            for (int c = 0; c < M::NC; ++c) K[c] += Bl[c * NT + T0] * (((M::ODD >> (M::C0 + c)) & 1u) ? sn : cs);
            TapSum<Q, T0 + 1, NT, T, M>::run(Bl, tr, K);
        }
    }
};

template <int Q, int NQ>
struct QLoop {
    template <class F>
    __device__ __forceinline__ static void run(F&& f) {
        f(std::integral_constant<int, Q>{});
        QLoop<Q + 1, NQ>::run(f);
    }
};
template <int NQ>
struct QLoop<NQ, NQ> {
    template <class F>
    __device__ __forceinline__ static void run(F&&) {}
};

// block Lw*(N/8) (Lw lines), LDS Lw*line_pitch(N) + N complex.  From 512
// points on a line fills whole waves and its taps are wave-uniform (scalar
// loads); a 256-point line is half a wave, and the taps are per-lane loads.
template <class T, class M, int LG, int NT>
__global__ void __launch_bounds__(256) k_lastmul_f(Lines ln, M mul, cx<T>* S, const T* __restrict__ taps, int nct,
                                                   const cx<T>* __restrict__ twb) {
    static_assert(LG >= 8 && NT >= 1 && !M::RT_ODD, "specialised pass needs N >= 256");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    constexpr int NI = M::NIN, NO = M::NOUT, N = 1 << LG, Tn = N >> 3;
    const int tid = threadIdx.x, j = tid & (Tn - 1);
    // line slot: wave-uniform from 512 points on
    const int l = LG >= 9 ? __builtin_amdgcn_readfirstlane(tid >> (LG - 3)) : (tid >> (LG - 3));
    const int Lw = blockDim.x >> (LG - 3);
    const long li = (long)blockIdx.x * Lw + l;
    const bool ok = li < ln.nlines;
    const long lic = ok ? li : 0;
    cx<T>* tw = lds + (long)Lw * line_pitch(N);
    stage_twiddles(tw, twb, N);
    cx<T> vin[NI][8];
#pragma unroll
    for (int f = 0; f < NI; ++f) {
        const cx<T>* src = S + f * ln.fstride + lic * ln.pitch;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int p = j + Tn * q;
            vin[f][q] = (ok && p < ln.len) ? src[p] : cx<T>{T(0), T(0)};
        }
    }
    cx<T>* line = lds + l * line_pitch(N);
#pragma unroll
    for (int f = 0; f < NI; ++f) fft_line<-1>(vin[f], j, LG, tw, 0, line);
    // base trig factors of this thread (the table holds exp(-2 pi i e / N))
    TapTrig<T, NT> tr;
    {
        lds_ptr<const cx<T>> twv = as_lds(tw);
        const T h = T(0.70710678118654752440084436210484904);
#pragma unroll
        for (int t = 1; t < NT; ++t) {
            const cx<T> w = twv[(j * t) & (N - 1)];
            tr.c[t] = w.r;
            tr.s[t] = -w.i;
            tr.a[t] = (w.r + w.i) * h;
            tr.b[t] = (w.r - w.i) * h;
        }
    }
    const T* __restrict__ Bl = taps + (lic * nct + M::C0) * NT;
    auto kvals = [&](auto Qc, T* K) {
        constexpr int Q = decltype(Qc)::value;
#pragma unroll
        for (int c = 0; c < M::NC; ++c) K[c] = Bl[c * NT];
        TapSum<Q, 1, NT, T, M>::run(Bl, tr, K);
    };
    auto store = [&](int O, cx<T> (&w)[8]) {
        if (ok) {
            cx<T>* dst = S + (ln.out_off + O) * ln.fstride + li * ln.pitch;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int p = j + Tn * q;
                if (p < ln.len) dst[p] = w[q];
            }
        }
    };
    if constexpr (NO <= 3) {
        cx<T> w[NO][8];
        QLoop<0, 8>::run([&](auto Qc) {
            constexpr int Q = decltype(Qc)::value;
            T K[M::NC];
            kvals(Qc, K);
            cx<T> a[NI];
#pragma unroll
            for (int f = 0; f < NI; ++f) a[f] = vin[f][Q];
            if constexpr (has_all_out<M>::value) {
                // all outputs from one evaluation (the preconditioner's 3x3
                // inverse once per wavenumber)
                cx<T> o[NO];
                mul.all(K, a, o);
#pragma unroll
                for (int O = 0; O < NO; ++O) w[O][Q] = o[O];
            } else {
                OutLoop<0, NO>::run([&](auto Oc) {
                    constexpr int O = decltype(Oc)::value;
                    w[O][Q] = mul.template one<O>(K, a);
                });
            }
        });
#pragma unroll
        for (int O = 0; O < NO; ++O) {
            fft_line<1>(w[O], j, LG, tw, 0, line);
            store(O, w[O]);
        }
    } else {
        OutLoop<0, NO>::run([&](auto Oc) {
            constexpr int O = decltype(Oc)::value;
            cx<T> w[8];
            QLoop<0, 8>::run([&](auto Qc) {
                constexpr int Q = decltype(Qc)::value;
                T K[M::NC];
                kvals(Qc, K);
                cx<T> a[NI];
#pragma unroll
                for (int f = 0; f < NI; ++f) a[f] = vin[f][Q];
                w[Q] = mul.template one<O>(K, a);
            });
            fft_line<1>(w, j, LG, tw, 0, line);
            store(O, w);
        });
    }
}

// ----------------------------------------------------------------------------
// Last-axis pass by direct summation.  After the transforms along the other
// axes, the multiplier of component c along the last axis is a trigonometric
// polynomial of degree m (the taps): B_c[0] + sum_{t=1..m} B_c[t] trig(2 pi k t / n).
// Multiplying by it and transforming back is, exactly, a (2m+1)-point
// correlation along the line, since the line is zero beyond the body and the
// box leaves at least m zeros on each side (the periodic wrap only meets
// zeros):
//   even c:  w_c[0] g(z) + sum_t w_c[t] (g(z+t) + g(z-t))
//   odd c:   -i sum_t w_c[t] (g(z+t) - g(z-t))     (the i of i^P_c taken
//            out of the sine: i sin = (e^{+i} - e^{-i}) / 2)
// with w_c[t] the taps in the direct convention (1/(n1 n2) instead of the
// transform normalisation, no factor 2 for t > 0).  Each multiplier lists
// its terms (DTerm: output, input, component, sign, power of i, k_a).  For
// m = 3 this is ~170 arithmetic operations per point of the LPS force stage
// against ~530 for the FFT-multiply-FFT form of the same product.
//
// One wavefront per line, four lines per block.  The line is swept in
// chunks of 256 points, lane j holding the 4 consecutive points 4j .. 4j+3
// of the chunk in registers (coalesced loads and stores).  The neighbours up
// to 4 points away come from the lanes on either side by DPP whole-wave
// shifts.  Beyond the chunk ends: lane 63 loads the next chunk's first 4
// points (not yet overwritten: the outputs may replace the inputs in
// place), and lane 0 takes the previous chunk's last 4 input points, which
// lane 63 left in a small wave-private LDS slot before that chunk's stores.
// The taps are wave-uniform (scalar loads).
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
constexpr int DPP_WAVE_SHL1 = 0x130;   // lane i receives lane i+1
constexpr int DPP_WAVE_SHR1 = 0x138;   // lane i receives lane i-1

template <class T>
struct alignas(4 * sizeof(T)) cx2 {
    cx<T> a, b;
};

template <int N>
struct IPow {
    template <class T>
    __device__ __forceinline__ static cx<T> apply(cx<T> a) {
        if constexpr ((N & 3) == 0) return a;
        else if constexpr ((N & 3) == 1) return {-a.i, a.r};
        else if constexpr ((N & 3) == 2) return {-a.r, -a.i};
        else return {a.i, -a.r};
    }
};

// FP64: at least two waves per SIMD (<= 256 registers) keeps enough loads in
// flight; FP32 needs no bound.
template <class T, class M, int NT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 1 : 2)))
k_lastconv(Lines ln, M mul, cx<T>* S, const T* __restrict__ taps, int nct) {
    static_assert(!M::RT_ODD && NT >= 2 && NT <= 5, "direct pass: compile-time parities, at most 4 neighbours");
    constexpr int NI = M::NIN, NO = M::NOUT;
    constexpr bool LAZY = sizeof(T) == 8 && NI * NO > 16;
    const int lane = threadIdx.x & 63;
    const int l = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const long li = (long)blockIdx.x * (blockDim.x >> 6) + l;
    const bool ok = li < ln.nlines;    // wave-uniform
    const long lic = ok ? li : 0;
    const int len = ln.len, nch = (len + 255) >> 8;
    const T* __restrict__ Bl = taps + (lic * nct + M::C0) * NT;   // wave-uniform
    const T ka = mul.ka_value();
    __shared__ cx<T> halo_s[4 * NI * 4];
    lds_ptr<cx<T>> halo = as_lds(halo_s) + l * NI * 4;
    for (int ch = 0; ch < nch; ++ch) {
        const int z0 = ch * 256 + 4 * lane;
        // this lane's 4 points of an input field
        auto load_in = [&](int f, cx<T>(&dst)[4]) {
            const cx<T>* src = S + f * ln.fstride + lic * ln.pitch + z0;
            if (ok && z0 + 3 < len) {
                // 4 consecutive points; line starts are 16-point aligned
                const cx2<T> p0 = reinterpret_cast<const cx2<T>*>(src)[0];
                const cx2<T> p1 = reinterpret_cast<const cx2<T>*>(src)[1];
                dst[0] = p0.a; dst[1] = p0.b; dst[2] = p1.a; dst[3] = p1.b;
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    dst[q] = cx<T>{T(0), T(0)};
                    if (ok && z0 + q < len) dst[q] = src[q];
                }
            }
        };
        // every input's points loaded together, or (FP64 chains with many
        // inputs and outputs, whose points and outputs would not fit in the
        // registers of two waves) one input ahead of the arithmetic
        cx<T> cur[LAZY ? 2 : NI][4];
        if constexpr (LAZY) load_in(0, cur[0]);
        else {
#pragma unroll
            for (int f = 0; f < NI; ++f) load_in(f, cur[f]);
        }
        const int e0 = z0 + 4;   // lane 63: the next chunk's first points
        const bool edge_lane = ok && lane == 63;
        cx<T> out[NO][4];
#pragma unroll
        for (int o = 0; o < NO; ++o)
#pragma unroll
            for (int q = 0; q < 4; ++q) out[o][q] = cx<T>{T(0), T(0)};
#pragma unroll
        for (int J = 0; J < NI; ++J) {
            if constexpr (LAZY) {
                if (J + 1 < NI) load_in(J + 1, cur[(J + 1) & 1]);
            }
            // window of points z0 - 4 .. z0 + 7 of input J; lanes 0 and 63
            // load the points beyond the chunk ends themselves
            cx<T> edge[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) edge[q] = cx<T>{T(0), T(0)};
            if (edge_lane) {
                const cx<T>* src = S + J * ln.fstride + lic * ln.pitch;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (e0 + q < len) edge[q] = src[e0 + q];
            }
            if (lane == 0 && ch > 0) {
#pragma unroll
                for (int q = 0; q < 4; ++q) edge[q] = halo[J * 4 + q];
            }
            const cx<T>(&cj)[4] = cur[LAZY ? (J & 1) : J];
            cx<T> w[12];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                w[4 + q] = cj[q];
                const cx<T> a = {dpp_mov<DPP_WAVE_SHR1>(cj[q].r), dpp_mov<DPP_WAVE_SHR1>(cj[q].i)};
                const cx<T> b = {dpp_mov<DPP_WAVE_SHL1>(cj[q].r), dpp_mov<DPP_WAVE_SHL1>(cj[q].i)};
                w[q] = lane == 0 ? edge[q] : a;
                w[8 + q] = lane == 63 ? edge[q] : b;
            }
            // lane 63's input points are the next chunk's left neighbours (read
            // by lane 0 above, in program order, before this write)
            if (lane == 63) {
#pragma unroll
                for (int q = 0; q < 4; ++q) halo[J * 4 + q] = cj[q];
            }
            // neighbour sums at the 4 points, then every term that reads input J
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const cx<T> ctr = w[4 + q];
                cx<T> ev[NT], od[NT];
#pragma unroll
                for (int t = 1; t < NT; ++t) {
                    ev[t] = w[4 + q + t] + w[4 + q - t];
                    od[t] = w[4 + q + t] - w[4 + q - t];
                }
                OutLoop<0, NO>::run([&](auto Oc) {
                    constexpr int O = decltype(Oc)::value;
                    OutLoop<0, NI>::run([&](auto Jc) {
                        constexpr int JJ = decltype(Jc)::value;
                        constexpr DTerm tm = M::dterm(O, JJ);
                        if constexpr (tm.coef != 0) {
                            if (JJ == J) {
                                constexpr bool zo = (M::ODD >> (M::C0 + tm.c)) & 1u;
                                cx<T> sv;
                                if constexpr (zo) {
                                    sv = cscale(od[1], Bl[tm.c * NT + 1]);
#pragma unroll
                                    for (int t = 2; t < NT; ++t) sv = sv + cscale(od[t], Bl[tm.c * NT + t]);
                                } else {
                                    sv = cscale(ctr, Bl[tm.c * NT]);
#pragma unroll
                                    for (int t = 1; t < NT; ++t) sv = sv + cscale(ev[t], Bl[tm.c * NT + t]);
                                }
                                // i^ipow of the multiplier, times -i for a component odd along the line
                                sv = IPow<tm.ipow + (zo ? 3 : 0)>::apply(sv);
                                if constexpr (tm.ka) sv = cscale(sv, ka);
                                if constexpr (tm.coef == 1) out[O][q] = out[O][q] + sv;
                                else if constexpr (tm.coef == -1) out[O][q] = out[O][q] - sv;
                                else out[O][q] = out[O][q] + cscale(sv, T(tm.coef));
                            }
                        }
                    });
                });
            }
        }
        if (ok) {
#pragma unroll
            for (int o = 0; o < NO; ++o) {
                cx<T>* dst = S + (ln.out_off + o) * ln.fstride + li * ln.pitch + z0;
                if (z0 + 3 < len) {
                    reinterpret_cast<cx2<T>*>(dst)[0] = cx2<T>{out[o][0], out[o][1]};
                    reinterpret_cast<cx2<T>*>(dst)[1] = cx2<T>{out[o][2], out[o][3]};
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (z0 + q < len) dst[q] = out[o][q];
                }
            }
        }
    }
}

// ----------------------------------------------------------------------------
// (y, z) pass by direct summation (3D).  After the transform along x alone,
// the multiplier of component c at x-wavenumber kx is, over (y, z), a 2D
// trigonometric polynomial whose coefficients are the partial x-spectra
//   tau_c(kx; oy, oz) = sum_ox K_c(o) trig_c(2 pi kx ox / n1)
// (cos for a component even along x; sin, times i, for an odd one).
// Multiplying by it and transforming back along y and z is, exactly, the 2D
// correlation  out(y, z) = sum_{oy, oz} i^{p_x} tau_c(kx; oy, oz) g(y + oy, z + oz)
// over the body rows and planes: the box leaves at least one horizon of
// zeros beyond the body along y and z, so the periodic wrap meets only
// zeros.  K_c is even or odd along y and along z, so the four points
// (+-oy, +-oz) enter as sums or differences and only the taps with
// oy, oz >= 0 inside the horizon's quarter disc oy^2 + oz^2 <= MT^2 are
// stored (yz_tap numbers them).  Each multiplier term (DTerm) applies with
// the real factor coef * i^(ipow - #odd axes), the powers of i of the full
// 3D multiplier other than the x one being the y and z parities here.
//
// A block takes one x-wavenumber, a tile of YT consecutive rows y (one per
// thread) and a chunk of planes z, and sweeps the input planes in order
// (upwards in even chunks, downwards in odd ones).
// Each plane goes through LDS with MT halo rows on either side, so a thread
// forms its y-neighbour sums and differences there; the plane's
// contributions go into the accumulators of the 2 MT + 1 output planes it
// reaches (a register ring), and an output plane is stored as soon as its
// last input plane is in.  The inputs are loaded two (four for the light
// FP64 passes) planes ahead of the arithmetic.  Outputs go to other SA fields than the
// inputs (neighbouring chunks read each other's planes).
struct YZArgs {
    int b2, b3, h1, P2;
    long saf;              // field stride of SA
    int nyt, nzc, zc;      // y tiles, z chunks, planes per chunk
    int in_off, out_off;   // SA field slots of the inputs and of the outputs
    int nct;               // components per x-wavenumber in the taps table
};

__host__ __device__ constexpr int yz_tap(int MT, int a, int b) {
    int n = 0;
    for (int bb = 0; bb <= MT; ++bb)
        for (int aa = 0; aa <= MT; ++aa) {
            if (aa * aa + bb * bb > MT * MT) continue;
            if (aa == a && bb == b) return n;
            ++n;
        }
    return n;   // (a, b) outside the quarter disc: the number of taps
}
__host__ __device__ constexpr int yz_ntap(int MT) { return yz_tap(MT, MT + 1, MT + 1); }

// popcount of a 3-bit parity
__host__ __device__ constexpr int npar(int p) { return (p & 1) + ((p >> 1) & 1) + ((p >> 2) & 1); }

// Real factor of a term in the (y, z) form: coef * i^(ipow - #odd axes).
template <class M>
__host__ __device__ constexpr int yz_factor(DTerm t) {
    const int e = ((t.ipow - npar(M::par3(t.c))) % 4 + 4) % 4;
    return e == 0 ? t.coef : -t.coef;   // e is 0 or 2 for a real-space kernel
}

// The term of output O and input J in the (y, z) pass: dterm_yz when the
// multiplier has one (constant factors folded into extra tap components).
template <class M, class = void>
struct has_dterm_yz : std::false_type {};
template <class M>
struct has_dterm_yz<M, std::void_t<decltype(M::dterm_yz(0, 0))>> : std::true_type {};
template <class M>
__host__ __device__ constexpr DTerm yz_dterm(int O, int J) {
    if constexpr (has_dterm_yz<M>::value) return M::dterm_yz(O, J);
    else return M::dterm(O, J);
}

// Whether output O has a term of an input in [J0, J1) whose component has
// z-parity G.
template <class M, int O, int G, int J0, int J1>
__host__ __device__ constexpr bool yz_group_used() {
    for (int J = J0; J < J1; ++J) {
        const DTerm t = yz_dterm<M>(O, J);
        if (t.coef != 0 && ((M::par3(t.c) >> 2) & 1) == G) return true;
    }
    return false;
}

// q += (real factor) * i^{p_x} * sum_a tau_c(a, b) P(a): one term at z-offset b,
// P the y-neighbour sums (component even along y) or differences (odd).
// C: component (relative to the multiplier's first), PR: its odd axes, FR:
// the real factor, KA: times k_a.
template <class T, int MT, int NU, int C, int PR, int FR, bool KA, int b>
__device__ __forceinline__ void yz_term(cx<T>& q, const T* __restrict__ tk, const cx<T> (&pe)[MT + 1],
                                        const cx<T> (&po)[MT + 1], T ka) {
    constexpr bool px = PR & 1, py = (PR >> 1) & 1;
    constexpr int fr = FR;
    constexpr bool plain = !KA && (fr == 1 || fr == -1);
    cx<T> st = {T(0), T(0)};
    OutLoop<py ? 1 : 0, MT + 1>::run([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        if constexpr (a * a + b * b <= MT * MT) {
            const T w = tk[C * NU + yz_tap(MT, a, b)];
            const cx<T> P = py ? po[a] : pe[a];
            if constexpr (plain) {
                // straight into q, the sign and the i of an odd x-parity folded in
                const T sw = fr > 0 ? w : -w;
                if constexpr (px) { q.r -= sw * P.i; q.i += sw * P.r; }
                else { q.r += sw * P.r; q.i += sw * P.i; }
            } else {
                st.r += w * P.r;
                st.i += w * P.i;
            }
        }
    });
    if constexpr (!plain) {
        T sc = T(fr);
        if constexpr (KA) sc *= ka;
        if constexpr (px) { q.r -= sc * st.i; q.i += sc * st.r; }
        else { q.r += sc * st.r; q.i += sc * st.i; }
    }
}

template <class T, class M, int MT, int YT>
__global__ void __launch_bounds__(YT) k_yzconv(YZArgs a, M mul, cx<T>* S, const T* __restrict__ taps) {
    constexpr int NI = M::NIN, NO = M::NOUT, R = 2 * MT + 1, W = YT + 2 * MT, NU = yz_ntap(MT);
    // FP32 sums the terms of all inputs at once (their neighbour sums held
    // together) when there are few inputs; otherwise one input at a time
    constexpr bool YZ_GROUP = sizeof(T) == 4 && NI <= 4;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    lds_ptr<cx<T>> lds = as_lds(reinterpret_cast<cx<T>*>(smem_raw));
    // block -> (kx, y tile, z chunk): consecutive chunks of one (kx, tile) on one XCD
    const long nblk = (long)a.h1 * a.nyt * a.nzc;
    const long bq = nblk >> 3, br = nblk & 7;
    const long xcd = blockIdx.x & 7, bk = blockIdx.x >> 3;
    const long lin = xcd < br ? xcd * (bq + 1) + bk : br * (bq + 1) + (xcd - br) * bq + bk;
    const int zc = (int)(lin % a.nzc);
    const long t2 = lin / a.nzc;
    const int yt = (int)(t2 % a.nyt);
    const int kx = (int)(t2 / a.nyt);

    const int tid = threadIdx.x;
    const int y0 = yt * YT, y = y0 + tid;
    const bool yin = y < a.b2;
    // halo rows: threads 0 .. MT-1 the MT rows below the tile, MT .. 2MT-1 the MT above
    const bool hlo = tid < MT, hthr = tid < 2 * MT;
    const int yh = hlo ? y0 - MT + tid : y0 + YT + (tid - MT);
    const int ph = hlo ? tid : YT + tid;
    const bool hin = hthr && yh >= 0 && yh < a.b2;
    // block-uniform: a neighbouring tile exists (else the halo rows are zero,
    // written once below)
    const bool halo = a.nyt > 1;
    const int z0 = zc * a.zc, z1 = min(a.b3, z0 + a.zc);
    // odd chunks sweep their planes downwards, so that both chunks at a
    // chunk boundary sweep the planes around it at the same time (both at
    // their start or both at their end) and the halo planes they share are
    // fetched from HBM once; a downward sweep takes the second taps table,
    // whose components odd along z are negated (the plane at offset -b then
    // takes the place of the one at +b)
    const bool down = (zc & 1) != 0;   // block-uniform
    const int dz = down ? -1 : 1;
    const T* __restrict__ tk = taps + (down ? (long)a.h1 * a.nct * NU : 0L) + ((long)kx * a.nct + M::C0) * NU;
    const T ka = mul.ka_value();
    const long zs = (long)a.h1 * a.P2;
    const cx<T>* __restrict__ src = S + (long)a.in_off * a.saf + (long)kx * a.P2;
    cx<T>* __restrict__ dst = S + (long)a.out_off * a.saf + (long)kx * a.P2 + y;

    // ring of RR = 2 MT + 2 output planes (one more than the 2 MT + 1 an
    // input plane reaches, so that the sweep unrolls by an even count and the
    // two register sets of prefetched inputs alternate at compile time)
    constexpr int RR = R + 1;
    cx<T> acc[RR][NO];
#pragma unroll
    for (int r = 0; r < RR; ++r)
#pragma unroll
        for (int o = 0; o < NO; ++o) acc[r][o] = cx<T>{T(0), T(0)};
    // PF register sets of prefetched inputs (planes zi+1 .. zi+PF in flight):
    // four for the light dilatation-type passes in FP64 (NI * NO <= 4), else
    // two (in FP32 the extra registers cost more occupancy than they gain)
    // (one set for chains with many inputs, whose sets would crowd out the
    // accumulators)
    constexpr int PF = NI > 4 ? 1 : ((sizeof(T) == 8 && NI * NO <= 4 && RR % 4 == 0) ? 4 : 2);
    cx<T> nv[PF][NI], nh[PF][NI];   // row y, halo row yh
#pragma unroll
    for (int k = 0; k < PF; ++k)
#pragma unroll
        for (int J = 0; J < NI; ++J) nv[k][J] = nh[k][J] = cx<T>{T(0), T(0)};
    // straight-line loads: the plane index is clamped into the body (planes
    // outside it are never used) and rows beyond the body read row 0 and are
    // replaced by zeros
    const int yl = yin ? y : 0;
    auto load = [&](auto pc, int z) {
        constexpr int P = decltype(pc)::value;
        const cx<T>* __restrict__ sp = src + min(max(z, 0), a.b3 - 1) * zs;
#pragma unroll
        for (int J = 0; J < NI; ++J) {
            const cx<T> v = sp[J * a.saf + yl];
            nv[P][J] = yin ? v : cx<T>{T(0), T(0)};
        }
        if (halo) {
#pragma unroll
            for (int J = 0; J < NI; ++J) {
                nh[P][J] = cx<T>{T(0), T(0)};
                if (hin) nh[P][J] = sp[J * a.saf + yh];
            }
        }
    };
    // halo rows of both buffers start at zero (the only value they keep
    // when the tile has no neighbour on that side)
    if (hthr) {
#pragma unroll
        for (int J = 0; J < 2 * NI; ++J) lds[J * W + ph] = cx<T>{T(0), T(0)};
    }

    const int zb = down ? z1 - 1 + MT : z0 - MT;   // first input plane of the sweep
    const int nst = (z1 - z0) + 2 * MT;            // input planes swept
    OutLoop<0, PF>::run([&](auto kc) { load(kc, zb + dz * decltype(kc)::value); });
    for (int s0 = 0; s0 < nst; s0 += RR) {
        OutLoop<0, RR>::run([&](auto rc) {
            constexpr int rr = decltype(rc)::value, P = rr & 1, PS = rr % PF;
            const int s = s0 + rr;
            if (s >= nst) return;   // block-uniform
            const int zi = zb + dz * s;
            const bool act = zi >= 0 && zi < a.b3;   // block-uniform
            lds_ptr<cx<T>> row = lds + P * (NI * W);
            if (act) {
#pragma unroll
                for (int J = 0; J < NI; ++J) row[J * W + MT + tid] = nv[PS][J];
                if (halo) {
                    if (hthr) {
#pragma unroll
                        for (int J = 0; J < NI; ++J) row[J * W + ph] = nh[PS][J];
                    }
                }
                __syncthreads();
            }
            // the set just stored takes plane zi + PF (PF planes of arithmetic
            // to arrive)
            load(std::integral_constant<int, PS>{}, zi + dz * PF);
            if (act) {
                // per output and z-offset b, the terms of inputs J0 .. J1-1
                // even (G = 0) and odd (G = 1) along z: q0 and q1 reach output
                // plane zi - b as q0 + q1 and (b > 0) plane zi + b as q0 - q1.
                // The sums are chained to save adds: at b = 0 the G = 0 chain
                // starts from the accumulator itself; with both parities the
                // G = 1 chain starts from q0, giving s = q0 + q1, and the
                // other plane takes 2 q0 - s.
                auto terms = [&](auto j0c, auto j1c, const cx<T>(*pe)[MT + 1], const cx<T>(*po)[MT + 1]) {
                    constexpr int J0 = decltype(j0c)::value, J1 = decltype(j1c)::value;
                    OutLoop<0, NO>::run([&](auto Oc) {
                        constexpr int O = decltype(Oc)::value;
                        constexpr bool U0 = yz_group_used<M, O, 0, J0, J1>(), U1 = yz_group_used<M, O, 1, J0, J1>();
                        auto chain = [&](auto Gc, auto bc, cx<T>& q) {
                            constexpr int G = decltype(Gc)::value, b = decltype(bc)::value;
                            OutLoop<J0, J1>::run([&](auto Jc) {
                                constexpr int J = decltype(Jc)::value;
                                constexpr DTerm tm = yz_dterm<M>(O, J);
                                if constexpr (tm.coef != 0 && ((M::par3(tm.c) >> 2) & 1) == G) {
                                    yz_term<T, MT, NU, tm.c, M::par3(tm.c), yz_factor<M>(tm), tm.ka, b>(
                                        q, tk, pe[J - J0], po[J - J0], ka);
                                }
                            });
                        };
                        OutLoop<0, MT + 1>::run([&](auto bc) {
                            constexpr int b = decltype(bc)::value;
                            // input plane zi reaches output plane zi - b with oz = +b
                            // and, for b > 0, plane zi + b with oz = -b
                            constexpr int sm = (rr - b + RR) % RR, sp = (rr + b) % RR;
                            using I0 = std::integral_constant<int, 0>;
                            using I1 = std::integral_constant<int, 1>;
                            if constexpr (b == 0) {
                                if constexpr (U0) chain(I0{}, bc, acc[sm][O]);
                            } else if constexpr (U0 && U1) {
                                cx<T> q0 = {T(0), T(0)};
                                chain(I0{}, bc, q0);
                                cx<T> s = q0;
                                chain(I1{}, bc, s);
                                acc[sm][O] = acc[sm][O] + s;
                                acc[sp][O].r = (acc[sp][O].r + T(2) * q0.r) - s.r;
                                acc[sp][O].i = (acc[sp][O].i + T(2) * q0.i) - s.i;
                            } else if constexpr (U0) {
                                cx<T> q0 = {T(0), T(0)};
                                chain(I0{}, bc, q0);
                                acc[sm][O] = acc[sm][O] + q0;
                                acc[sp][O] = acc[sp][O] + q0;
                            } else if constexpr (U1) {
                                cx<T> q1 = {T(0), T(0)};
                                chain(I1{}, bc, q1);
                                acc[sm][O] = acc[sm][O] + q1;
                                acc[sp][O] = acc[sp][O] - q1;
                            }
                        });
                    });
                };
                // y-neighbour sums (pe) and differences (po) at this row
                auto nbr = [&](int J, cx<T>(&pe)[MT + 1], cx<T>(&po)[MT + 1]) {
                    pe[0] = row[J * W + MT + tid];
                    po[0] = cx<T>{T(0), T(0)};
#pragma unroll
                    for (int t = 1; t <= MT; ++t) {
                        const cx<T> up = row[J * W + MT + tid + t], dn = row[J * W + MT + tid - t];
                        pe[t] = up + dn;
                        po[t] = up - dn;
                    }
                };
                if constexpr (YZ_GROUP) {
                    // FP32: all inputs at once, one scatter per (output, parity, offset)
                    cx<T> pe[NI][MT + 1], po[NI][MT + 1];
#pragma unroll
                    for (int J = 0; J < NI; ++J) nbr(J, pe[J], po[J]);
                    terms(std::integral_constant<int, 0>{}, std::integral_constant<int, NI>{}, pe, po);
                } else {
                    // FP64: one input at a time (half the registers of the sums)
                    OutLoop<0, NI>::run([&](auto Jc) {
                        constexpr int J = decltype(Jc)::value;
                        cx<T> pe[1][MT + 1], po[1][MT + 1];
                        nbr(J, pe[0], po[0]);
                        terms(std::integral_constant<int, J>{}, std::integral_constant<int, J + 1>{}, pe, po);
                    });
                }
            }
            // output plane zi - MT has all its inputs
            constexpr int sd = (rr - MT + RR) % RR;
            const int zo = zi - dz * MT;
            if (zo >= z0 && zo < z1 && yin) {
#pragma unroll
                for (int o = 0; o < NO; ++o) dst[o * a.saf + zo * zs] = acc[sd][o];
            }
#pragma unroll
            for (int o = 0; o < NO; ++o) acc[sd][o] = cx<T>{T(0), T(0)};
        });
    }
}

// ----------------------------------------------------------------------------
// 3D y passes with a transpose, so that the z pass reads contiguous lines.
//   forward: SA [f][z][kx][y<b2]  --FFT along y-->  SB [f][kx][ky][z<Pz]
//   inverse: SB [f][kx][ky][z]    --iFFT along y--> SA [f][z][kx][y<b2]
// A block takes Lz consecutive body planes z0..z0+Lz-1 of one (f, kx), so
// every ky row of the transposed side is a contiguous run of Lz values.
// grid (ceil(b3/Lz), h1, F), block Lz*(n2/8), LDS Lz*(n2+1) complex.
template <class T, int LG>
__global__ void __launch_bounds__(1024) k_ytf(Geo g, const cx<T>* __restrict__ SA, cx<T>* __restrict__ SB,
                                              int Pz, const cx<T>* __restrict__ twb) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    const int lgN = LG > 0 ? LG : 31 - __clz(g.n2), N = 1 << lgN, Tn = N >> 3;
    const int Lz = blockDim.x / Tn;
    const int tid = threadIdx.x, j = tid % Tn, l = tid / Tn;
    const int kx = blockIdx.y, f = blockIdx.z;
    const int z0 = blockIdx.x * Lz, z = z0 + l;
    const bool ok = z < g.b3;
    cx<T> v[8];
    const cx<T>* src = SA + f * g.saf + ((long)(ok ? z : 0) * g.h1 + kx) * g.P2;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int p = j + Tn * q;
        v[q] = (ok && p < g.b2) ? src[p] : cx<T>{T(0), T(0)};
    }
    cx<T>* tw = lds + (long)Lz * line_pitch(N);
    stage_twiddles(tw, twb, N);
    cx<T>* line = lds + l * line_pitch(N);
    fft_line<-1>(v, j, lgN, tw, 0, line);
    __syncthreads();
    lds_ptr<cx<T>> linev = as_lds(line);
    lds_ptr<cx<T>> ldsv = as_lds(lds);
#pragma unroll
    for (int q = 0; q < 8; ++q) linev[j + Tn * q] = v[q];
    __syncthreads();
    // kk < Tn: the rows kk + Tn*i (i < 8) cover [0, N)
    const int ll = tid % Lz, kk = tid / Lz;
    if (z0 + ll < g.b3) {
        cx<T>* dst = SB + ((long)f * g.h1 + kx) * N * Pz + z0 + ll;
#pragma unroll
        for (int i = 0; i < 8; ++i) dst[(long)(kk + Tn * i) * Pz] = ldsv[ll * line_pitch(N) + kk + Tn * i];
    }
}

template <class T, int LG>
__global__ void __launch_bounds__(1024) k_yti(Geo g, const cx<T>* __restrict__ SB, cx<T>* __restrict__ SA,
                                              int Pz, const cx<T>* __restrict__ twb) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    const int lgN = LG > 0 ? LG : 31 - __clz(g.n2), N = 1 << lgN, Tn = N >> 3;
    const int Lz = blockDim.x / Tn;
    const int tid = threadIdx.x, j = tid % Tn, l = tid / Tn;
    const int kx = blockIdx.y, f = blockIdx.z;
    const int z0 = blockIdx.x * Lz, z = z0 + l;
    const int ll = tid % Lz, kk = tid / Lz;   // kk < Tn
    {
        // all eight loads of this thread in flight before the LDS stores
        const bool okr = z0 + ll < g.b3;
        const cx<T>* src = SB + ((long)f * g.h1 + kx) * N * Pz + z0 + ll;
        cx<T> t[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) t[i] = okr ? src[(long)(kk + Tn * i) * Pz] : cx<T>{T(0), T(0)};
        lds_ptr<cx<T>> ldsv = as_lds(lds);
#pragma unroll
        for (int i = 0; i < 8; ++i) ldsv[ll * line_pitch(N) + kk + Tn * i] = t[i];
    }
    cx<T>* tw = lds + (long)Lz * line_pitch(N);
    stage_twiddles(tw, twb, N);
    __syncthreads();
    cx<T>* line = lds + l * line_pitch(N);
    lds_ptr<cx<T>> linev = as_lds(line);
    cx<T> v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = linev[j + Tn * q];
    fft_line<1>(v, j, lgN, tw, 0, line);
    if (z < g.b3) {
        cx<T>* dst = SA + f * g.saf + ((long)z * g.h1 + kx) * g.P2;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int p = j + Tn * q;
            if (p < g.b2) dst[p] = v[q];
        }
    }
}

// ----------------------------------------------------------------------------
// Pass 5: transposed load of body rows from SA, c2r along x, epilogue.
// grid (ceil(b2/Lt), b3), block Tc*Lt; LDS Lt*(Nc+2) complex + reduction.
// partials: per block NRED doubles at (blockIdx.y*gridDim.x + blockIdx.x)*NRED.
// An epilogue with NCHAIN > 0 also returns NCHAIN values per node (fin_chain),
// which the pass transforms forward again (r2c) and stores to SAout: the c2r
// of one chain and the r2c of the next in one pass over the block's rows.
template <class F, class = void>
struct fin_chain_n : std::integral_constant<int, 0> {};
template <class F>
struct fin_chain_n<F, std::void_t<decltype(F::NCHAIN)>> : std::integral_constant<int, F::NCHAIN> {};

template <class T, class F, int LG>
__global__ void __launch_bounds__(512) k_xinv(Geo g, F fin, const cx<T>* __restrict__ SA,
                                               double* __restrict__ partials,
                                               const cx<T>* __restrict__ twb, cx<T>* __restrict__ SAout) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    constexpr int NO = F::NOUT, NG = node_group<T>();
    const int Nc = x_len<LG>(g), lgNc = x_lg<LG>(g), Tc = Nc >> 3;
    constexpr int XF = x_block_fixed<T, LG, fin_xrows<F>::value>();
    const int nthr = XF > 0 ? XF : (int)blockDim.x;
    const int Lt = nthr / Tc;
    const int tid = threadIdx.x, j = tid % Tc, l = tid / Tc;
    // block -> (row group, plane): when a block's transposed runs are shorter
    // than a 128-byte line (8 FP32 rows), consecutive row groups of a plane
    // go to one XCD (the hardware deals consecutive blocks to the 8 XCDs in
    // turn), so that the two blocks sharing a line meet in one L2
    const long nblk = (long)gridDim.x * gridDim.y, bq = nblk >> 3, br = nblk & 7;
    const long lin = (long)blockIdx.y * gridDim.x + blockIdx.x, xcd = lin & 7, bk = lin >> 3;
    const bool part_lines = Lt * (int)sizeof(cx<T>) < 128;   // block-uniform
    const long lg = !part_lines ? lin : (xcd < br ? xcd * (bq + 1) + bk : br * (bq + 1) + (xcd - br) * bq + bk);
    const int z = (int)(lg / gridDim.x);
    const int y0 = (int)(lg % gridDim.x) * Lt;
    const int y = y0 + l;
    const int pitch = row_pitch(Nc);
    cx<T>* row = lds + l * pitch;
    cx<T>* twn1 = lds + Lt * pitch;
    stage_table(twn1, twb + g.twn1, g.n1);
    // transposed load: thread (ll, kk < Tc) fetches the columns kk + Tc*i
    // (i < 8) and, for kk == 0, the Nyquist column Nc; the next field's
    // values are fetched while this field is transformed
    const int ll = tid % Lt, kk = tid / Lt;
    const bool okr = (y0 + ll) < g.b2;
    const cx<T>* src0 = SA + (long)z * g.h1 * g.P2 + y0 + ll;
    cx<T> pre[9];
    auto fetch = [&](int o) {
        const cx<T>* src = src0 + o * g.saf;
#pragma unroll
        for (int i = 0; i < 8; ++i) pre[i] = okr ? src[(long)(kk + Tc * i) * g.P2] : cx<T>{T(0), T(0)};
        pre[8] = (okr && kk == 0) ? src[(long)Nc * g.P2] : cx<T>{T(0), T(0)};
    };
    fetch(0);
    // flags of this thread's epilogue nodes, loaded ahead of the transforms
    // (the epilogue's static-field addresses depend on them)
    constexpr int RN = x_rn<LG>();
    const long nbase = ((long)z * g.b2 + y0) * g.b1;
    const int nval = min(Lt, g.b2 - y0) * g.b1;
    uint8_t cbv[RN];
#pragma unroll
    for (int r = 0; r < RN; ++r) {
        const int e = tid + nthr * r;
        cbv[r] = e < nval ? node_flags(fin, Nd{nbase, (uint32_t)e}) : uint8_t(0);
    }
    lds_ptr<cx<T>> rowv = as_lds(row);
    lds_ptr<cx<T>> ldsv = as_lds(lds);
    lds_ptr<const cx<T>> twv = as_lds(twn1);
    // complex point held in v[q] by this thread after the inverse transform:
    // j + Tc q (powers of two), s M + jj + (M/8) q (mixed radix, sub-line s)
    auto xpt = [&](int q) -> int {
        if constexpr (LG >= 0) return j + Tc * q;
        else {
            const int Tq = 1 << (lgNc - 3);
            return (j >> (lgNc - 3)) * (Tq << 3) + (j & (Tq - 1)) + Tq * q;
        }
    };
    // Each field: transposed spectra into the rows, c2r, then straight to the
    // epilogue layout (consecutive threads on consecutive nodes of the
    // block's run) through a flat [Lt][b1] staging area over the row
    // buffers, so only the per-node values nv stay in registers.
    lds_ptr<T> flat = as_lds(reinterpret_cast<T*>(lds));
    T nv[NO][RN];
#pragma unroll
    for (int o = 0; o < NO; ++o) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 8; ++i) ldsv[ll * pitch + kk + Tc * i] = pre[i];
        if (kk == 0) ldsv[ll * pitch + Nc] = pre[8];
        if (o + 1 < NO) fetch(o + 1);
        __syncthreads();
        // the complex half-spectrum point k of the packed c2r input, from the
        // r2c spectrum points k and Nc - k
        auto c2r_pre = [&](int k) -> cx<T> {
            cx<T> A = rowv[k];
            cx<T> B = cconj(rowv[Nc - k]);
            cx<T> w = cconj(twv[k]);
            cx<T> Dm = cmul(w, A - B);
            return (A + B) + cx<T>{-Dm.i, Dm.r};
        };
        cx<T> v[8];
        if constexpr (LG >= 0) {
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = c2r_pre(j + Tc * q);
            fft_line<1>(v, j, lgNc, twn1, 1, row);
        } else {
            // each thread forms the points of its sub-line s directly:
            // X[s + rad k2], k2 = jj + Tq q
            const int Tq = 1 << (lgNc - 3), s = j >> (lgNc - 3), jj = j & (Tq - 1);
            const int R = LG < -1 ? mix_R<LG>() : g.rad;
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = c2r_pre(s + R * (jj + Tq * q));
            fft_mixed_inv<mix_R<LG>(), mix_lgM<LG>(), T>(v, j, g.rad, lgNc, twn1, row);
        }
        __syncthreads();   // every row transform is done with its LDS
        if (y < g.b2) {
            if ((g.b1 & 1) == 0) {
                // one 2T store per pair (even b1: pairs start at even slots)
                lds_ptr<cx<T>> flat2 = (lds_ptr<cx<T>>)flat;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int x = 2 * xpt(q);
                    if (x < g.b1) flat2[(l * g.b1 + x) >> 1] = v[q];
                }
            } else {
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int x = 2 * xpt(q);
                    if (x < g.b1) flat[l * g.b1 + x] = v[q].r;
                    if (x + 1 < g.b1) flat[l * g.b1 + x + 1] = v[q].i;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RN; ++r) {
            const int e = tid + nthr * r;
            nv[o][r] = e < nval ? flat[e] : T(0);
        }
    }
    double red[F::NRED > 0 ? F::NRED : 1];
#pragma unroll
    for (int r = 0; r < (F::NRED > 0 ? F::NRED : 1); ++r) red[r] = 0.0;
    constexpr int NCH = fin_chain_n<F>::value;
    T chv[NCH > 0 ? NCH : 1][RN];
#pragma unroll
    for (int c = 0; c < (NCH > 0 ? NCH : 1); ++c)
#pragma unroll
        for (int r = 0; r < RN; ++r) chv[c][r] = T(0);
    auto run_fin = [&](auto full) {
#pragma unroll
        for (int r0 = 0; r0 < RN; r0 += NG) {
            typename F::Ld ld[NG];
#pragma unroll
            for (int q = 0; q < NG; ++q) {
                if (r0 + q >= RN) break;   // the last group of an RN that NG does not divide
                const int e = tid + nthr * (r0 + q);
                if (decltype(full)::value || e < nval) ld[q] = fin.load(Nd{nbase, (uint32_t)e}, cbv[r0 + q]);
            }
#pragma unroll
            for (int q = 0; q < NG; ++q) {
                if (r0 + q >= RN) break;
                const int e = tid + nthr * (r0 + q);
                if (decltype(full)::value || e < nval) {
                    T vv[NO];
#pragma unroll
                    for (int o = 0; o < NO; ++o) vv[o] = nv[o][r0 + q];
                    if constexpr (NCH > 0) {
                        T cn[NCH];
                        fin.fin_chain(Nd{nbase, (uint32_t)e}, ld[q], vv, red, cn);
#pragma unroll
                        for (int c = 0; c < NCH; ++c) chv[c][r0 + q] = cn[c];
                    } else {
                        fin.fin(Nd{nbase, (uint32_t)e}, ld[q], vv, red);
                    }
                }
            }
        }
    };
    if (nval == RN * nthr) run_fin(std::true_type{});   // branch-free, as in k_xfwd
    else run_fin(std::false_type{});
    if constexpr (NCH > 0) {
        // the twiddles are still in LDS after the row buffers
        static_assert(F::NRED == 0, "a chained epilogue has no reductions");
        r2c_store<T, NCH, RN, LG>(g, chv, SAout, lds, nthr, nval, z, y0);
    }
    if constexpr (F::NRED > 0) {
        __syncthreads();
        double* sm = reinterpret_cast<double*>(smem_raw);
        block_reduce_store<F::NRED>(red, partials + ((long)blockIdx.y * gridDim.x + blockIdx.x) * F::NRED, sm);
    }
}

// Deterministic final sum of per-block partials: out[r] = sum_b part[b*NR + r]
// (one block, fixed order tree), also written to host[r] when host is not
// null (the device address of a pinned host buffer).
static __global__ void k_reduce_final(const double* __restrict__ part, long nblk, int NR, double* __restrict__ out,
                                      double* __restrict__ host);

}  // namespace pdk
