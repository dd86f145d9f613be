// pd_ops.hpp -- per-node input generators, spectral multipliers and
// assembly epilogues of the FCBM-EC convolution chains.
//
// Every chain evaluates sums of the form (paper Eq. 13-14, 45)
//     sum_n a_n(x) [c_n (*) b_n](x)
// as: generator  -> b_n(x') on the body box (zero on the padding)
//     multiplier -> per wavenumber, combines F(b_n) with the kernel spectra
//     epilogue   -> a_n(x) times the convolutions, plus pointwise terms.
// Convolutions are correlations (K (*) g)(x) = sum_o K(o) g(x + o) over the
// horizon stencil, which is what the bond sums of Eq. 55 are; their
// multiplier is sum_o K(o) e^{+2 pi i k.o/n}.  The volume dV and the 1/N of
// the inverse DFT are folded into the kernel partial spectra (taps).
//
// Kernel component order inside a plan:
//   bond-based: C_ij (i <= j, sym index), then omega_0 (integrity plans)
//   LPS       : C_ij (6), then a0_i = omega xi_i (3)          [taps]
//               plus omega r^2 (static fields only)
// C_ij is even in every axis except i and j, a0_i is odd in axis i; a
// component odd in P axes has the multiplier i^P * (real sum).
#pragma once

#include <stdint.h>

#include "pd_fft.hpp"

namespace pdk {

__host__ __device__ constexpr int nsym(int D) { return D * (D + 1) / 2; }
__host__ __device__ constexpr int symi(int D, int i, int j) {
    return (i <= j) ? (i * D - (i * (i - 1)) / 2 + (j - i)) : (j * D - (j * (j - 1)) / 2 + (i - j));
}

// Weight kinds (match pd_weight_kind).
enum { WK_NONE = 0, WK_LAMBDA = 1, WK_SCALE = 2 };

// ----------------------------------------------------------------------------
// Node context shared by generators and epilogues.
//
// chiB[i] bit 0: the node is in the body; bit 1 (set only with bit 0): the
// node's whole horizon lies in the body ("interior"), so its static fields
// equal the constants stat_int (the same sums, in the same order) and are
// read from that small cached table instead of the per-node arrays; bit
// 2 + d: component d is an unknown (chi_Omega, only on the body).  The
// passes load chiB[i] ahead of the node's other loads and hand it to the
// generators' and epilogues' load steps, which take chi_Omega from it.
__device__ __forceinline__ uint8_t omega_bit(uint8_t cb, int d) { return (cb >> (2 + d)) & 1; }
// Node index of the x passes, split into a block-uniform part (the start of
// the block's run of body nodes) and a small per-thread part, so that every
// field access is a uniform base plus a 32-bit offset: the addressing mode
// with the base in scalar registers, instead of a 64-bit address per thread
// and field.
struct Nd {
    long base;      // block-uniform
    uint32_t off;   // per thread, < 2^20
};
// A block-uniform address, taken through readfirstlane so that it stays a
// scalar base (otherwise the compiler folds it into one 64-bit per-thread
// offset), as a global-memory pointer.
__device__ __forceinline__ __attribute__((address_space(1))) char* uniform_base(const void* p) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    return reinterpret_cast<__attribute__((address_space(1))) char*>(((uintptr_t)hi << 32) | lo);
}
// load / store of field p at node n
template <class T>
__device__ __forceinline__ T ldf(const T* p, Nd n) {
    auto b = uniform_base(p + n.base) + n.off * (uint32_t)sizeof(T);
    return *reinterpret_cast<const __attribute__((address_space(1))) T*>(b);
}
template <class T>
struct ident { using type = T; };
// Raise the step's non-finite flag (a plain store of 1: every writer stores
// the same value) when a new force or velocity value is NaN or infinite.
template <class T>
__device__ __forceinline__ void flag_nonfinite(double* flag, T Fn, T vn) {
    if (flag && !(__builtin_isfinite(Fn) && __builtin_isfinite(vn))) *flag = 1.0;
}
template <class T>
__device__ __forceinline__ void stf(T* p, Nd n, typename ident<T>::type v) {
    auto b = uniform_base(p + n.base) + n.off * (uint32_t)sizeof(T);
    *reinterpret_cast<__attribute__((address_space(1))) T*>(b) = v;
}
// load of element idx of a block-uniform array p + base (32-bit index)
template <class T>
__device__ __forceinline__ T ldo(const T* p, long base, uint32_t idx) {
    auto b = uniform_base(p + base) + idx * (uint32_t)sizeof(T);
    return *reinterpret_cast<const __attribute__((address_space(1))) T*>(b);
}
// address of field p at node n (for address selects)
template <class T>
__device__ __forceinline__ const T* adf(const T* p, Nd n) {
    return p + n.base + n.off;
}

template <class T>
struct NodeCtx {
    long nb;                   // body nodes
    const uint8_t* chiB;       // [nb] body | interior << 1 | chi_Omega[d] << (2 + d)
    const T* stat;             // static fields [nb][ncs] (a node's fields together)
    int ncs;                   // static fields per node
    const T* stat_int;         // [ncs] values at interior nodes (device copy)
    T sint[10];                // the same values, as kernel arguments
    double edge_frac;          // host bookkeeping: fraction of body-box nodes that
                               // read per-node static fields (not interior)
    // static field q (runtime index) at node i with flags cb (a select of
    // addresses, no branch)
    __device__ __forceinline__ T st(int q, Nd i, uint8_t cb) const {
        const T* a = (cb & 2) ? stat_int + q : stat + (i.base + i.off) * ncs + q;
        return *a;
    }
    // static fields Q0 .. Q0+N-1 at node i: the interior values at interior
    // nodes (no memory access), the node's own fields at the others (one
    // contiguous run), loaded under a branch that waves without edge nodes
    // skip
    template <int Q0, int N>
    __device__ __forceinline__ void st_range(Nd i, uint8_t cb, T* out) const {
#pragma unroll
        for (int k = 0; k < N; ++k) out[k] = sint[Q0 + k];
        if (!(cb & 2)) {
            const uint32_t o = i.off * (uint32_t)ncs + Q0;
#pragma unroll
            for (int k = 0; k < N; ++k) out[k] = ldo(stat, i.base * ncs, o + k);
        }
    }
};

// ============================================================================
// Generators.  Each node is handled in two steps so that a pass can issue the
// loads of a whole group of nodes before the first store of any of them:
//   Ld ld = load(i)               every load for node i, unconditional
//   gen(i, ld, in[NIN])           arithmetic, selects, stores, the inputs
// (all choices are selects; an optional array that is absent is replaced by
// one that is read anyway at the same index).
// ============================================================================

// Bond-based / LPS displacement inputs:  phi u_j  [, phi]  [, phi u_i u_j].
// VV = 1 first applies the embedded-constraint position update (Eq. 83)
//     u <- chi_O [u + dt v + c2 F] + (1 - chi_O) w   (written back to u)
// and, for integrity weights with failure on, lambda <- lambda && W <= Wc
// (Eq. 63, irreversible), written back to lambda.  INNER (VV): an inner step
// of a multi-step call without prescribed displacements (vhalf = 1, w = null
// at compile time): no loads or registers for F and w.
template <class T, int D, int WK, bool WPHI, bool ENERGY, bool VV, bool INNER = false>
struct GenU {
    static constexpr int NIN = D + (WPHI ? 1 : 0) + (ENERGY ? nsym(D) : 0);
    NodeCtx<T> c;
    T* u;                      // [D][nb] (updated in place when VV)
    const uint8_t* lam_in;     // integrity
    uint8_t* lam_out;          // VV + failure: updated integrity
    const T* s;                // scale weight
    const T* v; const T* F; const T* w; const T* W;
    T dt, c2, Wc;
    int fail;                  // VV: apply the failure rule
    // VV: v holds the half-step velocity v + dt/(2 rho) F (a step inside a
    // multi-step call), so the position update needs no F
    int vhalf;
    static_assert(!INNER || VV, "INNER is a Verlet position update");
    // algorithmic bytes moved per body node (reads + writes)
    __host__ double nbytes() const {
        const double t = sizeof(T);
        double b = D * t + 1;
        if (WK == WK_LAMBDA) b += 1;
        if (WK == WK_SCALE) b += t;
        if (VV) {
            b += D * ((INNER || vhalf ? 2 : 3) * t) + (!INNER && w ? D * t : 0.0);
            if (WK == WK_LAMBDA && fail) b += t + 1;
        }
        return b;
    }
    struct Ld {
        T u[D], v[VV ? D : 1], F[(VV && !INNER) ? D : 1], w[(VV && !INNER) ? D : 1];
        uint8_t o[VV ? D : 1];
        uint8_t chiB, lam;
        T s, W;
    };
    __device__ __forceinline__ Ld load(Nd i, uint8_t cb) const {
        Ld L;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const long k = d * c.nb;
            L.u[d] = ldf(u + k, i);
            if constexpr (VV) {
                L.v[d] = ldf(v + k, i);
                // no branch around a load (it would hold back the loads of the
                // node group): with vhalf the F slot re-reads v (a cache hit)
                // and is not used
                if constexpr (!INNER) {
                    L.F[d] = ldf((vhalf ? v : F) + k, i);
                    L.w[d] = ldf((w ? w : u) + k, i);
                }
                L.o[d] = omega_bit(cb, d);
            }
        }
        L.chiB = cb;
        L.lam = (WK == WK_LAMBDA) ? ldf(lam_in, i) : uint8_t(1);
        L.s = (WK == WK_SCALE) ? ldf(s, i) : T(1);
        L.W = (VV && WK == WK_LAMBDA) ? ldf(W, i) : T(0);
        return L;
    }
    __device__ __forceinline__ void gen(Nd i, const Ld& L, T (&in)[NIN]) const {
        T ud[D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            T x = L.u[d];
            if constexpr (VV && INNER) {
                const T xn = x + dt * L.v[d];
                x = L.o[d] ? xn : T(0);
                stf(u + d * c.nb, i, x);
            } else if constexpr (VV) {
                const T Fs = vhalf ? T(0) : L.F[d];
                const T xn = x + dt * L.v[d] + c2 * Fs;
                x = L.o[d] ? xn : (w ? L.w[d] : T(0));
                stf(u + d * c.nb, i, x);
            }
            ud[d] = x;
        }
        uint8_t l = L.lam;
        if constexpr (VV && WK == WK_LAMBDA) {
            const uint8_t keep = (l != 0 && L.W <= Wc) ? 1 : 0;
            if (fail) {
                l = keep;
                stf(lam_out, i, l);
            }
        }
        T phi = (L.chiB && l) ? T(1) : T(0);
        if constexpr (WK == WK_SCALE) phi *= L.s;
#pragma unroll
        for (int d = 0; d < D; ++d) in[d] = phi * ud[d];
        int o = D;
        if constexpr (WPHI) in[o++] = phi;
        if constexpr (ENERGY) {
#pragma unroll
            for (int a = 0; a < D; ++a)
#pragma unroll
                for (int b = a; b < D; ++b) in[o + symi(D, a, b)] = phi * ud[a] * ud[b];
        }
    }
};

// LPS stage B input: chi_B theta.
template <class T>
struct GenTheta {
    static constexpr int NIN = 1;
    NodeCtx<T> c;
    const T* theta;
    __host__ double nbytes() const { return sizeof(T) + 1.0; }
    struct Ld { T th; uint8_t chiB; };
    __device__ __forceinline__ Ld load(Nd i, uint8_t cb) const { return {ldf(theta, i), cb}; }
    __device__ __forceinline__ void gen(Nd, const Ld& L, T (&in)[1]) const { in[0] = L.chiB ? L.th : T(0); }
};

// Nonlinear bond-based inputs (Sec. 3.2): with h = |u|^2 / 2 and the mask chi,
//   chi u_j (D) | chi h (1) | chi u_a u_b, a <= b (nsym) | chi h u_i (D).
template <class T, int D>
struct GenNBB {
    static constexpr int NIN = 2 * D + 1 + nsym(D);
    NodeCtx<T> c;
    const T* u;
    __host__ double nbytes() const { return D * sizeof(T) + 1.0; }
    struct Ld { T u[D]; uint8_t chiB; };
    __device__ __forceinline__ Ld load(Nd i, uint8_t cb) const {
        Ld L;
#pragma unroll
        for (int d = 0; d < D; ++d) L.u[d] = ldf(u + d * c.nb, i);
        L.chiB = cb;
        return L;
    }
    __device__ __forceinline__ void gen(Nd, const Ld& L, T (&in)[NIN]) const {
        const T chi = L.chiB ? T(1) : T(0);
        T h = T(0);
#pragma unroll
        for (int d = 0; d < D; ++d) h += L.u[d] * L.u[d];
        h *= T(0.5);
        const T ch = chi * h;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            in[d] = chi * L.u[d];
            in[D + 1 + nsym(D) + d] = ch * L.u[d];
        }
        in[D] = ch;
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int b = a; b < D; ++b) in[D + 1 + symi(D, a, b)] = chi * L.u[a] * L.u[b];
    }
};

// Damage count input: chi_B lambda.
template <class T>
struct GenPhi {
    static constexpr int NIN = 1;
    NodeCtx<T> c;
    const uint8_t* lam;
    __host__ double nbytes() const { return 2.0; }
    struct Ld { uint8_t chiB, lam; };
    __device__ __forceinline__ Ld load(Nd i, uint8_t cb) const { return {cb, ldf(lam, i)}; }
    __device__ __forceinline__ void gen(Nd, const Ld& L, T (&in)[1]) const {
        in[0] = (L.chiB && L.lam) ? T(1) : T(0);
    }
};

// Weighted bond-based adjoint inputs: phi u_j, phi, phi g_i, and
// phi (g_i u_j + g_j u_i) for i < j, phi g_i u_i on the diagonal.
template <class T, int D, int WK>
struct GenAdj {
    static constexpr int NIN = 2 * D + 1 + nsym(D);
    NodeCtx<T> c;
    const T* u; const T* u2; const T* g; const uint8_t* lam; const T* s;
    __host__ double nbytes() const {
        const double t = sizeof(T);
        return (2 * D + (u2 ? D : 0)) * t + 1 + (WK == WK_SCALE ? t : 0.0) + (WK == WK_LAMBDA ? 1.0 : 0.0);
    }
    struct Ld { T u[D], u2[D], g[D]; uint8_t chiB, lam; T s; };
    __device__ __forceinline__ Ld load(Nd i, uint8_t cb) const {
        Ld L;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            L.u[d] = ldf(u + d * c.nb, i);
            L.u2[d] = ldf((u2 ? u2 : u) + d * c.nb, i);
            L.g[d] = ldf(g + d * c.nb, i);
        }
        L.chiB = cb;
        L.lam = (WK == WK_LAMBDA) ? ldf(lam, i) : uint8_t(1);
        L.s = (WK == WK_SCALE) ? ldf(s, i) : T(1);
        return L;
    }
    __device__ __forceinline__ void gen(Nd, const Ld& L, T (&in)[NIN]) const {
        T phi = (L.chiB && L.lam) ? T(1) : T(0);
        if constexpr (WK == WK_SCALE) phi *= L.s;
        T ud[D], gd[D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            ud[d] = L.u[d] + (u2 ? L.u2[d] : T(0));
            gd[d] = L.g[d];
            in[d] = phi * ud[d];
            in[D + 1 + d] = phi * gd[d];
        }
        in[D] = phi;
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int b = a; b < D; ++b)
                in[2 * D + 1 + symi(D, a, b)] = (a == b) ? phi * gd[a] * ud[a]
                                                         : phi * (gd[a] * ud[b] + gd[b] * ud[a]);
    }
};

// Plain scalar field (tests).
template <class T>
struct GenScalar {
    static constexpr int NIN = 1;
    const T* x;
    __device__ __forceinline__ uint8_t flags(Nd) const { return 0; }
    __host__ double nbytes() const { return sizeof(T); }
    struct Ld { T x; };
    __device__ __forceinline__ Ld load(Nd i, uint8_t cb) const { return {ldf(x, i)}; }
    __device__ __forceinline__ void gen(Nd, const Ld& L, T (&in)[1]) const { in[0] = L.x; }
};

// ============================================================================
// Multipliers: mul(K, kz, in, out); K[c] is the real kernel sum of component
// C0 + c at this wavenumber.
// ============================================================================

template <class T>
__device__ __forceinline__ cx<T> kmul(T k, cx<T> a) { return {k * a.r, k * a.i}; }
// multiply by i k
template <class T>
__device__ __forceinline__ cx<T> kmuli(T k, cx<T> a) { return {-k * a.i, k * a.r}; }

// One term of a multiplier, for the direct last-axis pass: output O takes
// coef * i^ipow * [ka] * (component c applied to input J).  coef == 0: none.
struct DTerm {
    int c, coef, ipow;
    bool ka;
};
__host__ __device__ constexpr bool sym_diag(int D, int c) {
    return c == 0 || (D == 2 ? c == 2 : (c == 3 || c == 5));
}
// Odd axes of the tensor component C_ij stored at symi(D, i, j): bit d set
// when exactly one of i, j equals d (xi_i xi_j / r^2 changes sign with o_d).
__host__ __device__ constexpr int sym_par(int D, int c) {
    for (int i = 0; i < D; ++i)
        for (int j = i; j < D; ++j)
            if (symi(D, i, j) == c) return (1 << i) ^ (1 << j);
    return 0;
}

// Bond-based: conv_i = sum_j M[C_ij] U_j; [G_c = M[C_c] Phi]; [E = sum_c m_c M[C_c] F_c]
// with M[C_ij] = K (i == j) or -K (i != j: two odd axes, i^2 = -1).
template <class T, int D, bool WPHI, bool ENERGY>
struct MulBB {
    static constexpr int NIN = D + (WPHI ? 1 : 0) + (ENERGY ? nsym(D) : 0);
    static constexpr int NOUT = D + (WPHI ? nsym(D) : 0) + (ENERGY ? 1 : 0);
    static constexpr int C0 = 0, NC = nsym(D);
    // components odd along the last axis (y in 2D: C_xy; z in 3D: C_xz, C_yz)
    static constexpr bool RT_ODD = false;
    static constexpr uint32_t ODD = (D == 2) ? (1u << 1) : ((1u << 2) | (1u << 4));
    __device__ __forceinline__ T ka_value() const { return T(0); }
    // odd axes (bits x, y, z) of component C0 + c
    static constexpr int DIM = D;
    __host__ __device__ static constexpr int par3(int c) { return sym_par(D, c); }
    __host__ __device__ static constexpr DTerm dterm(int O, int J) {
        if (O < D) return J < D ? DTerm{symi(D, O, J), O == J ? 1 : -1, 0, false} : DTerm{0, 0, 0, false};
        if (WPHI && O < D + nsym(D)) return J == D ? DTerm{O - D, sym_diag(D, O - D) ? 1 : -1, 0, false}
                                                   : DTerm{0, 0, 0, false};
        const int ib = D + (WPHI ? 1 : 0);
        if (J < ib || J >= ib + nsym(D)) return DTerm{0, 0, 0, false};
        return DTerm{J - ib, sym_diag(D, J - ib) ? 1 : -2, 0, false};
    }
    // components output O depends on
    template <int O>
    __host__ __device__ static constexpr uint32_t need() {
        if (O < D) {
            uint32_t m = 0;
            for (int j = 0; j < D; ++j) m |= 1u << symi(D, O, j);
            return m;
        }
        if (WPHI && O < D + nsym(D)) return 1u << (O - D);
        return (1u << nsym(D)) - 1u;
    }
    template <int O>
    __device__ __forceinline__ cx<T> one(const T* K, const cx<T>* in) const {
        cx<T> acc = {T(0), T(0)};
        if constexpr (O < D) {
#pragma unroll
            for (int j = 0; j < D; ++j) {
                T k = (O == j) ? K[symi(D, O, j)] : -K[symi(D, O, j)];
                acc = acc + kmul(k, in[j]);
            }
        } else if constexpr (WPHI && O < D + nsym(D)) {
            constexpr int c = O - D;
            constexpr bool diag = (c == 0) || (D == 2 ? c == 2 : (c == 3 || c == 5));
            acc = kmul(diag ? K[c] : -K[c], in[D]);
        } else {
            const int ib = D + (WPHI ? 1 : 0);
#pragma unroll
            for (int a = 0; a < D; ++a)
#pragma unroll
                for (int b = a; b < D; ++b) {
                    T k = (a == b) ? K[symi(D, a, b)] : -T(2) * K[symi(D, a, b)];
                    acc = acc + kmul(k, in[ib + symi(D, a, b)]);
                }
        }
        return acc;
    }
    __device__ __forceinline__ void mul(const T* K, int, const cx<T>* in, cx<T>* out) const {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            cx<T> acc = {T(0), T(0)};
#pragma unroll
            for (int j = 0; j < D; ++j) {
                T k = (i == j) ? K[symi(D, i, j)] : -K[symi(D, i, j)];
                acc = acc + kmul(k, in[j]);
            }
            out[i] = acc;
        }
        int o = D;
        if constexpr (WPHI) {
#pragma unroll
            for (int a = 0; a < D; ++a)
#pragma unroll
                for (int b = a; b < D; ++b) {
                    T k = (a == b) ? K[symi(D, a, b)] : -K[symi(D, a, b)];
                    out[o + symi(D, a, b)] = kmul(k, in[D]);
                }
            o += nsym(D);
        }
        if constexpr (ENERGY) {
            const int ib = D + (WPHI ? 1 : 0);
            cx<T> acc = {T(0), T(0)};
#pragma unroll
            for (int a = 0; a < D; ++a)
#pragma unroll
                for (int b = a; b < D; ++b) {
                    T k = (a == b) ? K[symi(D, a, b)] : -T(2) * K[symi(D, a, b)];
                    acc = acc + kmul(k, in[ib + symi(D, a, b)]);
                }
            out[o] = acc;
        }
    }
};

// LPS dilatation convolution: S = sum_i M[a0_i] U_i, M[a0_i] = i K.
template <class T>
struct MulLPSA {
    static constexpr int NIN = 3, NOUT = 1, C0 = 6, NC = 3;
    static constexpr bool RT_ODD = false;
    static constexpr uint32_t ODD = (1u << 2) | (1u << 4) | (1u << 8);
    __device__ __forceinline__ T ka_value() const { return T(0); }
    static constexpr int DIM = 3;
    __host__ __device__ static constexpr int par3(int c) { return 1 << c; }   // a0_c = omega xi_c
    __host__ __device__ static constexpr DTerm dterm(int, int J) { return DTerm{J, 1, 1, false}; }
    template <int O>
    __host__ __device__ static constexpr uint32_t need() { return 7u; }
    template <int O>
    __device__ __forceinline__ cx<T> one(const T* K, const cx<T>* in) const {
        cx<T> acc = kmuli(K[0], in[0]);
        acc = acc + kmuli(K[1], in[1]);
        return acc + kmuli(K[2], in[2]);
    }
    __device__ __forceinline__ void mul(const T* K, int, const cx<T>* in, cx<T>* out) const {
        cx<T> acc = kmuli(K[0], in[0]);
        acc = acc + kmuli(K[1], in[1]);
        acc = acc + kmuli(K[2], in[2]);
        out[0] = acc;
    }
};

// LPS force convolutions: conv_i = sum_j M[C_ij] U_j + k_a M[a0_i] Theta.
template <class T>
struct MulLPSB {
    static constexpr int NIN = 4, NOUT = 3, C0 = 0, NC = 9;
    static constexpr bool RT_ODD = false;
    static constexpr uint32_t ODD = (1u << 2) | (1u << 4) | (1u << 8);
    __device__ __forceinline__ T ka_value() const { return ka; }
    static constexpr int DIM = 3;
    // components: C_ij (0..5), a0_i (6..8); in the (y, z) taps also k_a a0_i (9..11)
    __host__ __device__ static constexpr int par3(int c) {
        return c < 6 ? sym_par(3, c) : 1 << (c < 9 ? c - 6 : c - 9);
    }
    __host__ __device__ static constexpr DTerm dterm(int O, int J) {
        return J < 3 ? DTerm{symi(3, O, J), O == J ? 1 : -1, 0, false} : DTerm{6 + O, 1, 1, true};
    }
    // the (y, z) pass reads k_a a0_i from the scaled components instead
    __host__ __device__ static constexpr DTerm dterm_yz(int O, int J) {
        return J < 3 ? dterm(O, J) : DTerm{9 + O, 1, 1, false};
    }
    T ka;
    template <int O>
    __host__ __device__ static constexpr uint32_t need() {
        return (1u << symi(3, O, 0)) | (1u << symi(3, O, 1)) | (1u << symi(3, O, 2)) | (1u << (6 + O));
    }
    template <int O>
    __device__ __forceinline__ cx<T> one(const T* K, const cx<T>* in) const {
        cx<T> acc = kmuli(ka * K[6 + O], in[3]);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            T k = (O == j) ? K[symi(3, O, j)] : -K[symi(3, O, j)];
            acc = acc + kmul(k, in[j]);
        }
        return acc;
    }
    __device__ __forceinline__ void mul(const T* K, int, const cx<T>* in, cx<T>* out) const {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            cx<T> acc = kmuli(ka * K[6 + i], in[3]);
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                T k = (i == j) ? K[symi(3, i, j)] : -K[symi(3, i, j)];
                acc = acc + kmul(k, in[j]);
            }
            out[i] = acc;
        }
    }
};

// Nonlinear bond-based multiplier (Sec. 3.2, the convolution form of
// Eq. 21-26 read with xi = x' - x).  Kernel components: C_ab =
// c xi_a xi_b (nsym), a_i = c xi_i (D), c = alpha omega / |xi|^2 (1), all
// with dV.  Inputs as GenNBB.  Outputs, every sum that the force later
// multiplies by the same local factor formed here in spectral space:
//   D_i  = sum_j C_ij (*) chi u_j + a_i (*) chi h + sum_j a_j (*) chi u_j u_i
//          + c (*) chi h u_i                                          (D)
//   S_ab = a_a (*) chi u_b + a_b (*) chi u_a + c (*) chi u_a u_b      (nsym)
//   t    = sum_j a_j (*) chi u_j + c (*) chi h                        (1)
//   c_j  = c (*) chi u_j                                              (D)
// Every (output, input) pair has at most one term: a multiple of the raw
// correlation with one component, whose multiplier is i^(#odd axes) times
// its real sum.
template <class T, int D>
struct MulNBB {
    static constexpr int NIN = 2 * D + 1 + nsym(D);
    static constexpr int NOUT = D + nsym(D) + 1 + D;
    static constexpr int C0 = 0, NC = nsym(D) + D + 1;
    static constexpr int DIM = D;
    static constexpr int CA = nsym(D), CC = nsym(D) + D;   // first a_i, the scalar c
    static constexpr bool RT_ODD = false;
    __host__ __device__ static constexpr int par3(int cc) {
        return cc < CA ? sym_par(D, cc) : (cc < CC ? 1 << (cc - CA) : 0);
    }
    // components odd along the last axis: C_xy, a_y (2D); C_xz, C_yz, a_z (3D)
    static constexpr uint32_t ODD = (D == 2) ? ((1u << 1) | (1u << 4)) : ((1u << 2) | (1u << 4) | (1u << 8));
    __device__ __forceinline__ T ka_value() const { return T(0); }
    __host__ __device__ static constexpr int npar3(int p) { return (p & 1) + ((p >> 1) & 1) + ((p >> 2) & 1); }
    // f times the raw correlation with component cc: f i^(#odd axes) K_cc
    __host__ __device__ static constexpr DTerm raw(int cc, int f = 1) {
        const int n = npar3(par3(cc));
        return DTerm{cc, (n & 2) ? -f : f, n & 1, false};
    }
    __host__ __device__ static constexpr DTerm dterm(int O, int J) {
        constexpr DTerm none{0, 0, 0, false};
        constexpr int JH = D, JU2 = D + 1, JHU = D + 1 + nsym(D);
        constexpr int OS = D, OT = D + nsym(D), OC = D + nsym(D) + 1;
        if (O < OS) {
            const int i = O;
            if (J < D) return raw(symi(D, i, J));
            if (J == JH) return raw(CA + i);
            if (J < JHU) {
                for (int a = 0; a < D; ++a)
                    for (int b = a; b < D; ++b)
                        if (JU2 + symi(D, a, b) == J) {
                            if (a == i) return raw(CA + b);
                            if (b == i) return raw(CA + a);
                        }
                return none;
            }
            return (J - JHU == i) ? raw(CC) : none;
        }
        if (O < OT) {
            for (int a = 0; a < D; ++a)
                for (int b = a; b < D; ++b)
                    if (OS + symi(D, a, b) == O) {
                        if (J == JU2 + symi(D, a, b)) return raw(CC);
                        if (a == b) return J == a ? raw(CA + a, 2) : none;
                        if (J == b) return raw(CA + a);
                        if (J == a) return raw(CA + b);
                    }
            return none;
        }
        if (O == OT) return J < D ? raw(CA + J) : (J == JH ? raw(CC) : none);
        return J == O - OC ? raw(CC) : none;
    }
    template <int O>
    __host__ __device__ static constexpr uint32_t need() {
        uint32_t m = 0;
        for (int J = 0; J < NIN; ++J)
            if (dterm(O, J).coef != 0) m |= 1u << dterm(O, J).c;
        return m;
    }
    template <int O>
    __device__ __forceinline__ cx<T> one(const T* K, const cx<T>* in) const {
        cx<T> acc = {T(0), T(0)};
#pragma unroll
        for (int J = 0; J < NIN; ++J) {
            const DTerm t = dterm(O, J);
            if (t.coef == 0) continue;
            const T k = T(t.coef) * K[t.c];
            acc = acc + (t.ipow ? kmuli(k, in[J]) : kmul(k, in[J]));
        }
        return acc;
    }
    template <int O>
    __device__ __forceinline__ void mul_from(const T* K, const cx<T>* in, cx<T>* out) const {
        if constexpr (O < NOUT) {
            out[O] = one<O>(K, in);
            mul_from<O + 1>(K, in, out);
        }
    }
    __device__ __forceinline__ void mul(const T* K, int, const cx<T>* in, cx<T>* out) const {
        mul_from<0>(K, in, out);
    }
};

// Damage count: omega_0 (*) (chi_B lambda) over the bonds (centre excluded).
template <class T, int D>
struct MulCount {
    static constexpr int NIN = 1, NOUT = 1, C0 = nsym(D), NC = 1;
    static constexpr bool RT_ODD = false;
    static constexpr uint32_t ODD = 0u;
    __device__ __forceinline__ T ka_value() const { return T(0); }
    static constexpr int DIM = D;
    __host__ __device__ static constexpr int par3(int) { return 0; }
    __host__ __device__ static constexpr DTerm dterm(int, int) { return DTerm{0, 1, 0, false}; }
    template <int O>
    __host__ __device__ static constexpr uint32_t need() { return 1u; }
    template <int O>
    __device__ __forceinline__ cx<T> one(const T* K, const cx<T>* in) const { return kmul(K[0], in[0]); }
    __device__ __forceinline__ void mul(const T* K, int, const cx<T>* in, cx<T>* out) const {
        out[0] = kmul(K[0], in[0]);
    }
};

// Weighted bond-based adjoint: conv_i (D), G_c (nsym), cg_i = C (*) phi g (D),
// E' = sum_c M[C_c] F(s_c) (1).
template <class T, int D>
struct MulAdj {
    static constexpr int NIN = 2 * D + 1 + nsym(D);
    static constexpr int NOUT = 2 * D + nsym(D) + 1;
    static constexpr int C0 = 0, NC = nsym(D);
    static constexpr bool RT_ODD = false;
    static constexpr uint32_t ODD = (D == 2) ? (1u << 1) : ((1u << 2) | (1u << 4));
    __device__ __forceinline__ T ka_value() const { return T(0); }
    static constexpr int DIM = D;
    __host__ __device__ static constexpr int par3(int c) { return sym_par(D, c); }
    __host__ __device__ static constexpr DTerm dterm(int O, int J) {
        if (O < D) return J < D ? DTerm{symi(D, O, J), O == J ? 1 : -1, 0, false} : DTerm{0, 0, 0, false};
        if (O < D + nsym(D)) return J == D ? DTerm{O - D, sym_diag(D, O - D) ? 1 : -1, 0, false}
                                           : DTerm{0, 0, 0, false};
        if (O < 2 * D + nsym(D)) {
            const int i = O - D - nsym(D), j = J - (D + 1);
            return (j >= 0 && j < D) ? DTerm{symi(D, i, j), i == j ? 1 : -1, 0, false} : DTerm{0, 0, 0, false};
        }
        const int q = J - (2 * D + 1);
        return (q >= 0 && q < nsym(D)) ? DTerm{q, sym_diag(D, q) ? 1 : -1, 0, false} : DTerm{0, 0, 0, false};
    }
    // outputs: conv_i (D) | G_c (nsym) | cg_i (D) | E' (1)
    template <int O>
    __host__ __device__ static constexpr uint32_t need() {
        if (O < D || (O >= D + nsym(D) && O < 2 * D + nsym(D))) {
            const int i = O < D ? O : O - D - nsym(D);
            uint32_t m = 0;
            for (int j = 0; j < D; ++j) m |= 1u << symi(D, i, j);
            return m;
        }
        if (O < D + nsym(D)) return 1u << (O - D);
        return (1u << nsym(D)) - 1u;
    }
    template <int O>
    __device__ __forceinline__ cx<T> one(const T* K, const cx<T>* in) const {
        cx<T> acc = {T(0), T(0)};
        if constexpr (O < D || (O >= D + nsym(D) && O < 2 * D + nsym(D))) {
            constexpr int i = O < D ? O : O - D - nsym(D);
            constexpr int base = O < D ? 0 : D + 1;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                T k = (i == j) ? K[symi(D, i, j)] : -K[symi(D, i, j)];
                acc = acc + kmul(k, in[base + j]);
            }
        } else if constexpr (O < D + nsym(D)) {
            constexpr int c = O - D;
            constexpr bool diag = (c == 0) || (D == 2 ? c == 2 : (c == 3 || c == 5));
            acc = kmul(diag ? K[c] : -K[c], in[D]);
        } else {
#pragma unroll
            for (int p = 0; p < D; ++p)
#pragma unroll
                for (int q = p; q < D; ++q) {
                    T k = (p == q) ? K[symi(D, p, q)] : -K[symi(D, p, q)];
                    acc = acc + kmul(k, in[2 * D + 1 + symi(D, p, q)]);
                }
        }
        return acc;
    }
    __device__ __forceinline__ void mul(const T* K, int, const cx<T>* in, cx<T>* out) const {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            cx<T> a = {T(0), T(0)}, b = {T(0), T(0)};
#pragma unroll
            for (int j = 0; j < D; ++j) {
                T k = (i == j) ? K[symi(D, i, j)] : -K[symi(D, i, j)];
                a = a + kmul(k, in[j]);
                b = b + kmul(k, in[D + 1 + j]);
            }
            out[i] = a;
            out[D + nsym(D) + i] = b;
        }
        cx<T> e = {T(0), T(0)};
#pragma unroll
        for (int p = 0; p < D; ++p)
#pragma unroll
            for (int q = p; q < D; ++q) {
                T k = (p == q) ? K[symi(D, p, q)] : -K[symi(D, p, q)];
                out[D + symi(D, p, q)] = kmul(k, in[D]);
                e = e + kmul(k, in[2 * D + 1 + symi(D, p, q)]);
            }
        out[2 * D + nsym(D)] = e;
    }
};

// Spectral preconditioner of the static solve: the inverse of the periodic,
// unmasked bond-based symbol (Ĉ(0) - M[C](k), the operator -L of the same
// kernel on the full periodic box, shifted by a multiple of the identity so
// that k = 0 is invertible), applied per wavenumber.  It is nonlocal along
// the last axis, so only the transform form of the last-axis pass applies.
// In tap units (Ĉ/Nfft), normalised by s0: out = (S')^-1 in * outscale with
// S' = k0n - kscale M[C](k), k0n = (Ĉ(0) + shift)/ (Nfft s0).
template <class T, int D>
struct MulPre {
    static constexpr int NIN = D, NOUT = D, C0 = 0, NC = nsym(D);
    static constexpr bool RT_ODD = false, NONLOCAL = true;
    static constexpr uint32_t ODD = (D == 2) ? (1u << 1) : ((1u << 2) | (1u << 4));
    T k0n[3];
    T kscale, outscale;
    __device__ __forceinline__ T ka_value() const { return T(0); }
    __host__ __device__ static constexpr DTerm dterm(int, int) { return DTerm{0, 0, 0, false}; }
    template <int O>
    __host__ __device__ static constexpr uint32_t need() { return (1u << nsym(D)) - 1u; }
    template <int O>
    __device__ __forceinline__ cx<T> one(const T* K, const cx<T>* in) const {
        // S'_ij = k0n_i [i == j] - kscale * (i == j ? K : -K)_ij  (symmetric)
        auto Sij = [&](int i, int j) {
            const T m = (i == j) ? K[symi(D, i, j)] : -K[symi(D, i, j)];
            return (i == j ? k0n[i] : T(0)) - kscale * m;
        };
        if constexpr (D == 2) {
            const T a = Sij(0, 0), b = Sij(1, 1), d = Sij(0, 1);
            const T inv = outscale / (a * b - d * d);
            const T r0 = (O == 0) ? b : -d, r1 = (O == 0) ? -d : a;
            return cscale(kmul(r0, in[0]) + kmul(r1, in[1]), inv);
        } else {
            const T a = Sij(0, 0), b = Sij(1, 1), c = Sij(2, 2);
            const T d = Sij(0, 1), e = Sij(0, 2), f = Sij(1, 2);
            // cofactors of the symmetric matrix [[a d e] [d b f] [e f c]]
            const T A00 = b * c - f * f, A01 = e * f - d * c, A02 = d * f - e * b;
            const T A11 = a * c - e * e, A12 = d * e - a * f, A22 = a * b - d * d;
            const T inv = outscale / (a * A00 + d * A01 + e * A02);
            T r0, r1, r2;
            if constexpr (O == 0) { r0 = A00; r1 = A01; r2 = A02; }
            else if constexpr (O == 1) { r0 = A01; r1 = A11; r2 = A12; }
            else { r0 = A02; r1 = A12; r2 = A22; }
            return cscale(kmul(r0, in[0]) + kmul(r1, in[1]) + kmul(r2, in[2]), inv);
        }
    }
    // All outputs from one evaluation of the symbol and its inverse (the
    // last-axis pass uses this when a multiplier provides it).
    __device__ __forceinline__ void all(const T* K, const cx<T>* in, cx<T>* out) const {
        auto Sij = [&](int i, int j) {
            const T m = (i == j) ? K[symi(D, i, j)] : -K[symi(D, i, j)];
            return (i == j ? k0n[i] : T(0)) - kscale * m;
        };
        if constexpr (D == 2) {
            const T a = Sij(0, 0), b = Sij(1, 1), d = Sij(0, 1);
            const T inv = outscale / (a * b - d * d);
            out[0] = cscale(kmul(b, in[0]) + kmul(-d, in[1]), inv);
            out[1] = cscale(kmul(-d, in[0]) + kmul(a, in[1]), inv);
        } else {
            const T a = Sij(0, 0), b = Sij(1, 1), c = Sij(2, 2);
            const T d = Sij(0, 1), e = Sij(0, 2), f = Sij(1, 2);
            const T A00 = b * c - f * f, A01 = e * f - d * c, A02 = d * f - e * b;
            const T A11 = a * c - e * e, A12 = d * e - a * f, A22 = a * b - d * d;
            const T inv = outscale / (a * A00 + d * A01 + e * A02);
            out[0] = cscale(kmul(A00, in[0]) + kmul(A01, in[1]) + kmul(A02, in[2]), inv);
            out[1] = cscale(kmul(A01, in[0]) + kmul(A11, in[1]) + kmul(A12, in[2]), inv);
            out[2] = cscale(kmul(A02, in[0]) + kmul(A12, in[1]) + kmul(A22, in[2]), inv);
        }
    }
};

// Preconditioner input: chi_O r (r in TR, converted to the chain type).
template <class T, int D, class TR>
struct GenMasked {
    static constexpr int NIN = D;
    NodeCtx<T> c;
    const TR* r;
    __host__ double nbytes() const { return D * double(sizeof(TR)) + 1.0; }
    struct Ld { TR r[D]; uint8_t o[D]; };
    __device__ __forceinline__ Ld load(Nd i, uint8_t cb) const {
        Ld L;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            L.r[d] = ldf(r + d * c.nb, i);
            L.o[d] = omega_bit(cb, d);
        }
        return L;
    }
    __device__ __forceinline__ void gen(Nd, const Ld& L, T (&in)[D]) const {
#pragma unroll
        for (int d = 0; d < D; ++d) in[d] = L.o[d] ? T(L.r[d]) : T(0);
    }
};

// Test multiplier: a single kernel component odd in P axes, i^P K.
template <class T>
struct MulTest {
    static constexpr int NIN = 1, NOUT = 1, C0 = 0, NC = 1;
    static constexpr bool RT_ODD = true;   // parity comes with the test kernel
    static constexpr uint32_t ODD = 0u;
    __device__ __forceinline__ T ka_value() const { return T(0); }
    int P;
    template <int O>
    __host__ __device__ static constexpr uint32_t need() { return 1u; }
    template <int O>
    __device__ __forceinline__ cx<T> one(const T* K, const cx<T>* in) const {
        return mul_ipow(kmul(K[0], in[0]), P);
    }
    __device__ __forceinline__ void mul(const T* K, int, const cx<T>* in, cx<T>* out) const {
        out[0] = mul_ipow(kmul(K[0], in[0]), P);
    }
};

// ============================================================================
// Epilogues, in two steps like the generators:
//   Ld ld = load(i)                 every load for node i, unconditional
//   fin(i, ld, val[NOUT], red)      val are the (normalised) convolutions at
//                                   node i; arithmetic, selects, stores and
//                                   the partial sums red[NRED]
// ============================================================================

// Bond-based force / Verlet finish.
//   L_i = phi (conv_i - sum_j G_ij u_j)          (Eq. 18, 46, 100 with weights)
//   W   = 1/2 phi (E - 2 u_j conv_j + u_i u_j G_ij) (Eq. 47, 102)
// G is the static chi_B field (WPHI = false) or comes from the chain.
// VV: F' = L + b, v <- chi_O [v + c1 (F + F')]  (Eq. 84); optional energy
// partial sums (KE, PE, EXT, |chi_O F'|^2).
template <class T, int D, int WK, bool WPHI, bool ENERGY, bool VV, bool ENRED>
struct FinBB {
    static constexpr int NOUT = D + (WPHI ? nsym(D) : 0) + (ENERGY ? 1 : 0);
    static constexpr int NRED = ENRED ? 4 : 0;
    NodeCtx<T> c;
    const T* u; const uint8_t* lam; const T* s;
    T* L; T* Wout;
    T* v; T* F; const T* b;   // VV
    T c1, rho;
    double* nanflag;          // VV: set to 1 on a non-finite F' or v (null: no check)
    int vh_in, vh_out;        // VV: half-step velocity in / out (as FinLin)
    __host__ double nbytes() const {
        const double t = sizeof(T);
        double r = D * t + 1 + (WK == WK_LAMBDA ? 1.0 : 0.0) + (WK == WK_SCALE ? t : 0.0);
        if (!WPHI) r += nsym(D) * t * c.edge_frac;
        if (ENERGY) r += t;
        if (VV) r += D * ((2 + (vh_in ? 0 : 1) + (vh_out ? 0 : 1)) * t) + (b ? D * t : 0.0);
        else r += D * t;
        return r;
    }
    struct Ld {
        T u[D], G[WPHI ? 1 : nsym(D)];
        T v[VV ? D : 1], F[VV ? D : 1], b[VV ? D : 1];
        uint8_t o[VV ? D : 1];
        uint8_t chiB, lam;
        T s;
    };
    __device__ __forceinline__ Ld load(Nd i, uint8_t cb) const {
        Ld Q;
#pragma unroll
        for (int d = 0; d < D; ++d) Q.u[d] = ldf(u + d * c.nb, i);
        if constexpr (!WPHI) c.template st_range<0, nsym(D)>(i, cb, Q.G);
        if constexpr (VV) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const long k = d * c.nb;
                Q.v[d] = ldf(v + k, i);
                Q.F[d] = ldf((vh_in ? v : F) + k, i);   // with vh_in: a cache hit, unused
                Q.o[d] = omega_bit(cb, d);
            }
            if (b) {   // kernel-uniform
#pragma unroll
                for (int d = 0; d < D; ++d) Q.b[d] = ldf(b + d * c.nb, i);
            }
        }
        Q.chiB = cb;
        Q.lam = (WK == WK_LAMBDA) ? ldf(lam, i) : uint8_t(1);
        Q.s = (WK == WK_SCALE) ? ldf(s, i) : T(1);
        return Q;
    }
    __device__ __forceinline__ void fin(Nd i, const Ld& Q, const T (&val)[NOUT], double* red) const {
        T phi = (Q.chiB && Q.lam) ? T(1) : T(0);
        if constexpr (WK == WK_SCALE) phi *= Q.s;
        T Gm[nsym(D)];
#pragma unroll
        for (int q = 0; q < nsym(D); ++q) Gm[q] = WPHI ? val[D + q] : Q.G[WPHI ? 0 : q];
        T Li[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            T acc = val[a];
#pragma unroll
            for (int bb = 0; bb < D; ++bb) acc -= Gm[symi(D, a, bb)] * Q.u[bb];
            Li[a] = phi * acc;
        }
        if constexpr (ENERGY) {
            T e = val[D + (WPHI ? nsym(D) : 0)];
#pragma unroll
            for (int a = 0; a < D; ++a) {
                e -= T(2) * Q.u[a] * val[a];
#pragma unroll
                for (int bb = 0; bb < D; ++bb) e += Q.u[a] * Q.u[bb] * Gm[symi(D, a, bb)];
            }
            stf(Wout, i, T(0.5) * phi * e);
        }
        if constexpr (VV) {
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const long k = a * c.nb;
                const T bk = b ? Q.b[a] : T(0);
                T Fn = Li[a] + bk;
                const T Fo = vh_in ? T(0) : Q.F[a];
                T vn = Q.o[a] ? Q.v[a] + c1 * (Fo + Fn) : T(0);
                if (vh_out) {
                    stf(v + k, i, Q.o[a] ? vn + c1 * Fn : T(0));
                } else {
                    stf(v + k, i, vn);
                    stf(F + k, i, Fn);
                }
                flag_nonfinite(nanflag, Fn, vn);
                if constexpr (ENRED) {
                    red[0] += 0.5 * double(rho) * double(vn) * double(vn);
                    red[1] += -0.5 * double(Q.u[a]) * double(Li[a]);
                    red[2] += -double(bk) * double(Q.u[a]);
                    red[3] += Q.o[a] ? double(Fn) * double(Fn) : 0.0;
                }
            }
        } else {
#pragma unroll
            for (int a = 0; a < D; ++a) stf(L + a * c.nb, i, Li[a]);
        }
    }
};

// LPS dilatation (Eq. 96 with the sign reading of Eq. 93):
//   theta = 3 chi / m (S - g_i u_i),  0 where chi = 0 or m = 0.
template <class T>
struct FinTheta {
    static constexpr int NOUT = 1, NRED = 0;
    NodeCtx<T> c;
    const T* u; T* theta;
    __host__ double nbytes() const { return 4.0 * sizeof(T) + 4.0 * sizeof(T) * c.edge_frac + 1.0; }
    struct Ld { T m, g[3], u[3]; uint8_t chiB; };
    __device__ __forceinline__ Ld load(Nd i, uint8_t cb) const {
        Ld Q;
        T st[4];
        c.template st_range<6, 4>(i, cb, st);
        Q.m = st[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            Q.g[d] = st[d];
            Q.u[d] = ldf(u + d * c.nb, i);
        }
        Q.chiB = cb;
        return Q;
    }
    __device__ __forceinline__ T value(const Ld& Q, T S) const {
        T acc = S;
#pragma unroll
        for (int d = 0; d < 3; ++d) acc -= Q.g[d] * Q.u[d];
        const bool on = Q.chiB && Q.m != T(0);
        return on ? T(3) / (on ? Q.m : T(1)) * acc : T(0);
    }
    __device__ __forceinline__ void fin(Nd i, const Ld& Q, const T (&val)[1], double*) const {
        stf(theta, i, value(Q, val[0]));
    }
};

// The dilatation stage's epilogue chained to the force stage's generator:
// theta stored as by FinTheta and also handed on (chi theta = theta, zero off
// the body) for the r2c of the force stage in the same pass.
template <class T>
struct FinThetaChain : FinTheta<T> {
    static constexpr int NCHAIN = 1;
    __host__ double nbytes() const { return FinTheta<T>::nbytes(); }
    __device__ __forceinline__ void fin_chain(Nd i, const typename FinTheta<T>::Ld& Q, const T (&val)[1], double*,
                                              T (&next)[1]) const {
        const T th = this->value(Q, val[0]);
        stf(this->theta, i, th);
        next[0] = th;
    }
};

// LPS force (Eq. 95 with the sign reading of Eq. 92):
//   L_i = chi (conv_i + k_a theta g_i - G_ij u_j), conv_i including k_a a (*) chi theta.
// MODE 0: write L;  MODE 1: Verlet finish (as FinBB);  MODE 2: CG operator
// Ap = -chi_O L with partial sum p.Ap;  MODE 3: FP64 residual
// r = chi_O (L + b) with partial |r|^2.  INNER (MODE 1): an inner step of a
// multi-step call, vh_in = vh_out = 1 at compile time, so the epilogue keeps
// no registers for F and issues no load for it; it also makes the next
// step's position update u <- chi_O (u + dt vh') (the caller has no
// prescribed displacement w), with u and vh' already in registers; in FP64
// it also hands chi u of the new positions to the pass's forward transform
// (NCHAIN = D: the next step's first stage starts from those spectra).  In
// FP32 the chained pass ran slower than the two passes it replaces (0.440
// against 0.277 + 0.15 ms at 256^3), so there the next step's first pass is
// the plain chi u transform.
template <class T, int D, int MODE, bool ENRED, bool LPS, bool INNER = false>
struct FinLin {
    // Shared by bond-based (static G, LPS = false) and LPS for the solver / VV modes.
    static constexpr int NOUT = D;
    static constexpr int NRED = (MODE == 1) ? (ENRED ? 4 : 0) : ((MODE >= 2) ? 1 : 0);
    // the FP32 velocity-update pass runs 8 rows per block (measured faster
    // than 16 on the 256^3 step; the other x passes are faster with 16)
    static constexpr int XROWS = (MODE == 1 && sizeof(T) == 4) ? 8 : 0;
    NodeCtx<T> c;
    T ka;
    const T* u; const T* theta;
    T* L; T* v; T* F; const T* b;
    T c1, rho;
    T* u_next; T dt;   // INNER: the position update of the next step (u_next = u)
    double* nanflag;   // MODE 1: set to 1 on a non-finite F' or v (null: no check)
    // MODE 1, steps inside a multi-step call: v holds the half-step velocity
    // vh = v + c1 F on entry (vh_in; F is not read) and receives
    // vh' = v' + c1 F' on exit (vh_out; F is not written); both 1 when INNER
    int vh_in, vh_out;
    static_assert(!INNER || (MODE == 1 && !ENRED), "INNER is a Verlet step without energy sums");
    static constexpr int NCHAIN = (INNER && sizeof(T) == 8) ? D : 0;
    __host__ __device__ bool vhi() const { return INNER || vh_in; }
    __host__ __device__ bool vho() const { return INNER || vh_out; }
    __host__ double nbytes() const {
        const double t = sizeof(T);
        double r = D * t + 1 + nsym(D) * t * c.edge_frac + (LPS ? t + D * t * c.edge_frac : 0.0);
        if (MODE == 0) r += D * t;
        else if (MODE == 1) r += D * ((2 + (vhi() ? 0 : 1) + (vho() ? 0 : 1) + (INNER ? 1 : 0)) * t) + (b ? D * t : 0.0);
        else if (MODE == 2) r += D * t;
        else r += D * (2 * t);
        return r;
    }
    static constexpr bool HAS_O = MODE >= 1;
    struct Ld {
        T u[D], G[nsym(D)], g[LPS ? D : 1], th;
        T v[MODE == 1 ? D : 1], F[(MODE == 1 && !INNER) ? D : 1], b[(MODE == 1 || MODE == 3) ? D : 1];
        uint8_t o[HAS_O ? D : 1];
        uint8_t chiB;
    };
    __device__ __forceinline__ Ld load(Nd i, uint8_t cb) const {
        Ld Q;
        Q.chiB = cb;
#pragma unroll
        for (int d = 0; d < D; ++d) Q.u[d] = ldf(u + d * c.nb, i);
        if constexpr (LPS) {
            // G_ij and g_i are consecutive static fields 0 .. 8
            T st[nsym(D) + D];
            c.template st_range<0, nsym(D) + D>(i, cb, st);
#pragma unroll
            for (int q = 0; q < nsym(D); ++q) Q.G[q] = st[q];
#pragma unroll
            for (int d = 0; d < D; ++d) Q.g[d] = st[nsym(D) + d];
            Q.th = ldf(theta, i);
        } else {
            c.template st_range<0, nsym(D)>(i, cb, Q.G);
            Q.th = T(0);
        }
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const long k = d * c.nb;
            if constexpr (HAS_O) Q.o[d] = omega_bit(cb, d);
            if constexpr (MODE == 1) {
                Q.v[d] = ldf(v + k, i);
                if constexpr (!INNER) Q.F[d] = ldf((vh_in ? v : F) + k, i);   // with vh_in: a cache hit, unused
            }
            if constexpr (MODE == 3) Q.b[d] = ldf(b + k, i);
        }
        if constexpr (MODE == 1) {
            if (b) {   // kernel-uniform
#pragma unroll
                for (int d = 0; d < D; ++d) Q.b[d] = ldf(b + d * c.nb, i);
            }
        }
        return Q;
    }
    __device__ __forceinline__ void fin(Nd i, const Ld& Q, const T (&val)[D], double* red) const {
        T next[D];
        apply<false>(i, Q, val, red, next);
    }
    __device__ __forceinline__ void fin_chain(Nd i, const Ld& Q, const T (&val)[D], double* red,
                                              T (&next)[D]) const {
        apply<true>(i, Q, val, red, next);
    }
    template <bool CH>
    __device__ __forceinline__ void apply(Nd i, const Ld& Q, const T (&val)[D], double* red, T (&next)[D]) const {
        const T chi = Q.chiB ? T(1) : T(0);
#pragma unroll
        for (int a = 0; a < D; ++a) {
            T acc = val[a];
#pragma unroll
            for (int bb = 0; bb < D; ++bb) acc -= Q.G[symi(D, a, bb)] * Q.u[bb];
            if constexpr (LPS) acc += ka * Q.th * Q.g[a];
            T La = chi * acc;
            const long k = a * c.nb;
            if constexpr (MODE == 0) {
                stf(L + k, i, La);
            } else if constexpr (MODE == 1) {
                const T bk = b ? Q.b[a] : T(0);
                T Fn = La + bk;
                T Fo = T(0);
                if constexpr (!INNER) Fo = vh_in ? T(0) : Q.F[a];
                const T vf = Q.v[a] + c1 * (Fo + Fn);
                T vn = Q.o[a] ? vf : T(0);
                if (vho()) {
                    const T vh2 = Q.o[a] ? vn + c1 * Fn : T(0);
                    stf(v + k, i, vh2);
                    // the same expressions as the position update and the
                    // chi u input of GenU
                    if constexpr (INNER) {
                        const T un = Q.o[a] ? Q.u[a] + dt * vh2 : T(0);
                        stf(u_next + k, i, un);
                        if constexpr (CH) next[a] = chi * un;
                    }
                } else {
                    stf(v + k, i, vn);
                    stf(F + k, i, Fn);
                }
                flag_nonfinite(nanflag, Fn, vn);
                if constexpr (ENRED) {
                    red[0] += 0.5 * double(rho) * double(vn) * double(vn);
                    red[1] += -0.5 * double(Q.u[a]) * double(La);
                    red[2] += -double(bk) * double(Q.u[a]);
                    red[3] += Q.o[a] ? double(Fn) * double(Fn) : 0.0;
                }
            } else if constexpr (MODE == 2) {
                T ap = Q.o[a] ? -La : T(0);
                stf(L + k, i, ap);
                red[0] += double(Q.u[a]) * double(ap);
            } else {
                T r = Q.o[a] ? La + Q.b[a] : T(0);
                stf(L + k, i, r);
                red[0] += double(r) * double(r);
            }
        }
    }
};

// Nonlinear bond-based force (Sec. 3.2): with h = |u|^2 / 2 and the static
// sums P_ab = C_ab (*) chi, q_i = a_i (*) chi, p = c (*) chi (plan time),
//   L_i = chi [ D_i - sum_j (P_ij + S_ij) u_j - t u_i
//               + sum_j (q_j + c_j) u_j u_i + (q_i + c_i) h - p h u_i ].
template <class T, int D>
struct FinNBB {
    static constexpr int NOUT = D + nsym(D) + 1 + D, NRED = 0;
    NodeCtx<T> c;
    const T* u;
    T* L;
    __host__ double nbytes() const {
        const double t = sizeof(T);
        return 2.0 * D * t + 1.0 + (nsym(D) + D + 1) * t * c.edge_frac;
    }
    struct Ld { T u[D], st[nsym(D) + D + 1]; uint8_t chiB; };
    __device__ __forceinline__ Ld load(Nd i, uint8_t cb) const {
        Ld Q;
#pragma unroll
        for (int d = 0; d < D; ++d) Q.u[d] = ldf(u + d * c.nb, i);
        c.template st_range<0, nsym(D) + D + 1>(i, cb, Q.st);
        Q.chiB = cb;
        return Q;
    }
    __device__ __forceinline__ void fin(Nd i, const Ld& Q, const T (&val)[NOUT], double*) const {
        constexpr int OS = D, OT = D + nsym(D), OC = OT + 1;
        const T chi = Q.chiB ? T(1) : T(0);
        T h = T(0), qcu = T(0);
#pragma unroll
        for (int d = 0; d < D; ++d) {
            h += Q.u[d] * Q.u[d];
            qcu += (Q.st[nsym(D) + d] + val[OC + d]) * Q.u[d];
        }
        h *= T(0.5);
        const T p = Q.st[nsym(D) + D];
        const T lu = qcu - val[OT] - p * h;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            T t = val[a] + lu * Q.u[a] + (Q.st[nsym(D) + a] + val[OC + a]) * h;
#pragma unroll
            for (int j = 0; j < D; ++j) t -= (Q.st[symi(D, a, j)] + val[OS + symi(D, a, j)]) * Q.u[j];
            stf(L + a * c.nb, i, chi * t);
        }
    }
};

// Damage index: cnt = rint(omega_0 (*) phi) + phi(x), beta(x) static,
// d = 1 - phi cnt / beta on chi_B.
template <class T>
struct FinCount {
    static constexpr int NOUT = 1, NRED = 0;
    NodeCtx<T> c;
    int beta_comp;
    const uint8_t* lam; T* d;
    __host__ double nbytes() const { return 2.0 + sizeof(T) + sizeof(T) * c.edge_frac; }
    struct Ld { T st; uint8_t chiB, lam; };
    __device__ __forceinline__ Ld load(Nd i, uint8_t cb) const { return {c.st(beta_comp, i, cb), cb, ldf(lam, i)}; }
    __device__ __forceinline__ void fin(Nd i, const Ld& Q, const T (&val)[1], double*) const {
        int phi = (Q.chiB && Q.lam) ? 1 : 0;
        long cnt = (long)rint(val[0]) + phi;
        long beta = (long)rint(Q.st) + (Q.chiB ? 1 : 0);
        stf(d, i, Q.chiB ? T(1.0 - double(phi * cnt) / double(beta > 0 ? beta : 1)) : T(0));
    }
};

// Weighted bond-based adjoint epilogue:
//   u_bar_i = phi (cg_i - G_ij g_j)
//   phi_bar = g_i (conv_i - G_ij u_j) + u_j cg_j - E'
//   s_bar   = chi_B phi_bar  (scale weights, phi = chi_B s)
template <class T, int D, int WK>
struct FinAdj {
    static constexpr int NOUT = 2 * D + nsym(D) + 1;
    static constexpr int NRED = 0;
    NodeCtx<T> c;
    const T* u; const T* u2; const T* g; const uint8_t* lam; const T* s;
    T* ubar; T* wbar;
    T wscale;       // wbar = wscale * chi_B phi_bar (+ previous value if accumulate)
    int accumulate;
    __host__ double nbytes() const {
        const double t = sizeof(T);
        return (2 * D + (u2 ? D : 0)) * t + 1 + (WK == WK_SCALE ? t : 0.0) + (ubar ? D * t : 0.0) +
               (wbar ? (accumulate ? 2 : 1) * t : 0.0);
    }
    struct Ld { T u[D], u2[D], g[D]; uint8_t chiB, lam; T s, wb; };
    __device__ __forceinline__ Ld load(Nd i, uint8_t cb) const {
        Ld Q;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            Q.u[d] = ldf(u + d * c.nb, i);
            Q.u2[d] = ldf((u2 ? u2 : u) + d * c.nb, i);
            Q.g[d] = ldf(g + d * c.nb, i);
        }
        Q.chiB = cb;
        Q.lam = (WK == WK_LAMBDA) ? ldf(lam, i) : uint8_t(1);
        Q.s = (WK == WK_SCALE) ? ldf(s, i) : T(1);
        Q.wb = (wbar && accumulate) ? ldf(wbar, i) : T(0);
        return Q;
    }
    __device__ __forceinline__ void fin(Nd i, const Ld& Q, const T (&val)[NOUT], double*) const {
        T phi = (Q.chiB && Q.lam) ? T(1) : T(0);
        if constexpr (WK == WK_SCALE) phi *= Q.s;
        T ud[D], gd[D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            ud[d] = Q.u[d] + (u2 ? Q.u2[d] : T(0));
            gd[d] = Q.g[d];
        }
        T pb = -val[2 * D + nsym(D)];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            T acc_u = val[D + nsym(D) + a];
            T acc_c = val[a];
#pragma unroll
            for (int bb = 0; bb < D; ++bb) {
                T Gab = val[D + symi(D, a, bb)];
                acc_u -= Gab * gd[bb];
                acc_c -= Gab * ud[bb];
            }
            if (ubar) stf(ubar + a * c.nb, i, phi * acc_u);
            pb += gd[a] * acc_c + ud[a] * val[D + nsym(D) + a];
        }
        if (wbar) {
            T add = Q.chiB ? wscale * pb : T(0);
            stf(wbar, i, accumulate ? Q.wb + add : add);
        }
    }
};

// Preconditioner output z = chi_O (M^-1 chi_O r), stored as TZ, with the
// partial sum r . z (FP64) for the preconditioned CG.
template <class T, int D, class TR, class TZ>
struct FinPre {
    static constexpr int NOUT = D, NRED = 1;
    NodeCtx<T> c;
    const TR* r;
    TZ* z;
    __host__ double nbytes() const { return D * double(sizeof(TR) + sizeof(TZ)) + 1.0; }
    struct Ld { TR r[D]; uint8_t o[D]; };
    __device__ __forceinline__ Ld load(Nd i, uint8_t cb) const {
        Ld Q;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            Q.r[d] = ldf(r + d * c.nb, i);
            Q.o[d] = omega_bit(cb, d);
        }
        return Q;
    }
    __device__ __forceinline__ void fin(Nd i, const Ld& Q, const T (&val)[D], double* red) const {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const TZ zd = Q.o[d] ? TZ(val[d]) : TZ(0);
            stf(z + d * c.nb, i, zd);
            red[0] += double(Q.r[d]) * double(zd);
        }
    }
};

// Plain scalar output (tests).
template <class T>
struct FinScalar {
    static constexpr int NOUT = 1, NRED = 0;
    T* out;
    __device__ __forceinline__ uint8_t flags(Nd) const { return 0; }
    __host__ double nbytes() const { return sizeof(T); }
    struct Ld {};
    __device__ __forceinline__ Ld load(Nd, uint8_t) const { return {}; }
    __device__ __forceinline__ void fin(Nd i, const Ld&, const T (&val)[1], double*) const { stf(out, i, val[0]); }
};

}  // namespace pdk
