// pd_impl.hpp -- plan creation, convolution chains, elementwise kernels and
// solvers of the FCBM-EC library (internal).  Included by pd_fcbm.hip (the C
// entry points) and by pd_inst.hip, which instantiates the per-dtype
// implementations in units of their own so that they compile in parallel.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <type_traits>
#include <vector>

#include "pd_plan.hpp"

using namespace pdk;


#define PD_TRY(...)                                \
    do {                                           \
        pd_status s_ = (__VA_ARGS__);              \
        if (s_ != PD_OK) return s_;                \
    } while (0)
#define HIP_TRY(x) PD_TRY(pdh::check(x))

namespace pdi {

constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------- plan kernels

// Partial spectra ("taps") of the kernel components, FP64 accumulation:
//   B_c[t](k') = sc_t * sum_{o in S, o_last = t} K_c(o) prod_{d<last} trig_{p_cd}(2 pi k_d o_d / n_d)
// with trig = cos for even and sin for odd axes (Eq. 56-58: the kernel
// spectrum as a quadrature sum over the horizon, split along the last axis).
// Transform convention (spectral multiply): sc_0 = 1/Nfft, sc_t = 2/Nfft;
// direct convention (line correlation): sc_t = n_last/Nfft for every t.
// Layout [k' (line)][component][tap]: the taps of one line are contiguous.
template <class T>
__global__ void k_taps(int dim, int n1, int n2, int h1, long NP, int ntap, int ns,
                       const int* __restrict__ offs, const double* __restrict__ kval, int kstride,
                       int nct, const uint8_t* __restrict__ par, const double* __restrict__ tw64, int twn1,
                       double sc0, double sc1, T* __restrict__ taps) {
    long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= NP * ntap) return;
    const long p = idx % NP;
    const int t = (int)(idx / NP);
    int kx, ky = 0;
    if (dim == 2) kx = (int)p;
    else { kx = (int)(p / n2); ky = (int)(p % n2); }
    const int last = dim - 1;
    double acc[12];
    for (int c = 0; c < nct; ++c) acc[c] = 0.0;
    const double* twx = tw64 + 2 * twn1;  // complex FP64 table of length n1
    const double* twy = tw64 + 2 * n2;    // of length n2 (a power of two) at [n2, 2 n2)
    for (int s = 0; s < ns; ++s) {
        const int ox = offs[3 * s], oy = offs[3 * s + 1], oz = offs[3 * s + 2];
        const int ol = (last == 1) ? oy : oz;
        if (ol != t) continue;
        int ex = (int)(((long)kx * ox) % n1);
        if (ex < 0) ex += n1;
        const double cxv = twx[2 * ex], sxv = -twx[2 * ex + 1];
        double cyv = 1.0, syv = 0.0;
        if (dim == 3) {
            int ey = (int)(((long)ky * oy) % n2);
            if (ey < 0) ey += n2;
            cyv = twy[2 * ey];
            syv = -twy[2 * ey + 1];
        }
        for (int c = 0; c < nct; ++c) {
            double f = par[3 * c] ? sxv : cxv;
            if (dim == 3) f *= par[3 * c + 1] ? syv : cyv;
            acc[c] += kval[(long)s * kstride + c] * f;
        }
    }
    const double sc = t ? sc1 : sc0;
    for (int c = 0; c < nct; ++c) taps[((long)p * nct + c) * ntap + t] = T(acc[c] * sc);
}

// Partial x-spectra over the (y, z) quarter disc, FP64 accumulation:
//   tau_c(kx; a, b) = sc * sum_{o in S, o_y = a, o_z = b} K_c(o) trig_{p_cx}(2 pi kx o_x / n1)
// for a, b >= 0, a^2 + b^2 <= MT^2 (tap u = yz_tap(MT, a, b)); sc = 1/n1,
// the normalisation of the unnormalised x transform pair.  The taps at
// negative o_y, o_z follow from the parities of K_c.  Layout [kx][c][u],
// with nx extra components after the nct ones (scaled copies, so that a
// constant factor of a multiplier term is folded into its taps).
template <class T>
__global__ void k_taps_yz(int n1, int h1, int MT, int nu, int ns, const int* __restrict__ offs,
                          const double* __restrict__ kval, int kstride, int nct, const uint8_t* __restrict__ par,
                          const double* __restrict__ tw64, int twn1, double sc, int nx, int x0, double xs,
                          T* __restrict__ taps) {
    long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)h1 * nu) return;
    const int kx = (int)(idx / nu), u = (int)(idx % nu);
    int ta = -1, tb = -1;
    for (int b = 0; b <= MT && ta < 0; ++b)
        for (int a = 0; a <= MT; ++a)
            if (a * a + b * b <= MT * MT && yz_tap(MT, a, b) == u) { ta = a; tb = b; break; }
    double acc[12];
    for (int c = 0; c < nct; ++c) acc[c] = 0.0;
    const double* twx = tw64 + 2 * twn1;
    for (int s = 0; s < ns; ++s) {
        if (offs[3 * s + 1] != ta || offs[3 * s + 2] != tb) continue;
        int ex = (int)(((long)kx * offs[3 * s]) % n1);
        if (ex < 0) ex += n1;
        const double cxv = twx[2 * ex], sxv = -twx[2 * ex + 1];
        for (int c = 0; c < nct; ++c) acc[c] += kval[(long)s * kstride + c] * (par[3 * c] ? sxv : cxv);
    }
    // nx extra components: xs times components x0 .. x0+nx-1 (LPS: k_a a0_i)
    const int nall = nct + nx;
    // second table (after the first): components odd along z negated
    T* rev = taps + (long)h1 * nall * nu;
    for (int c = 0; c < nct; ++c) {
        const T t = T(acc[c] * sc);
        taps[((long)kx * nall + c) * nu + u] = t;
        rev[((long)kx * nall + c) * nu + u] = par[3 * c + 2] ? -t : t;
    }
    for (int c = 0; c < nx; ++c) {
        const T t = T(acc[x0 + c] * sc * xs);
        taps[((long)kx * nall + nct + c) * nu + u] = t;
        rev[((long)kx * nall + nct + c) * nu + u] = par[3 * (x0 + c) + 2] ? -t : t;
    }
}

// Static embedded-constraint fields by direct quadrature over the horizon
// (the paper allows P = C (*) 1 either by quadrature or by FFT, Sec. 3.1):
//   stat_c(x) = sum_{o in S} chi_B(x + o) K_c(o)   on the body box,
// stored node-major (stat[i * ncs + c]).
// Also the node flags: flags[i] = chiB[i] | 2 when the node's whole horizon
// lies in the body (then stat equals the interior sums: every bond counted,
// same order), and bit 2 + d = chi_Omega of component d (zero outside the
// body), so that the passes read no separate chi_Omega bytes.
template <class T>
__global__ void k_static(int b1, int b2, int b3, int ns, const int* __restrict__ offs,
                         const double* __restrict__ kval, int ncs, const uint8_t* __restrict__ chiB,
                         const uint8_t* __restrict__ chiO, int D, T* __restrict__ stat,
                         uint8_t* __restrict__ flags, long nb) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    const int x = (int)(i % b1), y = (int)((i / b1) % b2), z = (int)(i / ((long)b1 * b2));
    double acc[12];
    for (int c = 0; c < ncs; ++c) acc[c] = 0.0;
    int inside = 0;
    for (int s = 0; s < ns; ++s) {
        const int xx = x + offs[3 * s], yy = y + offs[3 * s + 1], zz = z + offs[3 * s + 2];
        if (xx < 0 || xx >= b1 || yy < 0 || yy >= b2 || zz < 0 || zz >= b3) continue;
        if (!chiB[((long)zz * b2 + yy) * b1 + xx]) continue;
        ++inside;
        for (int c = 0; c < ncs; ++c) acc[c] += kval[(long)s * ncs + c];
    }
    for (int c = 0; c < ncs; ++c) stat[i * ncs + c] = T(acc[c]);
    int f = chiB[i] ? (inside == ns ? 3 : 1) : 0;
    for (int d = 0; d < D; ++d) f |= (chiB[i] && chiO[d * nb + i]) ? (4 << d) : 0;
    flags[i] = (uint8_t)f;
}

template <class T>
__global__ void k_fill(T* p, long n, T v) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace pdi

namespace pdk {

static __global__ void k_reduce_final(const double* __restrict__ part, long nblk, int NR, double* __restrict__ out,
                                      double* __restrict__ host) {
    __shared__ double sm[256];
    for (int r = 0; r < NR; ++r) {
        double s = 0;
        for (long b = threadIdx.x; b < nblk; b += blockDim.x) s += part[b * NR + r];
        sm[threadIdx.x] = s;
        __syncthreads();
        for (int w = blockDim.x / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            out[r] = sm[0];
            if (host) host[r] = sm[0];
        }
        __syncthreads();
    }
}

}  // namespace pdk

namespace pdi {

// ------------------------------------------------------------------ helpers

inline bool is_pow2(long v) { return v > 0 && (v & (v - 1)) == 0; }

// Radix R of an x length n1 = 2 R 2^p (R = 3, 5 or 9, 2^p >= 8); 1 for a
// power of two, 0 for any other length.
inline int x_radix(long n1) {
    if (is_pow2(n1)) return 1;
    for (int R : {3, 5, 9})
        if (n1 % (2 * R) == 0 && is_pow2(n1 / (2 * R)) && n1 / (2 * R) >= 8) return R;
    return 0;
}

template <class T>
inline cx<T>* SAp(pd_plan p) { return reinterpret_cast<cx<T>*>(p->SA); }
template <class T>
inline cx<T>* SBp(pd_plan p) { return reinterpret_cast<cx<T>*>(p->SB); }
template <class T>
inline const cx<T>* TWp(pd_plan p) { return reinterpret_cast<const cx<T>*>(p->tw); }

template <class T>
NodeCtx<T> ctx(pd_plan p) {
    NodeCtx<T> c;
    c.nb = p->nb;
    c.chiB = p->chiB;
    c.stat = reinterpret_cast<const T*>(p->stat);
    c.ncs = p->ncs;
    c.stat_int = reinterpret_cast<const T*>(p->stat_int);
    for (int q = 0; q < 10; ++q) c.sint[q] = T(q < p->ncs ? p->stat_int_h[q] : 0.0);
    c.edge_frac = p->nb > 0 ? (double)p->n_edge / (double)p->nb : 0.0;
    return c;
}

// Lengths with compile-time specialisations of the x and y passes (the
// 512^3 box: 256-point complex rows along x, 512-point lines along y; the
// 256-point x box: 128-point rows); any other length runs the
// runtime-length kernels (LG = 0).  The specialised x passes also assume a
// body no longer than half the x box (b1 <= Nc).
constexpr int kFastLgX = 8, kFastLgX2 = 7, kFastLgY = 9;

inline bool x_fast(const Geo& g) {
    return g.b1 <= g.Nc && (g.Nc == (1 << kFastLgX) || g.Nc == (1 << kFastLgX2));
}

template <class T>
int rows_per_block(pd_plan p, int want = 0) {
    const Geo& g = p->geo;
    const int Tc = g.Nc / 8;
    int Lt = g.rad != 1 ? xrows_mixed<T>() : (want > 0 ? want : xrows<T>());
    while (Lt > 1 && Tc * Lt > 512) Lt >>= 1;
    // few rows (2D plates, small blocks): fewer rows per block, down to two
    // (16-byte runs in the transposed stores), until the grid has a block for
    // each of the 256 compute units
    if (!x_fast(g))
        while (Lt > 2 && (long)((g.b2 + Lt - 1) / Lt) * g.b3 < 256) Lt >>= 1;
    while (Lt > 1 && ((size_t)Lt * row_pitch(p->geo.Nc) + tw_lds_len(p->geo.n1)) * sizeof(cx<T>) > (size_t)p->max_lds) Lt >>= 1;
    return Lt;
}

template <class T>
int cols_per_block(pd_plan p, int nc_taps) {
    const int Tn = p->geo.n3 / 8;
    int Lc = (sizeof(T) == 4) ? 16 : 8;
    while (Lc > 1 && Tn * Lc > 512) Lc >>= 1;
    while (Lc > p->geo.n2) Lc >>= 1;
    auto need = [&](int L) {
        return (size_t)p->geo.n3 * L * sizeof(cx<T>) + (size_t)L * nc_taps * p->ntap * sizeof(T);
    };
    while (Lc > 1 && need(Lc) > (size_t)p->max_lds) Lc >>= 1;
    return Lc;
}

template <class K>
void allow_lds(K kern, size_t bytes) {
    if (bytes > 65536) (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Records a pair of events around one launch when timing is enabled.
struct ProfScope {
    pd_plan p;
    hipStream_t st;
    hipEvent_t a = nullptr;
    ProfScope(pd_plan p_, hipStream_t st_) : p(p_), st(st_) {
        if (p->prof && hipEventCreate(&a) == hipSuccess) (void)hipEventRecord(a, st);
    }
    void done(const char* name, double bytes) {
        if (!p->prof || !a) return;
        hipEvent_t b;
        if (hipEventCreate(&b) != hipSuccess) return;
        (void)hipEventRecord(b, st);
        ProfRec r;
        std::snprintf(r.name, sizeof(r.name), "%s", name);
        r.a = a;
        r.b = b;
        r.bytes = bytes;
        p->prof->push_back(r);
        a = nullptr;
    }
};

template <class T>
long xinv_blocks(pd_plan p) {
    const int Lt = rows_per_block<T>(p);
    return (long)((p->geo.b2 + Lt - 1) / Lt) * p->geo.b3;
}

// Pass 1
template <class T, class G, int LG>
pd_status launch_xfwd_lg(pd_plan p, const G& gen, cx<T>* SA, hipStream_t st) {
    const Geo& g = p->geo;
    const int Tc = g.Nc / 8, Lt = rows_per_block<T>(p);
    if (x_block_fixed<T, LG>() > 0 && Tc * Lt != x_block_fixed<T, LG>()) return PD_EUNSUPPORTED;
    dim3 grid((g.b2 + Lt - 1) / Lt, g.b3), block(Tc * Lt);
    size_t lds = ((size_t)Lt * row_pitch(g.Nc) + tw_lds_len(g.n1)) * sizeof(cx<T>);
    allow_lds(k_xfwd<T, G, LG>, lds);
    ProfScope ps(p, st);
    hipLaunchKernelGGL((k_xfwd<T, G, LG>), grid, block, lds, st, g, gen, SA, TWp<T>(p));
    if (p->prof) {
        char nm[32];
        std::snprintf(nm, sizeof nm, "xfwd_%d", G::NIN);
        ps.done(nm, gen.nbytes() * (double)g.nb + (double)G::NIN * g.b3 * g.h1 * g.b2 * sizeof(cx<T>));
    }
    return pdh::check(hipGetLastError());
}
// Mixed-radix x lengths with compile-time kernels (the minimum-padding x
// grids of a 256-node body: n1 = 384, 320, 288; FP32): the launch
// configuration must have the fixed block shape, else the runtime-length
// kernel runs.
template <class T>
int x_mixed_lg(pd_plan p) {
    const Geo& g = p->geo;
    const int Tc = g.Nc / 8, Lt = rows_per_block<T>(p);
    auto fits = [&](int R, int lgM) {
        const int rn = R == 3 ? 11 : (R == 5 ? 13 : 15);   // x_rn of the specialisation
        return g.rad == R && g.lgM == lgM && Tc * Lt == ((R << lgM) / 8) * xrows_mixed<T>() &&
               8 * g.b1 <= rn * g.Nc;
    };
    if (fits(3, 6)) return mix_lg(3, 6);
    if (fits(5, 5)) return mix_lg(5, 5);
    if (fits(9, 4)) return mix_lg(9, 4);
    return -1;
}

template <class T, class G>
pd_status launch_xfwd(pd_plan p, const G& gen, cx<T>* SA, hipStream_t st) {
    if (p->geo.rad != 1) {
        // compile-time mixed lengths in FP32 only (FP64 takes the runtime kernel)
        if constexpr (sizeof(T) == 4) {
            switch (x_mixed_lg<T>(p)) {
                case mix_lg(3, 6): return launch_xfwd_lg<T, G, mix_lg(3, 6)>(p, gen, SA, st);
                case mix_lg(5, 5): return launch_xfwd_lg<T, G, mix_lg(5, 5)>(p, gen, SA, st);
                case mix_lg(9, 4): return launch_xfwd_lg<T, G, mix_lg(9, 4)>(p, gen, SA, st);
                default: break;
            }
        }
        return launch_xfwd_lg<T, G, -1>(p, gen, SA, st);
    }
    if (p->geo.b1 <= p->geo.Nc) {
        if (p->geo.Nc == (1 << kFastLgX)) return launch_xfwd_lg<T, G, kFastLgX>(p, gen, SA, st);
        if (p->geo.Nc == (1 << kFastLgX2)) return launch_xfwd_lg<T, G, kFastLgX2>(p, gen, SA, st);
    }
    return launch_xfwd_lg<T, G, 0>(p, gen, SA, st);
}

// Last-axis pass over contiguous lines.  Default: direct line correlation
// (taps_d, horizons up to 4 spacings along the last axis); otherwise the
// FFT-multiply-FFT form (taps), specialised for 512-point lines with 4 taps
// or with runtime lengths.
template <class T, class M, int NT>
pd_status launch_lastconv(pd_plan p, const Lines& ln, const M& mul, cx<T>* S, const T* taps_d, int nct,
                          hipStream_t st) {
    // one wavefront per line, four lines per block (one when there are too
    // few lines to give every compute unit two blocks, as on the 2D plates);
    // no LDS; line starts must be 16-point aligned (the pitches of SA and SB
    // are)
    if ((ln.pitch & 15) || (ln.fstride & 15)) return PD_EINVAL;
    const int Lw = ln.nlines >= 4L * 512 ? 4 : 1;
    dim3 grid((unsigned)((ln.nlines + Lw - 1) / Lw)), block(64 * Lw);
    hipLaunchKernelGGL((k_lastconv<T, M, NT>), grid, block, 0, st, ln, mul, S, taps_d, nct);
    return PD_OK;
}

// Multipliers that are not trigonometric polynomials of the taps along the
// last axis (the preconditioner) declare NONLOCAL and take a transform form.
template <class M, class = void>
struct is_nonlocal : std::false_type {};
template <class M>
struct is_nonlocal<M, std::void_t<decltype(M::NONLOCAL)>> : std::integral_constant<bool, M::NONLOCAL> {};

template <class T, class M>
pd_status launch_lastmul(pd_plan p, const Lines& ln, const M& mul, cx<T>* S, const T* taps, const T* taps_d,
                         int ntap, int nct, uint32_t oddmask, hipStream_t st) {
    const int Tn = ln.N / 8;
    ProfScope ps(p, st);
    // the direct line correlation holds 4 points of every input and output
    // per lane: beyond 16 fields in FP64 it spills heavily (13 + 13: 8.6 ms
    // against 2.4 ms for the transform form on the 128^3 block)
    constexpr bool direct_ok = !M::RT_ODD && !is_nonlocal<M>::value && !(sizeof(T) == 8 && M::NIN + M::NOUT > 16);
    int path = 2;   // 0 direct, 1 specialised FFT, 2 generic FFT
    if constexpr (direct_ok) {
        if ((p->lastaxis == PD_LASTAXIS_AUTO || p->lastaxis == PD_LASTAXIS_YFFT) && taps_d && ntap >= 2 && ntap <= 5)
            path = 0;
    }
    if constexpr (!M::RT_ODD) {
        if (path != 0 && p->lastaxis != PD_LASTAXIS_FFT_GENERIC && (ln.N == 512 || ln.N == 256) && ntap == 4)
            path = 1;
    }
    if (path == 0) {
        if constexpr (direct_ok) {
            pd_status s = PD_OK;
            switch (ntap) {
                case 2: s = launch_lastconv<T, M, 2>(p, ln, mul, S, taps_d, nct, st); break;
                case 3: s = launch_lastconv<T, M, 3>(p, ln, mul, S, taps_d, nct, st); break;
                case 4: s = launch_lastconv<T, M, 4>(p, ln, mul, S, taps_d, nct, st); break;
                default: s = launch_lastconv<T, M, 5>(p, ln, mul, S, taps_d, nct, st); break;
            }
            PD_TRY(s);
        }
    } else if (path == 1) {
        if constexpr (!M::RT_ODD) {
            // 512-point lines: 4 per block; 256-point lines (the 128^3 cube's
            // preconditioner): 8 per block, two per wave
            auto go = [&](auto lgc) -> pd_status {
                constexpr int LG = decltype(lgc)::value, NT = 4;
                const int Lw = 2048 >> LG;   // 256 threads
                const size_t lds = ((size_t)Lw * line_pitch(1 << LG) + tw_lds_len(1 << LG)) * sizeof(cx<T>);
                if (lds > (size_t)p->max_lds) return PD_EUNSUPPORTED;
                dim3 grid((unsigned)((ln.nlines + Lw - 1) / Lw)), block(Lw * ((1 << LG) / 8));
                allow_lds(k_lastmul_f<T, M, LG, NT>, lds);
                hipLaunchKernelGGL((k_lastmul_f<T, M, LG, NT>), grid, block, lds, st, ln, mul, S, taps, nct,
                                   TWp<T>(p));
                return PD_OK;
            };
            PD_TRY(ln.N == 512 ? go(std::integral_constant<int, 9>{}) : go(std::integral_constant<int, 8>{}));
        }
    } else {
        int Lw = std::max(1, 256 / Tn);
        auto need = [&](int L) {
            return ((size_t)L * line_pitch(ln.N) + tw_lds_len(ln.N)) * sizeof(cx<T>) +
                   (size_t)L * M::NC * ntap * sizeof(T);
        };
        while (Lw > 1 && need(Lw) > (size_t)p->max_lds) Lw >>= 1;
        size_t lds = need(Lw);
        dim3 grid((unsigned)((ln.nlines + Lw - 1) / Lw)), block(Lw * Tn);
        allow_lds(k_lastmul<T, M>, lds);
        hipLaunchKernelGGL((k_lastmul<T, M>), grid, block, lds, st, ln, mul, S, taps, ntap, nct, oddmask, TWp<T>(p));
    }
    if (p->prof) {
        char nm[32];
        std::snprintf(nm, sizeof nm, "%s_%dx%d", path == 0 ? "lastconv" : "lastmul", M::NIN, M::NOUT);
        ps.done(nm, (double)(M::NIN + M::NOUT) * ln.nlines * ln.len * sizeof(cx<T>) +
                        (double)M::NC * ntap * ln.nlines * sizeof(T));
    }
    return pdh::check(hipGetLastError());
}

// (y, z) direct pass (3D), for horizons of radius MT = 2 or 3 spacings in
// (y, z).  A multiplier qualifies when its terms have compile-time parities
// (par3) and are local, the ring of 2 MT + 1 output planes fits in at most
// 128 registers per thread, and it is one of the chains built with the pass
// (the force, Verlet and static chains: LPS dilatation and force, unweighted
// bond-based); the weighted bond-based and adjoint chains, with up to 13
// outputs, take the y transform path.
template <class M, class = void>
struct has_par3 : std::false_type {};
template <class M>
struct has_par3<M, std::void_t<decltype(M::par3(0))>> : std::true_type {};

template <class T, class M, int MT>
constexpr bool yz_fits() {
    return M::NOUT * (2 * MT + 1) * 2 * (int)(sizeof(T) / 4) <= 128;
}
// Outputs O0 .. O1-1 of a multiplier: a (y, z) pass holds the accumulators
// of all its outputs in registers, so a chain with many outputs (the 3D
// nonlinear model's 13) runs the pass once per group of outputs, each
// reading all the inputs.
template <class M, int O0, int O1>
struct MulOutRange {
    static constexpr int NIN = M::NIN, NOUT = O1 - O0, C0 = M::C0, NC = M::NC;
    static constexpr bool RT_ODD = M::RT_ODD;
    static constexpr uint32_t ODD = M::ODD;
    M m;
    __device__ __forceinline__ auto ka_value() const { return m.ka_value(); }
    __host__ __device__ static constexpr int par3(int c) { return M::par3(c); }
    __host__ __device__ static constexpr DTerm dterm(int O, int J) { return M::dterm(O0 + O, J); }
    // the transform forms of the last-axis pass
    template <int O>
    __host__ __device__ static constexpr uint32_t need() { return M::template need<O0 + O>(); }
    template <int O, class TK, class TI>
    __device__ __forceinline__ auto one(const TK* K, const TI* in) const { return m.template one<O0 + O>(K, in); }
};
template <class T, class M>
struct is_nbb3_range : std::false_type {};
template <class T, int O0, int O1>
struct is_nbb3_range<T, MulOutRange<MulNBB<T, 3>, O0, O1>> : std::true_type {};

template <class T, class M>
constexpr bool yz_capable() {
    return std::is_same<M, MulLPSA<T>>::value || std::is_same<M, MulLPSB<T>>::value ||
           std::is_same<M, MulBB<T, 3, false, false>>::value || is_nbb3_range<T, M>::value;
}

template <class T, class M, int MT, int YT>
pd_status launch_yzconv_t(pd_plan p, const M& mul, int in_off, int out_off, hipStream_t st) {
    const Geo& g = p->geo;
    YZArgs a;
    a.b2 = g.b2; a.b3 = g.b3; a.h1 = g.h1; a.P2 = g.P2;
    a.saf = g.saf;
    a.nyt = (g.b2 + YT - 1) / YT;
    // planes per chunk: the chunk count nearest to ~20 waves per CU of 256
    // CUs, and chunks of at least 4 MT planes.  A chunk sweeps 2 MT halo
    // planes beyond its own (their loads and arithmetic are repeated by the
    // neighbouring chunk), so fewer, longer chunks do less work, while too
    // few blocks leave CUs idle at the end: at the 256^3 body five chunks of
    // 52 planes (1285 blocks) ran both LPS passes 5-12 % faster than 16
    // chunks of 16 planes, and the 128^3 body keeps 12-plane chunks.
    const long tiles = (long)g.h1 * a.nyt;
    const long den = tiles * YT;
    const long want = std::max(1L, (256L * 20 * 64 + den / 2) / den);
    int zc = (int)std::max<long>(4L * MT, (g.b3 + want - 1) / want);
    zc = std::min(zc, g.b3);
    a.zc = zc;
    a.nzc = (g.b3 + zc - 1) / zc;
    a.in_off = in_off; a.out_off = out_off;
    a.nct = p->nct_yz;
    const long nblk = tiles * a.nzc;
    const size_t lds = (size_t)2 * M::NIN * (YT + 2 * MT) * sizeof(cx<T>);
    if (lds > (size_t)p->max_lds || nblk > 0x7fffffffL) return PD_EUNSUPPORTED;
    allow_lds(k_yzconv<T, M, MT, YT>, lds);
    hipLaunchKernelGGL((k_yzconv<T, M, MT, YT>), dim3((unsigned)nblk), dim3(YT), lds, st, a, mul, SAp<T>(p),
                       reinterpret_cast<const T*>(p->taps_yz));
    return PD_OK;
}

template <class T, class M>
pd_status launch_yzconv(pd_plan p, const M& mul, int in_off, int out_off, hipStream_t st) {
    pd_status s = PD_EUNSUPPORTED;
    ProfScope ps(p, st);
    const bool wide = p->geo.b2 > 128;
    auto go = [&](auto mtc) {
        constexpr int MT = decltype(mtc)::value;
        if constexpr (yz_fits<T, M, MT>()) {
            s = wide ? launch_yzconv_t<T, M, MT, 256>(p, mul, in_off, out_off, st)
                     : launch_yzconv_t<T, M, MT, 128>(p, mul, in_off, out_off, st);
        }
    };
    switch (p->yz_mt) {
        case 2: go(std::integral_constant<int, 2>{}); break;
        case 3: go(std::integral_constant<int, 3>{}); break;
        default: break;
    }
    PD_TRY(s);
    if (p->prof) {
        const Geo& g = p->geo;
        char nm[32];
        std::snprintf(nm, sizeof nm, "yzconv_%dx%d", M::NIN, M::NOUT);
        ps.done(nm, (double)(M::NIN + M::NOUT) * g.b3 * g.h1 * g.b2 * sizeof(cx<T>) +
                        (double)M::NC * p->yz_nu * g.h1 * sizeof(T));
    }
    return pdh::check(hipGetLastError());
}

// The (y, z) pass kernels are instantiated once per (dtype, multiplier), in
// instantiation units of their own (pd_inst.hip, parts 4 and 5).
template <class T> using YzBB = MulBB<T, 3, false, false>;
#define PD_YZ_LIST_A(X, T) X(T, MulLPSB<T>)
#define PD_YZ_LIST_B(X, T) X(T, MulLPSA<T>) X(T, YzBB<T>)
#define PD_YZ_DECL(T, M) extern template pd_status launch_yzconv<T, M>(pd_plan, const M&, int, int, hipStream_t);
#if !defined(PD_INST_PART) || (PD_INST_PART != 4 && PD_INST_PART != 5)
PD_YZ_LIST_A(PD_YZ_DECL, float)
PD_YZ_LIST_A(PD_YZ_DECL, double)
PD_YZ_LIST_B(PD_YZ_DECL, float)
PD_YZ_LIST_B(PD_YZ_DECL, double)
#endif

// The 3D nonlinear chain's (y, z) pass: the 13 outputs in groups of 7 (FP32)
// or 3 (FP64), whose accumulators fit the registers of one pass; inputs in
// SA slots [0, 13), outputs to [out_off, out_off + 13).  Instantiated in its
// own unit (pd_inst.hip, part 6).
template <class T, int O0, int O1> using YzNBB = MulOutRange<MulNBB<T, 3>, O0, O1>;
template <class T>
constexpr int nbb_yz_group() { return sizeof(T) == 4 ? 7 : 3; }
template <class T, int O0>
pd_status nbb_yz_from(pd_plan p, int out_off, hipStream_t st) {
    constexpr int NO = MulNBB<T, 3>::NOUT;
    if constexpr (O0 >= NO) {
        return PD_OK;
    } else {
        constexpr int O1 = (O0 + nbb_yz_group<T>() < NO) ? O0 + nbb_yz_group<T>() : NO;
        PD_TRY((launch_yzconv<T, YzNBB<T, O0, O1>>(p, YzNBB<T, O0, O1>{}, 0, out_off + O0, st)));
        return nbb_yz_from<T, O1>(p, out_off, st);
    }
}
template <class T>
pd_status nbb_yz(pd_plan p, int out_off, hipStream_t st) { return nbb_yz_from<T, 0>(p, out_off, st); }
#if !defined(PD_INST_PART) || PD_INST_PART != 6
extern template pd_status nbb_yz<float>(pd_plan, int, hipStream_t);
extern template pd_status nbb_yz<double>(pd_plan, int, hipStream_t);
#endif

// The 2D nonlinear chain's line correlation along y in groups of 2 outputs
// (FP64), inputs in SA slots [0, 8), outputs to [out_off, out_off + 8).
template <class T, int O0>
pd_status nbb2_lines_from(pd_plan p, int out_off, hipStream_t st) {
    constexpr int NO = MulNBB<T, 2>::NOUT;
    if constexpr (O0 >= NO) {
        return PD_OK;
    } else {
        constexpr int O1 = O0 + 2 < NO ? O0 + 2 : NO;
        const Geo& g = p->geo;
        Lines ln{(long)g.h1, (long)g.P2, g.saf, g.b2, g.n2, out_off + O0};
        PD_TRY((launch_lastmul<T>(p, ln, MulOutRange<MulNBB<T, 2>, O0, O1>{}, SAp<T>(p),
                                  reinterpret_cast<const T*>(p->taps), reinterpret_cast<const T*>(p->taps_d),
                                  p->ntap, p->nct, p->oddmask, st)));
        return nbb2_lines_from<T, O1>(p, out_off, st);
    }
}

// Whether a chain takes the (y, z) direct pass: 3D plan tables, the default
// kernel choice, and a multiplier that qualifies at the plan's radius.
template <class T, class M>
bool use_yz(pd_plan p) {
    if constexpr (!yz_capable<T, M>()) return false;
    else {
        if (p->geo.dim != 3 || !p->taps_yz || p->lastaxis != PD_LASTAXIS_AUTO) return false;
        switch (p->yz_mt) {
            case 2: return yz_fits<T, M, 2>();
            case 3: return yz_fits<T, M, 3>();
            default: return false;
        }
    }
}

// planes per block of the transposing y passes
template <class T>
int planes_per_block(pd_plan p) {
    const int Tn = p->geo.n2 / 8;
    int Lz = (sizeof(T) == 4) ? 16 : 8;
    while (Lz > 1 && Tn * Lz > 1024) Lz >>= 1;
    while (Lz > 1 && ((size_t)Lz * line_pitch(p->geo.n2) + tw_lds_len(p->geo.n2)) * sizeof(cx<T>) > (size_t)p->max_lds) Lz >>= 1;
    return Lz;
}

// 3D y passes with transpose; F fields starting at SA field 0 / SB field fb.
template <class T, int SIGN, int LG>
pd_status launch_ytrans_lg(pd_plan p, int F, int fb, hipStream_t st) {
    const Geo& g = p->geo;
    const int Tn = g.n2 / 8, Lz = planes_per_block<T>(p);
    dim3 grid((g.b3 + Lz - 1) / Lz, g.h1, F), block(Lz * Tn);
    size_t lds = ((size_t)Lz * line_pitch(g.n2) + tw_lds_len(g.n2)) * sizeof(cx<T>);
    cx<T>* SB = SBp<T>(p) + (long)fb * p->sbf;
    ProfScope ps(p, st);
    if (SIGN < 0) {
        allow_lds(k_ytf<T, LG>, lds);
        hipLaunchKernelGGL((k_ytf<T, LG>), grid, block, lds, st, g, SAp<T>(p), SB, p->Pz, TWp<T>(p));
    } else {
        allow_lds(k_yti<T, LG>, lds);
        hipLaunchKernelGGL((k_yti<T, LG>), grid, block, lds, st, g, SB, SAp<T>(p), p->Pz, TWp<T>(p));
    }
    if (p->prof) {
        char nm[32];
        std::snprintf(nm, sizeof nm, "%s_%d", SIGN < 0 ? "ytf" : "yti", g.n2);
        ps.done(nm, (double)F * g.b3 * g.h1 * (g.b2 + g.n2) * sizeof(cx<T>));
    }
    return pdh::check(hipGetLastError());
}
template <class T, int SIGN>
pd_status launch_ytrans(pd_plan p, int F, int fb, hipStream_t st) {
    if (F <= 0) return PD_OK;
    if (p->geo.n2 == (1 << kFastLgY)) return launch_ytrans_lg<T, SIGN, kFastLgY>(p, F, fb, st);
    return launch_ytrans_lg<T, SIGN, 0>(p, F, fb, st);
}

// Pass 5 (+ deterministic reduction into p->red when F::NRED > 0)
template <class T, class F, int LG>
pd_status launch_xinv_lg(pd_plan p, const F& fin, const cx<T>* SA, hipStream_t st, cx<T>* SAout = nullptr) {
    const Geo& g = p->geo;
    constexpr int XF = x_block_fixed<T, LG, fin_xrows<F>::value>();
    const int Tc = g.Nc / 8, Lt = rows_per_block<T>(p, fin_xrows<F>::value);
    if (XF > 0 && Tc * Lt != XF) return PD_EUNSUPPORTED;
    dim3 grid((g.b2 + Lt - 1) / Lt, g.b3), block(Tc * Lt);
    size_t lds = ((size_t)Lt * row_pitch(g.Nc) + tw_lds_len(g.n1)) * sizeof(cx<T>);
    size_t red_lds = (size_t)((Tc * Lt + 63) / 64) * 8 * sizeof(double);
    lds = std::max(lds, red_lds);
    const long nblk = (long)grid.x * grid.y;
    if (F::NRED > 0 && nblk * F::NRED > p->partials_cap) return PD_EINVAL;
    allow_lds(k_xinv<T, F, LG>, lds);
    ProfScope ps(p, st);
    constexpr int NCH = fin_chain_n<F>::value;
    if (NCH > 0 && !SAout) return PD_EINVAL;
    hipLaunchKernelGGL((k_xinv<T, F, LG>), grid, block, lds, st, g, fin, SA, p->partials, TWp<T>(p), SAout);
    if (p->prof) {
        char nm[32];
        if (NCH > 0) std::snprintf(nm, sizeof nm, "xinvfwd_%d_%d", F::NOUT, NCH);
        else std::snprintf(nm, sizeof nm, "xinv_%d", F::NOUT);
        ps.done(nm, fin.nbytes() * (double)g.nb + (double)(F::NOUT + NCH) * g.b3 * g.h1 * g.b2 * sizeof(cx<T>));
    }
    PD_TRY(pdh::check(hipGetLastError()));
    if (F::NRED > 0) {
        hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, st, p->partials, nblk, F::NRED, p->red,
                           (double*)nullptr);
        PD_TRY(pdh::check(hipGetLastError()));
    }
    return PD_OK;
}
template <class T, class F>
pd_status launch_xinv(pd_plan p, const F& fin, const cx<T>* SA, hipStream_t st, cx<T>* SAout = nullptr) {
    if (p->geo.rad != 1) {
        if constexpr (sizeof(T) == 4) {
            switch (x_mixed_lg<T>(p)) {
                case mix_lg(3, 6): return launch_xinv_lg<T, F, mix_lg(3, 6)>(p, fin, SA, st, SAout);
                case mix_lg(5, 5): return launch_xinv_lg<T, F, mix_lg(5, 5)>(p, fin, SA, st, SAout);
                case mix_lg(9, 4): return launch_xinv_lg<T, F, mix_lg(9, 4)>(p, fin, SA, st, SAout);
                default: break;
            }
        }
        return launch_xinv_lg<T, F, -1>(p, fin, SA, st, SAout);
    }
    if (p->geo.b1 <= p->geo.Nc) {
        if (p->geo.Nc == (1 << kFastLgX)) return launch_xinv_lg<T, F, kFastLgX>(p, fin, SA, st, SAout);
        if (p->geo.Nc == (1 << kFastLgX2)) return launch_xinv_lg<T, F, kFastLgX2>(p, fin, SA, st, SAout);
    }
    return launch_xinv_lg<T, F, 0>(p, fin, SA, st, SAout);
}

// One full chain.  3D: sb_off is the SB field slot the generator's fields go
// to; the multiplier reads SB slots [0, M::NIN) and writes slots
// [out_off, out_off + M::NOUT) (out_off > 0 keeps the input spectra for a
// later chain, as the LPS dilatation stage does for the force stage).
template <class T, class G, class M, class F>
pd_status run_chain(pd_plan p, const G& gen, const M& mul, const F& fin, hipStream_t st, int sb_off = 0,
                    int out_off = 0, const T* taps = nullptr, int ntap = 0, int nct = 1,
                    uint32_t oddmask = 0xffffffffu) {
    static_assert(M::NOUT == F::NOUT, "multiplier/epilogue mismatch");
    const Geo& g = p->geo;
    const T* taps_d = nullptr;   // direct-convention taps (plan tables only)
    if (!taps) {
        taps = reinterpret_cast<const T*>(p->taps);
        taps_d = reinterpret_cast<const T*>(p->taps_d);
        ntap = p->ntap;
        nct = p->nct;
        oddmask = p->oddmask;
    }
    if (std::max(G::NIN, M::NOUT) > p->saf_cap) return PD_EINVAL;
    if constexpr (yz_capable<T, M>()) {
        if (taps_d && use_yz<T, M>(p)) {
            // x transform, (y, z) direct pass, inverse x transform; the generator
            // writes SA slots [sb_off, sb_off + G::NIN), the multiplier reads
            // [0, M::NIN) and writes after its inputs
            const int wo = std::max(out_off, M::NIN);
            if (sb_off + G::NIN > p->saf_cap || wo + M::NOUT > p->saf_cap) return PD_EINVAL;
            PD_TRY(launch_xfwd<T>(p, gen, SAp<T>(p) + (long)sb_off * g.saf, st));
            PD_TRY((launch_yzconv<T, M>(p, mul, 0, wo, st)));
            return launch_xinv<T>(p, fin, SAp<T>(p) + (long)wo * g.saf, st);
        }
    }
    PD_TRY(launch_xfwd<T>(p, gen, SAp<T>(p), st));
    if (g.dim == 2) {
        if (G::NIN != M::NIN) return PD_EINVAL;
        Lines ln{(long)g.h1, (long)g.P2, g.saf, g.b2, g.n2, 0};
        PD_TRY(launch_lastmul<T>(p, ln, mul, SAp<T>(p), taps, taps_d, ntap, nct, oddmask, st));
    } else {
        if (sb_off + G::NIN > p->sbf_cap || M::NIN > p->sbf_cap || out_off + M::NOUT > p->sbf_cap) return PD_EINVAL;
        PD_TRY((launch_ytrans<T, -1>(p, G::NIN, sb_off, st)));
        Lines ln{(long)g.h1 * g.n2, (long)p->Pz, p->sbf, g.b3, g.n3, out_off};
        PD_TRY(launch_lastmul<T>(p, ln, mul, SBp<T>(p), taps, taps_d, ntap, nct, oddmask, st));
        PD_TRY((launch_ytrans<T, 1>(p, M::NOUT, out_off, st)));
    }
    PD_TRY(launch_xinv<T>(p, fin, SAp<T>(p), st));
    return PD_OK;
}

// ----------------------------------------------------------------- stencil
struct Bond {
    int o[3];
    double xi[3];
    double r;
};

inline std::vector<Bond> make_stencil(int dim, const double* dx, double delta) {
    std::vector<Bond> S;
    int M[3] = {0, 0, 0};
    for (int d = 0; d < dim; ++d) M[d] = (int)std::floor(delta / dx[d] + 1e-9) + 1;
    const double lim = delta * delta * (1.0 + 1e-10);
    for (int oz = -M[2]; oz <= M[2]; ++oz)
        for (int oy = -M[1]; oy <= M[1]; ++oy)
            for (int ox = -M[0]; ox <= M[0]; ++ox) {
                if (!ox && !oy && !oz) continue;
                Bond b;
                b.o[0] = ox; b.o[1] = oy; b.o[2] = oz;
                double r2 = 0;
                for (int d = 0; d < 3; ++d) {
                    b.xi[d] = (d < dim) ? b.o[d] * dx[d] : 0.0;
                    r2 += b.xi[d] * b.xi[d];
                }
                if (r2 > lim) continue;
                b.r = std::sqrt(r2);
                S.push_back(b);
            }
    return S;
}

// Bond-based micromodulus constant for omega = 1/r (influence 0) or 1:
// alpha = 2 lambda_target / (A_d * int_0^delta omega r^(d+1) dr), with the
// isotropic angular moments A_2 = pi/4, A_3 = 4 pi/15 and the Lame constant
// lambda_target = 3E/8 (2D plane stress, nu = 1/3) or 2E/5 (3D, nu = 1/4);
// for 2D and omega = 1/r this is the paper's alpha = 9E/(pi delta^3).
inline double bb_alpha(int dim, int influence, double E, double delta) {
    const double I = influence == 0 ? std::pow(delta, dim + 1) / (dim + 1) : std::pow(delta, dim + 2) / (dim + 2);
    const double A = dim == 2 ? kPi / 4.0 : 4.0 * kPi / 15.0;
    const double lam = dim == 2 ? 3.0 * E / 8.0 : 2.0 * E / 5.0;
    return 2.0 * lam / (A * I);
}

// Twiddle buffer: exp(-2 pi i e / N) for every power of two N <= P at complex
// entries [N, 2N), P the largest power-of-two axis length, and, when the x
// length n1 is not a power of two, the length-n1 table at [2P, 2P + n1)
// (*twn1 receives the offset of the n1 table either way).
template <class T>
void twiddles_host(int P, int n1, std::vector<T>& out, int* twn1) {
    const bool mixed = !is_pow2(n1);
    *twn1 = mixed ? 2 * P : n1;
    out.assign((size_t)2 * (2 * P + (mixed ? n1 : 0)), T(0));
    auto put = [&](int N, size_t at) {
        for (int e = 0; e < N; ++e) {
            long double a = -2.0L * 3.141592653589793238462643383279502884L * (long double)e / (long double)N;
            out[2 * (at + e)] = (T)cosl(a);
            out[2 * (at + e) + 1] = (T)sinl(a);
        }
    };
    for (int N = 1; N <= P; N <<= 1) put(N, (size_t)N);
    if (mixed) put(n1, (size_t)2 * P);
}

// Largest eigenvalue of the periodic operator's symbol, sampled on a
// coarse set of wavenumbers (the maximum sits at large |k|), used for the
// explicit time-step bound dt <= 2/sqrt(lambda_max/rho).
inline double symbol_lambda_max(pd_plan p, const std::vector<Bond>& S) {
    const int D = p->dim;
    double best = 0;
    const int nsmp = 16;
    int lim[3] = {nsmp, nsmp, D == 3 ? nsmp : 0};
    for (int a = 0; a <= lim[0]; ++a)
        for (int b = 0; b <= lim[1]; ++b)
            for (int c = 0; c <= lim[2]; ++c) {
                double kk[3] = {a * 0.5 / nsmp, b * 0.5 / nsmp, c * 0.5 / nsmp};  // cycles per node
                double Mx[3][3] = {{0}}, sv[3] = {0, 0, 0};
                for (const Bond& bd : S) {
                    double ph = 0;
                    for (int d = 0; d < D; ++d) ph += 2 * kPi * kk[d] * bd.o[d];
                    const double om = p->influence == 0 ? 1.0 / bd.r : 1.0;
                    double coef = (p->kern.model == PD_LPS_LINEAR) ? 30.0 * p->mu / p->m0 : p->alpha;
                    coef *= om / (bd.r * bd.r) * p->dV * (1.0 - std::cos(ph));
                    for (int i = 0; i < D; ++i)
                        for (int j = 0; j < D; ++j) Mx[i][j] += coef * bd.xi[i] * bd.xi[j];
                    for (int i = 0; i < D; ++i) sv[i] += om * bd.xi[i] * std::sin(ph) * p->dV;
                }
                if (p->kern.model == PD_LPS_LINEAR)
                    for (int i = 0; i < D; ++i)
                        for (int j = 0; j < D; ++j) Mx[i][j] += 3.0 * p->ka * sv[i] * sv[j];
                // Gershgorin bound of the symmetric matrix
                for (int i = 0; i < D; ++i) {
                    double r = 0;
                    for (int j = 0; j < D; ++j) r += std::fabs(Mx[i][j]);
                    best = std::max(best, r);
                }
            }
    return best;
}

template <class T>
pd_status build_device_tables(pd_plan p, const std::vector<Bond>& S, hipStream_t st) {
    const int D = p->dim;
    // components
    std::vector<double> kv;          // [ns][ncs]
    std::vector<uint8_t> par;        // [nct][3]
    const int ns = (int)S.size();
    auto om = [&](double r) { return p->influence == 0 ? 1.0 / r : 1.0; };
    int nct = 0, ncs = 0;
    if (p->kern.model == PD_BB_LINEAR) {
        nct = nsym(D) + (p->kern.weight == PD_WEIGHT_INTEGRITY ? 1 : 0);
        ncs = nct;
    } else if (p->kern.model == PD_BB_NONLINEAR) {
        nct = nsym(D) + D + 1;   // C_ab, a_i, c
        ncs = nct;
    } else {
        nct = 9;
        ncs = 10;
    }
    kv.assign((size_t)ns * ncs, 0.0);
    par.assign((size_t)nct * 3, 0);
    const double cC = (p->kern.model == PD_LPS_LINEAR) ? 30.0 * p->mu / p->m0 : p->alpha;
    for (int s = 0; s < ns; ++s) {
        const Bond& bd = S[s];
        const double w = om(bd.r);
        for (int i = 0; i < D; ++i)
            for (int j = i; j < D; ++j)
                kv[(size_t)s * ncs + symi(D, i, j)] = cC * w * bd.xi[i] * bd.xi[j] / (bd.r * bd.r) * p->dV;
        if (p->kern.model == PD_BB_LINEAR) {
            if (p->kern.weight == PD_WEIGHT_INTEGRITY) kv[(size_t)s * ncs + nsym(D)] = 1.0;
        } else if (p->kern.model == PD_BB_NONLINEAR) {
            // Eq. 24: a_i = c xi_i, c = alpha omega / |xi|^2 (with dV)
            const double cc = cC * w / (bd.r * bd.r) * p->dV;
            for (int i = 0; i < D; ++i) kv[(size_t)s * ncs + nsym(D) + i] = cc * bd.xi[i];
            kv[(size_t)s * ncs + nsym(D) + D] = cc;
        } else {
            for (int i = 0; i < 3; ++i) kv[(size_t)s * ncs + 6 + i] = w * bd.xi[i] * p->dV;
            kv[(size_t)s * ncs + 9] = w * bd.r * bd.r * p->dV;
        }
    }
    p->oddmask = 0;
    for (int i = 0; i < D; ++i)
        for (int j = i; j < D; ++j) {
            const int c = symi(D, i, j);
            for (int d = 0; d < D; ++d) par[3 * c + d] = ((i == d) + (j == d)) & 1;
        }
    if (p->kern.model == PD_LPS_LINEAR)
        for (int i = 0; i < 3; ++i) par[3 * (6 + i) + i] = 1;
    if (p->kern.model == PD_BB_NONLINEAR)
        for (int i = 0; i < D; ++i) par[3 * (nsym(D) + i) + i] = 1;
    for (int c = 0; c < nct; ++c)
        if (par[3 * c + (D - 1)]) p->oddmask |= 1u << c;
    p->nct = nct;
    p->ncs = ncs;
    p->beta_comp = (p->kern.weight == PD_WEIGHT_INTEGRITY && p->kern.model == PD_BB_LINEAR) ? nsym(D) : -1;

    int mlast = 0;
    std::vector<int> offs((size_t)ns * 3);
    for (int s = 0; s < ns; ++s) {
        for (int d = 0; d < 3; ++d) offs[3 * s + d] = S[s].o[d];
        mlast = std::max(mlast, std::abs(S[s].o[D - 1]));
    }
    p->ntap = mlast + 1;
    if (p->ntap > 9) return PD_EUNSUPPORTED;
    {
        // preconditioner constants: Ĉ(0)_ii = sum_o C_ii(o) dV; the shift is a
        // quarter of the mean diagonal of the symbol at the first nonzero
        // wavenumber along x, sum_o C_ii(o) (1 - cos(2 pi o_x / n1)) dV
        const double nf = (double)p->nfft;
        double sh = 0.0;
        for (int i = 0; i < 3; ++i) p->pre_k0[i] = 0.0;
        for (int s = 0; s < ns; ++s) {
            const double cx1 = 1.0 - std::cos(2.0 * kPi * S[s].o[0] / p->geo.n1);
            for (int i = 0; i < D; ++i) {
                const double c = kv[(size_t)s * ncs + symi(D, i, i)];
                p->pre_k0[i] += c;
                sh += c * cx1;
            }
        }
        p->pre_shift = 0.25 * sh / D / nf;
        for (int i = 0; i < 3; ++i) p->pre_k0[i] /= nf;
        p->pre_s0 = p->pre_k0[0] > 0 ? p->pre_k0[0] : 1.0;
    }

    if (D == 2 && p->kern.model == PD_BB_LINEAR) {
        // per-bond constants of the direct strain-energy sum (Eq. 42 with the
        // bond weights of Eq. 46): xi and alpha omega / |xi|^2 dV
        std::vector<T> et((size_t)ns * 4, T(0));
        int emt = 0;
        for (int q = 0; q < ns; ++q) {
            const Bond& bd = S[q];
            et[4 * (size_t)q + 0] = T(bd.xi[0]);
            et[4 * (size_t)q + 1] = T(bd.xi[1]);
            et[4 * (size_t)q + 2] = T(p->alpha * om(bd.r) / (bd.r * bd.r) * p->dV);
            emt = std::max(emt, std::max(std::abs(bd.o[0]), std::abs(bd.o[1])));
        }
        p->emt = emt;
        HIP_TRY(hipMalloc(&p->etab, sizeof(T) * et.size()));
        HIP_TRY(hipMemcpy(p->etab, et.data(), sizeof(T) * et.size(), hipMemcpyHostToDevice));
        p->bytes += sizeof(T) * et.size();
    }
    HIP_TRY(hipMalloc(&p->offs_dev, sizeof(int) * offs.size()));
    HIP_TRY(hipMalloc(&p->kval_dev, sizeof(double) * kv.size()));
    uint8_t* par_dev = nullptr;
    HIP_TRY(hipMalloc(&par_dev, par.size()));
    HIP_TRY(hipMemcpyAsync(p->offs_dev, offs.data(), sizeof(int) * offs.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(p->kval_dev, kv.data(), sizeof(double) * kv.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(par_dev, par.data(), par.size(), hipMemcpyHostToDevice, st));

    const Geo& g = p->geo;
    const long NP = (D == 2) ? (long)g.h1 : (long)g.h1 * g.n2;
    HIP_TRY(hipMalloc(&p->taps, sizeof(T) * NP * p->ntap * nct));
    HIP_TRY(hipMalloc(&p->taps_d, sizeof(T) * NP * p->ntap * nct));
    p->bytes += 2 * sizeof(T) * NP * p->ntap * nct;
    {
        long n = NP * p->ntap;
        const double inv = 1.0 / (double)p->nfft, nl = (double)(D == 2 ? g.n2 : g.n3);
        hipLaunchKernelGGL((k_taps<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, D, g.n1, g.n2, g.h1, NP,
                           p->ntap, ns, p->offs_dev, p->kval_dev, ncs, nct, par_dev, p->tw64, g.twn1,
                           inv, 2.0 * inv, reinterpret_cast<T*>(p->taps));
        HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL((k_taps<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, D, g.n1, g.n2, g.h1, NP,
                           p->ntap, ns, p->offs_dev, p->kval_dev, ncs, nct, par_dev, p->tw64, g.twn1,
                           nl * inv, nl * inv, reinterpret_cast<T*>(p->taps_d));
        HIP_TRY(hipGetLastError());
    }
    // (y, z) direct pass: needs every bond inside the quarter-disc footprint
    // of radius MT = max(|o_y|, |o_z|), 2 or 3
    p->yz_mt = p->yz_nu = 0;
    if (D == 3) {
        int mt = 0;
        for (int s = 0; s < ns; ++s) mt = std::max(mt, std::max(std::abs(S[s].o[1]), std::abs(S[s].o[2])));
        bool fits = mt >= 2 && mt <= 3;
        for (int s = 0; s < ns && fits; ++s)
            fits = S[s].o[1] * S[s].o[1] + S[s].o[2] * S[s].o[2] <= mt * mt;
        if (fits) {
            p->yz_mt = mt;
            p->yz_nu = yz_ntap(mt);
            // LPS: three more components, k_a a0_i, for the force stage's k_a term
            const int nx = (p->kern.model == PD_LPS_LINEAR) ? 3 : 0;
            p->nct_yz = nct + nx;
            const long n = (long)g.h1 * p->yz_nu;
            HIP_TRY(hipMalloc(&p->taps_yz, 2 * sizeof(T) * n * p->nct_yz));
            p->bytes += 2 * sizeof(T) * n * p->nct_yz;
            hipLaunchKernelGGL((k_taps_yz<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g.n1, g.h1, mt,
                               p->yz_nu, ns, p->offs_dev, p->kval_dev, ncs, nct, par_dev, p->tw64, g.twn1,
                               1.0 / (double)g.n1, nx, 6, p->ka, reinterpret_cast<T*>(p->taps_yz));
            HIP_TRY(hipGetLastError());
        }
    }
    HIP_TRY(hipMalloc(&p->stat, sizeof(T) * p->nb * ncs));
    p->bytes += sizeof(T) * p->nb * ncs;
    uint8_t* flags = nullptr;
    HIP_TRY(hipMalloc(&flags, p->nb));
    hipLaunchKernelGGL((k_static<T>), dim3((unsigned)((p->nb + 255) / 256)), dim3(256), 0, st, g.b1, g.b2, g.b3, ns,
                       p->offs_dev, p->kval_dev, ncs, p->chiB, p->chiO, D, reinterpret_cast<T*>(p->stat), flags,
                       p->nb);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
        (void)hipFree(flags);
        return PD_EDEVICE;
    }
    (void)hipFree(p->chiB);
    p->chiB = flags;   // body | interior << 1 | chi_Omega[d] << (2 + d)
    {
        // nodes that read per-node static fields (everything not interior),
        // for the byte accounting of the passes
        std::vector<uint8_t> fh((size_t)p->nb);
        HIP_TRY(hipMemcpy(fh.data(), flags, p->nb, hipMemcpyDeviceToHost));
        long ne = 0;
        for (long i = 0; i < p->nb; ++i) ne += (fh[(size_t)i] & 2) ? 0 : 1;
        p->n_edge = ne;
    }
    {
        // interior values: every bond counted, summed in the same order as k_static
        std::vector<T> si((size_t)ncs);
        for (int c = 0; c < ncs; ++c) {
            double acc = 0.0;
            for (int s = 0; s < ns; ++s) acc += kv[(size_t)s * ncs + c];
            si[(size_t)c] = T(acc);
            if (c < 10) p->stat_int_h[c] = (double)si[(size_t)c];
        }
        HIP_TRY(hipMalloc(&p->stat_int, sizeof(T) * ncs));
        HIP_TRY(hipMemcpy(p->stat_int, si.data(), sizeof(T) * ncs, hipMemcpyHostToDevice));
    }
    HIP_TRY(hipStreamSynchronize(st));
    (void)hipFree(par_dev);
    return PD_OK;
}

inline void plan_free(pd_plan p) {
    if (!p) return;
    if (p->stream0) (void)hipStreamSynchronize(p->stream0);
    void* bufs[] = {p->tw, p->tw64, p->taps, p->taps_d, p->taps_yz, p->stat, p->stat_int, p->chiB, p->chiO, p->SA, p->SB, p->theta,
                    p->vtmp, p->vtmp2, p->partials, p->red, p->offs_dev, p->kval_dev, p->etab};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    if (p->red_host) (void)hipHostFree(p->red_host);
    for (hipEvent_t e : p->lag_ev)
        if (e) (void)hipEventDestroy(e);
    if (p->prof) {
        for (ProfRec& r : *p->prof) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        delete p->prof;
    }
    if (p->sub32) plan_free(p->sub32);
    delete p;
}

template <class T>
pd_status plan_alloc(pd_plan p, hipStream_t st, const uint8_t* chiB_h, const uint8_t* chiO_h) {
    const Geo& g = p->geo;
    const int D = p->dim;
    // twiddles
    int P = 1;
    while (P < std::max(std::max(g.n2, g.n3), is_pow2(g.n1) ? g.n1 : 1)) P <<= 1;
    {
        std::vector<T> tw;
        int off = 0;
        twiddles_host<T>(P, g.n1, tw, &off);
        HIP_TRY(hipMalloc(&p->tw, sizeof(T) * tw.size()));
        HIP_TRY(hipMemcpyAsync(p->tw, tw.data(), sizeof(T) * tw.size(), hipMemcpyHostToDevice, st));
        std::vector<double> tw64;
        twiddles_host<double>(P, g.n1, tw64, &off);
        p->geo.twn1 = off;
        HIP_TRY(hipMalloc(&p->tw64, sizeof(double) * tw64.size()));
        HIP_TRY(hipMemcpyAsync(p->tw64, tw64.data(), sizeof(double) * tw64.size(), hipMemcpyHostToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    // masks
    std::vector<uint8_t> cb((size_t)p->nb, 1), co((size_t)p->nb * D, 1);
    if (chiB_h)
        for (long i = 0; i < p->nb; ++i) cb[i] = chiB_h[i] ? 1 : 0;
    for (int d = 0; d < D; ++d)
        for (long i = 0; i < p->nb; ++i)
            co[(size_t)d * p->nb + i] = chiO_h ? (chiO_h[(size_t)d * p->nb + i] ? 1 : 0) : cb[i];
    // a constrained or unknown component only makes sense on the body
    for (int d = 0; d < D; ++d)
        for (long i = 0; i < p->nb; ++i) co[(size_t)d * p->nb + i] &= cb[i];
    HIP_TRY(hipMalloc(&p->chiB, p->nb));
    HIP_TRY(hipMalloc(&p->chiO, p->nb * D));
    HIP_TRY(hipMemcpy(p->chiB, cb.data(), p->nb, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(p->chiO, co.data(), p->nb * D, hipMemcpyHostToDevice));
    p->bytes += p->nb * (D + 1);
    // workspaces: field capacities by model
    int capA, capB = 0, capC = 0;
    if (D == 2) {
        // weighted + energy: in D+1+nsym, out D+nsym+1; adjoint: in 2D+1+nsym, out 2D+nsym+1
        capA = 2 * D + 1 + nsym(D) + 1;
    } else {
        // LPS: 3 + 1 inputs and the 3 outputs of the (y, z) direct pass
        capA = (p->kern.model == PD_LPS_LINEAR) ? 7 : (2 * D + 1 + nsym(D) + 1);
        capB = (p->kern.model == PD_LPS_LINEAR) ? 4 : (2 * D + 1 + nsym(D) + 1);
        capC = (p->kern.model == PD_LPS_LINEAR) ? 3 : (2 * D + nsym(D) + 1);
    }
    if (p->kern.model == PD_BB_LINEAR && p->kern.weight == PD_WEIGHT_NONE) {
        // unweighted bond-based: force (D) or force+energy (D+1+nsym)
        capA = std::max(capA, D + 1 + nsym(D));
    }
    if (p->kern.model == PD_BB_NONLINEAR) {
        // 8 inputs and 8 outputs in 2D, 13 and 13 in 3D (the (y, z) pass and
        // the grouped FP64 line correlation keep the inputs and write the
        // outputs after them; the y transform path works in place)
        capA = std::max(capA, 2 * (2 * D + 1 + nsym(D)));
        if (D == 3) capB = std::max(capB, 2 * D + 1 + nsym(D));
    }
    p->saf_cap = capA;
    p->sbf_cap = std::max(capB, capC);
    p->scf_cap = 0;
    size_t szA = sizeof(cx<T>) * (size_t)g.saf * capA;
    HIP_TRY(hipMalloc(&p->SA, szA));
    p->bytes += szA;
    if (D == 3) {
        size_t szB = sizeof(cx<T>) * (size_t)p->sbf * std::max(capB, capC);
        HIP_TRY(hipMalloc(&p->SB, szB));
        p->bytes += szB;
    }
    if (p->kern.model == PD_LPS_LINEAR) {
        HIP_TRY(hipMalloc(&p->theta, sizeof(T) * p->nb));
        p->bytes += sizeof(T) * p->nb;
    }
    HIP_TRY(hipMalloc(&p->vtmp, 2 * sizeof(T) * p->nb * D));
    HIP_TRY(hipMalloc(&p->vtmp2, 2 * sizeof(T) * p->nb * D));
    p->bytes += 4 * sizeof(T) * p->nb * D;
    {
        // (the fewest rows per block any x pass takes: 8 for the Verlet c2r)
        const int Lt = std::min(rows_per_block<T>(p), rows_per_block<T>(p, 8));
        long nblk = (long)((g.b2 + Lt - 1) / Lt) * g.b3;
        p->partials_cap = std::max(nblk * 8, 4096L);
        HIP_TRY(hipMalloc(&p->partials, sizeof(double) * p->partials_cap));
        HIP_TRY(hipMalloc(&p->red, sizeof(double) * 16));
        HIP_TRY(hipHostMalloc(&p->red_host, sizeof(double) * 16, hipHostMallocDefault));
        // the device address of the pinned buffer, for reductions that write
        // their result straight to the host (null: results are copied)
        if (hipHostGetDevicePointer((void**)&p->red_host_dev, p->red_host, 0) != hipSuccess) {
            p->red_host_dev = nullptr;
            (void)hipGetLastError();
        }
        // the solver's lagged residual reads wait on these (created once, so
        // that a solve creates no runtime objects)
        for (hipEvent_t& e : p->lag_ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    return PD_OK;
}

inline pd_status plan_create_impl(const pd_grid* grid, const pd_horizon* hz, const pd_kernel* kern, const pd_mask* mask,
                           pd_dtype dtype, int flags, hipStream_t st, pd_plan* out) {
    if (!grid || !hz || !kern || !out) return PD_EINVAL;
    *out = nullptr;
    const int D = grid->dim;
    if (D != 2 && D != 3) return PD_EINVAL;
    if (kern->model == PD_LPS_LINEAR && D != 3) return PD_EUNSUPPORTED;
    if (kern->model != PD_BB_LINEAR && kern->model != PD_LPS_LINEAR && kern->model != PD_BB_NONLINEAR)
        return PD_EINVAL;
    if (kern->model == PD_BB_NONLINEAR && (kern->weight != PD_WEIGHT_NONE || (flags & PD_PLAN_MIXED)))
        return PD_EUNSUPPORTED;
    if (kern->model == PD_LPS_LINEAR && kern->weight != PD_WEIGHT_NONE) return PD_EUNSUPPORTED;
    if (dtype != PD_F32 && dtype != PD_F64) return PD_EINVAL;
    if (!(hz->delta > 0) || (hz->influence != 0 && hz->influence != 1)) return PD_EINVAL;
    if (!(kern->E > 0)) return PD_EINVAL;
    if (kern->model == PD_LPS_LINEAR && !(kern->nu > -1.0 && kern->nu < 0.5)) return PD_EINVAL;
    for (int d = 0; d < 3; ++d) {
        const bool active = d < D;
        const long n = grid->fft_n[d], b = grid->body_n[d];
        if (!active) {
            if (n != 1 || b != 1) return PD_EINVAL;
            continue;
        }
        if (!(grid->dx[d] > 0)) return PD_EINVAL;
        if (b < 1 || n < 1) return PD_EINVAL;
        // x: a power of two, or 2 R 2^p with R = 3, 5, 9 and 2^p >= 8 (the
        // complex half-length is transformed by one radix-R step and R
        // power-of-two transforms); y and z: powers of two
        if (!is_pow2(n) && !(d == 0 && x_radix(n) > 1)) return PD_EUNSUPPORTED;
        const long lo = 16, hi = (d == 0) ? 2048 : 1024;
        if (n < lo || n > hi) return PD_EUNSUPPORTED;
        const long m = (long)std::ceil(hz->delta / grid->dx[d] * (1.0 - 1e-12));
        if (n - b < m) return PD_EINVAL;  // a bond would wrap around the periodic box
    }
    pd_plan p = new pd_plan_s();
    std::memset(p, 0, sizeof(*p));
    p->lastaxis = PD_LASTAXIS_AUTO;
    p->dim = D;
    for (int d = 0; d < 3; ++d) {
        p->n[d] = (int)grid->fft_n[d];
        p->b[d] = (int)grid->body_n[d];
        p->dx[d] = d < D ? grid->dx[d] : 1.0;
    }
    p->delta = hz->delta;
    p->influence = hz->influence;
    p->kern = *kern;
    p->dtype = dtype;
    p->flags = flags;
    p->stream0 = st;
    (void)hipGetDevice(&p->device);
    int maxsm = 65536;
    if (hipDeviceGetAttribute(&maxsm, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device) != hipSuccess) maxsm = 65536;
    p->max_lds = std::max(32768, maxsm);
    Geo& g = p->geo;
    g.dim = D;
    g.n1 = p->n[0]; g.n2 = p->n[1]; g.n3 = p->n[2];
    g.b1 = p->b[0]; g.b2 = p->b[1]; g.b3 = p->b[2];
    g.Nc = g.n1 / 2;
    g.h1 = g.Nc + 1;
    g.rad = x_radix(g.n1);
    {
        int lg = 0;
        while ((g.rad << (lg + 1)) <= g.Nc) ++lg;
        g.lgM = lg;   // Nc = rad 2^lgM
    }
    g.P2 = ((g.b2 + 15) / 16) * 16;
    g.nb = (long)g.b1 * g.b2 * g.b3;
    g.saf = (long)g.b3 * g.h1 * g.P2;
    g.sbf = (long)g.b3 * g.h1 * g.n2;
    p->Pz = ((g.b3 + 15) / 16) * 16;
    p->sbf = (long)g.h1 * g.n2 * p->Pz;
    p->nb = g.nb;
    p->nfft = (long)g.n1 * g.n2 * g.n3;
    p->dV = p->dx[0] * p->dx[1] * (D == 3 ? p->dx[2] : 1.0);

    std::vector<Bond> S = make_stencil(D, p->dx, p->delta);
    p->ns = (int)S.size();
    if (p->ns == 0) { delete p; return PD_EINVAL; }
    p->m0 = 0;
    for (const Bond& bd : S) p->m0 += (p->influence == 0 ? 1.0 / bd.r : 1.0) * bd.r * bd.r * p->dV;
    p->alpha = bb_alpha(D, p->influence, kern->E, p->delta);
    if (kern->model == PD_LPS_LINEAR) {
        p->kappa = kern->E / (3.0 * (1.0 - 2.0 * kern->nu));
        p->mu = kern->E / (2.0 * (1.0 + kern->nu));
        p->ka = (3.0 * p->kappa - 5.0 * p->mu) / p->m0;
    }
    p->Wc = (kern->weight == PD_WEIGHT_INTEGRITY && kern->G0 > 0) ? kern->G0 / p->delta : 0.0;
    const double lmax = symbol_lambda_max(p, S);
    p->dt_max = (lmax > 0 && kern->rho > 0) ? 2.0 / std::sqrt(lmax / kern->rho) : 0.0;

    pd_status s = (dtype == PD_F32) ? plan_alloc<float>(p, st, mask ? mask->chi_B : nullptr, mask ? mask->chi_Omega : nullptr)
                                    : plan_alloc<double>(p, st, mask ? mask->chi_B : nullptr, mask ? mask->chi_Omega : nullptr);
    if (s == PD_OK)
        s = (dtype == PD_F32) ? build_device_tables<float>(p, S, st) : build_device_tables<double>(p, S, st);
    if (s == PD_OK && (flags & PD_PLAN_MIXED)) {
        if (dtype != PD_F64) s = PD_EINVAL;
        else s = plan_create_impl(grid, hz, kern, mask, PD_F32, 0, st, &p->sub32);
        if (s == PD_OK) p->sub32->parent = p;
    }
    if (s != PD_OK) {
        plan_free(p);
        return s;
    }
    *out = p;
    return PD_OK;
}

// ------------------------------------------------------- strain energy
// Strain energy density of the weighted linearized bond-based solid by
// direct bond sums (Eq. 42 with the bond weights of Eq. 46/100, as Eq. 47
// defines it before its convolution form, Eq. 64/102):
//   W(x) = 1/2 phi(x) sum_o phi(x + o) alpha omega (xi . eta)^2 / |xi|^2 dV,
// eta = u(x + o) - u(x), phi = chi_B lambda or chi_B s, zero beyond the body
// box.  The convolution form expands (xi . eta)^2 into terms of order
// (chi u)^2 that cancel down to (u' - u)^2: in FP32, once displacements reach
// a grid spacing (a split plate), the cancellation error exceeds W_c.  The
// direct sum forms eta first.  A block takes a tile of EW_TX x EW_TY nodes;
// u and phi of the tile and a halo of M nodes go through LDS; each thread
// sums the bonds of one node in stencil order (bond constants are
// block-uniform: scalar loads).
constexpr int EW_TX = 64, EW_TY = 4;
template <class T, int WK>
__global__ void __launch_bounds__(EW_TX * EW_TY)
k_energy_bb2d(int b1, int b2, int ns, int M, const int* __restrict__ offs, const T* __restrict__ et,
              const T* __restrict__ u, const uint8_t* __restrict__ chiB, const uint8_t* __restrict__ lam,
              const T* __restrict__ s, T* __restrict__ W) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* su0 = reinterpret_cast<T*>(smem_raw);
    const int PX = EW_TX + 2 * M, PY = EW_TY + 2 * M;
    T* su1 = su0 + PX * PY;
    T* sph = su1 + PX * PY;
    const long nb = (long)b1 * b2;
    const int x0 = blockIdx.x * EW_TX, y0 = blockIdx.y * EW_TY;
    for (int q = threadIdx.x; q < PX * PY; q += blockDim.x) {
        const int gx = x0 - M + q % PX, gy = y0 - M + q / PX;
        const bool in = gx >= 0 && gx < b1 && gy >= 0 && gy < b2;
        const long k = in ? (long)gy * b1 + gx : 0;
        T ph = (in && (chiB[k] & 1)) ? T(1) : T(0);
        if constexpr (WK == WK_LAMBDA) ph = (in && lam[k]) ? ph : T(0);
        if constexpr (WK == WK_SCALE) ph *= in ? s[k] : T(0);
        su0[q] = in ? u[k] : T(0);
        su1[q] = in ? u[nb + k] : T(0);
        sph[q] = ph;
    }
    __syncthreads();
    const int tx = threadIdx.x % EW_TX, ty = threadIdx.x / EW_TX;
    const int gx = x0 + tx, gy = y0 + ty;
    if (gx >= b1 || gy >= b2) return;
    const int c = (ty + M) * PX + tx + M;
    const T u0 = su0[c], u1 = su1[c], pc = sph[c];
    T acc = T(0);
    for (int q = 0; q < ns; ++q) {
        const int n = c + offs[3 * q + 1] * PX + offs[3 * q];
        const T e = et[4 * q] * (su0[n] - u0) + et[4 * q + 1] * (su1[n] - u1);
        acc += et[4 * q + 2] * e * e * sph[n];
    }
    W[(long)gy * b1 + gx] = T(0.5) * pc * acc;
}

template <class T>
pd_status launch_energy(pd_plan p, const T* u, const uint8_t* lam, const T* s, T* W, hipStream_t st) {
    if (p->dim != 2 || !p->etab || !W) return PD_EUNSUPPORTED;
    const Geo& g = p->geo;
    const int M = p->emt;
    const size_t lds = (size_t)3 * (EW_TX + 2 * M) * (EW_TY + 2 * M) * sizeof(T);
    if (lds > (size_t)p->max_lds) return PD_EUNSUPPORTED;
    dim3 grid((g.b1 + EW_TX - 1) / EW_TX, (g.b2 + EW_TY - 1) / EW_TY), block(EW_TX * EW_TY);
    ProfScope ps(p, st);
    auto go = [&](auto kern) {
        allow_lds(kern, lds);
        hipLaunchKernelGGL(kern, grid, block, lds, st, g.b1, g.b2, p->ns, M, p->offs_dev,
                           reinterpret_cast<const T*>(p->etab), u, p->chiB, lam, s, W);
    };
    if (p->kern.weight == PD_WEIGHT_INTEGRITY) go(k_energy_bb2d<T, WK_LAMBDA>);
    else if (p->kern.weight == PD_WEIGHT_SCALE) go(k_energy_bb2d<T, WK_SCALE>);
    else go(k_energy_bb2d<T, WK_NONE>);
    if (p->prof) {
        const double t = sizeof(T);
        double per = 2 * t + 1 + t + (p->kern.weight == PD_WEIGHT_INTEGRITY ? 1.0 : 0.0) +
                     (p->kern.weight == PD_WEIGHT_SCALE ? t : 0.0);
        ps.done("energy_direct", per * (double)g.nb);
    }
    return pdh::check(hipGetLastError());
}

// ------------------------------------------------------------------ force
// The two LPS chains: the dilatation (generator gA, epilogue fA writing
// theta) and the force (multiplier mB, epilogue fB).  With the (y, z) pass
// the dilatation's c2r and the force stage's r2c of chi theta run as one
// pass (FinThetaChain): x transform of chi u -> SA 0..2, (y, z) dilatation
// -> SA 4, c2r + theta + r2c -> SA 3, (y, z) force stage SA 0..3 -> SA
// 4..6, c2r + epilogue.
// have_spectra: slots 0 .. 2 already hold the chi u spectra (made by the
// previous step's chained epilogue), so the first pass is skipped.  A
// chained force-stage epilogue (FB::NCHAIN > 0) transforms its outputs into
// slots 0 .. 2, which the force stage's (y, z) pass has finished reading.
template <class T>
bool lps_yz(pd_plan p) {
    return use_yz<T, MulLPSA<T>>(p) && use_yz<T, MulLPSB<T>>(p);
}
template <class T, class GA, class FB>
pd_status run_lps(pd_plan p, const GA& gA, const FinTheta<T>& fA, const MulLPSB<T>& mB, const FB& fB,
                  hipStream_t st, bool have_spectra = false) {
    constexpr bool CHAIN = fin_chain_n<FB>::value > 0;
    if (lps_yz<T>(p)) {
        const Geo& g = p->geo;
        cx<T>* SA = SAp<T>(p);
        if (p->saf_cap < 7) return PD_EINVAL;
        if (!have_spectra) PD_TRY(launch_xfwd<T>(p, gA, SA, st));
        PD_TRY((launch_yzconv<T, MulLPSA<T>>(p, MulLPSA<T>{}, 0, 4, st)));
        FinThetaChain<T> fc{};
        static_cast<FinTheta<T>&>(fc) = fA;
        PD_TRY(launch_xinv<T>(p, fc, SA + 4 * g.saf, st, SA + 3 * g.saf));
        PD_TRY((launch_yzconv<T, MulLPSB<T>>(p, mB, 0, 4, st)));
        return launch_xinv<T>(p, fB, SA + 4 * g.saf, st, CHAIN ? SA : nullptr);
    }
    if (have_spectra || CHAIN) return PD_EINVAL;   // only the (y, z) path chains the steps
    PD_TRY(run_chain<T>(p, gA, MulLPSA<T>{}, fA, st, 0, 3));
    GenTheta<T> gB{};
    gB.c = ctx<T>(p);
    gB.theta = fA.theta;
    return run_chain<T>(p, gB, mB, fB, st, 3);
}

template <class T>
pd_status force_impl(pd_plan p, const T* u, const void* weight, T* L, T* W, hipStream_t st) {
    const int D = p->dim;
    const pd_weight_kind wk = p->kern.weight;
    if (wk != PD_WEIGHT_NONE && !weight) return PD_EINVAL;
    if (p->kern.model == PD_LPS_LINEAR) {
        if (W) return PD_EUNSUPPORTED;
        // stage A: dilatation
        GenU<T, 3, WK_NONE, false, false, false> gA{};
        gA.c = ctx<T>(p);
        gA.u = const_cast<T*>(u);
        FinTheta<T> fA{};
        fA.c = ctx<T>(p);
        fA.u = u;
        fA.theta = reinterpret_cast<T*>(p->theta);
        // stage B: force
        MulLPSB<T> mB{};
        mB.ka = T(p->ka);
        FinLin<T, 3, 0, false, true> fB{};
        fB.c = ctx<T>(p);
        fB.ka = T(p->ka);
        fB.u = u;
        fB.theta = reinterpret_cast<const T*>(p->theta);
        fB.L = L;
        return run_lps<T>(p, gA, fA, mB, fB, st);
    }
    if (p->kern.model == PD_BB_NONLINEAR) {
        if (W) return PD_EUNSUPPORTED;
        auto nbb = [&](auto Dc) -> pd_status {
            constexpr int DD = decltype(Dc)::value;
            GenNBB<T, DD> gg{};
            gg.c = ctx<T>(p);
            gg.u = u;
            FinNBB<T, DD> ff{};
            ff.c = ctx<T>(p);
            ff.u = u;
            ff.L = L;
            if constexpr (DD == 3) {
                // x transform, the (y, z) pass in output groups, inverse x
                // transform (the y-transform path otherwise)
                constexpr int NI = MulNBB<T, 3>::NIN, NO = MulNBB<T, 3>::NOUT;
                if (use_yz<T, YzNBB<T, 0, nbb_yz_group<T>()>>(p) && p->saf_cap >= NI + NO) {
                    PD_TRY(launch_xfwd<T>(p, gg, SAp<T>(p), st));
                    PD_TRY(nbb_yz<T>(p, NI, st));
                    return launch_xinv<T>(p, ff, SAp<T>(p) + (long)NI * p->geo.saf, st);
                }
            } else if constexpr (sizeof(T) == 8) {
                // FP64 2D: the line correlation in four groups of 2 outputs
                // (with more outputs per group the points of the 8 inputs and
                // the outputs exceed the registers of two waves and spill),
                // written after the inputs
                constexpr int NI = MulNBB<T, 2>::NIN, NO = MulNBB<T, 2>::NOUT;
                if (p->lastaxis == PD_LASTAXIS_AUTO && p->saf_cap >= NI + NO) {
                    PD_TRY(launch_xfwd<T>(p, gg, SAp<T>(p), st));
                    PD_TRY((nbb2_lines_from<T, 0>(p, NI, st)));
                    return launch_xinv<T>(p, ff, SAp<T>(p) + (long)NI * p->geo.saf, st);
                }
            }
            return run_chain<T>(p, gg, MulNBB<T, DD>{}, ff, st);
        };
        return p->dim == 2 ? nbb(std::integral_constant<int, 2>{}) : nbb(std::integral_constant<int, 3>{});
    }
    // bond-based
    auto go = [&](auto Dc) -> pd_status {
        constexpr int DD = decltype(Dc)::value;
        if (wk == PD_WEIGHT_NONE && !W) {
            GenU<T, DD, WK_NONE, false, false, false> gg{};
            gg.c = ctx<T>(p);
            gg.u = const_cast<T*>(u);
            FinLin<T, DD, 0, false, false> ff{};
            ff.c = ctx<T>(p);
            ff.u = u;
            ff.L = L;
            return run_chain<T>(p, gg, MulBB<T, DD, false, false>{}, ff, st);
        }
        if constexpr (DD == 3) {
            return PD_EUNSUPPORTED;  // weighted bond-based chains are built for 2D plates
        } else {
        auto weighted = [&](auto WKc) -> pd_status {
            constexpr int WK = decltype(WKc)::value;
            const uint8_t* lam = (WK == WK_LAMBDA) ? reinterpret_cast<const uint8_t*>(weight) : nullptr;
            const T* s = (WK == WK_SCALE) ? reinterpret_cast<const T*>(weight) : nullptr;
            if (W && p->energy_form == 1) {
                // the convolution form of W (Eq. 102) in the same chain
                GenU<T, DD, WK, true, true, false> gg{};
                gg.c = ctx<T>(p);
                gg.u = const_cast<T*>(u);
                gg.lam_in = lam;
                gg.s = s;
                FinBB<T, DD, WK, true, true, false, false> ff{};
                ff.c = ctx<T>(p);
                ff.u = u; ff.lam = lam; ff.s = s; ff.L = L; ff.Wout = W;
                return run_chain<T>(p, gg, MulBB<T, DD, true, true>{}, ff, st);
            } else {
                GenU<T, DD, WK, true, false, false> gg{};
                gg.c = ctx<T>(p);
                gg.u = const_cast<T*>(u);
                gg.lam_in = lam;
                gg.s = s;
                FinBB<T, DD, WK, true, false, false, false> ff{};
                ff.c = ctx<T>(p);
                ff.u = u; ff.lam = lam; ff.s = s; ff.L = L;
                PD_TRY(run_chain<T>(p, gg, MulBB<T, DD, true, false>{}, ff, st));
                return W ? launch_energy<T>(p, u, lam, s, W, st) : PD_OK;
            }
        };
        if (wk == PD_WEIGHT_INTEGRITY) return weighted(std::integral_constant<int, WK_LAMBDA>{});
        if (wk == PD_WEIGHT_SCALE) return weighted(std::integral_constant<int, WK_SCALE>{});
        return weighted(std::integral_constant<int, WK_NONE>{});
        }
    };
    return D == 2 ? go(std::integral_constant<int, 2>{}) : go(std::integral_constant<int, 3>{});
}

}  // namespace pdi

// ------------------------------------------------------- elementwise kernels
namespace pdi {

constexpr int EW_THREADS = 256;

// grid-stride elementwise kernels use at most 2048 blocks (partials capacity)
inline unsigned ew_blocks(long n) { return (unsigned)std::max<long>(1, std::min<long>((n + EW_THREADS - 1) / EW_THREADS, 2048L)); }

// y[k] += x[k]  (k < n)
template <class T>
__global__ void k_add(T* __restrict__ y, const T* __restrict__ x, long n) {
    for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) y[k] += x[k];
}

// u = chi_O u + (1 - chi_O) w   and   t = (1 - chi_O) w
template <class T>
__global__ void k_constrain(T* __restrict__ u, T* __restrict__ t, const T* __restrict__ w,
                            const uint8_t* __restrict__ chiO, long n) {
    for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
        const T wk = w ? w[k] : T(0);
        if (u) u[k] = chiO[k] ? u[k] : wk;
        if (t) t[k] = chiO[k] ? T(0) : wk;
    }
}

// Block partial sums of NR FP64 accumulators, written to part[blockIdx*NR].
template <int NR>
__device__ __forceinline__ void ew_block_reduce(double (&acc)[NR], double* part) {
    __shared__ double sm[(EW_THREADS / 64) * 4];
    block_reduce_store<NR>(acc, part + (long)blockIdx.x * NR, sm);
}

// CG coefficients stay on the device: alpha = rho / (p . Ap) and
// beta = rho_new / rho are formed by every thread from the reduction results
// (0 when the denominator is 0), so no scalar travels through the host.
__device__ __forceinline__ double dev_ratio(const double* __restrict__ num, const double* __restrict__ den) {
    const double d = den[0];
    return d != 0.0 ? num[0] / d : 0.0;
}
// Thread 0 of block 0 keeps rho_new for the next iteration's alpha (a slot
// that no thread of the launch reads).
__device__ __forceinline__ void keep_rho(double* __restrict__ save, const double* __restrict__ num) {
    if (save && blockIdx.x == 0 && threadIdx.x == 0) save[0] = num[0];
}

// CG update: x += a p; r -= a Ap; partial |r|^2, a = num / den.  (types may
// differ: x is the iterate precision, r/p/Ap the operator precision)
template <class TX, class T>
__global__ void k_cg_update(TX* __restrict__ x, const T* __restrict__ p, T* __restrict__ r, const T* __restrict__ Ap,
                            const double* __restrict__ num, const double* __restrict__ den, long n,
                            double* __restrict__ part) {
    const double a = dev_ratio(num, den);
    double acc[1] = {0.0};
    for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
        x[k] = TX(double(x[k]) + a * double(p[k]));
        T rk = T(double(r[k]) - a * double(Ap[k]));
        r[k] = rk;
        acc[0] += double(rk) * double(rk);
    }
    ew_block_reduce<1>(acc, part);
}

// p = r + b p, b = num / den
template <class T>
__global__ void k_cg_dir(T* __restrict__ p, const T* __restrict__ r, const double* __restrict__ num,
                         const double* __restrict__ den, double* __restrict__ save, long n) {
    const double b = dev_ratio(num, den);
    keep_rho(save, num);
    for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x)
        p[k] = T(double(r[k]) + b * double(p[k]));
}

// Mixed-precision CG vectors: the iterate and residual in FP64, the
// direction in FP32, the precision the operator reads it in.
// p32 = (float) r
static __global__ void k_cgm_start(float* __restrict__ p32, const double* __restrict__ r, long n) {
    for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x)
        p32[k] = float(r[k]);
}
// x += a p32 (FP64 iterate);  r32 -= a Ap32 (formed in FP64, stored in
// FP32: the recursively updated residual is replaced by the FP64 one before
// its rounding accumulates); partial |r32|^2 in FP64, a = num / den
static __global__ void k_cgm_update(double* __restrict__ x, const float* __restrict__ p32, float* __restrict__ r32,
                                    const float* __restrict__ Ap32, const double* __restrict__ num,
                                    const double* __restrict__ den, long n, double* __restrict__ part) {
    const double a = dev_ratio(num, den);
    double acc[1] = {0.0};
    for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
        x[k] += a * double(p32[k]);
        const float rk = float(double(r32[k]) - a * double(Ap32[k]));
        r32[k] = rk;
        acc[0] += double(rk) * double(rk);
    }
    ew_block_reduce<1>(acc, part);
}
// p32 = (float) (r + b p32), b = num / den
static __global__ void k_cgm_dir(float* __restrict__ p32, const float* __restrict__ r32,
                                 const double* __restrict__ num, const double* __restrict__ den,
                                 double* __restrict__ save, long n) {
    const double b = dev_ratio(num, den);
    keep_rho(save, num);
    for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x)
        p32[k] = float(double(r32[k]) + b * double(p32[k]));
}
// r32 = (float) r (the FP64 residual of a replacement)
static __global__ void k_to32(float* __restrict__ r32, const double* __restrict__ r, long n) {
    for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x)
        r32[k] = float(r[k]);
}

// Preconditioned CG directions: p = z + b p, b = num / den
template <class T>
__global__ void k_pcg_dir(T* __restrict__ p, const T* __restrict__ z, const double* __restrict__ num,
                          const double* __restrict__ den, double* __restrict__ save, long n) {
    const double b = dev_ratio(num, den);
    keep_rho(save, num);
    for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x)
        p[k] = T(double(z[k]) + b * double(p[k]));
}
// mixed, preconditioned: p32 = (float) (z32 + b p32), b = num / den
static __global__ void k_pcgm_dir(float* __restrict__ p32, const float* __restrict__ z32,
                                  const double* __restrict__ num, const double* __restrict__ den,
                                  double* __restrict__ save, long n) {
    const double b = dev_ratio(num, den);
    keep_rho(save, num);
    for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x)
        p32[k] = float(double(z32[k]) + b * double(p32[k]));
}

// Verlet adjoint helpers
template <class T>
__global__ void k_mask_copy(T* __restrict__ a, const T* __restrict__ vb, const uint8_t* __restrict__ chiO, long n) {
    for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x)
        a[k] = chiO[k] ? vb[k] : T(0);
}
// ut = chi_O (ub + c1 La)
template <class T>
__global__ void k_vva_ut(T* __restrict__ ut, const T* __restrict__ ub, const T* __restrict__ La, T c1,
                         const uint8_t* __restrict__ chiO, long n) {
    for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x)
        ut[k] = chiO[k] ? ub[k] + c1 * La[k] : T(0);
}
// ub = c1 La + ut + c2 Lut;  vb = a + dt ut;  bb += c2 ut + 2 c1 a (bb may be null)
template <class T>
__global__ void k_vva_final(T* __restrict__ ub, T* __restrict__ vb, T* __restrict__ bb, const T* __restrict__ a,
                            const T* __restrict__ ut, const T* __restrict__ La, const T* __restrict__ Lut, T c1, T c2,
                            T dt, long n) {
    for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
        const T ak = a[k], utk = ut[k];
        ub[k] = c1 * La[k] + utk + c2 * Lut[k];
        vb[k] = ak + dt * utk;
        if (bb) bb[k] += c2 * utk + T(2) * c1 * ak;
    }
}

template <int NR>
pd_status ew_finish(pd_plan p, unsigned nblk, double* out, hipStream_t st, double* host = nullptr) {
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, st, p->partials, (long)nblk, NR, out, host);
    return pdh::check(hipGetLastError());
}

inline pd_status fetch_red(pd_plan p, int n, hipStream_t st, double* dst) {
    HIP_TRY(hipMemcpyAsync(p->red_host, p->red, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int i = 0; i < n; ++i) dst[i] = p->red_host[i];
    return PD_OK;
}

// ------------------------------------------------------------ operator kinds
// Apply one linear chain with a FinLin epilogue: MODE 0 force, 2 CG operator
// Ap = -chi_O L(x), 3 residual chi_O (L(x) + b).  Unweighted plans only.
template <class T, int MODE>
pd_status lin_apply(pd_plan p, const T* x, T* out, const T* b, hipStream_t st) {
    const int D = p->dim;
    if (p->kern.model == PD_LPS_LINEAR) {
        GenU<T, 3, WK_NONE, false, false, false> gA{};
        gA.c = ctx<T>(p);
        gA.u = const_cast<T*>(x);
        FinTheta<T> fA{};
        fA.c = ctx<T>(p);
        fA.u = x;
        fA.theta = reinterpret_cast<T*>(p->theta);
        MulLPSB<T> mB{};
        mB.ka = T(p->ka);
        FinLin<T, 3, MODE, false, true> fB{};
        fB.c = ctx<T>(p);
        fB.ka = T(p->ka);
        fB.u = x;
        fB.theta = reinterpret_cast<const T*>(p->theta);
        fB.L = out;
        fB.b = b;
        return run_lps<T>(p, gA, fA, mB, fB, st);
    }
    auto go = [&](auto Dc) -> pd_status {
        constexpr int DD = decltype(Dc)::value;
        GenU<T, DD, WK_NONE, false, false, false> gg{};
        gg.c = ctx<T>(p);
        gg.u = const_cast<T*>(x);
        FinLin<T, DD, MODE, false, false> ff{};
        ff.c = ctx<T>(p);
        ff.u = x;
        ff.L = out;
        ff.b = b;
        return run_chain<T>(p, gg, MulBB<T, DD, false, false>{}, ff, st);
    };
    return D == 2 ? go(std::integral_constant<int, 2>{}) : go(std::integral_constant<int, 3>{});
}

// --------------------------------------------------------------- Verlet
// Spectral preconditioner z = chi_O M^-1 chi_O r (M: periodic unmasked
// bond-based symbol, see MulPre); p->red[0] = r . z.  T is the chain
// precision, r is read as TR and z stored as TZ.
template <class T, class TR, class TZ>
pd_status precond_apply(pd_plan p, const TR* r, TZ* z, hipStream_t st) {
    auto go = [&](auto Dc) -> pd_status {
        constexpr int DD = decltype(Dc)::value;
        GenMasked<T, DD, TR> gg{};
        gg.c = ctx<T>(p);
        gg.r = r;
        MulPre<T, DD> mm{};
        const double s0 = p->pre_s0;
        for (int i = 0; i < 3; ++i) mm.k0n[i] = T((p->pre_k0[i] + p->pre_shift) / s0);
        mm.kscale = T(1.0 / s0);
        mm.outscale = T(1.0 / ((double)p->nfft * (double)p->nfft * s0));
        FinPre<T, DD, TR, TZ> ff{};
        ff.c = ctx<T>(p);
        ff.r = r;
        ff.z = z;
        return run_chain<T>(p, gg, mm, ff, st);
    };
    return p->dim == 2 ? go(std::integral_constant<int, 2>{}) : go(std::integral_constant<int, 3>{});
}

// One EC velocity-Verlet step.  vh_in / vh_out (inside a multi-step call): v
// holds the half-step velocity v + dt/(2 rho) F on entry / is left holding
// it on exit, and F is then neither read nor written.  drifted: the
// previous step already made this step's position update; *drift_out: this
// step made the next one's.
template <class T, bool ENRED>
pd_status verlet_one(pd_plan p, pd_state* S, const T* b, const T* w, T dt, double* nanflag, int vh_in, int vh_out,
                     int drifted, int* drift_out, hipStream_t st) {
    *drift_out = 0;
    const int D = p->dim;
    const T rho = T(p->kern.rho);
    const T c1 = dt / (T(2) * rho), c2 = dt * dt / (T(2) * rho);
    T* u = reinterpret_cast<T*>(S->u);
    T* v = reinterpret_cast<T*>(S->v);
    T* F = reinterpret_cast<T*>(S->F);
    if (p->kern.model == PD_LPS_LINEAR) {
        FinTheta<T> fA{};
        fA.c = ctx<T>(p);
        fA.u = u;
        fA.theta = reinterpret_cast<T*>(p->theta);
        MulLPSB<T> mB{};
        mB.ka = T(p->ka);
        // whether the inner epilogue also transforms the next chi u (FP64)
        constexpr bool CH = fin_chain_n<FinLin<T, 3, 1, false, true, true>>::value > 0;
        auto go = [&](auto gA, auto fB) -> pd_status {
            gA.c = ctx<T>(p);
            gA.u = u; gA.v = v; gA.F = F; gA.w = w; gA.dt = dt; gA.c2 = c2; gA.vhalf = vh_in;
            fB.c = ctx<T>(p);
            fB.ka = T(p->ka); fB.u = u; fB.theta = reinterpret_cast<const T*>(p->theta);
            fB.v = v; fB.F = F; fB.b = b; fB.c1 = c1; fB.rho = rho; fB.nanflag = nanflag;
            fB.vh_in = vh_in; fB.vh_out = vh_out;
            fB.u_next = u; fB.dt = dt;
            // after a chained step the chi u spectra of this step are in place
            return run_lps<T>(p, gA, fA, mB, fB, st, CH && drifted != 0);
        };
        // The inner steps of a call (no F read or written; no prescribed
        // displacement) run generator and epilogue instances of their own,
        // with the half-step flags fixed at compile time and no registers or
        // loads for F and w.  The inner epilogue also makes the next step's
        // position update (12 B per node and step less), after which that
        // step's first pass is the plain chi u transform (GenP); in FP64, on
        // the (y, z) path, the epilogue also transforms chi u, and the next
        // step starts at its first (y, z) pass.  (256^3 FP32: the instances
        // ran the force-stage c2r pass 10 % and the first x pass 6 % faster.)
        using GenG = GenU<T, 3, WK_NONE, false, false, true>;
        using FinG = FinLin<T, 3, 1, ENRED, true>;
        if constexpr (!ENRED) {
            using GenI = GenU<T, 3, WK_NONE, false, false, true, true>;
            using GenP = GenU<T, 3, WK_NONE, false, false, false>;
            using FinI = FinLin<T, 3, 1, false, true, true>;
            const bool fi = vh_in && vh_out && !w && (!CH || lps_yz<T>(p));
            *drift_out = fi ? 1 : 0;
            if (drifted) return fi ? go(GenP{}, FinI{}) : go(GenP{}, FinG{});
            if (vh_in && !w) return fi ? go(GenI{}, FinI{}) : go(GenI{}, FinG{});
        }
        if (drifted) return PD_EINVAL;   // not reached: only the inner epilogue chains
        return go(GenG{}, FinG{});
    }
    auto go = [&](auto Dc) -> pd_status {
        constexpr int DD = decltype(Dc)::value;
        const pd_weight_kind wk = p->kern.weight;
        if (wk == PD_WEIGHT_NONE) {
            GenU<T, DD, WK_NONE, false, false, true> gg{};
            gg.c = ctx<T>(p);
            gg.u = u; gg.v = v; gg.F = F; gg.w = w; gg.dt = dt; gg.c2 = c2; gg.vhalf = vh_in;
            FinLin<T, DD, 1, ENRED, false> ff{};
            ff.c = ctx<T>(p);
            ff.u = u; ff.v = v; ff.F = F; ff.b = b; ff.c1 = c1; ff.rho = rho; ff.nanflag = nanflag;
            ff.vh_in = vh_in; ff.vh_out = vh_out;
            return run_chain<T>(p, gg, MulBB<T, DD, false, false>{}, ff, st);
        }
        if constexpr (DD == 3) {
            return PD_EUNSUPPORTED;
        } else {
        auto weighted = [&](auto WKc, auto Ec) -> pd_status {
            constexpr int WK = decltype(WKc)::value;
            constexpr bool E = decltype(Ec)::value;
            GenU<T, DD, WK, true, E, true> gg{};
            gg.c = ctx<T>(p);
            gg.u = u; gg.v = v; gg.F = F; gg.w = w; gg.dt = dt; gg.c2 = c2; gg.vhalf = vh_in;
            gg.lam_in = S->lambda; gg.lam_out = S->lambda; gg.s = reinterpret_cast<const T*>(S->s);
            gg.W = reinterpret_cast<const T*>(S->W); gg.Wc = T(p->Wc); gg.fail = (S->W && p->Wc > 0) ? 1 : 0;
            FinBB<T, DD, WK, true, E, true, ENRED> ff{};
            ff.c = ctx<T>(p);
            ff.u = u; ff.lam = S->lambda; ff.s = reinterpret_cast<const T*>(S->s); ff.Wout = reinterpret_cast<T*>(S->W);
            ff.v = v; ff.F = F; ff.b = b; ff.c1 = c1; ff.rho = rho; ff.nanflag = nanflag;
            ff.vh_in = vh_in; ff.vh_out = vh_out;
            return run_chain<T>(p, gg, MulBB<T, DD, true, E>{}, ff, st);
        };
        if (wk == PD_WEIGHT_INTEGRITY) {
            if (S->W && p->energy_form == 1)
                return weighted(std::integral_constant<int, WK_LAMBDA>{}, std::true_type{});
            PD_TRY(weighted(std::integral_constant<int, WK_LAMBDA>{}, std::false_type{}));
            // W of the new state (u, lambda after this step's update) decides
            // the next step's failures
            if (S->W) return launch_energy<T>(p, u, S->lambda, nullptr, reinterpret_cast<T*>(S->W), st);
            return PD_OK;
        }
        return weighted(std::integral_constant<int, WK_SCALE>{}, std::false_type{});
        }
    };
    return D == 2 ? go(std::integral_constant<int, 2>{}) : go(std::integral_constant<int, 3>{});
}

template <class T>
pd_status force_impl_any(pd_plan p, const T* u, const void* weight, T* L, T* W, hipStream_t st);

// slot of red / red_host holding the Verlet call's non-finite flag
constexpr int kNanSlot = 12;

template <class T>
pd_status verlet_impl(pd_plan p, pd_state* S, const T* b, const T* w, double dt, int nsteps, double* energy,
                      hipStream_t st) {
    if (!S || !S->u || !S->v || !S->F) return PD_EINVAL;
    if (!(dt > 0) || nsteps < 0) return PD_EINVAL;
    if (p->dt_max > 0 && dt > p->dt_max) return PD_EINVAL;
    if (p->kern.weight == PD_WEIGHT_INTEGRITY && !S->lambda) return PD_EINVAL;
    if (p->kern.weight == PD_WEIGHT_SCALE && !S->s) return PD_EINVAL;
    if (p->kern.weight == PD_WEIGHT_INTEGRITY && p->Wc > 0 && !S->W) return PD_EINVAL;
    const long n = p->nb * p->dim;
    if (S->step == 0) {
        const void* wgt = (p->kern.weight == PD_WEIGHT_INTEGRITY) ? (const void*)S->lambda
                          : (p->kern.weight == PD_WEIGHT_SCALE) ? (const void*)S->s : nullptr;
        T* Wp = (p->kern.weight == PD_WEIGHT_INTEGRITY && S->W) ? reinterpret_cast<T*>(S->W) : nullptr;
        PD_TRY(force_impl_any<T>(p, reinterpret_cast<const T*>(S->u), wgt, reinterpret_cast<T*>(S->F), Wp, st));
        if (b) {
            hipLaunchKernelGGL(k_add<T>, dim3(ew_blocks(n)), dim3(EW_THREADS), 0, st, reinterpret_cast<T*>(S->F), b, n);
            HIP_TRY(hipGetLastError());
        }
    }
    // Non-finite flag of the velocity updates: slot kNanSlot of the pinned
    // host buffer, written by the epilogue through its mapped address (or a
    // device slot copied back), cleared here and read once, after the last
    // step of the call.
    double* flag = nullptr;
    if (nsteps > 0) {
        if (p->red_host_dev) {
            p->red_host[kNanSlot] = 0.0;
            flag = p->red_host_dev + kNanSlot;
        } else {
            flag = p->red + kNanSlot;
            hipLaunchKernelGGL(k_fill<double>, dim3(1), dim3(64), 0, st, flag, 1L, 0.0);
            HIP_TRY(hipGetLastError());
        }
    }
    // Between the steps of one call the half-step velocity
    // vh = v + dt/(2 rho) F is carried in v instead of (v, F): the position
    // update is u + dt vh and the velocity update vh' = vh + dt/rho F'
    // (the same Verlet step, Eq. 83-84, regrouped), so the inner steps read
    // and write no F; the first step reads (v, F) and the last writes them.
    // Steps with energy output, and calls with PD_STATE_EXACT_STEPS, keep
    // (v, F) throughout.
    const bool kdk = !energy && !(S->flags & PD_STATE_EXACT_STEPS);
    int drifted = 0;   // u already holds this step's updated positions
    for (int k = 0; k < nsteps; ++k) {
        const int vh_in = (kdk && k > 0) ? 1 : 0, vh_out = (kdk && k + 1 < nsteps) ? 1 : 0;
        int drift = 0;
        if (energy) {
            PD_TRY((verlet_one<T, true>(p, S, b, w, T(dt), flag, 0, 0, 0, &drift, st)));
            double r[4];
            PD_TRY(fetch_red(p, 4, st, r));
            const double dV = p->dV;
            energy[4 * k + 0] = r[0] * dV;
            energy[4 * k + 1] = r[1] * dV;
            energy[4 * k + 2] = r[2] * dV;
            energy[4 * k + 3] = (r[0] + r[1] + r[2]) * dV - dt * dt / (8.0 * p->kern.rho) * r[3] * dV;
            for (int q = 0; q < 4; ++q)
                if (!std::isfinite(energy[4 * k + q])) return PD_ENUMERIC;
        } else {
            PD_TRY((verlet_one<T, false>(p, S, b, w, T(dt), flag, vh_in, vh_out, drifted, &drift, st)));
        }
        drifted = drift;
        S->step += 1;
    }
    if (nsteps > 0) {
        if (!p->red_host_dev)
            HIP_TRY(hipMemcpyAsync(p->red_host + kNanSlot, flag, sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (p->red_host[kNanSlot] != 0.0) return PD_ENUMERIC;
    }
    return PD_OK;
}

// -------------------------------------------------------------- force
template <class T>
pd_status force_impl_any(pd_plan p, const T* u, const void* weight, T* L, T* W, hipStream_t st) {
    return force_impl<T>(p, u, weight, L, W, st);
}

// ------------------------------------------------------------- adjoint
template <class T>
pd_status adjoint_impl(pd_plan p, const T* u, const T* u2, const void* weight, const T* g, T* ubar, T* wbar,
                       T wscale, int accumulate, hipStream_t st) {
    if (!wbar) {
        if (!ubar) return PD_OK;
        if (p->kern.weight == PD_WEIGHT_NONE) return lin_apply<T, 0>(p, g, ubar, nullptr, st);
        return force_impl<T>(p, g, weight, ubar, nullptr, st);
    }
    if (p->kern.weight != PD_WEIGHT_SCALE || p->kern.model != PD_BB_LINEAR) return PD_EUNSUPPORTED;
    if (!weight) return PD_EINVAL;
    if (p->dim != 2) return PD_EUNSUPPORTED;
    auto go = [&](auto Dc) -> pd_status {
        constexpr int DD = decltype(Dc)::value;
        GenAdj<T, DD, WK_SCALE> gg{};
        gg.c = ctx<T>(p);
        gg.u = u; gg.u2 = u2; gg.g = g; gg.s = reinterpret_cast<const T*>(weight);
        FinAdj<T, DD, WK_SCALE> ff{};
        ff.c = ctx<T>(p);
        ff.u = u; ff.u2 = u2; ff.g = g; ff.s = reinterpret_cast<const T*>(weight);
        ff.ubar = ubar; ff.wbar = wbar; ff.wscale = wscale; ff.accumulate = accumulate;
        return run_chain<T>(p, gg, MulAdj<T, DD>{}, ff, st);
    };
    return go(std::integral_constant<int, 2>{});
}

template <class T>
pd_status verlet_adjoint_impl(pd_plan p, const T* un, const T* unp1, const T* s, T* ub, T* vb, T* sb, T* bb,
                              double dt, hipStream_t st) {
    if (!un || !unp1 || !ub || !vb) return PD_EINVAL;
    if (p->kern.weight == PD_WEIGHT_INTEGRITY) return PD_EUNSUPPORTED;
    if (p->kern.weight == PD_WEIGHT_SCALE && !s) return PD_EINVAL;
    const long n = p->nb * p->dim;
    // scratch: a, La, ut, Lut  (4 vector fields of T)
    T* a = reinterpret_cast<T*>(p->vtmp);
    T* La = a + n;            // vtmp and vtmp2 each hold two vector fields
    T* ut = reinterpret_cast<T*>(p->vtmp2);
    T* Lut = ut + n;
    const T rho = T(p->kern.rho), c1 = T(dt / (2.0 * p->kern.rho)), c2 = T(dt * dt / (2.0 * p->kern.rho));
    (void)rho;
    const void* wgt = (p->kern.weight == PD_WEIGHT_SCALE) ? (const void*)s : nullptr;
    hipLaunchKernelGGL(k_mask_copy<T>, dim3(ew_blocks(n)), dim3(EW_THREADS), 0, st, a, (const T*)vb, p->chiO, n);
    HIP_TRY(hipGetLastError());
    PD_TRY(adjoint_impl<T>(p, un, unp1, wgt, a, La, sb, c1, 1, st));
    hipLaunchKernelGGL(k_vva_ut<T>, dim3(ew_blocks(n)), dim3(EW_THREADS), 0, st, ut, (const T*)ub, (const T*)La, c1,
                       p->chiO, n);
    HIP_TRY(hipGetLastError());
    PD_TRY(adjoint_impl<T>(p, un, nullptr, wgt, ut, Lut, sb, c2, 1, st));
    hipLaunchKernelGGL(k_vva_final<T>, dim3(ew_blocks(n)), dim3(EW_THREADS), 0, st, ub, vb, bb, (const T*)a,
                       (const T*)ut, (const T*)La, (const T*)Lut, c1, c2, T(dt), n);
    return pdh::check(hipGetLastError());
}

// --------------------------------------------------------- static solve
// The host reads the residual norm of each CG iteration one iteration late:
// the reduction writes the value to pinned host memory as well (or it is
// copied there behind the iteration's kernels) and the host waits for it
// only after the next iteration is queued, so the device never idles on a
// host round trip.  Slots 8 and 9 of red_host.
struct LagRead {
    hipEvent_t ev[2] = {nullptr, nullptr};   // the plan's events
    double* h = nullptr;
    double* hd = nullptr;   // device address of h (the reduction writes it), or null
    pd_status init(pd_plan p) {
        h = p->red_host + 8;
        hd = p->red_host_dev ? p->red_host_dev + 8 : nullptr;
        ev[0] = p->lag_ev[0];
        ev[1] = p->lag_ev[1];
        return (ev[0] && ev[1]) ? PD_OK : PD_EDEVICE;
    }
    // host slot of iteration k as the reduction kernel addresses it
    double* dslot(int k) const { return hd ? hd + (k & 1) : nullptr; }
    pd_status post(int k, const double* src, hipStream_t st) {
        if (!hd) HIP_TRY(hipMemcpyAsync(h + (k & 1), src, sizeof(double), hipMemcpyDeviceToHost, st));
        return pdh::check(hipEventRecord(ev[k & 1], st));
    }
    pd_status get(int k, double* v) {
        HIP_TRY(hipEventSynchronize(ev[k & 1]));
        *v = h[k & 1];
        return std::isfinite(*v) ? PD_OK : PD_ENUMERIC;
    }
};
// Device slots of red used by the solvers: [0] the operator's or the
// preconditioner's reduction, [2] |r|^2 of the last update, [6 + (k & 1)]
// rho of iteration k (r.r, or r.z when preconditioned).
constexpr int kRedRR = 2, kRedRho = 6;

// Drive a CG loop whose iterations are queued by issue(k): issue more while
// the lagged |r|^2 is above stop2, then confirm on the last iteration's value
// (CG residuals are not monotone, so the extra iteration queued behind the
// converged one is checked too) and continue if it is not converged.
template <class Issue>
pd_status cg_drive(LagRead& lag, double stop2, int maxit, int* issued_out, double* rr_out, Issue&& issue) {
    int issued = 0;
    double rr = *rr_out;
    while (rr > stop2 && issued < maxit) {
        bool hint = false;
        while (issued < maxit && !hint) {
            PD_TRY(issue(issued));
            ++issued;
            if (issued >= 2) {
                double v;
                PD_TRY(lag.get(issued - 2, &v));
                hint = v <= stop2;
            }
        }
        PD_TRY(lag.get(issued - 1, &rr));
    }
    *issued_out = issued;
    *rr_out = rr;
    return PD_OK;
}

// Plain CG in the plan precision on A = -chi_O L chi_O; x holds the full
// displacement (constrained components already = w).  Vectors r, pp, Ap of
// type T.  Returns the number of operator applications used.
template <class T, class TX>
pd_status cg_run(pd_plan p, TX* x_unused, T* xT, T* r, T* pp, T* Ap, double rr0, double stop2, int maxit, int* its,
                 int* applies, double* rr_out, hipStream_t st) {
    (void)x_unused;
    const long n = p->nb * p->dim;
    const unsigned nb = ew_blocks(n);
    double* dev = p->red;
    LagRead lag;
    PD_TRY(lag.init(p));
    HIP_TRY(hipMemcpyAsync(pp, r, sizeof(T) * n, hipMemcpyDeviceToDevice, st));
    p->red_host[kRedRho] = rr0;
    HIP_TRY(hipMemcpyAsync(dev + kRedRho, p->red_host + kRedRho, sizeof(double), hipMemcpyHostToDevice, st));
    auto issue = [&](int k) -> pd_status {
        double* rho = dev + kRedRho + (k & 1);
        double* rho_new = dev + kRedRho + ((k + 1) & 1);
        PD_TRY((lin_apply<T, 2>(p, pp, Ap, nullptr, st)));   // red[0] = p.Ap
        hipLaunchKernelGGL((k_cg_update<T, T>), dim3(nb), dim3(EW_THREADS), 0, st, xT, (const T*)pp, r, (const T*)Ap,
                           (const double*)rho, (const double*)dev, n, p->partials);
        PD_TRY(ew_finish<1>(p, nb, rho_new, st, lag.dslot(k)));
        PD_TRY(lag.post(k, rho_new, st));
        hipLaunchKernelGGL(k_cg_dir<T>, dim3(nb), dim3(EW_THREADS), 0, st, pp, (const T*)r, (const double*)rho_new,
                           (const double*)rho, (double*)nullptr, n);
        return pdh::check(hipGetLastError());
    };
    int it = 0;
    double rr = rr0;
    PD_TRY(cg_drive(lag, stop2, maxit, &it, &rr, issue));
    *its = it;
    *applies = it;
    *rr_out = rr;
    return PD_OK;
}

// Device memory a solve needs for its vectors (each one 256-byte aligned):
// r and t in FP64, then FP64 p and Ap (plain and preconditioned FP64), z
// (preconditioned FP64), or FP32 p, Ap and r (mixed) and z (mixed,
// preconditioned).
inline size_t solve_vec_bytes(long n, size_t elem) { return ((size_t)n * elem + 255) & ~(size_t)255; }
inline size_t solve_workspace_bytes(pd_plan p, int options) {
    const long n = p->nb * p->dim;
    const bool mixed = (options & PD_SOLVE_MIXED) != 0, pre = (options & PD_SOLVE_PRECOND) != 0;
    size_t tot = 2 * solve_vec_bytes(n, 8);
    if (!mixed) tot += (pre ? 3 : 2) * solve_vec_bytes(n, 8);
    else tot += (pre ? 4 : 3) * solve_vec_bytes(n, 4);
    return tot;
}

// The solve's vectors come from hipMalloc (freed before return) or, when ws
// is non-null, from the ws_bytes of device memory at ws (nothing is
// allocated; the caller guarantees ws_bytes >= solve_workspace_bytes).
inline pd_status static_solve_impl(pd_plan p, const double* b, const double* w, double* u, double rtol, int maxit,
                                   int options, pd_solve_info* info, hipStream_t st, void* ws = nullptr,
                                   size_t ws_bytes = 0) {
    const bool mixed = (options & PD_SOLVE_MIXED) != 0, pre = (options & PD_SOLVE_PRECOND) != 0;
    if (options & ~(PD_SOLVE_MIXED | PD_SOLVE_PRECOND)) return PD_EINVAL;
    if (p->dtype != PD_F64) return PD_EINVAL;
    if (p->kern.weight != PD_WEIGHT_NONE) return PD_EUNSUPPORTED;
    if (!b || !u || !(rtol > 0) || maxit <= 0) return PD_EINVAL;
    if (mixed && !p->sub32) return PD_EINVAL;
    if (ws && ws_bytes < solve_workspace_bytes(p, options)) return PD_EINVAL;
    const long n = p->nb * p->dim;
    pd_solve_info inf{};
    double *r = nullptr, *pp = nullptr, *Ap = nullptr, *t = nullptr, *z = nullptr;
    float *p32 = nullptr, *Ap32 = nullptr, *z32 = nullptr, *r32 = nullptr;
    size_t ws_off = 0;
    auto cleanup = [&]() {
        if (ws) return;
        void* bufs[] = {r, pp, Ap, t, z, p32, Ap32, z32, r32};
        for (void* q : bufs)
            if (q) (void)hipFree(q);
    };
    auto fail = [&](pd_status s) { cleanup(); return s; };
    auto vec = [&](auto** q, size_t elem) -> pd_status {
        if (!ws) return pdh::check(hipMalloc(q, elem * n));
        *q = reinterpret_cast<std::remove_pointer_t<decltype(q)>>(static_cast<unsigned char*>(ws) + ws_off);
        ws_off += solve_vec_bytes(n, elem);
        return PD_OK;
    };
#define SOLVE_TRY(x)                       \
    do {                                   \
        pd_status s2_ = (x);               \
        if (s2_ != PD_OK) return fail(s2_); \
    } while (0)
    SOLVE_TRY(vec(&r, sizeof(double)));
    SOLVE_TRY(vec(&t, sizeof(double)));
    // x = chi_O u + (1 - chi_O) w ; t = (1 - chi_O) w
    hipLaunchKernelGGL(k_constrain<double>, dim3(ew_blocks(n)), dim3(EW_THREADS), 0, st, u, t, w, p->chiO, n);
    SOLVE_TRY(pdh::check(hipGetLastError()));
    // |rhs|^2 = |chi_O (L((1 - chi_O) w) + b)|^2
    SOLVE_TRY((lin_apply<double, 3>(p, t, r, b, st)));
    double v[3];
    SOLVE_TRY(fetch_red(p, 1, st, v));
    inf.applies_fp64 += 1;
    double bn2 = v[0] > 0 ? v[0] : 1.0;
    const double stop2 = rtol * rtol * bn2;
    // r = chi_O (L(x) + b)
    SOLVE_TRY((lin_apply<double, 3>(p, u, r, b, st)));
    SOLVE_TRY(fetch_red(p, 1, st, v));
    inf.applies_fp64 += 1;
    double rr = v[0];
    pd_status result = PD_OK;
    const unsigned nb = ew_blocks(n);
    if (!mixed && !pre) {
        SOLVE_TRY(vec(&pp, sizeof(double)));
        SOLVE_TRY(vec(&Ap, sizeof(double)));
        int its = 0, app = 0;
        double rr_end = rr;
        SOLVE_TRY((cg_run<double, double>(p, u, u, r, pp, Ap, rr, stop2, maxit, &its, &app, &rr_end, st)));
        inf.iters_fp64 = its;
        inf.applies_fp64 += app;
    } else if (!mixed) {
        // preconditioned CG in FP64
        SOLVE_TRY(vec(&pp, sizeof(double)));
        SOLVE_TRY(vec(&Ap, sizeof(double)));
        SOLVE_TRY(vec(&z, sizeof(double)));
        double* dev = p->red;
        int it = 0;
        if (rr > stop2) {
            LagRead lag;
            SOLVE_TRY(lag.init(p));
            SOLVE_TRY((precond_apply<double, double, double>(p, r, z, st)));   // red[0] = r.z
            inf.precond_applies += 1;
            SOLVE_TRY(pdh::check(hipMemcpyAsync(dev + kRedRho, dev, sizeof(double), hipMemcpyDeviceToDevice, st)));
            SOLVE_TRY(pdh::check(hipMemcpyAsync(pp, z, sizeof(double) * n, hipMemcpyDeviceToDevice, st)));
            auto issue = [&](int k) -> pd_status {
                double* rho = dev + kRedRho + (k & 1);
                double* rho_new = dev + kRedRho + ((k + 1) & 1);
                PD_TRY((lin_apply<double, 2>(p, pp, Ap, nullptr, st)));   // red[0] = p.Ap
                hipLaunchKernelGGL((k_cg_update<double, double>), dim3(nb), dim3(EW_THREADS), 0, st, u,
                                   (const double*)pp, r, (const double*)Ap, (const double*)rho, (const double*)dev, n,
                                   p->partials);
                PD_TRY(ew_finish<1>(p, nb, dev + kRedRR, st, lag.dslot(k)));
                PD_TRY(lag.post(k, dev + kRedRR, st));
                PD_TRY((precond_apply<double, double, double>(p, r, z, st)));   // red[0] = r.z
                hipLaunchKernelGGL(k_pcg_dir<double>, dim3(nb), dim3(EW_THREADS), 0, st, pp, (const double*)z,
                                   (const double*)dev, (const double*)rho, rho_new, n);
                return pdh::check(hipGetLastError());
            };
            SOLVE_TRY(cg_drive(lag, stop2, maxit, &it, &rr, issue));
            inf.applies_fp64 += it;
            inf.precond_applies += it;
        }
        inf.iters_fp64 = it;
    } else {
        // CG with the operator (and the preconditioner, if any) applied in
        // FP32 (sub32 plan), with the iterate updated and every inner
        // product accumulated in FP64, and the direction and the recursively
        // updated residual kept in FP32 (the precision the operator reads
        // the direction in; each residual update is formed in FP64).  The
        // residual is replaced by the FP64 residual chi_O (L x + b) whenever
        // it has dropped by a factor 10 since the last replacement and at
        // the end (residual replacement keeps the FP32 operator's errors and
        // the residual's rounding from accumulating), so the returned
        // iterate meets rtol in FP64.  The host sees |r|^2 one iteration
        // late, so a replacement follows the iteration queued behind the one
        // that triggered it.
        pd_plan q = p->sub32;
        SOLVE_TRY(vec(&p32, sizeof(float)));
        SOLVE_TRY(vec(&Ap32, sizeof(float)));
        SOLVE_TRY(vec(&r32, sizeof(float)));
        if (pre) SOLVE_TRY(vec(&z32, sizeof(float)));
        double* dev = q->red;
        LagRead lag;
        SOLVE_TRY(lag.init(q));
        hipLaunchKernelGGL(k_to32, dim3(nb), dim3(EW_THREADS), 0, st, r32, (const double*)r, n);
        // rho = r.z (preconditioned) or r.r; the direction starts from z or r
        if (pre) {
            if (rr > stop2) {
                SOLVE_TRY((precond_apply<float, float, float>(q, r32, z32, st)));   // q->red[0] = r.z
                inf.precond_applies += 1;
                SOLVE_TRY(pdh::check(hipMemcpyAsync(dev + kRedRho, dev, sizeof(double), hipMemcpyDeviceToDevice, st)));
            }
            SOLVE_TRY(pdh::check(hipMemcpyAsync(p32, z32, sizeof(float) * n, hipMemcpyDeviceToDevice, st)));
        } else {
            q->red_host[kRedRho] = rr;
            SOLVE_TRY(pdh::check(hipMemcpyAsync(dev + kRedRho, q->red_host + kRedRho, sizeof(double),
                                                hipMemcpyHostToDevice, st)));
            hipLaunchKernelGGL(k_cgm_start, dim3(nb), dim3(EW_THREADS), 0, st, p32, (const double*)r, n);
        }
        SOLVE_TRY(pdh::check(hipGetLastError()));
        auto issue = [&](int k) -> pd_status {
            double* rho = dev + kRedRho + (k & 1);
            double* rho_new = dev + kRedRho + ((k + 1) & 1);
            PD_TRY((lin_apply<float, 2>(q, p32, Ap32, nullptr, st)));   // q->red[0] = p32 . Ap32
            hipLaunchKernelGGL(k_cgm_update, dim3(nb), dim3(EW_THREADS), 0, st, u, (const float*)p32, r32,
                               (const float*)Ap32, (const double*)rho, (const double*)dev, n, q->partials);
            PD_TRY(ew_finish<1>(q, nb, dev + kRedRR, st, lag.dslot(k)));
            PD_TRY(lag.post(k, dev + kRedRR, st));
            if (pre) {
                PD_TRY((precond_apply<float, float, float>(q, r32, z32, st)));   // q->red[0] = r.z
                hipLaunchKernelGGL(k_pcgm_dir, dim3(nb), dim3(EW_THREADS), 0, st, p32, (const float*)z32,
                                   (const double*)dev, (const double*)rho, rho_new, n);
            } else {
                hipLaunchKernelGGL(k_cgm_dir, dim3(nb), dim3(EW_THREADS), 0, st, p32, (const float*)r32,
                                   (const double*)(dev + kRedRR), (const double*)rho, rho_new, n);
            }
            return pdh::check(hipGetLastError());
        };
        double rr_rep = rr;   // |r|^2 at the last replacement
        int it = 0, fresh = 0;  // iterations from `fresh` on follow the last replacement
        while (rr > stop2 && it < maxit) {
            SOLVE_TRY(issue(it));
            ++it;
            inf.iters_fp32 += 1;
            inf.applies_fp32 += 1;
            if (pre) inf.precond_applies += 1;
            if (it - 2 < fresh) continue;
            double rr_lag;
            SOLVE_TRY(lag.get(it - 2, &rr_lag));
            if (rr_lag <= stop2 || rr_lag <= 1e-2 * rr_rep) {
                // residual replacement in FP64, after the queued iteration
                SOLVE_TRY((lin_apply<double, 3>(p, u, r, b, st)));
                hipLaunchKernelGGL(k_to32, dim3(nb), dim3(EW_THREADS), 0, st, r32, (const double*)r, n);
                SOLVE_TRY(fetch_red(p, 1, st, v));
                inf.applies_fp64 += 1;
                inf.iters_fp64 += 1;
                if (!std::isfinite(v[0])) return fail(PD_ENUMERIC);
                rr = rr_rep = v[0];
                fresh = it;
                if (!pre) {
                    // the next alpha uses |r|^2 of the replaced residual
                    const int sl = kRedRho + (it & 1);
                    q->red_host[sl] = rr;
                    SOLVE_TRY(pdh::check(hipMemcpyAsync(dev + sl, q->red_host + sl, sizeof(double),
                                                        hipMemcpyHostToDevice, st)));
                }
            }
        }
    }
    // true FP64 residual of the returned iterate
    SOLVE_TRY((lin_apply<double, 3>(p, u, r, b, st)));
    SOLVE_TRY(fetch_red(p, 1, st, v));
    inf.applies_fp64 += 1;
    inf.rel_res = std::sqrt(v[0] / bn2);
    if (!(inf.rel_res <= rtol)) result = std::isfinite(inf.rel_res) ? PD_ENOTCONV : PD_ENUMERIC;
    if (info) *info = inf;
    cleanup();
#undef SOLVE_TRY
    return result;
}

// ---------------------------------------------------------- damage index
template <class T>
pd_status damage_impl(pd_plan p, const uint8_t* lam, T* d, hipStream_t st) {
    if (p->kern.model != PD_BB_LINEAR || p->kern.weight != PD_WEIGHT_INTEGRITY) return PD_EUNSUPPORTED;
    if (!lam || !d) return PD_EINVAL;
    auto go = [&](auto Dc) -> pd_status {
        constexpr int DD = decltype(Dc)::value;
        GenPhi<T> gg{};
        gg.c = ctx<T>(p);
        gg.lam = lam;
        FinCount<T> ff{};
        ff.c = ctx<T>(p);
        ff.beta_comp = p->beta_comp;
        ff.lam = lam;
        ff.d = d;
        return run_chain<T>(p, gg, MulCount<T, DD>{}, ff, st);
    };
    if (p->dim != 2) return PD_EUNSUPPORTED;
    return go(std::integral_constant<int, 2>{});
}

// ------------------------------------------------------------ test chain
// Correlation with the separable kernel K(o) = prod_d k_d(o_d), k_d(o) =
// [o = s_d] + (-1)^{p_d} [o = -s_d] (s_d > 0) or [o = 0] (s_d = 0).
template <class T>
pd_status test_conv_impl(pd_plan p, const T* x, const int* sh, int parity, T* out, hipStream_t st) {
    const int D = p->dim;
    std::vector<int> offs;
    std::vector<double> kv;
    int P = 0;
    for (int d = 0; d < D; ++d) {
        if (sh[d] < 0) return PD_EINVAL;
        if (((parity >> d) & 1) && sh[d] == 0) return PD_EINVAL;
        P += (parity >> d) & 1;
    }
    int cnt[3] = {1, 1, 1};
    for (int d = 0; d < D; ++d) cnt[d] = sh[d] ? 2 : 1;
    for (int a = 0; a < cnt[0]; ++a)
        for (int bq = 0; bq < cnt[1]; ++bq)
            for (int c = 0; c < cnt[2]; ++c) {
                int sg[3] = {a ? -1 : 1, bq ? -1 : 1, c ? -1 : 1};
                double val = 1.0;
                for (int d = 0; d < D; ++d)
                    if (((parity >> d) & 1) && sg[d] < 0) val = -val;
                offs.push_back(sg[0] * sh[0]);
                offs.push_back(sg[1] * sh[1]);
                offs.push_back(D == 3 ? sg[2] * sh[2] : 0);
                kv.push_back(val);
            }
    const int ns = (int)kv.size();
    const int ntap = sh[D - 1] + 1;
    if (ntap > 9) return PD_EUNSUPPORTED;
    uint8_t par[3] = {(uint8_t)(parity & 1), (uint8_t)((parity >> 1) & 1), (uint8_t)((parity >> 2) & 1)};
    const Geo& g = p->geo;
    const long NP = (D == 2) ? (long)g.h1 : (long)g.h1 * g.n2;
    int* od = nullptr;
    double* kd = nullptr;
    uint8_t* pd = nullptr;
    T* taps = nullptr;
    pd_status s = PD_OK;
    s = pdh::check(hipMalloc(&od, sizeof(int) * offs.size()));
    if (s == PD_OK) s = pdh::check(hipMalloc(&kd, sizeof(double) * kv.size()));
    if (s == PD_OK) s = pdh::check(hipMalloc(&pd, 3));
    if (s == PD_OK) s = pdh::check(hipMalloc(&taps, sizeof(T) * NP * ntap));
    if (s == PD_OK) {
        (void)hipMemcpyAsync(od, offs.data(), sizeof(int) * offs.size(), hipMemcpyHostToDevice, st);
        (void)hipMemcpyAsync(kd, kv.data(), sizeof(double) * kv.size(), hipMemcpyHostToDevice, st);
        (void)hipMemcpyAsync(pd, par, 3, hipMemcpyHostToDevice, st);
        long nn = NP * ntap;
        hipLaunchKernelGGL((k_taps<T>), dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, D, g.n1, g.n2, g.h1, NP, ntap,
                           ns, od, kd, 1, 1, pd, p->tw64, g.twn1, 1.0 / (double)p->nfft, 2.0 / (double)p->nfft, taps);
        s = pdh::check(hipGetLastError());
    }
    if (s == PD_OK) {
        GenScalar<T> gg{};
        gg.x = x;
        MulTest<T> mm{};
        mm.P = P;
        FinScalar<T> ff{};
        ff.out = out;
        s = run_chain<T>(p, gg, mm, ff, st, 0, 0, taps, ntap, 1, (uint32_t)par[D - 1]);
    }
    (void)hipStreamSynchronize(st);
    if (od) (void)hipFree(od);
    if (kd) (void)hipFree(kd);
    if (pd) (void)hipFree(pd);
    if (taps) (void)hipFree(taps);
    return s;
}

inline hipStream_t S_(void* s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace pdi

// ===================================================================== C ABI

// The per-dtype implementation is instantiated once, in pd_inst.hip (each
// unit defines its share after these declarations); every other use only
// refers to it, so no unit compiles what another one holds.
namespace pdi {
#define PD_EXTERN(T)                                                                                               \
    extern template pd_status plan_alloc<T>(pd_plan, hipStream_t, const uint8_t*, const uint8_t*);                \
    extern template pd_status build_device_tables<T>(pd_plan, const std::vector<Bond>&, hipStream_t);             \
    extern template pd_status force_impl<T>(pd_plan, const T*, const void*, T*, T*, hipStream_t);                 \
    extern template pd_status adjoint_impl<T>(pd_plan, const T*, const T*, const void*, const T*, T*, T*, T, int, \
                                              hipStream_t);                                                       \
    extern template pd_status damage_impl<T>(pd_plan, const uint8_t*, T*, hipStream_t);                           \
    extern template pd_status test_conv_impl<T>(pd_plan, const T*, const int*, int, T*, hipStream_t);             \
    extern template pd_status verlet_impl<T>(pd_plan, pd_state*, const T*, const T*, double, int, double*,        \
                                             hipStream_t);                                                        \
    extern template pd_status verlet_adjoint_impl<T>(pd_plan, const T*, const T*, const T*, T*, T*, T*, T*,       \
                                                     double, hipStream_t);                                        \
    extern template pd_status cg_run<T, T>(pd_plan, T*, T*, T*, T*, T*, double, double, int, int*, int*, double*, \
                                           hipStream_t);                                                          \
    extern template pd_status lin_apply<T, 3>(pd_plan, const T*, T*, const T*, hipStream_t);                      \
    extern template pd_status lin_apply<T, 2>(pd_plan, const T*, T*, const T*, hipStream_t);                      \
    extern template pd_status precond_apply<T, double, T>(pd_plan, const double*, T*, hipStream_t);
PD_EXTERN(float)
extern template pd_status precond_apply<float, float, float>(pd_plan, const float*, float*, hipStream_t);
PD_EXTERN(double)
#undef PD_EXTERN
}  // namespace pdi
