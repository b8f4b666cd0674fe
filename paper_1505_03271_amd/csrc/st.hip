// Streaming lattice Boltzmann step (arXiv:1505.03271 sec. 2.1, eq:ST) with
// dt = dx = 1.  Push form: each thread reads the populations of its own cell
// once (coalesced), collides them,
//   f' = f~ + (f_eq - f~)/tau~ + (1 - 1/(2 tau~)) F,   g' = g~ + (g_eq - g~)/tau~_g,
// and writes f'_a to the neighbour x + c_a.  A population whose neighbour
// lies beyond a wall returns to its own cell in the opposite direction
// (half-way bounce-back; the wall sits on the cell face as in the FV
// scheme); on the isothermal y walls g returns as 2 w_a T_w - g'_a
// (anti-bounce-back).  Every destination slot is written exactly once, so
// the step is a permutation of the collided values.  With RAW the collision
// is skipped and the stored words are moved unchanged.
#include <type_traits>

#include "lb_kernels.h"

namespace lbk {

// destination slot of population a of the cell (i, j): the neighbour's slot,
// or the opposite slot of the cell itself beyond a wall; yhit = -1 / +1 for a
// bottom / top wall hit (the thermal anti-bounce-back), drow the row written
struct StDest {
    int64_t slot;
    int yhit, drow;
};
__device__ inline StDest st_dest(const StArgs& A, const int i, const int j, const int a) {
    int ti = i + cx(a), tj = j + cy(a);
    bool hit = false;
    StDest d;
    d.yhit = 0;
    if (tj < 0 || tj >= A.ny) {
        if (A.wall_y) { hit = true; d.yhit = tj < 0 ? -1 : 1; } else tj = tj < 0 ? tj + A.ny : tj - A.ny;
    }
    if (ti < 0 || ti >= A.nx) {
        if (A.wall_x) hit = true; else ti = ti < 0 ? ti + A.nx : ti - A.nx;
    }
    const int64_t cell = int64_t(j) * A.nx + i;
    d.slot = hit ? int64_t(opp(a)) * A.plane + cell : int64_t(a) * A.plane + int64_t(tj) * A.nx + ti;
    d.drow = hit ? j : tj;
    return d;
}

// the collision of one cell from its decoded populations: f' and g' of
// every population before the wall rules and the storage offsets
template <class R, bool TH>
__device__ __forceinline__ void st_collide(const StArgs& A, const R* f, const R* g, R* fp, R* gp) {
    StageConst<R> k;
    k.hdt = R(0.5);
    k.ax = R(A.ax);
    k.ay = R(A.ay);
    k.bg = R(A.bg);
    k.T0 = R(A.T0);
    k.k1 = k.kh = k.k1g = 0;
    const R tt = R(A.tau + 0.5), ttg = R(A.tau_g + 0.5);
    const R kc = R(1) / tt, kf = R(1) - R(0.5) / tt, kcg = R(1) / ttg;
    Macro<R> m = macro<R, TH>(f, g, k);
    EqForce<R> e;
    eq_force(m, e);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const R wr = wt<R>(a) * m.rho;
        fp[a] = f[a] + kc * (wr * e.poly[a] - f[a]) + kf * wr * e.frc[a];
        if (TH) gp[a] = g[a] + kcg * (wt<R>(a) * m.T * e.poly[a] - g[a]);
    }
}

// the values stored for population a of a collided cell at its destination
template <class R, class S, bool TH>
__device__ inline R st_out_f(const StArgs& A, const int a, const R fp) {
    const R rf = R(A.ref_f);
    return Codec<S>::offset ? fp - wt<R>(a) * rf : fp;
}
template <class R, class S, bool TH>
__device__ inline R st_out_g(const StArgs& A, const int a, R gp, const StDest& d, const R rg) {
    if (d.yhit != 0) gp = R(2) * wt<R>(a) * (d.yhit < 0 ? R(A.T_bottom) : R(A.T_top)) - gp;
    const R rgd = A.tref ? R(A.tref[d.drow]) : rg;
    return Codec<S>::offset ? gp - wt<R>(a) * rgd : gp;
}

template <class R, class S, bool TH, bool RAW>
__global__ void __launch_bounds__(256) st_step(StArgs A) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= A.nx) return;
    const int64_t plane = A.plane;
    const int64_t cell = int64_t(j) * A.nx + i;
    const S* src = static_cast<const S*>(A.src);
    S* dst = static_cast<S*>(A.dst);

    StDest d[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) d[a] = st_dest(A, i, j, a);

    if (RAW) {
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            dst[d[a].slot] = src[int64_t(a) * plane + cell];
            if (TH) dst[9 * plane + d[a].slot] = src[9 * plane + int64_t(a) * plane + cell];
        }
        return;
    }

    // g is stored relative to the row's thermal reference when one is kept
    const R rf = R(A.ref_f), rg = A.tref ? R(A.tref[j]) : R(A.ref_g);
    R f[9], g[9], fp[9], gp[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        R x = Codec<S>::template load<R>(src + a * plane + cell);
        f[a] = Codec<S>::offset ? x + wt<R>(a) * rf : x;
        if (TH) {
            R y = Codec<S>::template load<R>(src + (9 + a) * plane + cell);
            g[a] = Codec<S>::offset ? y + wt<R>(a) * rg : y;
        }
    }
    st_collide<R, TH>(A, f, g, fp, gp);
    if (A.bad) raise_flag(A.bad, !__builtin_isfinite(TH ? fp[0] + gp[0] : fp[0]));
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        Codec<S>::template store<R>(dst + d[a].slot, st_out_f<R, S, TH>(A, a, fp[a]));
        if (TH) Codec<S>::template store<R>(dst + 9 * plane + d[a].slot, st_out_g<R, S, TH>(A, a, gp[a], d[a], rg));
    }
}

// 16-bit or FP32 storage on grids of even width: a thread takes two
// neighbouring cells of a row, reads each population of both as one word
// (32 or 64 bits) and writes the populations that stay in their column
// (c_x = 0: rest, up, down, and their wall bounce-backs) as one word too; the
// others move to different words and are written one by one.  The
// arithmetic of each cell is that of st_step.
template <class S> struct PairWord;
template <> struct PairWord<bf16_t> { using W = uint32_t; };
template <> struct PairWord<f16_t> { using W = uint32_t; };
template <> struct PairWord<float> { using W = uint64_t; };

template <class S> __device__ inline S pair_part(const typename PairWord<S>::W w, const int q) {
    if constexpr (sizeof(S) == 2) return S{uint16_t(w >> (16 * q))};
    else return __builtin_bit_cast(S, uint32_t(w >> (32 * q)));
}
template <class S> __device__ inline typename PairWord<S>::W pair_word(const S lo, const S hi) {
    using W = typename PairWord<S>::W;
    if constexpr (sizeof(S) == 2) return W(lo.bits) | (W(hi.bits) << 16);
    else return W(__builtin_bit_cast(uint32_t, lo)) | (W(__builtin_bit_cast(uint32_t, hi)) << 32);
}

template <class R, class S, bool TH>
__global__ void __launch_bounds__(256) st_step_pair(StArgs A) {
    using W = typename PairWord<S>::W;
    const int i0 = 2 * (blockIdx.x * 256 + threadIdx.x);
    const int j = blockIdx.y;
    if (i0 >= A.nx) return;
    const int64_t plane = A.plane;
    const int64_t cell = int64_t(j) * A.nx + i0;   // even: the pair is one aligned word
    const W* src = reinterpret_cast<const W*>(static_cast<const S*>(A.src));
    S* dst = static_cast<S*>(A.dst);
    W* dstw = reinterpret_cast<W*>(dst);
    const R rf = R(A.ref_f), rg = A.tref ? R(A.tref[j]) : R(A.ref_g);
    R f[2][9], g[2][9], fp[2][9], gp[2][9];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const W w = src[(int64_t(a) * plane + cell) >> 1];
        const W v = TH ? src[(int64_t(9 + a) * plane + cell) >> 1] : W(0);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const S x = pair_part<S>(w, q);
            const R xr = Codec<S>::template load<R>(&x);
            f[q][a] = xr + wt<R>(a) * rf;
            if (TH) {
                const S y = pair_part<S>(v, q);
                const R yr = Codec<S>::template load<R>(&y);
                g[q][a] = yr + wt<R>(a) * rg;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) st_collide<R, TH>(A, f[q], g[q], fp[q], gp[q]);
    if (A.bad) raise_flag(A.bad, !__builtin_isfinite(TH ? (fp[0][0] + gp[0][0]) + (fp[1][0] + gp[1][0])
                                                        : fp[0][0] + fp[1][0]));
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const StDest d0 = st_dest(A, i0, j, a), d1 = st_dest(A, i0 + 1, j, a);
        S of[2], og[2];
        Codec<S>::template store<R>(&of[0], st_out_f<R, S, TH>(A, a, fp[0][a]));
        Codec<S>::template store<R>(&of[1], st_out_f<R, S, TH>(A, a, fp[1][a]));
        if (TH) {
            Codec<S>::template store<R>(&og[0], st_out_g<R, S, TH>(A, a, gp[0][a], d0, rg));
            Codec<S>::template store<R>(&og[1], st_out_g<R, S, TH>(A, a, gp[1][a], d1, rg));
        }
        if (cx(a) == 0) {   // both land in one aligned word (d1.slot = d0.slot + 1)
            dstw[d0.slot >> 1] = pair_word<S>(of[0], of[1]);
            if (TH) dstw[(9 * plane + d0.slot) >> 1] = pair_word<S>(og[0], og[1]);
        } else {
            dst[d0.slot] = of[0];
            dst[d1.slot] = of[1];
            if (TH) {
                dst[9 * plane + d0.slot] = og[0];
                dst[9 * plane + d1.slot] = og[1];
            }
        }
    }
}

template <class R, class S>
static hipError_t st_typed(bool thermal, bool raw, const StArgs& a, hipStream_t s) {
    dim3 grid((a.nx + 255) / 256, a.ny), block(256);
    if constexpr (!std::is_same<S, double>::value) {
        if (!raw && a.pairs && a.nx % 2 == 0) {
            const dim3 gp((a.nx / 2 + 255) / 256, a.ny);
            if (thermal) hipLaunchKernelGGL((st_step_pair<R, S, true>), gp, block, 0, s, a);
            else hipLaunchKernelGGL((st_step_pair<R, S, false>), gp, block, 0, s, a);
            return hipGetLastError();
        }
    }
    if (thermal) {
        if (raw) hipLaunchKernelGGL((st_step<R, S, true, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((st_step<R, S, true, false>), grid, block, 0, s, a);
    } else {
        if (raw) hipLaunchKernelGGL((st_step<R, S, false, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((st_step<R, S, false, false>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_st(int storage, bool thermal, bool stream_only, const StArgs& a, hipStream_t s) {
    switch (storage) {
        case ST_F64: return st_typed<double, double>(thermal, stream_only, a, s);
        case ST_F32: return st_typed<float, float>(thermal, stream_only, a, s);
        case ST_BF16: return st_typed<float, bf16_t>(thermal, stream_only, a, s);
        case ST_F16: return st_typed<float, f16_t>(thermal, stream_only, a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace lbk
