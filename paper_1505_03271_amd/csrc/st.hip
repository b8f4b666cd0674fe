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
#include "lb_kernels.h"

namespace lbk {

template <class R, class S, bool TH, bool RAW>
__global__ void __launch_bounds__(256) st_step(StArgs A) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= A.nx) return;
    const int64_t plane = A.plane;
    const int64_t cell = int64_t(j) * A.nx + i;
    const S* src = static_cast<const S*>(A.src);
    S* dst = static_cast<S*>(A.dst);

    // destination slot of each population
    int64_t slot[9];
    int yhit[9], drow[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        int ti = i + cx(a), tj = j + cy(a);
        bool hit = false;
        yhit[a] = 0;
        if (tj < 0 || tj >= A.ny) {
            if (A.wall_y) { hit = true; yhit[a] = tj < 0 ? -1 : 1; } else tj = tj < 0 ? tj + A.ny : tj - A.ny;
        }
        if (ti < 0 || ti >= A.nx) {
            if (A.wall_x) hit = true; else ti = ti < 0 ? ti + A.nx : ti - A.nx;
        }
        slot[a] = hit ? int64_t(opp(a)) * plane + cell : int64_t(a) * plane + int64_t(tj) * A.nx + ti;
        drow[a] = hit ? j : tj;
    }

    if (RAW) {
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            dst[slot[a]] = src[int64_t(a) * plane + cell];
            if (TH) dst[9 * plane + slot[a]] = src[9 * plane + int64_t(a) * plane + cell];
        }
        return;
    }

    // g is stored relative to the row's thermal reference when one is kept
    const R rf = R(A.ref_f), rg = A.tref ? R(A.tref[j]) : R(A.ref_g);
    R f[9], g[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        R x = Codec<S>::template load<R>(src + a * plane + cell);
        f[a] = Codec<S>::offset ? x + wt<R>(a) * rf : x;
        if (TH) {
            R y = Codec<S>::template load<R>(src + (9 + a) * plane + cell);
            g[a] = Codec<S>::offset ? y + wt<R>(a) * rg : y;
        }
    }
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
    const R Tb = R(A.T_bottom), Tt = R(A.T_top);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const R wr = wt<R>(a) * m.rho;
        R fp = f[a] + kc * (wr * e.poly[a] - f[a]) + kf * wr * e.frc[a];
        R x = Codec<S>::offset ? fp - wt<R>(a) * rf : fp;
        Codec<S>::template store<R>(dst + slot[a], x);
        if (TH) {
            R gp = g[a] + kcg * (wt<R>(a) * m.T * e.poly[a] - g[a]);
            if (yhit[a] != 0) gp = R(2) * wt<R>(a) * (yhit[a] < 0 ? Tb : Tt) - gp;
            const R rgd = A.tref ? R(A.tref[drow[a]]) : rg;
            R y = Codec<S>::offset ? gp - wt<R>(a) * rgd : gp;
            Codec<S>::template store<R>(dst + 9 * plane + slot[a], y);
        }
    }
}

template <class R, class S>
static hipError_t st_typed(bool thermal, bool raw, const StArgs& a, hipStream_t s) {
    dim3 grid((a.nx + 255) / 256, a.ny), block(256);
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
