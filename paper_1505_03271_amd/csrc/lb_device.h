// Device-side building blocks shared by the liblb kernels: the D2Q9 lattice,
// the storage codec for populations, and the local kinetic model (moments,
// equilibrium, Guo force) of arXiv:1505.03271 sec. 2.1, 2.2.4 and sec. 5.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace lbk {

// ---- D2Q9 lattice: index a has velocity (CX[a], CY[a]) ------------------
// The ordering is the one documented in include/lb.h.
__host__ __device__ constexpr int cx(int a) {
    return a == 1 || a == 5 || a == 8 ? 1 : (a == 3 || a == 6 || a == 7 ? -1 : 0);
}
__host__ __device__ constexpr int cy(int a) {
    return a == 2 || a == 5 || a == 6 ? 1 : (a == 4 || a == 7 || a == 8 ? -1 : 0);
}
// lattice weight by speed class: rest 4/9, axis 1/9, diagonal 1/36
template <class R>
__host__ __device__ constexpr R wt(int a) {
    return a == 0 ? R(4) / R(9) : (a <= 4 ? R(1) / R(9) : R(1) / R(36));
}
// population moving opposite to a
__host__ __device__ constexpr int opp(int a) {
    return a == 0 ? 0 : (a <= 4 ? (a + 1) % 4 + 1 : (a + 1) % 4 + 5);
}
static_assert(opp(1) == 3 && opp(2) == 4 && opp(3) == 1 && opp(4) == 2, "D2Q9 opposite (axes)");
static_assert(opp(5) == 7 && opp(6) == 8 && opp(7) == 5 && opp(8) == 6, "D2Q9 opposite (diagonals)");

// ---- storage codec -------------------------------------------------------
// F64 is stored as is.  F32/BF16/F16 store the offset p - w_a * ref, which
// removes the O(1) rest part so the narrow formats keep their precision for
// the deviation from the reference state.  Conversions round to nearest even.
struct bf16_t { uint16_t bits; };
struct f16_t { uint16_t bits; };

template <class S> struct Codec;

template <> struct Codec<double> {
    static constexpr bool offset = false;
    template <class R> __device__ static R load(const double* p) { return R(*p); }
    template <class R> __device__ static void store(double* p, R v) { *p = double(v); }
};

template <> struct Codec<float> {
    static constexpr bool offset = true;
    template <class R> __device__ static R load(const float* p) { return R(*p); }
    template <class R> __device__ static void store(float* p, R v) { *p = float(v); }
};

__device__ inline float bf16_bits_to_float(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }
__device__ inline uint16_t float_to_bf16_bits(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u)  // inf / nan: keep, quiet the nan
        return uint16_t((u >> 16) | ((u & 0x007fffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);       // round to nearest, ties to even
    return uint16_t(u >> 16);
}

template <> struct Codec<bf16_t> {
    static constexpr bool offset = true;
    template <class R> __device__ static R load(const bf16_t* p) { return R(bf16_bits_to_float(p->bits)); }
    // v_cvt_pk_bf16_f32: round to nearest even, as float_to_bf16_bits for finite values
    template <class R> __device__ static void store(bf16_t* p, R v) {
        p->bits = __builtin_bit_cast(uint16_t, (__bf16)float(v));
    }
};

template <> struct Codec<f16_t> {
    static constexpr bool offset = true;
    template <class R> __device__ static R load(const f16_t* p) {
        return R(__half2float(__ushort_as_half(p->bits)));
    }
    template <class R> __device__ static void store(f16_t* p, R v) {
        float x = float(v);
        asm("" : "+v"(x));   // round the FP32 value (no fused multiply-add-convert)
        p->bits = __half_as_ushort(__float2half_rn(x));
    }
};

// ---- moment-split storage ------------------------------------------------
// A cell keeps the conserved moments of its populations in FP32,
//   m = (rho - rho_ref, j_x, j_y, T - T_r),   j = sum c f~,
// and, in a 16-bit format, the residual r_a = f~_a - E_a(m) of each
// population from the forced equilibrium E = f_eq - dt/2 F (Guo) at the
// velocity u = j / rho + dt/2 a; for g, E = g_eq = w T (f_eq / (w rho)).  E
// carries the moments m exactly, so the residuals have zero mass and
// momentum: r0, r1 and r2 of f and r0 of g follow from the stored ones,
//   r1 = r3 - r5 + r6 + r7 - r8,  r2 = r4 - r5 - r6 + r7 + r8,  r0 = -sum r,
// and the 16-bit words never carry a conserved quantity.  Only the non-
// equilibrium part, which relaxes every step, is rounded to 16 bits; the
// slowly changing moments keep FP32 resolution, so increments far below a
// 16-bit ulp of the populations are not lost.  The 16-bit values hold
// r * RSCALE (2^10 for IEEE half, whose range is narrow; 1 for bfloat16).
template <class N> struct Split { uint16_t bits; };
using bf16s_t = Split<bf16_t>;
using f16s_t = Split<f16_t>;
template <class S> struct is_split { static constexpr bool value = false; };
template <class N> struct is_split<Split<N>> { static constexpr bool value = true; };
template <class S> struct split_scale { static constexpr float value = 1.0f; };
template <> struct split_scale<f16s_t> { static constexpr float value = 1024.0f; };

// Residual slot of (species s, population a), -1 when it is derived:
// slots 0..5 hold f r3..r8, slots 6..13 hold g r1..r8.
__host__ __device__ constexpr int split_slot(int s, int a) {
    return s == 0 ? (a >= 3 ? a - 3 : -1) : (a >= 1 ? 5 + a : -1);
}
// Byte layout of a split state with `cells` cells (each record is read by
// one lane with one 16- or 12-byte load):
//   thermal:      [float4 m per cell][8 residuals (16 B) per cell][6 residuals (12 B) per cell]
//   not thermal:  [float3 m per cell][6 residuals (12 B) per cell]
// Thermal residual slots 0..7 are in the first residual plane, 8..13 in the
// second; not thermal, slots 0..5 in the one plane.
struct SplitLayout {
    bool thermal;
    int64_t cells;
    __host__ __device__ int64_t bytes() const { return (thermal ? 44 : 24) * cells; }
    // byte offset of moment q (0..3; 0..2 when not thermal) of cell c
    __host__ __device__ int64_t mom(int q, int64_t c) const { return (thermal ? 16 : 12) * c + 4 * q; }
    // byte offset of residual slot k of cell c
    __host__ __device__ int64_t res(int k, int64_t c) const {
        if (!thermal) return 12 * cells + 12 * c + 2 * k;
        if (k < 8) return 16 * cells + 16 * c + 2 * k;
        return 32 * cells + 12 * c + 2 * (k - 8);
    }
};

// ---- population layouts in device memory ---------------------------------
// SoA (ST scheme): element (s, a, c) at (s*9 + a) * plane + c.
// Grouped (FV schemes): each cell keeps four populations of a species side by
// side so one lane reads them with one wide load:
//   group 2s   : a = 1..4 (axis velocities) of species s, 4 elements per cell
//   group 2s+1 : a = 5..8 (diagonals)
//   rest plane : a = 0 of every species, nsp elements per cell
// i.e. element (s, a>0, c) at (2s + (a>4)) * 4 plane + 4c + (a-1)%4 and
// (s, 0, c) at 8 nsp plane + nsp c + s.
__host__ __device__ inline int64_t pop_index(bool grouped, int nsp, int64_t plane, int s, int a, int64_t c) {
    if (!grouped) return (int64_t(s) * 9 + a) * plane + c;
    if (a == 0) return int64_t(8) * nsp * plane + int64_t(nsp) * c + s;
    return (int64_t(2 * s + (a > 4 ? 1 : 0)) * 4) * plane + 4 * c + ((a - 1) & 3);
}

// ---- local kinetic model -----------------------------------------------
// Constants of one semi-implicit stage (eq:semi) or of the Euler step
// (eq:euler), all precomputed on the host:
//   hdt   velocity shift: u = sum c f / rho + hdt a   (dt/2; 0 for Euler)
//   k1    relaxation in the advected bracket: dt/(2 tau~)      (0 for Euler)
//   kh    force in the advected bracket: dt/2                   (0 for Euler)
//   kc    collision: dt/tau~                                  (dt/tau for Euler)
//   kf    force in the update: dt (1 - dt/(2 tau~))            (dt for Euler)
//   k1g, kcg   the same two relaxation constants for g
template <class R>
struct StageConst {
    R hdt, k1, kh, kc, kf, k1g, kcg;
    R ax, ay, bg, T0;  // a = (ax, ay + bg (T - T0))
};

template <class R>
struct Macro {
    R rho, ux, uy, T, ax, ay;
};

template <class R, bool TH>
__device__ inline Macro<R> macro(const R* f, const R* g, const StageConst<R>& k) {
    Macro<R> m;
    R rho = 0, jx = 0, jy = 0;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        rho += f[a];
        if (cx(a) != 0) jx += R(cx(a)) * f[a];
        if (cy(a) != 0) jy += R(cy(a)) * f[a];
    }
    R T = 0;
    if (TH) {
#pragma unroll
        for (int a = 0; a < 9; ++a) T += g[a];
    }
    m.rho = rho;
    m.T = T;
    m.ax = k.ax;
    m.ay = TH ? k.ay + k.bg * (T - k.T0) : k.ay;
    R ir = R(1) / rho;
    m.ux = jx * ir + k.hdt * m.ax;
    m.uy = jy * ir + k.hdt * m.ay;
    return m;
}

// Equilibrium divided by w_a rho:  1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u
// Guo force divided by w_a rho (eq:F2):  3 (c - u).a + 9 (c.u)(c.a)
template <class R>
struct EqForce {
    R poly[9];
    R frc[9];
};

template <class R>
__device__ inline void eq_force(const Macro<R>& m, EqForce<R>& e) {
    const R uu = R(1.5) * (m.ux * m.ux + m.uy * m.uy);
    const R ua = m.ux * m.ax + m.uy * m.ay;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const R cu = R(cx(a)) * m.ux + R(cy(a)) * m.uy;
        const R ca = R(cx(a)) * m.ax + R(cy(a)) * m.ay;
        e.poly[a] = R(1) + R(3) * cu + R(4.5) * cu * cu - uu;
        e.frc[a] = R(3) * (ca - ua) + R(9) * cu * ca;
    }
}

// ---- non-finite flag -----------------------------------------------------
// A lane whose value is not finite raises the simulation's flag: one atomic
// per wave (its lowest such lane), through the vector memory path.  A
// blow-up makes every population of a cell non-finite within a step or two
// (each depends on the cell's density), so checking one value per species
// and cell suffices.
__device__ inline void raise_flag(int* flag, bool bad) {
    const uint64_t m = __builtin_amdgcn_ballot_w64(bad);
    if (m == 0 || !bad) return;
    const uint32_t below = __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
    if (below == 0) __hip_atomic_fetch_or(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace lbk
