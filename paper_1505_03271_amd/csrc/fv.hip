// Finite-volume lattice Boltzmann stage kernel (arXiv:1505.03271 sec. 2.2).
//
// Two launches make one semi-implicit + Heun step (eq:semi-heun):
//   predictor:  f~* = f~n - dt D(phi(f~n)) + C(f~n)            (eq:semi)
//   corrector:  f~n+1 = H + f~*/2 - dt/2 D(phi(f~*)),  H = (f~n + C(f~n)) / 2
// where the corrector reads f~n at its own cell and recomputes C(f~n).
// with, per population (sec. 2.2.2 and the force term of sec. 2.2.4),
//   phi = f~ + dt/(2 tau~)(f_eq - f~) + dt/2 F          (advected bracket)
//   C   = dt/tau~ (f_eq - f~) + dt (1 - dt/(2 tau~)) F   (collision + force)
//   D   = sum_faces (S/V) c.n [phi]_face                 (QUICK, sec. 2.2.3)
// The corrector is eq:semi-heun rearranged with f~* = f~n - dt Dn + Cn, so
// D(phi(f~n)) is never needed twice.  The single-pass schemes (eq:semi,
// eq:euler) use the predictor alone with their own constants.
//
// Offset arithmetic.  Populations are handled as offsets d = p - w_a ref
// (ref = rho_ref for f, the row's thermal reference Tr for g; ref = 0 for
// FP64 storage), exactly as they are stored.  Moments are rho = sum d + ref,
// j = sum c d, T = sum d_g + Tr.  The advected bracket is carried as
// phi - w_a ref, built from rho - ref and T - Tr so that no O(1) constant
// enters it: the four-point weights of a cell sum to zero, so a constant
// shift cancels from D, and leaving it out keeps the FP32 rounding of the
// weights (whose sum is zero only up to that rounding) from acting on it.
// Collision outputs are produced directly as offsets.
//
// Equilibrium and force are split by population pairs (a, inv(a)): with
// cu = c.u and ca = c.a,
//   f_eq / (w rho) = E +- O,   E = 1 + 9/2 cu^2 - 3/2 u.u,   O = 3 cu
//   F    / (w rho) = Fe +- Fo, Fe = 9 cu ca - 3 u.a,          Fo = 3 ca
// (Guo force, eq:F2, with cs^2 = 1/3).
//
// Flux.  For every cell the x (y) contribution of a population is a
// four-point stencil of phi along that axis; its weights combine the QUICK
// coefficients of the two faces, the sign of c, S/V = 1/dx and the update
// factor (dt, or dt/2 in the corrector) and are precomputed on the host:
//   c > 0:  nodes i-2 .. i+1,   c < 0:  nodes i-1 .. i+2.
//
// Mapping.  A work item of W lanes (FV_LANES, or 64 in narrow mode, four
// items to a block) owns a strip of up to W - 4 consecutive columns plus two
// halo columns on each side, one lane per column, and marches up a chunk of
// rows.  Each row is read once with
// coalesced buffer loads (x fastest in every population plane; one scalar
// offset per plane), the stage is evaluated once per cell, x neighbours come
// through LDS (double buffered, one barrier per row) and y neighbours from a
// ring of the last four rows kept in registers (the march is unrolled by four
// so the ring needs no moves).  y weights are uniform over the block (scalar
// loads); x weights are per lane and stay in registers.
//
// Boundaries ("Boundary conditions" of sec. 2.2): the bracket of a ghost cell
// is the mirror cell's with the opposite population (double reflection); for
// g on the y walls it is 2 w_a T_w - phi_inv(a) (isothermal anti-reflection).
// Periodic axes wrap.
#include <type_traits>

#include "lb_kernels.h"

namespace lbk {

// population pairs (a, inv(a)) with c_a = (PX, PY)
__device__ constexpr int pa(int p) { return p == 0 ? 1 : p == 1 ? 2 : p == 2 ? 5 : 6; }
__device__ constexpr int pb(int p) { return p == 0 ? 3 : p == 1 ? 4 : p == 2 ? 7 : 8; }
// populations with c_x != 0 (LDS slots) and with c_y = +1 / -1 (y ring)
__device__ constexpr int xpop(int p) { return p == 0 ? 1 : p == 1 ? 5 : p == 2 ? 8 : p == 3 ? 3 : p == 4 ? 6 : 7; }
__device__ constexpr int upop(int p) { return p == 0 ? 2 : p == 1 ? 5 : 6; }
__device__ constexpr int dpop(int p) { return p == 0 ? 4 : p == 1 ? 7 : 8; }

template <int N> struct Slot { static constexpr int value = N; };

// ---- raw buffer access: 32-bit lane offset, scalar per-plane offset ------
struct Buf {
    __amdgpu_buffer_rsrc_t r;
};
__device__ inline Buf make_buf(const void* p, uint32_t bytes) {
    // dword 3 for gfx9-family raw buffers: 32-bit data format, no swizzle
    return Buf{__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, int(bytes), 0x00020000)};
}

// Wide access to the grouped layout (pop_index): one group = the four
// populations a = 1..4 or a = 5..8 of a species at one cell, contiguous; the
// rest plane holds a = 0 of every species.  Loads return offsets in R.
typedef __attribute__((ext_vector_type(2))) unsigned u32x2;
typedef __attribute__((ext_vector_type(3))) unsigned u32x3;
typedef __attribute__((ext_vector_type(4))) unsigned u32x4;

__device__ inline double as_f64(unsigned lo, unsigned hi) {
    return __builtin_bit_cast(double, (uint64_t(hi) << 32) | uint64_t(lo));
}
__device__ inline unsigned f64_lo(double d) { return unsigned(__builtin_bit_cast(uint64_t, d)); }
__device__ inline unsigned f64_hi(double d) { return unsigned(__builtin_bit_cast(uint64_t, d) >> 32); }

// Stores wider than 64 bits take their whole byte offset in the VGPR operand
// and none in the SGPR one.  With an SGPR offset, a store of four dwords has
// been seen to take lanes 12..15 of every 16 of its first data register from
// the instruction after it, which overwrote that register (the compiler
// keeps a wait state between such a store and a write of its data only when
// the SGPR offset field is unused).  The extra VALU add per store is free.
__device__ inline void store_x4(Buf b, u32x4 x, uint32_t v, uint32_t s) {
    __builtin_amdgcn_raw_buffer_store_b128(x, b.r, v + s, 0u, 0);
}
__device__ inline void store_x3(Buf b, u32x3 x, uint32_t v, uint32_t s) {
    __builtin_amdgcn_raw_buffer_store_b96(x, b.r, v + s, 0u, 0);
}

template <class S> struct Io;
template <> struct Io<double> {
    template <class R> __device__ static void ld4(Buf b, uint32_t v, uint32_t s, R* d) {
        u32x4 x = __builtin_amdgcn_raw_buffer_load_b128(b.r, v, s, 0);
        u32x4 y = __builtin_amdgcn_raw_buffer_load_b128(b.r, v + 16, s, 0);
        d[0] = R(as_f64(x[0], x[1]));
        d[1] = R(as_f64(x[2], x[3]));
        d[2] = R(as_f64(y[0], y[1]));
        d[3] = R(as_f64(y[2], y[3]));
    }
    template <class R> __device__ static void st4(Buf b, uint32_t v, uint32_t s, const R* d) {
        const double a0 = d[0], a1 = d[1], a2 = d[2], a3 = d[3];
        store_x4(b, u32x4{f64_lo(a0), f64_hi(a0), f64_lo(a1), f64_hi(a1)}, v, s);
        store_x4(b, u32x4{f64_lo(a2), f64_hi(a2), f64_lo(a3), f64_hi(a3)}, v + 16, s);
    }
    template <class R, int N> __device__ static void ldr(Buf b, uint32_t v, uint32_t s, R* d) {
        if (N == 2) {
            u32x4 x = __builtin_amdgcn_raw_buffer_load_b128(b.r, v, s, 0);
            d[0] = R(as_f64(x[0], x[1]));
            d[1] = R(as_f64(x[2], x[3]));
        } else {
            u32x2 x = __builtin_amdgcn_raw_buffer_load_b64(b.r, v, s, 0);
            d[0] = R(as_f64(x[0], x[1]));
        }
    }
    template <class R, int N> __device__ static void str(Buf b, uint32_t v, uint32_t s, const R* d) {
        const double a0 = d[0];
        if (N == 2) {
            const double a1 = d[1];
            store_x4(b, u32x4{f64_lo(a0), f64_hi(a0), f64_lo(a1), f64_hi(a1)}, v, s);
        } else {
            __builtin_amdgcn_raw_buffer_store_b64(u32x2{f64_lo(a0), f64_hi(a0)}, b.r, v, s, 0);
        }
    }
};
template <> struct Io<float> {
    template <class R> __device__ static void ld4(Buf b, uint32_t v, uint32_t s, R* d) {
        u32x4 x = __builtin_amdgcn_raw_buffer_load_b128(b.r, v, s, 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) d[q] = R(__uint_as_float(x[q]));
    }
    template <class R> __device__ static void st4(Buf b, uint32_t v, uint32_t s, const R* d) {
        u32x4 x{__float_as_uint(float(d[0])), __float_as_uint(float(d[1])), __float_as_uint(float(d[2])),
                __float_as_uint(float(d[3]))};
        store_x4(b, x, v, s);
    }
    template <class R, int N> __device__ static void ldr(Buf b, uint32_t v, uint32_t s, R* d) {
        if (N == 2) {
            u32x2 x = __builtin_amdgcn_raw_buffer_load_b64(b.r, v, s, 0);
            d[0] = R(__uint_as_float(x[0]));
            d[1] = R(__uint_as_float(x[1]));
        } else {
            d[0] = R(__uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(b.r, v, s, 0)));
        }
    }
    template <class R, int N> __device__ static void str(Buf b, uint32_t v, uint32_t s, const R* d) {
        if (N == 2)
            __builtin_amdgcn_raw_buffer_store_b64(u32x2{__float_as_uint(float(d[0])), __float_as_uint(float(d[1]))},
                                                  b.r, v, s, 0);
        else
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(float(d[0])), b.r, v, s, 0);
    }
};
// 16-bit formats: two elements per dword, element k in bits 16 * (k % 2)
template <bool BF> struct Io16 {
    __device__ static float dec(uint32_t w, int hi) {
        const uint32_t h = hi ? (w >> 16) : (w & 0xffffu);
        if (BF) return __uint_as_float(h << 16);
        return float(__builtin_bit_cast(_Float16, uint16_t(h)));
    }
    __device__ static uint16_t enc(float x) {
        // x as an FP32 value: without this the compiler may fuse the
        // conversion with the multiply-add that produced x (v_fma_mixlo_f16,
        // one rounding from the exact result), so a value stored and the
        // same value rounded elsewhere could differ in the last bit
        asm("" : "+v"(x));
        if (BF) return __builtin_bit_cast(uint16_t, (__bf16)x);    // v_cvt_pk_bf16_f32: round to nearest even
        return __builtin_bit_cast(uint16_t, (_Float16)x);          // round to nearest even
    }
    // two values in one conversion instruction (round to nearest even)
    __device__ static uint32_t enc2(float lo, float hi) {
        typedef float f32x2 __attribute__((ext_vector_type(2)));
        typedef __bf16 b16x2 __attribute__((ext_vector_type(2)));
        typedef _Float16 h16x2 __attribute__((ext_vector_type(2)));
        asm("" : "+v"(lo), "+v"(hi));   // as in enc
        const f32x2 x{lo, hi};
        if (BF) return __builtin_bit_cast(uint32_t, __builtin_convertvector(x, b16x2));
        return __builtin_bit_cast(uint32_t, __builtin_convertvector(x, h16x2));
    }
    template <class R> __device__ static void ld4(Buf b, uint32_t v, uint32_t s, R* d) {
        u32x2 x = __builtin_amdgcn_raw_buffer_load_b64(b.r, v, s, 0);
        d[0] = R(dec(x[0], 0));
        d[1] = R(dec(x[0], 1));
        d[2] = R(dec(x[1], 0));
        d[3] = R(dec(x[1], 1));
    }
    template <class R> __device__ static void st4(Buf b, uint32_t v, uint32_t s, const R* d) {
        __builtin_amdgcn_raw_buffer_store_b64(u32x2{enc2(float(d[0]), float(d[1])), enc2(float(d[2]), float(d[3]))},
                                              b.r, v, s, 0);
    }
    template <class R, int N> __device__ static void ldr(Buf b, uint32_t v, uint32_t s, R* d) {
        if (N == 2) {
            uint32_t x = __builtin_amdgcn_raw_buffer_load_b32(b.r, v, s, 0);
            d[0] = R(dec(x, 0));
            d[1] = R(dec(x, 1));
        } else {
            d[0] = R(dec(__builtin_amdgcn_raw_buffer_load_b16(b.r, v, s, 0), 0));
        }
    }
    template <class R, int N> __device__ static void str(Buf b, uint32_t v, uint32_t s, const R* d) {
        if (N == 2) __builtin_amdgcn_raw_buffer_store_b32(enc2(float(d[0]), float(d[1])), b.r, v, s, 0);
        else __builtin_amdgcn_raw_buffer_store_b16(enc(float(d[0])), b.r, v, s, 0);
    }
};
template <> struct Io<bf16_t> : Io16<true> {};
template <> struct Io<f16_t> : Io16<false> {};

// All populations of one cell (offsets): f[0..8] and, if TH, g[0..8].
template <class R, class S, bool TH>
__device__ inline void load_cell(Buf b, uint32_t cell, uint32_t gbytes, uint32_t rest_off, R* f, R* g) {
    constexpr int NSP = TH ? 2 : 1;
    const uint32_t v4 = cell * uint32_t(4 * sizeof(S));
    Io<S>::template ld4<R>(b, v4, 0u, f + 1);
    Io<S>::template ld4<R>(b, v4, gbytes, f + 5);
    if (TH) {
        Io<S>::template ld4<R>(b, v4, 2 * gbytes, g + 1);
        Io<S>::template ld4<R>(b, v4, 3 * gbytes, g + 5);
    }
    R r0[2];
    Io<S>::template ldr<R, NSP>(b, cell * uint32_t(NSP * sizeof(S)), rest_off, r0);
    f[0] = r0[0];
    if (TH) g[0] = r0[NSP - 1];
}

template <class R, class S, bool TH>
__device__ inline void store_cell(Buf b, uint32_t cell, uint32_t gbytes, uint32_t rest_off, const R* f, const R* g) {
    constexpr int NSP = TH ? 2 : 1;
    const uint32_t v4 = cell * uint32_t(4 * sizeof(S));
    Io<S>::template st4<R>(b, v4, 0u, f + 1);
    Io<S>::template st4<R>(b, v4, gbytes, f + 5);
    if (TH) {
        Io<S>::template st4<R>(b, v4, 2 * gbytes, g + 1);
        Io<S>::template st4<R>(b, v4, 3 * gbytes, g + 5);
    }
    R r0[2] = {f[0], TH ? g[0] : R(0)};
    Io<S>::template str<R, NSP>(b, cell * uint32_t(NSP * sizeof(S)), rest_off, r0);
}

template <class R> __device__ inline R recip(R x) { return R(1) / x; }
template <> __device__ inline float recip<float>(float x) { return __builtin_amdgcn_rcpf(x); }

// One semi-implicit stage at a cell, in offset space.  Writes the advected
// brackets ph[s][a] (shifted by (1 - k1) w_a ref) of the moving populations
// and, when BASE, the offsets of f~ + C (all populations).  Tr is the
// thermal reference of the cell's row (g is stored as g - w_a Tr).
// stage_core takes the cell's macroscopic state (rho, T, u, a_y); stage
// computes it from the offsets.
template <class R, bool TH, bool BASE>
__device__ inline void stage_core(const R* df, const R* dg, const R rho_p, const R rho, const R T_p, const R T,
                                  const R ux, const R uy, const R ay, const StageK<R>& k, R (*ph)[9], R (*bs)[9]) {
    constexpr int NSP = TH ? 2 : 1;
    const R ax = k.ax;
    const R uu = R(1.5) * (ux * ux + uy * uy);
    const R ua3 = R(3) * (ux * ax + uy * ay);
    // rest population: no flux; base only
    if (BASE) {
        bs[0][0] = k.omkc * df[0] + wt<R>(0) * (k.kc * rho_p - rho * (k.kc * uu + k.kf * ua3));
        if (TH) bs[NSP - 1][0] = k.omkcg * dg[0] + k.kcg * wt<R>(0) * (T_p - T * uu);
    }
    // The weight w is common to a class of populations (axis 1/9, diagonal
    // 1/36), so it enters through per-class products: w rho, w k1 rho' (and
    // w kc rho'), and for g w k1g T, w k1g T' (and with kcg).
    const R k1r = k.k1 * rho_p, kcr = k.kc * rho_p;
    R wr[2], wk1[2], wkc[2], gT[2], gTp[2], cT[2], cTp[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const R w = wt<R>(c == 0 ? 1 : 5);
        wr[c] = w * rho;
        wk1[c] = w * k1r;
        wkc[c] = w * kcr;
        const R g1 = k.k1g * w, gc = k.kcg * w;
        gT[c] = g1 * T;
        gTp[c] = g1 * T_p;
        cT[c] = gc * T;
        cTp[c] = gc * T_p;
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int a = pa(p), b = pb(p);
        const int c = p < 2 ? 0 : 1;
        R cu, ca;
        if (p == 0) { cu = ux; ca = ax; }
        else if (p == 1) { cu = uy; ca = ay; }
        else if (p == 2) { cu = ux + uy; ca = ax + ay; }
        else { cu = uy - ux; ca = ay - ax; }
        const R Em = (R(4.5) * cu) * cu - uu;     // even part of f_eq / (w rho), minus 1
        const R Fe = (R(9) * cu) * ca - ua3;      // even part of F / (w rho)
        // advected bracket of f, minus w ref:
        //   w (k1 rho' + rho (k1 Em + kh Fe)) +- w rho (3 k1 cu + 3 kh ca)
        const R Pe = k.k1 * Em + k.kh * Fe;
        const R Po = k.k1x3 * cu + k.khx3 * ca;
        ph[0][a] = k.omk1 * df[a] + (wk1[c] + wr[c] * (Pe + Po));
        ph[0][b] = k.omk1 * df[b] + (wk1[c] + wr[c] * (Pe - Po));
        if (TH) {
            // bracket of g, minus w Tr: k1g w (T' + T Em +- 3 T cu)
            const R O = R(3) * cu;
            const R Ge = gTp[c] + gT[c] * Em, Go = gT[c] * O;
            ph[NSP - 1][a] = k.omk1g * dg[a] + (Ge + Go);
            ph[NSP - 1][b] = k.omk1g * dg[b] + (Ge - Go);
            if (BASE) {
                const R Ce = cTp[c] + cT[c] * Em, Co = cT[c] * O;
                bs[NSP - 1][a] = k.omkcg * dg[a] + (Ce + Co);
                bs[NSP - 1][b] = k.omkcg * dg[b] + (Ce - Co);
            }
        }
        if (BASE) {
            const R Ae = k.kc * Em + k.kf * Fe;
            const R Ao = k.kcx3 * cu + k.kfx3 * ca;
            bs[0][a] = k.omkc * df[a] + (wkc[c] + wr[c] * (Ae + Ao));
            bs[0][b] = k.omkc * df[b] + (wkc[c] + wr[c] * (Ae - Ao));
        }
    }
}

template <class R, bool TH, bool BASE>
__device__ inline void stage(const R* df, const R* dg, const StageK<R>& k, const R Tr, R (*ph)[9], R (*bs)[9]) {
    R rho_p = df[0], jx = 0, jy = 0;
#pragma unroll
    for (int a = 1; a < 9; ++a) {
        rho_p += df[a];
        if (cx(a) > 0) jx += df[a]; else if (cx(a) < 0) jx -= df[a];
        if (cy(a) > 0) jy += df[a]; else if (cy(a) < 0) jy -= df[a];
    }
    const R rho = rho_p + k.ref_f;
    R T_p = 0, T = 0, ay = k.ay;
    if (TH) {
        T_p = dg[0];
#pragma unroll
        for (int a = 1; a < 9; ++a) T_p += dg[a];
        T = T_p + Tr;
        ay = k.ay + k.bg * (T - k.T0);
    }
    const R ir = recip(rho);
    const R ux = jx * ir + k.hdt * k.ax, uy = jy * ir + k.hdt * ay;
    stage_core<R, TH, BASE>(df, dg, rho_p, rho, T_p, T, ux, uy, ay, k, ph, bs);
}

// ---- moment-split cells (storage BF16S / F16S) ---------------------------
// Layout (SplitLayout, with G = 8 bytes x cells = group_bytes): thermal
// cells keep m as a float4 at 16 c, residual slots 0..7 at 2G + 16 c and
// 8..13 at 4G + 12 c; other cells keep m as three floats at 12 c and the
// residuals at 1.5 G + 12 c.  One wide load per record and lane.
template <class S> struct Narrow;
template <> struct Narrow<bf16s_t> : Io16<true> {};
template <> struct Narrow<f16s_t> : Io16<false> {};

// A split record as loaded: the words stay packed (11 or 6 registers) until
// decode_split, which is placed where the values are used, so the wait for
// a load sits there and not at the load.
template <bool TH> struct SplitRaw {
    u32x4 m;  // moments (thermal: 4 words; otherwise words 0..2)
    u32x4 p;  // residual slots 0..7 (otherwise 0..5 in words 0..2)
    u32x3 t;  // residual slots 8..13 (thermal only)
};

template <class S, bool TH>
__device__ inline void load_split_raw(Buf b, uint32_t cell, uint32_t G, SplitRaw<TH>& w) {
    const uint32_t v12 = cell * 12u;
    if (TH) {
        const uint32_t v16 = cell * 16u;
        w.m = __builtin_amdgcn_raw_buffer_load_b128(b.r, v16, 0u, 0);
        w.p = __builtin_amdgcn_raw_buffer_load_b128(b.r, v16, 2 * G, 0);
        w.t = __builtin_amdgcn_raw_buffer_load_b96(b.r, v12, 4 * G, 0);
    } else {
        const u32x3 x = __builtin_amdgcn_raw_buffer_load_b96(b.r, v12, 0u, 0);
        const u32x3 p = __builtin_amdgcn_raw_buffer_load_b96(b.r, v12, G + G / 2, 0);
        w.m = u32x4{x[0], x[1], x[2], 0u};
        w.p = u32x4{p[0], p[1], p[2], 0u};
    }
}

template <class R, class S, bool TH>
__device__ inline void decode_split(const SplitRaw<TH>& w, R* m, R* rf, R* rg) {
    using IO = Narrow<S>;
    constexpr float irs = 1.0f / split_scale<S>::value;
    auto d = [&](uint32_t x, int hi) __attribute__((always_inline)) { return R(IO::dec(x, hi) * irs); };
#pragma unroll
    for (int q = 0; q < 3; ++q) m[q] = R(__uint_as_float(w.m[q]));
    m[3] = TH ? R(__uint_as_float(w.m[3])) : R(0);
    rf[3] = d(w.p[0], 0); rf[4] = d(w.p[0], 1); rf[5] = d(w.p[1], 0); rf[6] = d(w.p[1], 1);
    rf[7] = d(w.p[2], 0); rf[8] = d(w.p[2], 1);
    if (TH) {
        rg[1] = d(w.p[3], 0); rg[2] = d(w.p[3], 1);
        rg[3] = d(w.t[0], 0); rg[4] = d(w.t[0], 1); rg[5] = d(w.t[1], 0); rg[6] = d(w.t[1], 1);
        rg[7] = d(w.t[2], 0); rg[8] = d(w.t[2], 1);
    }
}

// Macroscopic state of a split cell from its moments.
template <class R, bool TH>
__device__ inline void split_macro(const R* m, const StageK<R>& k, const R Tr, R& rho, R& T, R& ux, R& uy, R& ay) {
    rho = m[0] + k.ref_f;
    T = TH ? m[3] + Tr : R(0);
    ay = TH ? k.ay + k.bg * (T - k.T0) : k.ay;
    const R ir = recip(rho);
    ux = m[1] * ir + k.hdt * k.ax;
    uy = m[2] * ir + k.hdt * ay;
}

// Offsets of the forced equilibrium, e_a = E_a - w_a ref: for f
// w (m0 + rho (P_a - 1 - hdt F_a / (w rho))), for g w (m3 + T (P_a - 1)),
// with P = f_eq / (w rho).  Small terms only, so FP32 keeps them exact to
// its own resolution.
template <class R, bool TH, class Fn>
__device__ inline void split_eq(const R* m, const R rho, const R T, const R ux, const R uy, const R ay,
                                const StageK<R>& k, const R q, Fn&& put) {
    const R uu = R(1.5) * (ux * ux + uy * uy);
    const R ua3 = R(3) * (ux * k.ax + uy * ay);
    put(0, 0, wt<R>(0) * (m[0] + rho * (k.hdt * ua3 - uu)));
    if (TH) put(1, 0, wt<R>(0) * (m[3] - T * uu));
    const R wr[2] = {wt<R>(1) * rho, wt<R>(5) * rho}, wp[2] = {wt<R>(1) * m[0], wt<R>(5) * m[0]};
    const R wT[2] = {wt<R>(1) * T, wt<R>(5) * T}, wTp[2] = {wt<R>(1) * m[3], wt<R>(5) * m[3]};
    const R wq[2] = {wt<R>(1) * q, wt<R>(5) * q};  // heat-flux reference w c_y q of a c_y = +1 population
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int a = pa(p), b = pb(p);
        R cu, ca;
        if (p == 0) { cu = ux; ca = k.ax; }
        else if (p == 1) { cu = uy; ca = ay; }
        else if (p == 2) { cu = ux + uy; ca = k.ax + ay; }
        else { cu = uy - ux; ca = ay - k.ax; }
        const R Em = (R(4.5) * cu) * cu - uu;
        const R O = R(3) * cu;
        const R Qe = Em - k.hdt * ((R(9) * cu) * ca - ua3);
        const R Qo = O - k.hdt * (R(3) * ca);
        const int c = p < 2 ? 0 : 1;
        put(0, a, wp[c] + wr[c] * (Qe + Qo));
        put(0, b, wp[c] + wr[c] * (Qe - Qo));
        if (TH) {
            // equilibrium plus the reference (+- wq for the pairs along y)
            const R A = wTp[c] + wT[c] * Em;
            const R B = p == 0 ? wT[c] * O : wT[c] * O + wq[c];
            put(1, a, A + B);
            put(1, b, A - B);
        }
    }
}

// The stage of a split cell, straight from its moments and residuals r
// (f~ = f_eq - dt/2 F + r, g = g_eq + r_g).  With P = f_eq / (w rho) =
// 1 + (E - 1) +- O per opposite pair and F / (w rho) = Fe +- Fo:
//   phi - w ref   = w (rho' + rho ((E-1 + cP Fe) +- (O + cP Fo))) + (1 - k1) r,  cP = kh - (1 - k1) dt/2
//   f~ + C - w ref = w (rho' + rho ((E-1 + cB Fe) +- (O + cB Fo))) + (1 - kc) r, cB = kf - (1 - kc) dt/2
//   f~ - w ref    = w (rho' + rho ((E-1 - dt/2 Fe) +- (O - dt/2 Fo))) + r
//   phi_g - w Tr  = w (T' + T (E-1 +- O)) + (1 - k1g) r_g,  and likewise with kcg, or r_g alone
// (rho' = rho - ref, T' = T - Tr).  The stored g residual of a population
// with velocity c is r_g - w c_y q, q the row's heat-flux reference.  On entry df, dg hold the stored
// residuals (f: a = 3..8, g: a = 1..8); the rest follow from zero mass and
// momentum.  With NEED_D they are replaced by the offsets d of all
// populations.
template <class R, bool TH, bool BASE, bool NEED_D>
__device__ inline void stage_split(const R* m, R* df, R* dg, const StageK<R>& k, const R Tr, const R q, R (*ph)[9],
                                   R (*bs)[9]) {
    constexpr int NSP = TH ? 2 : 1;
    df[1] = df[3] - df[5] + df[6] + df[7] - df[8];
    df[2] = df[4] - df[5] - df[6] + df[7] + df[8];
    df[0] = -(((df[1] + df[2]) + (df[3] + df[4])) + ((df[5] + df[6]) + (df[7] + df[8])));
    if (TH) dg[0] = -(((dg[1] + dg[2]) + (dg[3] + dg[4])) + ((dg[5] + dg[6]) + (dg[7] + dg[8])));
    R rho, T, ux, uy, ay;
    split_macro<R, TH>(m, k, Tr, rho, T, ux, uy, ay);
    const R uu = R(1.5) * (ux * ux + uy * uy);
    const R ua3 = R(3) * (ux * k.ax + uy * ay);
    const R rp = m[0], Tp = TH ? m[3] : R(0);
    constexpr R w0 = wt<R>(0);
    // w rho, w rho', w T, w T' of the axis (1/9) and diagonal (1/36) classes
    const R wr[2] = {wt<R>(1) * rho, wt<R>(5) * rho}, wp[2] = {wt<R>(1) * rp, wt<R>(5) * rp};
    const R wT[2] = {wt<R>(1) * T, wt<R>(5) * T}, wTp[2] = {wt<R>(1) * Tp, wt<R>(5) * Tp};
    const R wq[2] = {wt<R>(1) * q, wt<R>(5) * q};
    // rest population: no flux
    if (BASE) {
        bs[0][0] = w0 * (rp - rho * (uu + k.cB * ua3)) + k.omkc * df[0];
        if (TH) bs[NSP - 1][0] = w0 * (Tp - T * uu) + k.omkcg * dg[0];
    }
    if (NEED_D) {
        df[0] = w0 * (rp + rho * (k.hdt * ua3 - uu)) + df[0];
        if (TH) dg[0] = w0 * (Tp - T * uu) + dg[0];
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int a = pa(p), b = pb(p);
        const int c = p < 2 ? 0 : 1;
        R cu, ca;
        if (p == 0) { cu = ux; ca = k.ax; }
        else if (p == 1) { cu = uy; ca = ay; }
        else if (p == 2) { cu = ux + uy; ca = k.ax + ay; }
        else { cu = uy - ux; ca = ay - k.ax; }
        const R Em = (R(4.5) * cu) * cu - uu;
        const R O = R(3) * cu;
        const R Fe = (R(9) * cu) * ca - ua3;
        const R Fo = R(3) * ca;
        const R ra = df[a], rb = df[b];
        const R PE = Em + k.cP * Fe, PO = O + k.cP * Fo;
        ph[0][a] = (wp[c] + wr[c] * (PE + PO)) + k.omk1 * ra;
        ph[0][b] = (wp[c] + wr[c] * (PE - PO)) + k.omk1 * rb;
        // g: the residual is the stored one plus the reference +- wq (pairs
        // along y), which enters each formula through its odd part
        R GA = 0, GO = 0;
        if (TH) {
            GA = wTp[c] + wT[c] * Em;
            GO = wT[c] * O;
            const R B = p == 0 ? GO : GO + k.omk1g * wq[c];
            ph[NSP - 1][a] = (GA + B) + k.omk1g * dg[a];
            ph[NSP - 1][b] = (GA - B) + k.omk1g * dg[b];
        }
        if (BASE) {
            const R BE = Em + k.cB * Fe, BO = O + k.cB * Fo;
            bs[0][a] = (wp[c] + wr[c] * (BE + BO)) + k.omkc * ra;
            bs[0][b] = (wp[c] + wr[c] * (BE - BO)) + k.omkc * rb;
            if (TH) {
                const R B = p == 0 ? GO : GO + k.omkcg * wq[c];
                bs[NSP - 1][a] = (GA + B) + k.omkcg * dg[a];
                bs[NSP - 1][b] = (GA - B) + k.omkcg * dg[b];
            }
        }
        if (NEED_D) {
            const R QE = Em - k.hdt * Fe, QO = O - k.hdt * Fo;
            df[a] = (wp[c] + wr[c] * (QE + QO)) + ra;
            df[b] = (wp[c] + wr[c] * (QE - QO)) + rb;
            if (TH) {
                const R B = p == 0 ? GO : GO + wq[c];
                dg[a] = (GA + B) + dg[a];
                dg[b] = (GA - B) + dg[b];
            }
        }
    }
}

// Offsets d of a cell -> its split record: moments (FP32 words) and rounded
// residuals (16-bit words), as stored.  Returns m0 + m3, which is finite
// exactly when the moments are.
// X2: df, dg hold twice the offsets (exactly: every operation that formed
// them scales by two without rounding differently), halved here where it
// costs least, in the four moments and inside the residuals' subtraction.
template <class R, class S, bool TH, bool X2 = false>
__device__ inline R encode_split(const R* df, const R* dg, const StageK<R>& k, const R Tr, const R q,
                                 SplitRaw<TH>& w) {
    using IO = Narrow<S>;
    constexpr float rs = split_scale<S>::value;
    constexpr R hx = X2 ? R(0.5) : R(1);
    R m[4];
    m[0] = hx * (((df[0] + (df[1] + df[2])) + (df[3] + df[4])) + ((df[5] + df[6]) + (df[7] + df[8])));
    m[1] = hx * (((df[1] - df[3]) + (df[5] - df[6])) + (df[8] - df[7]));
    m[2] = hx * (((df[2] - df[4]) + (df[5] + df[6])) - (df[7] + df[8]));
    m[3] = TH ? hx * (((dg[0] + (dg[1] + dg[2])) + (dg[3] + dg[4])) + ((dg[5] + dg[6]) + (dg[7] + dg[8]))) : R(0);
    R rho, T, ux, uy, ay;
    split_macro<R, TH>(m, k, Tr, rho, T, ux, uy, ay);
    R rf[9], rg[9];
    split_eq<R, TH>(m, rho, T, ux, uy, ay, k, q, [&](int s, int a, R e) __attribute__((always_inline)) {
        if (s == 0) rf[a] = hx * df[a] - e; else rg[a] = hx * dg[a] - e;
    });
    auto e2 = [&](R lo, R hi) __attribute__((always_inline)) { return IO::enc2(float(lo) * rs, float(hi) * rs); };
    w.m = u32x4{__float_as_uint(float(m[0])), __float_as_uint(float(m[1])), __float_as_uint(float(m[2])),
                __float_as_uint(float(m[3]))};
    if (TH) {
        w.p = u32x4{e2(rf[3], rf[4]), e2(rf[5], rf[6]), e2(rf[7], rf[8]), e2(rg[1], rg[2])};
        w.t = u32x3{e2(rg[3], rg[4]), e2(rg[5], rg[6]), e2(rg[7], rg[8])};
    } else {
        w.p = u32x4{e2(rf[3], rf[4]), e2(rf[5], rf[6]), e2(rf[7], rf[8]), 0u};
        w.t = u32x3{0u, 0u, 0u};
    }
    return m[0] + m[3];
}

template <bool TH>
__device__ inline void store_split_raw(Buf b, uint32_t cell, uint32_t G, const SplitRaw<TH>& w) {
    const uint32_t v12 = cell * 12u;
    if (TH) {
        const uint32_t v16 = cell * 16u;
        store_x4(b, w.m, v16, 0u);
        store_x4(b, w.p, v16, 2 * G);
        store_x3(b, w.t, v12, 4 * G);
    } else {
        store_x3(b, u32x3{w.m[0], w.m[1], w.m[2]}, v12, 0u);
        store_x3(b, u32x3{w.p[0], w.p[1], w.p[2]}, v12, G + G / 2);
    }
}

// Offsets d of a cell -> moments (FP32) and rounded residuals, stored.
// Returns m0 + m3, which is finite exactly when the stored moments are.
template <class R, class S, bool TH, bool X2 = false>
__device__ inline R store_split(Buf b, uint32_t cell, uint32_t G, const R* df, const R* dg, const StageK<R>& k,
                                const R Tr, const R q) {
    SplitRaw<TH> w;
    const R chk = encode_split<R, S, TH, X2>(df, dg, k, Tr, q, w);
    store_split_raw<TH>(b, cell, G, w);
    return chk;
}

// Make this row's LDS writes visible to the other lanes of the item.  A
// 64-lane item (one wave) only needs the wave's own LDS operations kept in
// program order (the LDS executes a wave's instructions in order); a block-
// wide item needs a workgroup barrier.
template <int W> __device__ inline void lanes_sync() {
    if (W == 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// Work item of block b.  Blocks are dealt to the eight XCDs round robin, so
// block b runs on XCD b % 8; items are numbered chunk-major (adjacent strips
// of a chunk are consecutive) and each XCD takes a contiguous range of them,
// so strips that share halo columns run side by side on one XCD and meet in
// its L2.
__device__ inline int xcd_item(int b, int n_items) {
    const int per_xcd = (n_items + 7) / 8;
    return (b % 8) * per_xcd + b / 8;
}

// Roles of fv_item: a stage launch of its own (the predictor, a single-pass
// scheme, or the corrector), or one half of a fused step, which runs the
// predictor and the corrector of one Heun step side by side in one block
// (see fv_fused).
enum { FV_ALONE = 0, FV_FIRST = 1, FV_SECOND = 2 };
// LDS rings of the fused step: rows of f~* (FP32 offsets) handed from the
// first half to the second one step after they are formed, and rows of the
// collision base f~n + C(f~n) handed three steps after they are computed
constexpr int FV_RING = 2, FV_RING_B = 4;
// words of the whole hand-over area of a fused step, per lane
template <class S, bool TH> constexpr int fused_ring_words() { return (FV_RING + FV_RING_B) * (TH ? 18 : 9); }

// One FV stage over work item `item` (strip item % n_strips, chunk
// item / n_strips) of the simulation described by A, on W lanes (lane t;
// lds: this item's exchange rows).  In a fused step (MODE != FV_ALONE) the
// strips carry a halo of four columns; the first half (the predictor) forms
// f~* on the rows and columns the second half's stencils reach and hands
// every formed row, in its stored form, to the second half through `ring`,
// with the collision base f~n + C(f~n) of each row of the chunk; the second
// half (the corrector) reads its input rows there one step of the march
// after they were formed, takes its own cells' base from the ring instead
// of recomputing it, and stores f~n+1.  Both halves meet at one barrier per
// step of the march: a ring row is written before a step's barrier and read
// after it, and rewritten only after the next one.
template <class R, class S, bool TH, bool CORR, int W, int MODE = FV_ALONE>
__device__ __forceinline__ void fv_item(const FvArgs<R>& A, const int item, const int t,
                                        R (*lds)[6 * (TH ? 2 : 1)][W], uint32_t* ring = nullptr) {
    static_assert(MODE == FV_ALONE || (W == FV_LANES && (MODE == FV_SECOND) == CORR && sizeof(R) == 4),
                  "fused halves: wide items, FP32 arithmetic, the predictor first");
    constexpr int NSP = TH ? 2 : 1;
    constexpr int HW = MODE == FV_ALONE ? FV_HALO : FV_FUSED_HALO;
    const int strip = item % A.n_strips, chunk = item / A.n_strips;
    const int x0 = strip * A.strip_w;
    const int own = min(A.strip_w, A.nx - x0);
    const int lanes = own + 2 * HW;
    if ((t & ~63) >= lanes) return;  // a wave without columns of this strip leaves (barriers count live waves)

    // ---- this lane's column (ghost columns mirror or wrap) ----
    const int xg = x0 - HW + t;
    int col = xg;
    bool mx = false;   // ghost column of a no-slip wall
    bool dxg = false;  // ghost column of a fixed-density boundary (density rho_S on its face)
    R rho_S = R(1);
    if (xg < 0) {
        if (A.wall_x) { col = -xg - 1; mx = A.wall_x == 1; dxg = A.wall_x == 2; rho_S = A.rho_x0; }
        else col = xg + A.nx;
    } else if (xg >= A.nx) {
        if (A.wall_x) { col = 2 * A.nx - 1 - xg; mx = A.wall_x == 1; dxg = A.wall_x == 2; rho_S = A.rho_x1; }
        else col = xg - A.nx;
    }
    if (t >= lanes) { col = 0; mx = false; dxg = false; }  // idle lane of a live wave
    const bool owned = t >= HW && t < HW + own;
    // cells whose new values are formed: the owned ones, and in the first
    // half of a fused step every lane whose stencil lies in the strip
    const bool formed = MODE == FV_FIRST ? (t >= 2 && t < lanes - 2) : owned;

    R xc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) xc[q] = formed ? A.xcoef[col * 8 + q] : R(0);

    const uint32_t gb = A.group_bytes, ro = A.rest_off;
    const uint32_t nxu = uint32_t(A.nx), colu = uint32_t(col);
    const Buf bsrc = make_buf(A.src, A.state_bytes);
    const Buf bdst = make_buf(A.dst, A.state_bytes);
    const Buf baux = make_buf(A.aux, A.state_bytes);

    const int y0 = chunk * A.chunk_h;
    const int y1 = min(y0 + A.chunk_h, A.ny);
    const StageK<R> k = A.k;
    typedef const __attribute__((address_space(4))) R CR;
    // rows formed by the first half of a fused step (those the second
    // half's stencils reach; at a y wall only the rows inside)
    const int f_lo = A.wall_y ? max(y0 - 2, 0) : y0 - 2;
    const int f_hi = A.wall_y ? min(y1 + 2, A.ny) : y1 + 2;
    // the fused halves' hand-over rings: [FV_RING][9 NSP][W] words of f~*
    // offsets, then [FV_RING_B][9 NSP][W] words of collision bases
    constexpr int RW = 9 * NSP;
    auto ring_at = [&](const int row, const int w) __attribute__((always_inline)) -> uint32_t& {
        const int slot = (row - (y0 - 4) + 4 * FV_RING) % FV_RING;
        return ring[(slot * RW + w) * W + t];
    };
    auto base_at = [&](const int row, const int w) __attribute__((always_inline)) -> R& {
        const int slot = (row - (y0 - 4)) % FV_RING_B;
        return reinterpret_cast<R*>(ring + FV_RING * RW * W)[(slot * (9 * NSP) + w) * W + t];
    };
    // a fused step at a bottom wall: the second half's ghost rows -1 and -2
    // are the mirrors of rows 0 and 1, which the first half forms after
    // them; the second half skips those two steps and writes the ghost rows
    // into its rings when it computes rows 0 and 1 (items of a fused step
    // are at least two rows high: only the first chunk starts below row 2)
    const bool ghost_later = MODE == FV_SECOND && A.wall_y && y0 == 0;

    // rings: phi of c_y=+1 and c_y=-1 populations of the last four rows,
    // partial updates (all but the y flux) of the last two rows
    R UP[4][NSP][3], DN[4][NSP][3], U[2][NSP][9];
    R TRg[4] = {0, 0, 0, 0};  // thermal reference of the rows in the UP/DN rings
    R QRg[4] = {0, 0, 0, 0};  // heat-flux reference of those rows (split storage)
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int s = 0; s < NSP; ++s)
#pragma unroll
            for (int p = 0; p < 3; ++p) UP[q][s][p] = DN[q][s][p] = R(0);
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int s = 0; s < NSP; ++s)
#pragma unroll
            for (int a = 0; a < 9; ++a) U[q][s][a] = R(0);

    // One row of the march.  The body is free of block-uniform branches (so
    // the unrolled rings stay in fixed registers): every row is exchanged
    // through LDS, ghost rows are selected arithmetically (in the trips that
    // may hold them), and only the stores and the owned lanes' flux are
    // masked.
    // Storage row of march row r (ghost rows mirror or wrap; rows past the
    // chunk end, the padding of the last unrolled trip, are clamped).
    auto map_row = [&](const int r) __attribute__((always_inline)) {
        int row = r;
        if (r < 0) row = A.wall_y ? -r - 1 : r + A.ny;
        else if (r >= A.ny) row = A.wall_y ? 2 * A.ny - 1 - r : r - A.ny;
        return min(max(row, 0), A.ny - 1);
    };
    // Rows are loaded one row ahead of their use (software pipelining): the
    // loads of row r+1 are in flight while row r is computed.  The FP64
    // instance (the parity path) loads each row where it is used: two rows of
    // f and g (and the corrector's own-cell input) in double would not fit
    // next to its rings in registers.
    constexpr bool AHEAD = sizeof(R) == 4;
    // The corrector's own-cell input goes one row ahead only for 16-bit
    // storage, whose prefetched words stay packed two to a register.
    constexpr bool AHEAD_OWN = AHEAD && sizeof(S) == 2 && !is_split<S>::value;
    // Moment-split storage keeps the prefetched records packed (PR, AR) and
    // decodes a row where it is used: the stencil record at the top of its
    // row, the corrector's own-cell record only for the base.
    constexpr bool SPLIT = is_split<S>::value;
    // whether the stage input is a split record (the second half of a fused
    // step reads FP32 offsets from the ring)
    constexpr bool SPLIT_IN = SPLIT && MODE != FV_SECOND;
    // The halves of a fused step with g keep a lane's twelve exchanged
    // brackets together in LDS (three 16-byte words per lane, those moving
    // to +x first), so a neighbour's values come in a few wide reads.
    constexpr bool XT = TH && MODE != FV_ALONE && sizeof(R) == 4;
    auto xslot = [](int s, int p) { return (p < 3 ? 0 : 6) + 3 * s + p % 3; };
    // LATE: the second half into split storage encodes and stores its
    // finished row after the row's barrier, behind the exchange reads, so
    // that the encoder's arithmetic covers their latency
    constexpr bool LATE = XT && MODE == FV_SECOND && SPLIT;   // (measured: faster with split storage only)
    // neighbour lanes of the exchange, clamped to the item (lanes whose flux
    // is formed never reach the clamp)
    const int lm2 = max(t - 2, 0), lm1 = max(t - 1, 0), lp1 = min(t + 1, W - 1), lp2 = min(t + 2, W - 1);
    // The second half of a fused step into split storage works with twice
    // its update (base f~n + C(f~n) + f~* and the flux weights of dt, not
    // dt/2): scaling by two is exact, so every value it forms is exactly
    // twice that of the plain form, and the encoder halves the moments (four
    // products instead of eighteen here).
    constexpr bool X2 = SPLIT && MODE == FV_SECOND;
    R PF[2][9], PG[2][9], PH[2][9], PHG[2][9];
    SplitRaw<TH> PR[2], AR[2];

    auto load_any = [&](const Buf& b, uint32_t cell, R* f, R* g) __attribute__((always_inline)) {
        if constexpr (!SPLIT) load_cell<R, S, TH>(b, cell, gb, ro, f, g);
    };
    // row of the corrector's own-cell input (f~n): rows outside the grid are
    // clamped (their results are not used)
    auto own_row = [&](const int r) __attribute__((always_inline)) { return min(max(r, 0), A.ny - 1); };
    auto prefetch = [&](const int r, auto slot_tag) __attribute__((always_inline)) {
        constexpr int Q = decltype(slot_tag)::value & 1;
        const uint32_t cell = uint32_t(map_row(r)) * nxu + colu;
        if constexpr (SPLIT) {
            load_split_raw<S, TH>(bsrc, cell, gb, PR[Q]);
        } else {
            load_any(bsrc, cell, PF[Q], PG[Q]);
            if (CORR && AHEAD_OWN && MODE == FV_ALONE && formed)  // the corrector's own-cell input (f~n)
                load_any(baux, uint32_t(own_row(r)) * nxu + colu, PH[Q], PHG[Q]);
        }
    };
    // The corrector's own-cell record of the next row is requested after the
    // row's barrier, away from the burst of the next row's stencil loads at
    // the top of the row (every lane: row and column are in range).
    auto prefetch_own = [&](const int r, auto slot_tag) __attribute__((always_inline)) {
        constexpr int Q = decltype(slot_tag)::value & 1;
        if constexpr (SPLIT)
            if (CORR && MODE == FV_ALONE) load_split_raw<S, TH>(baux, uint32_t(own_row(r)) * nxu + colu, gb, AR[Q]);
    };
    // The second half of a fused step reads its input row from the ring, at
    // the row where it is used (the row after it may still be in the making).
    // A ghost row at a y wall reads its mirror row.
    auto ring_read = [&](const int r, auto slot_tag) __attribute__((always_inline)) {
        constexpr int Q = decltype(slot_tag)::value & 1;
        const int src = (A.wall_y && (r < 0 || r >= A.ny)) ? map_row(r) : r;
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            PF[Q][a] = __uint_as_float(ring_at(src, a));
            if (TH) PG[Q][a] = __uint_as_float(ring_at(src, 9 + a));
        }
    };
    // store the offsets of a cell of a row whose thermal reference is trow,
    // and note whether the cell is finite (its moments; otherwise its rest
    // populations): the item raises the non-finite flag once, at its end
    bool bad = false;
    auto store_any = [&](const Buf& b, uint32_t cell, const R* f, const R* g, const R trow, const R qrow)
                         __attribute__((always_inline)) {
        R chk;
        if constexpr (SPLIT) {
            chk = store_split<R, S, TH, X2>(b, cell, gb, f, g, k, trow, qrow);
        } else {
            store_cell<R, S, TH>(b, cell, gb, ro, f, g);
            chk = TH ? f[0] + g[0] : f[0];
        }
        bad = bad || !__builtin_isfinite(chk);
    };
    // first half of a fused step: hand the formed row of f~* to the second
    // half as FP32 offsets (it is never stored)
    auto store_hand = [&](const int j, const R* f, const R* g) __attribute__((always_inline)) {
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            ring_at(j, a) = __float_as_uint(float(f[a]));
            if (TH) ring_at(j, 9 + a) = __float_as_uint(float(g[a]));
        }
    };

    // GH = 1 or 2: rows 0 and 1 of the corrector's first trip at a bottom
    // wall, which also write the ghost rows -1 and -2 (0: any other row; the
    // rows that write ghost rows are separate copies, so the march itself
    // carries no code for them).  YG: the row may lie beyond a y wall.
    auto row_step = [&](const int r, auto slot_tag, auto gh_tag, auto yg_tag) __attribute__((always_inline)) {
        constexpr int SL = decltype(slot_tag)::value;  // (r - y0 + 2) mod 4
        constexpr int GH = MODE == FV_SECOND ? decltype(gh_tag)::value : 0;
        const bool my = decltype(yg_tag)::value && A.wall_y && (r < 0 || r >= A.ny);
        // thermal reference of this row (uniform; ghost rows use their mirror's)
        R Tr = k.ref_g, Qr = 0;
        if (TH && A.tref) Tr = ((const CR*)A.tref)[map_row(r)];
        if (SPLIT && TH && A.qref) Qr = ((const CR*)A.qref)[map_row(r)];
        // wall temperature for the anti-reflection of the shifted brackets
        const R Tw = (r < 0 ? A.Tb : A.Tt) - Tr;

        if (MODE == FV_SECOND) ring_read(r, Slot<SL>{});
        else if (!AHEAD) prefetch(r, Slot<SL>{});
        R df[9], dg[9], mm[4];
        if constexpr (SPLIT_IN) {
            // While stores are outstanding the compiler waits for all vector
            // memory operations at the first use of a load, so the decode of
            // this row's stencil record comes first and the next row's is
            // requested right after it.
            decode_split<R, S, TH>(PR[SL & 1], mm, df, dg);
            __builtin_amdgcn_sched_barrier(0);
            if (AHEAD && MODE != FV_SECOND) prefetch(r + 1, Slot<SL + 1>{});
        } else {
#pragma unroll
            for (int a = 0; a < 9; ++a) {
                df[a] = PF[SL & 1][a];
                if (TH) dg[a] = PG[SL & 1][a];
            }
            if (AHEAD && MODE != FV_SECOND) prefetch(r + 1, Slot<SL + 1>{});
            if (CORR && !AHEAD_OWN && MODE == FV_ALONE && formed)  // own-cell input of this row, used after the stage
                load_any(baux, uint32_t(own_row(r)) * nxu + colu, PH[SL & 1], PHG[SL & 1]);
        }

        R ph[NSP][9], bs[NSP][9];
        if constexpr (SPLIT_IN) {  // decodes df, dg to offsets in place
            if (CORR) stage_split<R, TH, false, true>(mm, df, dg, k, Tr, Qr, ph, bs);
            else stage_split<R, TH, true, false>(mm, df, dg, k, Tr, Qr, ph, bs);
        } else {
            if (CORR) stage<R, TH, false>(df, dg, k, Tr, ph, bs);
            else stage<R, TH, true>(df, dg, k, Tr, ph, bs);
        }
        // ghost row (y walls): double reflection of f, anti-reflection of g
        {
            R tmp[NSP][9];
#pragma unroll
            for (int s = 0; s < NSP; ++s)
#pragma unroll
                for (int a = 1; a < 9; ++a) tmp[s][a] = ph[s][a];
#pragma unroll
            for (int a = 1; a < 9; ++a) {
                ph[0][a] = my ? tmp[0][opp(a)] : tmp[0][a];
                if (TH) ph[NSP - 1][a] = my ? R(2) * wt<R>(a) * Tw - tmp[NSP - 1][opp(a)] : tmp[NSP - 1][a];
            }
        }
        if (MODE == FV_ALONE && mx) {  // ghost column (x walls; fused steps have none): double reflection of both species
#pragma unroll
            for (int s = 0; s < NSP; ++s) {
                R tmp[9];
#pragma unroll
                for (int a = 1; a < 9; ++a) tmp[a] = ph[s][a];
#pragma unroll
                for (int a = 1; a < 9; ++a) ph[s][a] = tmp[opp(a)];
            }
        }
        if (MODE == FV_ALONE && !TH && A.wall_x == 2) {
            // ghost column of a fixed-density boundary ("Boundary conditions",
            // second rule): the ghost density 2 rho_S - rho (linear through
            // the face value and the mirror cell) rescales the mirror cell's
            // brackets: phi_ghost = s phi, s = (2 rho_S - rho) / rho, i.e.
            // phi - w ref -> s (phi - w ref) + (s - 1) w ref.  Flow only.
            R rho;
            if constexpr (SPLIT_IN) rho = mm[0] + k.ref_f;
            else {
                rho = df[0];
#pragma unroll
                for (int a = 1; a < 9; ++a) rho += df[a];
                rho += k.ref_f;
            }
            const R sc = dxg ? (R(2) * rho_S - rho) / rho : R(1);
            const R sr = (sc - R(1)) * k.ref_f;
#pragma unroll
            for (int a = 1; a < 9; ++a) ph[0][a] = sc * ph[0][a] + wt<R>(a) * sr;
        }

        // ---- y flux: finish row j = r - 2 (phi rows j-2 .. j+2) before the
        //      partial update of row r takes over the U slot of row j ----
        const int j = r - 2;
        // y weights of row j: uniform, read as scalar loads (constant address
        // space) in uniform control flow, so no vector-memory wait is needed
        R yc[8];
        {
            const CR* yw = (const CR*)(A.ycoef) + int64_t(map_row(j)) * 8;   // (a periodic row wraps)
#pragma unroll
            for (int q = 0; q < 8; ++q) yc[q] = yw[q];
        }
        // A per-row thermal reference shifts the brackets of g by
        // w_a Tr(row); across rows the shift does not cancel from the y
        // stencil, so its flux is added back (uniform per row).  The weights
        // sum to zero, so the flux is taken of Tr(row) - Tr(j), which keeps
        // it free of the rounding of that sum.
        R sU = 0, sD = 0;
        if (TH && A.tref) {
            const R tj = TRg[(SL + 2) & 3];
            sU = yc[0] * (TRg[SL] - tj) + yc[1] * (TRg[(SL + 1) & 3] - tj) + yc[3] * (TRg[(SL + 3) & 3] - tj);
            sD = yc[4] * (TRg[(SL + 1) & 3] - tj) + yc[6] * (TRg[(SL + 3) & 3] - tj) + yc[7] * (Tr - tj);
        }
        R out[NSP][9];
        bool store_late = false;
        if (MODE == FV_FIRST ? (formed && j >= f_lo && j < f_hi) : (owned && j >= y0 && j < y1)) {
#pragma unroll
            for (int s = 0; s < NSP; ++s) {
#pragma unroll
                for (int a = 0; a < 9; ++a) out[s][a] = U[SL & 1][s][a];
#pragma unroll
                for (int p = 0; p < 3; ++p) {
                    // c_y = +1: rows j-2 .. j+1 = r-4 .. r-1  (ring slots SL, SL+1, SL+2, SL+3)
                    out[s][upop(p)] -= yc[0] * UP[SL][s][p] + yc[1] * UP[(SL + 1) & 3][s][p] +
                                       yc[2] * UP[(SL + 2) & 3][s][p] + yc[3] * UP[(SL + 3) & 3][s][p];
                    // c_y = -1: rows j-1 .. j+2 = r-3 .. r
                    out[s][dpop(p)] -= yc[4] * DN[(SL + 1) & 3][s][p] + yc[5] * DN[(SL + 2) & 3][s][p] +
                                       yc[6] * DN[(SL + 3) & 3][s][p] + yc[7] * ph[s][dpop(p)];
                    if (TH && s == NSP - 1) {
                        out[s][upop(p)] -= wt<R>(upop(p)) * sU;
                        out[s][dpop(p)] -= wt<R>(dpop(p)) * sD;
                    }
                }
            }
            if (MODE == FV_FIRST)
                store_hand(j, out[0], out[NSP - 1]);
            else if (LATE)
                store_late = true;
            else
                store_any(bdst, uint32_t(j) * nxu + colu, out[0], out[NSP - 1], TRg[(SL + 2) & 3], QRg[(SL + 2) & 3]);
        }

        // ---- x flux and partial update (all but the y flux) of row r ----
        const int b = SL & 1;
        if constexpr (XT) {
            R xv[12];
#pragma unroll
            for (int s = 0; s < NSP; ++s)
#pragma unroll
                for (int p = 0; p < 6; ++p) xv[xslot(s, p)] = ph[s][xpop(p)];
            float4* xw = reinterpret_cast<float4*>(&lds[b][0][0] + 12 * t);
#pragma unroll
            for (int q = 0; q < 3; ++q) xw[q] = float4{xv[4 * q], xv[4 * q + 1], xv[4 * q + 2], xv[4 * q + 3]};
        } else {
#pragma unroll
            for (int s = 0; s < NSP; ++s)
#pragma unroll
                for (int p = 0; p < 6; ++p) lds[b][s * 6 + p][t] = ph[s][xpop(p)];
        }
        lanes_sync<W>();
        R Lm2[12], Lm1[12], Lp1[12], Lp2[12];
        auto x_reads = [&]() __attribute__((always_inline)) {
            const R* xb = &lds[b][0][0];
            auto ld4 = [&](R* o, int lane, int q) __attribute__((always_inline)) {
                const float4 x = *reinterpret_cast<const float4*>(xb + 12 * lane + q);
                o[q] = x.x; o[q + 1] = x.y; o[q + 2] = x.z; o[q + 3] = x.w;
            };
            auto ld2 = [&](R* o, int lane, int q) __attribute__((always_inline)) {
                const float2 x = *reinterpret_cast<const float2*>(xb + 12 * lane + q);
                o[q] = x.x; o[q + 1] = x.y;
            };
            // (reads issued for every lane take clamped neighbours; inside
            // the flux block the lanes are those whose flux is formed)
            const int m2 = LATE ? lm2 : t - 2, m1 = LATE ? lm1 : t - 1, p1 = LATE ? lp1 : t + 1, p2 = LATE ? lp2 : t + 2;
            ld4(Lm2, m2, 0); ld2(Lm2, m2, 4);
            ld4(Lm1, m1, 0); ld4(Lm1, m1, 4); ld4(Lm1, m1, 8);
            ld4(Lp1, p1, 0); ld4(Lp1, p1, 4); ld4(Lp1, p1, 8);
            ld2(Lp2, p2, 6); ld4(Lp2, p2, 8);
        };
        if constexpr (LATE) {
            // the exchange reads first, then the store of the finished row
            // while they arrive
            x_reads();
            if (store_late)
                store_any(bdst, uint32_t(j) * nxu + colu, out[0], out[NSP - 1], TRg[(SL + 2) & 3], QRg[(SL + 2) & 3]);
        }
        if (SPLIT && CORR && AHEAD && MODE == FV_ALONE) {
            __builtin_amdgcn_sched_barrier(0);
            prefetch_own(r + 1, Slot<SL + 1>{});
            __builtin_amdgcn_sched_barrier(0);
        }
        // (the partial update of a row is kept only where a later row's y
        // flux finishes it: rows the half forms or owns)
        if (formed && (MODE == FV_FIRST ? (r >= f_lo && r < f_hi) : (r >= y0 && r < y1))) {
            R base[NSP][9];
            if (CORR) {
                // f~n+1 = (f~n + C(f~n) + f~*)/2 - dt/2 D(phi*): C from f~n at this
                // cell (in a fused step, from the first half, which computed it)
                R phn[NSP][9], bn[NSP][9];
                if constexpr (MODE == FV_SECOND) {
#pragma unroll
                    for (int s = 0; s < NSP; ++s)
#pragma unroll
                        for (int a = 0; a < 9; ++a) bn[s][a] = base_at(r, s * 9 + a);
                } else if constexpr (SPLIT) {
                    R hm[4], hf[9], hg[9];
                    decode_split<R, S, TH>(AR[SL & 1], hm, hf, hg);
                    stage_split<R, TH, true, false>(hm, hf, hg, k, Tr, Qr, phn, bn);
                } else {
                    stage<R, TH, true>(PH[SL & 1], PHG[SL & 1], k, Tr, phn, bn);
                }
#pragma unroll
                for (int a = 0; a < 9; ++a) {
                    base[0][a] = X2 ? bn[0][a] + df[a] : R(0.5) * (bn[0][a] + df[a]);
                    if (TH) base[NSP - 1][a] = X2 ? bn[NSP - 1][a] + dg[a] : R(0.5) * (bn[NSP - 1][a] + dg[a]);
                }
            } else {
#pragma unroll
                for (int s = 0; s < NSP; ++s)
#pragma unroll
                    for (int a = 0; a < 9; ++a) base[s][a] = bs[s][a];
                if (MODE == FV_FIRST && r >= y0 && r < y1) {   // the second half's base of this row
#pragma unroll
                    for (int s = 0; s < NSP; ++s)
#pragma unroll
                        for (int a = 0; a < 9; ++a) base_at(r, s * 9 + a) = bs[s][a];
                }
            }
            if constexpr (XT && !LATE) x_reads();
#pragma unroll
            for (int s = 0; s < NSP; ++s) {
#pragma unroll
                for (int p = 0; p < 6; ++p) {
                    const int a = xpop(p);
                    const R* L = lds[b][s * 6 + p];
                    const R v = ph[s][a];
                    R d;
                    if constexpr (XT) {
                        const int q = xslot(s, p);
                        if (cx(a) > 0)
                            d = xc[0] * Lm2[q] + xc[1] * Lm1[q] + xc[2] * v + xc[3] * Lp1[q];
                        else
                            d = xc[4] * Lm1[q] + xc[5] * v + xc[6] * Lp1[q] + xc[7] * Lp2[q];
                    } else if (cx(a) > 0)
                        d = xc[0] * L[t - 2] + xc[1] * L[t - 1] + xc[2] * v + xc[3] * L[t + 1];
                    else
                        d = xc[4] * L[t - 1] + xc[5] * v + xc[6] * L[t + 1] + xc[7] * L[t + 2];
                    base[s][a] -= d;
                }
#pragma unroll
                for (int a = 0; a < 9; ++a) U[SL & 1][s][a] = base[s][a];
            }
        }
        // ---- push this row into the rings ----
        TRg[SL] = Tr;
        QRg[SL] = Qr;
#pragma unroll
        for (int s = 0; s < NSP; ++s)
#pragma unroll
            for (int p = 0; p < 3; ++p) {
                UP[SL][s][p] = ph[s][upop(p)];
                DN[SL][s][p] = ph[s][dpop(p)];
            }
        // ghost rows -1 (at row 0) and -2 (at row 1) of a fused step at a
        // bottom wall, as the ghost-row code above forms them from the mirror
        // row: double reflection of f, anti-reflection of g (opp(upop(p)) =
        // dpop(p)); the slots are those of rows r - 1 and r - 3
        if constexpr (GH != 0) {
            const R Twb = A.Tb - Tr;
            auto ghost = [&](auto g_tag) __attribute__((always_inline)) {
                constexpr int G = decltype(g_tag)::value;
                TRg[G] = Tr;
                QRg[G] = Qr;
#pragma unroll
                for (int p = 0; p < 3; ++p) {
                    UP[G][0][p] = ph[0][dpop(p)];
                    DN[G][0][p] = ph[0][upop(p)];
                    if (TH) {
                        UP[G][NSP - 1][p] = R(2) * wt<R>(upop(p)) * Twb - ph[NSP - 1][dpop(p)];
                        DN[G][NSP - 1][p] = R(2) * wt<R>(dpop(p)) * Twb - ph[NSP - 1][upop(p)];
                    }
                }
            };
            ghost(Slot<GH == 1 ? (SL + 3) & 3 : (SL + 1) & 3>{});
        }
    };

    // Rows y0-2 .. y1+1 in trips of four; the trip may run up to three rows
    // past y1+1 (their results are never stored).  A chunk of height 4k
    // needs exactly k+1 trips.  The first half of a fused step marches two
    // rows further each way (rows y0-4 .. y1+3 of f~n) and forms row j of
    // f~* at its step j - y0 + 6; the second half reads row r at step
    // r - y0 + 7, five idle steps after the first half began, and both
    // halves end on the same count of barriers.
    const int r0 = MODE == FV_FIRST ? y0 - 4 : y0 - 2;
    const int r1 = MODE == FV_FIRST ? y1 + 3 : y1 + 1;
    const int steps1 = ((y1 + 3) - (y0 - 4) + 4) / 4 * 4;      // march steps of the first half
    const int steps2 = ((y1 + 1) - (y0 - 2) + 4) / 4 * 4;      // of the second
    const int before = MODE == FV_SECOND ? 5 : 0;               // idle steps before the march
    const int total = max(steps1, 5 + steps2);
    for (int q = 0; q < before; ++q) lanes_sync<W>();
    if (AHEAD && MODE != FV_SECOND) prefetch(r0, Slot<0>{});
    if (AHEAD && MODE == FV_ALONE) prefetch_own(r0, Slot<0>{});
    int r = r0;
    if constexpr (MODE == FV_SECOND) {
        if (ghost_later) {   // the first trip (rows -2 .. 1): the ghost rows come with rows 0 and 1
            lanes_sync<W>();
            lanes_sync<W>();
            row_step(0, Slot<2>{}, Slot<1>{}, Slot<1>{});
            row_step(1, Slot<3>{}, Slot<2>{}, Slot<1>{});
            r += 4;
        }
    }
    auto trip = [&](const int r, auto yg_tag) __attribute__((always_inline)) {
        row_step(r, Slot<0>{}, Slot<0>{}, yg_tag);
        row_step(r + 1, Slot<1>{}, Slot<0>{}, yg_tag);
        row_step(r + 2, Slot<2>{}, Slot<0>{}, yg_tag);
        row_step(r + 3, Slot<3>{}, Slot<0>{}, yg_tag);
    };
    // Fused halves march the trips that may hold rows beyond a y wall (whose
    // brackets are reflected) apart from the others, which carry no code for
    // the reflection: the first half's trips below row 0, then every trip
    // inside the grid, then those reaching row ny.  (The second half has
    // none below row 0 at a wall: its first trip is the one above.)
    if constexpr (MODE == FV_ALONE) {
        for (; r <= r1; r += 4) {
            row_step(r, Slot<0>{}, Slot<0>{}, Slot<1>{});
            row_step(r + 1, Slot<1>{}, Slot<0>{}, Slot<1>{});
            row_step(r + 2, Slot<2>{}, Slot<0>{}, Slot<1>{});
            row_step(r + 3, Slot<3>{}, Slot<0>{}, Slot<1>{});
        }
    } else {
        if (MODE == FV_FIRST && A.wall_y)
            for (; r <= r1 && r < 0; r += 4) trip(r, Slot<1>{});
        for (; r <= r1 && !(A.wall_y && r + 3 >= A.ny); r += 4) trip(r, Slot<0>{});
        for (; r <= r1; r += 4) trip(r, Slot<1>{});
    }
    if (MODE != FV_ALONE)
        for (int q = before + (MODE == FV_FIRST ? steps1 : steps2); q < total; ++q) lanes_sync<W>();
    if (A.bad) raise_flag(A.bad, bad);
}

// ---- fused step: the predictor and the corrector of one Heun step ----
// A block of 2 x FV_LANES lanes on one strip: the first FV_LANES run the
// predictor (eq:semi) over the strip and two cells beyond it (rows and
// columns), forming f~* where the corrector's stencils reach, and hand each
// formed row, as it would be stored, to the others through an LDS ring,
// with the collision base f~n + C(f~n) of the strip's cells; the others run
// the corrector (eq:semi-heun) on those rows and store f~n+1.  Each half
// runs the code of the separate launch (the same arithmetic in the same
// order, on the same stored values), so the results are those of a
// predictor launch followed by a corrector launch, bit for bit, while a step
// reads f~n once and writes f~n+1 once.  Each wave holds one stage's rings,
// so two waves (one of each half) share a SIMD.  x is periodic (with x walls
// the host uses separate launches); items are wide strips.
template <class R, class S, bool TH>
__device__ __forceinline__ void fused_halves(const FvArgs<R>& A, const int item, R (*x1)[6 * (TH ? 2 : 1)][FV_LANES],
                                             R (*x2)[6 * (TH ? 2 : 1)][FV_LANES], uint32_t* ring) {
    if (threadIdx.x < FV_LANES) {
        fv_item<R, S, TH, false, FV_LANES, FV_FIRST>(A, item, threadIdx.x, x1, ring);
    } else {
        FvArgs<R> C = A;   // the corrector's flux weights
        if (!is_split<S>::value) {   // (split storage: twice them, see fv_item)
            C.xcoef = A.xcoef2;
            C.ycoef = A.ycoef2;
        }
        fv_item<R, S, TH, true, FV_LANES, FV_SECOND>(C, item, threadIdx.x - FV_LANES, x2, ring);
    }
}
// (without g a half holds few enough registers for two blocks per CU)
template <class R, class S, bool TH>
__global__ void __launch_bounds__(2 * FV_LANES, TH ? 1 : 2) fv_fused(FvArgs<R> A) {
    constexpr int NSP = TH ? 2 : 1;
    // (16-byte aligned: with g a lane's exchanged values are read as 16-byte words)
    __shared__ __attribute__((aligned(16))) R x1[2][6 * NSP][FV_LANES];
    __shared__ __attribute__((aligned(16))) R x2[2][6 * NSP][FV_LANES];
    __shared__ uint32_t ring[fused_ring_words<S, TH>() * FV_LANES];
    const int b = xcd_item(blockIdx.x, A.n_items);
    if (b >= A.n_items) return;
    fused_halves<R, S, TH>(A, b, x1, x2, ring);
}

// Fused steps of many simulations in one launch (serving): a work list of
// (simulation, local item) pairs over a table of two argument blocks per
// simulation, one per direction of its pair of state buffers, chosen by its
// phase (0: the state is in the first buffer, 1: in the second; the tick
// kernel flips it after each step the simulation takes).  A simulation with
// no steps left is skipped.  Every item runs the code of fv_fused, so a
// simulation's result does not depend on what else shares the launch.
template <class R, class S, bool TH>
__global__ void __launch_bounds__(2 * FV_LANES, TH ? 1 : 2)
    fv_fused_multi(const FvArgs<R>* args, const int2* items, int n_items, const int64_t* left, const int* phase) {
    constexpr int NSP = TH ? 2 : 1;
    // (16-byte aligned: with g a lane's exchanged values are read as 16-byte words)
    __shared__ __attribute__((aligned(16))) R x1[2][6 * NSP][FV_LANES];
    __shared__ __attribute__((aligned(16))) R x2[2][6 * NSP][FV_LANES];
    __shared__ uint32_t ring[fused_ring_words<S, TH>() * FV_LANES];
    const int b = xcd_item(blockIdx.x, n_items);
    if (b >= n_items) return;
    const int2 it = items[b];
    if (left[it.x] <= 0) return;
    // the argument block is uniform over the item: scalar loads
    static_assert(sizeof(FvArgs<R>) % 4 == 0, "argument block in words");
    typedef const __attribute__((address_space(4))) uint32_t CW;
    const int ph = __builtin_amdgcn_readfirstlane(phase[it.x]);
    CW* src = (CW*)(args + 2 * it.x + ph);
    uint32_t words[sizeof(FvArgs<R>) / 4];
#pragma unroll
    for (int q = 0; q < int(sizeof(FvArgs<R>) / 4); ++q) words[q] = src[q];
    FvArgs<R> A;
    __builtin_memcpy(&A, words, sizeof(FvArgs<R>));
    fused_halves<R, S, TH>(A, it.y, x1, x2, ring);
}
// Blocks per CU the register budget is sized for: two waves per SIMD (FP32
// arithmetic) or one (FP64).
template <class R> constexpr int FV_MIN_BLOCKS = (sizeof(R) == 4 ? 8 : 4) * 64 / FV_LANES;

// Block b runs one wide item (FV_LANES lanes) or, in narrow mode, four
// independent 64-lane items, one per wave: narrow strips waste fewer lanes
// on grids whose width is not close to a multiple of FV_LANES - 4.  A wave
// of a narrow block synchronises with itself only.
template <class R, class S, bool TH, bool CORR>
__device__ __forceinline__ void fv_block(const FvArgs<R>& A, const int item, const bool narrow, R* lds_mem) {
    constexpr int NSP = TH ? 2 : 1;
    if (narrow) {
        const int w = threadIdx.x >> 6;
        fv_item<R, S, TH, CORR, 64>(A, item, threadIdx.x & 63,
                                    reinterpret_cast<R(*)[6 * NSP][64]>(lds_mem + w * (2 * 6 * NSP * 64)));
    } else {
        fv_item<R, S, TH, CORR, FV_LANES>(A, item, threadIdx.x, reinterpret_cast<R(*)[6 * NSP][FV_LANES]>(lds_mem));
    }
}

// One simulation: arguments by value.
template <class R, class S, bool TH, bool CORR>
__global__ void __launch_bounds__(FV_LANES, FV_MIN_BLOCKS<R>) fv_pass(FvArgs<R> A) {
    __shared__ R lds_mem[2 * 6 * (TH ? 2 : 1) * FV_LANES];
    const int nb = A.narrow ? (A.n_items + 3) / 4 : A.n_items;
    const int b = xcd_item(blockIdx.x, nb);
    if (b >= nb) return;
    if (A.narrow) {
        const int item = 4 * b + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        if (item >= A.n_items) return;
        fv_block<R, S, TH, CORR>(A, item, true, lds_mem);
    } else {
        fv_block<R, S, TH, CORR>(A, b, false, lds_mem);
    }
}

// Many simulations in one launch (serving): a table of per-simulation
// arguments (predictor and corrector entry per simulation), a work list of
// (simulation, local item) pairs, the n_wide items of wide-strip members
// first, then the n_narrow items of narrow-strip members (four to a block),
// and per-simulation remaining steps; the items of a simulation that has
// finished are skipped.  Every item runs the same code as in fv_pass, so a
// simulation's result does not depend on what else shares the launch.
template <class R, class S, bool TH, bool CORR>
__global__ void __launch_bounds__(FV_LANES, FV_MIN_BLOCKS<R>)
    fv_pass_multi(const FvArgs<R>* args, const int2* items, int n_wide, int n_narrow, const int64_t* left) {
    __shared__ R lds_mem[2 * 6 * (TH ? 2 : 1) * FV_LANES];
    const int nb = n_wide + (n_narrow + 3) / 4;
    const int b = xcd_item(blockIdx.x, nb);
    if (b >= nb) return;
    const bool narrow = b >= n_wide;
    int idx = b;
    if (narrow) {
        const int k = 4 * (b - n_wide) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        if (k >= n_narrow) return;
        idx = n_wide + k;
    }
    const int2 it = items[idx];
    if (left[it.x] <= 0) return;
    // the argument block is uniform over the item: copy it word by word with
    // scalar loads
    static_assert(sizeof(FvArgs<R>) % 4 == 0, "argument block in words");
    typedef const __attribute__((address_space(4))) uint32_t CW;
    CW* src = (CW*)(args + 2 * it.x + (CORR ? 1 : 0));
    uint32_t words[sizeof(FvArgs<R>) / 4];
#pragma unroll
    for (int q = 0; q < int(sizeof(FvArgs<R>) / 4); ++q) words[q] = src[q];
    FvArgs<R> A;
    __builtin_memcpy(&A, words, sizeof(FvArgs<R>));
    if (A.bad && *(volatile const int*)A.bad) return;  // a member that blew up is not stepped further
    fv_block<R, S, TH, CORR>(A, it.y, narrow, lds_mem);
}

// One group step done: every member that stepped has one step less to go,
// its state moved to its other buffer (phase != NULL: fused steps), and
// (every[i] > 0) counts towards its next renewal of the thermal references,
// due[i] = 1 when the step count reaches it (as lb_step does).
__global__ void tick_kernel(int64_t* left, int n, const int64_t* every, int64_t* since, int* due, int* phase) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int d = 0;
    if (left[i] > 0) {
        left[i] -= 1;
        if (phase) phase[i] ^= 1;
        if (every && every[i] > 0 && ++since[i] >= every[i]) {
            since[i] = 0;
            d = 1;
        }
    }
    if (due) due[i] = d;
}

template <class R, class S>
static hipError_t launch_multi_typed(bool thermal, bool corrector, const void* args, const int2* items, int n_wide,
                                     int n_narrow, const int64_t* left, hipStream_t s) {
    const FvArgs<R>* a = static_cast<const FvArgs<R>*>(args);
    const int nb = n_wide + (n_narrow + 3) / 4;
    dim3 grid(8 * ((nb + 7) / 8)), block(FV_LANES);
    if (thermal) {
        if (corrector)
            hipLaunchKernelGGL((fv_pass_multi<R, S, true, true>), grid, block, 0, s, a, items, n_wide, n_narrow, left);
        else
            hipLaunchKernelGGL((fv_pass_multi<R, S, true, false>), grid, block, 0, s, a, items, n_wide, n_narrow, left);
    } else {
        if (corrector)
            hipLaunchKernelGGL((fv_pass_multi<R, S, false, true>), grid, block, 0, s, a, items, n_wide, n_narrow, left);
        else
            hipLaunchKernelGGL((fv_pass_multi<R, S, false, false>), grid, block, 0, s, a, items, n_wide, n_narrow, left);
    }
    return hipGetLastError();
}

hipError_t launch_fv_multi(int storage, bool thermal, bool corrector, const void* args, const int2* items,
                           int n_wide, int n_narrow, const int64_t* left, hipStream_t s) {
    if (n_wide + n_narrow <= 0) return hipSuccess;
    switch (storage) {
        case ST_F64: return launch_multi_typed<double, double>(thermal, corrector, args, items, n_wide, n_narrow, left, s);
        case ST_F32: return launch_multi_typed<float, float>(thermal, corrector, args, items, n_wide, n_narrow, left, s);
        case ST_BF16: return launch_multi_typed<float, bf16_t>(thermal, corrector, args, items, n_wide, n_narrow, left, s);
        case ST_F16: return launch_multi_typed<float, f16_t>(thermal, corrector, args, items, n_wide, n_narrow, left, s);
        case ST_BF16S: return launch_multi_typed<float, bf16s_t>(thermal, corrector, args, items, n_wide, n_narrow, left, s);
        case ST_F16S: return launch_multi_typed<float, f16s_t>(thermal, corrector, args, items, n_wide, n_narrow, left, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_tick(int64_t* left, int n, const int64_t* every, int64_t* since, int* due, int* phase,
                       hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(tick_kernel, dim3((n + 255) / 256), dim3(256), 0, s, left, n, every, since, due, phase);
    return hipGetLastError();
}

size_t fv_args_bytes(int storage) { return storage == ST_F64 ? sizeof(FvArgs<double>) : sizeof(FvArgs<float>); }

template <class R, class S>
static hipError_t launch_typed(bool thermal, bool corrector, const void* args, hipStream_t s) {
    const FvArgs<R>& A = *static_cast<const FvArgs<R>*>(args);
    const int nb = A.narrow ? (A.n_items + 3) / 4 : A.n_items;
    dim3 grid(8 * ((nb + 7) / 8)), block(FV_LANES);
    if (thermal) {
        if (corrector)
            hipLaunchKernelGGL((fv_pass<R, S, true, true>), grid, block, 0, s, A);
        else
            hipLaunchKernelGGL((fv_pass<R, S, true, false>), grid, block, 0, s, A);
    } else {
        if (corrector)
            hipLaunchKernelGGL((fv_pass<R, S, false, true>), grid, block, 0, s, A);
        else
            hipLaunchKernelGGL((fv_pass<R, S, false, false>), grid, block, 0, s, A);
    }
    return hipGetLastError();
}

template <class R, class S>
static hipError_t launch_fused_typed(bool thermal, const void* args, hipStream_t s) {
    const FvArgs<R>& A = *static_cast<const FvArgs<R>*>(args);
    if (A.chunk_h < 2) return hipErrorInvalidValue;   // items of at least two rows (the bottom wall's first trip)
    dim3 grid(8 * ((A.n_items + 7) / 8)), block(2 * FV_LANES);
    if (thermal) hipLaunchKernelGGL((fv_fused<R, S, true>), grid, block, 0, s, A);
    else hipLaunchKernelGGL((fv_fused<R, S, false>), grid, block, 0, s, A);
    return hipGetLastError();
}

hipError_t launch_fv_fused(int storage, bool thermal, const void* args, hipStream_t s) {
    switch (storage) {
        case ST_F32: return launch_fused_typed<float, float>(thermal, args, s);
        case ST_BF16: return launch_fused_typed<float, bf16_t>(thermal, args, s);
        case ST_F16: return launch_fused_typed<float, f16_t>(thermal, args, s);
        case ST_BF16S: return launch_fused_typed<float, bf16s_t>(thermal, args, s);
        case ST_F16S: return launch_fused_typed<float, f16s_t>(thermal, args, s);
    }
    return hipErrorInvalidValue;   // FP64 storage uses separate launches
}

template <class R, class S>
static hipError_t launch_fused_multi_typed(bool thermal, const void* args, const int2* items, int n_items,
                                           const int64_t* left, const int* phase, hipStream_t s) {
    const FvArgs<R>* a = static_cast<const FvArgs<R>*>(args);
    dim3 grid(8 * ((n_items + 7) / 8)), block(2 * FV_LANES);
    if (thermal) hipLaunchKernelGGL((fv_fused_multi<R, S, true>), grid, block, 0, s, a, items, n_items, left, phase);
    else hipLaunchKernelGGL((fv_fused_multi<R, S, false>), grid, block, 0, s, a, items, n_items, left, phase);
    return hipGetLastError();
}

hipError_t launch_fv_fused_multi(int storage, bool thermal, const void* args, const int2* items, int n_items,
                                 const int64_t* left, const int* phase, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    switch (storage) {
        case ST_F32: return launch_fused_multi_typed<float, float>(thermal, args, items, n_items, left, phase, s);
        case ST_BF16: return launch_fused_multi_typed<float, bf16_t>(thermal, args, items, n_items, left, phase, s);
        case ST_F16: return launch_fused_multi_typed<float, f16_t>(thermal, args, items, n_items, left, phase, s);
        case ST_BF16S: return launch_fused_multi_typed<float, bf16s_t>(thermal, args, items, n_items, left, phase, s);
        case ST_F16S: return launch_fused_multi_typed<float, f16s_t>(thermal, args, items, n_items, left, phase, s);
    }
    return hipErrorInvalidValue;   // FP64 storage uses separate launches
}

template <class R, class S>
static int fused_resident_typed(bool thermal) {
    int per_cu = 0, dev = 0, cus = 0;
    const void* k = thermal ? (const void*)fv_fused<R, S, true> : (const void*)fv_fused<R, S, false>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 2 * FV_LANES, 0) != hipSuccess) return 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return per_cu * cus;
}

int fv_fused_resident_blocks(int storage, bool thermal) {
    switch (storage) {
        case ST_F32: return fused_resident_typed<float, float>(thermal);
        case ST_BF16: return fused_resident_typed<float, bf16_t>(thermal);
        case ST_F16: return fused_resident_typed<float, f16_t>(thermal);
        case ST_BF16S: return fused_resident_typed<float, bf16s_t>(thermal);
        case ST_F16S: return fused_resident_typed<float, f16s_t>(thermal);
    }
    return 0;
}

template <class R, class S>
static int resident_typed(bool thermal, bool corrector) {
    int per_cu = 0, dev = 0, cus = 0;
    const void* k;
    if (thermal) k = corrector ? (const void*)fv_pass<R, S, true, true> : (const void*)fv_pass<R, S, true, false>;
    else k = corrector ? (const void*)fv_pass<R, S, false, true> : (const void*)fv_pass<R, S, false, false>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, FV_LANES, 0) != hipSuccess) return 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return per_cu * cus;
}

int fv_resident_blocks(int storage, bool thermal, bool corrector) {
    switch (storage) {
        case ST_F64: return resident_typed<double, double>(thermal, corrector);
        case ST_F32: return resident_typed<float, float>(thermal, corrector);
        case ST_BF16: return resident_typed<float, bf16_t>(thermal, corrector);
        case ST_F16: return resident_typed<float, f16_t>(thermal, corrector);
        case ST_BF16S: return resident_typed<float, bf16s_t>(thermal, corrector);
        case ST_F16S: return resident_typed<float, f16s_t>(thermal, corrector);
    }
    return 0;
}

hipError_t launch_fv_pass(int storage, bool thermal, bool corrector, const void* args, hipStream_t s) {
    switch (storage) {
        case ST_F64: return launch_typed<double, double>(thermal, corrector, args, s);
        case ST_F32: return launch_typed<float, float>(thermal, corrector, args, s);
        case ST_BF16: return launch_typed<float, bf16_t>(thermal, corrector, args, s);
        case ST_F16: return launch_typed<float, f16_t>(thermal, corrector, args, s);
        case ST_BF16S: return launch_typed<float, bf16s_t>(thermal, corrector, args, s);
        case ST_F16S: return launch_typed<float, f16s_t>(thermal, corrector, args, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace lbk
