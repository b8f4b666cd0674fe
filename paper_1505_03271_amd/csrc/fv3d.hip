// Three-dimensional FV-LB step on D3Q19 (arXiv:1505.03271 sec. 2.2, the
// lattice of the paper's own runs: "Boundary conditions", last paragraph,
// and sec. 5).  Gravity and the isothermal walls are along z.
//
// One FV stage is two kernels, one thread per cell:
//   fv3_stage   decode the cell, compute its advected brackets
//               phi = f~ + dt/(2 tau~)(f_eq - f~) + dt/2 F   (g: no force)
//               of the 18 moving populations and write them to a scratch
//               buffer (shifted by w_a ref as in the 2D kernel);
//   fv3_update  the QUICK flux divergence D from the scratch buffer along each
//               axis a population moves on (four-point cell stencils with the
//               update factor folded in, ghosts mirrored with the opposite
//               population, or wrapped), the cell's own collision base, and
//               the new state:
//                 predictor / single stage:  f~ + C(f~) - dt D(phi)
//                 Heun corrector:            (f~n + C(f~n) + f~*)/2 - dt/2 D(phi*)
// The flux + update kernel works on 32 x 4 x 4 tiles whose brackets and halo
// brackets are staged in LDS population by population (fv3_update_tiled);
// it also leaves the brackets of its output for the next pass in a second
// scratch buffer, so that only the first pass after a new state runs the
// stage kernel.  fv3_update, one thread per cell reading every stencil point
// from the scratch buffer, computes the same operations in the same order.
// The scratch round trip moves the brackets through HBM once more than a
// fused kernel would.
//
// Storage: FP64 (parity path) or FP32 offsets p - w_a ref, populations as
// (s * 19 + a) * cells + cell, x fastest.
#include <type_traits>
#include <utility>

#include "lb_kernels.h"

namespace lbk {

// ---- D3Q19: rest, 6 axis velocities, 12 edge velocities; opposite pairs adjacent
__host__ __device__ constexpr int c3(int a, int d) {
    constexpr int t[19][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
                              {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
                              {-1, 0, 1}, {0, 1, 1},   {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
    return t[a][d];
}
template <class R> __host__ __device__ constexpr R w3(int a) {
    return a == 0 ? R(1) / R(3) : (a <= 6 ? R(1) / R(18) : R(1) / R(36));
}
__host__ __device__ constexpr int opp3(int a) { return a == 0 ? 0 : ((a & 1) ? a + 1 : a - 1); }
static_assert(opp3(1) == 2 && opp3(2) == 1 && opp3(7) == 8 && opp3(18) == 17, "D3Q19 opposite pairs");

template <class S> struct Store3;
template <> struct Store3<double> {
    static constexpr bool offset = false;
    __device__ static double ld(const double* p) { return *p; }
    __device__ static void st(double* p, double v) { *p = v; }
};
template <> struct Store3<float> {
    static constexpr bool offset = true;
    __device__ static float ld(const float* p) { return *p; }
    __device__ static void st(float* p, float v) { *p = v; }
};

// decoded offsets of one cell, and its macroscopic state
template <class R, class S, bool TH>
__device__ inline void load3(const S* st, int64_t cells, int64_t c, R* df, R* dg) {
#pragma unroll
    for (int a = 0; a < 19; ++a) {
        df[a] = R(Store3<S>::ld(st + int64_t(a) * cells + c));
        if (TH) dg[a] = R(Store3<S>::ld(st + int64_t(19 + a) * cells + c));
    }
}

template <class R, bool TH>
struct Mac3 {
    R rho_p, rho, T_p, T, u[3], acc[3];
};

template <class R, bool TH>
__device__ inline Mac3<R, TH> macro3(const R* df, const R* dg, const StageK<R>& k, const R az) {
    Mac3<R, TH> m;
    R rp = 0, j[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < 19; ++a) {
        rp += df[a];
#pragma unroll
        for (int d = 0; d < 3; ++d)
            if (c3(a, d) > 0) j[d] += df[a];
            else if (c3(a, d) < 0) j[d] -= df[a];
    }
    m.rho_p = rp;
    m.rho = rp + k.ref_f;
    m.T_p = 0;
    if (TH) {
#pragma unroll
        for (int a = 0; a < 19; ++a) m.T_p += dg[a];
    }
    m.T = m.T_p + k.ref_g;
    m.acc[0] = k.ax;
    m.acc[1] = k.ay;
    m.acc[2] = TH ? az + k.bg * (m.T - k.T0) : az;
    const R ir = R(1) / m.rho;
#pragma unroll
    for (int d = 0; d < 3; ++d) m.u[d] = j[d] * ir + k.hdt * m.acc[d];
    return m;
}

// poly - 1 and frc of population a: f_eq / (w rho) - 1, F / (w rho)
template <class R, bool TH>
__device__ inline void eqf3(const Mac3<R, TH>& m, int a, R& pm1, R& frc) {
    const R uu = m.u[0] * m.u[0] + m.u[1] * m.u[1] + m.u[2] * m.u[2];
    const R ua = m.u[0] * m.acc[0] + m.u[1] * m.acc[1] + m.u[2] * m.acc[2];
    const R cu = R(c3(a, 0)) * m.u[0] + R(c3(a, 1)) * m.u[1] + R(c3(a, 2)) * m.u[2];
    const R ca = R(c3(a, 0)) * m.acc[0] + R(c3(a, 1)) * m.acc[1] + R(c3(a, 2)) * m.acc[2];
    pm1 = R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu;
    frc = R(3) * (ca - ua) + R(9) * cu * ca;
}

// base = f~ + C(f~) - w ref of every population (offsets)
template <class R, bool TH>
__device__ inline void base3(const R* df, const R* dg, const Mac3<R, TH>& m, const StageK<R>& k, R* bf, R* bg) {
#pragma unroll
    for (int a = 0; a < 19; ++a) {
        R pm1, frc;
        eqf3<R, TH>(m, a, pm1, frc);
        bf[a] = k.omkc * df[a] + w3<R>(a) * (k.kc * m.rho_p + m.rho * (k.kc * pm1 + k.kf * frc));
        if (TH) bg[a] = k.omkcg * dg[a] + k.kcg * w3<R>(a) * (m.T_p + m.T * pm1);
    }
}

// brackets phi - w ref (f) and phi - w ref_g (g) of the 18 moving
// populations of a decoded cell, written to phi[(s * 18 + a - 1) * cells + c]
template <class R, bool TH, int a>
__device__ __forceinline__ void bracket3(const StageK<R>& k, const R* df, const R* dg, const Mac3<R, TH>& m, R* phi,
                                         const int64_t cells, const int64_t c) {
    R pm1, frc;
    eqf3<R, TH>(m, a, pm1, frc);
    phi[int64_t(a - 1) * cells + c] = k.omk1 * df[a] + w3<R>(a) * (k.k1 * m.rho_p + m.rho * (k.k1 * pm1 + k.kh * frc));
    if (TH) phi[int64_t(18 + a - 1) * cells + c] = k.omk1g * dg[a] + k.k1g * w3<R>(a) * (m.T_p + m.T * pm1);
}
template <class R, bool TH, int... as>
__device__ __forceinline__ void brackets3(const StageK<R>& k, const R* df, const R* dg, const Mac3<R, TH>& m, R* phi,
                                          const int64_t cells, const int64_t c, std::integer_sequence<int, as...>) {
    (bracket3<R, TH, as + 1>(k, df, dg, m, phi, cells, c), ...);
}

template <class R, class S, bool TH>
__global__ void __launch_bounds__(256) fv3_stage(Fv3Args<R> A) {
    const int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (c >= A.cells) return;
    R df[19], dg[19];
    load3<R, S, TH>(static_cast<const S*>(A.src), A.cells, c, df, dg);
    const Mac3<R, TH> m = macro3<R, TH>(df, dg, A.k, A.az);
    brackets3<R, TH>(A.k, df, dg, m, A.phi, A.cells, c, std::make_integer_sequence<int, 18>{});
}

// bracket of population a of species s at index q along `axis` of the cell
// (i[0], i[1], i[2]); ghosts as in the 2D kernel
template <class R>
__device__ inline R phi_at(const Fv3Args<R>& A, int s, int a, int axis, int q, const int* i) {
    const int n = A.n[axis];
    int p[3] = {i[0], i[1], i[2]};
    int b = a;
    bool anti = false;
    if (q >= 0 && q < n) {
        p[axis] = q;
    } else if (!A.wall[axis]) {
        p[axis] = q < 0 ? q + n : q - n;
    } else {
        p[axis] = q < 0 ? -q - 1 : 2 * n - 1 - q;
        b = opp3(a);
        anti = s == 1 && axis == 2;
    }
    const int64_t cell = (int64_t(p[2]) * A.n[1] + p[1]) * A.n[0] + p[0];
    const R v = A.phi[int64_t(s * 18 + b - 1) * A.cells + cell];
    if (!anti) return v;
    // isothermal anti-reflection of the shifted bracket: 2 w (T_w - ref_g) - phi_inv
    return R(2) * w3<R>(a) * ((q < 0 ? A.Tb : A.Tt) - A.k.ref_g) - v;
}

// The update of cell c (all populations).
template <class R, class S, bool TH, bool CORR>
__device__ __forceinline__ void update_cell(const Fv3Args<R>& A, const int64_t c) {
    constexpr int NSP = TH ? 2 : 1;
    const int i[3] = {int(c % A.n[0]), int((c / A.n[0]) % A.n[1]), int(c / (int64_t(A.n[0]) * A.n[1]))};
    const StageK<R>& k = A.k;
    const int64_t stride[3] = {1, int64_t(A.n[0]), int64_t(A.n[0]) * A.n[1]};
    bool inner[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) inner[d] = i[d] >= 2 && i[d] + 2 < A.n[d];
    const S* own = static_cast<const S*>(CORR ? A.aux : A.src);
    const S* star = static_cast<const S*>(A.src);
    S* dst = static_cast<S*>(A.dst);
    // the cell's macroscopic state (f~n in the corrector, else the stage input)
    Mac3<R, TH> m;
    {
        R df[19], dg[19];
        load3<R, S, TH>(own, A.cells, c, df, dg);
        m = macro3<R, TH>(df, dg, k, A.az);
    }
    // population by population: base = f~ + C(f~) (corrector: (f~n + C + f~*)/2),
    // minus the flux divergence, stored at once (short live ranges)
#pragma unroll
    for (int s = 0; s < NSP; ++s)
#pragma unroll
        for (int a = 0; a < 19; ++a) {
            const int64_t e = int64_t(s * 19 + a) * A.cells + c;
            const R d = R(Store3<S>::ld(own + e));
            R pm1, frc;
            eqf3<R, TH>(m, a, pm1, frc);
            R b = s == 0 ? k.omkc * d + w3<R>(a) * (k.kc * m.rho_p + m.rho * (k.kc * pm1 + k.kf * frc))
                         : k.omkcg * d + k.kcg * w3<R>(a) * (m.T_p + m.T * pm1);
            if (CORR) b = R(0.5) * (b + R(Store3<S>::ld(star + e)));
            if (a > 0) {
                const R* pa = A.phi + int64_t(s * 18 + a - 1) * A.cells;
#pragma unroll
                for (int axis = 0; axis < 3; ++axis) {
                    const int cd = c3(a, axis);
                    if (cd == 0) continue;
                    const R* w = A.coef[axis] + int64_t(i[axis]) * 8 + (cd > 0 ? 0 : 4);
                    const int q0 = cd > 0 ? -2 : -1;
                    if (inner[axis]) {  // all four points inside: plain strided loads
#pragma unroll
                        for (int q = 0; q < 4; ++q) b -= w[q] * pa[c + (q0 + q) * stride[axis]];
                    } else {
#pragma unroll
                        for (int q = 0; q < 4; ++q) b -= w[q] * phi_at<R>(A, s, a, axis, i[axis] + q0 + q, i);
                    }
                }
            }
            Store3<S>::st(dst + e, S(b));
        }
}

template <class R, class S, bool TH, bool CORR>
__global__ void __launch_bounds__(256) fv3_update(Fv3Args<R> A) {
    const int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (c >= A.cells) return;
    update_cell<R, S, TH, CORR>(A, c);
}

// ---- tiled update ---------------------------------------------------------
// A block updates a tile of T3X x T3Y x T3Z cells.  Population by population,
// the brackets of the tile and of the halo cells its stencils reach (two
// cells beyond each face along each axis the population moves on: a cross,
// no edges or corners) are staged in LDS, so a bracket is read from the
// scratch buffer about once per tile rather than four times per axis and
// cell.  The arithmetic is that of fv3_update, in the same order.
// (tiles 8 deep in z, 1024 threads, ran at the same rate at 256^3)
constexpr int T3X = 32, T3Y = 4, T3Z = 4, T3N = T3X * T3Y * T3Z;
constexpr int T3G = 1;    // moving populations staged per barrier
// populations whose staged loads are in flight ahead of the one being
// updated: four in the predictor, two in the corrector (whose staged values
// carry f~* as well; two keep it within 128 VGPRs, see below)
template <bool CORR> constexpr int T3PD = CORR ? 2 : 4;
constexpr int T3S = 8;   // tiles per z column of the block order (see fv3_update_tiled)
constexpr int L3X = T3X + 4, L3Y = T3Y + 4, L3Z = T3Z + 4, L3N = L3X * L3Y * L3Z;
static_assert(T3Y == 4 && (T3Z == 4 || T3Z == 8),
              "one thread per y-halo cell (the four halo rows map to the tile's four); the z-halo planes "
              "map to the first four planes of the tile");
static_assert((4 * T3Y * T3Z) % 64 == 0 && (T3X * T3Y * 4) % 64 == 0, "halo-staging threads are whole waves");
static_assert(18 % T3G == 0, "groups of populations divide a species");
static_assert(T3G <= T3PD<true> && T3G <= T3PD<false>,
              "a group's staged values are all in flight before its first write");
__device__ constexpr int l3(int x, int y, int z) { return ((z + 2) * L3Y + (y + 2)) * L3X + (x + 2); }

// Source of one staged bracket: the cell it is read at, whether that is a
// wall mirror (the opposite population is read) and at which z wall the
// thermal bracket is anti-reflected.  Positions more than two cells outside
// the domain, or outside along two axes, are never read by a cell's stencil.
enum { SRC_VALID = 1, SRC_MIRROR = 2, SRC_ZLO = 4, SRC_ZHI = 8 };
struct Src3 {
    int64_t cell;
    int flags;
};

template <class R>
__device__ inline Src3 src3(const Fv3Args<R>& A, const int* g) {
    int p[3], out = 0, flags = SRC_VALID;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int q = g[d], n = A.n[d];
        if (q >= 0 && q < n) {
            p[d] = q;
            continue;
        }
        if (q < -2 || q > n + 1) return Src3{0, 0};
        ++out;
        if (!A.wall[d]) {
            p[d] = q < 0 ? q + n : q - n;
        } else {
            p[d] = q < 0 ? -q - 1 : 2 * n - 1 - q;
            flags |= SRC_MIRROR;
            if (d == 2) flags |= q < 0 ? SRC_ZLO : SRC_ZHI;
        }
    }
    if (out > 1) return Src3{0, 0};
    return Src3{(int64_t(p[2]) * A.n[1] + p[1]) * A.n[0] + p[0], flags};
}

// bracket of population a of species s at a staged source, as read (the
// thermal anti-reflection at a z wall is applied when it is staged, so that
// the load can stay in flight until then).  Positions that no stencil reads
// point at cell 0 and are loaded all the same: branch-free loads keep the
// compiler's count of loads in flight exact.
template <class R, int s, int a>
__device__ inline R fetch3(const Fv3Args<R>& A, const Src3& q) {
    const int b = (q.flags & SRC_MIRROR) ? opp3(a) : a;
    return A.phi[int64_t(s * 18 + b - 1) * A.cells + q.cell];
}

// the staged value of a fetched bracket (as phi_at): at a z wall the
// thermal bracket is anti-reflected, 2 w (T_w - ref_g) - phi_inv, with
// zw = 2 (T_w - ref_g) of the position (the same exact product)
template <class R, int s, int a>
__device__ inline R staged3(const Src3& q, const R zw, const R v) {
    if (s == 0 || !(q.flags & (SRC_ZLO | SRC_ZHI))) return v;
    return w3<R>(a) * zw - v;
}

// the values one thread stages for population (s, a): its own position and
// one halo cell along each axis the population moves on
template <class R>
struct Stage3 {
    R own, x, y, z;
    R star;   // Heun corrector: f~* of the population at the own cell
};
template <class R, int s, int a>
__device__ inline Stage3<R> fetch_pop(const Fv3Args<R>& A, const Src3* q, const bool xh, const bool zh,
                                      const int64_t c, const bool corr) {
    Stage3<R> v;
    v.own = fetch3<R, s, a>(A, q[0]);
    // (the stage input of the corrector is f~*, stored in the state's own precision R)
    v.star = corr ? static_cast<const R*>(A.src)[int64_t(s * 19 + a) * A.cells + c] : R(0);
    v.x = c3(a, 0) && xh ? fetch3<R, s, a>(A, q[1]) : R(0);
    v.y = c3(a, 1) ? fetch3<R, s, a>(A, q[2]) : R(0);
    v.z = c3(a, 2) && zh ? fetch3<R, s, a>(A, q[3]) : R(0);
    return v;
}

// the first T3PD moving populations' staged values
template <class R, bool TH, bool CORR, int p>
__device__ __forceinline__ void fetch_first(const Fv3Args<R>& A, const Src3* q, const bool xh, const bool zh,
                                            const int64_t c, Stage3<R>* v) {
    if constexpr (p < T3PD<CORR> && p < 18 * (TH ? 2 : 1)) {
        v[p] = fetch_pop<R, p / 18, p % 18 + 1>(A, q, xh, zh, c, CORR);
        fetch_first<R, TH, CORR, p + 1>(A, q, xh, zh, c, v);
    }
}

// a value the whole wave holds alike, kept in a scalar register
__device__ inline float wave_uniform(const float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
}
__device__ inline double wave_uniform(const double x) {
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(u)), hi = __builtin_amdgcn_readfirstlane(uint32_t(u >> 32));
    return __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
}
static_assert((T3X * T3Y) % 64 == 0, "a wave lies in one z plane of the tile");

// Everything a thread of the tiled kernel carries from population to population.
template <class R, bool TH>
struct Tile3 {
    Src3 q[4];        // staged positions: own, x halo, y halo, z halo
    int li[4];        // their LDS indices
    bool xh, zh;      // stages an x-halo cell / a z-halo cell (whole waves)
    bool mine;        // owns a cell of the domain
    R zw[4];          // 2 (T_w - ref_g) at the z wall a staged position mirrors (else 0)
    int64_t c;        // own cell (cell 0 for threads outside the domain)
    R bf[19], bg[19]; // own record, then its collision bases, then the new values
    R w[3][8];        // flux weights of the own position along each axis
};

// collision bases of the own cell in place of its record (Heun corrector:
// (f~n + C(f~n) + f~*) / 2), as in fv3_update.  The new values are stored
// only after every population's flux: vector loads and stores share one
// completion counter, so a store issued between a staged load and its use
// would make that use wait for the store as well.
template <class R, class S, bool TH, bool CORR, int s, int a>
__device__ __forceinline__ void tile_base(const Fv3Args<R>& A, Tile3<R, TH>& T, const Mac3<R, TH>& m) {
    const StageK<R>& k = A.k;
    R pm1, frc;
    eqf3<R, TH>(m, a, pm1, frc);
    R& d = s == 0 ? T.bf[a] : T.bg[a];
    R b = s == 0 ? k.omkc * d + w3<R>(a) * (k.kc * m.rho_p + m.rho * (k.kc * pm1 + k.kf * frc))
                 : k.omkcg * d + k.kcg * w3<R>(a) * (m.T_p + m.T * pm1);
    // the corrector's f~* term of a moving population is added when the
    // population is staged (its load travels with the staged brackets)
    if (CORR && a == 0)
        b = R(0.5) * (b + R(Store3<S>::ld(static_cast<const S*>(A.src) + int64_t(s * 19 + a) * A.cells + T.c)));
    d = b;
}
template <class R, class S, bool TH, bool CORR, int s, int... as>
__device__ __forceinline__ void tile_bases(const Fv3Args<R>& A, Tile3<R, TH>& T, const Mac3<R, TH>& m,
                                           std::integer_sequence<int, as...>) {
    (tile_base<R, S, TH, CORR, s, as>(A, T, m), ...);
}

// the new values (indices fixed at compile time, so the arrays stay in registers)
template <class R, class S, bool TH, int s, int... as>
__device__ __forceinline__ void tile_stores(const Fv3Args<R>& A, const Tile3<R, TH>& T,
                                            std::integer_sequence<int, as...>) {
    S* dst = static_cast<S*>(A.dst);
    ((Store3<S>::st(dst + int64_t(s * 19 + as) * A.cells + T.c, S(s == 0 ? T.bf[as] : T.bg[as]))), ...);
}

// Moving populations are staged T3G at a time (one barrier per group):
// write the group's staged values, synchronise, put the loads of later
// populations in flight, then apply the group's fluxes.
template <class R, bool TH, bool CORR, int p>
__device__ __forceinline__ void tile_write(const Fv3Args<R>& A, R (*lds)[T3G][L3N], Tile3<R, TH>& T,
                                           const Stage3<R>* v) {
    constexpr int s = p / 18, a = p % 18 + 1;
    R* L = lds[(p / T3G) & 1][p % T3G];
    const Stage3<R>& u = v[p % T3PD<CORR>];
    L[T.li[0]] = staged3<R, s, a>(T.q[0], T.zw[0], u.own);
    if (c3(a, 0) && T.xh) L[T.li[1]] = staged3<R, s, a>(T.q[1], T.zw[1], u.x);
    if (c3(a, 1)) L[T.li[2]] = staged3<R, s, a>(T.q[2], T.zw[2], u.y);
    if (c3(a, 2) && T.zh) L[T.li[3]] = staged3<R, s, a>(T.q[3], T.zw[3], u.z);
    if (CORR) {
        R& b = s == 0 ? T.bf[a] : T.bg[a];
        b = R(0.5) * (b + u.star);
    }
}

template <class R, bool TH, bool CORR, int p>
__device__ __forceinline__ void tile_prefetch(const Fv3Args<R>& A, const Tile3<R, TH>& T, Stage3<R>* v) {
    if constexpr (p + T3PD<CORR> < 18 * (TH ? 2 : 1)) {
        constexpr int p2 = p + T3PD<CORR>;
        v[p % T3PD<CORR>] = fetch_pop<R, p2 / 18, p2 % 18 + 1>(A, T.q, T.xh, T.zh, T.c, CORR);
    }
}

template <class R, class S, bool TH, bool CORR, int p>
__device__ __forceinline__ void tile_update(const Fv3Args<R>& A, R (*lds)[T3G][L3N], Tile3<R, TH>& T) {
    constexpr int s = p / 18, a = p % 18 + 1;
    const R* L = lds[(p / T3G) & 1][p % T3G];
    R& b = s == 0 ? T.bf[a] : T.bg[a];
#pragma unroll
    for (int axis = 0; axis < 3; ++axis) {
        const int cd = c3(a, axis);
        if (cd == 0) continue;
        const R* wq = T.w[axis] + (cd > 0 ? 0 : 4);
        const int q0 = cd > 0 ? -2 : -1;
        const int st = axis == 0 ? 1 : axis == 1 ? L3X : L3X * L3Y;
#pragma unroll
        for (int j = 0; j < 4; ++j) b -= wq[j] * L[T.li[0] + (q0 + j) * st];
    }
    // the value is final here: keep the compiler from sinking this
    // population's arithmetic (and its LDS values) down to the stores
    asm volatile("" : "+v"(b));
}

template <class R, class S, bool TH, bool CORR, int g, int... js>
__device__ __forceinline__ void tile_group(const Fv3Args<R>& A, R (*lds)[T3G][L3N], Tile3<R, TH>& T,
                                           Stage3<R>* v, std::integer_sequence<int, js...>) {
    (tile_write<R, TH, CORR, g * T3G + js>(A, lds, T, v), ...);
    __syncthreads();
    (tile_prefetch<R, TH, CORR, g * T3G + js>(A, T, v), ...);
    (tile_update<R, S, TH, CORR, g * T3G + js>(A, lds, T), ...);
}

template <class R, class S, bool TH, bool CORR, int... gs>
__device__ __forceinline__ void tile_groups(const Fv3Args<R>& A, R (*lds)[T3G][L3N], Tile3<R, TH>& T,
                                            Stage3<R>* v, std::integer_sequence<int, gs...>) {
    (tile_group<R, S, TH, CORR, gs>(A, lds, T, v, std::make_integer_sequence<int, T3G>{}), ...);
}

// The tile's new state and, when phi_next is set, the brackets of that state
// for the next stage (the stage kernel's arithmetic on the same values), so
// that the next pass needs no stage kernel.
// FP32 passes are held to 128 VGPRs, two blocks per CU, without spills
// (one block per CU with more registers was the slower of the two).
template <class R, bool CORR>
constexpr int T3_WAVES_PER_SIMD = sizeof(R) == 4 ? 4 : 1;

template <class R, class S, bool TH, bool CORR>
__global__ void __launch_bounds__(T3N, (T3_WAVES_PER_SIMD<R, CORR>)) fv3_update_tiled(Fv3Args<R> A) {
    static_assert(std::is_same<R, S>::value, "3D states are stored in their arithmetic type");
    __shared__ R lds[2][T3G][L3N];
    const int t = threadIdx.x;
    const int tx = t % T3X, ty = (t / T3X) % T3Y, tz = t / (T3X * T3Y);
    // one tile per block.  Blocks are dealt to the eight XCDs round robin;
    // block b takes unit (b % 8) * per + b / 8 of the tiles ordered z fastest
    // within columns of T3S tiles, then x, then y, then column, so that the
    // blocks an XCD runs at once are z and x neighbours and meet in its L2 on
    // the halo planes and columns they share
    const int nxt = (A.n[0] + T3X - 1) / T3X, nyt = (A.n[1] + T3Y - 1) / T3Y;
    const int nzt = (A.n[2] + T3Z - 1) / T3Z, ncol = (nzt + T3S - 1) / T3S;
    const int per = (T3S * nxt * nyt * ncol + 7) / 8;
    const int u = int(blockIdx.x % 8) * per + int(blockIdx.x / 8);
    if (u >= T3S * nxt * nyt * ncol) return;   // the whole block
    const int zt = (u / (T3S * nxt * nyt)) * T3S + u % T3S;
    if (zt >= nzt) return;                     // a short last column: the whole block
    const int o[3] = {((u / T3S) % nxt) * T3X, ((u / (T3S * nxt)) % nyt) * T3Y, zt * T3Z};
    const int i[3] = {o[0] + tx, o[1] + ty, o[2] + tz};
    Tile3<R, TH> T;
    T.mine = i[0] < A.n[0] && i[1] < A.n[1] && i[2] < A.n[2];
    // the four positions this thread stages: its own, an x-halo cell
    // (wave 0 only), a y-halo cell and a z-halo cell
    T.q[0] = src3(A, i);
    T.li[0] = l3(tx, ty, tz);
    T.xh = __builtin_amdgcn_readfirstlane(t) < 4 * T3Y * T3Z;   // uniform branches
    T.zh = __builtin_amdgcn_readfirstlane(t) < 4 * T3X * T3Y;
    {
        const int h = t & 3, hy = (t >> 2) % T3Y, hz = ((t >> 2) / T3Y) % T3Z;
        const int rx = h < 2 ? h - 2 : T3X + h - 2;
        const int g[3] = {o[0] + rx, o[1] + hy, o[2] + hz};
        T.q[1] = T.xh ? src3(A, g) : Src3{0, 0};
        T.li[1] = l3(rx, hy, hz);
    }
    {
        const int ry = ty < 2 ? ty - 2 : T3Y + ty - 2;
        const int g[3] = {i[0], o[1] + ry, i[2]};
        T.q[2] = src3(A, g);
        T.li[2] = l3(tx, ry, tz);
    }
    {
        const int rz = tz < 2 ? tz - 2 : T3Z + (tz & 3) - 2;   // threads of the first four planes
        const int g[3] = {i[0], i[1], o[2] + rz};
        T.q[3] = src3(A, g);
        T.li[3] = l3(tx, ty, rz);
    }
    {
        const R zlo = R(2) * (A.Tb - A.k.ref_g), zhi = R(2) * (A.Tt - A.k.ref_g);
#pragma unroll
        for (int k = 0; k < 4; ++k)
            T.zw[k] = (T.q[k].flags & SRC_ZLO) ? zlo : (T.q[k].flags & SRC_ZHI) ? zhi : R(0);
    }
    T.c = T.mine ? (int64_t(i[2]) * A.n[1] + i[1]) * A.n[0] + i[0] : 0;
    Stage3<R> v[T3PD<CORR>];
    fetch_first<R, TH, CORR, 0>(A, T.q, T.xh, T.zh, T.c, v);
    // own record, macroscopic state and the flux weights of the cell along
    // each axis (threads outside the domain read cell 0 and the last
    // weights, without branches, and store nothing)
    load3<R, S, TH>(static_cast<const S*>(CORR ? A.aux : A.src), A.cells, T.c, T.bf, T.bg);
    if constexpr (!TH)
#pragma unroll
        for (int a = 0; a < 19; ++a) T.bg[a] = R(0);
    {
        const Mac3<R, TH> m = macro3<R, TH>(T.bf, T.bg, A.k, A.az);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int64_t id = i[d] < A.n[d] ? i[d] : A.n[d] - 1;
#pragma unroll
            for (int j = 0; j < 8; ++j)   // a wave shares its z plane: z weights are wave-uniform
                T.w[d][j] = d == 2 ? wave_uniform(A.coef[d][id * 8 + j]) : A.coef[d][id * 8 + j];
        }
        tile_bases<R, S, TH, CORR, 0>(A, T, m, std::make_integer_sequence<int, 19>{});
        if constexpr (TH) tile_bases<R, S, TH, CORR, 1>(A, T, m, std::make_integer_sequence<int, 19>{});
    }
    constexpr int NG = 18 * (TH ? 2 : 1) / T3G;
    tile_groups<R, S, TH, CORR>(A, lds, T, v, std::make_integer_sequence<int, NG>{});
    if (T.mine) {
        tile_stores<R, S, TH, 0>(A, T, std::make_integer_sequence<int, 19>{});
        if constexpr (TH) tile_stores<R, S, TH, 1>(A, T, std::make_integer_sequence<int, 19>{});
        if (A.phi_next) {
            const Mac3<R, TH> m = macro3<R, TH>(T.bf, T.bg, A.k, A.az);
            brackets3<R, TH>(A.k, T.bf, T.bg, m, A.phi_next, A.cells, T.c, std::make_integer_sequence<int, 18>{});
        }
    }
}

template <class R, class S, bool TH, bool CORR>
static void launch_update3(const Fv3Args<R>& A, hipStream_t st) {
    if (A.gather) {
        const dim3 grid(unsigned((A.cells + 255) / 256)), block(256);
        hipLaunchKernelGGL((fv3_update<R, S, TH, CORR>), grid, block, 0, st, A);
    } else {
        const int nxt = (A.n[0] + T3X - 1) / T3X, nyt = (A.n[1] + T3Y - 1) / T3Y;
        const int ncol = ((A.n[2] + T3Z - 1) / T3Z + T3S - 1) / T3S;
        const dim3 grid(unsigned(8 * ((T3S * nxt * nyt * ncol + 7) / 8)));   // as the kernel's unit count
        hipLaunchKernelGGL((fv3_update_tiled<R, S, TH, CORR>), grid, dim3(T3N), 0, st, A);
    }
}

template <class R, class S>
static hipError_t fv3_typed(bool thermal, bool corrector, const void* args, hipStream_t st) {
    const Fv3Args<R>& A = *static_cast<const Fv3Args<R>*>(args);
    const dim3 grid(unsigned((A.cells + 255) / 256)), block(256);
    if (thermal) {
        if (A.stage) hipLaunchKernelGGL((fv3_stage<R, S, true>), grid, block, 0, st, A);
        if (corrector) launch_update3<R, S, true, true>(A, st);
        else launch_update3<R, S, true, false>(A, st);
    } else {
        if (A.stage) hipLaunchKernelGGL((fv3_stage<R, S, false>), grid, block, 0, st, A);
        if (corrector) launch_update3<R, S, false, true>(A, st);
        else launch_update3<R, S, false, false>(A, st);
    }
    return hipGetLastError();
}

hipError_t launch_fv3(int storage, bool thermal, bool corrector, const void* args, hipStream_t s) {
    switch (storage) {
        case ST_F64: return fv3_typed<double, double>(thermal, corrector, args, s);
        case ST_F32: return fv3_typed<float, float>(thermal, corrector, args, s);
    }
    return hipErrorInvalidValue;
}

size_t fv3_args_bytes(int storage) { return storage == ST_F64 ? sizeof(Fv3Args<double>) : sizeof(Fv3Args<float>); }

// ---- initial state, moments, populations and FP64 diagnostics ------------

template <class S>
__device__ inline double ld3(const Aux3Args& A, int s, int a, int64_t c) {
    const S* st = static_cast<const S*>(A.state);
    const double x = double(Store3<S>::ld(st + int64_t(s * 19 + a) * A.cells + c));
    return Store3<S>::offset ? x + w3<double>(a) * (s ? A.ref_g : A.ref_f) : x;
}

__device__ inline void macro3d(const Aux3Args& A, const double* f, const double* g, double* rho, double* u,
                               double* T, double* acc) {
    double r = 0, j[3] = {0, 0, 0}, t = 0;
    for (int a = 0; a < 19; ++a) {
        r += f[a];
        for (int d = 0; d < 3; ++d) j[d] += c3(a, d) * f[a];
        if (A.thermal) t += g[a];
    }
    acc[0] = A.a[0];
    acc[1] = A.a[1];
    acc[2] = A.a[2] + (A.thermal ? A.bg * (t - A.T0) : 0.0);
    for (int d = 0; d < 3; ++d) u[d] = j[d] / r + A.hdt * acc[d];
    *rho = r;
    *T = t;
}

template <class S>
__global__ void init3_kernel(Aux3Args A, const double* rho, const double* ux, const double* uy, const double* uz,
                             const double* T) {
    const int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (c >= A.cells) return;
    S* st = static_cast<S*>(A.state);
    const double u[3] = {ux[c], uy[c], uz[c]};
    const double Tc = A.thermal ? T[c] : 0.0;
    const double acc[3] = {A.a[0], A.a[1], A.a[2] + (A.thermal ? A.bg * (Tc - A.T0) : 0.0)};
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2], ua = u[0] * acc[0] + u[1] * acc[1] + u[2] * acc[2];
    for (int a = 0; a < 19; ++a) {
        const double cu = c3(a, 0) * u[0] + c3(a, 1) * u[1] + c3(a, 2) * u[2];
        const double ca = c3(a, 0) * acc[0] + c3(a, 1) * acc[1] + c3(a, 2) * acc[2];
        const double feq = w3<double>(a) * rho[c] * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * uu);
        const double F = w3<double>(a) * rho[c] * (3 * (ca - ua) + 9 * cu * ca);
        double v = feq - A.hdt * F;
        if (Store3<S>::offset) v -= w3<double>(a) * A.ref_f;
        Store3<S>::st(st + int64_t(a) * A.cells + c, S(v));
        if (A.thermal) {
            double gv = w3<double>(a) * Tc * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * uu);
            if (Store3<S>::offset) gv -= w3<double>(a) * A.ref_g;
            Store3<S>::st(st + int64_t(19 + a) * A.cells + c, S(gv));
        }
    }
}

template <class S>
__global__ void moments3_kernel(Aux3Args A, double* rho, double* ux, double* uy, double* uz, double* T,
                                double* pops) {
    const int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (c >= A.cells) return;
    double f[19], g[19];
    for (int a = 0; a < 19; ++a) {
        f[a] = ld3<S>(A, 0, a, c);
        g[a] = A.thermal ? ld3<S>(A, 1, a, c) : 0.0;
    }
    if (pops) {
        for (int a = 0; a < 19; ++a) {
            pops[int64_t(a) * A.cells + c] = f[a];
            if (A.thermal) pops[int64_t(19 + a) * A.cells + c] = g[a];
        }
        return;
    }
    double r, u[3], t, acc[3];
    macro3d(A, f, g, &r, u, &t, acc);
    rho[c] = r;
    ux[c] = u[0];
    uy[c] = u[1];
    uz[c] = u[2];
    T[c] = t;
}

__device__ inline double bsum3(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < int(blockDim.x >> 6); ++w) r += sh[w];
    return r;
}

template <class S>
__global__ void __launch_bounds__(256) diag3_kernel(Diag3Args D, double* partial) {
    __shared__ double sh[4];
    const Aux3Args& A = D.a;
    const int nx = A.n[0], ny = A.n[1], nz = A.n[2];
    double acc[D_COUNT];
    for (int q = 0; q < D_COUNT; ++q) acc[q] = 0.0;
    auto cellT = [&](int64_t c) {
        double t = 0.0;
        for (int a = 0; a < 19; ++a) t += ld3<S>(A, 1, a, c);
        return t;
    };
    for (int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x; c < A.cells; c += int64_t(gridDim.x) * 256) {
        const int i = int(c % nx), j = int((c / nx) % ny), l = int(c / (int64_t(nx) * ny));
        const double v = A.dx[i] * A.dy[j] * A.dz[l];
        double f[19], g[19];
        for (int a = 0; a < 19; ++a) {
            f[a] = ld3<S>(A, 0, a, c);
            g[a] = A.thermal ? ld3<S>(A, 1, a, c) : 0.0;
            if (!isfinite(f[a]) || !isfinite(g[a])) acc[D_BAD] = 1.0;
        }
        double r, u[3], t, ac[3];
        macro3d(A, f, g, &r, u, &t, ac);
        acc[D_MASS] += v * r;
        acc[D_EKIN] += v * 0.5 * r * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        acc[D_ETH] += v * t;
        acc[D_UT] += v * u[2] * t;
        acc[D_VOL] += v;
        if (D.walls && (l == 0 || l == nz - 1)) {
            const int l2 = l == 0 ? 1 : nz - 2;
            const double T2 = cellT((int64_t(l2) * ny + j) * nx + i);
            const double w = A.dx[i] * A.dy[j] * D.inv_area;
            if (l == 0) acc[D_NUB] += w * D.nu_scale * (D.nub[0] * D.Tb + D.nub[1] * t + D.nub[2] * T2);
            if (l == nz - 1) acc[D_NUT] += w * D.nu_scale * (D.nut[0] * D.Tt + D.nut[1] * t + D.nut[2] * T2);
        }
    }
    for (int q = 0; q < D_COUNT; ++q) {
        const double r = bsum3(acc[q], sh);
        if (threadIdx.x == 0) partial[int64_t(blockIdx.x) * D_COUNT + q] = r;
    }
}

__global__ void __launch_bounds__(256) diag3_fold(const double* partial, int nblocks, double* out) {
    __shared__ double sh[4];
    for (int q = 0; q < D_COUNT; ++q) {
        double acc = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += 256) {
            const double p = partial[int64_t(b) * D_COUNT + q];
            acc = (q == D_BAD) ? fmax(acc, p) : acc + p;
        }
        double r = bsum3(acc, sh);
        if (q == D_BAD) r = r > 0.0 ? 1.0 : 0.0;
        if (threadIdx.x == 0) out[q] = r;
    }
}

template <class S>
static hipError_t aux3_typed(int what, const Aux3Args& a, const double* const* in, double* const* out,
                             hipStream_t s) {
    const dim3 grid(unsigned((a.cells + 255) / 256)), block(256);
    switch (what) {
        case 0: hipLaunchKernelGGL(init3_kernel<S>, grid, block, 0, s, a, in[0], in[1], in[2], in[3], in[4]); break;
        case 1:
            hipLaunchKernelGGL(moments3_kernel<S>, grid, block, 0, s, a, out[0], out[1], out[2], out[3], out[4],
                               nullptr);
            break;
        case 2:
            hipLaunchKernelGGL(moments3_kernel<S>, grid, block, 0, s, a, nullptr, nullptr, nullptr, nullptr, nullptr,
                               out[0]);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_aux3(int storage, int what, const Aux3Args& a, const double* const* in, double* const* out,
                       hipStream_t s) {
    switch (storage) {
        case ST_F64: return aux3_typed<double>(what, a, in, out, s);
        case ST_F32: return aux3_typed<float>(what, a, in, out, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_diag3(int storage, const Diag3Args& d, double* partial, double* out, hipStream_t s) {
    const int64_t want = (d.a.cells + 255) / 256;
    const int nb = int(want < DIAG_BLOCKS ? want : DIAG_BLOCKS);
    switch (storage) {
        case ST_F64: hipLaunchKernelGGL(diag3_kernel<double>, dim3(nb), dim3(256), 0, s, d, partial); break;
        case ST_F32: hipLaunchKernelGGL(diag3_kernel<float>, dim3(nb), dim3(256), 0, s, d, partial); break;
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(diag3_fold, dim3(1), dim3(256), 0, s, partial, nb, out);
    return hipGetLastError();
}

}  // namespace lbk
