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
// fv3_update, one thread per cell reading every stencil point from the
// scratch buffer, computes the same operations in the same order.  The
// two-kernel form moves the brackets through HBM once more than a fused
// kernel would.
//
// Storage: FP64 (parity path) or FP32 offsets p - w_a ref, populations as
// (s * 19 + a) * cells + cell, x fastest.
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

template <class R, class S, bool TH>
__global__ void __launch_bounds__(256) fv3_stage(Fv3Args<R> A) {
    const int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (c >= A.cells) return;
    R df[19], dg[19];
    load3<R, S, TH>(static_cast<const S*>(A.src), A.cells, c, df, dg);
    const Mac3<R, TH> m = macro3<R, TH>(df, dg, A.k, A.az);
    const StageK<R>& k = A.k;
#pragma unroll
    for (int a = 1; a < 19; ++a) {
        R pm1, frc;
        eqf3<R, TH>(m, a, pm1, frc);
        // phi - w ref (f) and phi - w ref_g (g)
        A.phi[int64_t(a - 1) * A.cells + c] =
            k.omk1 * df[a] + w3<R>(a) * (k.k1 * m.rho_p + m.rho * (k.k1 * pm1 + k.kh * frc));
        if (TH)
            A.phi[int64_t(18 + a - 1) * A.cells + c] = k.omk1g * dg[a] + k.k1g * w3<R>(a) * (m.T_p + m.T * pm1);
    }
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
constexpr int T3X = 32, T3Y = 4, T3Z = 4, T3N = T3X * T3Y * T3Z;
constexpr int T3PD = 3;   // populations whose staged loads are in flight ahead of the one being updated
constexpr int L3X = T3X + 4, L3Y = T3Y + 4, L3Z = T3Z + 4, L3N = L3X * L3Y * L3Z;
static_assert(T3Y == 4 && T3Z == 4, "one thread per halo cell: the four halo rows / planes map to the tile's four");
static_assert(4 * T3Y * T3Z <= T3N, "x halo cells fit the block");
__device__ constexpr int l3(int x, int y, int z) { return ((z + 2) * L3Y + (y + 2)) * L3X + (x + 2); }

// Source of one staged bracket: the cell it is read at, whether that is a
// wall mirror (the opposite population is read) and at which z wall the
// thermal bracket is anti-reflected.  Positions more than two cells outside
// the domain, or outside along two axes, are never read by a cell's stencil
// and are not loaded.
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

// bracket of population a of species s at a staged source (as phi_at)
template <class R, int s, int a>
__device__ inline R fetch3(const Fv3Args<R>& A, const Src3& q) {
    if (!(q.flags & SRC_VALID)) return R(0);
    const int b = (q.flags & SRC_MIRROR) ? opp3(a) : a;
    const R v = A.phi[int64_t(s * 18 + b - 1) * A.cells + q.cell];
    if (s == 0 || !(q.flags & (SRC_ZLO | SRC_ZHI))) return v;
    return R(2) * w3<R>(a) * (((q.flags & SRC_ZLO) ? A.Tb : A.Tt) - A.k.ref_g) - v;
}

// the staged values one thread contributes for population (s, a): its own
// position and one halo cell along each axis the population moves on
template <class R>
struct Stage3 {
    R own, x, y, z;
};
template <class R, int s, int a>
__device__ inline Stage3<R> fetch_pop(const Fv3Args<R>& A, const Src3* q) {
    Stage3<R> v;
    v.own = fetch3<R, s, a>(A, q[0]);
    v.x = c3(a, 0) ? fetch3<R, s, a>(A, q[1]) : R(0);
    v.y = c3(a, 1) ? fetch3<R, s, a>(A, q[2]) : R(0);
    v.z = c3(a, 2) ? fetch3<R, s, a>(A, q[3]) : R(0);
    return v;
}

// the first T3PD moving populations' staged values
template <class R, bool TH, int p>
__device__ __forceinline__ void fetch_first(const Fv3Args<R>& A, const Src3* q, Stage3<R>* v) {
    if constexpr (p < T3PD && p < 18 * (TH ? 2 : 1)) {
        v[p] = fetch_pop<R, p / 18, p % 18 + 1>(A, q);
        fetch_first<R, TH, p + 1>(A, q, v);
    }
}

template <class R, class S, bool TH, bool CORR, int s, int a>
__device__ __forceinline__ void tiled_pop(const Fv3Args<R>& A, R (*lds)[L3N], const Src3* q, const int* li,
                                          const bool xh, Stage3<R>* v, const bool mine, const int64_t c,
                                          const R* df, const R* dg, const Mac3<R, TH>& m, const R (*w)[8]) {
    constexpr int NSP = TH ? 2 : 1;
    const StageK<R>& k = A.k;
    const int64_t e = int64_t(s * 19 + a) * A.cells + c;
    R pm1, frc;
    eqf3<R, TH>(m, a, pm1, frc);
    const R d = s == 0 ? df[a] : dg[a];
    R b = s == 0 ? k.omkc * d + w3<R>(a) * (k.kc * m.rho_p + m.rho * (k.kc * pm1 + k.kf * frc))
                 : k.omkcg * d + k.kcg * w3<R>(a) * (m.T_p + m.T * pm1);
    if (CORR && mine) b = R(0.5) * (b + R(Store3<S>::ld(static_cast<const S*>(A.src) + e)));
    if (a > 0) {
        constexpr int p = s * 18 + a - 1;   // moving population 0 .. 18 NSP - 1
        R* L = lds[p & 1];
        Stage3<R>& u = v[p % T3PD];
        L[li[0]] = u.own;
        if (c3(a, 0) && xh) L[li[1]] = u.x;
        if (c3(a, 1)) L[li[2]] = u.y;
        if (c3(a, 2)) L[li[3]] = u.z;
        __syncthreads();
        // later populations' loads are in flight during this one's flux
        if constexpr (p + T3PD < 18 * NSP) {
            constexpr int s2 = (p + T3PD) / 18, a2 = (p + T3PD) % 18 + 1;
            u = fetch_pop<R, s2, a2>(A, q);
        }
#pragma unroll
        for (int axis = 0; axis < 3; ++axis) {
            const int cd = c3(a, axis);
            if (cd == 0) continue;
            const R* wq = w[axis] + (cd > 0 ? 0 : 4);
            const int q0 = cd > 0 ? -2 : -1;
            const int st = axis == 0 ? 1 : axis == 1 ? L3X : L3X * L3Y;
#pragma unroll
            for (int j = 0; j < 4; ++j) b -= wq[j] * L[li[0] + (q0 + j) * st];
        }
    }
    if (mine) Store3<S>::st(static_cast<S*>(A.dst) + e, S(b));
}

template <class R, class S, bool TH, bool CORR, int s, int... as>
__device__ __forceinline__ void tiled_species(const Fv3Args<R>& A, R (*lds)[L3N], const Src3* q, const int* li,
                                              const bool xh, Stage3<R>* v, const bool mine, const int64_t c,
                                              const R* df, const R* dg, const Mac3<R, TH>& m, const R (*w)[8],
                                              std::integer_sequence<int, as...>) {
    (tiled_pop<R, S, TH, CORR, s, as>(A, lds, q, li, xh, v, mine, c, df, dg, m, w), ...);
}

template <class R, class S, bool TH, bool CORR>
__global__ void __launch_bounds__(T3N) fv3_update_tiled(Fv3Args<R> A) {
    __shared__ R lds[2][L3N];
    const int t = threadIdx.x;
    const int tx = t % T3X, ty = (t / T3X) % T3Y, tz = t / (T3X * T3Y);
    const int o[3] = {int(blockIdx.x) * T3X, int(blockIdx.y) * T3Y, int(blockIdx.z) * T3Z};
    const int i[3] = {o[0] + tx, o[1] + ty, o[2] + tz};
    const bool mine = i[0] < A.n[0] && i[1] < A.n[1] && i[2] < A.n[2];
    // the four positions this thread stages: its own, an x-halo cell
    // (threads 0 .. 4 T3Y T3Z - 1), a y-halo cell and a z-halo cell
    Src3 q[4];
    int li[4];
    q[0] = src3(A, i);
    li[0] = l3(tx, ty, tz);
    const bool xh = t < 4 * T3Y * T3Z;
    {
        const int h = t & 3, hy = (t >> 2) & 3, hz = (t >> 4) & 3;
        const int rx = h < 2 ? h - 2 : T3X + h - 2;
        const int g[3] = {o[0] + rx, o[1] + hy, o[2] + hz};
        q[1] = xh ? src3(A, g) : Src3{0, 0};
        li[1] = l3(rx, hy, hz);
    }
    {
        const int ry = ty < 2 ? ty - 2 : T3Y + ty - 2;
        const int g[3] = {i[0], o[1] + ry, i[2]};
        q[2] = src3(A, g);
        li[2] = l3(tx, ry, tz);
    }
    {
        const int rz = tz < 2 ? tz - 2 : T3Z + tz - 2;
        const int g[3] = {i[0], i[1], o[2] + rz};
        q[3] = src3(A, g);
        li[3] = l3(tx, ty, rz);
    }
    Stage3<R> v[T3PD];
    fetch_first<R, TH, 0>(A, q, v);
    // own record (f~n in the corrector, else the stage input), macroscopic
    // state and the flux weights of the cell along each axis
    const int64_t c = mine ? (int64_t(i[2]) * A.n[1] + i[1]) * A.n[0] + i[0] : 0;
    R df[19], dg[19], w[3][8];
    Mac3<R, TH> m{};
    if (mine) {
        load3<R, S, TH>(static_cast<const S*>(CORR ? A.aux : A.src), A.cells, c, df, dg);
        m = macro3<R, TH>(df, dg, A.k, A.az);
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int j = 0; j < 8; ++j) w[d][j] = A.coef[d][int64_t(i[d]) * 8 + j];
    } else {
#pragma unroll
        for (int a = 0; a < 19; ++a) df[a] = dg[a] = R(0);
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int j = 0; j < 8; ++j) w[d][j] = R(0);
        m.rho = R(1);
    }
    tiled_species<R, S, TH, CORR, 0>(A, lds, q, li, xh, v, mine, c, df, dg, m, w,
                                     std::make_integer_sequence<int, 19>{});
    if constexpr (TH)
        tiled_species<R, S, TH, CORR, 1>(A, lds, q, li, xh, v, mine, c, df, dg, m, w,
                                         std::make_integer_sequence<int, 19>{});
}

template <class R, class S, bool TH, bool CORR>
static void launch_update3(const Fv3Args<R>& A, hipStream_t st) {
    if (A.gather) {
        const dim3 grid(unsigned((A.cells + 255) / 256)), block(256);
        hipLaunchKernelGGL((fv3_update<R, S, TH, CORR>), grid, block, 0, st, A);
    } else {
        const dim3 grid(unsigned((A.n[0] + T3X - 1) / T3X), unsigned((A.n[1] + T3Y - 1) / T3Y),
                        unsigned((A.n[2] + T3Z - 1) / T3Z));
        hipLaunchKernelGGL((fv3_update_tiled<R, S, TH, CORR>), grid, dim3(T3N), 0, st, A);
    }
}

template <class R, class S>
static hipError_t fv3_typed(bool thermal, bool corrector, const void* args, hipStream_t st) {
    const Fv3Args<R>& A = *static_cast<const Fv3Args<R>*>(args);
    const dim3 grid(unsigned((A.cells + 255) / 256)), block(256);
    if (thermal) {
        hipLaunchKernelGGL((fv3_stage<R, S, true>), grid, block, 0, st, A);
        if (corrector) launch_update3<R, S, true, true>(A, st);
        else launch_update3<R, S, true, false>(A, st);
    } else {
        hipLaunchKernelGGL((fv3_stage<R, S, false>), grid, block, 0, st, A);
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
