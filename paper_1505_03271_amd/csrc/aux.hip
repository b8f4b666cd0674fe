// Initial state, field export and FP64 diagnostics of liblb.
//
// All arithmetic here is double precision: the stored words are decoded
// exactly (every storage format widens exactly to double) and the moments
// follow the relations of arXiv:1505.03271 sec. 2.1 and "Force term"
// (rho = sum f~, u = sum c f~ / rho + dt/2 a) and sec. 5 (T = sum g~).
#include <type_traits>

#include "lb_kernels.h"

namespace lbk {

// population a of species sp at cell c, decoded to double
// reference of species sp at cell c: ref, or the row's thermal reference
__device__ inline double ref_at(const AuxArgs& A, int sp, int64_t c, double ref) {
    return (sp == 1 && A.tref) ? double(A.tref[c / A.nx]) : ref;
}

template <class S>
__device__ inline double get_pop(const AuxArgs& A, const S* st, int sp, int a, int64_t c, double ref) {
    const int nsp = A.thermal ? 2 : 1;
    ref = ref_at(A, sp, c, ref);
    double x = Codec<S>::template load<double>(st + pop_index(A.grouped, nsp, A.plane, sp, a, c));
    return Codec<S>::offset ? x + wt<double>(a) * ref : x;
}

template <class S>
__device__ inline void put_pop(const AuxArgs& A, S* st, int sp, int a, int64_t c, double ref, double v) {
    const int nsp = A.thermal ? 2 : 1;
    ref = ref_at(A, sp, c, ref);
    double x = Codec<S>::offset ? v - wt<double>(a) * ref : v;
    Codec<S>::template store<double>(st + pop_index(A.grouped, nsp, A.plane, sp, a, c), x);
}

// ---- moment-split cells (SplitLayout), decoded and encoded in double ----
template <class S> __device__ inline double split_get(const char* st, int64_t off) {
    const uint16_t b = *reinterpret_cast<const uint16_t*>(st + off);
    double x;
    if constexpr (std::is_same<S, bf16s_t>::value) x = double(bf16_bits_to_float(b));
    else x = double(__half2float(__ushort_as_half(b)));
    return x / double(split_scale<S>::value);
}
template <class S> __device__ inline void split_put(char* st, int64_t off, double r) {
    const float x = float(r * double(split_scale<S>::value));
    uint16_t b;
    if constexpr (std::is_same<S, bf16s_t>::value) b = float_to_bf16_bits(x);
    else b = __half_as_ushort(__float2half_rn(x));
    *reinterpret_cast<uint16_t*>(st + off) = b;
}

// Offsets e_a = E_a - w_a ref of the forced equilibrium at moments m (f:
// E = f_eq - dt/2 F, g: E = g_eq), with the row reference Tr of g.
__device__ inline void split_eq_d(const AuxArgs& A, const double* m, double Tr, double (*e)[9]) {
    const double rho = m[0] + A.ref_f, T = A.thermal ? m[3] + Tr : 0.0;
    const double ay = A.thermal ? A.ay + A.bg * (T - A.T0) : A.ay;
    const double ux = m[1] / rho + A.hdt * A.ax, uy = m[2] / rho + A.hdt * ay;
    const double uu = 1.5 * (ux * ux + uy * uy), ua = ux * A.ax + uy * ay;
    for (int a = 0; a < 9; ++a) {
        const double cu = cx(a) * ux + cy(a) * uy, ca = cx(a) * A.ax + cy(a) * ay;
        const double pm1 = 3.0 * cu + 4.5 * cu * cu - uu;          // f_eq / (w rho) - 1
        const double fr = 3.0 * (ca - ua) + 9.0 * cu * ca;         // F / (w rho)
        e[0][a] = wt<double>(a) * (m[0] + rho * (pm1 - A.hdt * fr));
        e[1][a] = A.thermal ? wt<double>(a) * (m[3] + T * pm1) : 0.0;
    }
}

__device__ inline SplitLayout split_layout(const AuxArgs& A) { return SplitLayout{A.thermal != 0, A.plane}; }
__device__ inline double row_ref(const AuxArgs& A, int64_t c) { return A.tref ? double(A.tref[c / A.nx]) : A.ref_g; }
// heat-flux reference of the row of cell c: the stored g residual of
// population a is r_a - w_a c_ay q
__device__ inline double row_qref(const AuxArgs& A, int64_t c) { return A.qref ? double(A.qref[c / A.nx]) : 0.0; }

template <class S> __device__ inline void split_moments(const AuxArgs& A, int64_t c, double* m) {
    const SplitLayout L = split_layout(A);
    const char* st = static_cast<const char*>(A.state);
    for (int q = 0; q < 4; ++q)
        m[q] = (q < 3 || A.thermal) ? double(*reinterpret_cast<const float*>(st + L.mom(q, c))) : 0.0;
}

// populations p[s][a] of cell c
template <class S> __device__ inline void split_decode_d(const AuxArgs& A, int64_t c, double (*p)[9]) {
    const SplitLayout L = split_layout(A);
    const char* st = static_cast<const char*>(A.state);
    double m[4], e[2][9], r[2][9];
    split_moments<S>(A, c, m);
    for (int s = 0; s < 2; ++s)
        for (int a = 0; a < 9; ++a) {
            const int k = split_slot(s, a);
            r[s][a] = (k >= 0 && (s == 0 || A.thermal)) ? split_get<S>(st, L.res(k, c)) : 0.0;
        }
    const double q = row_qref(A, c);
    for (int a = 1; a < 9; ++a) r[1][a] += wt<double>(a) * cy(a) * q;  // zero mass: slot 0 is unchanged
    r[0][1] = r[0][3] - r[0][5] + r[0][6] + r[0][7] - r[0][8];
    r[0][2] = r[0][4] - r[0][5] - r[0][6] + r[0][7] + r[0][8];
    for (int s = 0; s < 2; ++s) {
        double t = 0.0;
        for (int a = 1; a < 9; ++a) t += r[s][a];
        r[s][0] = -t;
    }
    const double Tr = row_ref(A, c);
    split_eq_d(A, m, Tr, e);
    for (int a = 0; a < 9; ++a) {
        p[0][a] = e[0][a] + r[0][a] + wt<double>(a) * A.ref_f;
        p[1][a] = A.thermal ? e[1][a] + r[1][a] + wt<double>(a) * Tr : 0.0;
    }
}

template <class S> __device__ inline void split_encode_d(const AuxArgs& A, int64_t c, const double (*p)[9]) {
    const SplitLayout L = split_layout(A);
    char* st = static_cast<char*>(A.state);
    const double Tr = row_ref(A, c);
    double d[2][9], m[4] = {0.0, 0.0, 0.0, 0.0}, e[2][9];
    for (int a = 0; a < 9; ++a) {
        d[0][a] = p[0][a] - wt<double>(a) * A.ref_f;
        d[1][a] = A.thermal ? p[1][a] - wt<double>(a) * Tr : 0.0;
        m[0] += d[0][a];
        m[1] += cx(a) * d[0][a];
        m[2] += cy(a) * d[0][a];
        m[3] += d[1][a];
    }
    for (int q = 0; q < 4; ++q) m[q] = double(float(m[q]));  // the stored moments
    for (int q = 0; q < (A.thermal ? 4 : 3); ++q) *reinterpret_cast<float*>(st + L.mom(q, c)) = float(m[q]);
    split_eq_d(A, m, Tr, e);
    const double q = row_qref(A, c);
    for (int s = 0; s < (A.thermal ? 2 : 1); ++s)
        for (int a = 0; a < 9; ++a) {
            const int k = split_slot(s, a);
            if (k >= 0) split_put<S>(st, L.res(k, c), d[s][a] - e[s][a] - (s ? wt<double>(a) * cy(a) * q : 0.0));
        }
}

__device__ inline StageConst<double> aux_const(const AuxArgs& a) {
    StageConst<double> k{};
    k.hdt = a.hdt;
    k.ax = a.ax;
    k.ay = a.ay;
    k.bg = a.bg;
    k.T0 = a.T0;
    return k;
}

// f~ = f_eq - dt/2 F and g~ = (T/rho) f_eq (appendix A)
template <class S>
__global__ void init_kernel(AuxArgs A, const double* rho, const double* ux, const double* uy, const double* T) {
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= A.plane) return;
    Macro<double> m;
    m.rho = rho[c];
    m.ux = ux[c];
    m.uy = uy[c];
    m.T = A.thermal ? T[c] : 0.0;
    m.ax = A.ax;
    m.ay = A.thermal ? A.ay + A.bg * (m.T - A.T0) : A.ay;
    EqForce<double> e;
    eq_force(m, e);
    if constexpr (is_split<S>::value) {
        double p[2][9];
        for (int a = 0; a < 9; ++a) {
            const double wr = wt<double>(a) * m.rho;
            p[0][a] = wr * e.poly[a] - A.hdt * wr * e.frc[a];
            p[1][a] = wt<double>(a) * m.T * e.poly[a];
        }
        split_encode_d<S>(A, c, p);
    } else {
        S* st = static_cast<S*>(A.state);
        for (int a = 0; a < 9; ++a) {
            const double wr = wt<double>(a) * m.rho;
            put_pop(A, st, 0, a, c, A.ref_f, wr * e.poly[a] - A.hdt * wr * e.frc[a]);
            if (A.thermal) put_pop(A, st, 1, a, c, A.ref_g, wt<double>(a) * m.T * e.poly[a]);
        }
    }
}

template <class S>
__device__ inline Macro<double> cell_macro(const AuxArgs& A, int64_t c) {
    if constexpr (is_split<S>::value) {  // the stored moments
        double mm[4];
        split_moments<S>(A, c, mm);
        Macro<double> m;
        m.rho = mm[0] + A.ref_f;
        m.T = A.thermal ? mm[3] + row_ref(A, c) : 0.0;
        m.ax = A.ax;
        m.ay = A.thermal ? A.ay + A.bg * (m.T - A.T0) : A.ay;
        m.ux = mm[1] / m.rho + A.hdt * m.ax;
        m.uy = mm[2] / m.rho + A.hdt * m.ay;
        return m;
    } else {
        const S* st = static_cast<const S*>(A.state);
        double f[9], g[9];
        for (int a = 0; a < 9; ++a) {
            f[a] = get_pop(A, st, 0, a, c, A.ref_f);
            g[a] = A.thermal ? get_pop(A, st, 1, a, c, A.ref_g) : 0.0;
        }
        StageConst<double> k = aux_const(A);
        return A.thermal ? macro<double, true>(f, g, k) : macro<double, false>(f, g, k);
    }
}

template <class S>
__global__ void moments_kernel(AuxArgs A, double* rho, double* ux, double* uy, double* T) {
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= A.plane) return;
    Macro<double> m = cell_macro<S>(A, c);
    rho[c] = m.rho;
    ux[c] = m.ux;
    uy[c] = m.uy;
    T[c] = m.T;
}

template <class S>
__global__ void get_pops_kernel(AuxArgs A, double* out) {
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= A.plane) return;
    const int ns = A.thermal ? 2 : 1;
    if constexpr (is_split<S>::value) {
        double p[2][9];
        split_decode_d<S>(A, c, p);
        for (int s = 0; s < ns; ++s)
            for (int a = 0; a < 9; ++a) out[(s * 9 + a) * A.plane + c] = p[s][a];
    } else {
        const S* st = static_cast<const S*>(A.state);
        for (int s = 0; s < ns; ++s)
            for (int a = 0; a < 9; ++a)
                out[(s * 9 + a) * A.plane + c] = get_pop(A, st, s, a, c, s ? A.ref_g : A.ref_f);
    }
}

template <class S>
__global__ void set_pops_kernel(AuxArgs A, const double* in) {
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= A.plane) return;
    const int ns = A.thermal ? 2 : 1;
    if constexpr (is_split<S>::value) {
        double p[2][9];
        for (int s = 0; s < 2; ++s)
            for (int a = 0; a < 9; ++a) p[s][a] = s < ns ? in[(s * 9 + a) * A.plane + c] : 0.0;
        split_encode_d<S>(A, c, p);
    } else {
        S* st = static_cast<S*>(A.state);
        for (int s = 0; s < ns; ++s)
            for (int a = 0; a < 9; ++a)
                put_pop(A, st, s, a, c, s ? A.ref_g : A.ref_f, in[(s * 9 + a) * A.plane + c]);
    }
}

// ---- per-row thermal reference update ----------------------------------
// One block per row: the row mean of T becomes the row's new reference and
// every stored g of the row is re-encoded, d_new = d_old + w_a (old - new).
// Split storage also renews the heat-flux reference q: 3 times the row mean
// of sum_a c_ay r_a (sum_a w_a c_ay^2 = 1/3), and each stored residual of a
// population along y moves by w_a c_ay (q_old - q_new) (one rounding).
template <class S>
__device__ __forceinline__ void rebase_row(const AuxArgs& A, const int j) {
    __shared__ double red[2][4];
    __shared__ float newref, newq;
    S* st = static_cast<S*>(A.state);
    constexpr bool SPLIT = is_split<S>::value;
    const bool with_q = SPLIT && A.qref;
    const float oldq = with_q ? A.qref[j] : 0.0f;
    double sum = 0.0, flux = 0.0;
    for (int i = threadIdx.x; i < A.nx; i += 256) {
        const int64_t c = int64_t(j) * A.nx + i;
        if constexpr (SPLIT) {
            sum += cell_macro<S>(A, c).T;
            if (with_q) {
                const SplitLayout L = split_layout(A);
                const char* sb = static_cast<const char*>(A.state);
                for (int a = 1; a < 9; ++a)
                    if (cy(a)) flux += cy(a) * split_get<S>(sb, L.res(split_slot(1, a), c));
            }
        } else {
            for (int a = 0; a < 9; ++a) sum += get_pop(A, st, 1, a, c, A.ref_g);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        sum += __shfl_down(sum, o, 64);
        flux += __shfl_down(flux, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = sum;
        red[1][threadIdx.x >> 6] = flux;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        newref = float((red[0][0] + red[0][1] + red[0][2] + red[0][3]) / A.nx);
        // stored residuals are r - w c_y q_old: their mean flux is mean(sum c_y r) - q_old / 3
        newq = with_q ? float(3.0 * (red[1][0] + red[1][1] + red[1][2] + red[1][3]) / A.nx + double(oldq)) : 0.0f;
    }
    __syncthreads();
    const float oldref = A.tref[j];
    const float nr = newref, nq = newq;
    for (int i = threadIdx.x; i < A.nx; i += 256) {
        const int64_t c = int64_t(j) * A.nx + i;
        if constexpr (SPLIT) {  // the moment T - Tr, and the residuals along y
            const SplitLayout L = split_layout(A);
            char* sb = static_cast<char*>(A.state);
            float* m3 = reinterpret_cast<float*>(sb + L.mom(3, c));
            *m3 = float(double(*m3) + (double(oldref) - double(nr)));
            if (with_q)
                for (int a = 1; a < 9; ++a)
                    if (cy(a)) {
                        const int64_t off = L.res(split_slot(1, a), c);
                        split_put<S>(sb, off, split_get<S>(sb, off) + wt<double>(a) * cy(a) * (double(oldq) - double(nq)));
                    }
        } else {
            const int nsp = 2;
            for (int a = 0; a < 9; ++a) {
                S* p = st + pop_index(A.grouped, nsp, A.plane, 1, a, c);
                const double d = Codec<S>::template load<double>(p);
                Codec<S>::template store<double>(p, d + wt<double>(a) * (double(oldref) - double(nr)));
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const_cast<float*>(A.tref)[j] = nr;
        if (with_q) const_cast<float*>(A.qref)[j] = nq;
    }
    __syncthreads();   // the shared reduction slots are free for the next row
}

template <class S>
__global__ void __launch_bounds__(256) rebase_kernel(AuxArgs A) {
    rebase_row<S>(A, blockIdx.x);
}

// Serving: the rows of many simulations (items = (simulation, row)); a
// simulation's rows are renewed only when due[simulation] is set, which the
// step counter kernel decides.  Blocks stride over the items.
template <class S>
__global__ void __launch_bounds__(256) rebase_multi_kernel(const AuxArgs* args, const int2* items, int n_items,
                                                           const int* due, const int* phase) {
    for (int q = blockIdx.x; q < n_items; q += gridDim.x) {
        const int2 it = items[q];
        if (!due[it.x]) continue;   // uniform over the block
        // two argument blocks per simulation: its state in the first or the
        // second buffer (the phase of fused group steps; 0 without)
        const AuxArgs A = args[2 * it.x + (phase ? phase[it.x] : 0)];
        rebase_row<S>(A, it.y);
    }
}

template <class S>
static hipError_t rebase_typed(const AuxArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(rebase_kernel<S>, dim3(a.ny), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <class S>
static hipError_t rebase_multi_typed(const AuxArgs* args, const int2* items, int n_items, const int* due,
                                     const int* phase, hipStream_t s) {
    const int blocks = n_items < 2048 ? n_items : 2048;
    hipLaunchKernelGGL(rebase_multi_kernel<S>, dim3(blocks), dim3(256), 0, s, args, items, n_items, due, phase);
    return hipGetLastError();
}

hipError_t launch_rebase_multi(int storage, const AuxArgs* args, const int2* items, int n_items, const int* due,
                               const int* phase, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    switch (storage) {
        case ST_F32: return rebase_multi_typed<float>(args, items, n_items, due, phase, s);
        case ST_BF16: return rebase_multi_typed<bf16_t>(args, items, n_items, due, phase, s);
        case ST_F16: return rebase_multi_typed<f16_t>(args, items, n_items, due, phase, s);
        case ST_BF16S: return rebase_multi_typed<bf16s_t>(args, items, n_items, due, phase, s);
        case ST_F16S: return rebase_multi_typed<f16s_t>(args, items, n_items, due, phase, s);
    }
    return hipSuccess;
}

hipError_t launch_rebase(int storage, const AuxArgs& a, hipStream_t s) {
    if (!a.tref || !a.thermal) return hipSuccess;
    switch (storage) {
        case ST_F32: return rebase_typed<float>(a, s);
        case ST_BF16: return rebase_typed<bf16_t>(a, s);
        case ST_F16: return rebase_typed<f16_t>(a, s);
        case ST_BF16S: return rebase_typed<bf16s_t>(a, s);
        case ST_F16S: return rebase_typed<f16s_t>(a, s);
    }
    return hipSuccess;
}

// ---- diagnostics -------------------------------------------------------

__device__ inline double block_sum(double v, double* sh) {
    // wave64 tree, then the four wave sums in order
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
__global__ void __launch_bounds__(256) diag_kernel(DiagArgs D, double* partial) {
    __shared__ double sh[4];
    const AuxArgs& A = D.a;
    const S* st = static_cast<const S*>(A.state);
    double acc[D_COUNT];
    for (int q = 0; q < D_COUNT; ++q) acc[q] = 0.0;
    const int ns = A.thermal ? 2 : 1;
    for (int64_t c = int64_t(blockIdx.x) * 256 + threadIdx.x; c < A.plane; c += int64_t(gridDim.x) * 256) {
        const int i = int(c % A.nx), j = int(c / A.nx);
        const double v = A.dx[i] * A.dy[j];
        Macro<double> m = cell_macro<S>(A, c);
        acc[D_MASS] += v * m.rho;
        acc[D_EKIN] += v * 0.5 * m.rho * (m.ux * m.ux + m.uy * m.uy);
        acc[D_ETH] += v * m.T;
        acc[D_UT] += v * m.uy * m.T;
        acc[D_VOL] += v;
        if constexpr (is_split<S>::value) {
            double p[2][9];
            split_decode_d<S>(A, c, p);
            for (int s = 0; s < ns; ++s)
                for (int a = 0; a < 9; ++a)
                    if (!isfinite(p[s][a])) acc[D_BAD] = 1.0;
        } else {
            for (int s = 0; s < ns; ++s)
                for (int a = 0; a < 9; ++a) {
                    const double p = get_pop(A, st, s, a, c, 0.0);
                    if (!isfinite(p)) acc[D_BAD] = 1.0;
                }
        }
        if (D.walls && (j == 0 || j == A.ny - 1)) {
            const int j2 = j == 0 ? 1 : A.ny - 2;
            const double T2 = cell_macro<S>(A, int64_t(j2) * A.nx + i).T;
            const double w = A.dx[i] * D.inv_Lx;
            if (j == 0)
                acc[D_NUB] += w * D.nu_scale * (D.nub[0] * D.Tb + D.nub[1] * m.T + D.nub[2] * T2);
            if (j == A.ny - 1)
                acc[D_NUT] += w * D.nu_scale * (D.nut[0] * D.Tt + D.nut[1] * m.T + D.nut[2] * T2);
        }
    }
    for (int q = 0; q < D_COUNT; ++q) {
        double r = block_sum(acc[q], sh);
        if (threadIdx.x == 0) partial[int64_t(blockIdx.x) * D_COUNT + q] = r;
    }
}

template <class S>
__global__ void __launch_bounds__(256) profile_kernel(AuxArgs A, double inv_Lx, double* out) {
    __shared__ double sh[4];
    const int j = blockIdx.x;
    double acc[PROFILE_ROWS] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < A.nx; i += 256) {
        const int64_t c = int64_t(j) * A.nx + i;
        const Macro<double> m = cell_macro<S>(A, c);
        const double w = A.dx[i] * inv_Lx;
        acc[0] += w * m.T;
        acc[1] += w * m.T * m.T;
        acc[2] += w * m.ux * m.ux;
        acc[3] += w * m.uy * m.uy;
        acc[4] += w * m.uy * m.T;
    }
    for (int q = 0; q < PROFILE_ROWS; ++q) {
        const double r = block_sum(acc[q], sh);
        if (threadIdx.x == 0) out[int64_t(q) * A.ny + j] = r;
    }
}

template <class S>
static hipError_t profiles_typed(const AuxArgs& a, double inv_Lx, double* out, hipStream_t s) {
    hipLaunchKernelGGL(profile_kernel<S>, dim3(a.ny), dim3(256), 0, s, a, inv_Lx, out);
    return hipGetLastError();
}

hipError_t launch_profiles(int storage, const AuxArgs& a, double inv_Lx, double* out, hipStream_t s) {
    switch (storage) {
        case ST_F64: return profiles_typed<double>(a, inv_Lx, out, s);
        case ST_F32: return profiles_typed<float>(a, inv_Lx, out, s);
        case ST_BF16: return profiles_typed<bf16_t>(a, inv_Lx, out, s);
        case ST_F16: return profiles_typed<f16_t>(a, inv_Lx, out, s);
        case ST_BF16S: return profiles_typed<bf16s_t>(a, inv_Lx, out, s);
        case ST_F16S: return profiles_typed<f16s_t>(a, inv_Lx, out, s);
    }
    return hipErrorInvalidValue;
}

__global__ void __launch_bounds__(256) diag_fold(const double* partial, int nblocks, double* out, DiagFinal fin) {
    __shared__ double sh[4];
    for (int q = 0; q < D_COUNT; ++q) {
        double acc = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += 256) {
            double p = partial[int64_t(b) * D_COUNT + q];
            acc = (q == D_BAD) ? fmax(acc, p) : acc + p;
        }
        double r;
        if (q == D_BAD) {
            // any block flagged: sum of flags > 0
            r = block_sum(acc, sh);
            r = r > 0.0 ? 1.0 : 0.0;
        } else {
            r = block_sum(acc, sh);
        }
        if (threadIdx.x == 0) out[q] = r;
    }
    // the values lb_diagnostics reports: wall Nusselt numbers only with
    // isothermal walls, and the volume Nusselt number in place of sum V u_y T
    if (fin.finish && threadIdx.x == 0) {
        const double ut = out[D_UT], vol = out[D_VOL];
        out[D_NUB] = fin.walls ? out[D_NUB] : 0.0;
        out[D_NUT] = fin.walls ? out[D_NUT] : 0.0;
        out[D_UT] = fin.walls ? 1.0 + fin.H * (ut / vol) / (fin.kappa * fin.dT) : 0.0;
    }
}

template <class S>
static hipError_t aux_typed(int what, const AuxArgs& a, const double* p0, const double* p1, const double* p2,
                            const double* p3, double* o0, double* o1, double* o2, double* o3, hipStream_t s) {
    const int64_t blocks = (a.plane + 255) / 256;
    switch (what) {
        case 0: hipLaunchKernelGGL(init_kernel<S>, dim3(blocks), dim3(256), 0, s, a, p0, p1, p2, p3); break;
        case 1: hipLaunchKernelGGL(moments_kernel<S>, dim3(blocks), dim3(256), 0, s, a, o0, o1, o2, o3); break;
        case 2: hipLaunchKernelGGL(get_pops_kernel<S>, dim3(blocks), dim3(256), 0, s, a, o0); break;
        case 3: hipLaunchKernelGGL(set_pops_kernel<S>, dim3(blocks), dim3(256), 0, s, a, p0); break;
    }
    return hipGetLastError();
}

static hipError_t aux_dispatch(int storage, int what, const AuxArgs& a, const double* p0, const double* p1,
                               const double* p2, const double* p3, double* o0, double* o1, double* o2,
                               double* o3, hipStream_t s) {
    switch (storage) {
        case ST_F64: return aux_typed<double>(what, a, p0, p1, p2, p3, o0, o1, o2, o3, s);
        case ST_F32: return aux_typed<float>(what, a, p0, p1, p2, p3, o0, o1, o2, o3, s);
        case ST_BF16: return aux_typed<bf16_t>(what, a, p0, p1, p2, p3, o0, o1, o2, o3, s);
        case ST_F16: return aux_typed<f16_t>(what, a, p0, p1, p2, p3, o0, o1, o2, o3, s);
        case ST_BF16S: return aux_typed<bf16s_t>(what, a, p0, p1, p2, p3, o0, o1, o2, o3, s);
        case ST_F16S: return aux_typed<f16s_t>(what, a, p0, p1, p2, p3, o0, o1, o2, o3, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_init(int storage, const AuxArgs& a, const double* rho, const double* ux, const double* uy,
                       const double* T, hipStream_t s) {
    return aux_dispatch(storage, 0, a, rho, ux, uy, T, nullptr, nullptr, nullptr, nullptr, s);
}
hipError_t launch_moments(int storage, const AuxArgs& a, double* rho, double* ux, double* uy, double* T,
                          hipStream_t s) {
    return aux_dispatch(storage, 1, a, nullptr, nullptr, nullptr, nullptr, rho, ux, uy, T, s);
}
hipError_t launch_get_pops(int storage, const AuxArgs& a, double* out, hipStream_t s) {
    return aux_dispatch(storage, 2, a, nullptr, nullptr, nullptr, nullptr, out, nullptr, nullptr, nullptr, s);
}
hipError_t launch_set_pops(int storage, const AuxArgs& a, const double* in, hipStream_t s) {
    return aux_dispatch(storage, 3, a, in, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, s);
}

int diag_blocks(int64_t cells) {
    const int64_t want = (cells + 255) / 256;
    return int(want < DIAG_BLOCKS ? want : DIAG_BLOCKS);
}

hipError_t launch_diagnostics(int storage, const DiagArgs& d, double* partial, double* out, hipStream_t s,
                              const DiagFinal& fin) {
    const int nb = diag_blocks(d.a.plane);
    switch (storage) {
        case ST_F64: hipLaunchKernelGGL(diag_kernel<double>, dim3(nb), dim3(256), 0, s, d, partial); break;
        case ST_F32: hipLaunchKernelGGL(diag_kernel<float>, dim3(nb), dim3(256), 0, s, d, partial); break;
        case ST_BF16: hipLaunchKernelGGL(diag_kernel<bf16_t>, dim3(nb), dim3(256), 0, s, d, partial); break;
        case ST_F16: hipLaunchKernelGGL(diag_kernel<f16_t>, dim3(nb), dim3(256), 0, s, d, partial); break;
        case ST_BF16S: hipLaunchKernelGGL(diag_kernel<bf16s_t>, dim3(nb), dim3(256), 0, s, d, partial); break;
        case ST_F16S: hipLaunchKernelGGL(diag_kernel<f16s_t>, dim3(nb), dim3(256), 0, s, d, partial); break;
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(diag_fold, dim3(1), dim3(256), 0, s, partial, nb, out, fin);
    return hipGetLastError();
}

}  // namespace lbk
