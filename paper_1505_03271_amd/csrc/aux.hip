// Initial state, field export and FP64 diagnostics of liblb.
//
// All arithmetic here is double precision: the stored words are decoded
// exactly (every storage format widens exactly to double) and the moments
// follow the relations of arXiv:1505.03271 sec. 2.1 and "Force term"
// (rho = sum f~, u = sum c f~ / rho + dt/2 a) and sec. 5 (T = sum g~).
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
    S* st = static_cast<S*>(A.state);
    Macro<double> m;
    m.rho = rho[c];
    m.ux = ux[c];
    m.uy = uy[c];
    m.T = A.thermal ? T[c] : 0.0;
    m.ax = A.ax;
    m.ay = A.thermal ? A.ay + A.bg * (m.T - A.T0) : A.ay;
    EqForce<double> e;
    eq_force(m, e);
    for (int a = 0; a < 9; ++a) {
        const double wr = wt<double>(a) * m.rho;
        put_pop(A, st, 0, a, c, A.ref_f, wr * e.poly[a] - A.hdt * wr * e.frc[a]);
        if (A.thermal) put_pop(A, st, 1, a, c, A.ref_g, wt<double>(a) * m.T * e.poly[a]);
    }
}

template <class S>
__device__ inline Macro<double> cell_macro(const AuxArgs& A, int64_t c) {
    const S* st = static_cast<const S*>(A.state);
    double f[9], g[9];
    for (int a = 0; a < 9; ++a) {
        f[a] = get_pop(A, st, 0, a, c, A.ref_f);
        g[a] = A.thermal ? get_pop(A, st, 1, a, c, A.ref_g) : 0.0;
    }
    StageConst<double> k = aux_const(A);
    return A.thermal ? macro<double, true>(f, g, k) : macro<double, false>(f, g, k);
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
    const S* st = static_cast<const S*>(A.state);
    const int ns = A.thermal ? 2 : 1;
    for (int s = 0; s < ns; ++s)
        for (int a = 0; a < 9; ++a)
            out[(s * 9 + a) * A.plane + c] = get_pop(A, st, s, a, c, s ? A.ref_g : A.ref_f);
}

template <class S>
__global__ void set_pops_kernel(AuxArgs A, const double* in) {
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= A.plane) return;
    S* st = static_cast<S*>(A.state);
    const int ns = A.thermal ? 2 : 1;
    for (int s = 0; s < ns; ++s)
        for (int a = 0; a < 9; ++a)
            put_pop(A, st, s, a, c, s ? A.ref_g : A.ref_f, in[(s * 9 + a) * A.plane + c]);
}

// ---- per-row thermal reference update ----------------------------------
// One block per row: the row mean of T becomes the row's new reference and
// every stored g of the row is re-encoded, d_new = d_old + w_a (old - new).
template <class S>
__global__ void __launch_bounds__(256) rebase_kernel(AuxArgs A) {
    __shared__ double red[4];
    __shared__ float newref;
    const int j = blockIdx.x;
    S* st = static_cast<S*>(A.state);
    double sum = 0.0;
    for (int i = threadIdx.x; i < A.nx; i += 256) {
        const int64_t c = int64_t(j) * A.nx + i;
        for (int a = 0; a < 9; ++a) sum += get_pop(A, st, 1, a, c, A.ref_g);
    }
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_down(sum, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) newref = float((red[0] + red[1] + red[2] + red[3]) / A.nx);
    __syncthreads();
    const float oldref = A.tref[j];
    const float nr = newref;
    for (int i = threadIdx.x; i < A.nx; i += 256) {
        const int64_t c = int64_t(j) * A.nx + i;
        const int nsp = 2;
        for (int a = 0; a < 9; ++a) {
            S* p = st + pop_index(A.grouped, nsp, A.plane, 1, a, c);
            const double d = Codec<S>::template load<double>(p);
            Codec<S>::template store<double>(p, d + wt<double>(a) * (double(oldref) - double(nr)));
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) const_cast<float*>(A.tref)[j] = nr;
}

template <class S>
static hipError_t rebase_typed(const AuxArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(rebase_kernel<S>, dim3(a.ny), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_rebase(int storage, const AuxArgs& a, hipStream_t s) {
    if (!a.tref || !a.thermal) return hipSuccess;
    switch (storage) {
        case ST_F32: return rebase_typed<float>(a, s);
        case ST_BF16: return rebase_typed<bf16_t>(a, s);
        case ST_F16: return rebase_typed<f16_t>(a, s);
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
        for (int s = 0; s < ns; ++s)
            for (int a = 0; a < 9; ++a) {
                const double p = get_pop(A, st, s, a, c, 0.0);
                if (!isfinite(p)) acc[D_BAD] = 1.0;
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

__global__ void __launch_bounds__(256) diag_fold(const double* partial, int nblocks, double* out) {
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

hipError_t launch_diagnostics(int storage, const DiagArgs& d, double* partial, double* out, hipStream_t s) {
    const int64_t want = (d.a.plane + 255) / 256;
    const int nb = int(want < DIAG_BLOCKS ? want : DIAG_BLOCKS);
    switch (storage) {
        case ST_F64: hipLaunchKernelGGL(diag_kernel<double>, dim3(nb), dim3(256), 0, s, d, partial); break;
        case ST_F32: hipLaunchKernelGGL(diag_kernel<float>, dim3(nb), dim3(256), 0, s, d, partial); break;
        case ST_BF16: hipLaunchKernelGGL(diag_kernel<bf16_t>, dim3(nb), dim3(256), 0, s, d, partial); break;
        case ST_F16: hipLaunchKernelGGL(diag_kernel<f16_t>, dim3(nb), dim3(256), 0, s, d, partial); break;
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(diag_fold, dim3(1), dim3(256), 0, s, partial, nb, out);
    return hipGetLastError();
}

}  // namespace lbk
