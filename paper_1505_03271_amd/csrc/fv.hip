// Finite-volume lattice Boltzmann stage kernel (arXiv:1505.03271 sec. 2.2).
//
// One launch evaluates, for every cell, one semi-implicit stage fused with
// the QUICK face fluxes:
//   phi = f~ + dt/(2 tau~)(f_eq - f~) + dt/2 F         (advected bracket, eq:semi)
//   C   = dt/tau~ (f_eq - f~) + dt (1 - dt/(2 tau~)) F  (collision + force)
//   D   = sum_faces (S/V) c.n [phi]_face                (QUICK, sec. 2.2.3)
// and writes
//   predictor / single pass:  f~*   = f~n - dt D(phi(f~n)) + C(f~n)          (eq:semi)
//   corrector:                f~n+1 = (f~n + f~* + C(f~n))/2 - dt/2 D(phi(f~*))
// The corrector form is eq:semi-heun rewritten with f~* = f~n - dt Dn + Cn,
// so D(phi(f~n)) never has to be recomputed and f~n+1 can overwrite f~n: each
// cell reads f~n only at itself, and f~* (with halo) from the other buffer.
//
// Mapping: a block of FV_LANES lanes owns a strip of up to FV_LANES - 4
// consecutive columns plus two halo columns on each side (one lane per
// column) and marches up a chunk of rows.  Each row is loaded once with
// coalesced accesses (x fastest in every population plane), the stage is
// evaluated once per cell, x-face neighbours are exchanged through LDS
// (double buffered, one barrier per row), and y-face neighbours are kept in a
// rolling register window of the last rows.  The y-face weights and 1/dy are
// uniform over the block (scalar loads); the x-face weights are per lane and
// stay in registers for the whole march.
//
// Boundaries ("Boundary conditions" of sec. 2.2): the advected bracket phi of
// a ghost cell is that of its mirror cell with the opposite population
// (double reflection); for g on the y walls the anti-reflection
// -phi_inv(a) + 2 w_a T_w imposes the wall temperature.  Periodic axes wrap.
#include "lb_kernels.h"

namespace lbk {

// populations with c_x != 0, in the order (+1, +1, +1, -1, -1, -1)
__device__ constexpr int xpop(int p) { return p == 0 ? 1 : p == 1 ? 5 : p == 2 ? 8 : p == 3 ? 3 : p == 4 ? 6 : 7; }
// populations with c_y = +1 and c_y = -1
__device__ constexpr int upop(int p) { return p == 0 ? 2 : p == 1 ? 5 : 6; }
__device__ constexpr int dpop(int p) { return p == 0 ? 4 : p == 1 ? 7 : 8; }

template <class R, class S>
__device__ inline void load_pops(const S* base, int64_t plane, int64_t cell, R ref, R* v) {
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        R x = Codec<S>::template load<R>(base + a * plane + cell);
        v[a] = Codec<S>::offset ? x + wt<R>(a) * ref : x;
    }
}

template <class R, class S>
__device__ inline void store_pops(S* base, int64_t plane, int64_t cell, R ref, const R* v) {
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        R x = Codec<S>::offset ? v[a] - wt<R>(a) * ref : v[a];
        Codec<S>::template store<R>(base + a * plane + cell, x);
    }
}

// One semi-implicit stage at a cell: the advected brackets phi (and, when
// WANT_C, the collision increments C) of f and g.
template <class R, bool TH, bool WANT_C>
__device__ inline void stage(const R* f, const R* g, const StageConst<R>& k, R (*ph)[9], R (*C)[9]) {
    Macro<R> m = macro<R, TH>(f, g, k);
    EqForce<R> e;
    eq_force(m, e);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const R wr = wt<R>(a) * m.rho;
        const R feq = wr * e.poly[a];
        const R F = wr * e.frc[a];
        const R neq = feq - f[a];
        ph[0][a] = f[a] + k.k1 * neq + k.kh * F;
        if (WANT_C) C[0][a] = k.kc * neq + k.kf * F;
        if (TH) {
            const R geq = wt<R>(a) * m.T * e.poly[a];
            const R gneq = geq - g[a];
            ph[1][a] = g[a] + k.k1g * gneq;
            if (WANT_C) C[1][a] = k.kcg * gneq;
        }
    }
}

template <class R, class S, bool TH, bool CORR>
__global__ void __launch_bounds__(FV_LANES) fv_pass(FvArgs<R> A) {
    constexpr int NSP = TH ? 2 : 1;
    __shared__ R lds[2][6 * NSP][FV_LANES];

    const int t = threadIdx.x;
    const int x0 = blockIdx.x * A.strip_w;
    const int own = min(A.strip_w, A.nx - x0);
    const int lanes = own + 2 * FV_HALO;
    if ((t & ~63) >= lanes) return;  // a wave with no column of this strip leaves (barriers count live waves)

    // ---- this lane's column (ghost columns mirror or wrap) ----
    const int xg = x0 - FV_HALO + t;
    int col = xg;
    bool mx = false;
    if (xg < 0) {
        if (A.wall_x) { col = -xg - 1; mx = true; } else col = xg + A.nx;
    } else if (xg >= A.nx) {
        if (A.wall_x) { col = 2 * A.nx - 1 - xg; mx = true; } else col = xg - A.nx;
    }
    if (t >= lanes) { col = 0; mx = false; }  // idle lane of a live wave
    const bool owned = t >= FV_HALO && t < FV_HALO + own;

    R xl[6], xr[6], idx_c = 0;
#pragma unroll
    for (int q = 0; q < 6; ++q) { xl[q] = 0; xr[q] = 0; }
    if (owned) {
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            xl[q] = A.m.xw[col * 6 + q];
            xr[q] = A.m.xw[(col + 1) * 6 + q];
        }
        idx_c = A.m.idx[col];
    }

    const S* src = static_cast<const S*>(A.src);
    const S* loc = static_cast<const S*>(A.loc);
    S* dst = static_cast<S*>(A.dst);
    const int64_t plane = A.plane;
    const int y0 = blockIdx.y * A.chunk_h;
    const int y1 = min(y0 + A.chunk_h, A.ny);

    // rolling state of the march
    R P3[NSP][3], P2[NSP][3], P1[NSP][3];  // phi of c_y=+1 populations at rows r-3, r-2, r-1
    R M2[NSP][3], M1[NSP][3];              // phi of c_y=-1 populations at rows r-2, r-1
    R Fp[NSP][6];                          // y-face values of the face below the row being finished
    R U1[NSP][9], U2[NSP][9];              // partial updates of rows r-1, r-2 (all but the y flux)
#pragma unroll
    for (int s = 0; s < NSP; ++s) {
#pragma unroll
        for (int q = 0; q < 3; ++q) { P3[s][q] = P2[s][q] = P1[s][q] = M2[s][q] = M1[s][q] = 0; }
#pragma unroll
        for (int q = 0; q < 6; ++q) Fp[s][q] = 0;
#pragma unroll
        for (int a = 0; a < 9; ++a) { U1[s][a] = U2[s][a] = 0; }
    }

    for (int r = y0 - 2; r <= y1 + 1; ++r) {
        int row = r;
        bool my = false;
        R Tw = 0;
        if (r < 0) {
            if (A.wall_y) { row = -r - 1; my = true; Tw = A.T_bottom; } else row = r + A.ny;
        } else if (r >= A.ny) {
            if (A.wall_y) { row = 2 * A.ny - 1 - r; my = true; Tw = A.T_top; } else row = r - A.ny;
        }
        const int64_t cell = int64_t(row) * A.nx + col;
        const bool out_row = r >= y0 && r < y1;

        R f[9], g[9];
        load_pops<R, S>(src, plane, cell, A.ref_f, f);
        if (TH) load_pops<R, S>(src + 9 * plane, plane, cell, A.ref_g, g);

        R ph[NSP][9], C[NSP][9];
        if (CORR)
            stage<R, TH, false>(f, g, A.k, ph, C);
        else
            stage<R, TH, true>(f, g, A.k, ph, C);

        // ghost rows: double reflection (f), anti-reflection about T_w (g)
        if (my) {
            R tmp[9];
#pragma unroll
            for (int a = 0; a < 9; ++a) tmp[a] = ph[0][a];
#pragma unroll
            for (int a = 0; a < 9; ++a) ph[0][a] = tmp[opp(a)];
            if (TH) {
#pragma unroll
                for (int a = 0; a < 9; ++a) tmp[a] = ph[NSP - 1][a];
#pragma unroll
                for (int a = 0; a < 9; ++a) ph[NSP - 1][a] = R(2) * wt<R>(a) * Tw - tmp[opp(a)];
            }
        }
        // ghost columns: double reflection of both species (x walls are adiabatic)
        if (mx) {
#pragma unroll
            for (int s = 0; s < NSP; ++s) {
                R tmp[9];
#pragma unroll
                for (int a = 0; a < 9; ++a) tmp[a] = ph[s][a];
#pragma unroll
                for (int a = 0; a < 9; ++a) ph[s][a] = tmp[opp(a)];
            }
        }

        // ---- x fluxes and the partial update of an output row ----
        R U0[NSP][9];
        if (out_row) {
            const int b = r & 1;
#pragma unroll
            for (int s = 0; s < NSP; ++s)
#pragma unroll
                for (int p = 0; p < 6; ++p) lds[b][s * 6 + p][t] = ph[s][xpop(p)];
            __syncthreads();
            if (owned) {
                R base[NSP][9];
                if (CORR) {
                    // C(f~n) at this cell; f~* is f here
                    R fn[9], gn[9], phn[NSP][9], Cn[NSP][9];
                    const int64_t oc = int64_t(r) * A.nx + col;
                    load_pops<R, S>(loc, plane, oc, A.ref_f, fn);
                    if (TH) load_pops<R, S>(loc + 9 * plane, plane, oc, A.ref_g, gn);
                    stage<R, TH, true>(fn, gn, A.k, phn, Cn);
#pragma unroll
                    for (int a = 0; a < 9; ++a) {
                        base[0][a] = R(0.5) * (fn[a] + f[a] + Cn[0][a]);
                        if (TH) base[NSP - 1][a] = R(0.5) * (gn[a] + g[a] + Cn[NSP - 1][a]);
                    }
                } else {
#pragma unroll
                    for (int a = 0; a < 9; ++a) {
                        base[0][a] = f[a] + C[0][a];
                        if (TH) base[NSP - 1][a] = g[a] + C[NSP - 1][a];
                    }
                }
#pragma unroll
                for (int s = 0; s < NSP; ++s) {
#pragma unroll
                    for (int a = 0; a < 9; ++a) U0[s][a] = base[s][a];
#pragma unroll
                    for (int p = 0; p < 6; ++p) {
                        const int a = xpop(p);
                        const R* L = lds[b][s * 6 + p];
                        const R v = ph[s][a];
                        R Fr, Fl;
                        if (cx(a) > 0) {
                            const R m1 = L[t - 1], m2 = L[t - 2], p1 = L[t + 1];
                            Fr = xr[0] * v + xr[1] * p1 + xr[2] * m1;
                            Fl = xl[0] * m1 + xl[1] * v + xl[2] * m2;
                        } else {
                            const R m1 = L[t - 1], p1 = L[t + 1], p2 = L[t + 2];
                            Fr = xr[3] * p1 + xr[4] * v + xr[5] * p2;
                            Fl = xl[3] * v + xl[4] * m1 + xl[5] * p1;
                        }
                        U0[s][a] -= A.dt_update * R(cx(a)) * (Fr - Fl) * idx_c;
                    }
                }
            }
        }

        // ---- y faces: face between rows r-2 and r-1 (face index r-1) ----
        if (r >= y0 + 1) {
            const R* yw = A.m.yw + int64_t(r - 1) * 6;
            const R w0 = yw[0], w1 = yw[1], w2 = yw[2], w3 = yw[3], w4 = yw[4], w5 = yw[5];
            R Fc[NSP][6];
#pragma unroll
            for (int s = 0; s < NSP; ++s) {
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    Fc[s][q] = w0 * P2[s][q] + w1 * P1[s][q] + w2 * P3[s][q];
                    Fc[s][3 + q] = w3 * M1[s][q] + w4 * M2[s][q] + w5 * ph[s][dpop(q)];
                }
            }
            if (r >= y0 + 2 && owned) {
                const int j = r - 2;
                const R iy = A.m.idy[j];
                R out[NSP][9];
#pragma unroll
                for (int s = 0; s < NSP; ++s) {
#pragma unroll
                    for (int a = 0; a < 9; ++a) out[s][a] = U2[s][a];
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        out[s][upop(q)] -= A.dt_update * (Fc[s][q] - Fp[s][q]) * iy;
                        out[s][dpop(q)] += A.dt_update * (Fc[s][3 + q] - Fp[s][3 + q]) * iy;
                    }
                }
                const int64_t oc = int64_t(j) * A.nx + col;
                store_pops<R, S>(dst, plane, oc, A.ref_f, out[0]);
                if (TH) store_pops<R, S>(dst + 9 * plane, plane, oc, A.ref_g, out[NSP - 1]);
            }
#pragma unroll
            for (int s = 0; s < NSP; ++s)
#pragma unroll
                for (int q = 0; q < 6; ++q) Fp[s][q] = Fc[s][q];
        }

        // ---- advance the windows ----
#pragma unroll
        for (int s = 0; s < NSP; ++s) {
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                P3[s][q] = P2[s][q];
                P2[s][q] = P1[s][q];
                P1[s][q] = ph[s][upop(q)];
                M2[s][q] = M1[s][q];
                M1[s][q] = ph[s][dpop(q)];
            }
#pragma unroll
            for (int a = 0; a < 9; ++a) {
                U2[s][a] = U1[s][a];
                U1[s][a] = out_row ? U0[s][a] : R(0);
            }
        }
    }
}

template <class R, class S>
static hipError_t launch_typed(bool thermal, bool corrector, const void* args, int n_strips, int n_chunks,
                               hipStream_t s) {
    const FvArgs<R>& A = *static_cast<const FvArgs<R>*>(args);
    dim3 grid(n_strips, n_chunks), block(FV_LANES);
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

hipError_t launch_fv_pass(int storage, bool thermal, bool corrector, const void* args, int n_strips,
                          int n_chunks, hipStream_t s) {
    switch (storage) {
        case ST_F64: return launch_typed<double, double>(thermal, corrector, args, n_strips, n_chunks, s);
        case ST_F32: return launch_typed<float, float>(thermal, corrector, args, n_strips, n_chunks, s);
        case ST_BF16: return launch_typed<float, bf16_t>(thermal, corrector, args, n_strips, n_chunks, s);
        case ST_F16: return launch_typed<float, f16_t>(thermal, corrector, args, n_strips, n_chunks, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace lbk
