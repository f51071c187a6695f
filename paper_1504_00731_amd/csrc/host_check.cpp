// Host build of the kernels' per-interface arithmetic (wt_flux.hpp and the
// headers it includes), for CPU tests of that arithmetic without a GPU.  The
// loops below only gather each interface's stencil with the kernels' boundary
// index maps and take flux differences in the kernels' order; every FP64
// operation on the data is the one the device code performs.
#include <cstdint>
#include <cstdlib>
#include <vector>

#include "wt_bc.hpp"
#include "wt_flux.hpp"
#include "wt_pack.hpp"

namespace {

using wt::map_index;
using wt::reflected;

template <int NDIM>
struct HostStencil {
    double uu[6][NDIM + 2], ff[6][NDIM + 2], vv[6][NDIM], ss[6], hh[6], pp[6];
    static constexpr bool kPressure = true;
    double U(int k, int c) const { return uu[k][c]; }
    double f(int k, int c) const { return ff[k][c]; }
    double p(int k) const { return pp[k]; }
    double v(int k, int d) const { return vv[k][d]; }
    double sr(int k) const { return ss[k]; }
    double H(int k) const { return hh[k]; }
};

struct HostSpeeds {
    const double *al;
    bool walls;
    double operator()(int s) const
    {
        return wt::split_speed([this](int k) { return al[k]; }, s, walls);
    }
};

struct HostScalar {
    double uu[6], ff[6];
    double u(int k) const { return uu[k]; }
    double f(int k) const { return ff[k]; }
};

template <int NDIM, int DIR, int PREC>
int euler_sweep(const int64_t *n, double dx, int bc, const double *al, double gamma, double eps,
                double aR, const double *u, double *D, bool first)
{
    constexpr bool FAST = wt::fast_math<PREC>();
    constexpr int M = NDIM + 2;
    const int64_t N = n[0] * n[1] * n[2];
    const int64_t nd = n[DIR];
    const int64_t sd = DIR == 0 ? 1 : (DIR == 1 ? n[0] : n[0] * n[1]);
    std::vector<double> F((size_t)(nd + 1) * M);
    int bad = 0;
    for (int64_t cell = 0; cell < N; ++cell) {
        const int64_t coord = (cell / sd) % nd;
        if (coord != 0) continue;                 // one pass per pencil
        const int64_t base = cell;
        for (int64_t i = -1; i < nd; ++i) {
            HostStencil<NDIM> S;
            for (int k = 0; k < 6; ++k) {
                const int64_t idx = base + map_index(i - 2 + k, nd, bc) * sd;
                double uc[M];
                for (int c = 0; c < M; ++c) uc[c] = u[c * N + idx];
                if (reflected(i - 2 + k, nd, bc)) uc[1 + DIR] = -uc[1 + DIR];
                double p, H;
                if (!wt::euler_cell<NDIM, FAST>(uc, gamma, S.vv[k], p, H)) bad = 1;
                for (int c = 0; c < M; ++c) S.uu[k][c] = uc[c];
                wt::euler_normal_flux<NDIM, DIR>(uc, S.vv[k], p, S.ff[k]);
                S.ss[k] = FAST ? wt::sqrt_fast(uc[0]) : wt::sqrt_rn(uc[0]);
                S.hh[k] = H;
                S.pp[k] = p;
            }
            if (!wt::euler_interface_flux<NDIM, DIR, PREC>(S, HostSpeeds{al, bc == WT_REFLECTIVE}, gamma,
                                                        wt::WenoConst{eps, aR, 1.0 / eps},
                                                        &F[(i + 1) * M]))
                bad = 1;
        }
        for (int64_t i = 0; i < nd; ++i)
            for (int c = 0; c < M; ++c) {
                const double Dd = FAST ? (F[(i + 1) * M + c] - F[i * M + c]) * (1.0 / dx)
                                       : wt::div_rn(F[(i + 1) * M + c] - F[i * M + c], dx);
                const int64_t o = c * N + base + i * sd;
                D[o] = first ? Dd : D[o] + Dd;
            }
    }
    return bad;
}

}  // namespace

extern "C" {

// The finishing steps of the device division and square root, for tests.
double wth_div_finish(double q, double a, double b) { return wt::div_finish(q, a, b); }
double wth_sqrt_finish(double s, double x) { return wt::sqrt_finish(s, x); }
double wth_div_by_recip(double a, double b, double y) { return wt::div_by_recip(a, b, y); }
double wth_div_by_recip_checked(double a, double b, double y)
{
    return wt::div_by_recip_checked(a, b, y);
}
double wth_recip_refine(double b, double y0) { return wt::recip_refine(b, y0); }

// The boundary index map and mirror flag, for CPU checks of their range.
int64_t wth_map_index(int64_t i, int64_t n, int bc) { return wt::map_index(i, n, bc); }
int wth_reflected(int64_t i, int64_t n, int bc) { return wt::reflected(i, n, bc) ? 1 : 0; }

double wth_weno_fp32(const double *s, double eps, double aR)
{
    return wt::weno_theta_fp32_recon(s, eps, (float)aR);
}

double wth_weno(const double *s, double eps, double aR)
{
    return wt::weno_theta(s[0], s[1], s[2], s[3], s[4], s[5], eps, aR, 1.0 / eps);
}

double wth_weno_fast(const double *s, double eps, double aR)
{
    return wt::weno_theta_fast(s[0], s[1], s[2], s[3], s[4], s[5], eps, aR);
}

// The packed-chunk rules of the batched 2D passes, for CPU checks of their tables:
// the chunks of nl lines of W interfaces (at most cap; returns their number), and
// the staged rows, stencil base and staged point of a chunk.
int wth_pack_chunks(int W, int nl, int qt, int rmax, int32_t *q0, int32_t *nq, int cap)
{
    int k = 0;
    wt::pack_chunks(W, nl, qt, rmax, [&](int a, int n) {
        if (k < cap) {
            q0[k] = a;
            nq[k] = n;
        }
        ++k;
    });
    return k;
}
void wth_pack_limits(int *lim)
{
    lim[0] = wt::kPackLanes;
    lim[1] = wt::kPackQt;
    lim[2] = wt::kPackRows;
}
int wth_pack_rows(int q0, int nq, int W) { return wt::pack_rows(q0, nq, W); }
int wth_pack_base(int q0, int q, int W) { return wt::pack_base(q0, q, W); }
void wth_pack_point(int q0, int row, int W, int *line, int *g) { wt::pack_point(q0, row, W, line, g); }

}  // extern "C"

namespace {

template <int PREC>
int host_rhs(int sys, int ndim, const int64_t *n, const double *dx, const int *bc,
             const double *alpha, double gamma, double eps, double aR, const double *u,
             const double *f, double *L, const double *grav)
{
    if (sys != 2) {
        const int64_t nn = n[0];
        std::vector<double> F((size_t)nn + 1);
        for (int64_t i = -1; i < nn; ++i) {
            HostScalar S;
            for (int k = 0; k < 6; ++k) {
                const int64_t idx = map_index(i - 2 + k, nn, bc[0]);
                S.uu[k] = u[idx];
                S.ff[k] = f[idx];
            }
            F[i + 1] = wt::scalar_interface_flux<PREC>(S, alpha[0], wt::WenoConst{eps, aR, 1.0 / eps});
        }
        for (int64_t i = 0; i < nn; ++i) L[i] = -wt::div_rn(F[i + 1] - F[i], dx[0]);
        return 0;
    }
    const int M = ndim + 2;
    const int64_t N = n[0] * n[1] * n[2];
    std::vector<double> D((size_t)N * M);
    int bad = 0;
    if (ndim == 1) {
        bad |= euler_sweep<1, 0, PREC>(n, dx[0], bc[0], alpha, gamma, eps, aR, u, D.data(), true);
    } else if (ndim == 2) {
        bad |= euler_sweep<2, 0, PREC>(n, dx[0], bc[0], alpha, gamma, eps, aR, u, D.data(), true);
        bad |= euler_sweep<2, 1, PREC>(n, dx[1], bc[1], alpha + 5, gamma, eps, aR, u, D.data(), false);
    } else {
        bad |= euler_sweep<3, 0, PREC>(n, dx[0], bc[0], alpha, gamma, eps, aR, u, D.data(), true);
        bad |= euler_sweep<3, 1, PREC>(n, dx[1], bc[1], alpha + 5, gamma, eps, aR, u, D.data(), false);
        bad |= euler_sweep<3, 2, PREC>(n, dx[2], bc[2], alpha + 10, gamma, eps, aR, u, D.data(), false);
    }
    for (int64_t k = 0; k < N * M; ++k) L[k] = -D[k];
    if (grav && (grav[0] != 0.0 || grav[1] != 0.0 || grav[2] != 0.0))
        for (int64_t j = 0; j < N; ++j) {
            // the final sweep's source term, in its order
            const double rho = u[j];
            double e = 0.0;
            for (int d = 0; d < ndim; ++d) {
                const double md = u[(1 + d) * N + j];
                L[(1 + d) * N + j] = L[(1 + d) * N + j] + (-(grav[d] * rho));
                e = d == 0 ? grav[0] * md : e + grav[d] * md;
            }
            L[(ndim + 1) * N + j] = L[(ndim + 1) * N + j] + (-e);
        }
    return bad;
}

}  // namespace

extern "C" {

// Full L(u) for the Euler equations (alpha: [ndim][5] LF speeds per field) or
// for a 1D scalar state with given flux values f (alpha[0]), in precision mode
// prec (0: plain FP64 order, 1: FP32 reconstruction, 2: fast FP64).
int wth_rhs(int prec, int sys, int ndim, const int64_t *n, const double *dx, const int *bc,
            const double *alpha, double gamma, double eps, double aR, const double *u,
            const double *f, double *L, const double *grav)
{
    if (prec == 1) return host_rhs<1>(sys, ndim, n, dx, bc, alpha, gamma, eps, aR, u, f, L, grav);
    if (prec == 2) return host_rhs<2>(sys, ndim, n, dx, bc, alpha, gamma, eps, aR, u, f, L, grav);
    return host_rhs<0>(sys, ndim, n, dx, bc, alpha, gamma, eps, aR, u, f, L, grav);
}

}  // extern "C"
