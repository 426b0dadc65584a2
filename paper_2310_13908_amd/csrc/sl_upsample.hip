// sl_upsample.hip -- the upsampling step around the sum (Sec. 3.4, "Upsampling"; the
// right-hand-side algorithm of Sec. 3.6, its upsampling, single-layer and downsampling steps):
//
//   u = I_d S^{delta_u}[I_u f]  evaluated on the upsampled surface X_u = I_u X,
//
// with I_u, I_d per-patch cubic-spline interpolation between the n x n grid of a patch and a grid
// of factor n x factor n nodes (parameters j pi / (n + 1) and j pi / (factor n + 1), j >= 1; the
// fine count is factor^2 N, the count of the paper's upsampling table).  The nodes, the density and
// the area element are upsampled by the same operator (X_u = I_u X, F_u = I_u F, W_u = I_u W), and
// the fine weights are w_u = psi_u W_u h_u^2 (eq. (smoothint) on the fine grid, with the POU values
// psi_u of the fine nodes given by the caller); delta_u is eq. (regparam) on the fine grid.
//
// Splines: not-a-knot cubic splines (de Boor's default) on the uniform parameter grid; the end
// pieces are extended where the fine grid reaches past the first or last coarse node.  Each 1-D
// operator is a dense matrix built on the host once per (n, factor) and kept on the device;
// a field on a patch resamples as A F B^T (two small kernels).
#include <math.h>

#include <vector>

#include "sl_internal.h"

namespace sl {

namespace {

// Second derivatives M of the not-a-knot cubic spline through y on the uniform grid of spacing
// h (N >= 4).  The not-a-knot rows M0 - 2 M1 + M2 = 0 (and at the other end) turn the first and
// last interior rows into 6 M1 = r1 and 6 M_{N-2} = r_{N-2}; the rows in between are tridiagonal.
void notaknot_moments(const std::vector<double> &y, double h, std::vector<double> &M)
{
    const int N = (int)y.size();
    std::vector<double> r(N, 0.0);
    for (int j = 1; j + 1 < N; ++j) r[j] = 6.0 * (y[j - 1] - 2.0 * y[j] + y[j + 1]) / (h * h);
    M.assign(N, 0.0);
    M[1] = r[1] / 6.0;
    M[N - 2] = r[N - 2] / 6.0;
    // rows 2..N-3: M_{j-1} + 4 M_j + M_{j+1} = r_j, with M_1 and M_{N-2} known (Thomas)
    const int lo = 2, hi = N - 3;
    if (hi >= lo) {
        const int m = hi - lo + 1;
        std::vector<double> c(m), d(m);
        for (int k = 0; k < m; ++k) {
            const int j = lo + k;
            double rhs = r[j];
            if (j == lo) rhs -= M[1];
            if (j == hi) rhs -= M[N - 2];
            const double b = 4.0 - (k > 0 ? c[k - 1] : 0.0);
            c[k] = 1.0 / b;
            d[k] = (rhs - (k > 0 ? d[k - 1] : 0.0)) / b;
        }
        for (int k = m - 1; k >= 0; --k) M[lo + k] = d[k] - (k + 1 < m ? c[k] * M[lo + k + 1] : 0.0);
    }
    M[0] = 2.0 * M[1] - M[2];
    M[N - 1] = 2.0 * M[N - 2] - M[N - 3];
}

// Matrix (rows = targets t_a, columns = data nodes) of the spline through unit data vectors on the
// nodes (j + 1) h, j = 0..N-1, evaluated at the targets.
std::vector<double> spline_matrix(int N, double h, const std::vector<double> &t)
{
    const int T = (int)t.size();
    std::vector<double> A((size_t)T * N, 0.0), y(N), M;
    for (int j = 0; j < N; ++j) {
        std::fill(y.begin(), y.end(), 0.0);
        y[j] = 1.0;
        notaknot_moments(y, h, M);
        for (int a = 0; a < T; ++a) {
            int k = (int)floor(t[a] / h) - 1;          // interval [(k+1) h, (k+2) h]
            k = k < 0 ? 0 : (k > N - 2 ? N - 2 : k);
            const double tk = (k + 1) * h, tk1 = (k + 2) * h;
            const double L = tk1 - t[a], R = t[a] - tk;
            const double ck = y[k] / h - M[k] * h / 6.0, ck1 = y[k + 1] / h - M[k + 1] * h / 6.0;
            A[(size_t)a * N + j] =
                M[k] * L * L * L / (6.0 * h) + M[k + 1] * R * R * R / (6.0 * h) + ck * L + ck1 * R;
        }
    }
    return A;
}

// G[p] = A F[p] B^T for every patch p: F (n_from x n_from), A and B (n_to x n_from).  Stage 1:
// T[p][j][b] = sum_k F[p][j][k] B[b][k]; stage 2: G[p][a][b] = sum_j A[a][j] T[p][j][b].
__global__ __launch_bounds__(256) void k_resample_cols(int64_t n_patches, int nf, int nt,
                                                       const double *__restrict__ F,
                                                       const double *__restrict__ B,
                                                       double *__restrict__ T)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (p, j, b)
    if (e >= n_patches * nf * nt) return;
    const int b = (int)(e % nt);
    const int64_t pj = e / nt;                                          // p * nf + j
    const double *f = F + pj * nf, *w = B + (int64_t)b * nf;
    double s = 0.0;
    for (int k = 0; k < nf; ++k) s = fma(f[k], w[k], s);
    T[e] = s;
}

__global__ __launch_bounds__(256) void k_resample_rows(int64_t n_patches, int nf, int nt,
                                                       const double *__restrict__ T,
                                                       const double *__restrict__ A,
                                                       double *__restrict__ G)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (p, a, b)
    if (e >= n_patches * nt * nt) return;
    const int b = (int)(e % nt);
    const int a = (int)((e / nt) % nt);
    const int64_t p = e / ((int64_t)nt * nt);
    const double *t = T + p * nf * nt + b, *w = A + (int64_t)a * nf;
    double s = 0.0;
    for (int j = 0; j < nf; ++j) s = fma(w[j], t[(int64_t)j * nt], s);
    G[e] = s;
}

// w = psi W_u h^2 per fine node.
__global__ __launch_bounds__(256) void k_fine_weights(int64_t n, const double *__restrict__ psi,
                                                      const double *__restrict__ Wu, double h2,
                                                      double *__restrict__ w)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    w[p] = psi[p] * Wu[p] * h2;
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

// Resample one field of every patch: G = A F B^T, T scratch of n_patches * nf * nt.
hipError_t resample(int64_t n_patches, int nf, int nt, const double *F, const double *A, const double *B,
                    double *T, double *G, hipStream_t st)
{
    hipLaunchKernelGGL(k_resample_cols, dim3(blocks_for(n_patches * nf * nt)), dim3(256), 0, st, n_patches,
                       nf, nt, F, B, T);
    hipLaunchKernelGGL(k_resample_rows, dim3(blocks_for(n_patches * nt * nt)), dim3(256), 0, st, n_patches,
                       nf, nt, T, A, G);
    return hipGetLastError();
}

}  // namespace

}  // namespace sl

using namespace sl;

extern "C" {

sl_status sl_eval_upsampled(sl_ctx *ctx, sl_precision prec, int64_t n_patches, int64_t n, int factor,
                            const double *x, const double *y, const double *z, const double *W,
                            const double *psi_up, const double *fx, const double *fy, const double *fz,
                            double C, double mu, double *ux, double *uy, double *uz, void *stream)
{
    if (!ctx) return fail(SL_EINVAL, "sl_eval_upsampled: ctx is NULL");
    if (prec != SL_FP64 && prec != SL_MIXED) return fail(SL_EINVAL, "sl_eval_upsampled: unknown precision");
    if (n_patches < 1 || n < 4 || n > 4096 || factor < 1 || factor > 8)
        return fail(SL_EINVAL, "sl_eval_upsampled: need n_patches >= 1, 4 <= n <= 4096, 1 <= factor <= 8");
    const int64_t nf = (int64_t)factor * n;
    if (n_patches > ((int64_t)1 << 30) / (nf * nf)) return fail(SL_EINVAL, "sl_eval_upsampled: more than 2^30 fine points");
    if (!(isfinite(C) && C > 0.0) || !(isfinite(mu) && mu > 0.0))
        return fail(SL_EINVAL, "sl_eval_upsampled: C and mu must be finite and > 0");
    if (!x || !y || !z || !W || !psi_up || !fx || !fy || !fz || !ux || !uy || !uz)
        return fail(SL_EINVAL, "sl_eval_upsampled: NULL array");
    struct Guard {   // the context's device for the call, the caller's afterwards
        int prev = -1;
        ~Guard() { if (prev >= 0) (void)hipSetDevice(prev); }
    } guard;
    if (hipGetDevice(&guard.prev) != hipSuccess) guard.prev = -1;
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(SL_EHIP, "sl_eval_upsampled: hipSetDevice failed");
    const hipStream_t st = (hipStream_t)stream;
    // spline matrices for (n, factor): up (nf x n), down (n x nf)
    double *mats = nullptr;
    {
        std::lock_guard<std::mutex> l(ctx->mu);
        const int64_t key = n * 16 + factor;
        auto it = ctx->splines.find(key);
        if (it != ctx->splines.end()) {
            mats = it->second;
        } else {
            const double hc = M_PI / (double)(n + 1), hf = M_PI / (double)(nf + 1);
            std::vector<double> tf(nf), tc(n);
            for (int64_t a = 0; a < nf; ++a) tf[a] = (a + 1) * hf;
            for (int64_t a = 0; a < n; ++a) tc[a] = (a + 1) * hc;
            const std::vector<double> U = spline_matrix((int)n, hc, tf);
            const std::vector<double> D = spline_matrix((int)nf, hf, tc);
            std::vector<double> all;
            all.reserve(U.size() + D.size());
            all.insert(all.end(), U.begin(), U.end());
            all.insert(all.end(), D.begin(), D.end());
            hipError_t e = hipMalloc(&mats, all.size() * sizeof(double));
            if (e == hipSuccess) e = hipMemcpy(mats, all.data(), all.size() * sizeof(double), hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                if (mats) (void)hipFree(mats);
                return hip_fail(e, "sl_eval_upsampled: spline matrices");
            }
            ctx->splines[key] = mats;
        }
    }
    const double *U = mats, *D = mats + nf * n;
    const int64_t Nf = n_patches * nf * nf;
    // workspace: 9 fine fields (x, y, z, W, f (3), w, delta) and u (3); scratch T
    const int64_t scratch = n_patches * nf * nf;     // >= n_patches * n * nf and n_patches * nf * n
    void *base = nullptr;
    hipError_t e = ws_alloc(ctx, &base, (size_t)(12 * Nf + scratch) * sizeof(double), st);
    if (e != hipSuccess) return hip_fail(e, "sl_eval_upsampled: workspace");
    double *Ws = static_cast<double *>(base);
    double *X[3] = {Ws, Ws + Nf, Ws + 2 * Nf}, *Wu = Ws + 3 * Nf;
    double *Fu[3] = {Ws + 4 * Nf, Ws + 5 * Nf, Ws + 6 * Nf};
    double *wu = Ws + 7 * Nf, *du = Ws + 8 * Nf, *Uu[3] = {Ws + 9 * Nf, Ws + 10 * Nf, Ws + 11 * Nf};
    double *T = Ws + 12 * Nf;
    const double *xin[3] = {x, y, z}, *fin[3] = {fx, fy, fz};
    double *uout[3] = {ux, uy, uz};
    for (int c = 0; c < 3 && e == hipSuccess; ++c) {
        e = resample(n_patches, (int)n, (int)nf, xin[c], U, U, T, X[c], st);
        if (e == hipSuccess) e = resample(n_patches, (int)n, (int)nf, fin[c], U, U, T, Fu[c], st);
    }
    if (e == hipSuccess) e = resample(n_patches, (int)n, (int)nf, W, U, U, T, Wu, st);
    const double hf = M_PI / (double)(nf + 1);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_fine_weights, dim3(blocks_for(Nf)), dim3(256), 0, st, Nf, psi_up, Wu, hf * hf, wu);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = launch_patch_delta(n_patches, nf, X[0], X[1], X[2], C, du, st);
    sl_status s = SL_OK;
    if (e == hipSuccess)
        s = sl_eval(ctx, prec, Nf, X[0], X[1], X[2], wu, Fu[0], Fu[1], Fu[2], Nf, nullptr, nullptr, nullptr, 0.0,
                    du, mu, Uu[0], Uu[1], Uu[2], stream);
    for (int c = 0; c < 3 && e == hipSuccess && s == SL_OK; ++c)
        e = resample(n_patches, (int)nf, (int)n, Uu[c], D, D, T, uout[c], st);
    const hipError_t ef = hipFreeAsync(base, st);
    if (s != SL_OK) return s;
    if (e != hipSuccess) return hip_fail(e, "sl_eval_upsampled: kernel launch");
    if (ef != hipSuccess) return hip_fail(ef, "sl_eval_upsampled: hipFreeAsync");
    return SL_OK;
}

}  // extern "C"
