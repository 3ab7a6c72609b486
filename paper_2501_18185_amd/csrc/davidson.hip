// Block Davidson-Liu over mw_sigma (the paper diagonalises through products
// sigma = H X that use only the nonzero elements of H, recomputed each time;
// section 2.4).  The host drives the iteration; every operation over N-long
// vectors runs in the kernels below, and only m x m subspace data crosses to
// the host once per step.
//
// Iteration (lowest nroots roots):
//   V orthonormal basis (vector-major [m][N]), W = H V.
//   G = V^H W (m x m, Hermitian) -> eigenpairs (theta_k, y_k), lowest nroots.
//   X_k = V y_k, AX_k = W y_k, r_k = AX_k - theta_k X_k; stop when every
//   ||r_k||_2 <= tol.  t_k = r_k / (theta_k - H_II) (|denominator| >= 1e-12,
//   sign kept); two passes of Gram-Schmidt against V; drop ||t|| < 1e-10.
//   Collapse V to the Ritz vectors when it would exceed max(8 nroots, 24).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <functional>
#include <vector>

#include "dev_common.h"
#include "mw_internal.h"

namespace mw {

namespace {

constexpr int DOT_BLOCKS = 256;

// partial[b][q] = sum over this block's slice of conj(X_{a_q}) Y_{b_q}
template <bool CPLX>
__global__ __launch_bounds__(256) void k_dots(const typename Scal<CPLX>::T *X, const typename Scal<CPLX>::T *Y,
                                              int64_t N, const int *ia, const int *ib, int npairs,
                                              typename Scal<CPLX>::T *partial)
{
    using T = typename Scal<CPLX>::T;
    __shared__ T red[256];
    for (int q = 0; q < npairs; q++) {
        const T *x = X + (size_t)ia[q] * N;
        const T *y = Y + (size_t)ib[q] * N;
        T acc = sc_zero(T());
        for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < N; t += (int64_t)gridDim.x * blockDim.x)
            acc = sc_add(acc, sc_mul(sc_conj(x[t]), y[t]));
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] = sc_add(red[threadIdx.x], red[threadIdx.x + s]);
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[(size_t)blockIdx.x * npairs + q] = red[0];
        __syncthreads();
    }
}

// out_k = beta_k * out_k + sum_a coef[a][k] X_a   for k < nout (out vectors
// are rows of OUT starting at out0)
template <bool CPLX>
__global__ __launch_bounds__(256) void k_lincomb(const typename Scal<CPLX>::T *X, int na, int64_t N,
                                                 const typename Scal<CPLX>::T *coef, int nout,
                                                 typename Scal<CPLX>::T *OUT, const double *beta)
{
    using T = typename Scal<CPLX>::T;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < N; t += (int64_t)gridDim.x * blockDim.x) {
        for (int k = 0; k < nout; k++) {
            T acc = sc_zero(T());
            for (int a = 0; a < na; a++) acc = sc_add(acc, sc_mul(coef[a * nout + k], X[(size_t)a * N + t]));
            T o = acc;
            if (beta[k] != 0.0) {  // never read OUT when it is overwritten
                const T prev = OUT[(size_t)k * N + t];
                if constexpr (CPLX) o = make_double2(beta[k] * prev.x + acc.x, beta[k] * prev.y + acc.y);
                else o = beta[k] * prev + acc;
            }
            OUT[(size_t)k * N + t] = o;
        }
    }
}

// t = r / (theta - H_II) with the denominator clamped
template <bool CPLX>
__global__ __launch_bounds__(256) void k_precond(const typename Scal<CPLX>::T *Rv, const typename Scal<CPLX>::T *diag,
                                                 double theta, int64_t N, typename Scal<CPLX>::T *T_out)
{
    using T = typename Scal<CPLX>::T;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < N; t += (int64_t)gridDim.x * blockDim.x) {
        double dg;
        if constexpr (CPLX) dg = diag[t].x;
        else dg = diag[t];
        double den = theta - dg;
        if (fabs(den) < 1e-12) den = den < 0 ? -1e-12 : 1e-12;
        T r = Rv[t];
        if constexpr (CPLX) T_out[t] = make_double2(r.x / den, r.y / den);
        else T_out[t] = r / den;
    }
}

// vector-major [m][N] <-> interleaved [N][m]
template <typename T>
__global__ __launch_bounds__(256) void k_pack(const T *src, int m, int64_t N, T *dst, int to_interleaved)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < (int64_t)m * N;
         t += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = t / m;
        int k = (int)(t - i * m);
        if (to_interleaved) dst[t] = src[(size_t)k * N + i];
        else dst[(size_t)k * N + i] = src[t];
    }
}

using cd = std::complex<double>;

// cyclic Jacobi for a Hermitian m x m matrix (row-major); eigenvalues
// ascending in w, eigenvectors in the columns of V
static void jacobi_eigh(int m, std::vector<cd> A, std::vector<double> &w, std::vector<cd> &V)
{
    V.assign((size_t)m * m, cd(0));
    for (int i = 0; i < m; i++) V[(size_t)i * m + i] = 1.0;
    for (int sweep = 0; sweep < 100; sweep++) {
        double off = 0, dn = 0;
        for (int i = 0; i < m; i++)
            for (int j = 0; j < m; j++) (i == j ? dn : off) += std::norm(A[(size_t)i * m + j]);
        if (off <= 1e-30 * std::max(dn, 1e-300)) break;
        for (int p = 0; p < m; p++)
            for (int q = p + 1; q < m; q++) {
                cd apq = A[(size_t)p * m + q];
                double a = std::abs(apq);
                if (a < 1e-300) continue;
                double app = A[(size_t)p * m + p].real(), aqq = A[(size_t)q * m + q].real();
                cd ph = apq / a;  // e^{i phi}
                double tau = (aqq - app) / (2 * a);
                double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1 + tau * tau));
                double c = 1 / std::sqrt(1 + t * t), s = t * c;
                // rotation J: columns p, q: [c, s ph; -s conj(ph), c]
                for (int k = 0; k < m; k++) {
                    cd akp = A[(size_t)k * m + p], akq = A[(size_t)k * m + q];
                    A[(size_t)k * m + p] = c * akp - s * std::conj(ph) * akq;
                    A[(size_t)k * m + q] = s * ph * akp + c * akq;
                }
                for (int k = 0; k < m; k++) {
                    cd apk = A[(size_t)p * m + k], aqk = A[(size_t)q * m + k];
                    A[(size_t)p * m + k] = c * apk - s * ph * aqk;
                    A[(size_t)q * m + k] = s * std::conj(ph) * apk + c * aqk;
                }
                for (int k = 0; k < m; k++) {
                    cd vkp = V[(size_t)k * m + p], vkq = V[(size_t)k * m + q];
                    V[(size_t)k * m + p] = c * vkp - s * std::conj(ph) * vkq;
                    V[(size_t)k * m + q] = s * ph * vkp + c * vkq;
                }
            }
    }
    std::vector<int> idx(m);
    for (int i = 0; i < m; i++) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(),
                     [&](int a, int b) { return A[(size_t)a * m + a].real() < A[(size_t)b * m + b].real(); });
    std::vector<cd> V2((size_t)m * m);
    w.resize(m);
    for (int j = 0; j < m; j++) {
        w[j] = A[(size_t)idx[j] * m + idx[j]].real();
        for (int k = 0; k < m; k++) V2[(size_t)k * m + j] = V[(size_t)k * m + idx[j]];
    }
    V = V2;
}

template <bool CPLX>
struct Davidson {
    using T = typename Scal<CPLX>::T;
    // sigma of k packed vectors ([N][k] in, [N][k] out) on stream s
    std::function<mw_status(int, const T *, T *)> sigma;
    const T *diag;   // [N] preconditioner diagonal (device)
    hipStream_t s;
    int R, mmax;
    int64_t N;
    // device buffers carved from the caller's work area
    T *V, *W, *X, *AX, *Rv, *Tn, *packA, *packB, *coef, *dpart;
    double *beta;
    int *ia, *ib;
    std::vector<cd> Gh;  // host subspace matrix (mmax x mmax)

    static size_t bytes(int R, int64_t N) { return bytes_m(std::max(8 * R, 24) + R, R, N); }

    // the same buffers for a basis of at most mmax vectors
    static size_t bytes_m(int mmax, int R, int64_t N)
    {
        const size_t sb = sizeof(T);
        size_t b = 0;
        auto take = [&](size_t x) { b = (b + 255) & ~(size_t)255; b += x; };
        take((size_t)mmax * N * sb);        // V
        take((size_t)mmax * N * sb);        // W
        take((size_t)R * N * sb);           // X
        take((size_t)R * N * sb);           // AX
        take((size_t)R * N * sb);           // residuals
        take((size_t)R * N * sb);           // new vectors
        take((size_t)R * N * sb);           // packed in
        take((size_t)R * N * sb);           // packed out
        take((size_t)mmax * mmax * sb);     // coefficients
        take((size_t)DOT_BLOCKS * mmax * R * sb);  // dot partials
        take((size_t)mmax * 8);             // beta
        take((size_t)2 * mmax * R * 4);     // pair indices
        return b + 256;
    }

    void carve(char *base)
    {
        size_t off = 0;
        const size_t sb = sizeof(T);
        auto take = [&](size_t x) { off = (off + 255) & ~(size_t)255; char *p = base + off; off += x; return p; };
        V = (T *)take((size_t)mmax * N * sb);
        W = (T *)take((size_t)mmax * N * sb);
        X = (T *)take((size_t)R * N * sb);
        AX = (T *)take((size_t)R * N * sb);
        Rv = (T *)take((size_t)R * N * sb);
        Tn = (T *)take((size_t)R * N * sb);
        packA = (T *)take((size_t)R * N * sb);
        packB = (T *)take((size_t)R * N * sb);
        coef = (T *)take((size_t)mmax * mmax * sb);
        dpart = (T *)take((size_t)DOT_BLOCKS * mmax * R * sb);
        beta = (double *)take((size_t)mmax * 8);
        ia = (int *)take((size_t)mmax * R * 4);
        ib = (int *)take((size_t)mmax * R * 4);
    }

    static cd to_c(double x) { return cd(x, 0); }
    static cd to_c(double2 x) { return cd(x.x, x.y); }
    static void from_c(cd v, double &x) { x = v.real(); }
    static void from_c(cd v, double2 &x) { x = make_double2(v.real(), v.imag()); }

    unsigned grid() const { return (unsigned)std::min<int64_t>((N + 255) / 256, 4096); }

    // dots conj(A_{a_q}) . B_{b_q} for the given pairs; blocking
    bool dots(const T *A, const T *B, const std::vector<int> &a, const std::vector<int> &b, std::vector<cd> &out)
    {
        const int np = (int)a.size();
        out.assign(np, cd(0));
        if (!np) return true;
        for (int c0 = 0; c0 < np; c0 += mmax * R) {
            int cnt = std::min(np - c0, mmax * R);
            if (hipMemcpyAsync(ia, a.data() + c0, cnt * 4, hipMemcpyHostToDevice, s) != hipSuccess) return false;
            if (hipMemcpyAsync(ib, b.data() + c0, cnt * 4, hipMemcpyHostToDevice, s) != hipSuccess) return false;
            hipLaunchKernelGGL(k_dots<CPLX>, dim3(DOT_BLOCKS), dim3(256), 0, s, A, B, N, ia, ib, cnt, dpart);
            std::vector<T> h((size_t)DOT_BLOCKS * cnt);
            if (hipMemcpyAsync(h.data(), dpart, h.size() * sizeof(T), hipMemcpyDeviceToHost, s) != hipSuccess)
                return false;
            if (hipStreamSynchronize(s) != hipSuccess) return false;
            for (int q = 0; q < cnt; q++) {
                cd acc = 0;
                for (int blk = 0; blk < DOT_BLOCKS; blk++) acc += to_c(h[(size_t)blk * cnt + q]);
                out[c0 + q] = acc;
            }
        }
        return true;
    }

    // OUT_k = beta_k OUT_k + sum_a C[a][k] X_a
    bool lincomb(const T *Xs, int na, const std::vector<cd> &C, int nout, T *OUT, const std::vector<double> &bt)
    {
        std::vector<T> ch((size_t)na * nout);
        for (size_t i = 0; i < ch.size(); i++) from_c(C[i], ch[i]);
        if (na && hipMemcpyAsync(coef, ch.data(), ch.size() * sizeof(T), hipMemcpyHostToDevice, s) != hipSuccess)
            return false;
        if (hipMemcpyAsync(beta, bt.data(), nout * 8, hipMemcpyHostToDevice, s) != hipSuccess) return false;
        hipLaunchKernelGGL(k_lincomb<CPLX>, dim3(grid()), dim3(256), 0, s, Xs, na, N, coef, nout, OUT, beta);
        // the host arrays must stay valid until the copies ran
        return hipStreamSynchronize(s) == hipSuccess;
    }

    // W rows [first, first+k) = H V rows [first, first+k)
    mw_status apply_h(int first, int k)
    {
        hipLaunchKernelGGL(k_pack<T>, dim3(grid()), dim3(256), 0, s, V + (size_t)first * N, k, N, packA, 1);
        mw_status st = sigma(k, packA, packB);
        if (st != MW_OK) return st;
        hipLaunchKernelGGL(k_pack<T>, dim3(grid()), dim3(256), 0, s, packB, k, N, W + (size_t)first * N, 0);
        return MW_OK;
    }

    // Gram-Schmidt of row `row` of V against rows [0, row); returns the norm
    bool orthonormalize(int row, double &norm)
    {
        T *t = V + (size_t)row * N;
        for (int pass = 0; pass < 2 && row > 0; pass++) {
            std::vector<int> a(row), b(row, row);
            for (int i = 0; i < row; i++) a[i] = i;
            std::vector<cd> ov;
            if (!dots(V, V, a, b, ov)) return false;
            std::vector<cd> C(row);
            for (int i = 0; i < row; i++) C[i] = -ov[i];
            if (!lincomb(V, row, C, 1, t, std::vector<double>{1.0})) return false;
        }
        std::vector<cd> nn;
        if (!dots(V, V, std::vector<int>{row}, std::vector<int>{row}, nn)) return false;
        norm = std::sqrt(std::max(nn[0].real(), 0.0));
        if (norm >= 1e-10) {
            std::vector<cd> C;
            if (!lincomb(V, 0, C, 1, t, std::vector<double>{1.0 / norm})) return false;
        }
        return true;
    }

    mw_status run(const void *c0, void *c_out, double *evals, double tol, int max_iter, int *iters)
    {
        const int msub = std::max(8 * R, 24);
        Gh.assign((size_t)mmax * mmax, cd(0));
        // start: orthonormalised c0
        hipLaunchKernelGGL(k_pack<T>, dim3(grid()), dim3(256), 0, s, (const T *)c0, R, N, V, 0);
        int m = 0;
        for (int k = 0; k < R; k++) {
            if (k != m)
                if (hipMemcpyAsync(V + (size_t)m * N, V + (size_t)k * N, N * sizeof(T), hipMemcpyDeviceToDevice, s) !=
                    hipSuccess)
                    return fail(MW_EHIP, "copy failed");
            double nrm;
            if (!orthonormalize(m, nrm)) return fail(MW_EHIP, "Gram-Schmidt failed");
            if (nrm >= 1e-10) m++;
        }
        if (m < R) return fail(MW_EINVAL, "start vectors are linearly dependent");
        mw_status st = apply_h(0, m);
        if (st != MW_OK) return st;
        int newfirst = 0;
        std::vector<double> theta(R);
        std::vector<cd> Y;
        bool converged = false;
        int it = 0;
        for (it = 1; it <= max_iter; it++) {
            // G[a][b] for b in the new rows (and its conjugate mirror)
            std::vector<int> a, b;
            for (int bb = newfirst; bb < m; bb++)
                for (int aa = 0; aa < m; aa++) { a.push_back(aa); b.push_back(bb); }
            std::vector<cd> gv;
            if (!dots(V, W, a, b, gv)) return fail(MW_EHIP, "dot products failed");
            for (size_t q = 0; q < gv.size(); q++) {
                Gh[(size_t)a[q] * mmax + b[q]] = gv[q];
                Gh[(size_t)b[q] * mmax + a[q]] = std::conj(gv[q]);
            }
            std::vector<cd> G((size_t)m * m);
            for (int i = 0; i < m; i++)
                for (int j = 0; j < m; j++)
                    G[(size_t)i * m + j] = 0.5 * (Gh[(size_t)i * mmax + j] + std::conj(Gh[(size_t)j * mmax + i]));
            std::vector<double> w;
            std::vector<cd> E;
            jacobi_eigh(m, G, w, E);
            Y.assign((size_t)m * R, cd(0));
            for (int i = 0; i < m; i++)
                for (int k = 0; k < R; k++) Y[(size_t)i * R + k] = E[(size_t)i * m + k];
            for (int k = 0; k < R; k++) theta[k] = w[k];
            std::vector<double> zero(R, 0.0);
            if (!lincomb(V, m, Y, R, X, zero) || !lincomb(W, m, Y, R, AX, zero)) return fail(MW_EHIP, "Ritz failed");
            // residuals r_k = AX_k - theta_k X_k
            if (hipMemcpyAsync(Rv, AX, (size_t)R * N * sizeof(T), hipMemcpyDeviceToDevice, s) != hipSuccess)
                return fail(MW_EHIP, "copy failed");
            for (int k = 0; k < R; k++) {
                std::vector<cd> C{cd(-theta[k], 0)};
                if (!lincomb(X + (size_t)k * N, 1, C, 1, Rv + (size_t)k * N, std::vector<double>{1.0}))
                    return fail(MW_EHIP, "residual failed");
            }
            std::vector<int> ka(R);
            for (int k = 0; k < R; k++) ka[k] = k;
            std::vector<cd> rn;
            if (!dots(Rv, Rv, ka, ka, rn)) return fail(MW_EHIP, "norms failed");
            bool all = true;
            for (int k = 0; k < R; k++) all = all && std::sqrt(std::max(rn[k].real(), 0.0)) <= tol;
            if (all) { converged = true; break; }
            if (it == max_iter) break;
            // corrections
            int nnew = 0;
            for (int k = 0; k < R; k++) {
                if (std::sqrt(std::max(rn[k].real(), 0.0)) <= tol) continue;
                hipLaunchKernelGGL(k_precond<CPLX>, dim3(grid()), dim3(256), 0, s, Rv + (size_t)k * N,
                                   diag, theta[k], N, Tn + (size_t)nnew * N);
                nnew++;
            }
            if (m + nnew > msub) {
                // collapse onto the Ritz vectors
                if (hipMemcpyAsync(V, X, (size_t)R * N * sizeof(T), hipMemcpyDeviceToDevice, s) != hipSuccess ||
                    hipMemcpyAsync(W, AX, (size_t)R * N * sizeof(T), hipMemcpyDeviceToDevice, s) != hipSuccess)
                    return fail(MW_EHIP, "collapse failed");
                std::fill(Gh.begin(), Gh.end(), cd(0));
                for (int k = 0; k < R; k++) Gh[(size_t)k * mmax + k] = theta[k];
                m = R;
            }
            newfirst = m;
            for (int k = 0; k < nnew; k++) {
                if (hipMemcpyAsync(V + (size_t)m * N, Tn + (size_t)k * N, N * sizeof(T), hipMemcpyDeviceToDevice, s) !=
                    hipSuccess)
                    return fail(MW_EHIP, "copy failed");
                double nrm;
                if (!orthonormalize(m, nrm)) return fail(MW_EHIP, "Gram-Schmidt failed");
                if (nrm >= 1e-10) m++;
            }
            if (m == newfirst) break;  // no new direction: stagnation
            st = apply_h(newfirst, m - newfirst);
            if (st != MW_OK) return st;
        }
        hipLaunchKernelGGL(k_pack<T>, dim3(grid()), dim3(256), 0, s, X, R, N, (T *)c_out, 1);
        if (hipStreamSynchronize(s) != hipSuccess) return fail(MW_EHIP, "final sync failed");
        for (int k = 0; k < R; k++) evals[k] = theta[k];
        *iters = std::min(it, max_iter);
        if (!converged) return fail(MW_ENOCONV, "Davidson did not converge");
        return MW_OK;
    }

    // Gram-Schmidt of row `row` of V against rows [0, row) with the same
    // combination applied to W, so that W stays H V; returns the norm
    bool orthonormalize_vw(int row, double &norm)
    {
        T *t = V + (size_t)row * N, *tw = W + (size_t)row * N;
        for (int pass = 0; pass < 2 && row > 0; pass++) {
            std::vector<int> a(row), b(row, row);
            for (int i = 0; i < row; i++) a[i] = i;
            std::vector<cd> ov;
            if (!dots(V, V, a, b, ov)) return false;
            std::vector<cd> C(row);
            for (int i = 0; i < row; i++) C[i] = -ov[i];
            if (!lincomb(V, row, C, 1, t, std::vector<double>{1.0}) ||
                !lincomb(W, row, C, 1, tw, std::vector<double>{1.0}))
                return false;
        }
        std::vector<cd> nn;
        if (!dots(V, V, std::vector<int>{row}, std::vector<int>{row}, nn)) return false;
        norm = std::sqrt(std::max(nn[0].real(), 0.0));
        if (norm >= 1e-10) {
            std::vector<cd> C;
            if (!lincomb(V, 0, C, 1, t, std::vector<double>{1.0 / norm}) ||
                !lincomb(W, 0, C, 1, tw, std::vector<double>{1.0 / norm}))
                return false;
        }
        return true;
    }

    // Iterative vector interaction over a search space of fixed dimension
    // (at most 3R): the current vectors X, their first-order corrections
    // t_k = (r_k - eps_k x_k) / (theta_k - H_II) (Olsen's choice of eps_k
    // makes t_k orthogonal to x_k) and the directions of the last step
    // P = X_new - X_old (X_old^H X_new), whose H P is carried along.  Each
    // step diagonalises H in that space and keeps R Ritz pairs: the lowest
    // (target NaN) or those nearest the target energy, without the roots
    // below them.  One sigma of the corrections per step (and of the
    // directions in the last steps, see below).  Buffers: V, W
    // rows [0, 3R) for the space, rows [3R, 4R) for P and H P (mmax = 4R).
    mw_status run_ivi(const void *c0, void *c_out, double *evals, double tol, int max_iter, int *iters,
                      double target)
    {
        const bool lowest = std::isnan(target);
        T *Pv = V + (size_t)3 * R * N, *PA = W + (size_t)3 * R * N;
        hipLaunchKernelGGL(k_pack<T>, dim3(grid()), dim3(256), 0, s, (const T *)c0, R, N, V, 0);
        int m = 0;
        for (int k = 0; k < R; k++) {
            if (k != m)
                if (hipMemcpyAsync(V + (size_t)m * N, V + (size_t)k * N, N * sizeof(T), hipMemcpyDeviceToDevice, s) !=
                    hipSuccess)
                    return fail(MW_EHIP, "copy failed");
            double nrm;
            if (!orthonormalize(m, nrm)) return fail(MW_EHIP, "Gram-Schmidt failed");
            if (nrm >= 1e-10) m++;
        }
        if (m < R) return fail(MW_EINVAL, "start vectors are linearly dependent");
        mw_status st = apply_h(0, m);
        if (st != MW_OK) return st;
        int np = 0;
        std::vector<double> theta(R);
        bool converged = false;
        int it = 0;
        for (it = 1; it <= max_iter; it++) {
            // Rayleigh-Ritz in the current space
            std::vector<int> a, b;
            for (int bb = 0; bb < m; bb++)
                for (int aa = 0; aa < m; aa++) { a.push_back(aa); b.push_back(bb); }
            std::vector<cd> gv;
            if (!dots(V, W, a, b, gv)) return fail(MW_EHIP, "dot products failed");
            std::vector<cd> G((size_t)m * m);
            for (size_t q = 0; q < gv.size(); q++) G[(size_t)a[q] * m + b[q]] = gv[q];
            for (int i = 0; i < m; i++)
                for (int j = 0; j < i; j++) {
                    const cd v = 0.5 * (G[(size_t)i * m + j] + std::conj(G[(size_t)j * m + i]));
                    G[(size_t)i * m + j] = v;
                    G[(size_t)j * m + i] = std::conj(v);
                }
            for (int i = 0; i < m; i++) G[(size_t)i * m + i] = cd(G[(size_t)i * m + i].real(), 0.0);
            std::vector<double> w;
            std::vector<cd> E;
            jacobi_eigh(m, G, w, E);
            std::vector<int> sel(m);
            for (int i = 0; i < m; i++) sel[i] = i;
            if (!lowest)
                std::stable_sort(sel.begin(), sel.end(),
                                 [&](int x, int y) { return std::fabs(w[x] - target) < std::fabs(w[y] - target); });
            sel.resize(R);
            std::sort(sel.begin(), sel.end());   // ascending energy among the kept
            std::vector<cd> Y((size_t)m * R), Ytp((size_t)std::max(m - R, 0) * R);
            for (int i = 0; i < m; i++)
                for (int k = 0; k < R; k++) {
                    Y[(size_t)i * R + k] = E[(size_t)i * m + sel[k]];
                    if (i >= R) Ytp[(size_t)(i - R) * R + k] = E[(size_t)i * m + sel[k]];
                }
            for (int k = 0; k < R; k++) theta[k] = w[sel[k]];
            std::vector<double> zero(R, 0.0);
            if (!lincomb(V, m, Y, R, X, zero) || !lincomb(W, m, Y, R, AX, zero)) return fail(MW_EHIP, "Ritz failed");
            np = 0;
            if (m > R) {
                // the step's direction outside the old X (its H P alike)
                if (!lincomb(V + (size_t)R * N, m - R, Ytp, R, Pv, zero) ||
                    !lincomb(W + (size_t)R * N, m - R, Ytp, R, PA, zero))
                    return fail(MW_EHIP, "direction failed");
                np = R;
            }
            if (hipMemcpyAsync(V, X, (size_t)R * N * sizeof(T), hipMemcpyDeviceToDevice, s) != hipSuccess ||
                hipMemcpyAsync(W, AX, (size_t)R * N * sizeof(T), hipMemcpyDeviceToDevice, s) != hipSuccess)
                return fail(MW_EHIP, "copy failed");
            // residuals r_k = AX_k - theta_k X_k
            if (hipMemcpyAsync(Rv, AX, (size_t)R * N * sizeof(T), hipMemcpyDeviceToDevice, s) != hipSuccess)
                return fail(MW_EHIP, "copy failed");
            for (int k = 0; k < R; k++) {
                std::vector<cd> C{cd(-theta[k], 0)};
                if (!lincomb(X + (size_t)k * N, 1, C, 1, Rv + (size_t)k * N, std::vector<double>{1.0}))
                    return fail(MW_EHIP, "residual failed");
            }
            std::vector<int> ka(R);
            for (int k = 0; k < R; k++) ka[k] = k;
            std::vector<cd> rn;
            if (!dots(Rv, Rv, ka, ka, rn)) return fail(MW_EHIP, "norms failed");
            bool all = true;
            for (int k = 0; k < R; k++) all = all && std::sqrt(std::max(rn[k].real(), 0.0)) <= tol;
            if (all) { converged = true; break; }
            if (it == max_iter) break;
            // first-order corrections of the unconverged roots, then the
            // directions of the last step
            m = R;
            for (int k = 0; k < R; k++) {
                if (std::sqrt(std::max(rn[k].real(), 0.0)) <= tol) continue;
                T *t = V + (size_t)m * N;
                hipLaunchKernelGGL(k_precond<CPLX>, dim3(grid()), dim3(256), 0, s, Rv + (size_t)k * N, diag, theta[k],
                                   N, t);
                // Olsen: t - eps u with u = x / (theta - H_II) and eps
                // = <x, t> / <x, u>, so that the correction is orthogonal
                // to x (first order in the residual)
                hipLaunchKernelGGL(k_precond<CPLX>, dim3(grid()), dim3(256), 0, s, X + (size_t)k * N, diag, theta[k],
                                   N, Tn);
                std::vector<cd> xt, xu;
                if (!dots(X + (size_t)k * N, t, std::vector<int>{0}, std::vector<int>{0}, xt) ||
                    !dots(X + (size_t)k * N, Tn, std::vector<int>{0}, std::vector<int>{0}, xu))
                    return fail(MW_EHIP, "dot products failed");
                if (std::abs(xu[0]) > 1e-300) {
                    std::vector<cd> C{-xt[0] / xu[0]};
                    if (!lincomb(Tn, 1, C, 1, t, std::vector<double>{1.0})) return fail(MW_EHIP, "correction failed");
                }
                double nrm;
                if (!orthonormalize(m, nrm)) return fail(MW_EHIP, "Gram-Schmidt failed");
                if (nrm >= 1e-10) m++;
            }
            if (m > R && (st = apply_h(R, m - R)) != MW_OK) return st;
            // H P is carried along with P, but normalising a direction that
            // Gram-Schmidt left short divides the rounding error of its
            // carried product by that length: below 1e-2 the products of
            // the directions are computed afresh (near convergence only)
            const int p0 = m;
            bool fresh = false;
            for (int k = 0; k < np; k++) {
                if (hipMemcpyAsync(V + (size_t)m * N, Pv + (size_t)k * N, N * sizeof(T), hipMemcpyDeviceToDevice, s) !=
                        hipSuccess ||
                    hipMemcpyAsync(W + (size_t)m * N, PA + (size_t)k * N, N * sizeof(T), hipMemcpyDeviceToDevice, s) !=
                        hipSuccess)
                    return fail(MW_EHIP, "copy failed");
                double nrm;
                if (!orthonormalize_vw(m, nrm)) return fail(MW_EHIP, "Gram-Schmidt failed");
                if (nrm >= 1e-10) {
                    m++;
                    fresh = fresh || nrm < 1e-2;
                }
            }
            if (fresh && (st = apply_h(p0, m - p0)) != MW_OK) return st;
            if (m == R) break;  // no new direction: stagnation
        }
        hipLaunchKernelGGL(k_pack<T>, dim3(grid()), dim3(256), 0, s, X, R, N, (T *)c_out, 1);
        if (hipStreamSynchronize(s) != hipSuccess) return fail(MW_EHIP, "final sync failed");
        for (int k = 0; k < R; k++) evals[k] = theta[k];
        *iters = std::min(it, max_iter);
        if (!converged) return fail(MW_ENOCONV, "iVI did not converge");
        return MW_OK;
    }
};

}  // namespace
}  // namespace mw

using namespace mw;

extern "C" const mw::DevPlan *mw_internal_devplan(mw_plan plan);

extern "C" mw_status mw_davidson_work_bytes(mw_plan plan, int32_t nroots, size_t *bytes)
{
    if (!plan || !bytes) return fail(MW_EINVAL, "NULL argument");
    const DevPlan *d = mw_internal_devplan(plan);
    if (!d) return fail(MW_EWORKSPACE, "plan has no workspace");
    if (nroots < 1 || nroots > d->max_roots) return fail(MW_EINVAL, "nroots must be in 1..max_roots");
    *bytes = d->kind == MW_SPINOR ? Davidson<true>::bytes(nroots, d->ndet) : Davidson<false>::bytes(nroots, d->ndet);
    return MW_OK;
}

template <bool CPLX>
static mw_status run_davidson(mw_plan plan, const DevPlan *d, int32_t nroots, const void *c0, void *c_out,
                              double *evals, double tol, int32_t max_iter, int32_t *iters, void *work,
                              hipStream_t s)
{
    using T = typename Scal<CPLX>::T;
    Davidson<CPLX> D;
    D.sigma = [plan, s](int k, const T *in, T *out) { return mw_sigma(plan, k, in, out, (mw_stream_t)s); };
    D.diag = (const T *)d->diag;
    D.s = s;
    D.R = nroots;
    D.mmax = std::max(8 * nroots, 24) + nroots;
    D.N = d->ndet;
    D.carve((char *)work);
    return D.run(c0, c_out, evals, tol, max_iter, iters);
}

extern "C" mw_status mw_davidson(mw_plan plan, int32_t nroots, const void *c0, void *c_out, double *evals, double tol,
                                 int32_t max_iter, int32_t *iters, void *work, size_t work_bytes, mw_stream_t stream)
{
    if (!plan) return fail(MW_EINVAL, "plan is NULL");
    const DevPlan *d = mw_internal_devplan(plan);
    if (!d) return fail(MW_EWORKSPACE, "plan has no workspace");
    if (nroots < 1 || nroots > d->max_roots) return fail(MW_EINVAL, "nroots must be in 1..max_roots");
    if (!c0 || !c_out || !evals || !iters || !work) return fail(MW_EINVAL, "NULL argument");
    if (!(tol > 0) || max_iter < 1) return fail(MW_EINVAL, "tol must be > 0 and max_iter >= 1");
    if (nroots > d->ndet) return fail(MW_EINVAL, "more roots than determinants");
    size_t need;
    mw_status st = mw_davidson_work_bytes(plan, nroots, &need);
    if (st != MW_OK) return st;
    if (work_bytes < need) return fail(MW_EWORKSPACE, "work area too small");
    if (((uintptr_t)work) & 255) return fail(MW_EWORKSPACE, "work area must be 256-byte aligned");
    if (d->kind == MW_SPINOR)
        return run_davidson<true>(plan, d, nroots, c0, c_out, evals, tol, max_iter, iters, work, (hipStream_t)stream);
    return run_davidson<false>(plan, d, nroots, c0, c_out, evals, tol, max_iter, iters, work, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// Iterative vector interaction (section 2.4): fixed search space of 3R
// vectors, lowest roots or the roots nearest a target energy
// ---------------------------------------------------------------------------

extern "C" mw_status mw_ivi_work_bytes(mw_plan plan, int32_t nroots, size_t *bytes)
{
    if (!plan || !bytes) return fail(MW_EINVAL, "NULL argument");
    const DevPlan *d = mw_internal_devplan(plan);
    if (!d) return fail(MW_EWORKSPACE, "plan has no workspace");
    if (nroots < 1 || nroots > d->max_roots) return fail(MW_EINVAL, "nroots must be in 1..max_roots");
    *bytes = d->kind == MW_SPINOR ? Davidson<true>::bytes_m(4 * nroots, nroots, d->ndet)
                                  : Davidson<false>::bytes_m(4 * nroots, nroots, d->ndet);
    return MW_OK;
}

template <bool CPLX>
static mw_status run_ivi_t(mw_plan plan, const DevPlan *d, int32_t nroots, double target, const void *c0,
                           void *c_out, double *evals, double tol, int32_t max_iter, int32_t *iters, void *work,
                           hipStream_t s)
{
    using T = typename Scal<CPLX>::T;
    Davidson<CPLX> D;
    D.sigma = [plan, s](int k, const T *in, T *out) { return mw_sigma(plan, k, in, out, (mw_stream_t)s); };
    D.diag = (const T *)d->diag;
    D.s = s;
    D.R = nroots;
    D.mmax = 4 * nroots;
    D.N = d->ndet;
    D.carve((char *)work);
    return D.run_ivi(c0, c_out, evals, tol, max_iter, iters, target);
}

extern "C" mw_status mw_ivi(mw_plan plan, int32_t nroots, double target, const void *c0, void *c_out, double *evals,
                            double tol, int32_t max_iter, int32_t *iters, void *work, size_t work_bytes,
                            mw_stream_t stream)
{
    if (!plan) return fail(MW_EINVAL, "plan is NULL");
    const DevPlan *d = mw_internal_devplan(plan);
    if (!d) return fail(MW_EWORKSPACE, "plan has no workspace");
    if (nroots < 1 || nroots > d->max_roots) return fail(MW_EINVAL, "nroots must be in 1..max_roots");
    if (!c0 || !c_out || !evals || !iters || !work) return fail(MW_EINVAL, "NULL argument");
    if (!(tol > 0) || max_iter < 1) return fail(MW_EINVAL, "tol must be > 0 and max_iter >= 1");
    if (std::isinf(target)) return fail(MW_EINVAL, "target must be finite (NaN for the lowest roots)");
    if (nroots > d->ndet) return fail(MW_EINVAL, "more roots than determinants");
    size_t need;
    mw_status st = mw_ivi_work_bytes(plan, nroots, &need);
    if (st != MW_OK) return st;
    if (work_bytes < need) return fail(MW_EWORKSPACE, "work area too small");
    if (((uintptr_t)work) & 255) return fail(MW_EWORKSPACE, "work area must be 256-byte aligned");
    if (d->kind == MW_SPINOR)
        return run_ivi_t<true>(plan, d, nroots, target, c0, c_out, evals, tol, max_iter, iters, work,
                               (hipStream_t)stream);
    return run_ivi_t<false>(plan, d, nroots, target, c0, c_out, evals, tol, max_iter, iters, work,
                            (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// Davidson in a CSF basis: sigma through mw_csf_sigma, preconditioned with
// the determinant diagonal carried into the CSF basis,
// D_mu = sum_I T_I,mu^2 H_II (the CSF diagonal without its off-diagonal
// determinant couplings inside the configuration).
// ---------------------------------------------------------------------------

extern "C" int mw_internal_csf_dims(mw_csf csf, mw_plan *plan, int64_t *ndet, int64_t *ncsf);
extern "C" mw_status mw_internal_csf_diag(mw_csf csf, const double *hdiag, double *out, hipStream_t s);

static size_t csf_dav_bytes(int R, int64_t ndet, int64_t ncsf, int mmax)
{
    size_t b = Davidson<false>::bytes_m(mmax, R, ncsf);
    b = (b + 255) & ~(size_t)255;
    b += (size_t)2 * ndet * R * 8;   // determinant vectors of mw_csf_sigma
    b = (b + 255) & ~(size_t)255;
    b += (size_t)ncsf * 8;           // preconditioner diagonal
    return b + 256;
}

extern "C" mw_status mw_csf_davidson_work_bytes(mw_csf csf, int32_t nroots, size_t *bytes)
{
    mw_plan plan;
    int64_t ndet, ncsf;
    if (!csf || !bytes) return fail(MW_EINVAL, "NULL argument");
    if (!mw_internal_csf_dims(csf, &plan, &ndet, &ncsf))
        return fail(MW_EWORKSPACE, "CSF basis has no workspace: call mw_csf_upload first");
    const DevPlan *d = mw_internal_devplan(plan);
    if (!d) return fail(MW_EWORKSPACE, "the plan has no workspace");
    if (nroots < 1 || nroots > d->max_roots) return fail(MW_EINVAL, "nroots must be in 1..max_roots of the plan");
    *bytes = csf_dav_bytes(nroots, ndet, ncsf, std::max(8 * nroots, 24) + nroots);
    return MW_OK;
}

// solver 0: Davidson (mmax = max(8R, 24) + R); 1: iVI (mmax = 4R)
static mw_status csf_solve(int solver, mw_csf csf, int32_t nroots, double target, const double *c0, double *c_out,
                           double *evals, double tol, int32_t max_iter, int32_t *iters, void *work,
                           size_t work_bytes, mw_stream_t stream)
{
    mw_plan plan;
    int64_t ndet, ncsf;
    if (!csf) return fail(MW_EINVAL, "csf is NULL");
    if (!mw_internal_csf_dims(csf, &plan, &ndet, &ncsf))
        return fail(MW_EWORKSPACE, "CSF basis has no workspace: call mw_csf_upload first");
    if (!c0 || !c_out || !evals || !iters || !work) return fail(MW_EINVAL, "NULL argument");
    if (!(tol > 0) || max_iter < 1) return fail(MW_EINVAL, "tol must be > 0 and max_iter >= 1");
    if (solver == 1 && std::isinf(target)) return fail(MW_EINVAL, "target must be finite (NaN for the lowest roots)");
    const DevPlan *d = mw_internal_devplan(plan);
    if (!d) return fail(MW_EWORKSPACE, "the plan has no workspace");
    if (nroots < 1 || nroots > d->max_roots) return fail(MW_EINVAL, "nroots must be in 1..max_roots of the plan");
    if (nroots > ncsf) return fail(MW_EINVAL, "more roots than CSFs");
    const int mmax = solver == 1 ? 4 * nroots : std::max(8 * nroots, 24) + nroots;
    if (work_bytes < csf_dav_bytes(nroots, ndet, ncsf, mmax)) return fail(MW_EWORKSPACE, "work area too small");
    if (((uintptr_t)work) & 255) return fail(MW_EWORKSPACE, "work area must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    size_t off = (Davidson<false>::bytes_m(mmax, nroots, ncsf) + 255) & ~(size_t)255;
    double *dwork = (double *)((char *)work + off);
    off = (off + (size_t)2 * ndet * nroots * 8 + 255) & ~(size_t)255;
    double *pdiag = (double *)((char *)work + off);
    mw_status st = mw_internal_csf_diag(csf, (const double *)d->diag, pdiag, s);
    if (st != MW_OK) return st;
    Davidson<false> D;
    D.sigma = [csf, dwork, s](int k, const double *in, double *out) {
        return mw_csf_sigma(csf, k, in, out, dwork, (mw_stream_t)s);
    };
    D.diag = pdiag;
    D.s = s;
    D.R = nroots;
    D.mmax = mmax;
    D.N = ncsf;
    D.carve((char *)work);
    if (solver == 1) return D.run_ivi(c0, c_out, evals, tol, max_iter, iters, target);
    return D.run(c0, c_out, evals, tol, max_iter, iters);
}

extern "C" mw_status mw_csf_ivi_work_bytes(mw_csf csf, int32_t nroots, size_t *bytes)
{
    mw_plan plan;
    int64_t ndet, ncsf;
    if (!csf || !bytes) return fail(MW_EINVAL, "NULL argument");
    if (!mw_internal_csf_dims(csf, &plan, &ndet, &ncsf))
        return fail(MW_EWORKSPACE, "CSF basis has no workspace: call mw_csf_upload first");
    const DevPlan *d = mw_internal_devplan(plan);
    if (!d) return fail(MW_EWORKSPACE, "the plan has no workspace");
    if (nroots < 1 || nroots > d->max_roots) return fail(MW_EINVAL, "nroots must be in 1..max_roots of the plan");
    *bytes = csf_dav_bytes(nroots, ndet, ncsf, 4 * nroots);
    return MW_OK;
}

extern "C" mw_status mw_csf_ivi(mw_csf csf, int32_t nroots, double target, const double *c0, double *c_out,
                                double *evals, double tol, int32_t max_iter, int32_t *iters, void *work,
                                size_t work_bytes, mw_stream_t stream)
{
    return csf_solve(1, csf, nroots, target, c0, c_out, evals, tol, max_iter, iters, work, work_bytes, stream);
}

extern "C" mw_status mw_csf_davidson(mw_csf csf, int32_t nroots, const double *c0, double *c_out, double *evals,
                                     double tol, int32_t max_iter, int32_t *iters, void *work, size_t work_bytes,
                                     mw_stream_t stream)
{
    return csf_solve(0, csf, nroots, 0.0, c0, c_out, evals, tol, max_iter, iters, work, work_bytes, stream);
}
