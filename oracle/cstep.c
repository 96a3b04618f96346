/*
 * Plain FP64 stabilised leapfrog (Kolar-Pozun & Kosec, arXiv 2508.18205,
 * Section 5, eq. 19) for the 2D TMz fields and for 3D, one half update per
 * call.
 *
 * TEST INFRASTRUCTURE ONLY: part of the CPU oracle.  Only the tests, the
 * package smoke check and the CPU-baseline leg of the benchmark may call it.
 * It shares no code with the GPU library.
 *
 * The same arithmetic as oracle/step.py (h_update / e_update) written as
 * loops over nodes, so that node sets of a million nodes can be advanced for
 * thousands of steps: every operator is D^L f(x_i) = sum_j w_ij f(x_j)
 * (eq. 16), summed in slot order, with
 *   Hx <- Hx - a (D^dy Ez - gamma D^hv Hx)
 *   Hy <- Hy + a (D^dx Ez + gamma D^hv Hy)
 *   Ez <- keep_i (Ez + kappa_i (D^dx Hy_new - D^dy Hx_new + gamma D^hv Ez))
 * a = dt / mu0, kappa_i = dt / (eps0 eps_r,i), keep_i = 0 on PEC wall nodes.
 * OpenMP over nodes only; built with -O2 -ffp-contract=off (no fused
 * multiply-adds, each product and sum rounded on its own).
 *
 * Layouts (row-major, original node order): E [N], H [N][2], curl indices
 * ci [N][n] (int64), curl weights cw [N][2][n] (x then y), HV indices hi
 * [N][nh], HV weights hw [N][nh].  Output buffers must not alias inputs.
 */
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static double dsum(const double* w, const int64_t* idx, int n, const double* f, int stride, int comp) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += w[j] * f[idx[j] * stride + comp];
    return s;
}

/* H^{n+1} from E^n and H^n (first two lines of eq. 19). */
void oracle_h_update_tm(int64_t N, const double* E, const double* H, double* Hout, int n, const int64_t* ci,
                        const double* cw, int nh, const int64_t* hi, const double* hw, double a, double gamma) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        const double* wx = cw + i * 2 * n;
        const double* wy = wx + n;
        const int64_t* c = ci + i * n;
        const double dxE = dsum(wx, c, n, E, 1, 0);
        const double dyE = dsum(wy, c, n, E, 1, 0);
        double hvx = 0.0, hvy = 0.0;
        if (nh > 0) {
            hvx = dsum(hw + i * nh, hi + i * nh, nh, H, 2, 0);
            hvy = dsum(hw + i * nh, hi + i * nh, nh, H, 2, 1);
        }
        Hout[2 * i + 0] = H[2 * i + 0] - a * (dyE - gamma * hvx);
        Hout[2 * i + 1] = H[2 * i + 1] + a * (dxE + gamma * hvy);
    }
}

/* E^{n+1} from E^n and H^{n+1} (last line of eq. 19), then the PEC factor.
 * kappa: [N] per-node values, or NULL to use kappa0 everywhere. */
void oracle_e_update_tm(int64_t N, const double* E, const double* Hn, double* Eout, int n, const int64_t* ci,
                        const double* cw, int nh, const int64_t* hi, const double* hw, const double* kappa,
                        double kappa0, double gamma, const double* keep) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        const double* wx = cw + i * 2 * n;
        const double* wy = wx + n;
        const int64_t* c = ci + i * n;
        const double dxHy = dsum(wx, c, n, Hn, 2, 1);
        const double dyHx = dsum(wy, c, n, Hn, 2, 0);
        double hv = 0.0;
        if (nh > 0) hv = dsum(hw + i * nh, hi + i * nh, nh, E, 1, 0);
        const double k = kappa ? kappa[i] : kappa0;
        const double br = dxHy - dyHx + gamma * hv;
        Eout[i] = (E[i] + k * br) * keep[i];
    }
}

/*
 * 3D: the full discrete curl of eq. 19, E [N][3], H [N][3] (x, y, z), curl
 * weights cw [N][3][n] (D^dx, D^dy, D^dz rows), with
 *   curl F = (D^dy Fz - D^dz Fy, D^dz Fx - D^dx Fz, D^dx Fy - D^dy Fx)
 *   H_c <- H_c - a (curl_c E - gamma D^hv H_c)
 *   E_c <- keep_ic (E_c + kappa_i (curl_c H_new + gamma D^hv E_c))
 * keep [N][3]: 0 for an E component tangential to a PEC wall at the node.
 */
static void curl3(const double* cw, const int64_t* c, int n, const double* F, double out[3]) {
    const double* wx = cw;
    const double* wy = cw + n;
    const double* wz = cw + 2 * n;
    const double dyFz = dsum(wy, c, n, F, 3, 2), dzFy = dsum(wz, c, n, F, 3, 1);
    const double dzFx = dsum(wz, c, n, F, 3, 0), dxFz = dsum(wx, c, n, F, 3, 2);
    const double dxFy = dsum(wx, c, n, F, 3, 1), dyFx = dsum(wy, c, n, F, 3, 0);
    out[0] = dyFz - dzFy;
    out[1] = dzFx - dxFz;
    out[2] = dxFy - dyFx;
}

/* H^{n+1} from E^n and H^n (3D). */
void oracle_h_update_3d(int64_t N, const double* E, const double* H, double* Hout, int n, const int64_t* ci,
                        const double* cw, int nh, const int64_t* hi, const double* hw, double a, double gamma) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double cu[3];
        curl3(cw + i * 3 * n, ci + i * n, n, E, cu);
        for (int c = 0; c < 3; ++c) {
            const double hv = nh > 0 ? dsum(hw + i * nh, hi + i * nh, nh, H, 3, c) : 0.0;
            Hout[3 * i + c] = H[3 * i + c] - a * (cu[c] - gamma * hv);
        }
    }
}

/* E^{n+1} from E^n and H^{n+1} (3D), then the PEC factors.  kappa: [N]
 * per-node values, or NULL to use kappa0 everywhere. */
void oracle_e_update_3d(int64_t N, const double* E, const double* Hn, double* Eout, int n, const int64_t* ci,
                        const double* cw, int nh, const int64_t* hi, const double* hw, const double* kappa,
                        double kappa0, double gamma, const double* keep) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double cu[3];
        curl3(cw + i * 3 * n, ci + i * n, n, Hn, cu);
        const double k = kappa ? kappa[i] : kappa0;
        for (int c = 0; c < 3; ++c) {
            const double hv = nh > 0 ? dsum(hw + i * nh, hi + i * nh, nh, E, 3, c) : 0.0;
            Eout[3 * i + c] = (E[3 * i + c] + k * (cu[c] + gamma * hv)) * keep[3 * i + c];
        }
    }
}

/* Number of OpenMP threads a parallel region uses (reported by the
 * benchmark's CPU baseline). */
int oracle_threads(void) {
    int t = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            t = omp_get_num_threads();
#endif
        }
    }
    return t;
}

/* Sets the OpenMP thread count of later calls (the benchmark's one-core
 * figure); values below 1 are ignored. */
void oracle_set_threads(int t) {
#ifdef _OPENMP
    if (t >= 1) omp_set_num_threads(t);
#else
    (void)t;
#endif
}
