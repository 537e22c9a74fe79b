// Ground-state and dynamics solvers on gfx950, built on the plan's NUFFT potential.
//
// Ground state (Sec. 3.1, Eqs. 'gf-eq2', 'gf-colb2', 'gffg33'): gradient flow with discrete
// normalization, backward Euler in time, Fourier pseudospectral in space, potential lagged at
// phi^n.  The backward-Euler step is implicit in the whole linear part,
//     (1/tau - Delta/2 + W) phi1 = phi^n / tau,   W = V + beta varphi^n,
// solved by preconditioned conjugate gradients.  The preconditioner is the Fourier multiplier
// D = 1/(1/tau + a + |mu|^2/2), a = (max W + min W)/2.  The search direction is kept in Fourier
// space, so one iteration costs two complex FFTs: r -> r^, and (p^ + i K p^) -> (p, K p) with
// K = |mu|^2/2 (both p and K p are real, so they share one inverse transform).
// Stopping rule max|phi^{n+1} - phi^n| / tau <= eps0 (Sec. 3.2); energies, chemical potential and
// virial identity as in Sec. 3.2.  All reductions are FP64.
//
// Dynamics (Sec. 4.1, Eqs. 'sps-eq65'-'sps-eq68'): Strang splitting; the kinetic flow is exact
// in Fourier space, the potential flow psi <- exp(-i (V + beta varphi) dt) psi is exact because
// |psi| does not change during it.  Order 4 composes three Strang steps (Yoshida).  Phase
// arguments are formed in FP64.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "exec.h"
#include "fft_dev.h"
#include "nufft_dev.h"
#include "nlf_internal.h"

namespace nlf {

constexpr int RB_T = 256;      // threads per block of the pointwise/reduction kernels
constexpr int MAXBLK = 256;    // reduction partials per field

template <typename T> __device__ __forceinline__ V2<T> mkc(T x, T y);
template <> __device__ __forceinline__ float2 mkc<float>(float x, float y) { return make_float2(x, y); }
template <> __device__ __forceinline__ double2 mkc<double>(double x, double y) { return make_double2(x, y); }

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    return v;
}
// block-wide reductions (blockDim = RB_T); the result is valid in every thread
__device__ double block_sum(double v) {
    __shared__ double sh[RB_T / 64];
    __shared__ double res;
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0;
        for (int i = 0; i < RB_T / 64; ++i) s += sh[i];
        res = s;
    }
    __syncthreads();
    double r = res;
    __syncthreads();
    return r;
}
__device__ double block_max(double v) {
    __shared__ double sh[RB_T / 64];
    __shared__ double res;
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = sh[0];
        for (int i = 1; i < RB_T / 64; ++i) s = fmax(s, sh[i]);
        res = s;
    }
    __syncthreads();
    double r = res;
    __syncthreads();
    return r;
}
// sum of the nblk partials of one field (every block recomputes it; nblk <= MAXBLK)
__device__ double sum_parts(const double* part, int nblk) {
    double v = (threadIdx.x < nblk) ? part[threadIdx.x] : 0.0;
    return block_sum(v);
}
__device__ double max_parts(const double* part, int nblk) {
    double v = (threadIdx.x < nblk) ? part[threadIdx.x] : -1e308;
    return block_max(v);
}
// -(min over the partials), computed as a max of negated values
__device__ double max_parts_neg(const double* part, int nblk) {
    double v = (threadIdx.x < nblk) ? -part[threadIdx.x] : -1e308;
    return block_max(v);
}

// Grid geometry handed to the solver kernels.
struct Geo {
    int dim;
    int n[3];
    int lg[3];        // log2 n_i (grid sizes are powers of two)
    double L[3], h[3];
    long long N;
    double dv;        // prod h_i
};

// per-axis indices by shifts and masks (no 64-bit division per element)
__device__ __forceinline__ void coords(const Geo& g, long long i, double x[3], int j[3]) {
    long long r = i;
    for (int a = g.dim - 1; a >= 0; --a) {
        j[a] = (int)(r & (g.n[a] - 1));
        r >>= g.lg[a];
        x[a] = -g.L[a] + j[a] * g.h[a];
    }
}
// linear index of the frequency -k of linear index i (per axis l -> (n - l) mod n)
__device__ __forceinline__ long long neg_index(const Geo& g, long long i) {
    long long r = i, out = 0;
    int sh = 0;
    for (int a = g.dim - 1; a >= 0; --a) {
        const int l = (int)(r & (g.n[a] - 1));
        r >>= g.lg[a];
        out |= (long long)((g.n[a] - l) & (g.n[a] - 1)) << sh;
        sh += g.lg[a];
    }
    return out;
}

// The residuals of fields 2q and 2q+1 share one complex transform, z = r_2q + i r_2q+1 (both real):
// field b writes its part of z, and reads its own spectrum back as (Z(k) + conj Z(-k)) / 2 (even b)
// or (Z(k) - conj Z(-k)) / (2i) (odd b).  The extraction is exact for any real other part, but that
// part must stay of the residuals' size: after the transform the buffer holds a spectrum, so a field
// whose partner is not writing this iteration (retired, or absent in an odd batch) clears the
// partner's part (lone = true).
template <typename T>
__device__ __forceinline__ void put_resid(V2<T>* zf, long long N, int b, long long i, T v, bool lone) {
    V2<T>* z = zf + (long long)(b >> 1) * N + i;
    if (lone) *z = (b & 1) ? mkc<T>((T)0, v) : mkc<T>(v, (T)0);
    else reinterpret_cast<T*>(z)[b & 1] = v;
}
template <typename T>
__device__ __forceinline__ void pair_spec(const V2<T>* zf, long long N, int b, long long i, long long ni, double& re,
                                          double& im) {
    const V2<T> z = zf[(long long)(b >> 1) * N + i], zm = zf[(long long)(b >> 1) * N + ni];
    if ((b & 1) == 0) {
        re = 0.5 * ((double)z.x + (double)zm.x);
        im = 0.5 * ((double)z.y - (double)zm.y);
    } else {
        re = 0.5 * ((double)z.y + (double)zm.y);
        im = -0.5 * ((double)z.x - (double)zm.x);
    }
}

// |mu|^2 of the discrete Fourier mode at flat index i (mu_l = pi l / L, l in [-n/2, n/2))
__device__ __forceinline__ double mu2(const Geo& g, long long i) {
    long long r = i;
    double s = 0;
    for (int a = g.dim - 1; a >= 0; --a) {
        int l = (int)(r & (g.n[a] - 1));
        r >>= g.lg[a];
        if (l >= g.n[a] / 2) l -= g.n[a];
        double m = 3.14159265358979323846 * l / g.L[a];
        s += m * m;
    }
    return s;
}

// Per-field parameters and scalars live in device memory: Fld[b].
struct Fld {
    double beta, g2[3];          // beta, gamma_i^2
    double tau;
    double a;                    // preconditioner shift
    double rz, rz_old, pAp, rr, bb;
    double norm2, res;
    double cgtol;                // inner relative tolerance of the current solve
    double cgtol_min;            // the caller's (final) inner tolerance
    int cg_last;                 // iterations of the current solve
    int done_at;                 // outer step at which the field retired
    int conv;                    // PCG converged
    int done;                    // outer flow converged (field retired)
    int cg_iters;
    int first;                   // first PCG iteration of the current solve
    int nonfinite;
    int steps;                   // outer steps taken while the field was active
    double best_res;             // persistent executor, FP32 stage of a mixed schedule: best residual
    int stall;                   //   so far and checks since it last improved by 10%
};

__device__ __forceinline__ double trapV(const Geo& g, const Fld& f, const double* Vext, long long i, const double x[3]) {
    if (Vext) return Vext[i];
    double v = 0;
    for (int a = 0; a < g.dim; ++a) v += f.g2[a] * x[a] * x[a];
    return 0.5 * v;
}

// ---- ground-state kernels -------------------------------------------------------------------
// HO Gaussian initial guess prod (gamma_i/pi)^{1/4} exp(-gamma_i x_i^2 / 2) (Sec. 3.2 "Gaussian")
template <typename T>
__global__ void k_ho_init(Geo g, const Fld* fl, T* phi) {
    const int b = blockIdx.y;
    const Fld f = fl[b];
    for (long long i = (long long)blockIdx.x * RB_T + threadIdx.x; i < g.N; i += (long long)gridDim.x * RB_T) {
        double x[3];
        int j[3];
        coords(g, i, x, j);
        double v = 1;
        for (int a = 0; a < g.dim; ++a) {
            double ga = sqrt(f.g2[a]);
            v *= pow(ga / 3.14159265358979323846, 0.25) * exp(-0.5 * ga * x[a] * x[a]);
        }
        phi[(long long)b * g.N + i] = (T)v;
    }
}

// partial sums of h^d sum v^2 (norm2) per field
template <typename T>
__device__ __forceinline__ void norm2_part_body(Geo g, const Fld* fl, const T* v, double* part, VBlk vb) {
    const int b = vb.y;
    if (fl[b].done) return;
    double s = 0;
    for (long long i = (long long)vb.x * RB_T + threadIdx.x; i < g.N; i += (long long)vb.gx * RB_T) {
        double a = (double)v[(long long)b * g.N + i];
        s += a * a;
    }
    s = block_sum(s);
    if (threadIdx.x == 0) part[b * MAXBLK + vb.x] = s * g.dv;
}

// phi <- v / ||v||; optionally residual max|phi_new - phi_old|/tau partials; rho = phi^2
template <typename T>
__device__ __forceinline__ void normalize_body(Geo g, Fld* fl, const T* v, T* phi, T* rho, const double* part_n, double* part_r,
                            int nblk, int track_res, VBlk vb) {
    const int b = vb.y;
    if (fl[b].done) return;
    const double nrm = sqrt(sum_parts(part_n + b * MAXBLK, nblk));
    const double inv = 1.0 / nrm;
    const double tau = fl[b].tau;
    double m = 0;
    for (long long i = (long long)vb.x * RB_T + threadIdx.x; i < g.N; i += (long long)vb.gx * RB_T) {
        long long k = (long long)b * g.N + i;
        double nv = (double)v[k] * inv;
        if (track_res) m = fmax(m, fabs(nv - (double)phi[k]) / tau);
        phi[k] = (T)nv;
        rho[k] = (T)(nv * nv);
    }
    if (track_res) {
        m = block_max(m);
        if (threadIdx.x == 0) part_r[b * MAXBLK + vb.x] = m;
    }
    if (vb.x == 0 && threadIdx.x == 0) fl[b].norm2 = nrm * nrm;
}

// outer residual max|phi^{n+1} - phi^n| / tau; retire the field at eps0.  The next inner solve
// only needs to be accurate relative to the size of the step it computes, so its tolerance
// follows the residual down to the caller's tolerance: max(cg_tol, min(1e-3, 1e-3 tau res)).
// The step count lives on the device (Fld::steps) so that the launch can be replayed from a graph.
template <typename T>
__device__ __forceinline__ void residual_final_body(Fld* fl, const double* part_r, int nblk, double eps0, VBlk vb) {
    const int b = vb.x;
    if (fl[b].done) return;
    double r = max_parts(part_r + b * MAXBLK, nblk);
    if (threadIdx.x == 0) {
        const int step = fl[b].steps + 1;
        fl[b].steps = step;
        fl[b].res = r;
        if (!(r == r) || r > 1e300) fl[b].nonfinite = 1;
        if (r <= eps0) {
            fl[b].done = 1;
            fl[b].done_at = step;
        }
        fl[b].cgtol = fmax(fl[b].cgtol_min, fmin(1e-3, 1e-3 * fl[b].tau * r));
    }
}

// W = V + beta varphi; partial max/min of W for the preconditioner shift; cw = (phi, 0)
template <typename T>
__device__ __forceinline__ void gf_prep_body(Geo g, const Fld* fl, const double* Vext, const T* pot, const T* phi, T* W,
                          V2<T>* cw, double* part_mx, double* part_mn, VBlk vb) {
    const int b = vb.y;
    if (fl[b].done) return;
    const Fld f = fl[b];
    double mx = -1e308, mn = 1e308;
    for (long long i = (long long)vb.x * RB_T + threadIdx.x; i < g.N; i += (long long)vb.gx * RB_T) {
        double x[3];
        int j[3];
        coords(g, i, x, j);
        long long k = (long long)b * g.N + i;
        double w = trapV(g, f, Vext, i, x) + f.beta * (double)pot[k];
        W[k] = (T)w;
        mx = fmax(mx, w);
        mn = fmin(mn, w);
        cw[k] = mkc<T>(phi[k], (T)0);
    }
    mx = block_max(mx);
    mn = -block_max(-mn);
    if (threadIdx.x == 0) {
        part_mx[b * MAXBLK + vb.x] = mx;
        part_mn[b * MAXBLK + vb.x] = mn;
    }
}

// after FFT(phi): cw <- K cw / N  (K = |mu|^2/2)
template <typename T>
__device__ __forceinline__ void kin_apply_body(Geo g, const Fld* fl, V2<T>* cw, VBlk vb) {
    const int b = vb.y;
    if (fl[b].done) return;
    const double invN = 1.0 / (double)g.N;
    for (long long i = (long long)vb.x * RB_T + threadIdx.x; i < g.N; i += (long long)vb.gx * RB_T) {
        long long k = (long long)b * g.N + i;
        double s = 0.5 * mu2(g, i) * invN;
        V2<T> v = cw[k];
        cw[k] = mkc<T>((T)(v.x * s), (T)(v.y * s));
    }
}

// preconditioner shift a (one block per field).  The Fourier multiplier 1/(1/tau + a + K) matches
// A = 1/tau + K + W up to the factor (1/tau + W)/(1/tau + a), which ranges over
// [(1/tau + min W), (1/tau + max W)] / (1/tau + a); the geometric mean
// 1/tau + a = sqrt((1/tau + min W)(1/tau + max W)) minimises the ratio of its extremes.
__device__ __forceinline__ void shift_body(Fld* fl, const double* part_mx, const double* part_mn, int nblk, VBlk vb) {
    const int b = vb.x;
    if (fl[b].done) return;
    double mx = max_parts(part_mx + b * MAXBLK, nblk);
    double v = (threadIdx.x < nblk) ? -part_mn[b * MAXBLK + threadIdx.x] : -1e308;
    double mn = -block_max(v);
    if (threadIdx.x == 0) {
        const double it = 1.0 / fl[b].tau;
        const double lo = it + mn, hi = it + mx;
        fl[b].a = (lo > 0.0) ? sqrt(lo * hi) - it : 0.5 * (mx + mn);
    }
}

// PCG start: x = phi, r = b - A x = -(K phi + W phi) (with b = phi/tau), r into its pair
// transform zf; bb partials
template <typename T>
__device__ __forceinline__ void pcg_init_body(Geo g, Fld* fl, const T* phi, const T* W, const V2<T>* kphi, T* x, T* r, V2<T>* zf,
                           double* part_bb, VBlk vb) {
    const int b = vb.y;
    if (fl[b].done) return;
    const double tau = fl[b].tau;
    // Start from c phi^n with c = |x| of the previous step's solution (~ 1/(1 + tau mu) for the
    // current chemical potential mu): r0 = (1 - c) phi/tau - c H phi = c (mu phi - H phi), the
    // eigen-residual, which vanishes as the flow converges.  The first step starts from phi^n.
    const double c = (fl[b].steps > 0 && fl[b].norm2 > 0.0) ? sqrt(fl[b].norm2) : 1.0;
    // the partner field runs this kernel too unless it has retired from the flow or is absent
    const bool lone = ((b ^ 1) >= (int)vb.gy) || fl[b ^ 1].done;
    double s = 0;
    for (long long i = (long long)vb.x * RB_T + threadIdx.x; i < g.N; i += (long long)vb.gx * RB_T) {
        long long k = (long long)b * g.N + i;
        double p = (double)phi[k];
        double ri = (1.0 - c) * p / tau - c * ((double)kphi[k].x + (double)W[k] * p);
        x[k] = (T)(c * p);
        r[k] = (T)ri;
        put_resid<T>(zf, g.N, b, i, (T)ri, lone);
        s += (p / tau) * (p / tau);
    }
    s = block_sum(s);
    if (threadIdx.x == 0) part_bb[b * MAXBLK + vb.x] = s;
    if (vb.x == 0 && threadIdx.x == 0) {
        fl[b].conv = 0;
        fl[b].first = 1;
        fl[b].rz_old = 0;
        fl[b].cg_last = 0;
    }
}

__device__ __forceinline__ void bb_final_body(Fld* fl, const double* part_bb, int nblk, VBlk vb) {
    const int b = vb.x;
    if (fl[b].done) return;
    double s = sum_parts(part_bb + b * MAXBLK, nblk);
    if (threadIdx.x == 0) fl[b].bb = s;
}

// rz = sum D |r^|^2 / N (Parseval), D = 1/(1/tau + a + K); r^ from the pair transform zf
template <typename T>
__device__ __forceinline__ void pcg_rz_body(Geo g, const Fld* fl, const V2<T>* zf, double* part_rz, VBlk vb) {
    const int b = vb.y;
    if (fl[b].done || fl[b].conv) return;
    const double c0 = 1.0 / fl[b].tau + fl[b].a;
    double s = 0;
    for (long long i = (long long)vb.x * RB_T + threadIdx.x; i < g.N; i += (long long)vb.gx * RB_T) {
        double vx, vy;
        pair_spec<T>(zf, g.N, b, i, neg_index(g, i), vx, vy);
        double d = 1.0 / (c0 + 0.5 * mu2(g, i));
        s += d * (vx * vx + vy * vy);
    }
    s = block_sum(s);
    if (threadIdx.x == 0) part_rz[b * MAXBLK + vb.x] = s / (double)g.N;
}

// p^ = D r^ + beta p^ (beta = rz / rz_old), cw = (p^ + i K p^) / N for the inverse transform
template <typename T>
__device__ __forceinline__ void pcg_dir_body(Geo g, Fld* fl, const V2<T>* zf, V2<T>* cw, V2<T>* ph, const double* part_rz, int nblk, VBlk vb) {
    const int b = vb.y;
    if (fl[b].done || fl[b].conv) return;
    const double rz = sum_parts(part_rz + b * MAXBLK, nblk);
    const double rzo = fl[b].rz_old;
    const double beta = (fl[b].first || !(rzo > 0.0)) ? 0.0 : rz / rzo;
    const double c0 = 1.0 / fl[b].tau + fl[b].a;
    const double invN = 1.0 / (double)g.N;
    for (long long i = (long long)vb.x * RB_T + threadIdx.x; i < g.N; i += (long long)vb.gx * RB_T) {
        long long k = (long long)b * g.N + i;
        double m2 = mu2(g, i);
        double d = 1.0 / (c0 + 0.5 * m2);
        double rx, ry;
        pair_spec<T>(zf, g.N, b, i, neg_index(g, i), rx, ry);
        double px = d * rx, py = d * ry;
        if (beta != 0.0) {   // the previous direction is never read on a restart (it may be unset)
            V2<T> pv = ph[k];
            px += beta * (double)pv.x;
            py += beta * (double)pv.y;
        }
        ph[k] = mkc<T>((T)px, (T)py);
        double kk = 0.5 * m2;
        // (p^ + i K p^) = (px - K py, py + K px)
        cw[k] = mkc<T>((T)((px - kk * py) * invN), (T)((py + kk * px) * invN));
    }
    if (vb.x == 0 && threadIdx.x == 0) fl[b].rz = rz;
}

// p = Re cw, K p = Im cw; Ap = K p + (1/tau + W) p; pAp partials
template <typename T>
__device__ __forceinline__ void pcg_apply_body(Geo g, const Fld* fl, const V2<T>* cw, const T* W, T* p, T* Ap, double* part_pap, VBlk vb) {
    const int b = vb.y;
    if (fl[b].done || fl[b].conv) return;
    const double it = 1.0 / fl[b].tau;
    double s = 0;
    for (long long i = (long long)vb.x * RB_T + threadIdx.x; i < g.N; i += (long long)vb.gx * RB_T) {
        long long k = (long long)b * g.N + i;
        V2<T> v = cw[k];
        double pv = (double)v.x;
        double ap = (double)v.y + (it + (double)W[k]) * pv;
        p[k] = (T)pv;
        Ap[k] = (T)ap;
        s += pv * ap;
    }
    s = block_sum(s);
    if (threadIdx.x == 0) part_pap[b * MAXBLK + vb.x] = s;
}

// a = rz / pAp; x += a p; r -= a Ap; r into its pair transform zf; rr partials
template <typename T>
__device__ __forceinline__ void pcg_update_body(Geo g, const Fld* fl, const T* p, const T* Ap, T* x, T* r, V2<T>* zf,
                             const double* part_pap, double* part_rr, int nblk, VBlk vb) {
    const int b = vb.y;
    if (fl[b].done || fl[b].conv) return;
    const double pap = sum_parts(part_pap + b * MAXBLK, nblk);
    // breakdown guard: A is symmetric positive definite, so pAp <= 0 (or a non-finite value) only
    // happens once rounding dominates the residual; the iterate is kept and the solve stops
    if (!(pap > 0.0) || !(fl[b].rz > 0.0) || !(pap < 1e300)) {
        if (threadIdx.x == 0) part_rr[b * MAXBLK + vb.x] = -1.0;
        return;
    }
    const double al = fl[b].rz / pap;
    // the partner writes its residual this iteration unless retired (flow or inner solve) or absent;
    // its conv flag only changes in k_pcg_check, after this kernel
    const bool lone = ((b ^ 1) >= (int)vb.gy) || fl[b ^ 1].done || fl[b ^ 1].conv;
    double s = 0;
    for (long long i = (long long)vb.x * RB_T + threadIdx.x; i < g.N; i += (long long)vb.gx * RB_T) {
        long long k = (long long)b * g.N + i;
        double xv = (double)x[k] + al * (double)p[k];
        double rv = (double)r[k] - al * (double)Ap[k];
        x[k] = (T)xv;
        r[k] = (T)rv;
        put_resid<T>(zf, g.N, b, i, (T)rv, lone);
        s += rv * rv;
    }
    s = block_sum(s);
    if (threadIdx.x == 0) part_rr[b * MAXBLK + vb.x] = s;
}

__device__ __forceinline__ void pcg_check_body(Fld* fl, const double* part_rr, int nblk, VBlk vb) {
    const int b = vb.x;
    if (fl[b].done || fl[b].conv) return;
    double rr = sum_parts(part_rr + b * MAXBLK, nblk);
    // a negative partial marks a breakdown stop of the update kernel (see k_pcg_update)
    double mn = -max_parts_neg(part_rr + b * MAXBLK, nblk);
    if (threadIdx.x == 0) {
        fl[b].rr = rr;
        fl[b].rz_old = fl[b].rz;
        fl[b].first = 0;
        fl[b].cg_iters += 1;
        fl[b].cg_last += 1;
        const double tol = fl[b].cgtol;
        if (mn < 0.0) fl[b].conv = 1;
        else if (!(rr == rr) || rr > 1e300) {
            fl[b].nonfinite = 1;
            fl[b].conv = 1;
        } else if (rr <= tol * tol * fl[b].bb) fl[b].conv = 1;
    }
}

// energies: partials of [Ekin, Epot, Eint, mass] (Ekin from |mu|^2 |phi^|^2 in Fourier space)
template <typename T>
__global__ void k_energy_part(Geo g, const Fld* fl, const double* Vext, const V2<T>* psi_hat, const V2<T>* psi_c,
                              const T* psi_r, const T* pot, double* part, int nblk_stride) {
    const int b = blockIdx.y;
    const Fld f = fl[b];
    double ek = 0, ep = 0, ei = 0, ms = 0;
    for (long long i = (long long)blockIdx.x * RB_T + threadIdx.x; i < g.N; i += (long long)gridDim.x * RB_T) {
        long long k = (long long)b * g.N + i;
        double x[3];
        int j[3];
        coords(g, i, x, j);
        V2<T> hv = psi_hat[k];
        ek += mu2(g, i) * ((double)hv.x * hv.x + (double)hv.y * hv.y);
        double dens;
        if (psi_c) {
            V2<T> v = psi_c[k];
            dens = (double)v.x * v.x + (double)v.y * v.y;
        } else {
            double v = (double)psi_r[k];
            dens = v * v;
        }
        ep += trapV(g, f, Vext, i, x) * dens;
        ei += (double)pot[k] * dens;
        ms += dens;
    }
    ek = block_sum(ek);
    ep = block_sum(ep);
    ei = block_sum(ei);
    ms = block_sum(ms);
    if (threadIdx.x == 0) {
        double* o = part + ((long long)b * nblk_stride + blockIdx.x) * 4;
        o[0] = 0.5 * g.dv * ek / (double)g.N;
        o[1] = g.dv * ep;
        o[2] = 0.5 * f.beta * g.dv * ei;
        o[3] = g.dv * ms;
    }
}

template <typename T>
__global__ void k_real_to_complex(long long count, const T* a, V2<T>* c) {
    for (long long i = (long long)blockIdx.x * RB_T + threadIdx.x; i < count; i += (long long)gridDim.x * RB_T)
        c[i] = mkc<T>(a[i], (T)0);
}

// ---- dynamics kernels -------------------------------------------------------------------------
// psi^ *= exp(-i |mu|^2 t / 2) / N   (exact kinetic flow over time t, with the FFT normalisation)
template <typename T>
__global__ void k_kin_phase(Geo g, int batch, V2<T>* psi, double t) {
    const int b = blockIdx.y;
    const double invN = 1.0 / (double)g.N;
    for (long long i = (long long)blockIdx.x * RB_T + threadIdx.x; i < g.N; i += (long long)gridDim.x * RB_T) {
        long long k = (long long)b * g.N + i;
        double ang = -0.5 * mu2(g, i) * t;
        double s, c;
        sincos(ang, &s, &c);
        V2<T> v = psi[k];
        double re = ((double)v.x * c - (double)v.y * s) * invN;
        double im = ((double)v.x * s + (double)v.y * c) * invN;
        psi[k] = mkc<T>((T)re, (T)im);
    }
}

template <typename T>
__global__ void k_density(long long count, const V2<T>* psi, T* rho) {
    for (long long i = (long long)blockIdx.x * RB_T + threadIdx.x; i < count; i += (long long)gridDim.x * RB_T) {
        V2<T> v = psi[i];
        rho[i] = (T)((double)v.x * v.x + (double)v.y * v.y);
    }
}

// psi *= exp(-i (V + beta varphi) t)
template <typename T>
__global__ void k_pot_phase(Geo g, const Fld* fl, const double* Vext, const T* pot, V2<T>* psi, double t) {
    const int b = blockIdx.y;
    const Fld f = fl[b];
    for (long long i = (long long)blockIdx.x * RB_T + threadIdx.x; i < g.N; i += (long long)gridDim.x * RB_T) {
        long long k = (long long)b * g.N + i;
        double x[3];
        int j[3];
        coords(g, i, x, j);
        double ang = -(trapV(g, f, Vext, i, x) + f.beta * (double)pot[k]) * t;
        double s, c;
        sincos(ang, &s, &c);
        V2<T> v = psi[k];
        psi[k] = mkc<T>((T)((double)v.x * c - (double)v.y * s), (T)((double)v.x * s + (double)v.y * c));
    }
}

template <typename T>
__global__ void k_copy_c(long long count, const V2<T>* a, V2<T>* b) {
    for (long long i = (long long)blockIdx.x * RB_T + threadIdx.x; i < count; i += (long long)gridDim.x * RB_T) b[i] = a[i];
}

template <typename A, typename Bt>
__device__ __forceinline__ void convert_body(long long count, const A* a, Bt* b, VBlk vb) {
    for (long long i = (long long)vb.x * RB_T + threadIdx.x; i < count; i += (long long)vb.gx * RB_T)
        b[i] = (Bt)a[i];
}
template <typename A, typename Bt>
__global__ void k_convert(long long count, const A* a, Bt* b) {
    convert_body<A, Bt>(count, a, b, hw_block());
}

// ---- step kernels as tasks ---------------------------------------------------------------------
// The kernels of a gradient-flow step take one argument record (the fields are the body's
// parameters), so that a launch can be recorded and replayed by the persistent executor.
template <typename T> struct Norm2T { Geo g; const Fld* fl; const T* v; double* part; };
template <typename T> struct NormalizeT { Geo g; Fld* fl; const T* v; T* phi; T* rho; const double* part_n; double* part_r; int nblk, track; };
template <typename T> struct ResidT { Fld* fl; const double* part_r; int nblk; double eps0; };
template <typename T> struct GfPrepT { Geo g; const Fld* fl; const double* Vext; const T* pot; const T* phi; T* W; V2<T>* cw; double* part_mx; double* part_mn; };
template <typename T> struct KinT { Geo g; const Fld* fl; V2<T>* cw; };
struct ShiftT { Fld* fl; const double* part_mx; const double* part_mn; int nblk; };
template <typename T> struct PcgInitT { Geo g; Fld* fl; const T* phi; const T* W; const V2<T>* kphi; T* x; T* r; V2<T>* zf; double* part_bb; };
struct BbT { Fld* fl; const double* part_bb; int nblk; };
template <typename T> struct RzT { Geo g; const Fld* fl; const V2<T>* zf; double* part_rz; };
template <typename T> struct DirT { Geo g; Fld* fl; const V2<T>* zf; V2<T>* cw; V2<T>* ph; const double* part_rz; int nblk; };
template <typename T> struct ApplyT { Geo g; const Fld* fl; const V2<T>* cw; const T* W; T* p; T* Ap; double* part_pap; };
template <typename T> struct UpdateT { Geo g; const Fld* fl; const T* p; const T* Ap; T* x; T* r; V2<T>* zf; const double* part_pap; double* part_rr; int nblk; };
struct CheckT { Fld* fl; const double* part_rr; int nblk; };
struct ToF64T { long long count; const float* a; double* b; };

template <typename T> __device__ __forceinline__ void apply(const Norm2T<T>& a, VBlk vb) { norm2_part_body<T>(a.g, a.fl, a.v, a.part, vb); }
template <typename T> __device__ __forceinline__ void apply(const NormalizeT<T>& a, VBlk vb) {
    normalize_body<T>(a.g, a.fl, a.v, a.phi, a.rho, a.part_n, a.part_r, a.nblk, a.track, vb);
}
template <typename T> __device__ __forceinline__ void apply(const ResidT<T>& a, VBlk vb) { residual_final_body<T>(a.fl, a.part_r, a.nblk, a.eps0, vb); }
template <typename T> __device__ __forceinline__ void apply(const GfPrepT<T>& a, VBlk vb) {
    gf_prep_body<T>(a.g, a.fl, a.Vext, a.pot, a.phi, a.W, a.cw, a.part_mx, a.part_mn, vb);
}
template <typename T> __device__ __forceinline__ void apply(const KinT<T>& a, VBlk vb) { kin_apply_body<T>(a.g, a.fl, a.cw, vb); }
__device__ __forceinline__ void apply(const ShiftT& a, VBlk vb) { shift_body(a.fl, a.part_mx, a.part_mn, a.nblk, vb); }
template <typename T> __device__ __forceinline__ void apply(const PcgInitT<T>& a, VBlk vb) {
    pcg_init_body<T>(a.g, a.fl, a.phi, a.W, a.kphi, a.x, a.r, a.zf, a.part_bb, vb);
}
__device__ __forceinline__ void apply(const BbT& a, VBlk vb) { bb_final_body(a.fl, a.part_bb, a.nblk, vb); }
template <typename T> __device__ __forceinline__ void apply(const RzT<T>& a, VBlk vb) { pcg_rz_body<T>(a.g, a.fl, a.zf, a.part_rz, vb); }
template <typename T> __device__ __forceinline__ void apply(const DirT<T>& a, VBlk vb) {
    pcg_dir_body<T>(a.g, a.fl, a.zf, a.cw, a.ph, a.part_rz, a.nblk, vb);
}
template <typename T> __device__ __forceinline__ void apply(const ApplyT<T>& a, VBlk vb) {
    pcg_apply_body<T>(a.g, a.fl, a.cw, a.W, a.p, a.Ap, a.part_pap, vb);
}
template <typename T> __device__ __forceinline__ void apply(const UpdateT<T>& a, VBlk vb) {
    pcg_update_body<T>(a.g, a.fl, a.p, a.Ap, a.x, a.r, a.zf, a.part_pap, a.part_rr, a.nblk, vb);
}
__device__ __forceinline__ void apply(const CheckT& a, VBlk vb) { pcg_check_body(a.fl, a.part_rr, a.nblk, vb); }
__device__ __forceinline__ void apply(const ToF64T& a, VBlk vb) { convert_body<float, double>(a.count, a.a, a.b, vb); }

template <class A>
__global__ void __launch_bounds__(RB_T) k_task(A a) {
    apply(a, hw_block());
}

template <typename T> constexpr int tk(int kd, int kf) { return std::is_same<T, double>::value ? kd : kf; }

// Launch one step kernel, or record it while a recorder is installed.
template <class A>
static int launch_task(nlf_plan* p, int kind, dim3 grid, const A& a) {
    if (Recorder* r = recorder()) return record(r, kind, grid, 0, a);
    hipLaunchKernelGGL((k_task<A>), grid, dim3(RB_T), 0, p->stream, a);
    NLF_HIP(hipGetLastError());
    return NLF_OK;
}

// ---- host side ----------------------------------------------------------------------------------
struct SolverWs {
    void* phi = nullptr;   // real [B][N] (GS) / unused
    void* x = nullptr;
    void* r = nullptr;
    void* p = nullptr;
    void* Ap = nullptr;
    void* W = nullptr;
    void* rho = nullptr;
    void* pot = nullptr;
    void* cw = nullptr;    // complex [B][N]
    void* ph = nullptr;    // complex [B][N]
    void* zf = nullptr;    // complex [(B+1)/2][N]: residual transforms of field pairs
    Fld* fl = nullptr;
    double* part = nullptr;    // 8 arrays of [B][MAXBLK]
    double* epart = nullptr;   // [B][MAXBLK][4]
};

static int ws_get(nlf_plan* p, SolverWs& w) {
    const size_t es = elem_size(p->prec) / 2, ec = elem_size(p->prec);
    const size_t B = p->batch, N = p->N;
    NLF_TRY(dev_alloc(p, &w.phi, B * N * es));
    NLF_TRY(dev_alloc(p, &w.x, B * N * es));
    NLF_TRY(dev_alloc(p, &w.r, B * N * es));
    NLF_TRY(dev_alloc(p, &w.p, B * N * es));
    NLF_TRY(dev_alloc(p, &w.Ap, B * N * es));
    NLF_TRY(dev_alloc(p, &w.W, B * N * es));
    NLF_TRY(dev_alloc(p, &w.rho, B * N * es));
    NLF_TRY(dev_alloc(p, &w.pot, B * N * es));
    NLF_TRY(dev_alloc(p, &w.cw, B * N * ec));
    NLF_TRY(dev_alloc(p, &w.ph, B * N * ec));
    NLF_TRY(dev_alloc(p, &w.zf, (B + 1) / 2 * N * ec));
    // the unpaired half of an odd batch stays 0; cleared on the plan's stream, ahead of the solve's
    // kernels (a fill on the legacy default stream is not ordered against a non-blocking stream)
    NLF_HIP(hipMemsetAsync(w.zf, 0, (B + 1) / 2 * N * ec, p->stream));
    NLF_TRY(dev_alloc(p, (void**)&w.fl, B * sizeof(Fld)));
    NLF_TRY(dev_alloc(p, (void**)&w.part, 8 * B * MAXBLK * sizeof(double)));
    NLF_TRY(dev_alloc(p, (void**)&w.epart, B * MAXBLK * 4 * sizeof(double)));
    return NLF_OK;
}

static Geo geo_of(const nlf_plan* p) {
    Geo g{};
    g.dim = p->dim;
    g.N = p->N;
    g.dv = 1;
    for (int i = 0; i < 3; ++i) {
        g.n[i] = p->n[i];
        g.L[i] = p->L[i];
        g.h[i] = p->h[i];
        g.lg[i] = 0;
        while ((1 << g.lg[i]) < p->n[i]) ++g.lg[i];
    }
    for (int i = 0; i < p->dim; ++i) g.dv *= p->h[i];
    return g;
}

static int nblocks(const nlf_plan* p) { return (int)std::min<long long>((p->N + RB_T - 1) / RB_T, MAXBLK); }

static void sws_delete(void* q) { delete static_cast<SolverWs*>(q); }

static int solver_ws(nlf_plan* p, SolverWs** out) {
    if (!p->sws) {
        SolverWs* w = new (std::nothrow) SolverWs();
        if (!w) return set_error(NLF_ENOMEM, "host allocation failed");
        int st = ws_get(p, *w);
        if (st != NLF_OK) {
            delete w;
            return st;
        }
        p->sws = w;
        p->sws_free = sws_delete;
    }
    *out = static_cast<SolverWs*>(p->sws);
    return NLF_OK;
}

static dim3 flat_grid(long long count) {
    return dim3((unsigned)std::max<long long>(1, std::min<long long>((count + RB_T - 1) / RB_T, 4096)));
}

// Energies of the fields: rho must hold |psi|^2 unless psi_c is given; out[b*4+q] = Ekin, Epot,
// Eint, mass.
template <typename T>
static int energies_t(nlf_plan* p, const Geo& g, SolverWs& w, const double* Vext, const void* psi_c,
                      const void* psi_r, std::vector<double>& out) {
    const int B = p->batch, nb = nblocks(p);
    const long long cnt = (long long)B * g.N;
    if (psi_c) {
        hipLaunchKernelGGL((k_density<T>), flat_grid(cnt), dim3(RB_T), 0, p->stream, cnt, (const V2<T>*)psi_c, (T*)w.rho);
        hipLaunchKernelGGL((k_copy_c<T>), flat_grid(cnt), dim3(RB_T), 0, p->stream, cnt, (const V2<T>*)psi_c, (V2<T>*)w.cw);
    } else {
        hipLaunchKernelGGL((k_real_to_complex<T>), flat_grid(cnt), dim3(RB_T), 0, p->stream, cnt, (const T*)psi_r,
                           (V2<T>*)w.cw);
    }
    NLF_HIP(hipGetLastError());
    NLF_TRY(potential(p, w.rho, w.pot));
    NLF_TRY(fft_full(p, w.cw, -1, B));
    hipLaunchKernelGGL((k_energy_part<T>), dim3(nb, B), dim3(RB_T), 0, p->stream, g, w.fl, Vext, (const V2<T>*)w.cw,
                       (const V2<T>*)psi_c, (const T*)psi_r, (const T*)w.pot, w.epart, nb);
    NLF_HIP(hipGetLastError());
    std::vector<double> h((size_t)B * nb * 4);
    NLF_HIP(hipMemcpyAsync(h.data(), w.epart, h.size() * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    NLF_HIP(hipStreamSynchronize(p->stream));
    out.assign((size_t)B * 4, 0.0);
    for (int b = 0; b < B; ++b)
        for (int i = 0; i < nb; ++i)
            for (int q = 0; q < 4; ++q) out[b * 4 + q] += h[((size_t)b * nb + i) * 4 + q];
    return NLF_OK;
}

static int read_flds(nlf_plan* p, SolverWs& w, std::vector<Fld>& fh) {
    NLF_HIP(hipMemcpyAsync(fh.data(), w.fl, fh.size() * sizeof(Fld), hipMemcpyDeviceToHost, p->stream));
    NLF_HIP(hipStreamSynchronize(p->stream));
    return NLF_OK;
}

struct GsParams {
    double tau, eps0, cg_tol;
    int max_iter, check_every, cg_max;
    int stall_stop;      // retire a field whose residual stopped decreasing (precision floor)
    int graphs;          // replay captured HIP graphs of the step's launches
};

static GsParams gs_params(const nlf_plan* p, const nlf_gf_opts* gf) {
    GsParams g;
    g.tau = (gf && gf->tau > 0) ? gf->tau : 1e-2;
    g.eps0 = (gf && gf->eps0 > 0) ? gf->eps0 : 1e-10;
    g.max_iter = (gf && gf->max_iter > 0) ? gf->max_iter : 100000;
    g.check_every = (gf && gf->check_every > 0) ? gf->check_every : 10;
    g.cg_tol = (gf && gf->cg_tol > 0) ? gf->cg_tol : (p->prec == NLF_F64 ? 1e-13 : 1e-6);
    g.cg_max = (gf && gf->cg_max_iter > 0) ? gf->cg_max_iter : 200;
    g.stall_stop = 0;
    g.graphs = (gf && gf->graph) ? 1 : 0;
    return g;
}

// A captured sequence of launches on the plan's stream, replayed with one hipGraphLaunch.  Capture
// records without executing; the body must only enqueue kernels (no synchronisation, no
// hipMemsetAsync: buffers are cleared by kernels).
struct StepGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    StepGraph() = default;
    StepGraph(const StepGraph&) = delete;
    StepGraph& operator=(const StepGraph&) = delete;
    ~StepGraph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

// Capture `body` into sg.  Returns false (HIP error state cleared, nothing enqueued) if the
// stream cannot be captured; the caller then launches directly.
template <class F>
static bool capture_graph(nlf_plan* p, StepGraph& sg, F&& body, int* rc) {
    *rc = NLF_OK;
    if (hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    *rc = body();
    hipGraph_t gr = nullptr;
    const hipError_t e = hipStreamEndCapture(p->stream, &gr);
    if (*rc != NLF_OK || e != hipSuccess || !gr) {
        (void)hipGetLastError();
        if (gr) (void)hipGraphDestroy(gr);
        if (*rc == NLF_OK) clear_error();
        return false;
    }
    if (hipGraphInstantiate(&sg.exec, gr, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipGraphDestroy(gr);
        sg.exec = nullptr;
        return false;
    }
    sg.graph = gr;
    return true;
}

// Run `body` directly, or (graphs on) capture it on first use and replay the graph.  A capture
// that fails turns graphs off for the rest of the solve (*graphs = false) and runs `body`.
template <class F>
static int run_step(nlf_plan* p, bool* graphs, StepGraph& sg, F&& body) {
    if (!*graphs) return body();
    if (!sg.exec) {
        int rc;
        if (!capture_graph(p, sg, body, &rc)) {
            *graphs = false;
            return body();
        }
    }
    NLF_HIP(hipGraphLaunch(sg.exec, p->stream));
    return NLF_OK;
}

// The legacy default stream cannot be captured.  While a solve runs on a plan created on it, the
// plan's work moves to a stream of its own (non-blocking, default priority), ordered after the
// caller's stream on entry and before it on exit.
struct SolveStream {
    nlf_plan* p;
    hipStream_t saved = nullptr;
    bool swapped = false;
    explicit SolveStream(nlf_plan* pl, bool want) : p(pl) {
        if (!want || p->stream != nullptr) return;
        if (!p->own_stream && hipStreamCreateWithFlags(&p->own_stream, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            p->own_stream = nullptr;
            return;
        }
        if (join(p->own_stream, p->stream)) {
            saved = p->stream;
            p->stream = p->own_stream;
            swapped = true;
        }
    }
    // make `later` wait for the work enqueued so far on `earlier`
    static bool join(hipStream_t later, hipStream_t earlier) {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        bool ok = hipEventRecord(e, earlier) == hipSuccess && hipStreamWaitEvent(later, e, 0) == hipSuccess;
        (void)hipEventDestroy(e);
        if (!ok) (void)hipGetLastError();
        return ok;
    }
    ~SolveStream() {
        if (!swapped) return;
        if (!join(saved, p->stream)) (void)hipStreamSynchronize(p->stream);
        p->stream = saved;
    }
};

// One plan's gradient-flow solve: its workspace, per-field state and partial-sum buffers.
template <typename T>
struct GsRun {
    nlf_plan* p = nullptr;
    SolverWs* w = nullptr;
    Geo g{};
    int B = 0, nb = 0;
    const double* Vext = nullptr;
    double eps0 = 0.0;
    std::vector<Fld> fh;
    double *part_n = nullptr, *part_r = nullptr, *part_mx = nullptr, *part_mn = nullptr;
    double *part_bb = nullptr, *part_rz = nullptr, *part_pap = nullptr, *part_rr = nullptr;
    dim3 grid;
};

// Workspace and the fields' parameters on the device (uploaded on the plan's stream).
template <typename T>
static int gs_prepare(nlf_plan* p, const nlf_phys* phys, const GsParams& gp, GsRun<T>& R) {
    NLF_TRY(solver_ws(p, &R.w));
    R.p = p;
    R.B = p->batch;
    R.nb = nblocks(p);
    R.g = geo_of(p);
    R.Vext = (const double*)phys[0].V_dev;
    R.eps0 = gp.eps0;
    R.fh.assign(R.B, Fld{});
    for (int b = 0; b < R.B; ++b) {
        Fld& f = R.fh[b];
        std::memset(&f, 0, sizeof(Fld));
        f.beta = phys[b].beta;
        for (int a = 0; a < 3; ++a) {
            double ga = (a < p->dim) ? phys[b].gamma[a] : 0.0;
            if (a < p->dim && !(ga > 0)) return set_error(NLF_EINVAL, "gamma[%d] of field %d must be positive", a, b);
            f.g2[a] = ga * ga;
        }
        f.tau = gp.tau;
        f.cgtol_min = gp.cg_tol;
        f.cgtol = std::max(gp.cg_tol, 1e-3);
        f.best_res = 1e300;
    }
    NLF_HIP(hipMemcpyAsync(R.w->fl, R.fh.data(), R.B * sizeof(Fld), hipMemcpyHostToDevice, p->stream));
    double* part = R.w->part;
    const long long stride = (long long)R.B * MAXBLK;
    R.part_n = part;
    R.part_r = part + 1 * stride;
    R.part_mx = part + 2 * stride;
    R.part_mn = part + 3 * stride;
    R.part_bb = part + 4 * stride;
    R.part_rz = part + 5 * stride;
    R.part_pap = part + 6 * stride;
    R.part_rr = part + 7 * stride;
    R.grid = dim3(R.nb, R.B);
    return NLF_OK;
}

// phi <- v / ||v|| (v may be phi itself), rho = phi^2, without tracking the residual.
template <typename T>
static int gs_normalise_from(GsRun<T>& R, const T* v) {
    SolverWs& w = *R.w;
    NLF_TRY(launch_task(R.p, tk<T>(TK_NORM2_D, TK_NORM2_F), R.grid, Norm2T<T>{R.g, w.fl, v, R.part_n}));
    return launch_task(R.p, tk<T>(TK_NORMALIZE_D, TK_NORMALIZE_F), R.grid,
                       NormalizeT<T>{R.g, w.fl, v, (T*)w.phi, (T*)w.rho, R.part_n, R.part_r, R.nb, 0});
}

// Initial state: psi0 (or the harmonic-oscillator Gaussian), normalised.
template <typename T>
static int gs_initial(GsRun<T>& R, const void* psi0) {
    nlf_plan* p = R.p;
    SolverWs& w = *R.w;
    const size_t rbytes = (size_t)R.B * R.g.N * (elem_size(p->prec) / 2);
    if (psi0) NLF_HIP(hipMemcpyAsync(w.phi, psi0, rbytes, hipMemcpyDeviceToDevice, p->stream));
    else hipLaunchKernelGGL((k_ho_init<T>), R.grid, dim3(RB_T), 0, p->stream, R.g, w.fl, (T*)w.phi);
    NLF_HIP(hipGetLastError());
    return gs_normalise_from<T>(R, (const T*)w.phi);
}

// The three parts of an outer step (Sec. 3.1, Eq. 'gf-eq2'); each only enqueues (or records) kernels.
// Set-up: the potential of rho = phi^2, W = V + beta varphi, the preconditioner shift, K phi, and the
// start of the inner solve.
template <typename T>
static int gs_setup(GsRun<T>& R) {
    nlf_plan* p = R.p;
    SolverWs& w = *R.w;
    const int B = R.B;
    NLF_TRY(potential(p, w.rho, w.pot));
    NLF_TRY(launch_task(p, tk<T>(TK_GFPREP_D, TK_GFPREP_F), R.grid,
                        GfPrepT<T>{R.g, w.fl, R.Vext, (const T*)w.pot, (const T*)w.phi, (T*)w.W, (V2<T>*)w.cw,
                                   R.part_mx, R.part_mn}));
    NLF_TRY(launch_task(p, TK_SHIFT, dim3(B), ShiftT{w.fl, R.part_mx, R.part_mn, R.nb}));
    NLF_TRY(fft_full(p, w.cw, -1, B));
    NLF_TRY(launch_task(p, tk<T>(TK_KIN_D, TK_KIN_F), R.grid, KinT<T>{R.g, w.fl, (V2<T>*)w.cw}));
    NLF_TRY(fft_full(p, w.cw, 1, B));
    NLF_TRY(launch_task(p, tk<T>(TK_PCGINIT_D, TK_PCGINIT_F), R.grid,
                        PcgInitT<T>{R.g, w.fl, (const T*)w.phi, (const T*)w.W, (const V2<T>*)w.cw, (T*)w.x, (T*)w.r,
                                    (V2<T>*)w.zf, R.part_bb}));
    return launch_task(p, TK_BB, dim3(B), BbT{w.fl, R.part_bb, R.nb});
}

// One inner (preconditioned conjugate-gradient) iteration; fields whose solve converged skip it.
template <typename T>
static int gs_cg(GsRun<T>& R) {
    nlf_plan* p = R.p;
    SolverWs& w = *R.w;
    const int B = R.B;
    NLF_TRY(fft_full(p, w.zf, -1, (B + 1) / 2));   // residuals of field pairs
    NLF_TRY(launch_task(p, tk<T>(TK_RZ_D, TK_RZ_F), R.grid, RzT<T>{R.g, w.fl, (const V2<T>*)w.zf, R.part_rz}));
    NLF_TRY(launch_task(p, tk<T>(TK_DIR_D, TK_DIR_F), R.grid,
                        DirT<T>{R.g, w.fl, (const V2<T>*)w.zf, (V2<T>*)w.cw, (V2<T>*)w.ph, R.part_rz, R.nb}));
    NLF_TRY(fft_full(p, w.cw, 1, B));
    NLF_TRY(launch_task(p, tk<T>(TK_APPLY_D, TK_APPLY_F), R.grid,
                        ApplyT<T>{R.g, w.fl, (const V2<T>*)w.cw, (const T*)w.W, (T*)w.p, (T*)w.Ap, R.part_pap}));
    NLF_TRY(launch_task(p, tk<T>(TK_UPDATE_D, TK_UPDATE_F), R.grid,
                        UpdateT<T>{R.g, w.fl, (const T*)w.p, (const T*)w.Ap, (T*)w.x, (T*)w.r, (V2<T>*)w.zf,
                                   R.part_pap, R.part_rr, R.nb}));
    return launch_task(p, TK_CHECK, dim3(B), CheckT{w.fl, R.part_rr, R.nb});
}

// Normalisation (Eq. 'gf-colb2'), the outer residual and the retirement of converged fields.
template <typename T>
static int gs_finish(GsRun<T>& R) {
    nlf_plan* p = R.p;
    SolverWs& w = *R.w;
    NLF_TRY(launch_task(p, tk<T>(TK_NORM2_D, TK_NORM2_F), R.grid, Norm2T<T>{R.g, w.fl, (const T*)w.x, R.part_n}));
    NLF_TRY(launch_task(p, tk<T>(TK_NORMALIZE_D, TK_NORMALIZE_F), R.grid,
                        NormalizeT<T>{R.g, w.fl, (const T*)w.x, (T*)w.phi, (T*)w.rho, R.part_n, R.part_r, R.nb, 1}));
    return launch_task(p, tk<T>(TK_RESID_D, TK_RESID_F), dim3(R.B), ResidT<T>{w.fl, R.part_r, R.nb, R.eps0});
}

// Energies, statistics and the output state (rho holds phi^2 from the last normalisation).  `steps`:
// outer steps run; stalled[b]: field b was retired at its precision floor, not at eps0.
template <typename T>
static int gs_end(GsRun<T>& R, const nlf_phys* phys, int steps, const std::vector<int>& stalled, void* psi,
                  nlf_gs_stats* stats, bool* all_done) {
    nlf_plan* p = R.p;
    SolverWs& w = *R.w;
    NLF_TRY(read_flds(p, w, R.fh));
    std::vector<double> e;
    NLF_TRY(energies_t<T>(p, R.g, w, R.Vext, nullptr, w.phi, e));
    bool all = true;
    for (int b = 0; b < R.B; ++b) {
        const Fld& f = R.fh[b];
        nlf_gs_stats& st = stats[b];
        st.iters = f.done ? f.done_at : steps;
        st.iters_fp32 = (sizeof(T) == 4) ? st.iters : 0;
        st.cg_iters = f.cg_iters;
        st.Ekin = e[b * 4 + 0];
        st.Epot = e[b * 4 + 1];
        st.Eint = e[b * 4 + 2];
        st.mass = e[b * 4 + 3];
        st.E = st.Ekin + st.Epot + st.Eint;
        st.mu = st.E + st.Eint;
        st.residual = f.res;
        st.virial = 2.0 * st.Ekin - 2.0 * st.Epot +
                    (p->kernel == NLF_LAPLACE2D ? phys[b].beta / (4.0 * 3.14159265358979323846) : st.Eint);
        st.persistent = 0;
        if (f.nonfinite) return set_error(NLF_ENONFINITE, "non-finite value in field %d", b);
        all = all && f.done && !stalled[b];
    }
    if (psi) {
        const size_t rbytes = (size_t)R.B * R.g.N * (elem_size(p->prec) / 2);
        NLF_HIP(hipMemcpyAsync(psi, w.phi, rbytes, hipMemcpyDeviceToDevice, p->stream));
    }
    NLF_HIP(hipStreamSynchronize(p->stream));
    *all_done = all;
    return NLF_OK;
}

template <typename T>
static int ground_state_t(nlf_plan* p, const nlf_phys* phys, const GsParams& gp, const void* psi0, void* psi,
                          nlf_gs_stats* stats) {
    SolveStream solve_stream(p, gp.graphs && !p->profiling);
    GsRun<T> R;
    NLF_TRY(gs_prepare<T>(p, phys, gp, R));
    NLF_TRY(gs_initial<T>(R, psi0));
    SolverWs& w = *R.w;
    const int B = R.B;
    const int max_iter = gp.max_iter, check_every = gp.check_every, cg_max = gp.cg_max;
    std::vector<Fld>& fh = R.fh;
    auto step_setup = [&]() -> int { return gs_setup<T>(R); };
    auto cg_block = [&]() -> int { return gs_cg<T>(R); };
    auto step_finish = [&]() -> int { return gs_finish<T>(R); };
    // Graphs are captured from the second outer step on (the first runs the launches directly,
    // which also sets the kernels' LDS attributes); stage profiling needs direct launches.
    StepGraph g_setup, g_cg, g_finish;
    bool want_graphs = gp.graphs && !p->profiling;

    int it = 0;
    bool all_done = false;
    int last_cg = 4;
    std::vector<double> best_res(B, 1e300);
    std::vector<int> stall(B, 0), stalled(B, 0);
    for (it = 1; it <= max_iter && !all_done; ++it) {
        bool graphs = want_graphs && it >= 2;
        NLF_TRY(run_step(p, &graphs, g_setup, step_setup));
        // convergence is read back first after about as many iterations as the previous solve took,
        // then every second iteration (each read is a stream synchronisation)
        int next_check = std::max(2, last_cg - 1);
        int most = 0;
        for (int cg = 0; cg < cg_max; ++cg) {
            NLF_TRY(run_step(p, &graphs, g_cg, cg_block));
            if (cg + 1 >= next_check) {
                NLF_TRY(read_flds(p, w, fh));
                bool all = true;
                for (int b = 0; b < B; ++b) {
                    all = all && (fh[b].done || fh[b].conv);
                    most = std::max(most, fh[b].cg_last);
                }
                if (all) break;
                next_check = cg + 3;
            }
        }
        last_cg = most;
        NLF_TRY(run_step(p, &graphs, g_finish, step_finish));
        if (it >= 2 && !graphs) want_graphs = false;
        if (it % check_every == 0 || it == max_iter) {
            NLF_TRY(read_flds(p, w, fh));
            all_done = true;
            bool retire = false;
            for (int b = 0; b < B; ++b) {
                if (fh[b].nonfinite) return set_error(NLF_ENONFINITE, "non-finite value in field %d at step %d", b, it);
                if (gp.stall_stop && !fh[b].done) {
                    // the residual of a precision-limited flow levels off at the rounding floor; a
                    // field that has not improved by 10% over three checks is retired
                    if (fh[b].res < 0.9 * best_res[b]) {
                        best_res[b] = fh[b].res;
                        stall[b] = 0;
                    } else if (++stall[b] >= 3) {
                        fh[b].done = 1;
                        fh[b].done_at = it;
                        stalled[b] = 1;
                        retire = true;
                    }
                }
                all_done = all_done && fh[b].done;
            }
            if (retire) NLF_HIP(hipMemcpyAsync(w.fl, fh.data(), B * sizeof(Fld), hipMemcpyHostToDevice, p->stream));
        }
    }
    bool all = false;
    NLF_TRY(gs_end<T>(R, phys, it - 1, stalled, psi, stats, &all));
    if (!all) return set_error(NLF_ENOCONV, "gradient flow did not reach eps0 = %g within %d steps", gp.eps0, max_iter);
    return NLF_OK;
}

// ---- persistent executor for batched ground states ------------------------------------------------
// nlf_ground_state_batch runs the gradient flow of every plan of the batch (plans of uneven grid
// size, each with its fields) in ONE cooperative launch: the kernels of one outer step of each plan
// are recorded once (set-up with the potential, one inner iteration, normalisation), and k_exec
// replays them on the device, the t-th recorded kernel of every plan together as one phase, with a
// grid barrier between phases.  The loops of the flow run on the device: an inner solve repeats
// until every field's conjugate-gradient solve has converged, the outer step until every field has
// retired at eps0 (a field retires on its own flag, its kernels then return at once).  With the
// mixed schedule the FP32 stage of every plan is followed, in the same launch, by the FP64 stage on
// the plans' FP64 twins.
constexpr int kMaxExecPlans = 16;

struct ExecStage {
    int n_init, n_setup, n_cg, n_fin;   // recorded kernels per list (equal for every plan)
    int init[kMaxExecPlans], setup[kMaxExecPlans], cg[kMaxExecPlans], fin[kMaxExecPlans];   // first task per plan
    Fld* fl[kMaxExecPlans];
    int stall_stop;                     // retire fields whose residual stopped decreasing (FP32 stage)
};
struct ExecProg {
    const TaskRec* tasks;
    int nplans, nstages;
    int B[kMaxExecPlans];
    ExecStage st[2];
    int max_iter, cg_max, check_every;
    unsigned long long* bar;            // barrier arrivals, zero at launch
    int* ctl;                           // [0] 1: a barrier timed out; [1 + s] outer steps of stage s
    unsigned long long timeout;         // per barrier, in wall_clock64() ticks
};

// Grid barrier of the cooperative launch: every workgroup arrives once per barrier; `passed` counts
// the arrivals the barrier waits for.  A barrier that has not completed after `timeout` ticks sets
// ctl[0]; every workgroup then leaves at its next barrier, so that the launch always ends.
__device__ __forceinline__ bool exec_barrier(const ExecProg& P, unsigned long long& passed) {
    __shared__ int ok;
    __syncthreads();
    passed += gridDim.x;
    if (threadIdx.x == 0) {
        __threadfence();   // release: the workgroup's stores (after the barrier above) reach memory
        atomicAdd(P.bar, 1ull);
        const unsigned long long t0 = wall_clock64();
        int good = 1;
        // relaxed polling, one acquire fence once every workgroup has arrived
        while (__hip_atomic_load(P.bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < passed) {
            if (__hip_atomic_load(P.ctl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                wall_clock64() - t0 > P.timeout) {
                atomicExch(P.ctl, 1);
                good = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __threadfence();
        ok = good && __hip_atomic_load(P.ctl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
    }
    __syncthreads();
    return ok;
}

__device__ __forceinline__ void run_task(const TaskRec& tk, VBlk vb, unsigned char* smem) {
    const void* a = tk.args;
    constexpr int NT = kExecThreads;
    switch (tk.kind) {
        case TK_ROWS_RHO_D: fft_rows_body<double, double, -1, LOAD_RHO, STORE_GRID, ExecRowCfg::E, true, NT>(*(const RowsArgs*)a, vb, smem); break;
        case TK_ROWS_RHO_F: fft_rows_body<float, float, -1, LOAD_RHO, STORE_GRID, ExecRowCfg::E, true, NT>(*(const RowsArgs*)a, vb, smem); break;
        case TK_ROWS_U_D: fft_rows_body<double, double, 1, LOAD_GRID, STORE_U, ExecRowCfg::E, true, NT>(*(const RowsArgs*)a, vb, smem); break;
        case TK_ROWS_U_DF: fft_rows_body<double, float, 1, LOAD_GRID, STORE_U, ExecRowCfg::E, true, NT>(*(const RowsArgs*)a, vb, smem); break;
        case TK_ROWS_FWD_D: fft_rows_body<double, double, -1, LOAD_GRID, STORE_GRID, ExecRowCfg::E, true, NT>(*(const RowsArgs*)a, vb, smem); break;
        case TK_ROWS_FWD_F: fft_rows_body<float, float, -1, LOAD_GRID, STORE_GRID, ExecRowCfg::E, true, NT>(*(const RowsArgs*)a, vb, smem); break;
        case TK_ROWS_INV_D: fft_rows_body<double, double, 1, LOAD_GRID, STORE_GRID, ExecRowCfg::E, true, NT>(*(const RowsArgs*)a, vb, smem); break;
        case TK_ROWS_INV_F: fft_rows_body<float, float, 1, LOAD_GRID, STORE_GRID, ExecRowCfg::E, true, NT>(*(const RowsArgs*)a, vb, smem); break;
        case TK_COLS_PFWD_D: fft_cols_body<double, -1, true, false, NT, ExecColCfg::E, true>(*(const ColsArgs*)a, vb, smem); break;
        case TK_COLS_PFWD_F: fft_cols_body<float, -1, true, false, NT, ExecColCfg::E, true>(*(const ColsArgs*)a, vb, smem); break;
        case TK_COLS_PINV_D: fft_cols_body<double, 1, false, true, NT, ExecColCfg::E, true>(*(const ColsArgs*)a, vb, smem); break;
        case TK_COLS_FWD_D: fft_cols_body<double, -1, false, false, NT, ExecColCfg::E, true>(*(const ColsArgs*)a, vb, smem); break;
        case TK_COLS_FWD_F: fft_cols_body<float, -1, false, false, NT, ExecColCfg::E, true>(*(const ColsArgs*)a, vb, smem); break;
        case TK_COLS_INV_D: fft_cols_body<double, 1, false, false, NT, ExecColCfg::E, true>(*(const ColsArgs*)a, vb, smem); break;
        case TK_COLS_INV_F: fft_cols_body<float, 1, false, false, NT, ExecColCfg::E, true>(*(const ColsArgs*)a, vb, smem); break;
        case TK_BINTERP_D: {
            const BinterpTask& t = *(const BinterpTask*)a;
            binterp2_body<double, 12>((const double2*)t.grid, t.gstride, t.na, t.ea, t.qq4, t.zero, t.zero16, vb, smem);
            break;
        }
        case TK_BINTERP_F: {
            const BinterpTask& t = *(const BinterpTask*)a;
            binterp2_32_body<7>((const float2*)t.grid, t.gstride, t.na, t.ea, t.qq4, t.qq1, t.zero, t.zero16, vb, smem);
            break;
        }
        case TK_MSPREAD_D: {
            const MspreadTask& t = *(const MspreadTask*)a;
            mspread_body<double, double, 12, 2, 128, false>((double2*)t.grid, t.gstride, (const double2*)t.cbuf, t.cstride,
                                                            t.na, t.items, t.nitems, t.cand, t.qq, t.ba, nullptr, 0, vb, smem);
            break;
        }
        case TK_MSPREAD_F: {
            const MspreadTask& t = *(const MspreadTask*)a;
            mspread32_body<7, 2, 128, false>((double2*)t.grid, t.gstride, (const float2*)t.cbuf, t.cstride, t.na, t.items,
                                             t.nitems, t.cand, t.qq, t.ba, nullptr, 0, vb, smem);
            break;
        }
        case TK_NORM2_D: apply(*(const Norm2T<double>*)a, vb); break;
        case TK_NORM2_F: apply(*(const Norm2T<float>*)a, vb); break;
        case TK_NORMALIZE_D: apply(*(const NormalizeT<double>*)a, vb); break;
        case TK_NORMALIZE_F: apply(*(const NormalizeT<float>*)a, vb); break;
        case TK_RESID_D: apply(*(const ResidT<double>*)a, vb); break;
        case TK_RESID_F: apply(*(const ResidT<float>*)a, vb); break;
        case TK_GFPREP_D: apply(*(const GfPrepT<double>*)a, vb); break;
        case TK_GFPREP_F: apply(*(const GfPrepT<float>*)a, vb); break;
        case TK_KIN_D: apply(*(const KinT<double>*)a, vb); break;
        case TK_KIN_F: apply(*(const KinT<float>*)a, vb); break;
        case TK_SHIFT: apply(*(const ShiftT*)a, vb); break;
        case TK_PCGINIT_D: apply(*(const PcgInitT<double>*)a, vb); break;
        case TK_PCGINIT_F: apply(*(const PcgInitT<float>*)a, vb); break;
        case TK_BB: apply(*(const BbT*)a, vb); break;
        case TK_RZ_D: apply(*(const RzT<double>*)a, vb); break;
        case TK_RZ_F: apply(*(const RzT<float>*)a, vb); break;
        case TK_DIR_D: apply(*(const DirT<double>*)a, vb); break;
        case TK_DIR_F: apply(*(const DirT<float>*)a, vb); break;
        case TK_APPLY_D: apply(*(const ApplyT<double>*)a, vb); break;
        case TK_APPLY_F: apply(*(const ApplyT<float>*)a, vb); break;
        case TK_UPDATE_D: apply(*(const UpdateT<double>*)a, vb); break;
        case TK_UPDATE_F: apply(*(const UpdateT<float>*)a, vb); break;
        case TK_CHECK: apply(*(const CheckT*)a, vb); break;
        case TK_TO_D: apply(*(const ToF64T*)a, vb); break;
        default: break;
    }
}

// One phase: the t-th task of every plan's list (first tasks offs[i]), their virtual blocks spread
// over the workgroups.  Each plan's count is rounded up to a multiple of 8, and the launch has a
// multiple of 8 workgroups, so a virtual block runs on the XCD that its index selects (workgroup w
// runs on XCD w mod 8), as in the kernels' own launches.
__device__ __forceinline__ void exec_phase(const ExecProg& P, const int* offs, int t, unsigned char* smem) {
    int base[kMaxExecPlans + 1];
    base[0] = 0;
    for (int i = 0; i < P.nplans; ++i) {
        const TaskRec& tk = P.tasks[offs[i] + t];
        base[i + 1] = base[i] + ((tk.gx * tk.gy * tk.gz + 7) & ~7);
    }
    for (int v = blockIdx.x; v < base[P.nplans]; v += gridDim.x) {
        int i = 0;
        while (v >= base[i + 1]) ++i;
        const TaskRec& tk = P.tasks[offs[i] + t];
        const int l = v - base[i];
        if (l >= tk.gx * tk.gy * tk.gz) continue;
        const VBlk vb{l % tk.gx, (l / tk.gx) % tk.gy, l / (tk.gx * tk.gy), tk.gx, tk.gy, tk.gz};
        run_task(tk, vb, smem);
        __syncthreads();   // the next virtual block reuses the LDS
    }
}

// any field of the stage still flowing (cg: still in its inner solve)
__device__ __forceinline__ bool exec_active(const ExecProg& P, const ExecStage& S, bool cg) {
    for (int i = 0; i < P.nplans; ++i)
        for (int b = 0; b < P.B[i]; ++b) {
            Fld* f = S.fl[i] + b;
            const int done = __hip_atomic_load(&f->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int conv = __hip_atomic_load(&f->conv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (!done && !(cg && conv)) return true;
        }
    return false;
}

// FP32 stage of the mixed schedule: a field whose residual has not improved by 10% over three checks
// has reached the FP32 floor and retires from the stage (one workgroup, between two barriers)
__device__ __forceinline__ void exec_stall(const ExecProg& P, const ExecStage& S, int step) {
    for (int i = 0; i < P.nplans; ++i)
        for (int b = threadIdx.x; b < P.B[i]; b += blockDim.x) {
            Fld* f = S.fl[i] + b;
            if (f->done) continue;
            if (f->res < 0.9 * f->best_res) {
                f->best_res = f->res;
                f->stall = 0;
            } else if (++f->stall >= 3) {
                f->done = 1;
                f->done_at = step;
            }
        }
}

__global__ void __launch_bounds__(kExecThreads, kExecWavesPerEU) k_exec(ExecProg P) {
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned long long passed = 0;
    int used = 0;   // outer steps of the earlier stage
    for (int s = 0; s < P.nstages; ++s) {
        const ExecStage& S = P.st[s];
        for (int t = 0; t < S.n_init; ++t) {
            exec_phase(P, S.init, t, smem);
            if (!exec_barrier(P, passed)) return;
        }
        const int max_steps = s == 0 ? P.max_iter : max(1, P.max_iter - used);
        int step = 0;
        while (step < max_steps && exec_active(P, S, false)) {
            for (int t = 0; t < S.n_setup; ++t) {
                exec_phase(P, S.setup, t, smem);
                if (!exec_barrier(P, passed)) return;
            }
            for (int it = 0; it < P.cg_max; ++it) {
                for (int t = 0; t < S.n_cg; ++t) {
                    exec_phase(P, S.cg, t, smem);
                    if (!exec_barrier(P, passed)) return;
                }
                if (!exec_active(P, S, true)) break;
            }
            for (int t = 0; t < S.n_fin; ++t) {
                exec_phase(P, S.fin, t, smem);
                if (!exec_barrier(P, passed)) return;
            }
            ++step;
            if (S.stall_stop && step % P.check_every == 0) {
                if (blockIdx.x == 0) exec_stall(P, S, step);
                if (!exec_barrier(P, passed)) return;
            }
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) P.ctl[1 + s] = step;
        used = step;
    }
}

// Record the kernels `fn` enqueues for the persistent executor into `out` (appended); returns the
// number recorded, or -1 if a launch has no executor body.
template <class F>
static int record_list(std::vector<TaskRec>& out, F&& fn) {
    Recorder rec;
    Recorder*& slot = recorder();
    Recorder* saved = slot;
    slot = &rec;
    const int st = fn();
    slot = saved;
    if (st != NLF_OK || rec.failed) return -1;
    out.insert(out.end(), rec.tasks.begin(), rec.tasks.end());
    return (int)rec.tasks.size();
}

// Can the batch run in the persistent executor: 2D plans of at most 256 points per axis (lines of
// at most 512 points on the oversampled grid), one precision, the default stencil widths, gather
// candidate lists, no stage timing, at most kMaxExecPlans plans.
static bool exec_eligible(int count, nlf_plan* const plans[], const nlf_gf_opts* gf) {
    if (!gf || !gf->persistent || gf->graph || count < 1 || count > kMaxExecPlans) return false;
    for (int i = 0; i < count; ++i) {
        const nlf_plan* p = plans[i];
        if (p->dim != 2 || p->sub || p->deterministic || p->profiling || !p->use_gather) return false;
        if (p->spread_mode != NLF_SPREAD_GATHER) return false;
        if (p->n[0] > 256 || p->n[1] > 256 || p->prec != plans[0]->prec) return false;
        if (p->msp != (p->prec == NLF_F64 ? 12 : 7)) return false;
        if (p->prec == NLF_F32 && p->t1_prec != NLF_F64) return false;
        if (p->kernel != NLF_COULOMB2D && p->kernel != NLF_LAPLACE2D && p->kernel != NLF_CONFINED2D) return false;
    }
    return true;
}

// The FP64 twin of an FP32 plan (mixed schedule), created on first use and owned by the plan.
static int twin_of(nlf_plan* p, nlf_plan** out) {
    if (!p->twin) {
        nlf_opts o = p->opts_copy;
        o.prec = NLF_F64;
        o.msp = 0;
        o.batch = p->batch;
        NLF_TRY(nlf_plan_create(&p->box_copy, p->kernel, &o, p->stream, &p->twin));
    }
    *out = p->twin;
    return NLF_OK;
}

// Record one stage's lists of every plan into `tasks` and the stage's table.
template <typename T>
static int record_stage(std::vector<GsRun<T>>& R, std::vector<TaskRec>& tasks, ExecStage& S,
                        const std::vector<GsRun<float>>* from32) {
    const int n = (int)R.size();
    int len[4] = {-2, -2, -2, -2};
    for (int i = 0; i < n; ++i) {
        GsRun<T>& r = R[i];
        nlf_plan* p = r.p;
        // the executor's spreading body takes 128-candidate blocks (the work items are unchanged)
        const int kc = p->spread_kc;
        p->spread_kc = 128;
        int l[4];
        const int off[4] = {(int)tasks.size(), 0, 0, 0};
        S.init[i] = off[0];
        l[0] = from32 ? record_list(tasks, [&]() -> int {
            const GsRun<float>& f = (*from32)[i];
            NLF_TRY(launch_task(p, TK_TO_D, flat_grid((long long)r.B * r.g.N),
                                ToF64T{(long long)r.B * r.g.N, (const float*)f.w->phi, (double*)r.w->phi}));
            return gs_normalise_from<T>(r, (const T*)r.w->phi);
        }) : 0;
        S.setup[i] = (int)tasks.size();
        l[1] = record_list(tasks, [&]() { return gs_setup<T>(r); });
        S.cg[i] = (int)tasks.size();
        l[2] = record_list(tasks, [&]() { return gs_cg<T>(r); });
        S.fin[i] = (int)tasks.size();
        l[3] = record_list(tasks, [&]() { return gs_finish<T>(r); });
        p->spread_kc = kc;
        for (int k = 0; k < 4; ++k) {
            if (l[k] < 0 || (len[k] != -2 && len[k] != l[k])) return set_error(NLF_EUNSUPPORTED, "plan %d: no executor program", i);
            len[k] = l[k];
        }
        S.fl[i] = r.w->fl;
    }
    S.n_init = len[0];
    S.n_setup = len[1];
    S.n_cg = len[2];
    S.n_fin = len[3];
    return NLF_OK;
}

// The persistent batched solve (see the executor above).  The launch goes on the first plan's
// stream, ordered after every plan's earlier work and before its later work.
template <typename T>
static int exec_batch(int count, nlf_plan* const plans[], const nlf_phys* const phys[], const nlf_gf_opts* gf,
                      const void* const psi0[], void* const psi[], nlf_gs_stats* const stats[]) {
    const bool mixed = std::is_same<T, float>::value && gf && gf->mixed;
    hipStream_t st0 = plans[0]->stream;
    for (int i = 1; i < count; ++i)
        if (!SolveStream::join(st0, plans[i]->stream)) return set_error(NLF_EHIP, "ordering the plans' streams failed");
    GsParams g0 = gs_params(plans[0], gf);
    if (mixed) {
        g0.eps0 = std::max(g0.eps0, (gf->eps_switch > 0) ? gf->eps_switch : 1e-5);
        g0.stall_stop = 1;
    }
    std::vector<GsRun<T>> R0(count);
    std::vector<GsRun<double>> R1(mixed ? count : 0);
    std::vector<TaskRec> tasks;
    ExecProg P{};
    P.nplans = count;
    P.nstages = mixed ? 2 : 1;
    for (int i = 0; i < count; ++i) {
        nlf_plan* p = plans[i];
        p->stream = st0;   // every plan's work of this call goes on the executor's stream
        NLF_TRY(gs_prepare<T>(p, phys[i], gs_params(p, gf), R0[i]));
        R0[i].eps0 = g0.eps0;
        // the FP32 stage's inner tolerance is that of an FP32 plan; the flags of the stage are set
        NLF_TRY(gs_initial<T>(R0[i], psi0 ? psi0[i] : nullptr));
        P.B[i] = p->batch;
    }
    P.st[0].stall_stop = g0.stall_stop;
    NLF_TRY(record_stage<T>(R0, tasks, P.st[0], nullptr));
    if (mixed) {
        for (int i = 0; i < count; ++i) {
            nlf_plan* tw;
            NLF_TRY(twin_of(plans[i], &tw));
            tw->stream = st0;
            if (!tw->use_gather || tw->spread_mode != NLF_SPREAD_GATHER)
                return set_error(NLF_EUNSUPPORTED, "plan %d: the FP64 twin does not spread by gather lists", i);
            GsParams g1 = gs_params(tw, gf);
            NLF_TRY(gs_prepare<double>(tw, phys[i], g1, R1[i]));
        }
        if constexpr (std::is_same<T, float>::value) NLF_TRY(record_stage<double>(R1, tasks, P.st[1], &R0));
    }
    // stage-0 state as gs_prepare wrote it, with the stall tracking of the executor
    P.max_iter = g0.max_iter;
    P.cg_max = g0.cg_max;
    P.check_every = g0.check_every;
    size_t lds = 0;
    for (const TaskRec& t : tasks) lds = std::max(lds, (size_t)t.lds);
    lds = std::max<size_t>(lds, Binterp2Lds<12>::bytes);
    lds = std::max<size_t>(lds, Binterp2Lds32<7>::bytes);
    lds = std::max<size_t>(lds, mspread_lds<128, false>());
    lds = std::max<size_t>(lds, mspread32_lds<128, false>());
    // device copies of the program and the control words
    TaskRec* dtasks = nullptr;
    unsigned long long* dctl = nullptr;
    NLF_HIP(hipMalloc(&dtasks, tasks.size() * sizeof(TaskRec)));
    if (hipMalloc(&dctl, 64) != hipSuccess) {
        (void)hipFree(dtasks);
        return set_error(NLF_ENOMEM, "hipMalloc of the executor's control words failed");
    }
    int rc = NLF_OK;
    int ctl[4] = {0, 0, 0, 0};
    do {
        if (hipMemcpyAsync(dtasks, tasks.data(), tasks.size() * sizeof(TaskRec), hipMemcpyHostToDevice, st0) != hipSuccess ||
            hipMemsetAsync(dctl, 0, 64, st0) != hipSuccess) {
            rc = set_error(NLF_EHIP, "uploading the executor program failed");
            break;
        }
        P.tasks = dtasks;
        P.bar = dctl;
        P.ctl = reinterpret_cast<int*>(dctl + 1);
        int rate_khz = 0, dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            rc = set_error(NLF_EHIP, "device attributes for the executor failed");
            break;
        }
        P.timeout = (unsigned long long)std::max(rate_khz, 1000) * 20000ull;   // 20 s per barrier
        if (lds > 64 * 1024 &&
            hipFuncSetAttribute((const void*)&k_exec, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) {
            rc = set_error(NLF_EHIP, "raising the executor's LDS to %zu bytes failed", lds);
            break;
        }
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)&k_exec, kExecThreads, lds) != hipSuccess ||
            per_cu < 1) {
            rc = set_error(NLF_EHIP, "the executor does not fit a CU (%zu bytes of LDS)", lds);
            break;
        }
        // kExecPerCU workgroups per CU (fewer if fewer fit): a grid barrier costs its workgroups'
        // fences (each an L2 write-back on this multi-XCD device) and polls
        const int nwg = std::max(8, cus / 8 * 8) * std::min(per_cu, kExecPerCU);
        void* args[] = {&P};
        if (hipLaunchCooperativeKernel((const void*)&k_exec, dim3(nwg), dim3(kExecThreads), args, (unsigned)lds, st0) !=
            hipSuccess) {
            (void)hipGetLastError();
            rc = set_error(NLF_EHIP, "cooperative launch of the executor (%d workgroups) failed", nwg);
            break;
        }
        if (hipMemcpyAsync(ctl, P.ctl, sizeof ctl, hipMemcpyDeviceToHost, st0) != hipSuccess ||
            hipStreamSynchronize(st0) != hipSuccess) {
            rc = set_error(NLF_EHIP, "the executor failed");
            break;
        }
        if (ctl[0]) rc = set_error(NLF_EHIP, "the executor's grid barrier timed out");
    } while (0);
    (void)hipFree(dtasks);
    (void)hipFree(dctl);
    if (rc != NLF_OK) return rc;
    // statistics, energies (FP64 state for the mixed schedule) and outputs
    int noconv = -1;
    for (int i = 0; i < count; ++i) {
        nlf_plan* p = plans[i];
        const int B = p->batch;
        std::vector<int> none(B, 0);
        bool all = false;
        if (!mixed) {
            NLF_TRY(gs_end<T>(R0[i], phys[i], ctl[1], none, psi[i], stats[i], &all));
        } else {
            std::vector<nlf_gs_stats> s0(B);
            NLF_TRY(read_flds(p, *R0[i].w, R0[i].fh));
            NLF_TRY(gs_end<double>(R1[i], phys[i], ctl[2], none, nullptr, stats[i], &all));
            for (int b = 0; b < B; ++b) {
                const Fld& f0 = R0[i].fh[b];
                const int it0 = f0.done ? f0.done_at : ctl[1];
                stats[i][b].iters += it0;
                stats[i][b].iters_fp32 = it0;
                stats[i][b].cg_iters += f0.cg_iters;
            }
            const long long cnt = (long long)B * p->N;
            hipLaunchKernelGGL((k_convert<double, float>), flat_grid(cnt), dim3(RB_T), 0, st0, cnt,
                               (const double*)R1[i].w->phi, (float*)psi[i]);
            NLF_HIP(hipGetLastError());
        }
        for (int b = 0; b < B; ++b) stats[i][b].persistent = 1;
        if (!all && noconv < 0) noconv = i;
    }
    NLF_HIP(hipStreamSynchronize(st0));
    if (noconv >= 0) return set_error(NLF_ENOCONV, "plan %d: the gradient flow did not reach eps0", noconv);
    return NLF_OK;
}

template <typename T>
static int evolve_t(nlf_plan* p, const nlf_phys* phys, const nlf_ts_opts* ts, void* psi, double* diag) {
    SolverWs* wp;
    NLF_TRY(solver_ws(p, &wp));
    SolverWs& w = *wp;
    const int B = p->batch, nb = nblocks(p);
    const Geo g = geo_of(p);
    const double dt = ts->dt;
    const int nsteps = ts->nsteps, order = ts->order ? ts->order : 2, de = ts->diag_every;
    if (!(dt > 0) || nsteps < 0 || (order != 2 && order != 4) || de < 0)
        return set_error(NLF_EINVAL, "need dt > 0, nsteps >= 0, order 2 or 4, diag_every >= 0");
    const double* Vext = (const double*)phys[0].V_dev;
    std::vector<Fld> fh(B);
    for (int b = 0; b < B; ++b) {
        std::memset(&fh[b], 0, sizeof(Fld));
        fh[b].beta = phys[b].beta;
        for (int a = 0; a < 3; ++a) fh[b].g2[a] = (a < p->dim) ? phys[b].gamma[a] * phys[b].gamma[a] : 0.0;
    }
    NLF_HIP(hipMemcpyAsync(w.fl, fh.data(), B * sizeof(Fld), hipMemcpyHostToDevice, p->stream));
    const dim3 grid(nb, B);
    // the phase kernels reduce nothing: as many blocks as the grid needs (up to 4096 per field),
    // not the MAXBLK of the reductions, so that large grids keep enough waves in flight
    const dim3 pgrid((unsigned)std::min<long long>((g.N + RB_T - 1) / RB_T, 4096), B);
    const long long cnt = (long long)B * g.N;
    double pending = 0.0;   // kinetic time not yet applied (adjacent half steps are merged)

    auto flush_kin = [&]() -> int {
        if (pending != 0.0) {
            NLF_TRY(fft_full(p, psi, -1, B));
            hipLaunchKernelGGL((k_kin_phase<T>), pgrid, dim3(RB_T), 0, p->stream, g, B, (V2<T>*)psi, pending);
            NLF_HIP(hipGetLastError());
            NLF_TRY(fft_full(p, psi, 1, B));
            pending = 0.0;
        }
        return NLF_OK;
    };
    auto strang = [&](double t) -> int {
        pending += 0.5 * t;
        NLF_TRY(flush_kin());
        hipLaunchKernelGGL((k_density<T>), flat_grid(cnt), dim3(RB_T), 0, p->stream, cnt, (const V2<T>*)psi, (T*)w.rho);
        NLF_HIP(hipGetLastError());
        NLF_TRY(potential(p, w.rho, w.pot));
        hipLaunchKernelGGL((k_pot_phase<T>), pgrid, dim3(RB_T), 0, p->stream, g, w.fl, Vext, (const T*)w.pot,
                           (V2<T>*)psi, t);
        NLF_HIP(hipGetLastError());
        pending += 0.5 * t;
        return NLF_OK;
    };
    auto record = [&](int slot) -> int {
        NLF_TRY(flush_kin());
        std::vector<double> e;
        NLF_TRY(energies_t<T>(p, g, w, Vext, psi, nullptr, e));
        for (int b = 0; b < B; ++b) {
            diag[((size_t)slot * B + b) * 2 + 0] = e[b * 4 + 3];
            diag[((size_t)slot * B + b) * 2 + 1] = e[b * 4 + 0] + e[b * 4 + 1] + e[b * 4 + 2];
        }
        return NLF_OK;
    };
    const double w1 = 1.0 / (2.0 - std::cbrt(2.0)), w0 = -std::cbrt(2.0) / (2.0 - std::cbrt(2.0));
    int slot = 0;
    if (de && diag) NLF_TRY(record(slot++));
    for (int s = 1; s <= nsteps; ++s) {
        if (order == 2) NLF_TRY(strang(dt));
        else {
            NLF_TRY(strang(w1 * dt));
            NLF_TRY(strang(w0 * dt));
            NLF_TRY(strang(w1 * dt));
        }
        if (de && diag && s % de == 0) NLF_TRY(record(slot++));
    }
    NLF_TRY(flush_kin());
    NLF_HIP(hipStreamSynchronize(p->stream));
    return NLF_OK;
}

int ho_guess(nlf_plan* p, const nlf_phys* phys, void* out) {
    SolverWs* wp;
    NLF_TRY(solver_ws(p, &wp));
    const int B = p->batch;
    std::vector<Fld> fh(B);
    for (int b = 0; b < B; ++b) {
        std::memset(&fh[b], 0, sizeof(Fld));
        for (int a = 0; a < 3; ++a) fh[b].g2[a] = (a < p->dim) ? phys[b].gamma[a] * phys[b].gamma[a] : 0.0;
    }
    NLF_HIP(hipMemcpyAsync(wp->fl, fh.data(), B * sizeof(Fld), hipMemcpyHostToDevice, p->stream));
    const Geo g = geo_of(p);
    dim3 grid(nblocks(p), B);
    if (p->prec == NLF_F64) hipLaunchKernelGGL((k_ho_init<double>), grid, dim3(RB_T), 0, p->stream, g, wp->fl, (double*)out);
    else hipLaunchKernelGGL((k_ho_init<float>), grid, dim3(RB_T), 0, p->stream, g, wp->fl, (float*)out);
    NLF_HIP(hipGetLastError());
    NLF_HIP(hipStreamSynchronize(p->stream));
    return NLF_OK;
}

}  // namespace nlf

using namespace nlf;

extern "C" {

int nlf_ground_state(nlf_plan* p, const nlf_phys* phys, const nlf_gf_opts* gf, const void* psi0, void* psi,
                     nlf_gs_stats* stats) {
    clear_error();
    if (!p || !phys || !psi || !stats) return set_error(NLF_EINVAL, "plan, phys, psi and stats must not be NULL");
    GsParams gp = gs_params(p, gf);
    if (p->prec == NLF_F64) return ground_state_t<double>(p, phys, gp, psi0, psi, stats);
    if (!(gf && gf->mixed)) return ground_state_t<float>(p, phys, gp, psi0, psi, stats);

    // mixed schedule: FP32 down to eps_switch (or the FP32 floor), then FP64 on the twin plan
    const double eps_final = gp.eps0;
    GsParams g1 = gp;
    g1.eps0 = std::max(eps_final, (gf->eps_switch > 0) ? gf->eps_switch : 1e-5);
    g1.stall_stop = 1;
    const int B = p->batch;
    std::vector<nlf_gs_stats> s1(B), s2(B);
    int st = ground_state_t<float>(p, phys, g1, psi0, psi, s1.data());
    if (st != NLF_OK && st != NLF_ENOCONV) return st;
    if (!p->twin) {
        nlf_opts o = p->opts_copy;
        o.prec = NLF_F64;
        o.msp = 0;
        o.batch = p->batch;
        NLF_TRY(nlf_plan_create(&p->box_copy, p->kernel, &o, p->stream, &p->twin));
    }
    SolverWs* w2;
    NLF_TRY(solver_ws(p->twin, &w2));
    const long long cnt = (long long)B * p->N;
    // the twin's x buffer carries the FP32 state in FP64 as the initial guess
    hipLaunchKernelGGL((k_convert<float, double>), flat_grid(cnt), dim3(RB_T), 0, p->stream, cnt, (const float*)psi,
                       (double*)w2->x);
    NLF_HIP(hipGetLastError());
    GsParams g2 = gs_params(p->twin, gf);
    g2.eps0 = eps_final;
    int used = 0;
    for (int b = 0; b < B; ++b) used = std::max(used, s1[b].iters);
    g2.max_iter = std::max(1, gp.max_iter - used);
    st = ground_state_t<double>(p->twin, phys, g2, w2->x, w2->Ap, s2.data());
    if (st != NLF_OK && st != NLF_ENOCONV) return st;
    hipLaunchKernelGGL((k_convert<double, float>), flat_grid(cnt), dim3(RB_T), 0, p->stream, cnt, (const double*)w2->Ap,
                       (float*)psi);
    NLF_HIP(hipGetLastError());
    NLF_HIP(hipStreamSynchronize(p->stream));
    for (int b = 0; b < B; ++b) {
        stats[b] = s2[b];
        stats[b].iters = s1[b].iters + s2[b].iters;
        stats[b].iters_fp32 = s1[b].iters;
        stats[b].cg_iters = s1[b].cg_iters + s2[b].cg_iters;
    }
    if (st == NLF_ENOCONV) return set_error(NLF_ENOCONV, "mixed-precision gradient flow did not reach eps0 = %g", eps_final);
    return NLF_OK;
}

int nlf_ground_state_batch(int count, nlf_plan* const plans[], const nlf_phys* const phys[], const nlf_gf_opts* gf,
                           const void* const psi0[], void* const psi[], nlf_gs_stats* const stats[]) {
    clear_error();
    if (count < 0 || (count > 0 && (!plans || !phys || !psi || !stats)))
        return set_error(NLF_EINVAL, "count must be >= 0 and the arrays non-NULL");
    for (int i = 0; i < count; ++i)
        if (!plans[i] || !phys[i] || !psi[i] || !stats[i]) return set_error(NLF_EINVAL, "entry %d has a NULL pointer", i);
    if (exec_eligible(count, plans, gf)) {
        // one persistent launch for the whole batch; the plans' streams are restored afterwards
        std::vector<hipStream_t> saved(count);
        for (int i = 0; i < count; ++i) saved[i] = plans[i]->stream;
        const int st = plans[0]->prec == NLF_F64 ? exec_batch<double>(count, plans, phys, gf, psi0, psi, stats)
                                                 : exec_batch<float>(count, plans, phys, gf, psi0, psi, stats);
        for (int i = 0; i < count; ++i) {
            plans[i]->stream = saved[i];
            if (plans[i]->twin) plans[i]->twin->stream = saved[i];
        }
        for (int i = 1; i < count; ++i) (void)SolveStream::join(saved[i], saved[0]);
        if (st != NLF_EUNSUPPORTED) return st;
        clear_error();   // a plan the executor cannot record: the threaded path below
    }
    int dev = 0;
    NLF_HIP(hipGetDevice(&dev));
    std::vector<int> status(count, NLF_OK);
    std::vector<std::string> msg(count);
    std::vector<std::thread> th;
    for (int i = 0; i < count; ++i) {
        th.emplace_back([&, i]() {
            if (hipSetDevice(dev) != hipSuccess) {
                status[i] = NLF_EHIP;
                msg[i] = "hipSetDevice failed in a solver thread";
                return;
            }
            status[i] = nlf_ground_state(plans[i], phys[i], gf, psi0 ? psi0[i] : nullptr, psi[i], stats[i]);
            msg[i] = nlf_last_error();
        });
    }
    for (auto& t : th) t.join();
    int noconv = -1;
    for (int i = 0; i < count; ++i) {
        if (status[i] != NLF_OK && status[i] != NLF_ENOCONV)
            return set_error(status[i], "plan %d: %s", i, msg[i].c_str());
        if (status[i] == NLF_ENOCONV && noconv < 0) noconv = i;
    }
    if (noconv >= 0) return set_error(NLF_ENOCONV, "plan %d: %s", noconv, msg[noconv].c_str());
    return NLF_OK;
}

int nlf_evolve(nlf_plan* p, const nlf_phys* phys, const nlf_ts_opts* ts, void* psi, double* diag) {
    clear_error();
    if (!p || !phys || !ts || !psi) return set_error(NLF_EINVAL, "plan, phys, ts and psi must not be NULL");
    return p->prec == NLF_F64 ? evolve_t<double>(p, phys, ts, psi, diag) : evolve_t<float>(p, phys, ts, psi, diag);
}

}  // extern "C"
