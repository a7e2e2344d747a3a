// Orbit fit of the progenitor (Sec. 2.2.2): one test particle integrated forward
// and backward from its present-day point in the host potential, compared with a
// stream track through a chi-squared statistic; Levenberg-Marquardt from many
// starts, and the Fisher matrix from the exact Hessian.
//
// Parameters are p = log10(M_NFW, rs_NFW, M_MN, a_MN, b_MN).  Derivatives are
// carried through the integrator in forward mode by jet arithmetic:
//   J1<5> : value and the five first derivatives (residuals with their Jacobian
//           rows, which is what Levenberg-Marquardt needs);
//   HD    : hyper-dual numbers v + a e1 + b e2 + c e1 e2 (e1^2 = e2^2 = 0), whose
//           e1 e2 part is the exact mixed second derivative along the two seeded
//           directions; fifteen lanes give the symmetric 5 x 5 Hessian.
// One lane integrates one orbit; a batch of starts (or of parameter pairs) fills
// the launch.  All arithmetic is FP64.
//
// Observables in the orbit-aligned frame (e1, e2, n) of the present-day point:
// phi1 accumulated as the sum of per-step turning angles atan(cross / dot) from
// phi1(0) = 0, phi2 = asin(x.n / |x|), d = |x|, v_r = x.v / |x|.  A track point
// (phi1_k; phi2_k, d_k, v_r,k) is compared with the linear interpolation along
// phi1 on the first segment, in time order from t = 0, whose phi1 interval holds
// phi1_k (forward branch for phi1_k >= 0, backward otherwise); a point that no
// segment reaches makes chi2 infinite.
#include <cmath>

#include "dnb_internal.h"
#include "../../include/dnb_orbitfit.h"

namespace dnb {

constexpr int NPAR = 5;
constexpr int NTRI = 15;           // packed upper triangle of a 5 x 5 matrix
constexpr double LN10 = 2.302585092994045684;

// ------------------------------------------------------------------- jets ---
template <int N>
struct J1 {
    double v;
    double d[N];
};

struct HD {
    double v, a, b, c;
};

__device__ inline double val(double x) { return x; }
template <int N> __device__ inline double val(const J1<N>& x) { return x.v; }
__device__ inline double val(const HD& x) { return x.v; }

// constant of the jet type
template <class T> __device__ inline T cst(double x);
template <> __device__ inline double cst<double>(double x) { return x; }
template <> __device__ inline J1<NPAR> cst<J1<NPAR>>(double x) {
    J1<NPAR> r;
    r.v = x;
#pragma unroll
    for (int i = 0; i < NPAR; ++i) r.d[i] = 0.0;
    return r;
}
template <> __device__ inline HD cst<HD>(double x) { return HD{x, 0.0, 0.0, 0.0}; }

// f(x) from f(val x), f'(val x), f''(val x)
__device__ inline double chain(double, double f, double, double) { return f; }
template <int N>
__device__ inline J1<N> chain(const J1<N>& x, double f, double f1, double) {
    J1<N> r;
    r.v = f;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = f1 * x.d[i];
    return r;
}
__device__ inline HD chain(const HD& x, double f, double f1, double f2) {
    return HD{f, f1 * x.a, f1 * x.b, f1 * x.c + f2 * x.a * x.b};
}

template <int N>
__device__ inline J1<N> operator+(const J1<N>& x, const J1<N>& y) {
    J1<N> r;
    r.v = x.v + y.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = x.d[i] + y.d[i];
    return r;
}
template <int N>
__device__ inline J1<N> operator-(const J1<N>& x, const J1<N>& y) {
    J1<N> r;
    r.v = x.v - y.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = x.d[i] - y.d[i];
    return r;
}
template <int N>
__device__ inline J1<N> operator*(const J1<N>& x, const J1<N>& y) {
    J1<N> r;
    r.v = x.v * y.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = x.v * y.d[i] + x.d[i] * y.v;
    return r;
}
template <int N>
__device__ inline J1<N> operator*(double s, const J1<N>& x) {
    J1<N> r;
    r.v = s * x.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = s * x.d[i];
    return r;
}
template <int N>
__device__ inline J1<N> operator+(const J1<N>& x, double s) {
    J1<N> r = x;
    r.v = x.v + s;
    return r;
}
template <int N> __device__ inline J1<N> operator-(const J1<N>& x) { return -1.0 * x; }

__device__ inline HD operator+(const HD& x, const HD& y) {
    return HD{x.v + y.v, x.a + y.a, x.b + y.b, x.c + y.c};
}
__device__ inline HD operator-(const HD& x, const HD& y) {
    return HD{x.v - y.v, x.a - y.a, x.b - y.b, x.c - y.c};
}
__device__ inline HD operator*(const HD& x, const HD& y) {
    return HD{x.v * y.v, x.v * y.a + x.a * y.v, x.v * y.b + x.b * y.v,
              x.v * y.c + x.a * y.b + x.b * y.a + x.c * y.v};
}
__device__ inline HD operator*(double s, const HD& x) {
    return HD{s * x.v, s * x.a, s * x.b, s * x.c};
}
__device__ inline HD operator+(const HD& x, double s) { return HD{x.v + s, x.a, x.b, x.c}; }
__device__ inline HD operator-(const HD& x) { return -1.0 * x; }

template <class T> __device__ inline T recip(const T& x) {
    const double r = 1.0 / val(x);
    return chain(x, r, -r * r, 2.0 * r * r * r);
}
__device__ inline double recip(double x) { return 1.0 / x; }
template <int N> __device__ inline J1<N> operator/(const J1<N>& x, const J1<N>& y) {
    return x * recip(y);
}
__device__ inline HD operator/(const HD& x, const HD& y) { return x * recip(y); }

template <class T> __device__ inline T jsqrt(const T& x) {
    const double s = sqrt(val(x));
    return chain(x, s, 0.5 / s, -0.25 / (s * val(x)));
}
template <class T> __device__ inline T jlog1p(const T& x) {
    const double u = 1.0 / (1.0 + val(x));
    return chain(x, log1p(val(x)), u, -u * u);
}
template <class T> __device__ inline T jatan(const T& x) {
    const double u = 1.0 / (1.0 + val(x) * val(x));
    return chain(x, atan(val(x)), u, -2.0 * val(x) * u * u);
}
template <class T> __device__ inline T jasin(const T& x) {
    const double q = 1.0 / (1.0 - val(x) * val(x));
    const double s = sqrt(q);
    return chain(x, asin(val(x)), s, val(x) * q * s);
}
template <class T> __device__ inline T jexp(const T& x) {
    const double e = exp(val(x));
    return chain(x, e, e, e);
}

// --------------------------------------------------------- host potential ---
template <class T>
struct PotT {
    double G;
    T m_nfw, rs, m_mn, a, b;
};

// a = -grad Phi of the NFW halo (scale mass) and the Miyamoto-Nagai disk.
template <class T>
__device__ inline void ext_acc(const PotT<T>& p, const T& x, const T& y, const T& z, T& ax,
                               T& ay, T& az) {
    const T r2 = x * x + y * y + z * z;
    ax = cst<T>(0.0); ay = cst<T>(0.0); az = cst<T>(0.0);
    if (val(r2) != 0.0) {
        const T r = jsqrt(r2);
        const T q = r / p.rs;
        T mu;
        if (val(q) < 1e-4)
            mu = q * q * (cst<T>(0.5) + q * (cst<T>(-2.0 / 3.0) + q * (cst<T>(0.75) - 0.8 * q)));
        else
            mu = jlog1p(q) - q / (q + 1.0);
        const T g = p.G * (p.m_nfw * mu / (r2 * r));
        ax = -(g * x); ay = -(g * y); az = -(g * z);
    }
    const T S = jsqrt(z * z + p.b * p.b);
    const T A = p.a + S;
    const T D2 = x * x + y * y + A * A;
    const T k = p.G * (p.m_mn / (D2 * jsqrt(D2)));
    ax = ax - k * x;
    ay = ay - k * y;
    if (val(S) != 0.0) az = az - k * z * A / S;
}

struct Frame {
    double e1[3], e2[3], n[3];
};

struct TrackModel {
    double w[6];
    double G, dt;      // step of the forward branch
    int64_t n_steps;
    double inv_sig[3];
    Frame fr;
};

// Observables of a point.
template <class T>
struct Obs {
    T u, w, phi1;          // in-plane coordinates and accumulated longitude
    T y[3];                // phi2, d, v_r
};

template <class T>
__device__ inline void observe(const Frame& f, const T (&x)[3], const T (&v)[3], Obs<T>& o) {
    o.u = f.e1[0] * x[0] + f.e1[1] * x[1] + f.e1[2] * x[2];
    o.w = f.e2[0] * x[0] + f.e2[1] * x[1] + f.e2[2] * x[2];
    const T xn = f.n[0] * x[0] + f.n[1] * x[1] + f.n[2] * x[2];
    const T d = jsqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    const T id = recip(d);
    o.y[0] = jasin(xn * id);
    o.y[1] = d;
    o.y[2] = (x[0] * v[0] + x[1] * v[1] + x[2] * v[2]) * id;
}

// One branch (sgn = +1 forward, -1 backward).  For every track point of the
// branch not yet matched, when the newest segment holds its phi1, calls
// emit(k, model values y[3]).  Returns the mask of points never reached.
template <class T, class Emit>
__device__ uint64_t run_branch(const TrackModel& m, const PotT<T>& p, double sgn,
                               const double* __restrict__ phi1_obs, int stride, int K,
                               uint64_t pending, Emit emit) {
    const double dt = sgn * m.dt, hdt = 0.5 * dt;
    T x[3] = {cst<T>(m.w[0]), cst<T>(m.w[1]), cst<T>(m.w[2])};
    T v[3] = {cst<T>(m.w[3]), cst<T>(m.w[4]), cst<T>(m.w[5])};
    T a[3];
    ext_acc(p, x[0], x[1], x[2], a[0], a[1], a[2]);
    Obs<T> prev;
    observe(m.fr, x, v, prev);
    prev.phi1 = cst<T>(0.0);
    for (int64_t s = 0; s < m.n_steps && pending; ++s) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T vh = v[c] + hdt * a[c];
            x[c] = x[c] + dt * vh;
            v[c] = vh;
        }
        ext_acc(p, x[0], x[1], x[2], a[0], a[1], a[2]);
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = v[c] + hdt * a[c];
        Obs<T> cur;
        observe(m.fr, x, v, cur);
        const T cross = prev.u * cur.w - prev.w * cur.u;
        const T dot = prev.u * cur.u + prev.w * cur.w;
        cur.phi1 = prev.phi1 + jatan(cross / dot);
        const double p0 = val(prev.phi1), p1 = val(cur.phi1);
        const double lo = fmin(p0, p1), hi = fmax(p0, p1);
        if (p0 != p1) {
            for (int k = 0; k < K; ++k) {
                const uint64_t bit = 1ull << k;
                const double t = phi1_obs[(int64_t)k * stride];
                if ((pending & bit) && lo <= t && t <= hi) {
                    pending &= ~bit;
                    const T wgt = (cst<T>(t) - prev.phi1) / (cur.phi1 - prev.phi1);
                    T y[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) y[c] = prev.y[c] + wgt * (cur.y[c] - prev.y[c]);
                    emit(k, y);
                }
            }
        }
        prev = cur;
    }
    return pending;
}

// Both branches; the masks split the track by the sign of phi1.
template <class T, class Emit>
__device__ bool run_track(const TrackModel& m, const PotT<T>& p, const double* __restrict__ phi1,
                          int stride, int K, Emit emit) {
    uint64_t fwd = 0, bwd = 0;
    for (int k = 0; k < K; ++k) {
        if (phi1[(int64_t)k * stride] >= 0.0) fwd |= 1ull << k;
        else bwd |= 1ull << k;
    }
    uint64_t left = 0;
    if (fwd) left |= run_branch(m, p, 1.0, phi1, stride, K, fwd, emit);
    if (bwd) left |= run_branch(m, p, -1.0, phi1, stride, K, bwd, emit);
    return left == 0;
}

// theta = 10^p as jets seeded on the chosen directions.
__device__ inline PotT<double> pot_of(const double* p, double G) {
    return PotT<double>{G, exp(LN10 * p[0]), exp(LN10 * p[1]), exp(LN10 * p[2]),
                        exp(LN10 * p[3]), exp(LN10 * p[4])};
}

__device__ inline PotT<J1<NPAR>> pot_of_j1(const double* p, double G) {
    J1<NPAR> t[NPAR];
#pragma unroll
    for (int i = 0; i < NPAR; ++i) {
        J1<NPAR> u = cst<J1<NPAR>>(p[i]);
        u.d[i] = 1.0;
        t[i] = jexp(LN10 * u);
    }
    return PotT<J1<NPAR>>{G, t[0], t[1], t[2], t[3], t[4]};
}

__device__ inline PotT<HD> pot_of_hd(const double* p, double G, int i, int j) {
    HD t[NPAR];
#pragma unroll
    for (int q = 0; q < NPAR; ++q) {
        HD u{p[q], q == i ? 1.0 : 0.0, q == j ? 1.0 : 0.0, 0.0};
        t[q] = jexp(LN10 * u);
    }
    return PotT<HD>{G, t[0], t[1], t[2], t[3], t[4]};
}

__device__ inline int tri(int i, int j) {   // i <= j
    return i * NPAR - i * (i - 1) / 2 + (j - i);
}

// ------------------------------------------------------------------ kernels --
// Model observables at the longitudes phi1 [K] for one parameter vector.
__global__ __launch_bounds__(64) void k_track_observe(TrackModel m, const double* __restrict__ p,
                                const double* __restrict__ phi1, int K, double* __restrict__ y) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    for (int k = 0; k < K; ++k) y[3 * k] = y[3 * k + 1] = y[3 * k + 2] = INFINITY;
    const PotT<double> pot = pot_of(p, m.G);
    run_track(m, pot, phi1, 1, K, [&](int k, const double (&v)[3]) {
        y[3 * k] = v[0]; y[3 * k + 1] = v[1]; y[3 * k + 2] = v[2];
    });
}

// chi2, J^T r and J^T J (packed) at p[b * p_stride] for every start b.
__global__ __launch_bounds__(64) void k_track_eval(TrackModel m, const double* __restrict__ trk, int K, int batch,
                             const double* __restrict__ p, int p_stride,
                             double* __restrict__ chi2, double* __restrict__ jtr,
                             double* __restrict__ jtj) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    const PotT<J1<NPAR>> pot = pot_of_j1(p + (int64_t)b * p_stride, m.G);
    double c2 = 0.0, g[NPAR] = {0, 0, 0, 0, 0}, h[NTRI];
#pragma unroll
    for (int q = 0; q < NTRI; ++q) h[q] = 0.0;
    const bool ok = run_track(m, pot, trk, 4, K, [&](int k, const J1<NPAR> (&y)[3]) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const J1<NPAR> r = m.inv_sig[c] * (y[c] + (-trk[4 * k + 1 + c]));
            c2 += r.v * r.v;
#pragma unroll
            for (int i = 0; i < NPAR; ++i) {
                g[i] += r.d[i] * r.v;
#pragma unroll
                for (int j = i; j < NPAR; ++j) h[tri(i, j)] += r.d[i] * r.d[j];
            }
        }
    });
    chi2[b] = ok ? c2 : INFINITY;
    if (jtr)
        for (int i = 0; i < NPAR; ++i) jtr[NPAR * b + i] = g[i];
    if (jtj)
        for (int q = 0; q < NTRI; ++q) jtj[NTRI * b + q] = h[q];
}

// d2 chi2 / dp_i dp_j: lane (b, q) handles the pair q of the upper triangle.
__global__ __launch_bounds__(64) void k_track_hessian(TrackModel m, const double* __restrict__ trk, int K, int batch,
                                const double* __restrict__ p, double* __restrict__ hess) {
    const int lane = blockIdx.x * blockDim.x + threadIdx.x;
    if (lane >= batch * NTRI) return;
    const int b = lane / NTRI, q = lane % NTRI;
    int i = 0, j = 0;
    for (int ii = 0, t = 0; ii < NPAR; ++ii)
        for (int jj = ii; jj < NPAR; ++jj, ++t)
            if (t == q) { i = ii; j = jj; }
    const PotT<HD> pot = pot_of_hd(p + (int64_t)NPAR * b, m.G, i, j);
    HD c2{0.0, 0.0, 0.0, 0.0};
    const bool ok = run_track(m, pot, trk, 4, K, [&](int k, const HD (&y)[3]) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const HD r = m.inv_sig[c] * (y[c] + (-trk[4 * k + 1 + c]));
            c2 = c2 + r * r;
        }
    });
    const double h = ok ? c2.c : NAN;
    hess[25 * b + 5 * i + j] = h;
    hess[25 * b + 5 * j + i] = h;
}

// Cholesky factor of the packed symmetric 5 x 5 matrix A (in place, lower
// triangle in L[i][j], j <= i).  False if A is not positive definite.
__device__ inline bool chol5(double (&L)[NPAR][NPAR]) {
    for (int j = 0; j < NPAR; ++j) {
        double s = L[j][j];
        for (int k = 0; k < j; ++k) s -= L[j][k] * L[j][k];
        if (!(s > 0.0)) return false;
        L[j][j] = sqrt(s);
        for (int i = j + 1; i < NPAR; ++i) {
            double t = L[i][j];
            for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
            L[i][j] = t / L[j][j];
        }
    }
    return true;
}

__device__ inline void chol5_solve(const double (&L)[NPAR][NPAR], double (&x)[NPAR]) {
    for (int i = 0; i < NPAR; ++i) {
        double t = x[i];
        for (int k = 0; k < i; ++k) t -= L[i][k] * x[k];
        x[i] = t / L[i][i];
    }
    for (int i = NPAR - 1; i >= 0; --i) {
        double t = x[i];
        for (int k = i + 1; k < NPAR; ++k) t -= L[k][i] * x[k];
        x[i] = t / L[i][i];
    }
}

// Fisher matrix F = H / 2 and covariance C = F^-1 (NaN if F is not positive definite).
__global__ void k_fisher_cov(int batch, const double* __restrict__ hess, double* __restrict__ cov) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    double L[NPAR][NPAR];
    for (int i = 0; i < NPAR; ++i)
        for (int j = 0; j < NPAR; ++j) L[i][j] = 0.5 * hess[25 * b + 5 * i + j];
    const bool ok = chol5(L);
    for (int j = 0; j < NPAR; ++j) {
        double e[NPAR] = {0, 0, 0, 0, 0};
        e[j] = 1.0;
        if (ok) chol5_solve(L, e);
        for (int i = 0; i < NPAR; ++i) cov[25 * b + 5 * i + j] = ok ? e[i] : NAN;
    }
}

// Levenberg-Marquardt state of one start.
struct LmState {
    double p[NPAR], pt[NPAR];   // current point, trial point
    double c, lam;              // chi2 at p, damping
    double g[NPAR];             // J^T r at p
    double h[NTRI];             // J^T J at p (packed)
};

// Trial point p - (J^T J + lam diag(J^T J))^-1 J^T r; the current point itself
// if the damped matrix is not positive definite (the step is then rejected).
__device__ inline void lm_trial(LmState& s) {
    double L[NPAR][NPAR];
    for (int i = 0; i < NPAR; ++i)
        for (int j = 0; j <= i; ++j) {
            const double a = s.h[tri(j, i)];
            L[i][j] = (i == j) ? a + s.lam * a : a;
        }
    double x[NPAR];
    for (int i = 0; i < NPAR; ++i) x[i] = -s.g[i];
    const bool ok = isfinite(s.c) && chol5(L);
    if (ok) chol5_solve(L, x);
    for (int i = 0; i < NPAR; ++i) s.pt[i] = ok ? s.p[i] + x[i] : s.p[i];
}

__global__ void k_lm_init(int batch, const double* __restrict__ p0, double lam0,
                          const double* __restrict__ c, const double* __restrict__ g,
                          const double* __restrict__ h, LmState* __restrict__ st) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    LmState s;
    for (int i = 0; i < NPAR; ++i) { s.p[i] = p0[NPAR * b + i]; s.g[i] = g[NPAR * b + i]; }
    for (int q = 0; q < NTRI; ++q) s.h[q] = h[NTRI * b + q];
    s.c = c[b];
    s.lam = lam0;
    lm_trial(s);
    st[b] = s;
}

// Accept the evaluated trial if chi2 decreased (lam / 10), else reject (lam x 10);
// then form the next trial.
__global__ void k_lm_update(int batch, const double* __restrict__ c, const double* __restrict__ g,
                            const double* __restrict__ h, LmState* __restrict__ st) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    LmState s = st[b];
    if (c[b] < s.c) {
        for (int i = 0; i < NPAR; ++i) { s.p[i] = s.pt[i]; s.g[i] = g[NPAR * b + i]; }
        for (int q = 0; q < NTRI; ++q) s.h[q] = h[NTRI * b + q];
        s.c = c[b];
        s.lam = fmax(s.lam / 10.0, 1e-12);
    } else {
        s.lam = fmin(s.lam * 10.0, 1e16);
    }
    lm_trial(s);
    st[b] = s;
}

__global__ void k_lm_final(int batch, const LmState* __restrict__ st, double* __restrict__ p,
                           double* __restrict__ chi2) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    for (int i = 0; i < NPAR; ++i) p[NPAR * b + i] = st[b].p[i];
    chi2[b] = st[b].c;
}

// ----------------------------------------------------------------- launchers --
static TrackModel track_model(const dnb_track_model& d) {
    TrackModel m;
    for (int i = 0; i < 6; ++i) m.w[i] = d.w_now[i];
    m.G = d.G;
    m.n_steps = d.n_steps;
    m.dt = d.dt_total / (double)d.n_steps;
    for (int c = 0; c < 3; ++c) m.inv_sig[c] = 1.0 / d.sigma[c];
    const double* x = d.w_now;
    const double* v = d.w_now + 3;
    double n[3] = {x[1] * v[2] - x[2] * v[1], x[2] * v[0] - x[0] * v[2], x[0] * v[1] - x[1] * v[0]};
    const double nn = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    const double xx = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    for (int c = 0; c < 3; ++c) { m.fr.n[c] = n[c] / nn; m.fr.e1[c] = x[c] / xx; }
    const double* a = m.fr.n;
    const double* e = m.fr.e1;
    m.fr.e2[0] = a[1] * e[2] - a[2] * e[1];
    m.fr.e2[1] = a[2] * e[0] - a[0] * e[2];
    m.fr.e2[2] = a[0] * e[1] - a[1] * e[0];
    return m;
}

hipError_t launch_track_observe(const dnb_track_model& md, int K, const double* phi1,
                                const double* p, double* y, hipStream_t st) {
    const TrackModel m = track_model(md);
    hipLaunchKernelGGL(k_track_observe, dim3(1), dim3(64), 0, st, m, p, phi1, K, y);
    return hipGetLastError();
}

hipError_t launch_track_eval(const dnb_track_model& md, const double* trk, int K, int batch,
                             const double* p, double* chi2, double* jtr, double* jtj,
                             hipStream_t st) {
    const TrackModel m = track_model(md);
    hipLaunchKernelGGL(k_track_eval, dim3((unsigned)cdiv(batch, 64)), dim3(64), 0, st, m, trk, K,
                       batch, p, NPAR, chi2, jtr, jtj);
    return hipGetLastError();
}

hipError_t launch_track_hessian(const dnb_track_model& md, const double* trk, int K, int batch,
                                const double* p, double* hess, double* cov, hipStream_t st) {
    const TrackModel m = track_model(md);
    hipLaunchKernelGGL(k_track_hessian, dim3((unsigned)cdiv((int64_t)batch * NTRI, 64)), dim3(64),
                       0, st, m, trk, K, batch, p, hess);
    if (cov)
        hipLaunchKernelGGL(k_fisher_cov, dim3((unsigned)cdiv(batch, 64)), dim3(64), 0, st, batch,
                           hess, cov);
    return hipGetLastError();
}

// Workspace: [batch] LmState, then chi2 [batch], J^T r [batch][5], J^T J [batch][15].
size_t lm_workspace_bytes(int64_t batch) {
    return (size_t)batch * (sizeof(LmState) + sizeof(double) * (1 + NPAR + NTRI));
}

hipError_t launch_track_lm(const dnb_track_model& md, const double* trk, int K, int batch,
                           double* p, int64_t n_iter, double lam0, double* chi2, void* work,
                           hipStream_t st) {
    const TrackModel m = track_model(md);
    LmState* s = (LmState*)work;
    double* c = (double*)(s + batch);
    double* g = c + batch;
    double* h = g + (int64_t)NPAR * batch;
    const dim3 grid((unsigned)cdiv(batch, 64)), blk(64);
    const int stride = (int)(sizeof(LmState) / sizeof(double));
    hipLaunchKernelGGL(k_track_eval, grid, blk, 0, st, m, trk, K, batch, (const double*)p, NPAR, c,
                       g, h);
    hipLaunchKernelGGL(k_lm_init, grid, blk, 0, st, batch, (const double*)p, lam0, c, g, h, s);
    const double* pt = (const double*)s + offsetof(LmState, pt) / sizeof(double);
    for (int64_t it = 0; it < n_iter; ++it) {
        hipLaunchKernelGGL(k_track_eval, grid, blk, 0, st, m, trk, K, batch, pt, stride, c, g, h);
        hipLaunchKernelGGL(k_lm_update, grid, blk, 0, st, batch, c, g, h, s);
    }
    hipLaunchKernelGGL(k_lm_final, grid, blk, 0, st, batch, s, p, chi2);
    return hipGetLastError();
}

}  // namespace dnb
