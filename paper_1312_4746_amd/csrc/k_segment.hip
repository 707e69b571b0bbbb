// Segmentation by convex relaxation on gfx950 (Sec. 3.2 energy, Sec. 4 convex
// relaxation and primal-dual iteration).
//
// Variables (label-major planes of N = H W values each, so that a thread per
// pixel reads every plane coalesced): the relaxed indicator functions u_i and
// their over-relaxed copy u_bar_i, the dual fields xi_i = (xi_x, xi_y), for a
// positive label cost the multipliers mu_i <= 0 and the label variables m_i,
// and the data term f_i = -l_i.  One launch is one iteration of the scheme:
//
//   xi^{t+1}  = P_Kg (xi^t + sigma_xi grad u_bar^t),   |xi(x)| <= lambda g(x) / 2
//   mu^{t+1}  = min(0, mu^t + sigma_mu (m_bar^t - u_bar^t))
//   m^{t+1}   = clamp(m^t - tau_m (nu + sum_x mu^{t+1}), 0, 1)
//   u^{t+1}   = P_simplex (u^t - tau_u (-div xi^{t+1} + f - mu^{t+1}))
//   u_bar^{t+1} = 2 u^{t+1} - u^t,   m_bar^{t+1} = 2 m^{t+1} - m^t
//
// with forward differences (zero across the last column and row) and the
// divergence as minus their adjoint.  div xi^{t+1} at x needs xi^{t+1} at x,
// x - 1 and x - W: each thread computes the new dual vectors of its left and
// upper neighbours again from the old ones (the same arithmetic as their own
// threads, so the same values) instead of waiting for them, which keeps an
// iteration to one launch with ping-pong buffers.  The pixel's L candidate
// values stay in registers for the simplex projection (Michelot's finite
// algorithm).  The m update needs sum_x mu^{t+1} over the whole image: the
// launch adds it up (one FP64 atomic per label and workgroup) and the next
// launch applies it.
//
// The arithmetic follows the oracle's order with no contraction of products
// into fused multiply-adds, so the FP64 instantiation matches it to rounding
// of the few reductions; the FP32 one is the production form.
//
// Workgroups are laid out per XCD (workgroup w runs on XCD w mod 8): XCD x
// takes a contiguous band of the image, so the rows above and below a
// workgroup's pixels are mostly in the same L2.
#include "cs_internal.h"
#include "../../include/cosparse.h"

namespace cs {

namespace {

constexpr int kXcds = 8;

// Logical block of workgroup b (a bijection of 0..nb-1): XCD x = b mod 8 takes
// the contiguous band of q + 1 blocks (x < nb mod 8) or q blocks (the others),
// q = floor(nb / 8), in order.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
    const int64_t q = nb / kXcds, rmd = nb % kXcds;
    const int64_t x = b % kXcds, i = b / kXcds;
    return x < rmd ? x * (q + 1) + i : rmd * (q + 1) + (x - rmd) * q + i;
}

template <typename T>
__device__ __forceinline__ void project_disc(T &qx, T &qy, T radius) {
#pragma clang fp contract(off)
    const T n = sqrt(qx * qx + qy * qy);
    if (n > radius) {
        const T s = radius / n;
        qx = qx * s;
        qy = qy * s;
    }
}

template <typename T>
__device__ __forceinline__ T block_sum(T v, T *red) {
    // fixed order: butterfly in each wave, then the four wave sums in order
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    return ((red[0] + red[1]) + red[2]) + red[3];
}

}  // namespace

// ---- edge metric g (Sec. 3.2) ----
// |grad I(x)| (FP64, forward differences over the three colour planes, zero
// across the last column and row) and a per-workgroup partial sum.
__global__ __launch_bounds__(256) void k_grad_mag(const float *rgb, int H, int W, double *mag, double *part) {
#pragma clang fp contract(off)
    __shared__ double red[4];
    const int64_t N = (int64_t)H * W;
    const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double m = 0.0;
    if (x < N) {
        const int c = (int)(x % W), r = (int)(x / W);
        double s = 0.0;
        for (int ch = 0; ch < 3; ++ch) {
            const float *P = rgb + (int64_t)ch * N;
            const double v = (double)P[x];
            const double dx = c < W - 1 ? (double)P[x + 1] - v : 0.0;
            const double dy = r < H - 1 ? (double)P[x + W] - v : 0.0;
            s = s + (dx * dx + dy * dy);
        }
        m = sqrt(s);
        mag[x] = m;
    }
    const double t = block_sum(m, red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// g(x) = exp(-|grad I| / gamma) / (2 gamma); gamma <= 0 selects the mean of
// |grad I| (every workgroup adds the partial sums in the same order).
template <typename T>
__global__ __launch_bounds__(256) void k_edge_weight(const double *mag, int64_t N, const double *part, int nparts,
                                                     double gamma, T *g, float *g32, double *gamma_out) {
#pragma clang fp contract(off)
    __shared__ double s_gamma;
    if (threadIdx.x == 0) {
        double gm = gamma;
        if (!(gm > 0.0)) {
            double s = 0.0;
            for (int i = 0; i < nparts; ++i) s = s + part[i];
            gm = s / (double)N;
        }
        s_gamma = gm;
        if (blockIdx.x == 0 && gamma_out) *gamma_out = gm;
    }
    __syncthreads();
    const double gm = s_gamma;
    const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (x >= N) return;
    const double v = exp(-mag[x] / gm) / (2.0 * gm);
    if (g) g[x] = (T)v;
    if (g32) g32[x] = (float)v;
}

// ---- initial state and the data term ----
template <typename T>
__global__ __launch_bounds__(256) void k_pd_init(PdArgs a, const float *loglik) {
    const int64_t N = a.N;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < (int64_t)a.L * N) {
        const int l = (int)(t / N);
        const int64_t x = t - (int64_t)l * N;
        T *f = (T *)a.f, *u = (T *)a.u[0], *ub = (T *)a.ub[0];
        T *px = (T *)a.px[0], *py = (T *)a.py[0];
        f[t] = -(T)loglik[x * a.L + l];
        const T u0 = (T)1 / (T)a.L;
        u[t] = u0;
        ub[t] = u0;
        px[t] = (T)0;
        py[t] = (T)0;
        if (a.mdl) ((T *)a.mu[0])[t] = (T)0;
    }
    if (t < (int64_t)a.L) {
        a.mval[t] = 1.0;  // m^0 = 1 (every label present)
    }
    if (a.mdl && t < (int64_t)(a.iters + 1) * a.L) a.msum[t] = 0.0;
}

// Per-label part of an iteration at pixel x: the new dual vector xi^{t+1}(x)
// (qx, qy), the new multiplier (mu_n, label cost only) and the candidate
// u^t - tau_u (-div xi^{t+1} + f - mu^{t+1}).  Reads only the current buffers.
template <typename T>
__device__ __forceinline__ T pd_label(const T *ub, const T *px, const T *py, const T *U, const T *F, const T *MU,
                                      int64_t x, int c, int r, int H, int W, T s_xi, T s_mu, T t_u, T mb, T rad,
                                      T rad_l, T rad_u, bool mdl, T &qx, T &qy, T &mu_n) {
#pragma clang fp contract(off)
    // every operand of the label loaded up front, the indices clamped into the
    // plane, so that the loads are in flight together (one memory round trip
    // per label); values of neighbours outside the image are not used
    const int64_t last = (int64_t)H * W - 1;
    auto at = [&](int64_t i) { return i < 0 ? (int64_t)0 : (i > last ? last : i); };
    const T ubc = ub[x], ubr = ub[at(x + 1)], ubd = ub[at(x + W)];
    const T ubl = ub[at(x - 1)], ubld = ub[at(x - 1 + W)];
    const T ubu = ub[at(x - W)], ubur = ub[at(x - W + 1)];
    const T pxc = px[x], pxl = px[at(x - 1)], pxu = px[at(x - W)];
    const T pyc = py[x], pyl = py[at(x - 1)], pyu = py[at(x - W)];
    const T uc = U[x], fc = F[x];
    const T muc = mdl ? MU[x] : (T)0;
    qx = pxc + s_xi * (c < W - 1 ? ubr - ubc : (T)0);
    qy = pyc + s_xi * (r < H - 1 ? ubd - ubc : (T)0);
    project_disc(qx, qy, rad);
    // xi^{t+1}_x(x - 1) and xi^{t+1}_y(x - W), as their own threads compute them
    T lx = 0, uy = 0;
    if (c > 0) {
        T ax = pxl + s_xi * (ubc - ubl);
        T ay = pyl + s_xi * (r < H - 1 ? ubld - ubl : (T)0);
        project_disc(ax, ay, rad_l);
        lx = ax;
    }
    if (r > 0) {
        T bx = pxu + s_xi * (c < W - 1 ? ubur - ubu : (T)0);
        T by = pyu + s_xi * (ubc - ubu);
        project_disc(bx, by, rad_u);
        uy = by;
    }
    // div xi^{t+1}(x) = xi_x(x) - xi_x(x - 1) + xi_y(x) - xi_y(x - W)
    T d = c < W - 1 ? qx : (T)0;
    d = d - lx;
    if (r < H - 1) d = d + qy;
    d = d - uy;
    T step = -d + fc;
    if (mdl) {
        mu_n = muc + s_mu * (mb - ubc);
        mu_n = mu_n < (T)0 ? mu_n : (T)0;
        step = step - mu_n;
    }
    return uc - t_u * step;
}

// Michelot's projection of v[0..L) onto the simplex: project onto the
// hyperplane sum = 1 of the coordinates in play, drop those below 0, repeat.
// Returns theta; coordinate l is v[l] - theta if bit l of *act is set, else 0.
template <typename T, int LMAX>
__device__ __forceinline__ T simplex_theta(const T (&v)[LMAX], int L, uint64_t *act_out) {
#pragma clang fp contract(off)
    uint64_t act = L >= 64 ? ~0ull : ((1ull << L) - 1ull);
    T theta = 0;
    for (;;) {
        T s = 0;
        int cnt = 0;
#pragma unroll
        for (int l = 0; l < LMAX; ++l)
            if (l < L) {
                const bool on = (act >> l) & 1ull;
                s = s + (on ? v[l] : (T)0);
                cnt += on;
            }
        theta = (s - (T)1) / (T)cnt;
        uint64_t drop = 0;
#pragma unroll
        for (int l = 0; l < LMAX; ++l)
            if (l < L && ((act >> l) & 1ull) && v[l] - theta < (T)0) drop |= 1ull << l;
        if (!drop) break;
        act &= ~drop;
    }
    *act_out = act;
    return theta;
}

// The same projection with the candidates in memory (v[l * stride], the
// thread's own stores): for label counts whose candidates do not fit in
// registers.
template <typename T>
__device__ __forceinline__ T simplex_theta_mem(const T *v, int64_t stride, int L, uint64_t *act_out) {
#pragma clang fp contract(off)
    uint64_t act = L >= 64 ? ~0ull : ((1ull << L) - 1ull);
    T theta = 0;
    for (;;) {
        T s = 0;
        int cnt = 0;
        for (int l = 0; l < L; ++l) {
            const bool on = (act >> l) & 1ull;
            s = s + (on ? v[l * stride] : (T)0);
            cnt += on;
        }
        theta = (s - (T)1) / (T)cnt;
        uint64_t drop = 0;
        for (int l = 0; l < L; ++l)
            if (((act >> l) & 1ull) && v[l * stride] - theta < (T)0) drop |= 1ull << l;
        if (!drop) break;
        act &= ~drop;
    }
    *act_out = act;
    return theta;
}

// One iteration t (buffers: cur = t & 1, next = cur ^ 1), label by label.  Up
// to 16 labels the candidates stay in registers for the projection; more
// (LMAX = 64) are parked in the next u plane, which the thread overwrites
// after the projection.  (Holding every label's dual vectors in registers
// until one store phase, for more loads in flight, measured slower: the
// registers halve the waves per SIMD.)
template <typename T, int LMAX, bool MDL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 8 : 4)))
void k_pd_iter(PdArgs a, int t) {
#pragma clang fp contract(off)
    constexpr bool kHold = LMAX <= 16;
    __shared__ T red[4];
    __shared__ double s_mb[LMAX];
    const int cur = t & 1, nxt = cur ^ 1;
    const int L = a.L, H = a.H, W = a.W;
    const int64_t N = a.N;
    const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
    const int64_t x = lb * 256 + threadIdx.x;
    const bool in = x < N;
    const int c = in ? (int)(x % W) : 0, r = in ? (int)(x / W) : 0;
    const T s_xi = (T)a.sigma_xi, s_mu = (T)a.sigma_mu, t_u = (T)a.tau_u;
    const T half_lam = (T)(0.5 * a.lambda);
    if (MDL) {
        // m^t and m_bar^t (kernel t = 0: m^0 = m_bar^0 = 1); workgroup 0 keeps m^t
        for (int l = threadIdx.x; l < L; l += 256) {
            double m, mprev;
            if (t == 0) {
                m = mprev = a.mval[l];
            } else {
                mprev = a.mval[(int64_t)(t - 1) * L + l];
                m = mprev - a.tau_m * (a.nu + a.msum[(int64_t)t * L + l]);
                m = m < 0.0 ? 0.0 : (m > 1.0 ? 1.0 : m);
                if (blockIdx.x == 0) a.mval[(int64_t)t * L + l] = m;
            }
            s_mb[l] = t == 0 ? m : 2.0 * m - mprev;
        }
        __syncthreads();
    }
    const T *U = (const T *)a.u[cur];
    const T *UB = (const T *)a.ub[cur];
    const T *PX = (const T *)a.px[cur];
    const T *PY = (const T *)a.py[cur];
    const T *F = (const T *)a.f;
    const T *G = (const T *)a.g;
    const T *MU = MDL ? (const T *)a.mu[cur] : nullptr;
    T *Un = (T *)a.u[nxt];
    T *UBn = (T *)a.ub[nxt];
    T *PXn = (T *)a.px[nxt];
    T *PYn = (T *)a.py[nxt];
    T *MUn = MDL ? (T *)a.mu[nxt] : nullptr;
    T rad = 0, rad_l = 0, rad_u = 0;
    if (in) {
        rad = half_lam * G[x];
        if (c > 0) rad_l = half_lam * G[x - 1];
        if (r > 0) rad_u = half_lam * G[x - W];
    }
    if constexpr (kHold) {
        T v[LMAX];
#pragma unroll
        for (int l = 0; l < LMAX; ++l) {
            v[l] = (T)0;
            if (l >= L) continue;
            T qx = 0, qy = 0, mu_n = 0;
            const int64_t o = (int64_t)l * N;
            if (in) {
                v[l] = pd_label(UB + o, PX + o, PY + o, U + o, F + o, MDL ? MU + o : nullptr, x, c, r, H, W, s_xi,
                                s_mu, t_u, MDL ? (T)s_mb[l] : (T)0, rad, rad_l, rad_u, MDL, qx, qy, mu_n);
                PXn[o + x] = qx;
                PYn[o + x] = qy;
                if constexpr (MDL) MUn[o + x] = mu_n;
            }
            if constexpr (MDL) {
                const T s = block_sum(mu_n, red);
                if (threadIdx.x == 0) atomicAdd(a.msum + (int64_t)(t + 1) * L + l, (double)s);
            }
        }
        if (!in) return;
        uint64_t act;
        const T theta = simplex_theta<T, LMAX>(v, L, &act);
        // u^t of every label loaded before any store (the loads in flight
        // together)
        T uo[LMAX];
#pragma unroll
        for (int l = 0; l < LMAX; ++l) uo[l] = l < L ? U[(int64_t)l * N + x] : (T)0;
        // the new values first, then every store (no wait between stores)
        T ubn[LMAX];
#pragma unroll
        for (int l = 0; l < LMAX; ++l) {
            v[l] = ((act >> l) & 1ull) ? v[l] - theta : (T)0;
            ubn[l] = (T)2 * v[l] - uo[l];
            // formed here, ahead of the stores (not sunk into the stores'
            // per-label branches, where each would wait for earlier stores)
            __asm__ volatile("" : "+v"(v[l]), "+v"(ubn[l]));
        }
#pragma unroll
        for (int l = 0; l < LMAX; ++l) {
            if (l >= L) continue;
            const int64_t o = (int64_t)l * N + x;
            UBn[o] = ubn[l];
            Un[o] = v[l];
        }
    } else {
        for (int l = 0; l < L; ++l) {
            T qx = 0, qy = 0, mu_n = 0;
            const int64_t o = (int64_t)l * N;
            if (in) {
                Un[o + x] = pd_label(UB + o, PX + o, PY + o, U + o, F + o, MDL ? MU + o : nullptr, x, c, r, H, W, s_xi,
                                     s_mu, t_u, MDL ? (T)s_mb[l] : (T)0, rad, rad_l, rad_u, MDL, qx, qy, mu_n);
                PXn[o + x] = qx;
                PYn[o + x] = qy;
                if (MDL) MUn[o + x] = mu_n;
            }
            if (MDL) {
                const T s = block_sum(mu_n, red);
                if (threadIdx.x == 0) atomicAdd(a.msum + (int64_t)(t + 1) * L + l, (double)s);
            }
        }
        if (!in) return;
        uint64_t act;
        const T theta = simplex_theta_mem<T>(Un + x, N, L, &act);
        for (int l = 0; l < L; ++l) {
            const int64_t o = (int64_t)l * N + x;
            const T un = ((act >> l) & 1ull) ? Un[o] - theta : (T)0;
            UBn[o] = (T)2 * un - U[o];
            Un[o] = un;
        }
    }
}

// The same iteration in two launches, for images too small to fill the chip
// with one thread per pixel: one thread per (pixel, label) forms the new dual
// vector (and multiplier) and the candidate, parked in the next u plane; then
// one thread per pixel projects its candidates onto the simplex.  The
// arithmetic is that of k_pd_iter element for element.
template <typename T, bool MDL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 8 : 4)))
void k_pd_dual(PdArgs a, int t, int nb) {
#pragma clang fp contract(off)
    __shared__ T red[4];
    __shared__ double s_mb;
    const int cur = t & 1, nxt = cur ^ 1;
    const int L = a.L, H = a.H, W = a.W;
    const int64_t N = a.N;
    // workgroup -> (label, pixel block): an XCD takes consecutive pixel blocks
    // of one label
    const int64_t lin = xcd_block(blockIdx.x, gridDim.x);
    const int l = (int)(lin / nb);
    const int64_t pb = lin - (int64_t)l * nb;
    const int64_t x = pb * 256 + threadIdx.x;
    const bool in = x < N;
    const int c = in ? (int)(x % W) : 0, r = in ? (int)(x / W) : 0;
    const T s_xi = (T)a.sigma_xi, s_mu = (T)a.sigma_mu, t_u = (T)a.tau_u;
    const T half_lam = (T)(0.5 * a.lambda);
    if (MDL) {
        if (threadIdx.x == 0) {
            double m, mprev;
            if (t == 0) {
                m = mprev = a.mval[l];
            } else {
                mprev = a.mval[(int64_t)(t - 1) * L + l];
                m = mprev - a.tau_m * (a.nu + a.msum[(int64_t)t * L + l]);
                m = m < 0.0 ? 0.0 : (m > 1.0 ? 1.0 : m);
                if (pb == 0) a.mval[(int64_t)t * L + l] = m;
            }
            s_mb = t == 0 ? m : 2.0 * m - mprev;
        }
        __syncthreads();
    }
    const int64_t o = (int64_t)l * N;
    const T *G = (const T *)a.g;
    T qx = 0, qy = 0, mu_n = 0;
    if (in) {
        const T rad = half_lam * G[x];
        const T rad_l = c > 0 ? half_lam * G[x - 1] : (T)0;
        const T rad_u = r > 0 ? half_lam * G[x - W] : (T)0;
        const T v = pd_label((const T *)a.ub[cur] + o, (const T *)a.px[cur] + o, (const T *)a.py[cur] + o,
                             (const T *)a.u[cur] + o, (const T *)a.f + o, MDL ? (const T *)a.mu[cur] + o : nullptr,
                             x, c, r, H, W, s_xi, s_mu, t_u, MDL ? (T)s_mb : (T)0, rad, rad_l, rad_u, MDL, qx, qy,
                             mu_n);
        ((T *)a.px[nxt])[o + x] = qx;
        ((T *)a.py[nxt])[o + x] = qy;
        if constexpr (MDL) ((T *)a.mu[nxt])[o + x] = mu_n;
        ((T *)a.u[nxt])[o + x] = v;  // the candidate, projected by k_pd_primal
    }
    if constexpr (MDL) {
        const T sm = block_sum(mu_n, red);
        if (threadIdx.x == 0) atomicAdd(a.msum + (int64_t)(t + 1) * L + l, (double)sm);
    }
}

template <typename T, int LMAX>
__global__ __launch_bounds__(256) void k_pd_primal(PdArgs a, int t) {
#pragma clang fp contract(off)
    const int cur = t & 1, nxt = cur ^ 1;
    const int L = a.L;
    const int64_t N = a.N;
    const int64_t x = xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    if (x >= N) return;
    const T *U = (const T *)a.u[cur];
    T *Un = (T *)a.u[nxt];
    T *UBn = (T *)a.ub[nxt];
    uint64_t act;
    if constexpr (LMAX <= 16) {
        // the candidates and u^t loaded together, the new values formed
        // before any store (as in k_pd_iter)
        T v[LMAX], uo[LMAX];
#pragma unroll
        for (int l = 0; l < LMAX; ++l) {
            v[l] = l < L ? Un[(int64_t)l * N + x] : (T)0;
            uo[l] = l < L ? U[(int64_t)l * N + x] : (T)0;
        }
        const T theta = simplex_theta<T, LMAX>(v, L, &act);
        T ubn[LMAX];
#pragma unroll
        for (int l = 0; l < LMAX; ++l) {
            v[l] = ((act >> l) & 1ull) ? v[l] - theta : (T)0;
            ubn[l] = (T)2 * v[l] - uo[l];
            __asm__ volatile("" : "+v"(v[l]), "+v"(ubn[l]));
        }
#pragma unroll
        for (int l = 0; l < LMAX; ++l) {
            if (l >= L) continue;
            const int64_t o = (int64_t)l * N + x;
            UBn[o] = ubn[l];
            Un[o] = v[l];
        }
    } else {
        const T theta = simplex_theta_mem<T>(Un + x, N, L, &act);
        for (int l = 0; l < L; ++l) {
            const int64_t o = (int64_t)l * N + x;
            const T un = ((act >> l) & 1ull) ? Un[o] - theta : (T)0;
            UBn[o] = (T)2 * un - U[o];
            Un[o] = un;
        }
    }
}

// Labels l(x) = argmax_i u_i(x) (ties to the lowest label) and u pixel-major.
template <typename T>
__global__ __launch_bounds__(256) void k_pd_labels(PdArgs a, int buf, int32_t *labels, float *u_out,
                                                   unsigned long long *used) {
    const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const T *U = (const T *)a.u[buf];
    uint64_t bit = 0;
    if (x < a.N) {
        int best = 0;
        T bv = U[x];
        for (int l = 0; l < a.L; ++l) {
            const T v = U[(int64_t)l * a.N + x];
            if (u_out) u_out[x * a.L + l] = (float)v;
            if (v > bv) {
                bv = v;
                best = l;
            }
        }
        labels[x] = best;
        bit = 1ull << best;
    }
    // labels present: OR over the wave, one atomic per wave
    for (int off = 32; off >= 1; off >>= 1) bit |= __shfl_xor(bit, off);
    if ((threadIdx.x & 63) == 0 && bit) atomicOr(used, (unsigned long long)bit);
}

// Per-workgroup partial energies in FP64: [0] the relaxed primal data and
// boundary terms, [1] the binary energy without the label cost, [2] the dual
// pixel terms, then L maxima of u_i (for the label-cost term of the primal).
template <typename T>
__global__ __launch_bounds__(256) void k_pd_energy(PdArgs a, int buf, const int32_t *labels, double *part) {
#pragma clang fp contract(off)
    __shared__ double red[4];
    const int64_t N = a.N;
    const int H = a.H, W = a.W, L = a.L;
    const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool in = x < N;
    const int c = in ? (int)(x % W) : 0, r = in ? (int)(x / W) : 0;
    const T *U = (const T *)a.u[buf], *PX = (const T *)a.px[buf], *PY = (const T *)a.py[buf];
    const T *F = (const T *)a.f, *G = (const T *)a.g;
    const T *MU = a.mdl ? (const T *)a.mu[buf] : nullptr;
    double prim = 0.0, bin = 0.0, dual = 0.0;
    if (in) {
        const double hg = 0.5 * a.lambda * (double)G[x];
        const int lx = labels[x];
        const int lr = c < W - 1 ? labels[x + 1] : lx, ld = r < H - 1 ? labels[x + W] : lx;
        double dmin = 0.0;
        for (int l = 0; l < L; ++l) {
            const int64_t o = (int64_t)l * N + x;
            const double u = (double)U[o];
            const double dx = c < W - 1 ? (double)U[o + 1] - u : 0.0;
            const double dy = r < H - 1 ? (double)U[o + W] - u : 0.0;
            prim = prim + (u * (double)F[o] + hg * sqrt(dx * dx + dy * dy));
            // binary segmentation: indicator of label l at x, x + 1, x + W
            const double bx = (double)(lr == l) - (double)(lx == l), by = (double)(ld == l) - (double)(lx == l);
            bin = bin + hg * sqrt(bx * bx + by * by);
            // dual: f - div xi (- mu)
            double d = c < W - 1 ? (double)PX[o] : 0.0;
            if (c > 0) d = d - (double)PX[o - 1];
            if (r < H - 1) d = d + (double)PY[o];
            if (r > 0) d = d - (double)PY[o - W];
            double q = -d + (double)F[o];
            if (a.mdl) q = q - (double)MU[o];
            dmin = l == 0 ? q : (q < dmin ? q : dmin);
        }
        bin = bin + (double)F[(int64_t)lx * N + x];
        dual = dmin;
    }
    double t0 = block_sum(prim, red);
    double t1 = block_sum(bin, red);
    double t2 = block_sum(dual, red);
    const int64_t stride = 3 + L;
    if (threadIdx.x == 0) {
        part[blockIdx.x * stride + 0] = t0;
        part[blockIdx.x * stride + 1] = t1;
        part[blockIdx.x * stride + 2] = t2;
    }
    if (a.mdl) {
        for (int l = 0; l < L; ++l) {
            double m = in ? (double)U[(int64_t)l * N + x] : 0.0;
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off));
            __syncthreads();
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
            __syncthreads();
            if (threadIdx.x == 0)
                part[blockIdx.x * stride + 3 + l] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
        }
    }
}

// The partial energies added in workgroup order (one workgroup); for a label
// cost also m^T, the label-cost terms and sum_i min(0, nu + sum_x mu_i).
// out: {primal, binary (without the label cost), dual}
__global__ __launch_bounds__(64) void k_pd_energy_final(PdArgs a, const double *part, int nparts, double *out) {
#pragma clang fp contract(off)
    // lane i sums the parts of its contiguous chunk in order (loads eight at a
    // time), then lane 0 adds the 64 lane sums in order: a fixed order
    __shared__ double s3[3][64];
    __shared__ double smx[64];
    const int lane = threadIdx.x;
    const int L = a.L;
    const int64_t stride = 3 + L;
    const int per = (nparts + 63) / 64, i0 = lane * per, i1 = i0 + per < nparts ? i0 + per : nparts;
    double p = 0.0, b = 0.0, d = 0.0;
    for (int i = i0; i < i1; i += 8) {
        double v[8][3];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int q = 0; q < 3; ++q) v[u][q] = i + u < i1 ? part[(int64_t)(i + u) * stride + q] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (i + u < i1) {
                p = p + v[u][0];
                b = b + v[u][1];
                d = d + v[u][2];
            }
    }
    s3[0][lane] = p;
    s3[1][lane] = b;
    s3[2][lane] = d;
    __syncthreads();
    double mdl_p = 0.0, mdl_d = 0.0;
    if (a.mdl) {
        for (int l = 0; l < L; ++l) {
            double mx = -INFINITY;
            for (int i = i0; i < i1; ++i) mx = fmax(mx, part[(int64_t)i * stride + 3 + l]);
            smx[lane] = mx;
            __syncthreads();
            if (lane == 0) {
                double m2 = smx[0];
                for (int q = 1; q < 64; ++q) m2 = fmax(m2, smx[q]);
                mdl_p = mdl_p + a.nu * m2;
                const double sl = a.nu + a.msum[(int64_t)a.iters * L + l];
                mdl_d = mdl_d + (sl < 0.0 ? sl : 0.0);
            }
            __syncthreads();
        }
    }
    if (lane == 0) {
        double pp = 0.0, bb = 0.0, dd = 0.0;
        for (int q = 0; q < 64; ++q) {
            pp = pp + s3[0][q];
            bb = bb + s3[1][q];
            dd = dd + s3[2][q];
        }
        out[0] = pp + mdl_p;
        out[1] = bb;
        out[2] = dd + mdl_d;
    }
}

// ---- launchers ----
// Two launches per iteration when one thread per pixel gives fewer waves than
// eight per SIMD of the chip.
bool pd_split(const LaunchCtx &lc, int64_t N) { return (N + 63) / 64 < (int64_t)lc.num_cu * 4 * 8; }

hipError_t launch_edge_weight(const LaunchCtx &lc, const float *rgb, int H, int W, double gamma, double *mag,
                              double *part, int precision, void *g, float *g32, double *gamma_out) {
    const int64_t N = (int64_t)H * W;
    const unsigned nb = (unsigned)((N + 255) / 256);
    hipLaunchKernelGGL(k_grad_mag, dim3(nb), dim3(256), 0, lc.stream, rgb, H, W, mag, part);
    if (precision == CS_FP64)
        hipLaunchKernelGGL(k_edge_weight<double>, dim3(nb), dim3(256), 0, lc.stream, mag, N, part, (int)nb, gamma,
                           (double *)g, g32, gamma_out);
    else
        hipLaunchKernelGGL(k_edge_weight<float>, dim3(nb), dim3(256), 0, lc.stream, mag, N, part, (int)nb, gamma,
                           (float *)g, g32, gamma_out);
    return hipGetLastError();
}

hipError_t launch_pd_init(const LaunchCtx &lc, const PdArgs &a, int precision, const float *loglik) {
    int64_t n = (int64_t)a.L * a.N;
    if (n < (int64_t)(a.iters + 1) * a.L) n = (int64_t)(a.iters + 1) * a.L;
    const dim3 grid((unsigned)((n + 255) / 256));
    if (precision == CS_FP64)
        hipLaunchKernelGGL(k_pd_init<double>, grid, dim3(256), 0, lc.stream, a, loglik);
    else
        hipLaunchKernelGGL(k_pd_init<float>, grid, dim3(256), 0, lc.stream, a, loglik);
    return hipGetLastError();
}

template <typename T>
static void pd_iter_launch(const LaunchCtx &lc, const PdArgs &a, int t) {
    const dim3 grid((unsigned)((a.N + 255) / 256));
    if (pd_split(lc, a.N)) {
        const int nb = (int)((a.N + 255) / 256);
        const dim3 g2((unsigned)((int64_t)nb * a.L));
        if (a.mdl)
            hipLaunchKernelGGL((k_pd_dual<T, true>), g2, dim3(256), 0, lc.stream, a, t, nb);
        else
            hipLaunchKernelGGL((k_pd_dual<T, false>), g2, dim3(256), 0, lc.stream, a, t, nb);
        if (a.L <= 16)
            hipLaunchKernelGGL((k_pd_primal<T, 16>), grid, dim3(256), 0, lc.stream, a, t);
        else
            hipLaunchKernelGGL((k_pd_primal<T, 64>), grid, dim3(256), 0, lc.stream, a, t);
        return;
    }
    if (a.L <= 16) {
        if (a.mdl)
            hipLaunchKernelGGL((k_pd_iter<T, 16, true>), grid, dim3(256), 0, lc.stream, a, t);
        else
            hipLaunchKernelGGL((k_pd_iter<T, 16, false>), grid, dim3(256), 0, lc.stream, a, t);
    } else {
        if (a.mdl)
            hipLaunchKernelGGL((k_pd_iter<T, 64, true>), grid, dim3(256), 0, lc.stream, a, t);
        else
            hipLaunchKernelGGL((k_pd_iter<T, 64, false>), grid, dim3(256), 0, lc.stream, a, t);
    }
}

hipError_t launch_pd_iter(const LaunchCtx &lc, const PdArgs &a, int precision, int t) {
    if (precision == CS_FP64)
        pd_iter_launch<double>(lc, a, t);
    else
        pd_iter_launch<float>(lc, a, t);
    return hipGetLastError();
}

template <typename T>
static hipError_t pd_finish(const LaunchCtx &lc, const PdArgs &a, int32_t *labels, float *u_out,
                            unsigned long long *used, double *part, double *energies) {
    const unsigned nb = (unsigned)((a.N + 255) / 256);
    const int buf = a.iters & 1;
    hipLaunchKernelGGL(k_pd_labels<T>, dim3(nb), dim3(256), 0, lc.stream, a, buf, labels, u_out, used);
    if (energies) {
        hipLaunchKernelGGL(k_pd_energy<T>, dim3(nb), dim3(256), 0, lc.stream, a, buf, labels, part);
        hipLaunchKernelGGL(k_pd_energy_final, dim3(1), dim3(64), 0, lc.stream, a, part, (int)nb, energies);
    }
    return hipGetLastError();
}

hipError_t launch_pd_finish(const LaunchCtx &lc, const PdArgs &a, int precision, int32_t *labels, float *u_out,
                            unsigned long long *used, double *part, double *energies) {
    if (precision == CS_FP64) return pd_finish<double>(lc, a, labels, u_out, used, part, energies);
    return pd_finish<float>(lc, a, labels, u_out, used, part, energies);
}

}  // namespace cs
