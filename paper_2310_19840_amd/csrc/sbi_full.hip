// sbi_full.hip -- the fully nonlinear W solve of one-dimensional grids: the
// boundary-integral equations of Sec. 2.3 with the remaining integrals I^(S)
// of App. A kept (Eq. con-V: V = sum_j V^(j) + I^(S), whose sum is the exact
// equation) and, over a variable bed, the bed's remainder I^(B) of App. B.
//
// Two-dimensional flow (one horizontal dimension): Green function -ln r with
// the image of the source in the bed z = -h, jump coefficient pi; for the
// periodic surface z = x + i eta(x), 0 <= x < L,
//
//   S[V] = pi phi_s + D[phi_s],
//   S[V](x_i) = int V(x') G dx',  D[f](x_i) = int f(x') dG/dn' sqrt(1 + eta_x'^2) dx',
//   G = -ln|2 sin(pi (z - z') / L)| - ln|2 sin(pi (z - conj(z') + 2 i h) / L)|.
//
// The solve iterates V_(n+1) = S0^-1 [pi phi_s + D[phi_s] - (S - S0)[V_n]]
// from V_0 = 0, where S0 is S on the undisturbed surface (Fourier multiplier
// (pi / |k|) (1 + exp(-2 |k| h))).  The kernels of S - S0 and D are smooth and
// periodic, so the trapezoidal rule over the grid is spectrally accurate;
// S0^-1 and the derivatives eta_x, eta_xx are circulant matrices on the grid
// (their discrete Fourier multipliers), applied by direct summation.  The work
// is O(n^2) per application: every kernel evaluates point pairs, split over
// workgroups along both the evaluation and the source points.  Deep water
// (k_1 h > 18, k_1 = 2 pi / L) drops the image terms.
//
// Over a variable bed z = b(x) = -h + delta(x) the image no longer applies; the
// bed is a boundary of its own with the potential phi_b on it (dphi/dn = 0):
//
//   S[V] = pi phi_s + D_SS[phi_s] + D_SB[phi_b]       at the surface points,
//   pi phi_b = S_BS[V] - D_BS[phi_s] - D_BB[phi_b]     at the bed points,
//
// (S, D without image; D_XY the double layer of boundary Y seen from the
// points of X, outward normals (-eta_x, 1) and (b_x, -1) times ds/dx).  A
// sweep updates phi_b from the bed equation with V_n, then
// V_(n+1) = S0^-1 [pi phi_s + D_SS[phi_s] + D_SB[phi_b] - (S - S_flat)[V_n]]
//           + S0^-1 (S0 - S_flat)[V_n],
// S0 the image form's flat operator, S_flat = pi / |k| that of the flat surface
// alone.  A bed too deep to matter (k_1 times the smallest depth beyond 18)
// keeps the image form, which then drops the image.
//
// One object per precision (SBI_REAL): fields and the pair arithmetic run in
// that type; the circulant tables, the slices of the pair sums and every
// accumulation are FP64 (the direct sums over n points would otherwise lose
// about log10(sqrt(n)) digits in FP32).
#include <hip/hip_runtime.h>
#include <math.h>

#include "sbi_device.hpp"
#include "sbi_full.hpp"
#include "sbi_kernels.hpp"

#ifndef SBI_REAL
#define SBI_REAL double
#endif

namespace sbi {

using Real = SBI_REAL;

constexpr int kFullThreads = 256;       // evaluation points per workgroup
constexpr double kDeepK1H = 18.0;       // exp(-2 k_1 h) < 1e-15 beyond this

__device__ __forceinline__ bool full_deep(const FullParams& p, int m) {
    return (2.0 * M_PI / p.lx) * p.href[m] > kDeepK1H;
}

// --- tables: S0^-1 (per member: its depth), eta_x and eta_xx circulants,
// sin^2(pi j / n), and the circulant cm of S0^-1 (S0 - S_flat) (multiplier
// exp(-2|k|h) / (1 + exp(-2|k|h))).  c[j] = (1/n) sum_m s(k_m) cos(2 pi m j / n) with
// s = |k| / (pi (1 + exp(-2 |k| h))), k_m the m-th discrete wavenumber (the
// Nyquist mode included); d1[j] = (1/n) sum_(0<m<n/2) (-2 k_m) sin(2 pi m j / n)
// (the Nyquist mode drops out of a first derivative of a real field);
// d2[j] = (1/n) sum_m (-k_m^2) cos(2 pi m j / n).
template <typename R>
__global__ void __launch_bounds__(kFullThreads) k_full_tables(const FullParams p) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.y;
    const int n = p.n;
    if (j >= n) return;
    const double dk = 2.0 * M_PI / p.lx;
    const bool deep = full_deep(p, m);
    const double h = p.href[m];
    double c = 0.0, cm = 0.0, d1 = 0.0, d2 = 0.0;
    for (int q = 1; q < n; ++q) {
        const int qq = q <= n / 2 ? q : n - q;
        const double k = dk * qq;
        // angle 2 pi q j / n reduced exactly in integers
        const long long r = ((long long)q * j) % n;
        const double cs = cospi(2.0 * (double)r / n);
        const double e2 = deep ? 0.0 : exp(-2.0 * k * h);
        const double s = k / (M_PI * (1.0 + e2));
        c += s * cs;
        cm += e2 / (1.0 + e2) * cs;  // S0^-1 (S0 - S_flat): exp(-2|k|h) / (1 + exp(-2|k|h))
        if (m == 0) {
            d2 -= k * k * cs;
            if (q < n / 2) d1 -= 2.0 * k * sinpi(2.0 * (double)r / n);
        }
    }
    static_cast<double*>(p.c0)[(long long)m * n + j] = c / n;
    if (p.cm) static_cast<double*>(p.cm)[(long long)m * n + j] = cm / n;
    {
        // the flat image's single-layer term 1/2 ln(sin^2(pi j / n) + sinh^2(2 pi h / L)) of this member
        const double sn = sinpi((double)j / n), sh = deep ? 0.0 : sinh(2.0 * M_PI * h / p.lx);
        static_cast<double*>(p.lfl)[(long long)m * n + j] = deep ? 0.0 : 0.5 * log(sn * sn + sh * sh);
    }
    if (m == 0) {
        static_cast<double*>(p.d1)[j] = d1 / n;
        static_cast<double*>(p.d2)[j] = d2 / n;
        const double sn = sinpi((double)j / n);
        static_cast<double*>(p.s2)[j] = sn * sn;
        static_cast<double*>(p.s2a)[j] = sinpi(2.0 * (double)j / n);
        static_cast<double*>(p.rs2)[j] = j == 0 ? 0.0 : 1.0 / (sn * sn);  // unused at j = 0 (the pair limit)
    }
}

// Circulant sums are split over kLanes lanes per output point (the lanes of
// an output take every kLanes-th source point, so the lanes of a wavefront
// read consecutive table and source entries) and folded by lane exchanges.
constexpr int kLanes = 16;
constexpr int kOutPerBlock = kFullThreads / kLanes;

__device__ __forceinline__ double lane_fold(double v) {
#pragma unroll
    for (int off = kLanes / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, kLanes);
    return v;
}

// --- b_x, b_xx of each member's bed (FP64 heights bz) at set-up
template <typename R>
__global__ void __launch_bounds__(kFullThreads) k_full_bedgeom(const FullParams p) {
    const int t = threadIdx.x;
    const int i = blockIdx.x * kOutPerBlock + t / kLanes;
    const int l = t % kLanes;
    const int m = blockIdx.z;
    const int n = p.n;
    const double* bz = static_cast<const double*>(p.bz) + (long long)m * n;
    const double* d1 = static_cast<const double*>(p.d1);
    const double* d2 = static_cast<const double*>(p.d2);
    double a1 = 0.0, a2 = 0.0;
    if (i < n)
        for (int j = l; j < n; j += kLanes) {
            const int d = (i - j + n) & (n - 1);
            a1 += d1[d] * bz[j];
            a2 += d2[d] * bz[j];
        }
    a1 = lane_fold(a1);
    a2 = lane_fold(a2);
    if (i < n && l == 0) {
        static_cast<double*>(p.bx)[(long long)m * n + i] = a1;
        static_cast<double*>(p.bxx)[(long long)m * n + i] = a2;
    }
}

__device__ __forceinline__ bool full_bed(const FullParams& p, int m) { return p.bed && p.bed[m]; }

// Decision of launch `sweep` from the residual of the previous one (the
// iteration mode's rules); every workgroup decides alike, the leader records.
__device__ __forceinline__ bool full_decided(const FullParams& p, Ctl* ctl, bool leader) {
    if (ctl->done) return true;
    double r, rmin;
    const int dec = sweep_decision(ctl, p.sweep, p.max_sweeps, p.tol, &r, &rmin);
    if (dec) {
        if (leader) ctl_commit(ctl, dec - 100, p.sweep, r);
        return true;
    }
    if (leader) {
        ctl->rmin = rmin;
        ctl->residual = r;
    }
    return false;
}

// --- pair sums over a slice of the source points, at the surface points.
// KIND 0: the double layer D[phi_s] (every member); KIND 1: the single layer
// (S - S0)[V_n] of the image-form members.  Partial sums go to
// part[split][member][point]; the consumer adds the slices in order.
// sinh of the small arguments of the pair kernels (scaled height differences
// pi (y_j - y_i) / L): below 1/8 by its Taylor series to the x^11 term, nested
// as x (1 + x^2/(2*3) (1 + x^2/(4*5) (...))), whose remainder is below 3e-21
// of the value there; beyond it by the library function.  A difference is
// passed as such (from exponentials of each point the sinh would lose its
// relative accuracy for nearby points).
template <typename R> __device__ __forceinline__ R sinh_series(R x) {
    if (fabs(x) >= R(0.125)) return sinh(x);
    const R x2 = x * x;
    R s = R(1) + x2 * R(1.0 / 110.0);
    s = R(1) + x2 * R(1.0 / 72.0) * s;
    s = R(1) + x2 * R(1.0 / 42.0) * s;
    s = R(1) + x2 * R(1.0 / 20.0) * s;
    s = R(1) + x2 * R(1.0 / 6.0) * s;
    return x * s;
}

// sinh and cosh of a small argument together: below 1/8 both by their Taylor
// series (cosh to the x^12 term, nested as 1 + x^2/(1*2) (1 + x^2/(3*4) (...)),
// remainder below 3e-24), beyond it the library sinh and cosh = sqrt(1 + sinh^2)
template <typename R> __device__ __forceinline__ R sinh_cosh_series(R x, R* ch) {
    if (fabs(x) >= R(0.125)) {
        const R sh = sinh(x);
        *ch = sqrt(R(1) + sh * sh);
        return sh;
    }
    const R x2 = x * x;
    R c = R(1) + x2 * R(1.0 / 132.0);
    c = R(1) + x2 * R(1.0 / 90.0) * c;
    c = R(1) + x2 * R(1.0 / 56.0) * c;
    c = R(1) + x2 * R(1.0 / 30.0) * c;
    c = R(1) + x2 * R(1.0 / 12.0) * c;
    *ch = R(1) + x2 * R(0.5) * c;
    return sinh_series(x);
}

template <typename R, int KIND>
__global__ void __launch_bounds__(kFullThreads) k_full_pairs(const FullParams p) {
    __shared__ R te[kFullThreads], tex[kFullThreads], tsrc[kFullThreads];
    const int t = threadIdx.x;
    const int i = blockIdx.x * kFullThreads + t;
    const int split = blockIdx.y;
    const int m = blockIdx.z;
    const int n = p.n;
    if (KIND == 1) {
        Ctl* ctl = p.ctl + m;
        const bool leader = blockIdx.x == 0 && blockIdx.y == 0 && t == 0;
        if (full_decided(p, ctl, leader)) return;  // workgroup-uniform
    }
    const long long mo = m * p.s_phys;
    const R* eta = static_cast<const R*>(p.eta) + mo;
    const R* ex = static_cast<const R*>(p.ex) + mo;
    if (KIND == 1 && full_bed(p, m)) return;  // the two-boundary surface pass serves it
    const R* src = static_cast<const R*>(KIND == 0 ? p.phi : p.vin) + mo;
    const double* s2 = static_cast<const double*>(p.s2);
    const double* rs2 = static_cast<const double*>(p.rs2);
    const double* s2at = static_cast<const double*>(p.s2a);
    const double* lfl = static_cast<const double*>(p.lfl) + (long long)m * n;
    const R pl = R(M_PI / p.lx);
    const bool deep = full_deep(p, m);
    const bool img = !deep && !full_bed(p, m);       // the image form keeps the bed's image
    const R b2h = R(2.0 * M_PI * p.href[m] / p.lx);  // 2 pi h / L
    // this point's values
    const bool on = i < n;
    const R etai = on ? eta[i] : R(0);
    const R exi = on ? ex[i] : R(0);
    double acc = 0.0;
    const int chunk = (n + gridDim.y - 1) / gridDim.y;
    const int jbeg = split * chunk, jend = min(n, jbeg + chunk);
    for (int j0 = jbeg; j0 < jend; j0 += kFullThreads) {
        __syncthreads();
        const int jl = j0 + t;
        if (jl < jend) {
            te[t] = eta[jl];
            tex[t] = ex[jl];
            tsrc[t] = src[jl];
        }
        __syncthreads();
        const int jn = min(kFullThreads, jend - j0);
        if (!on) continue;
        for (int jj = 0; jj < jn; ++jj) {
            const int j = j0 + jj;
            const int d = (j - i + n) & (n - 1);
            const R sa2 = R(s2[d]);                       // sin^2(pi (x_j - x_i) / L)
            // sinh of the scaled elevation difference, formed from the difference
            // itself (from exponentials of each point it would lose all relative
            // accuracy for nearby points)
            R chb;
            const R shb = sinh_cosh_series(pl * (te[jj] - etai), &chb);  // sinh(pi (eta_j - eta_i) / L)
            R kv;
            if (KIND == 1) {
                // -1/2 ln(1 + sinh^2 / sin^2); its limit -1/2 ln(1 + eta_x^2) at j = i
                kv = j == i ? R(-0.5) * log1p(exi * exi) : R(-0.5) * log1p(shb * shb * R(rs2[d]));
                if (img) {
                    // image minus flat image: -1/2 ln(sin^2 + sinh^2(pi (eta_i + eta_j + 2h) / L))
                    // + 1/2 ln(sin^2 + sinh^2(2 pi h / L))
                    const R shp = sinh_series(pl * (te[jj] + etai) + b2h);
                    kv += R(-0.5) * log(sa2 + shp * shp) + R(lfl[d]);
                }
            } else {
                // Im[(pi/L) cot(a + i b) (1 + i eta_x,j)], a = pi (x_j - x_i)/L, b = pi (eta_j - eta_i)/L:
                // cot(a + i b) = (sin 2a - i sinh 2b) / (2 (sin^2 a + sinh^2 b))
                const R s2a = R(s2at[d]);  // sin 2a
                if (j == i) {
                    kv = R(0);  // the curvature limit is added below
                } else {
                    const R den = R(2) * (sa2 + shb * shb);
                    kv = pl * (R(-2) * shb * chb + s2a * tex[jj]) / den;
                }
                if (img) {
                    // the image partner: b' = pi (eta_i + eta_j + 2h) / L
                    R chp;
                    const R shp = sinh_cosh_series(pl * (te[jj] + etai) + b2h, &chp);
                    const R den = R(2) * (sa2 + shp * shp);
                    kv += pl * (R(-2) * shp * chp + s2a * tex[jj]) / den;
                }
            }
            acc += (double)kv * (double)tsrc[jj];
        }
    }
    if (!on) return;
    const double dx = p.lx / n;
    double out = acc * dx;
    if (KIND == 0 && i >= jbeg && i < jend) {
        // the diagonal of the direct double layer: eta_xx / (2 (1 + eta_x^2))
        const double exx = (double)static_cast<const R*>(p.exx)[mo + i];
        out += dx * exx / (2.0 * (1.0 + (double)exi * (double)exi)) * (double)src[i];
    }
    static_cast<double*>(p.part)[((long long)split * p.batch + m) * n + i] = out;
}

// --- the single layer (S - S0)[V_n] of the image-form members from the
// symmetry of its kernel: K(i, j) = K(j, i) (both the direct part and the
// image depend on |eta_j - eta_i|, eta_i + eta_j and sin^2(pi (x_j - x_i)/L)).
// The n x n pairs split into tiles of kSymT x kSymT points; a workgroup takes
// tile (I, J), I <= J, evaluates each of its pairs once and adds K V_j to the
// row sums of its points i in block I and K V_i (reduced over a wavefront's
// rows) to the column sums of its points j in block J.  Row sums go to slice J
// of the points of block I, column sums to slice I of those of block J, so
// every point receives n / kSymT slices, one from each block, each written
// once; a diagonal tile (I = I) evaluates all its pairs and writes rows only.
constexpr int kSymT = kFullSymTile;
constexpr int kSymThreads = 2 * kSymT;  // two threads per row, each over half the tile's columns
static_assert(kSymT / 2 == 64, "a half tile's columns are the lanes of one wavefront");

template <typename R>
__global__ void __launch_bounds__(kSymThreads) k_full_sympairs(const FullParams p) {
    __shared__ R tej[kSymT], tvj[kSymT], tsj[kSymT], tcj[kSymT];
    __shared__ double colp[kSymThreads / 64][kSymT / 2];
    __shared__ double rowp[2][kSymT];
    const int t = threadIdx.x;
    const int m = blockIdx.z;
    const int n = p.n;
    const int nb = n / kSymT;
    {
        Ctl* ctl = p.ctl + m;
        const bool leader = blockIdx.x == 0 && t == 0;
        if (full_decided(p, ctl, leader)) return;  // workgroup-uniform
    }
    if (full_bed(p, m)) return;
    // tile (I, J), I <= J, of this workgroup's linear index (row-major upper triangle)
    int L = blockIdx.x, I = 0;
    while (L >= nb - I) {
        L -= nb - I;
        ++I;
    }
    const int J = I + L;
    const bool diag = I == J;
    const long long mo = m * p.s_phys;
    const R* eta = static_cast<const R*>(p.eta) + mo;
    const R* ex = static_cast<const R*>(p.ex) + mo;
    const R* v = static_cast<const R*>(p.vin) + mo;
    const double* s2 = static_cast<const double*>(p.s2);
    const double* rs2 = static_cast<const double*>(p.rs2);
    const double* lfl = static_cast<const double*>(p.lfl) + (long long)m * n;
    const R pl = R(M_PI / p.lx);
    const bool img = !full_deep(p, m);
    const R b2h = R(2.0 * M_PI * p.href[m] / p.lx);
    const int il = t % kSymT, hf = t / kSymT;
    const int i = I * kSymT + il;
    const R etai = eta[i], exi = ex[i];
    const double vi = (double)v[i];
    // the image's sinh(pi (eta_j + eta_i + 2h) / L) as sinh(a_j + b_i) =
    // sinh a_j cosh b_i + cosh a_j sinh b_i, a_j = pi eta_j / L, b_i = pi eta_i
    // / L + 2 pi h / L: one sinh and cosh per point instead of a sinh per pair
    // (with the bed below the surface b_i > |a_j|, so the second term
    // dominates the first and the sum does not cancel)
    R sbi = R(0), cbi = R(1);
    if (img) {
        const R b = pl * etai + b2h;
        sbi = sinh(b);
        cbi = cosh(b);
    }
    if (t < kSymT) {
        const R ej = eta[J * kSymT + t];
        tej[t] = ej;
        tvj[t] = v[J * kSymT + t];
        if (img) {
            tsj[t] = sinh(pl * ej);
            tcj[t] = cosh(pl * ej);
        }
    }
    __syncthreads();
    const int wv = t / 64, ln = t & 63;
    const int from = (ln + 1) & 63;
    double acc = 0.0, cacc = 0.0;
    for (int jj = 0; jj < kSymT / 2; ++jj) {
        // lane ln takes the columns of its half in the order ln, ln + 1, ...
        // (mod 64): at each step the lanes of a wavefront hold 64 different
        // columns, and the running column sum moves one lane down with its column
        const int jl = hf * (kSymT / 2) + ((ln + jj) & (kSymT / 2 - 1));
        const int j = J * kSymT + jl;
        const int d = (j - i + n) & (n - 1);
        const R sa2 = R(s2[d]);
        const R shb = sinh_series(pl * (tej[jl] - etai));
        R kv = j == i ? R(-0.5) * log1p(exi * exi) : R(-0.5) * log1p(shb * shb * R(rs2[d]));
        if (img) {
            const R shp = tsj[jl] * cbi + tcj[jl] * sbi;
            kv += R(-0.5) * log(sa2 + shp * shp) + R(lfl[d]);
        }
        acc += (double)kv * (double)tvj[jl];
        if (!diag) {
            // the pair seen from j: K V_i added to column jl's sum over this
            // wavefront's rows, which lane ln - 1 continues at the next step
            cacc += (double)kv * vi;
            cacc = __shfl(cacc, from, 64);
        }
    }
    rowp[hf][il] = acc;
    if (!diag) colp[wv][ln] = cacc;  // after 64 steps lane ln holds column ln of its half
    __syncthreads();
    if (t < kSymT) {
        const double dx = p.lx / n;
        double* part = static_cast<double*>(p.part);
        // rows of block I: slice J
        part[((long long)J * p.batch + m) * n + I * kSymT + t] = (rowp[0][t] + rowp[1][t]) * dx;
        if (!diag) {
            // columns of block J: slice I; column jl collects the two wavefronts of its half
            const int h2 = t / (kSymT / 2), q = t % (kSymT / 2);
            part[((long long)I * p.batch + m) * n + J * kSymT + t] = (colp[2 * h2][q] + colp[2 * h2 + 1][q]) * dx;
        }
    }
}

// --- the surface pass of the two-boundary members: (S - S_flat)[V_n] (no
// image; V_n absent at the first sweep) minus D_SB[phi_b] with the phi_b of
// this sweep, at the surface points over a slice of the source points
template <typename R>
__global__ void __launch_bounds__(kFullThreads) k_full_spairs(const FullParams p) {
    __shared__ R te[kFullThreads], tsrc[kFullThreads];
    __shared__ double tbz[kFullThreads], tbx[kFullThreads], tpb[kFullThreads];
    const int t = threadIdx.x;
    const int i = blockIdx.x * kFullThreads + t;
    const int split = blockIdx.y;
    const int m = blockIdx.z;
    const int n = p.n;
    {
        Ctl* ctl = p.ctl + m;
        const bool leader = blockIdx.x == 0 && blockIdx.y == 0 && t == 0;
        if (full_decided(p, ctl, leader)) return;  // workgroup-uniform
    }
    if (!full_bed(p, m)) return;
    const long long mo = m * p.s_phys, mb = (long long)m * n;
    const R* eta = static_cast<const R*>(p.eta) + mo;
    const R* ex = static_cast<const R*>(p.ex) + mo;
    const bool hasv = p.vin != nullptr;
    const R* src = hasv ? static_cast<const R*>(p.vin) + mo : nullptr;
    const double* bz = static_cast<const double*>(p.bz) + mb;
    const double* bxs = static_cast<const double*>(p.bx) + mb;
    const double* pbs = static_cast<const double*>(p.pbout) + mb;
    const double* s2 = static_cast<const double*>(p.s2);
    const double* rs2 = static_cast<const double*>(p.rs2);
    const double* s2at = static_cast<const double*>(p.s2a);
    const R pl = R(M_PI / p.lx);
    const double pld = M_PI / p.lx;
    const bool on = i < n;
    const R etai = on ? eta[i] : R(0);
    const R exi = on ? ex[i] : R(0);
    double acc = 0.0;
    const int chunk = (n + gridDim.y - 1) / gridDim.y;
    const int jbeg = split * chunk, jend = min(n, jbeg + chunk);
    for (int j0 = jbeg; j0 < jend; j0 += kFullThreads) {
        __syncthreads();
        const int jl = j0 + t;
        if (jl < jend) {
            te[t] = eta[jl];
            tsrc[t] = hasv ? src[jl] : R(0);
            tbz[t] = bz[jl];
            tbx[t] = bxs[jl];
            tpb[t] = pbs[jl];
        }
        __syncthreads();
        const int jn = min(kFullThreads, jend - j0);
        if (!on) continue;
        for (int jj = 0; jj < jn; ++jj) {
            const int j = j0 + jj;
            const int d = (j - i + n) & (n - 1);
            const R sa2 = R(s2[d]);
            const R s2a = R(s2at[d]);
            // the bed source (x_j, b_j): -D_SB = Im[(pi/L) cot(a + i b) (1 + i b_x,j)],
            // b = pi (b_j - eta_i) / L (the bed lies below every surface point)
            R ch;
            const R sh = sinh_cosh_series(R(pld * (tbz[jj] - (double)etai)), &ch);
            acc += (double)(pl * (R(-2) * sh * ch + s2a * R(tbx[jj])) / (R(2) * (sa2 + sh * sh))) * tpb[jj];
            if (hasv) {
                // the direct single layer minus the flat one, as in the image form
                const R shb = sinh_series(pl * (te[jj] - etai));
                const R kv = j == i ? R(-0.5) * log1p(exi * exi) : R(-0.5) * log1p(shb * shb * R(rs2[d]));
                acc += (double)kv * (double)tsrc[jj];
            }
        }
    }
    if (!on) return;
    static_cast<double*>(p.part)[((long long)split * p.batch + m) * n + i] = acc * (p.lx / n);
}

// --- pair sums at the bed points of two-boundary members, over a slice of
// the source points.  KIND 2: D_BS[phi_s] (surface sources); KIND 3:
// S_BS[V_n] - D_BB[phi_b] (surface and bed sources, phi_b of this sweep),
// which also decides the sweep.  With a = pi (x_j - x_i) / L and b the scaled
// height difference pi (y_j - y_i) / L of source and evaluation point:
// G = -1/2 ln(4 (sin^2 a + sinh^2 b)); the double layer of a surface source is
// Im[(pi/L) cot(a + i b) (1 + i eta_x,j)], that of a bed source
// -Im[(pi/L) cot(a + i b) (1 + i b_x,j)], with the curvature limit
// -b_xx / (2 (1 + b_x^2)) at coincident bed points.
template <typename R, int KIND>
__global__ void __launch_bounds__(kFullThreads) k_full_bpairs(const FullParams p) {
    __shared__ R te[kFullThreads], tex[kFullThreads], tsrc[kFullThreads];
    __shared__ double tbz[kFullThreads], tbx[kFullThreads], tpb[kFullThreads];
    const int t = threadIdx.x;
    const int i = blockIdx.x * kFullThreads + t;
    const int split = blockIdx.y;
    const int m = blockIdx.z;
    const int n = p.n;
    if (KIND == 3) {
        Ctl* ctl = p.ctl + m;
        const bool leader = blockIdx.x == 0 && blockIdx.y == 0 && t == 0;
        if (full_decided(p, ctl, leader)) return;  // workgroup-uniform
    }
    if (!full_bed(p, m)) return;
    const long long mo = m * p.s_phys, mb = (long long)m * n;
    const R* eta = static_cast<const R*>(p.eta) + mo;
    const R* ex = static_cast<const R*>(p.ex) + mo;
    const R* src = static_cast<const R*>(KIND == 2 ? p.phi : p.vin) + mo;
    const double* bz = static_cast<const double*>(p.bz) + mb;
    const double* bxs = static_cast<const double*>(p.bx) + mb;
    const double* pbs = KIND == 3 ? static_cast<const double*>(p.pbin) + mb : nullptr;
    const double* s2 = static_cast<const double*>(p.s2);
    const double* s2at = static_cast<const double*>(p.s2a);
    const R pl = R(M_PI / p.lx);
    const double pld = M_PI / p.lx;
    const bool on = i < n;
    const double bzi = on ? bz[i] : 0.0;
    double acc = 0.0;
    const int chunk = (n + gridDim.y - 1) / gridDim.y;
    const int jbeg = split * chunk, jend = min(n, jbeg + chunk);
    for (int j0 = jbeg; j0 < jend; j0 += kFullThreads) {
        __syncthreads();
        const int jl = j0 + t;
        if (jl < jend) {
            te[t] = eta[jl];
            tex[t] = ex[jl];
            tsrc[t] = src[jl];
            if (KIND == 3) {
                tbz[t] = bz[jl];
                tbx[t] = bxs[jl];
                tpb[t] = pbs[jl];
            }
        }
        __syncthreads();
        const int jn = min(kFullThreads, jend - j0);
        if (!on) continue;
        for (int jj = 0; jj < jn; ++jj) {
            const int j = j0 + jj;
            const int d = (j - i + n) & (n - 1);
            const R sa2 = R(s2[d]);
            const R s2a = R(s2at[d]);
            // the surface source (x_j, eta_j) seen from the bed point (x_i, b_i)
            R ch;
            const R sh = sinh_cosh_series(R(pld * ((double)te[jj] - bzi)), &ch);
            const R den = R(2) * (sa2 + sh * sh);
            if (KIND == 2) {
                acc += (double)(pl * (R(-2) * sh * ch + s2a * tex[jj]) / den) * (double)tsrc[jj];
            } else {
                acc += (double)(R(-0.5) * log(R(2) * den)) * (double)tsrc[jj];
                if (j != i) {
                    // minus the bed's double layer at (x_j, b_j)
                    R chb;
                    const R shb = sinh_cosh_series(R(pld * (tbz[jj] - bzi)), &chb);
                    const R denb = R(2) * (sa2 + shb * shb);
                    acc += (double)(pl * (R(-2) * shb * chb + s2a * R(tbx[jj])) / denb) * tpb[jj];
                }
            }
        }
    }
    if (!on) return;
    const double dx = p.lx / n;
    double out = acc * dx;
    if (KIND == 3 && i >= jbeg && i < jend) {
        // minus the diagonal of the bed's double layer: + b_xx / (2 (1 + b_x^2)) phi_b
        const double bxi = bxs[i], bxxi = static_cast<const double*>(p.bxx)[mb + i];
        out += dx * bxxi / (2.0 * (1.0 + bxi * bxi)) * pbs[i];
    }
    static_cast<double*>(p.part)[((long long)split * p.batch + m) * n + i] = out;
}

// --- rb = -D_BS[phi_s] of the two-boundary members (slices added in order)
template <typename R>
__global__ void k_full_rb(const FullParams p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.z;
    if (i >= p.n || !full_bed(p, m)) return;
    double a = 0.0;
    for (int s = 0; s < p.nsplit; ++s) a -= static_cast<const double*>(p.part)[((long long)s * p.batch + m) * p.n + i];
    static_cast<double*>(p.rb)[(long long)m * p.n + i] = a;
}

// --- phi_b of the next sweep, (rb + S_BS[V_n] - D_BB[phi_b]) / pi, for the
// undecided two-boundary members (no bed pass at the first sweep: V_0 = 0,
// phi_b = 0)
template <typename R>
__global__ void k_full_pb(const FullParams p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.z;
    if (i >= p.n || !full_bed(p, m) || p.ctl[m].done) return;
    const long long o = (long long)m * p.n + i;
    double a = static_cast<const double*>(p.rb)[o];
    if (p.pbin)
        for (int s = 0; s < p.nsplit; ++s) a += static_cast<const double*>(p.part)[((long long)s * p.batch + m) * p.n + i];
    static_cast<double*>(p.pbout)[o] = a / M_PI;
}

// --- rhs = pi phi_s + D[phi_s] (slices added in order)
template <typename R>
__global__ void k_full_rhs(const FullParams p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.z;
    if (i >= p.n) return;
    const long long mo = m * p.s_phys;
    double a = M_PI * (double)static_cast<const R*>(p.phi)[mo + i];
    for (int s = 0; s < p.nsplit; ++s) a += static_cast<const double*>(p.part)[((long long)s * p.batch + m) * p.n + i];
    static_cast<double*>(p.rhs)[(long long)m * p.n + i] = a;
}

// --- w = rhs - (S - S0)[V_n], or rhs - (S - S_flat)[V_n] + D_SB[phi_b] (the
// slices of the surface pass, in order; w = rhs at the first sweep of the
// image form, from V_0 = 0)
template <typename R>
__global__ void k_full_combine(const FullParams p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.z;
    if (i >= p.n) return;
    if (p.ctl[m].done) return;  // decided by this sweep's pair pass
    const long long o = (long long)m * p.n + i;
    double w = static_cast<const double*>(p.rhs)[o];
    // slices: those of the two-boundary surface pass, or of the image form's
    // single layer (nsym of the symmetric pass when it ran)
    const int ns = full_bed(p, m) ? p.nsplit : (p.nsym > 0 ? p.nsym : p.nsplit);
    if (p.vin || full_bed(p, m))
        for (int s = 0; s < ns; ++s) w -= static_cast<const double*>(p.part)[((long long)s * p.batch + m) * p.n + i];
    static_cast<double*>(p.w)[o] = w;
}

// --- V_(n+1) = S0^-1 w (+ S0^-1 (S0 - S_flat)[V_n] in the two-boundary form)
// in two passes.  The sum pass: workgroup (x, s) forms the kApOuts outputs of
// block x over source slice s; a thread forms kApR consecutive outputs over one
// of kApLanes ranges of the slice (its wavefront's: the source value is
// wave-uniform), keeping the kApR circulant entries c[i + r - j] as a window
// that moves by one entry per source point, so each step loads one table entry
// for kApR products; the ranges are added in LDS in a fixed order and the
// slice's sums go to the pair-pass slices, spent by then.  The finish pass adds
// the slices in order and takes the residual maxima max|V_(n+1) - V_n|,
// max|V_(n+1)| into the member's slot `sweep`.
constexpr int kApR = 4, kApLanes = 8, kApB = 16;
constexpr int kApThreads = 64 * kApLanes;
constexpr int kApOuts = 64 * kApR;  // outputs per workgroup
// source slices of the sum pass: enough workgroups to cover the chip at 4096
// points, each lane's range at least kApB points when n allows
__host__ __device__ constexpr int apply_slices(int n) { return n / 128 < 1 ? 1 : (n / 128 > 16 ? 16 : n / 128); }


// acc[k][r] += sum_j tab[k][(i0 + r - j) mod n] src_j over j in [jb, je), for
// NT tables against one source, in blocks of kApB source points whose table
// entries and source values are all requested before the block's products
// (one memory latency per block)
template <int NT, typename S>
__device__ __forceinline__ void circ_window(const double* const (&tab)[NT], const S* src, int i0, int jb, int je,
                                            int msk, double (&acc)[NT][kApR]) {
    double cw[NT][kApR];
#pragma unroll
    for (int k = 0; k < NT; ++k)
#pragma unroll
        for (int r = 0; r < kApR; ++r) cw[k][r] = tab[k][(i0 + r - jb) & msk];
    for (int j0 = jb; j0 < je; j0 += kApB) {
        double nx[NT][kApB], sv[kApB];
#pragma unroll
        for (int q = 0; q < kApB; ++q) {
            const int j = j0 + q;
#pragma unroll
            for (int k = 0; k < NT; ++k) nx[k][q] = tab[k][(i0 - j - 1) & msk];  // enters the window after point j
            sv[q] = j < je ? (double)src[j] : 0.0;  // a short range (small n) ends inside a block
        }
#pragma unroll
        for (int q = 0; q < kApB; ++q)
#pragma unroll
            for (int k = 0; k < NT; ++k) {
#pragma unroll
                for (int r = 0; r < kApR; ++r) acc[k][r] += cw[k][r] * sv[q];
#pragma unroll
                for (int r = kApR - 1; r > 0; --r) cw[k][r] = cw[k][r - 1];
                cw[k][0] = nx[k][q];
            }
    }
}

template <typename R>
__global__ void __launch_bounds__(kApThreads) k_full_apply(const FullParams p) {
    __shared__ double red[kApLanes][kApOuts];
    const int t = threadIdx.x;
    const int m = blockIdx.z;
    const int n = p.n;
    const int msk = n - 1;
    if (p.ctl[m].done) return;  // decided by this sweep's pair pass (workgroup-uniform)
    const long long mo = m * p.s_phys;
    const int lane = __builtin_amdgcn_readfirstlane(t / 64);
    const int o0 = (t & 63) * kApR;  // this thread's first output within the workgroup
    const int i0 = blockIdx.x * kApOuts + o0;
    const int ns = apply_slices(n);
    const int sl = n / ns;  // points per slice (n and ns are powers of two)
    const int jn = (sl + kApLanes - 1) / kApLanes;
    const int jb = blockIdx.y * sl + lane * jn, je = min(blockIdx.y * sl + sl, jb + jn);
    double acc[1][kApR];
#pragma unroll
    for (int r = 0; r < kApR; ++r) acc[0][r] = 0.0;
    if (jb < je) {
        const double* const c0[1] = {static_cast<const double*>(p.c0) + (long long)m * n};
        circ_window<1>(c0, static_cast<const double*>(p.w) + (long long)m * n, i0, jb, je, msk, acc);
        if (p.vin && full_bed(p, m)) {
            // + S0^-1 (S0 - S_flat)[V_n] of the two-boundary form
            const double* const cm[1] = {static_cast<const double*>(p.cm) + (long long)m * n};
            circ_window<1>(cm, static_cast<const R*>(p.vin) + mo, i0, jb, je, msk, acc);
        }
    }
#pragma unroll
    for (int r = 0; r < kApR; ++r) red[lane][o0 + r] = acc[0][r];
    __syncthreads();
    const int i = blockIdx.x * kApOuts + t;
    if (t < kApOuts && i < n) {
        double a = 0.0;
#pragma unroll
        for (int l = 0; l < kApLanes; ++l) a += red[l][t];
        static_cast<double*>(p.part)[((long long)blockIdx.y * p.batch + m) * n + i] = a;
    }
}

template <typename R>
__global__ void __launch_bounds__(kFullThreads) k_full_finish(const FullParams p) {
    const int t = threadIdx.x;
    const int i = blockIdx.x * kFullThreads + t;
    const int m = blockIdx.z;
    const int n = p.n;
    Ctl* ctl = p.ctl + m;
    if (ctl->done) return;  // workgroup-uniform
    const long long mo = m * p.s_phys;
    unsigned long long nu = 0ull, de = 0ull;
    if (i < n) {
        const int ns = apply_slices(n);
        double a = 0.0;
        for (int s2 = 0; s2 < ns; ++s2) a += static_cast<const double*>(p.part)[((long long)s2 * p.batch + m) * n + i];
        const R v = R(a);
        static_cast<R*>(p.vout)[mo + i] = v;
        const double vold = p.vin ? (double)static_cast<const R*>(p.vin)[mo + i] : 0.0;
        nu = abs_bits((double)v - vold);
        de = abs_bits((double)v);
        if (!isfinite((double)v)) nu = de = 0x7ff8000000000000ull;  // a NaN key outranks every finite one
    }
    block_reduce2_max_u64(nu, de);
    if (t == 0) {
        atomicMax(&ctl->slots->num[p.sweep], nu);
        atomicMax(&ctl->slots->den[p.sweep], de);
    }
}

// --- eta_x, eta_xx at every point: the circulant sums d1 * eta and d2 * eta
// by the apply's sum pass (both tables against eta; the ex slices first, then
// the exx slices, in the pair-pass slices, free at the start of a solve) and a
// pass that adds the slices in order
__host__ __device__ constexpr int geom_slices(int n) { return apply_slices(n) / 2 < 1 ? 1 : apply_slices(n) / 2; }

template <typename R>
__global__ void __launch_bounds__(kApThreads) k_full_geom(const FullParams p) {
    __shared__ double red[2][kApLanes][kApOuts];
    const int t = threadIdx.x;
    const int m = blockIdx.z;
    const int n = p.n;
    const int msk = n - 1;
    const int lane = __builtin_amdgcn_readfirstlane(t / 64);
    const int o0 = (t & 63) * kApR;
    const int i0 = blockIdx.x * kApOuts + o0;
    const int ns = geom_slices(n);
    const int sl = n / ns;
    const int jn = (sl + kApLanes - 1) / kApLanes;
    const int jb = blockIdx.y * sl + lane * jn, je = min(blockIdx.y * sl + sl, jb + jn);
    double acc[2][kApR];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int r = 0; r < kApR; ++r) acc[k][r] = 0.0;
    if (jb < je) {
        const double* const tab[2] = {static_cast<const double*>(p.d1), static_cast<const double*>(p.d2)};
        circ_window<2>(tab, static_cast<const R*>(p.eta) + m * p.s_phys, i0, jb, je, msk, acc);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int r = 0; r < kApR; ++r) red[k][lane][o0 + r] = acc[k][r];
    __syncthreads();
    const int i = blockIdx.x * kApOuts + t;
    if (t < kApOuts && i < n) {
        double* part = static_cast<double*>(p.part);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            double a = 0.0;
#pragma unroll
            for (int l = 0; l < kApLanes; ++l) a += red[k][l][t];
            part[((long long)(k * ns + blockIdx.y) * p.batch + m) * n + i] = a;
        }
    }
}

template <typename R>
__global__ void k_full_geomfin(const FullParams p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.z;
    const int n = p.n;
    if (i >= n) return;
    const int ns = geom_slices(n);
    const double* part = static_cast<const double*>(p.part);
    double a1 = 0.0, a2 = 0.0;
    for (int s = 0; s < ns; ++s) {
        a1 += part[((long long)s * p.batch + m) * n + i];
        a2 += part[((long long)(ns + s) * p.batch + m) * n + i];
    }
    static_cast<R*>(p.ex)[m * p.s_phys + i] = R(a1);
    static_cast<R*>(p.exx)[m * p.s_phys + i] = R(a2);
}

// --- the decided iterate V_s of every member (s = its sweep count) -> out
template <typename R>
__global__ void k_full_select(const FullParams p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.z;
    if (i >= p.n) return;
    const int s = p.ctl[m].sweeps;
    const long long mo = m * p.s_phys;
    static_cast<R*>(p.vfinal)[mo + i] = static_cast<const R*>(p.vbuf[s & 1])[mo + i];
}

// ---------------------------------------------------------------------------
template <> hipError_t launch_full_t<Real>(const FullParams& p, int what, hipStream_t s) {
    const int n = p.n;
    const int tiles = (n + kFullThreads - 1) / kFullThreads;
    const int outs = (n + kOutPerBlock - 1) / kOutPerBlock;
    switch (what) {
        case FULL_TABLES:
            hipLaunchKernelGGL(k_full_tables<Real>, dim3(tiles, p.batch), dim3(kFullThreads), 0, s, p);
            break;
        case FULL_GEOM: {
            hipLaunchKernelGGL(k_full_geom<Real>, dim3((n + kApOuts - 1) / kApOuts, geom_slices(n), p.batch),
                               dim3(kApThreads), 0, s, p);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k_full_geomfin<Real>, dim3(tiles, 1, p.batch), dim3(kFullThreads), 0, s, p);
            break;
        }
        case FULL_DOUBLE:
            hipLaunchKernelGGL((k_full_pairs<Real, 0>), dim3(tiles, p.nsplit, p.batch), dim3(kFullThreads), 0, s, p);
            break;
        case FULL_RHS:
            hipLaunchKernelGGL(k_full_rhs<Real>, dim3(tiles, 1, p.batch), dim3(kFullThreads), 0, s, p);
            break;
        case FULL_SINGLE:
            hipLaunchKernelGGL((k_full_pairs<Real, 1>), dim3(tiles, p.nsplit, p.batch), dim3(kFullThreads), 0, s, p);
            break;
        case FULL_COMBINE:
            hipLaunchKernelGGL(k_full_combine<Real>, dim3(tiles, 1, p.batch), dim3(kFullThreads), 0, s, p);
            break;
        case FULL_APPLY: {
            hipLaunchKernelGGL(k_full_apply<Real>, dim3((n + kApOuts - 1) / kApOuts, apply_slices(n), p.batch),
                               dim3(kApThreads), 0, s, p);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k_full_finish<Real>, dim3(tiles, 1, p.batch), dim3(kFullThreads), 0, s, p);
            break;
        }
        case FULL_SELECT:
            hipLaunchKernelGGL(k_full_select<Real>, dim3(tiles, 1, p.batch), dim3(kFullThreads), 0, s, p);
            break;
        case FULL_BEDGEOM:
            hipLaunchKernelGGL(k_full_bedgeom<Real>, dim3(outs, 1, p.batch), dim3(kFullThreads), 0, s, p);
            break;
        case FULL_RHSB:
            hipLaunchKernelGGL((k_full_bpairs<Real, 2>), dim3(tiles, p.nsplit, p.batch), dim3(kFullThreads), 0, s, p);
            break;
        case FULL_RB:
            hipLaunchKernelGGL(k_full_rb<Real>, dim3(tiles, 1, p.batch), dim3(kFullThreads), 0, s, p);
            break;
        case FULL_BED:
            hipLaunchKernelGGL((k_full_bpairs<Real, 3>), dim3(tiles, p.nsplit, p.batch), dim3(kFullThreads), 0, s, p);
            break;
        case FULL_SYM:
            if (n % kSymT != 0) return hipErrorInvalidValue;
            hipLaunchKernelGGL(k_full_sympairs<Real>, dim3((n / kSymT) * (n / kSymT + 1) / 2, 1, p.batch),
                               dim3(kSymThreads), 0, s, p);
            break;
        case FULL_SURF:
            hipLaunchKernelGGL(k_full_spairs<Real>, dim3(tiles, p.nsplit, p.batch), dim3(kFullThreads), 0, s, p);
            break;
        case FULL_PB:
            hipLaunchKernelGGL(k_full_pb<Real>, dim3(tiles, 1, p.batch), dim3(kFullThreads), 0, s, p);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace sbi
