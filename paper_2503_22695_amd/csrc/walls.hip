// Walled box ("Spatial Discretization": u* = 0 and u^{n+1}.n = 0 on the box
// faces) through its mirror image.  With the MAC ghost-cell convention
// (tangential ghost = minus the interior value, the wall-normal component on
// the wall faces held at zero) the walled operators are the restrictions of
// the periodic ones on the (2n)^3 grid of the box and its images: velocity
// components are odd across every wall, pressure is even (Neumann).  The
// image grid is an ordinary periodic context on the unit box, so its spacing
// is h/2 and every derivative carries its factor: Lap_h = Lap_{h/2} / 4 (the
// image context's viscosity is mu/4, the Poisson right-hand side is scaled by
// 4), D_h, G_h and C_h are half their h/2 versions, spreading at X/2 is 8 times
// the box's and interpolation is unchanged.  The projection's right-hand side
// is the box divergence mirrored evenly: the image divergence of a no-slip
// image field is not even across the walls.
//
// Index maps per axis (image index i' in 0..2n-1): a cell-centred axis maps
// i' >= n to 2n-1-i'; the wall-normal axis of a velocity component is
// face-centred, faces 0 and n are walls (value 0) and i' > n maps to 2n-i'.  A
// mirrored axis gives a factor -1 for velocity, +1 for pressure.
#include "internal.h"

namespace hipib {
namespace {

constexpr int WT = 256;

// returns the sign (0: a wall face) and the box index of image index ip
__device__ __forceinline__ int wall_src(int n, int ip, bool face, int* src) {
    if (face) {
        if (ip == 0 || ip == n) return 0;
        if (ip < n) { *src = ip; return 1; }
        *src = 2 * n - ip;
        return -1;
    }
    if (ip < n) { *src = ip; return 1; }
    *src = 2 * n - 1 - ip;
    return -1;
}

// mirroring modes: 0 even cell-centred scalar (pressure), 1 velocity (each
// component odd, face-centred along its own axis), 2 odd cell-centred scalar
// (one Dirichlet field, as the walled Helmholtz solve of hipib_mg_solve takes it)
enum { W_EVEN = 0, W_VELOCITY = 1, W_ODD = 2 };

// img[c][k'][j'][i'] = sign * box[c][k][j][i] (0 on wall faces), c < ncomp
__global__ void __launch_bounds__(WT)
k_wall_extend(const double* __restrict__ box, double* __restrict__ img, int n, int ncomp, int mode) {
    const int m = 2 * n;
    const int64_t M3 = (int64_t)m * m * m, N3 = (int64_t)n * n * n;
    const int64_t t = (int64_t)blockIdx.x * WT + threadIdx.x;
    if (t >= ncomp * M3) return;
    const int d = (int)(t / M3);
    const int64_t r = t - d * M3;
    const int ip = (int)(r % m), jp = (int)((r / m) % m), kp = (int)(r / ((int64_t)m * m));
    const bool vector = mode == W_VELOCITY;
    int i = 0, j = 0, k = 0;
    const int si = wall_src(n, ip, vector && d == 0, &i);
    const int sj = wall_src(n, jp, vector && d == 1, &j);
    const int sk = wall_src(n, kp, vector && d == 2, &k);
    double v = 0.0;
    if (si && sj && sk) {
        const double sg = mode == W_EVEN ? 1.0 : (double)(si * sj * sk);
        v = sg * box[d * N3 + i + (int64_t)n * (j + (int64_t)n * k)];
    }
    img[t] = v;
}

// box = the box part of img, the wall faces of velocity components zero
__global__ void __launch_bounds__(WT)
k_wall_restrict(const double* __restrict__ img, double* __restrict__ box, int n, int ncomp, int mode) {
    const bool vector = mode == W_VELOCITY;
    const int m = 2 * n;
    const int64_t M3 = (int64_t)m * m * m, N3 = (int64_t)n * n * n;
    const int64_t t = (int64_t)blockIdx.x * WT + threadIdx.x;
    if (t >= ncomp * N3) return;
    const int d = (int)(t / N3);
    const int64_t r = t - d * N3;
    const int i = (int)(r % n), j = (int)((r / n) % n), k = (int)(r / ((int64_t)n * n));
    const bool wall = vector && ((d == 0 && i == 0) || (d == 1 && j == 0) || (d == 2 && k == 0));
    box[t] = wall ? 0.0 : img[d * M3 + i + (int64_t)m * (j + (int64_t)m * k)];
}

// box[d] += scale * sum over the image cells mapping to it of sign * img, d <
// ncomp, summed in image-index order: the transpose of k_wall_extend for
// velocity (mode W_VELOCITY) or an even cell-centred scalar (W_EVEN)
__global__ void __launch_bounds__(WT)
k_wall_fold(const double* __restrict__ img, double* __restrict__ box, int n, int ncomp, int mode,
            double scale) {
    const bool vector = mode == W_VELOCITY;
    const int m = 2 * n;
    const int64_t M3 = (int64_t)m * m * m, N3 = (int64_t)n * n * n;
    const int64_t t = (int64_t)blockIdx.x * WT + threadIdx.x;
    if (t >= ncomp * N3) return;
    const int d = (int)(t / N3);
    const int64_t r = t - d * N3;
    const int ijk[3] = {(int)(r % n), (int)((r / n) % n), (int)(r / ((int64_t)n * n))};
    // per axis: the (up to two) image indices that map here, ascending, with signs
    int pre[3][2], sg[3][2], cnt[3];
    for (int a = 0; a < 3; ++a) {
        const int x = ijk[a];
        const int mirror = vector ? -1 : 1;
        if (vector && a == d) {   // face-centred: faces 1..n-1 come from x and 2n-x; face 0 is a wall
            cnt[a] = x == 0 ? 0 : 2;
            pre[a][0] = x; sg[a][0] = 1;
            pre[a][1] = 2 * n - x; sg[a][1] = mirror;
        } else {
            cnt[a] = 2;
            pre[a][0] = x; sg[a][0] = 1;
            pre[a][1] = 2 * n - 1 - x; sg[a][1] = mirror;
        }
    }
    double s = 0.0;
    for (int c = 0; c < cnt[2]; ++c)
        for (int b = 0; b < cnt[1]; ++b)
            for (int a = 0; a < cnt[0]; ++a)
                s += (double)(sg[0][a] * sg[1][b] * sg[2][c]) *
                     img[d * M3 + pre[0][a] + (int64_t)m * (pre[1][b] + (int64_t)m * pre[2][c])];
    box[t] = box[t] + scale * s;
}

// the transpose of k_wall_restrict: img = box values in the box part (velocity
// wall faces zero), zero in the images
__global__ void __launch_bounds__(WT)
k_wall_pad(const double* __restrict__ box, double* __restrict__ img, int n, int ncomp, int mode) {
    const bool vector = mode == W_VELOCITY;
    const int m = 2 * n;
    const int64_t M3 = (int64_t)m * m * m, N3 = (int64_t)n * n * n;
    const int64_t t = (int64_t)blockIdx.x * WT + threadIdx.x;
    if (t >= ncomp * M3) return;
    const int d = (int)(t / M3);
    const int64_t r = t - d * M3;
    const int ip = (int)(r % m), jp = (int)((r / m) % m), kp = (int)(r / ((int64_t)m * m));
    double v = 0.0;
    if (ip < n && jp < n && kp < n) {
        const bool wall = vector && ((d == 0 && ip == 0) || (d == 1 && jp == 0) || (d == 2 && kp == 0));
        if (!wall) v = box[d * N3 + ip + (int64_t)n * (jp + (int64_t)n * kp)];
    }
    img[t] = v;
}

// y = a x (element-wise), or y += a x
__global__ void __launch_bounds__(WT)
k_scale(const double* __restrict__ x, double* __restrict__ y, double a, int64_t count, int accumulate) {
    const int64_t t = (int64_t)blockIdx.x * WT + threadIdx.x;
    if (t >= count) return;
    y[t] = accumulate ? y[t] + a * x[t] : a * x[t];
}

unsigned blocks_for(int64_t count) { return (unsigned)((count + WT - 1) / WT); }

hipib_status extend(hipib_ctx* ctx, const double* box, double* img, int ncomp, int mode) {
    const int64_t M3 = ctx->img->n3;
    k_wall_extend<<<blocks_for(ncomp * M3), WT, 0, ctx->stream>>>(box, img, ctx->n, ncomp, mode);
    HIPIB_HIP(hipGetLastError());
    return HIPIB_OK;
}

hipib_status restrict_box(hipib_ctx* ctx, const double* img, double* box, int ncomp, int mode) {
    k_wall_restrict<<<blocks_for(ncomp * ctx->n3), WT, 0, ctx->stream>>>(img, box, ctx->n, ncomp, mode);
    HIPIB_HIP(hipGetLastError());
    return HIPIB_OK;
}

// box = fold(img) (box zeroed first) or box += fold(img)
hipib_status fold(hipib_ctx* ctx, const double* img, double* box, int ncomp, int mode, double s,
                  bool acc) {
    if (!acc) HIPIB_TRY(launch_zero(ctx, box, ncomp * ctx->n3));
    k_wall_fold<<<blocks_for(ncomp * ctx->n3), WT, 0, ctx->stream>>>(img, box, ctx->n, ncomp, mode, s);
    HIPIB_HIP(hipGetLastError());
    return HIPIB_OK;
}

hipib_status pad(hipib_ctx* ctx, const double* box, double* img, int ncomp, int mode) {
    k_wall_pad<<<blocks_for(ncomp * ctx->img->n3), WT, 0, ctx->stream>>>(box, img, ctx->n, ncomp, mode);
    HIPIB_HIP(hipGetLastError());
    return HIPIB_OK;
}

hipib_status scale(hipib_ctx* ctx, const double* x, double* y, double a, int64_t count, bool acc) {
    if (count <= 0) return HIPIB_OK;
    k_scale<<<blocks_for(count), WT, 0, ctx->stream>>>(x, y, a, count, acc ? 1 : 0);
    HIPIB_HIP(hipGetLastError());
    return HIPIB_OK;
}

template <typename T>
hipib_status alloc(hipib_ctx* ctx, T** p, size_t count) {
    (void)ctx;
    *p = nullptr;
    if (hipMalloc(reinterpret_cast<void**>(p), (count ? count : 1) * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(HIPIB_E_NOMEM, "hipMalloc of %zu bytes failed", count * sizeof(T));
    }
    return HIPIB_OK;
}

// positions on the image grid's unit box and their bins
hipib_status image_positions(hipib_ctx* ctx, const double* X) {
    HIPIB_TRY(scale(ctx, X, ctx->w_Xh, 0.5, 3 * (int64_t)ctx->nn, false));
    return launch_bin(ctx->img, ctx->w_Xh);
}

}  // namespace

hipib_status walled_create(hipib_ctx* ctx) {
    hipib_config c2 = ctx->cfg;
    c2.n = 2 * ctx->n;
    c2.mu = 0.25 * ctx->cfg.mu;
    c2.walls = 0;
    HIPIB_TRY(hipib_create(&c2, ctx->stream, &ctx->img));
    const int64_t M3 = ctx->img->n3;
    HIPIB_TRY(alloc(ctx, &ctx->w_u, 3 * (size_t)M3));
    HIPIB_TRY(alloc(ctx, &ctx->w_f, 3 * (size_t)M3));
    HIPIB_TRY(alloc(ctx, &ctx->w_g, 3 * (size_t)M3));
    HIPIB_TRY(alloc(ctx, &ctx->w_p, (size_t)M3));
    HIPIB_TRY(alloc(ctx, &ctx->w_b, (size_t)M3));
    HIPIB_TRY(alloc(ctx, &ctx->w_box, 3 * (size_t)ctx->n3));
    HIPIB_TRY(alloc(ctx, &ctx->w_fbox, 3 * (size_t)ctx->n3));
    return HIPIB_OK;
}

void walled_free(hipib_ctx* ctx) {
    if (ctx->img) (void)hipib_destroy(ctx->img);
    ctx->img = nullptr;
    double** bufs[] = {&ctx->w_u, &ctx->w_f, &ctx->w_g, &ctx->w_p, &ctx->w_b,
                       &ctx->w_box, &ctx->w_fbox, &ctx->w_Xh, &ctx->w_U, &ctx->w_ap, &ctx->w_ah};
    for (double** b : bufs) {
        (void)hipFree(*b);
        *b = nullptr;
    }
    ctx->w_nn = -1;
}

// the image context holds the nodes (no elements) for binning, spreading and
// interpolation on the image grid
hipib_status walled_set_nodes(hipib_ctx* ctx, const double* X_ref_host) {
    std::vector<double> half(3 * (size_t)ctx->nn);
    for (size_t t = 0; t < half.size(); ++t) half[t] = 0.5 * X_ref_host[t];
    HIPIB_TRY(hipib_set_mesh_elements(ctx->img, ctx->nn, ctx->nn ? half.data() : nullptr, 0, 8,
                                      nullptr, nullptr, nullptr));
    (void)hipFree(ctx->w_Xh);
    (void)hipFree(ctx->w_U);
    ctx->w_Xh = ctx->w_U = nullptr;
    HIPIB_TRY(alloc(ctx, &ctx->w_Xh, 3 * (size_t)ctx->nn));
    HIPIB_TRY(alloc(ctx, &ctx->w_U, 3 * (size_t)ctx->nn));
    ctx->w_nn = ctx->nn;
    return HIPIB_OK;
}

hipib_status walled_ns_step(hipib_ctx* ctx, const double* f, double* u, double* p) {
    hipib_ctx* img = ctx->img;
    img->stream = ctx->stream;
    const double rho = ctx->cfg.rho, dt = ctx->cfg.dt;
    int32_t cyc[4] = {0, 0, 0, 0};
    double rr[4] = {0, 0, 0, 0};
    HIPIB_TRY(extend(ctx, u, ctx->w_u, 3, W_VELOCITY));
    if (f) HIPIB_TRY(extend(ctx, f, ctx->w_f, 3, W_VELOCITY));
    else HIPIB_TRY(launch_zero(ctx, ctx->w_f, 3 * img->n3));
    HIPIB_TRY(extend(ctx, p, ctx->w_p, 1, W_EVEN));
    // g = (rho/dt) u - rho C_h(u) + f, C_h = C_{h/2} / 2; restricted (wall faces 0) and mirrored
    HIPIB_TRY(launch_rhs_build_coef(img, ctx->w_u, ctx->w_f, ctx->w_g, rho / dt, 0.5 * rho));
    HIPIB_TRY(restrict_box(ctx, ctx->w_g, ctx->w_box, 3, W_VELOCITY));
    HIPIB_TRY(extend(ctx, ctx->w_box, ctx->w_g, 3, W_VELOCITY));
    HIPIB_TRY(mg_solve(img, HIPIB_OP_HELMHOLTZ, 3, ctx->w_g, ctx->w_u, cyc, rr));
    HIPIB_TRY(restrict_box(ctx, ctx->w_u, ctx->w_box, 3, W_VELOCITY));
    HIPIB_TRY(extend(ctx, ctx->w_box, ctx->w_u, 3, W_VELOCITY));
    // b = 4 (-(rho/dt) D_h u*) = -2 (rho/dt) D_{h/2} u*: box part mirrored evenly
    HIPIB_TRY(launch_divergence_rhs_coef(img, ctx->w_u, ctx->w_b, 2.0 * (rho / dt)));
    HIPIB_TRY(restrict_box(ctx, ctx->w_b, ctx->w_box, 1, W_EVEN));
    HIPIB_TRY(extend(ctx, ctx->w_box, ctx->w_b, 1, W_EVEN));
    HIPIB_TRY(mg_remove_mean(img, ctx->w_b, 0));
    HIPIB_TRY(mg_solve(img, HIPIB_OP_POISSON, 1, ctx->w_b, ctx->w_p, cyc + 3, rr + 3));
    // u = u* - (dt/rho) G_h p, G_h = G_{h/2} / 2
    HIPIB_TRY(launch_project_coef(img, ctx->w_u, ctx->w_p, 0.5 * (dt / rho)));
    HIPIB_TRY(restrict_box(ctx, ctx->w_u, u, 3, W_VELOCITY));
    HIPIB_TRY(restrict_box(ctx, ctx->w_p, p, 1, W_EVEN));
    StepRecord rec;
    for (int t = 0; t < 4; ++t) {
        rec.cycles[t] = cyc[t];
        rec.relres[t] = rr[t];
    }
    ctx->recs.push_back(rec);
    return HIPIB_OK;
}

hipib_status walled_spread(hipib_ctx* ctx, const double* X, const double* F, double* f) {
    hipib_ctx* img = ctx->img;
    img->stream = ctx->stream;
    HIPIB_TRY(image_positions(ctx, X));
    HIPIB_TRY(launch_zero(ctx, ctx->w_f, 3 * img->n3));
    HIPIB_TRY(launch_spread(img, ctx->w_Xh, F, ctx->w_f));
    // f += (1/8) fold(image force): delta_h at X is 8 times delta_{h/2} at X/2
    return fold(ctx, ctx->w_f, f, 3, W_VELOCITY, 0.125, true);
}

hipib_status walled_interpolate(hipib_ctx* ctx, const double* X, const double* u, double* U) {
    hipib_ctx* img = ctx->img;
    img->stream = ctx->stream;
    HIPIB_TRY(image_positions(ctx, X));
    HIPIB_TRY(extend(ctx, u, ctx->w_u, 3, W_VELOCITY));
    return launch_interpolate(img, ctx->w_Xh, ctx->w_u, U, nullptr, 0.0);
}

hipib_status walled_ib_step(hipib_ctx* ctx, double* u, double* p, double* X, double pressure) {
    HIPIB_TRY(launch_fe_force(ctx, X, pressure, ctx->F));
    HIPIB_TRY(launch_zero(ctx, ctx->w_fbox, 3 * ctx->n3));
    HIPIB_TRY(walled_spread(ctx, X, ctx->F, ctx->w_fbox));
    HIPIB_TRY(walled_ns_step(ctx, ctx->w_fbox, u, p));
    HIPIB_TRY(sync_state(ctx));
    HIPIB_TRY(sync_state(ctx->img));
    HIPIB_TRY(position_status(ctx->img));
    if (ctx->st_host->numeric)
        return fail(HIPIB_E_NUMERIC, "non-positive Jacobian at a Gauss point (inverted element)");
    // U = J(X^n) u^{n+1} on the image grid (the bins of X^n / 2 are current), X += dt U
    HIPIB_TRY(extend(ctx, u, ctx->w_u, 3, W_VELOCITY));
    HIPIB_TRY(launch_interpolate(ctx->img, ctx->w_Xh, ctx->w_u, ctx->w_U, nullptr, 0.0));
    return scale(ctx, ctx->w_U, X, ctx->cfg.dt, 3 * (int64_t)ctx->nn, true);
}

// Reverse of walled_ib_step, given lam_u = dL/du^{n+1} (box) and lam_X =
// dL/dX^{n+1}: every mirror map contributes its transpose (extend -> fold,
// restrict -> pad), the periodic image-grid operators theirs (G^T = -D,
// D^T = -G, symmetric solves, C'(u)^T), spreading at X/2 the interpolation
// (S^T = J / h'^3), and the positions the factor 1/2 of X/2.  The adjoint
// solves start from the previous call's solutions (w_ap, w_ah; zero on the
// first call), as the periodic reverse step's do.  Image scratch: w_u, w_g,
// w_f (vectors), w_b (scalar); box scratch w_box, w_fbox.
hipib_status walled_adjoint_step(hipib_ctx* ctx, const double* u_n, const double* X_n,
                                 const double* u_np1, double pressure, double* lam_u, double* lam_X,
                                 double* dtheta) {
    hipib_ctx* img = ctx->img;
    img->stream = ctx->stream;
    HIPIB_TRY(adjoint_scratch(ctx));
    if (!ctx->w_ap || !ctx->w_ah) {   // first call: the solves' starts, zero
        if (!ctx->w_ap) HIPIB_TRY(alloc(ctx, &ctx->w_ap, (size_t)img->n3));
        if (!ctx->w_ah) HIPIB_TRY(alloc(ctx, &ctx->w_ah, 3 * (size_t)img->n3));
        HIPIB_TRY(launch_zero(ctx, ctx->w_ap, img->n3));
        HIPIB_TRY(launch_zero(ctx, ctx->w_ah, 3 * img->n3));
    }
    const double hp = img->h, hp3 = hp * hp * hp, rho = ctx->cfg.rho, dt = ctx->cfg.dt;
    const double a = rho / dt, b = 0.5 * rho, c = 0.5 * (dt / rho);
    const int64_t nn3 = 3 * (int64_t)ctx->nn, M3 = img->n3;
    HIPIB_TRY(image_positions(ctx, X_n));
    // X^{n+1} = X^n + dt J(X^n / 2) E u^{n+1}
    HIPIB_TRY(scale(ctx, lam_X, ctx->adj_sX, dt * hp3, nn3, false));      // sX = dt h'^3 lam_X'
    HIPIB_TRY(launch_zero(ctx, ctx->w_u, 3 * M3));
    if (ctx->nn > 0) HIPIB_TRY(launch_spread(img, ctx->w_Xh, ctx->adj_sX, ctx->w_u));   // J^T (dt lam_X')
    HIPIB_TRY(scale(ctx, lam_u, ctx->w_box, 1.0, 3 * ctx->n3, false));
    HIPIB_TRY(fold(ctx, ctx->w_u, ctx->w_box, 3, W_VELOCITY, 1.0, true));   // dL/du^{n+1}, box
    if (ctx->nn > 0) {
        HIPIB_TRY(extend(ctx, u_np1, ctx->w_g, 3, W_VELOCITY));
        HIPIB_TRY(launch_vjp_X(img, ctx->w_Xh, ctx->w_g, ctx->adj_sX, lam_X, 0.5 / (hp * hp3)));
    }
    // u^{n+1} = R(u_s - c G p), p = L^{-1} (mean-free) E_s R_s (-2a D u_s)
    HIPIB_TRY(pad(ctx, ctx->w_box, ctx->w_u, 3, W_VELOCITY));                // lam of image u^{n+1}
    HIPIB_TRY(launch_divergence_rhs_coef(img, ctx->w_u, ctx->w_b, -c));      // lam_p = c D lam
    HIPIB_TRY(mg_remove_mean(img, ctx->w_b, 0));
    HIPIB_TRY(mg_solve(img, HIPIB_OP_POISSON, 1, ctx->w_b, ctx->w_ap, nullptr, nullptr));
    HIPIB_TRY(mg_remove_mean(img, ctx->w_ap, 0));
    HIPIB_TRY(fold(ctx, ctx->w_ap, ctx->w_box, 1, W_EVEN, 1.0, false));
    HIPIB_TRY(pad(ctx, ctx->w_box, ctx->w_b, 1, W_EVEN));
    HIPIB_TRY(launch_project_coef(img, ctx->w_u, ctx->w_b, -2.0 * a));      // lam_us += 2a G lam_b
    // u_s = E R u*, u* = H^{-1} g_s, g_s = E R g
    HIPIB_TRY(fold(ctx, ctx->w_u, ctx->w_box, 3, W_VELOCITY, 1.0, false));
    HIPIB_TRY(pad(ctx, ctx->w_box, ctx->w_g, 3, W_VELOCITY));
    HIPIB_TRY(mg_solve(img, HIPIB_OP_HELMHOLTZ, 3, ctx->w_g, ctx->w_ah, nullptr, nullptr));
    HIPIB_TRY(fold(ctx, ctx->w_ah, ctx->w_box, 3, W_VELOCITY, 1.0, false));
    HIPIB_TRY(pad(ctx, ctx->w_box, ctx->w_u, 3, W_VELOCITY));               // lam_g (image)
    // g = a E u^n - b C'(E u^n) + E f
    HIPIB_TRY(extend(ctx, u_n, ctx->w_g, 3, W_VELOCITY));
    if (ctx->cfg.convection) HIPIB_TRY(launch_conv_vjp(img, ctx->w_g, ctx->w_u, ctx->w_f, a, -b));
    else HIPIB_TRY(scale(ctx, ctx->w_u, ctx->w_f, a, 3 * M3, false));
    HIPIB_TRY(fold(ctx, ctx->w_f, lam_u, 3, W_VELOCITY, 1.0, false));       // dL/du^n
    if (ctx->nn > 0) {
        // f = (1/8) E^T S(X/2) F
        HIPIB_TRY(fold(ctx, ctx->w_u, ctx->w_fbox, 3, W_VELOCITY, 1.0, false));   // dL/df (box)
        HIPIB_TRY(extend(ctx, ctx->w_fbox, ctx->w_g, 3, W_VELOCITY));
        HIPIB_TRY(launch_interpolate(img, ctx->w_Xh, ctx->w_g, ctx->adj_lamF, nullptr, 0.0));
        HIPIB_TRY(scale(ctx, ctx->adj_lamF, ctx->adj_lamF, 0.125 / hp3, nn3, false));
        HIPIB_TRY(launch_fe_force(ctx, X_n, pressure, ctx->F));
        HIPIB_TRY(launch_vjp_X(img, ctx->w_Xh, ctx->w_g, ctx->F, lam_X, 0.0625 / (hp * hp3)));
        HIPIB_TRY(adjoint_forces(ctx, X_n, pressure, ctx->adj_lamF, lam_X, dtheta));
    }
    HIPIB_TRY(sync_state(ctx));
    HIPIB_TRY(sync_state(ctx->img));
    HIPIB_TRY(position_status(ctx->img));
    if (ctx->st_host->numeric)
        return fail(HIPIB_E_NUMERIC, "non-positive Jacobian at a Gauss point (inverted element)");
    return HIPIB_OK;
}

// each component a cell-centred scalar: Poisson (Neumann, mirrored evenly,
// right-hand side times 4 for the image grid's unit-coefficient operator) or
// Helmholtz (Dirichlet, mirrored oddly; the image context's viscosity is mu/4)
hipib_status walled_solve(hipib_ctx* ctx, int op, int ncomp, const double* b, double* x,
                          int32_t* cycles, double* relres) {
    hipib_ctx* img = ctx->img;
    img->stream = ctx->stream;
    const bool poisson = op == HIPIB_OP_POISSON;
    const int mode = poisson ? W_EVEN : W_ODD;
    HIPIB_TRY(extend(ctx, b, ctx->w_g, ncomp, mode));
    HIPIB_TRY(extend(ctx, x, ctx->w_u, ncomp, mode));
    if (poisson) HIPIB_TRY(scale(ctx, ctx->w_g, ctx->w_g, 4.0, ncomp * img->n3, false));
    HIPIB_TRY(mg_solve(img, op, ncomp, ctx->w_g, ctx->w_u, cycles, relres));
    return restrict_box(ctx, ctx->w_u, x, ncomp, mode);
}

}  // namespace hipib
