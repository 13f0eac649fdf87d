/*
 * Plain, slow, FP64 CPU oracle of the voxel-parallel fitting hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the bench's CPU
 * baseline leg do.  It shares no code, header, table or helper with the HIP
 * library: every piece below is written out again from its definition.
 *
 * What it follows (paper = Chan et al., "GACELLE: GPU-accelerated tools for
 * model parameter estimation and image reconstruction", 2025):
 *   - whole-volume objective, paper §2.2.1 Eq. 2, with the optional weights
 *     of Eq. 1 and the regularised form of §2.4 Eq. 4;
 *   - gradient-moment optimisers Adam / SGDM / RMSProp and the three
 *     stopping criteria, paper §2.2.1 (Adam as defined by Kingma & Ba 2014);
 *   - total-variation regulariser R = |grad theta|, paper §2.4 Eq. 5 (grid);
 *   - Metropolis-Hastings with Gaussian likelihood, normal proposal with
 *     per-parameter step, burn-in ratio and thinning interval, pooled
 *     posterior mean / std, paper §2.2.2;
 *   - the mono-exponential model, paper §2.3.1 Eq. 3, and the other models of
 *     the registry (defined in the model section below);
 *   - Philox4x32-10 (Salmon et al., SC'11) and the Box-Muller transform
 *     (Box & Muller 1958) for the counter-based random streams that make
 *     CPU and GPU chains identical (paper §2.2.2, last paragraph).
 *
 * Readings of points the paper leaves open are stated where they are used.
 *
 * Parity unpinned: nothing here.  Every function has a pin in the CPU tests
 * (closed forms, library routines, brute force, analytic posteriors).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

enum { ORC_MONOEXP_T2S = 0, ORC_MONOEXP_R2S = 1, ORC_GRE3 = 2, ORC_DWI2 = 3, ORC_LINEAR3 = 4 };

/* ------------------------------------------------------------------------
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, §3 "Philox").
 * One round: two 32x32->64 products of words 0 and 2 with the fixed
 * multipliers; the outputs are permuted and the high halves are XORed with
 * the other two words and the round key.  The two key words are advanced by
 * the Weyl constants (golden ratio and sqrt(3)-1, as 32-bit fractions)
 * between rounds.
 * ------------------------------------------------------------------------ */
static void philox_round(uint32_t x[4], const uint32_t k[2]) {
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x[1] ^ k[0];
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x[3] ^ k[1];
    uint32_t y3 = lo0;
    x[0] = y0; x[1] = y1; x[2] = y2; x[3] = y3;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k[0] += 0x9E3779B9u; k[1] += 0xBB67AE85u; }
        philox_round(x, k);
    }
    out[0] = x[0]; out[1] = x[1]; out[2] = x[2]; out[3] = x[3];
}

/* Batch form for the tests: ctr[n][4] -> out[n][4] under one 64-bit seed
 * (key word 0 = low half, key word 1 = high half). */
void orc_philox_batch(uint64_t seed, const uint32_t *ctr, int64_t n, uint32_t *out) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int64_t i = 0; i < n; ++i) orc_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

/* Uniform on the open interval (0,1) from the top 23 bits of a word:
 * u = (floor(w / 2^9) + 1/2) / 2^23 = (2k+1) / 2^24 with k < 2^23, an odd
 * integer of at most 24 bits over a power of two: exact in binary32 and
 * binary64, so both precisions see the same number. */
double orc_uniform(uint32_t w) { return ((double)(w >> 9) + 0.5) / 8388608.0; }

/* Box-Muller: two independent standard normals from two uniforms. */
void orc_box_muller(double u1, double u2, double *z0, double *z1) {
    double r = sqrt(-2.0 * log(u1));
    *z0 = r * cos(2.0 * ORC_PI * u2);
    *z1 = r * sin(2.0 * ORC_PI * u2);
}

/* Draws of one MH step (voxel v of the job, chain c, iteration t).
 * Counter = (v, c | purpose << 16, t, block), key = seed.  Words are taken
 * in order across blocks; word pairs (2i, 2i+1) give normals 2i and 2i+1 by
 * Box-Muller; the word after the last pair gives the acceptance uniform. */
void orc_mh_draws(uint64_t seed, uint32_t v, uint32_t c, uint32_t t, int P,
                  double *z, double *u_acc) {
    int npairs = (P + 1) / 2;
    int nwords = 2 * npairs + 1;
    int nblk = (nwords + 3) / 4;
    uint32_t w[16];
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int b = 0; b < nblk; ++b) {
        uint32_t ctr[4] = {v, c | (0u << 16), t, (uint32_t)b};
        orc_philox4x32_10(ctr, key, w + 4 * b);
    }
    for (int i = 0; i < npairs; ++i) {
        double z0, z1;
        orc_box_muller(orc_uniform(w[2 * i]), orc_uniform(w[2 * i + 1]), &z0, &z1);
        if (2 * i < P) z[2 * i] = z0;
        if (2 * i + 1 < P) z[2 * i + 1] = z1;
    }
    *u_acc = orc_uniform(w[nwords - 1]);
}

/* Uniform initial state in the box: purpose 1, iteration 0; word p of the
 * consecutive blocks gives parameter p. */
void orc_init_uniform(uint64_t seed, uint32_t v, uint32_t c, int P,
                      const double *lb, const double *ub, double *theta) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int p = 0; p < P; ++p) {
        uint32_t ctr[4] = {v, c | (1u << 16), 0u, (uint32_t)(p / 4)};
        uint32_t w[4];
        orc_philox4x32_10(ctr, key, w);
        theta[p] = lb[p] + (ub[p] - lb[p]) * orc_uniform(w[p % 4]);
    }
}

/* ------------------------------------------------------------------------
 * Forward models.  Units: echo times in ms, T2* in ms, R2* in 1/s,
 * frequency shifts in Hz (phase 2*pi*df*TE*1e-3), b in s/mm^2 and
 * diffusivities in um^2/ms (b*D*1e-3 is dimensionless).
 *
 *  monoexp_t2s : s = S0 exp(-TE/T2*)                 (Eq. 3 in T2* form)
 *  monoexp_r2s : s = S0 exp(-TE*1e-3*R2*)            (Eq. 3)
 *  gre3        : s = sum_k A_k exp(-TE/T2*_k) exp(i 2 pi df_k TE 1e-3)
 *                three-pool complex multi-echo GRE of the T2*-based myelin
 *                water imaging family the paper supports (§2.1)
 *  dwi2        : s = f exp(-b 1e-3 Da (g.n)^2) + (1-f) exp(-b 1e-3 De),
 *                n = (sin th cos ph, sin th sin ph, cos th): stick + ball
 *  linear3     : s = sum_k A_k exp(-TE/tau_k), tau = (10, 30, 80) ms
 * Complex output: real parts of all echoes first, then imaginary parts.
 * ------------------------------------------------------------------------ */
typedef struct {
    int model, P, M, Meff;
    const double *te, *bval, *bvec;
} orc_model;

static int model_nparams(int model) {
    switch (model) {
        case ORC_MONOEXP_T2S: case ORC_MONOEXP_R2S: return 2;
        case ORC_GRE3: return 9;
        case ORC_DWI2: return 5;
        case ORC_LINEAR3: return 3;
    }
    return -1;
}

static int make_model(orc_model *m, int model, int M, const double *te,
                      const double *bval, const double *bvec) {
    m->model = model; m->M = M; m->te = te; m->bval = bval; m->bvec = bvec;
    m->P = model_nparams(model);
    if (m->P < 0) return -1;
    m->Meff = (model == ORC_GRE3) ? 2 * M : M;
    return 0;
}

static const double LIN3_TAU[3] = {10.0, 30.0, 80.0};

static void forward(const orc_model *m, const double *th, double *s) {
    int M = m->M;
    switch (m->model) {
    case ORC_MONOEXP_T2S:
        for (int j = 0; j < M; ++j) s[j] = th[0] * exp(-m->te[j] / th[1]);
        break;
    case ORC_MONOEXP_R2S:
        for (int j = 0; j < M; ++j) s[j] = th[0] * exp(-m->te[j] * 1e-3 * th[1]);
        break;
    case ORC_LINEAR3:
        for (int j = 0; j < M; ++j) {
            double a = 0.0;
            for (int k = 0; k < 3; ++k) a += th[k] * exp(-m->te[j] / LIN3_TAU[k]);
            s[j] = a;
        }
        break;
    case ORC_GRE3:
        for (int j = 0; j < M; ++j) {
            double re = 0.0, im = 0.0;
            for (int k = 0; k < 3; ++k) {
                double mag = th[k] * exp(-m->te[j] / th[3 + k]);
                double ph = 2.0 * ORC_PI * th[6 + k] * m->te[j] * 1e-3;
                re += mag * cos(ph);
                im += mag * sin(ph);
            }
            s[j] = re;
            s[M + j] = im;
        }
        break;
    case ORC_DWI2: {
        double n0 = sin(th[3]) * cos(th[4]), n1 = sin(th[3]) * sin(th[4]), n2 = cos(th[3]);
        for (int j = 0; j < M; ++j) {
            const double *g = m->bvec + 3 * j;
            double x = g[0] * n0 + g[1] * n1 + g[2] * n2;
            double b = m->bval[j] * 1e-3;
            s[j] = th[0] * exp(-b * th[1] * x * x) + (1.0 - th[0]) * exp(-b * th[2]);
        }
        break;
    }
    }
}

/* Analytic Jacobian J[j*P + p] = d s_j / d theta_p (derivatives of the
 * closed forms above). */
static void jacobian(const orc_model *m, const double *th, double *J) {
    int M = m->M, P = m->P;
    switch (m->model) {
    case ORC_MONOEXP_T2S:
        for (int j = 0; j < M; ++j) {
            double E = exp(-m->te[j] / th[1]);
            J[j * P + 0] = E;
            J[j * P + 1] = th[0] * E * m->te[j] / (th[1] * th[1]);
        }
        break;
    case ORC_MONOEXP_R2S:
        for (int j = 0; j < M; ++j) {
            double E = exp(-m->te[j] * 1e-3 * th[1]);
            J[j * P + 0] = E;
            J[j * P + 1] = -th[0] * E * m->te[j] * 1e-3;
        }
        break;
    case ORC_LINEAR3:
        for (int j = 0; j < M; ++j)
            for (int k = 0; k < 3; ++k) J[j * P + k] = exp(-m->te[j] / LIN3_TAU[k]);
        break;
    case ORC_GRE3:
        for (int j = 0; j < M; ++j) {
            double te = m->te[j];
            for (int k = 0; k < 3; ++k) {
                double E = exp(-te / th[3 + k]);
                double w = 2.0 * ORC_PI * te * 1e-3;
                double c = cos(w * th[6 + k]), sn = sin(w * th[6 + k]);
                double dT = th[k] * E * te / (th[3 + k] * th[3 + k]);
                /* real rows */
                J[j * P + k] = E * c;
                J[j * P + 3 + k] = dT * c;
                J[j * P + 6 + k] = -th[k] * E * w * sn;
                /* imaginary rows */
                J[(M + j) * P + k] = E * sn;
                J[(M + j) * P + 3 + k] = dT * sn;
                J[(M + j) * P + 6 + k] = th[k] * E * w * c;
            }
        }
        break;
    case ORC_DWI2: {
        double st = sin(th[3]), ct = cos(th[3]), sp = sin(th[4]), cp = cos(th[4]);
        double n0 = st * cp, n1 = st * sp, n2 = ct;
        double dt0 = ct * cp, dt1 = ct * sp, dt2 = -st;   /* dn/dtheta */
        double dp0 = -st * sp, dp1 = st * cp;             /* dn/dphi   */
        for (int j = 0; j < M; ++j) {
            const double *g = m->bvec + 3 * j;
            double x = g[0] * n0 + g[1] * n1 + g[2] * n2;
            double b = m->bval[j] * 1e-3;
            double Ea = exp(-b * th[1] * x * x), Ee = exp(-b * th[2]);
            double dx = -2.0 * th[0] * b * th[1] * x * Ea;   /* d s / d x */
            J[j * P + 0] = Ea - Ee;
            J[j * P + 1] = -th[0] * b * x * x * Ea;
            J[j * P + 2] = -(1.0 - th[0]) * b * Ee;
            J[j * P + 3] = dx * (g[0] * dt0 + g[1] * dt1 + g[2] * dt2);
            J[j * P + 4] = dx * (g[0] * dp0 + g[1] * dp1);
        }
        break;
    }
    }
}

int orc_nparams(int model) { return model_nparams(model); }

/* Forward of n voxels: theta[P][n] -> s[Meff][n]. */
int orc_forward(int model, int M, const double *te, const double *bval, const double *bvec,
                const double *theta, int64_t n, double *s) {
    orc_model m;
    if (make_model(&m, model, M, te, bval, bvec)) return -1;
    double th[16];
    double *sv = (double *)malloc(sizeof(double) * m.Meff);
    for (int64_t i = 0; i < n; ++i) {
        for (int p = 0; p < m.P; ++p) th[p] = theta[p * n + i];
        forward(&m, th, sv);
        for (int j = 0; j < m.Meff; ++j) s[j * n + i] = sv[j];
    }
    free(sv);
    return 0;
}

/* Jacobian of n voxels: J[n][Meff][P]. */
int orc_jacobian(int model, int M, const double *te, const double *bval, const double *bvec,
                 const double *theta, int64_t n, double *J) {
    orc_model m;
    if (make_model(&m, model, M, te, bval, bvec)) return -1;
    double th[16];
    for (int64_t i = 0; i < n; ++i) {
        for (int p = 0; p < m.P; ++p) th[p] = theta[p * n + i];
        jacobian(&m, th, J + i * (int64_t)m.Meff * m.P);
    }
    return 0;
}

/* Vector-Jacobian product: dtheta[P][n] = J^T ds for every voxel. */
int orc_vjp(int model, int M, const double *te, const double *bval, const double *bvec,
            const double *theta, int64_t n, const double *ds, double *dtheta) {
    orc_model m;
    if (make_model(&m, model, M, te, bval, bvec)) return -1;
    double th[16], *J = (double *)malloc(sizeof(double) * m.Meff * m.P);
    for (int64_t i = 0; i < n; ++i) {
        for (int p = 0; p < m.P; ++p) th[p] = theta[p * n + i];
        jacobian(&m, th, J);
        for (int p = 0; p < m.P; ++p) {
            double a = 0.0;
            for (int j = 0; j < m.Meff; ++j) a += J[j * m.P + p] * ds[j * n + i];
            dtheta[p * n + i] = a;
        }
    }
    free(J);
    return 0;
}

/* ------------------------------------------------------------------------
 * Data term of the whole-volume objective (Eq. 2 with weights, Eq. 1):
 *   D(theta) = 1/(N*Meff) * sum_{v in mask} sum_j |w_v (y_vj - s_vj)|^p,
 * p = 2 (L2, squared as in Eq. 1) or p = 1 (L1; a complex measurement counts
 * as its real and imaginary parts).  N = number of masked voxels.
 * Returns per-voxel terms (already scaled by 1/(N*Meff)) and dD/dtheta.
 * The L1 subgradient takes sign(0) = 0.
 * ------------------------------------------------------------------------ */
static double data_term(const orc_model *m, const double *th, const float *y, int64_t stride,
                        double w, int p, double scale, double *g, double *s, double *J) {
    forward(m, th, s);
    jacobian(m, th, J);
    double acc = 0.0;
    for (int q = 0; q < m->P; ++q) g[q] = 0.0;
    for (int j = 0; j < m->Meff; ++j) {
        double r = (double)y[j * stride] - s[j];
        double dr; /* d term / d s_j */
        if (p == 2) {
            acc += w * w * r * r;
            dr = -2.0 * w * w * r;
        } else {
            acc += fabs(w * r);
            dr = -w * (r > 0 ? 1.0 : (r < 0 ? -1.0 : 0.0));
        }
        for (int q = 0; q < m->P; ++q) g[q] += dr * J[j * m->P + q];
    }
    for (int q = 0; q < m->P; ++q) g[q] *= scale;
    return acc * scale;
}

/* Per-voxel loss and gradient on compacted arrays (used by the VJP tests):
 * theta[P][n], y[Meff][n] (float), w[n] or NULL; the loss is scaled by
 * `scale` (the caller passes 1/(N*Meff) for the objective's normalisation). */
int orc_loss_grad(int model, int M, const double *te, const double *bval, const double *bvec,
                  const double *theta, const float *y, const float *w, int64_t n, int p,
                  double scale, double *loss, double *grad) {
    orc_model m;
    if (make_model(&m, model, M, te, bval, bvec)) return -1;
    double th[16], g[16];
    double *s = (double *)malloc(sizeof(double) * m.Meff);
    double *J = (double *)malloc(sizeof(double) * m.Meff * m.P);
    for (int64_t i = 0; i < n; ++i) {
        for (int q = 0; q < m.P; ++q) th[q] = theta[q * n + i];
        double wi = w ? (double)w[i] : 1.0;
        loss[i] = data_term(&m, th, y + i, n, wi, p, scale, g, s, J);
        for (int q = 0; q < m.P; ++q) grad[q * n + i] = g[q];
    }
    free(s); free(J);
    return 0;
}

/* ------------------------------------------------------------------------
 * Total variation on a grid (Eq. 5, R = |grad theta|), read as the
 * anisotropic L1 norm of forward differences along x, y (and z in 3D),
 * counting only pairs whose two voxels are both inside the mask:
 *   R(u) = sum_{pairs (a,b)} |u_b - u_a|.
 * Subgradient with sign(0) = 0.  u and dR are full grids [nz][ny][nx];
 * dR is accumulated (+=) with weight `scale`.
 * ------------------------------------------------------------------------ */
double orc_tv(int nx, int ny, int nz, const uint8_t *mask, const double *u, int dim,
              double scale, double *dR) {
    double R = 0.0;
    int64_t sx = 1, sy = nx, sz = (int64_t)nx * ny;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int64_t a = z * sz + y * sy + x * sx;
                if (!mask[a]) continue;
                int64_t nb[3];
                int ok[3] = {x + 1 < nx, y + 1 < ny, dim == 3 && z + 1 < nz};
                nb[0] = a + sx; nb[1] = a + sy; nb[2] = a + sz;
                for (int d = 0; d < 3; ++d) {
                    if (!ok[d] || !mask[nb[d]]) continue;
                    double diff = u[nb[d]] - u[a];
                    R += fabs(diff);
                    if (dR) {
                        double sg = diff > 0 ? 1.0 : (diff < 0 ? -1.0 : 0.0);
                        dR[nb[d]] += scale * sg;
                        dR[a] -= scale * sg;
                    }
                }
            }
    return R;
}

/* ------------------------------------------------------------------------
 * Isotropic reading of the grid TV of Eq. 5: per masked voxel a, the
 * Euclidean norm of its forward differences (only those whose neighbour is
 * in the mask, along x, y and, in 3D, z):
 *   R(u) = sum_a G_a,  G_a = sqrt(sum_d (u_{a+e_d} - u_a)^2).
 * Subgradient: dG_a/du_{a+e_d} = D_d / G_a, dG_a/du_a = -sum_d D_d / G_a,
 * and 0 when G_a = 0.  dR is accumulated (+=) with weight `scale`.
 * ------------------------------------------------------------------------ */
double orc_tv_iso(int nx, int ny, int nz, const uint8_t *mask, const double *u, int dim,
                  double scale, double *dR) {
    double R = 0.0;
    int64_t sx = 1, sy = nx, sz = (int64_t)nx * ny;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int64_t a = z * sz + y * sy + x * sx;
                if (!mask[a]) continue;
                int64_t nb[3] = {a + sx, a + sy, a + sz};
                int ok[3] = {x + 1 < nx, y + 1 < ny, dim == 3 && z + 1 < nz};
                double D[3] = {0.0, 0.0, 0.0};
                double ss = 0.0;
                for (int d = 0; d < 3; ++d) {
                    ok[d] = ok[d] && mask[nb[d]];
                    if (!ok[d]) continue;
                    D[d] = u[nb[d]] - u[a];
                    ss += D[d] * D[d];
                }
                double Ga = sqrt(ss);
                R += Ga;
                if (dR && Ga > 0.0)
                    for (int d = 0; d < 3; ++d) {
                        if (!ok[d]) continue;
                        dR[nb[d]] += scale * D[d] / Ga;
                        dR[a] -= scale * D[d] / Ga;
                    }
            }
    return R;
}

/* ------------------------------------------------------------------------
 * Graph (surface-mesh) TV, the vertex form of Eq. 5 in the surface-fitting
 * demonstration (§2.6.1): for each vertex i the sum over its mesh neighbours
 * N(i) of |u_i - u_j|, summed over all vertices,
 *   R(u) = sum_i sum_{j in N(i)} |u_i - u_j|
 * (a symmetric adjacency counts every edge from both ends).  The adjacency is
 * CSR over the n vertices: neighbours of i are col[rowptr[i] .. rowptr[i+1]).
 * Subgradient with sign(0) = 0, accumulated (+=) with weight `scale`.
 * ------------------------------------------------------------------------ */
double orc_tv_graph(int64_t n, const int64_t *rowptr, const int32_t *col, const double *u,
                    double scale, double *dR) {
    double R = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            int64_t j = col[k];
            double diff = u[i] - u[j];
            R += fabs(diff);
            if (dR) {
                double sg = diff > 0 ? 1.0 : (diff < 0 ? -1.0 : 0.0);
                dR[i] += scale * sg;
                dR[j] -= scale * sg;
            }
        }
    return R;
}

/* ------------------------------------------------------------------------
 * Prior regulariser of Eq. 6: R = sum_v |(theta_v - mu_v) / sigma_v| for one
 * parameter map, theta = lb + (ub - lb) u.  The subgradient with respect to
 * u is sign(theta - mu) (ub - lb) / sigma (sign(0) = 0), accumulated (+=)
 * with weight `scale`.  Arrays are over n voxels.
 * ------------------------------------------------------------------------ */
double orc_prior(int64_t n, const double *u, double lb, double ub, const double *mu,
                 const double *sigma, double scale, double *dR) {
    double R = 0.0;
    for (int64_t v = 0; v < n; ++v) {
        double th = lb + (ub - lb) * u[v];
        double r = (th - mu[v]) / sigma[v];
        R += fabs(r);
        if (dR) {
            double sg = r > 0 ? 1.0 : (r < 0 ? -1.0 : 0.0);
            dR[v] += scale * sg * (ub - lb) / sigma[v];
        }
    }
    return R;
}

/* ------------------------------------------------------------------------
 * askadam: whole-volume gradient fit (paper §2.2.1, Eq. 2 / Eq. 4).
 *
 * Readings: bounds are enforced by optimising normalised coordinates
 * u = (theta - lb)/(ub - lb), clamped to [0,1] after every update; the loss
 * is D(theta(u)) + lambda/N * sum_{q in TV set} R(u_q); the gradient is
 * dD/du = (ub - lb) * dD/dtheta plus lambda/N * dR/du.  Iteration t
 * (1-based) evaluates the loss and gradient at u_{t-1}, records L_t, updates
 * to u_t and then tests the stopping rules:
 *   reason 1: L_t < tol;
 *   reason 2: |OLS slope of (s, L_s) over the last W iterations| < conv,
 *             tested once t >= W (W = convergence window, > 1);
 *   reason 0: t == n_iter.
 * The output is the last iterate theta(u_t).
 * Optimisers (g = gradient):
 *   Adam    m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 *           u -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)
 *   SGDM    vel = mom * vel - lr * g; u += vel
 *   RMSProp v = rho v + (1-rho) g^2; u -= lr * g / (sqrt(v) + eps)
 * ------------------------------------------------------------------------ */
typedef struct {
    int optimizer;               /* 0 Adam, 1 SGDM, 2 RMSProp */
    double lr, beta1, beta2, eps, momentum, rho;
    int n_iter, loss_p;
    double lambda;
    uint32_t tv_mask;
    int tv_dim;
    double tol, conv_value;
    int conv_window;
} orc_fit_opts;

static double ols_slope(const double *L, int W, int t_last) {
    /* slope of L against iteration index over t_last-W+1 .. t_last */
    double mx = 0.0, my = 0.0;
    for (int i = 0; i < W; ++i) { mx += (double)(t_last - W + 1 + i); my += L[i]; }
    mx /= W; my /= W;
    double sxy = 0.0, sxx = 0.0;
    for (int i = 0; i < W; ++i) {
        double dx = (double)(t_last - W + 1 + i) - mx;
        sxy += dx * (L[i] - my);
        sxx += dx * dx;
    }
    return sxy / sxx;
}

/* Regularisers of the loss (§2.4): TV (Eq. 5) on the maps of tv_mask in one of
 * three forms, and the prior (Eq. 6) on the maps of prior_mask.  Both are
 * divided by the number N of masked voxels, like the data term:
 *   L = D + lambda / N sum_{q in TV} R_TV(u_q)
 *         + prior_lambda / N sum_{q in prior} sum_v |(theta_qv - mu_qv) / sigma_qv|. */
typedef struct {
    int tv_kind;                 /* 0 anisotropic grid, 1 isotropic grid, 2 graph */
    int64_t graph_n;             /* graph: vertices = masked voxels in grid order */
    const int64_t *graph_rowptr; /* [graph_n + 1] */
    const int32_t *graph_col;    /* compact vertex indices */
    double prior_lambda;
    uint32_t prior_mask;
    const double *prior_mu;      /* [P][grid] */
    const double *prior_sigma;   /* [P][grid] */
} orc_reg;

int orc_askadam_reg(int model, int M, const double *te, const double *bval, const double *bvec,
                    int nx, int ny, int nz, const uint8_t *mask, const float *y,
                    const float *w, const double *lb, const double *ub, const double *x0,
                    int optimizer, double lr, double beta1, double beta2, double eps,
                    double momentum, double rho, int n_iter, int loss_p, double lambda,
                    uint32_t tv_mask, int tv_dim, const orc_reg *reg, double tol,
                    double conv_value, int conv_window, double *out_maps, double *loss_hist,
                    int *iters_run, int *stop_reason, int n_threads);

int orc_askadam(int model, int M, const double *te, const double *bval, const double *bvec,
                int nx, int ny, int nz, const uint8_t *mask, const float *y /*[Meff][grid]*/,
                const float *w /*[grid] or NULL*/, const double *lb, const double *ub,
                const double *x0 /*[P][grid] or NULL -> midpoint*/,
                int optimizer, double lr, double beta1, double beta2, double eps,
                double momentum, double rho, int n_iter, int loss_p, double lambda,
                uint32_t tv_mask, int tv_dim, double tol, double conv_value, int conv_window,
                double *out_maps /*[P][grid]*/, double *loss_hist /*[n_iter]*/,
                int *iters_run, int *stop_reason, int n_threads) {
    return orc_askadam_reg(model, M, te, bval, bvec, nx, ny, nz, mask, y, w, lb, ub, x0,
                           optimizer, lr, beta1, beta2, eps, momentum, rho, n_iter, loss_p,
                           lambda, tv_mask, tv_dim, NULL, tol, conv_value, conv_window,
                           out_maps, loss_hist, iters_run, stop_reason, n_threads);
}

int orc_askadam_reg(int model, int M, const double *te, const double *bval, const double *bvec,
                    int nx, int ny, int nz, const uint8_t *mask, const float *y,
                    const float *w, const double *lb, const double *ub, const double *x0,
                    int optimizer, double lr, double beta1, double beta2, double eps,
                    double momentum, double rho, int n_iter, int loss_p, double lambda,
                    uint32_t tv_mask, int tv_dim, const orc_reg *reg, double tol,
                    double conv_value, int conv_window, double *out_maps, double *loss_hist,
                    int *iters_run, int *stop_reason, int n_threads) {
    orc_model m;
    if (make_model(&m, model, M, te, bval, bvec)) return -1;
    int P = m.P;
    int64_t G = (int64_t)nx * ny * nz;
    int64_t N = 0;
    for (int64_t a = 0; a < G; ++a) N += mask[a] ? 1 : 0;
    if (N == 0) return -2;
    double scale = 1.0 / ((double)N * m.Meff);
    double *u = (double *)calloc((size_t)P * G, sizeof(double));
    double *mm = (double *)calloc((size_t)P * G, sizeof(double));
    double *vv = (double *)calloc((size_t)P * G, sizeof(double));
    double *gr = (double *)calloc((size_t)P * G, sizeof(double));
    double *lv = (double *)calloc((size_t)G, sizeof(double));
    for (int p = 0; p < P; ++p)
        for (int64_t a = 0; a < G; ++a) {
            double x = x0 ? x0[p * G + a] : 0.5 * (lb[p] + ub[p]);
            u[p * G + a] = mask[a] ? (x - lb[p]) / (ub[p] - lb[p]) : 0.0;
        }
    const int tv_kind = reg ? reg->tv_kind : 0;
    /* graph TV and the prior work on the masked voxels in grid order */
    int64_t *c2g = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
    {
        int64_t k = 0;
        for (int64_t a = 0; a < G; ++a)
            if (mask[a]) c2g[k++] = a;
    }
    if (tv_kind == 2 && lambda != 0.0 && tv_mask && (!reg->graph_rowptr || reg->graph_n != N)) {
        free(u); free(mm); free(vv); free(gr); free(lv); free(c2g);
        return -3;
    }
    double *uc = (double *)malloc(sizeof(double) * (size_t)N);
    double *gc = (double *)malloc(sizeof(double) * (size_t)N);
    double *muc = (double *)malloc(sizeof(double) * (size_t)N);
    double *sgc = (double *)malloc(sizeof(double) * (size_t)N);
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
    int t;
    int reason = 0;
    for (t = 1; t <= n_iter; ++t) {
        /* data term and its gradient, voxel by voxel */
#pragma omp parallel
        {
            double th[16], g[16];
            double *s = (double *)malloc(sizeof(double) * m.Meff);
            double *J = (double *)malloc(sizeof(double) * m.Meff * P);
#pragma omp for schedule(static)
            for (int64_t a = 0; a < G; ++a) {
                if (!mask[a]) { lv[a] = 0.0; for (int p = 0; p < P; ++p) gr[p * G + a] = 0.0; continue; }
                for (int p = 0; p < P; ++p) th[p] = lb[p] + (ub[p] - lb[p]) * u[p * G + a];
                double wi = w ? (double)w[a] : 1.0;
                lv[a] = data_term(&m, th, y + a, G, wi, loss_p, scale, g, s, J);
                for (int p = 0; p < P; ++p) gr[p * G + a] = (ub[p] - lb[p]) * g[p];
            }
            free(s); free(J);
        }
        double L = 0.0;
        for (int64_t a = 0; a < G; ++a) L += lv[a];
        /* regularisers */
        if (lambda != 0.0) {
            for (int p = 0; p < P; ++p) {
                if (!((tv_mask >> p) & 1u)) continue;
                const double sc = lambda / (double)N;
                if (tv_kind == 0) {
                    L += sc * orc_tv(nx, ny, nz, mask, u + p * G, tv_dim, sc, gr + p * G);
                } else if (tv_kind == 1) {
                    L += sc * orc_tv_iso(nx, ny, nz, mask, u + p * G, tv_dim, sc, gr + p * G);
                } else {
                    for (int64_t k = 0; k < N; ++k) { uc[k] = u[p * G + c2g[k]]; gc[k] = 0.0; }
                    L += sc * orc_tv_graph(N, reg->graph_rowptr, reg->graph_col, uc, sc, gc);
                    for (int64_t k = 0; k < N; ++k) gr[p * G + c2g[k]] += gc[k];
                }
            }
        }
        if (reg && reg->prior_lambda != 0.0) {
            for (int p = 0; p < P; ++p) {
                if (!((reg->prior_mask >> p) & 1u)) continue;
                const double sc = reg->prior_lambda / (double)N;
                for (int64_t k = 0; k < N; ++k) {
                    uc[k] = u[p * G + c2g[k]];
                    muc[k] = reg->prior_mu[p * G + c2g[k]];
                    sgc[k] = reg->prior_sigma[p * G + c2g[k]];
                    gc[k] = 0.0;
                }
                L += sc * orc_prior(N, uc, lb[p], ub[p], muc, sgc, sc, gc);
                for (int64_t k = 0; k < N; ++k) gr[p * G + c2g[k]] += gc[k];
            }
        }
        loss_hist[t - 1] = L;
        /* update */
        double c1 = 1.0 / (1.0 - pow(beta1, t)), c2 = 1.0 / (1.0 - pow(beta2, t));
        for (int p = 0; p < P; ++p)
            for (int64_t a = 0; a < G; ++a) {
                if (!mask[a]) continue;
                int64_t k = p * G + a;
                double g = gr[k], un;
                if (optimizer == 0) {
                    mm[k] = beta1 * mm[k] + (1.0 - beta1) * g;
                    vv[k] = beta2 * vv[k] + (1.0 - beta2) * g * g;
                    un = u[k] - lr * (mm[k] * c1) / (sqrt(vv[k] * c2) + eps);
                } else if (optimizer == 1) {
                    mm[k] = momentum * mm[k] - lr * g;
                    un = u[k] + mm[k];
                } else {
                    vv[k] = rho * vv[k] + (1.0 - rho) * g * g;
                    un = u[k] - lr * g / (sqrt(vv[k]) + eps);
                }
                u[k] = un < 0.0 ? 0.0 : (un > 1.0 ? 1.0 : un);
            }
        /* stopping rules */
        if (L < tol) { reason = 1; break; }
        if (conv_window > 1 && t >= conv_window &&
            fabs(ols_slope(loss_hist + t - conv_window, conv_window, t)) < conv_value) {
            reason = 2; break;
        }
    }
    if (t > n_iter) t = n_iter;
    *iters_run = t;
    *stop_reason = reason;
    for (int p = 0; p < P; ++p)
        for (int64_t a = 0; a < G; ++a)
            out_maps[p * G + a] = mask[a] ? lb[p] + (ub[p] - lb[p]) * u[p * G + a] : 0.0;
    free(u); free(mm); free(vv); free(gr); free(lv);
    free(c2g); free(uc); free(gc); free(muc); free(sgc);
    return 0;
}

/* ------------------------------------------------------------------------
 * Metropolis-Hastings, one chain per (voxel, chain) pair (paper §2.2.2).
 *
 * Target: uniform prior on the box [lb, ub] times the Gaussian likelihood
 *   logL(theta) = -1/(2 sigma^2) * sum_j w_v^2 (y_vj - s_j(theta))^2.
 * Step t = 0..n_iter-1: z ~ N(0, I) and u ~ U(0,1) from the counter-based
 * stream; proposal theta' = theta + step .* z; outside the box -> reject;
 * otherwise accept iff log(u) < logL(theta') - logL(theta) (ties reject).
 * After step t the state is retained when t >= burnin and
 * (t - burnin + 1) is a multiple of thin; retained samples of all chains are
 * pooled, mean and (n-1) standard deviation are the plain two-pass
 * definitions.  `vidx[i]` is the voxel index used in the random counters
 * (the voxel's position in the job's compacted order), so a subset of a big
 * volume reproduces the big run's chains exactly.
 * x0[C][P][n] is the initial state of every chain.
 * ------------------------------------------------------------------------ */
static double log_lik(const orc_model *m, const double *th, const float *y, int64_t stride,
                      double w, double inv2s2, double *s) {
    forward(m, th, s);
    double sse = 0.0;
    for (int j = 0; j < m->Meff; ++j) {
        double r = (double)y[j * stride] - s[j];
        sse += r * r;
    }
    return -inv2s2 * w * w * sse;
}

int64_t orc_mh_nkeep(int n_iter, int burnin, int thin) {
    if (n_iter <= burnin || thin <= 0) return 0;
    return (n_iter - burnin) / thin;
}

int orc_mh(int model, int M, const double *te, const double *bval, const double *bvec,
           int64_t n, const float *y /*[Meff][n]*/, const float *w /*[n] or NULL*/,
           const uint32_t *vidx, const double *lb, const double *ub,
           const double *x0 /*[C][P][n]*/, const double *step, double sigma, uint64_t seed,
           int n_chains, int n_iter, int burnin, int thin,
           double *samples /*[C][K][P][n] or NULL*/, double *mean /*[P][n]*/,
           double *sd /*[P][n]*/, int32_t *accept /*[C][n]*/, double *final_state /*[C][P][n]*/,
           double *final_logl /*[C][n] or NULL*/, double *min_margin /*[n] or NULL*/,
           int n_threads) {
    orc_model m;
    if (make_model(&m, model, M, te, bval, bvec)) return -1;
    int P = m.P;
    int64_t K = orc_mh_nkeep(n_iter, burnin, thin);
    double inv2s2 = 1.0 / (2.0 * sigma * sigma);
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel
    {
        double th[16], thp[16], z[16];
        double *s = (double *)malloc(sizeof(double) * m.Meff);
        double *keep = (double *)malloc(sizeof(double) * (size_t)(n_chains * K + 1) * P);
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < n; ++i) {
            double wi = w ? (double)w[i] : 1.0;
            double marg = INFINITY;
            int64_t kk = 0;
            for (int c = 0; c < n_chains; ++c) {
                for (int p = 0; p < P; ++p) th[p] = x0[((int64_t)c * P + p) * n + i];
                double ll = log_lik(&m, th, y + i, n, wi, inv2s2, s);
                int32_t acc = 0;
                for (int t = 0; t < n_iter; ++t) {
                    double ua;
                    orc_mh_draws(seed, vidx[i], (uint32_t)c, (uint32_t)t, P, z, &ua);
                    int inb = 1;
                    for (int p = 0; p < P; ++p) {
                        thp[p] = th[p] + step[p] * z[p];
                        if (!(thp[p] >= lb[p] && thp[p] <= ub[p])) inb = 0;
                    }
                    if (inb) {
                        double llp = log_lik(&m, thp, y + i, n, wi, inv2s2, s);
                        double d = llp - ll, lu = log(ua);
                        if (fabs(lu - d) < marg) marg = fabs(lu - d);
                        if (lu < d) {
                            for (int p = 0; p < P; ++p) th[p] = thp[p];
                            ll = llp;
                            ++acc;
                        }
                    }
                    if (t >= burnin && (t - burnin + 1) % thin == 0) {
                        for (int p = 0; p < P; ++p) keep[kk * P + p] = th[p];
                        if (samples) {
                            int64_t k = (t - burnin + 1) / thin - 1;
                            for (int p = 0; p < P; ++p)
                                samples[(((int64_t)c * K + k) * P + p) * n + i] = th[p];
                        }
                        ++kk;
                    }
                }
                accept[(int64_t)c * n + i] = acc;
                for (int p = 0; p < P; ++p) final_state[((int64_t)c * P + p) * n + i] = th[p];
                if (final_logl) final_logl[(int64_t)c * n + i] = ll;
            }
            for (int p = 0; p < P; ++p) {
                double sum = 0.0;
                for (int64_t k = 0; k < kk; ++k) sum += keep[k * P + p];
                double mu = kk > 0 ? sum / (double)kk : NAN;
                double ss = 0.0;
                for (int64_t k = 0; k < kk; ++k) {
                    double d = keep[k * P + p] - mu;
                    ss += d * d;
                }
                mean[p * n + i] = mu;
                sd[p * n + i] = kk > 1 ? sqrt(ss / (double)(kk - 1)) : NAN;
            }
            if (min_margin) min_margin[i] = marg;
        }
        free(s); free(keep);
    }
    return 0;
}

/* Log-likelihood of given states (tests use it for single-step checks). */
int orc_logl(int model, int M, const double *te, const double *bval, const double *bvec,
             const double *theta /*[P][n]*/, const float *y, const float *w, int64_t n,
             double sigma, double *out) {
    orc_model m;
    if (make_model(&m, model, M, te, bval, bvec)) return -1;
    double th[16];
    double *s = (double *)malloc(sizeof(double) * m.Meff);
    for (int64_t i = 0; i < n; ++i) {
        for (int p = 0; p < m.P; ++p) th[p] = theta[p * n + i];
        out[i] = log_lik(&m, th, y + i, n, w ? (double)w[i] : 1.0,
                         1.0 / (2.0 * sigma * sigma), s);
    }
    free(s);
    return 0;
}

/* ------------------------------------------------------------------------
 * Affine-invariant ensemble sampler (paper §2.2.2; Goodman & Weare 2010).
 *
 * K walkers per voxel split into halves S0 = {0..K/2-1}, S1 = {K/2..K-1};
 * iteration t updates S0 against S1, then S1 against the updated S0 (the
 * parallel form of the stretch move).  For walker k of half h the counter
 * (v, k | 2 << 16, t, 0) gives word 0 -> partner j = (other half start) +
 * floor(u0 K/2), word 1 -> z = ((a-1) u1 + 1)^2 / a (density ~ 1/sqrt(z) on
 * [1/a, a]), word 2 -> acceptance uniform; Y = X_j + z (X_k - X_j); outside
 * the box -> reject; accept iff log u2 < (P-1) log z + logL(Y) - logL(X_k).
 * Walkers start uniformly in [x0 - r, x0 + r], r = 1 % of the box width
 * (x = x0 + r (2u - 1) with u = word p % 4 of counter (v, k | 1 << 16, 0,
 * p / 4)), clamped to the box; x0_mode 1 starts them uniformly in the box.
 * Retention and moments as for MH, with walkers in place of chains.
 * ------------------------------------------------------------------------ */
int orc_ensemble(int model, int M, const double *te, const double *bval, const double *bvec,
                 int64_t n, const float *y, const float *w, const uint32_t *vidx,
                 const double *lb, const double *ub, const double *x0 /*[P][n]*/, int x0_mode,
                 double sigma, uint64_t seed, int K, double a, int n_iter, int burnin, int thin,
                 double *samples /*[K][S][P][n] or NULL*/, double *mean, double *sd,
                 int32_t *accept /*[K][n]*/, double *final_state /*[P][K][n]*/, int n_threads) {
    orc_model m;
    if (make_model(&m, model, M, te, bval, bvec)) return -1;
    if (K < 4 || K % 2) return -2;
    int P = m.P, hp = K / 2;
    int64_t S = orc_mh_nkeep(n_iter, burnin, thin);
    double inv2s2 = 1.0 / (2.0 * sigma * sigma);
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel
    {
        double *X = (double *)malloc(sizeof(double) * K * P);
        double *lp = (double *)malloc(sizeof(double) * K);
        int32_t *acc = (int32_t *)malloc(sizeof(int32_t) * K);
        double *keep = (double *)malloc(sizeof(double) * ((size_t)K * S + 1) * P);
        double *s = (double *)malloc(sizeof(double) * m.Meff);
        double Y[16];
#pragma omp for schedule(dynamic, 4)
        for (int64_t i = 0; i < n; ++i) {
            uint32_t v = vidx[i];
            double wi = w ? (double)w[i] : 1.0;
            for (int k = 0; k < K; ++k) {
                if (x0_mode == 1) {
                    orc_init_uniform(seed, v, (uint32_t)k, P, lb, ub, X + k * P);
                } else {
                    for (int p = 0; p < P; ++p) {
                        uint32_t ctr[4] = {v, (uint32_t)k | (1u << 16), 0u, (uint32_t)(p / 4)}, o[4];
                        orc_philox4x32_10(ctr, key, o);
                        double r = 0.01 * (ub[p] - lb[p]);
                        double x = x0[p * n + i] + r * (2.0 * orc_uniform(o[p % 4]) - 1.0);
                        X[k * P + p] = x < lb[p] ? lb[p] : (x > ub[p] ? ub[p] : x);
                    }
                }
                lp[k] = log_lik(&m, X + k * P, y + i, n, wi, inv2s2, s);
                acc[k] = 0;
            }
            int64_t kk = 0;
            for (int t = 0; t < n_iter; ++t) {
                for (int h = 0; h < 2; ++h) {
                    for (int ii = 0; ii < hp; ++ii) {
                        int k = h * hp + ii;
                        uint32_t ctr[4] = {v, (uint32_t)k | (2u << 16), (uint32_t)t, 0u}, o[4];
                        orc_philox4x32_10(ctr, key, o);
                        int j = (1 - h) * hp +
                                (int)((((uint64_t)(o[0] >> 9) * 2u + 1u) * (uint64_t)hp) >> 24);
                        double zt = (a - 1.0) * orc_uniform(o[1]) + 1.0;
                        double z = zt * zt / a;
                        int inb = 1;
                        for (int p = 0; p < P; ++p) {
                            Y[p] = X[j * P + p] + z * (X[k * P + p] - X[j * P + p]);
                            if (!(Y[p] >= lb[p] && Y[p] <= ub[p])) inb = 0;
                        }
                        if (!inb) continue;
                        double lpY = log_lik(&m, Y, y + i, n, wi, inv2s2, s);
                        if (log(orc_uniform(o[2])) < (double)(P - 1) * log(z) + lpY - lp[k]) {
                            for (int p = 0; p < P; ++p) X[k * P + p] = Y[p];
                            lp[k] = lpY;
                            ++acc[k];
                        }
                    }
                }
                if (t >= burnin && (t - burnin + 1) % thin == 0) {
                    int64_t q = (t - burnin + 1) / thin - 1;
                    for (int k = 0; k < K; ++k) {
                        for (int p = 0; p < P; ++p) {
                            keep[(kk + k) * P + p] = X[k * P + p];
                            if (samples) samples[(((int64_t)k * S + q) * P + p) * n + i] = X[k * P + p];
                        }
                    }
                    kk += K;
                }
            }
            for (int k = 0; k < K; ++k) {
                accept[(int64_t)k * n + i] = acc[k];
                for (int p = 0; p < P; ++p) final_state[((int64_t)p * K + k) * n + i] = X[k * P + p];
            }
            for (int p = 0; p < P; ++p) {
                double sum = 0.0;
                for (int64_t q = 0; q < kk; ++q) sum += keep[q * P + p];
                double mu = kk > 0 ? sum / (double)kk : NAN;
                double ss = 0.0;
                for (int64_t q = 0; q < kk; ++q) { double d = keep[q * P + p] - mu; ss += d * d; }
                mean[p * n + i] = mu;
                sd[p * n + i] = kk > 1 ? sqrt(ss / (double)(kk - 1)) : NAN;
            }
        }
        free(X); free(lp); free(acc); free(keep); free(s);
    }
    return 0;
}
