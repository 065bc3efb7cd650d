/*
 * lbora.c -- plain FP64 CPU oracle for the fluctuating D3Q19 lattice
 * Boltzmann update of Duenweg, Schiller & Ladd, "Statistical mechanics of
 * the fluctuating lattice Boltzmann equation" (arXiv:0707.1581).
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load this library.
 * It shares no code, header, table or constant with the GPU library: its
 * tables are built here from the velocity set and the polynomials of the
 * paper's Table II, its Philox generator is written here from the published
 * definition, and every step is the plain definition:
 *
 *   - moments m_k = sum_i e_ki n_i with dense 19x19 loops (Eq. modes with
 *     the unscaled Table II basis, Sec. III),
 *   - equilibrium populations by Eq. (derived_equil_distrib) with
 *     sigma_2 = c_s^2 = 1/3, projected onto the same basis,
 *   - per-mode update m* = m^eq + gamma_k (m - m^eq) + sqrt(mu rho w_k
 *     (1 - gamma_k^2)) r_k  (Eqs. updaterule and FDT, Sec. IV, with the
 *     normalisation of Eqs. xdef and evectors_orthonormal),
 *   - back-transform n*_i = a_i sum_k e_ki m*_k / w_k (completeness of the
 *     orthonormal basis, Eq. orthogonality),
 *   - push streaming n_i(r + c_i, t + 1) = n*_i(r, t) on a periodic box
 *     (Eq. LBE), into a second buffer.
 *
 * Lattice units throughout: b = h = 1, c_s^2 = 1/3, mu = kT / c_s^2
 * (Sec. VI, choice of parameters).  IEEE double, no reassociation.
 *
 * Readings of points the paper leaves open (velocity order, random-number
 * mapping, which rho scales the noise, step and site keys) are documented
 * next to the code that takes them.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 19

/* ------------------------------------------------------------------ */
/* Velocity set and weights (Sec. II: D3Q19, a^0 = 1/3, a^1 = 1/18,     */
/* a^sqrt2 = 1/36).  Order: rest; +x -x +y -y +z -z; then the twelve    */
/* diagonals in opposite pairs.  The opposite of i is i+1 (odd i) or    */
/* i-1 (even i > 0).                                                    */
/* ------------------------------------------------------------------ */
static const int VEL[Q][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static double weight_of(const int c[3]) {
  int c2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
  if (c2 == 0) return 1.0 / 3.0;
  if (c2 == 1) return 1.0 / 18.0;
  return 1.0 / 36.0;
}

/* Table II: the D3Q19 basis polynomial e_k(c), with c in lattice units. */
static double table2_poly(int k, const int c[3]) {
  double cx = c[0], cy = c[1], cz = c[2];
  double c2 = cx * cx + cy * cy + cz * cz;
  switch (k) {
    case 0: return 1.0;
    case 1: return cx;
    case 2: return cy;
    case 3: return cz;
    case 4: return c2 - 1.0;
    case 5: return 3.0 * cx * cx - c2;
    case 6: return cy * cy - cz * cz;
    case 7: return cx * cy;
    case 8: return cy * cz;
    case 9: return cz * cx;
    case 10: return (3.0 * c2 - 5.0) * cx;
    case 11: return (3.0 * c2 - 5.0) * cy;
    case 12: return (3.0 * c2 - 5.0) * cz;
    case 13: return (cy * cy - cz * cz) * cx;
    case 14: return (cz * cz - cx * cx) * cy;
    case 15: return (cx * cx - cy * cy) * cz;
    case 16: return 3.0 * c2 * c2 - 6.0 * c2 + 1.0;
    case 17: return (2.0 * c2 - 3.0) * (3.0 * cx * cx - c2);
    case 18: return (2.0 * c2 - 3.0) * (cy * cy - cz * cz);
  }
  return 0.0;
}

static double A[Q];      /* a_i                        */
static double E[Q][Q];   /* e_ki, [k][i]               */
static double W[Q];      /* w_k = sum_i a_i e_ki^2     */
static int tables_ready = 0;

static void build_tables(void) {
  if (tables_ready) return;
  for (int i = 0; i < Q; ++i) A[i] = weight_of(VEL[i]);
  for (int k = 0; k < Q; ++k) {
    double s = 0.0;
    for (int i = 0; i < Q; ++i) {
      E[k][i] = table2_poly(k, VEL[i]);
      s += A[i] * E[k][i] * E[k][i];
    }
    W[k] = s; /* the "length" of basis vector k, Sec. III */
  }
  tables_ready = 1;
}

/* Exported for the table pins: c[19][3], a[19], e[19][19] ([k][i]), w[19]. */
void ora_tables(int32_t* c, double* a, double* e, double* w) {
  build_tables();
  for (int i = 0; i < Q; ++i) {
    for (int d = 0; d < 3; ++d) c[3 * i + d] = VEL[i][d];
    a[i] = A[i];
  }
  for (int k = 0; k < Q; ++k) {
    w[k] = W[k];
    for (int i = 0; i < Q; ++i) e[Q * k + i] = E[k][i];
  }
}

/* ------------------------------------------------------------------ */
/* Random numbers.  The paper asks for independent unit Gaussians per   */
/* mode and step (Sec. IV) without naming a generator.  Reading:        */
/* Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11) keyed on the seed, */
/* counter (site, t mod 2^32, (stream << 16) | call, t >> 32), turned    */
/* into 24-bit uniforms and Box-Muller pairs as described below.        */
/* ------------------------------------------------------------------ */
static void philox_round(uint32_t x[4], uint32_t k0, uint32_t k1) {
  uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x[0];
  uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x[2];
  uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  uint32_t y0 = hi1 ^ x[1] ^ k0;
  uint32_t y2 = hi0 ^ x[3] ^ k1;
  x[0] = y0;
  x[1] = lo1;
  x[2] = y2;
  x[3] = lo0;
}

void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u; /* Weyl key increments of the published generator */
      k1 += 0xBB67AE85u;
    }
    philox_round(x, k0, k1);
  }
  for (int j = 0; j < 4; ++j) out[j] = x[j];
}

/* The word stream of one (seed, site, t, stream): word j is output word
 * j % 4 of Philox call j / 4, called with counter
 * (site, t mod 2^32, (stream << 16) | call, t >> 32) and key (seed mod 2^32,
 * seed >> 32).
 *
 * 24-bit chunks: every three consecutive words form one 96-bit big-endian
 * number that is cut into four 24-bit chunks, most significant first. */
void ora_uniform_chunks(uint64_t seed, uint32_t site, uint64_t t, uint32_t stream,
                        int32_t nchunks, uint32_t* out) {
  uint32_t words[64];
  int ntriples = (nchunks + 3) / 4;
  int nwords = 3 * ntriples;
  int ncalls = (nwords + 3) / 4;
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int call = 0; call < ncalls; ++call) {
    uint32_t ctr[4] = {site, (uint32_t)t, (stream << 16) | (uint32_t)call,
                       (uint32_t)(t >> 32)};
    ora_philox4x32_10(ctr, key, words + 4 * call);
  }
  for (int c = 0; c < nchunks; ++c) {
    const uint32_t* w = words + 3 * (c / 4);
    /* the 96-bit number w[0] w[1] w[2]; chunk c % 4 counted from the top */
    uint64_t hi64 = ((uint64_t)w[0] << 32) | w[1]; /* bits 95..32 */
    uint64_t lo64 = ((uint64_t)w[1] << 32) | w[2]; /* bits 63..0  */
    uint32_t v;
    switch (c % 4) {
      case 0: v = (uint32_t)(hi64 >> 40); break; /* bits 95..72 */
      case 1: v = (uint32_t)(hi64 >> 16); break; /* bits 71..48 */
      case 2: v = (uint32_t)(lo64 >> 24); break; /* bits 47..24 */
      default: v = (uint32_t)lo64; break;        /* bits 23..0  */
    }
    out[c] = v & 0xFFFFFFu;
  }
}

/* Box-Muller (Box & Muller 1958) on chunk pairs (2p, 2p+1):
 *   u1 = (chunk_2p + 1) 2^-24 in (0, 1],  u2 = chunk_2p+1 2^-24 in [0, 1),
 *   z_2p = sqrt(-2 ln u1) cos(2 pi u2),   z_2p+1 = sqrt(-2 ln u1) sin(2 pi u2).
 * Both uniforms are exact in binary32 and binary64. */
void ora_normals(uint64_t seed, uint32_t site, uint64_t t, uint32_t stream,
                 int32_t nnormals, double* z) {
  uint32_t ch[64];
  int npairs = (nnormals + 1) / 2;
  ora_uniform_chunks(seed, site, t, stream, 2 * npairs, ch);
  const double two_pi = 6.283185307179586476925286766559;
  for (int p = 0; p < npairs; ++p) {
    double u1 = ((double)ch[2 * p] + 1.0) * 0x1p-24;
    double u2 = (double)ch[2 * p + 1] * 0x1p-24;
    double r = sqrt(-2.0 * log(u1));
    z[2 * p] = r * cos(two_pi * u2);
    if (2 * p + 1 < nnormals) z[2 * p + 1] = r * sin(two_pi * u2);
  }
}

/* ------------------------------------------------------------------ */
/* Parameters and the per-mode rates (Sec. IV, "each mode ... its own   */
/* gamma_k"): k <= 3 conserved (gamma = 1); k = 4 bulk; k = 5..9 shear;  */
/* k = 10..15 odd (third-order) kinetic modes; k = 16..18 even           */
/* (fourth-order) kinetic modes.                                         */
/* ------------------------------------------------------------------ */
typedef struct {
  int64_t nx, ny, nz;
  double rho0;
  double kT;
  double gamma_bulk, gamma_shear, gamma_odd, gamma_even;
  uint64_t seed;
  int32_t thermal_modes; /* 0: all non-conserved modes; 1: stress modes only */
  int32_t reserved;
} ora_params;

static double mode_gamma(const ora_params* p, int k) {
  if (k <= 3) return 1.0;
  if (k == 4) return p->gamma_bulk;
  if (k <= 9) return p->gamma_shear;
  if (k <= 15) return p->gamma_odd;
  return p->gamma_even;
}

static int mode_thermalised(const ora_params* p, int k) {
  if (k <= 3) return 0;
  if (k <= 9) return 1;
  return p->thermal_modes == 0;
}

/* Eq. (derived_equil_distrib) with sigma_2 = c_s^2 = 1/3. */
void ora_equilibrium(double rho, const double u[3], double* neq) {
  build_tables();
  const double cs2 = 1.0 / 3.0;
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < Q; ++i) {
    double uc = u[0] * VEL[i][0] + u[1] * VEL[i][1] + u[2] * VEL[i][2];
    neq[i] = rho * A[i] * (1.0 + uc / cs2 + uc * uc / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
  }
}

/* One collision at one site, in place.  Returns 0, or -1 if rho <= 0 or
 * rho is not finite (the Gaussian model needs positive local mass). */
int ora_collide_site(const ora_params* p, double* n, uint32_t site, uint64_t t) {
  build_tables();
  double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < Q; ++i) {
    rho += n[i];
    for (int d = 0; d < 3; ++d) j[d] += n[i] * VEL[i][d];
  }
  if (!(rho > 0.0) || !isfinite(rho)) return -1;
  double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
  double neq[Q];
  ora_equilibrium(rho, u, neq);

  double m[Q], meq[Q], ms[Q];
  for (int k = 0; k < Q; ++k) {
    double s = 0.0, se = 0.0;
    for (int i = 0; i < Q; ++i) {
      s += E[k][i] * n[i];
      se += E[k][i] * neq[i];
    }
    m[k] = s;
    meq[k] = se;
  }

  double mu = 3.0 * p->kT; /* mu = kT / c_s^2 in lattice units */
  double r[16] = {0};
  if (p->kT > 0.0) ora_normals(p->seed, site, t, 0, 15, r);

  for (int k = 0; k < Q; ++k) {
    if (k <= 3) {
      ms[k] = m[k];
      continue;
    }
    double g = mode_gamma(p, k);
    double mk = meq[k] + g * (m[k] - meq[k]);
    if (p->kT > 0.0 && mode_thermalised(p, k)) {
      /* noise on mode k: sqrt(mu rho w_k (1 - gamma_k^2)) r, local rho */
      mk += sqrt(mu * rho * W[k] * (1.0 - g * g)) * r[k - 4];
    }
    ms[k] = mk;
  }

  for (int i = 0; i < Q; ++i) {
    double s = 0.0;
    for (int k = 0; k < Q; ++k) s += E[k][i] * ms[k] / W[k];
    n[i] = A[i] * s;
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Whole-lattice operations.  Layout of every lattice array: [q][z][y][x] */
/* with x fastest, absolute populations n_i.                              */
/* ------------------------------------------------------------------ */
static int64_t wrap(int64_t v, int64_t L) {
  v %= L;
  return v < 0 ? v + L : v;
}

/* One step: collide every site of n_in with noise keyed on t, push the
 * post-collision populations along c_i into n_out.  Returns the number of
 * sites with rho <= 0 (those sites stream their pre-collision values). */
int64_t ora_step(const ora_params* p, const double* n_in, double* n_out, uint64_t t) {
  build_tables();
  const int64_t nx = p->nx, ny = p->ny, nz = p->nz;
  const int64_t N = nx * ny * nz;
  int64_t bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
  for (int64_t z = 0; z < nz; ++z) {
    for (int64_t y = 0; y < ny; ++y) {
      for (int64_t x = 0; x < nx; ++x) {
        int64_t s = x + nx * (y + ny * z);
        double n[Q];
        for (int i = 0; i < Q; ++i) n[i] = n_in[i * N + s];
        if (ora_collide_site(p, n, (uint32_t)s, t) != 0) bad += 1;
        for (int i = 0; i < Q; ++i) {
          int64_t xd = wrap(x + VEL[i][0], nx);
          int64_t yd = wrap(y + VEL[i][1], ny);
          int64_t zd = wrap(z + VEL[i][2], nz);
          n_out[i * N + xd + nx * (yd + ny * zd)] = n[i];
        }
      }
    }
  }
  return bad;
}

/* nsteps steps starting at step count t0; n holds the state on entry and
 * on exit, tmp is a second buffer of the same size. */
int64_t ora_run(const ora_params* p, double* n, double* tmp, uint64_t t0, int64_t nsteps) {
  const int64_t N = p->nx * p->ny * p->nz;
  int64_t bad = 0;
  for (int64_t s = 0; s < nsteps; ++s) {
    bad += ora_step(p, n, tmp, t0 + (uint64_t)s);
    memcpy(n, tmp, sizeof(double) * (size_t)(Q * N));
  }
  return bad;
}

/* Initial states.  kind 0: rest, n_i = a_i rho0.  kind 1: thermal, every
 * normalised mode (conserved ones included) an independent unit Gaussian,
 * n_i = a_i rho0 + sqrt(mu rho0 a_i) sum_k ehat_ki z_k with
 * ehat_ki = sqrt(a_i / w_k) e_ki (Eqs. xdef, x_s, evectors_orthonormal);
 * normals from stream 1, normal k -> mode k.  kind 2: n_i = n_i^eq(rho, u)
 * from fields[4][N] = (rho, ux, uy, uz). */
int ora_init(const ora_params* p, int32_t kind, const double* fields, double* n) {
  build_tables();
  const int64_t N = p->nx * p->ny * p->nz;
  double mu = 3.0 * p->kT;
  if (kind == 2 && fields == NULL) return -1;
  if (kind < 0 || kind > 2) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < N; ++s) {
    double v[Q];
    if (kind == 0) {
      for (int i = 0; i < Q; ++i) v[i] = A[i] * p->rho0;
    } else if (kind == 1) {
      double z[Q + 1];
      ora_normals(p->seed, (uint32_t)s, 0, 1, Q, z);
      for (int i = 0; i < Q; ++i) {
        double x = 0.0;
        for (int k = 0; k < Q; ++k) x += sqrt(A[i] / W[k]) * E[k][i] * z[k];
        v[i] = A[i] * p->rho0 + sqrt(mu * p->rho0 * A[i]) * x;
      }
    } else {
      double u[3] = {fields[N + s], fields[2 * N + s], fields[3 * N + s]};
      ora_equilibrium(fields[s], u, v);
    }
    for (int i = 0; i < Q; ++i) n[i * N + s] = v[i];
  }
  return 0;
}

/* rho, jx, jy, jz per site (Eqs. defrho, defj): out[4][N]. */
void ora_moments(const ora_params* p, const double* n, double* out) {
  const int64_t N = p->nx * p->ny * p->nz;
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < N; ++s) {
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
      rho += n[i * N + s];
      for (int d = 0; d < 3; ++d) j[d] += n[i * N + s] * VEL[i][d];
    }
    out[s] = rho;
    for (int d = 0; d < 3; ++d) out[(d + 1) * N + s] = j[d];
  }
}

/* Unscaled modes of the deviation from rest, m_k = sum_i e_ki (n_i - a_i rho0),
 * out[19][N] (k = 0 gives rho - rho0; for k >= 1 the rest part vanishes). */
void ora_modes(const ora_params* p, const double* n, double* out) {
  build_tables();
  const int64_t N = p->nx * p->ny * p->nz;
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < N; ++s) {
    for (int k = 0; k < Q; ++k) {
      double acc = 0.0;
      for (int i = 0; i < Q; ++i) acc += E[k][i] * (n[i * N + s] - A[i] * p->rho0);
      out[k * N + s] = acc;
    }
  }
}

int32_t ora_num_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}

void ora_set_num_threads(int32_t n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
