/*
 * lbora.c -- plain FP64 CPU oracle for the fluctuating lattice Boltzmann
 * update (D3Q19 and D2Q9) of Duenweg, Schiller & Ladd, "Statistical
 * mechanics of the fluctuating lattice Boltzmann equation" (arXiv:0707.1581).
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load this library.
 * It shares no code, header, table or constant with the GPU library: its
 * tables are built here from the velocity sets and the polynomials of the
 * paper's Tables I and II, its Philox generator is written here from the published
 * definition, and every step is the plain definition:
 *
 *   - moments m_k = sum_i e_ki n_i with dense q x q loops (Eq. modes with
 *     the unscaled basis of Table II or Table I, Sec. III),
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

#define QMAX 19

/* ------------------------------------------------------------------ */
/* Lattices.  Two velocity sets of the paper (Sec. III): D3Q19 with the   */
/* basis of Table II and D2Q9 with the basis of Table I.  Both have three */
/* speeds (0, 1, sqrt 2) and c_s^2 = 1/3.  Velocity order: rest; the axis */
/* directions as (+x, -x, +y, -y[, +z, -z]); then the diagonals in        */
/* opposite pairs.  The opposite of i is i+1 (odd i) or i-1 (even i > 0). */
/* ------------------------------------------------------------------ */
enum { LAT_D3Q19 = 0, LAT_D2Q9 = 1, NLAT = 2 };

/* Mode classes (Sec. IV: each mode relaxes at its own rate, subject to   */
/* symmetry): conserved (mass, momentum), bulk stress, shear stress, odd  */
/* (third-order) and even (fourth-order) kinetic modes.                   */
enum { MODE_CONSERVED = 0, MODE_BULK, MODE_SHEAR, MODE_ODD, MODE_EVEN };

typedef struct {
  int q, d;
  int vel[QMAX][3];
  double a[QMAX];        /* a^{c_i}                    */
  double e[QMAX][QMAX];  /* e_ki, [k][i]               */
  double w[QMAX];        /* w_k = sum_i a_i e_ki^2     */
  int cls[QMAX];         /* mode class of k            */
} lattice;

static const int VEL_D3Q19[19][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static const int VEL_D2Q9[9][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};

/* Weights by speed.  D3Q19: a^0 = 1/3, a^1 = 1/18, a^sqrt2 = 1/36 (Sec. II).
 * D2Q9: the paper gives no numbers but states that normalisation and the
 * isotropy conditions sigma_2 = c_s^2, sigma_4 = sigma_2^2, kappa_4 = 0
 * (Eqs. equilcond2-4) fix the weights of a three-speed model.  With one
 * rest, four axis and four diagonal velocities: sum_i a_i c_ix^4 =
 * 2 a1 + 4 a2 must equal 3 sigma_4 = 3 * 4 a2 (kappa_4 = 0), so a1 = 4 a2;
 * sigma_4 = 4 a2 = (2 a1 + 4 a2)^2 = (12 a2)^2 gives a2 = 1/36, a1 = 1/9,
 * and a0 = 1 - 4 a1 - 4 a2 = 4/9, with c_s^2 = 2 a1 + 4 a2 = 1/3. */
static double weight_of(int lat, const int c[3]) {
  int c2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
  if (lat == LAT_D3Q19) return c2 == 0 ? 1.0 / 3.0 : (c2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
  return c2 == 0 ? 4.0 / 9.0 : (c2 == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
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

/* Table I: the D2Q9 basis polynomial e_k(c). */
static double table1_poly(int k, const int c[3]) {
  double cx = c[0], cy = c[1];
  double c2 = cx * cx + cy * cy;
  switch (k) {
    case 0: return 1.0;
    case 1: return cx;
    case 2: return cy;
    case 3: return 3.0 * c2 - 2.0;
    case 4: return 2.0 * cx * cx - c2;
    case 5: return cx * cy;
    case 6: return (3.0 * c2 - 4.0) * cx;
    case 7: return (3.0 * c2 - 4.0) * cy;
    case 8: return 9.0 * c2 * c2 - 15.0 * c2 + 2.0;
  }
  return 0.0;
}

/* Mode classes in table order: D3Q19 k = 0..3 conserved, 4 bulk, 5..9
 * shear, 10..15 odd, 16..18 even; D2Q9 k = 0..2 conserved, 3 bulk, 4..5
 * shear, 6..7 odd, 8 even (Sec. III: d + 1 conserved modes, one bulk mode,
 * d(d+1)/2 - 1 shear modes, then the kinetic modes). */
static int mode_class(int lat, int k) {
  if (lat == LAT_D3Q19) {
    if (k <= 3) return MODE_CONSERVED;
    if (k == 4) return MODE_BULK;
    if (k <= 9) return MODE_SHEAR;
    return k <= 15 ? MODE_ODD : MODE_EVEN;
  }
  if (k <= 2) return MODE_CONSERVED;
  if (k == 3) return MODE_BULK;
  if (k <= 5) return MODE_SHEAR;
  return k <= 7 ? MODE_ODD : MODE_EVEN;
}

static lattice LATS[NLAT];
static int tables_ready = 0;

static void build_tables(void) {
  if (tables_ready) return;
  for (int l = 0; l < NLAT; ++l) {
    lattice* L = &LATS[l];
    L->q = (l == LAT_D3Q19) ? 19 : 9;
    L->d = (l == LAT_D3Q19) ? 3 : 2;
    for (int i = 0; i < L->q; ++i) {
      for (int c = 0; c < 3; ++c) L->vel[i][c] = (l == LAT_D3Q19) ? VEL_D3Q19[i][c] : VEL_D2Q9[i][c];
      L->a[i] = weight_of(l, L->vel[i]);
    }
    for (int k = 0; k < L->q; ++k) {
      double s = 0.0;
      for (int i = 0; i < L->q; ++i) {
        L->e[k][i] = (l == LAT_D3Q19) ? table2_poly(k, L->vel[i]) : table1_poly(k, L->vel[i]);
        s += L->a[i] * L->e[k][i] * L->e[k][i];
      }
      L->w[k] = s; /* the "length" of basis vector k, Sec. III */
      L->cls[k] = mode_class(l, k);
    }
  }
  tables_ready = 1;
}

static const lattice* lattice_of(int32_t lat) {
  build_tables();
  return (lat >= 0 && lat < NLAT) ? &LATS[lat] : NULL;
}

/* Exported for the table pins: returns q and fills c[q][3], a[q], e[q][q]
 * ([k][i]) and w[q]; -1 for an unknown lattice. */
int32_t ora_tables(int32_t lat, int32_t* c, double* a, double* e, double* w) {
  const lattice* L = lattice_of(lat);
  if (!L) return -1;
  const int q = L->q;
  for (int i = 0; i < q; ++i) {
    for (int d = 0; d < 3; ++d) c[3 * i + d] = L->vel[i][d];
    a[i] = L->a[i];
  }
  for (int k = 0; k < q; ++k) {
    w[k] = L->w[k];
    for (int i = 0; i < q; ++i) e[q * k + i] = L->e[k][i];
  }
  return q;
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
/* Parameters and the per-mode rates (Sec. IV: every non-conserved mode  */
/* relaxes at a rate of its own, equal within a symmetry class): bulk,   */
/* shear, odd and even kinetic rates.                                    */
/* ------------------------------------------------------------------ */
typedef struct {
  int64_t nx, ny, nz;
  double rho0;
  double kT;
  double gamma_bulk, gamma_shear, gamma_odd, gamma_even;
  uint64_t seed;
  int32_t thermal_modes; /* 0: all non-conserved modes; 1: stress modes only */
  int32_t lattice;       /* LAT_D3Q19 or LAT_D2Q9 (then nz = 1)             */
} ora_params;

static double mode_gamma(const ora_params* p, int cls) {
  switch (cls) {
    case MODE_CONSERVED: return 1.0;
    case MODE_BULK: return p->gamma_bulk;
    case MODE_SHEAR: return p->gamma_shear;
    case MODE_ODD: return p->gamma_odd;
    default: return p->gamma_even;
  }
}

static int mode_thermalised(const ora_params* p, int cls) {
  if (cls == MODE_CONSERVED) return 0;
  if (cls == MODE_BULK || cls == MODE_SHEAR) return 1;
  return p->thermal_modes == 0;
}

/* A usable parameter set: known lattice, positive sizes, nz = 1 in 2D. */
static const lattice* params_lattice(const ora_params* p) {
  const lattice* L = lattice_of(p->lattice);
  if (!L || p->nx < 1 || p->ny < 1 || p->nz < 1) return NULL;
  if (L->d == 2 && p->nz != 1) return NULL;
  return L;
}

/* Eq. (derived_equil_distrib) with sigma_2 = c_s^2 = 1/3; u has three
 * components, of which a 2D lattice uses the first two. */
int ora_equilibrium(int32_t lat, double rho, const double u[3], double* neq) {
  const lattice* L = lattice_of(lat);
  if (!L) return -1;
  const double cs2 = 1.0 / 3.0;
  double uu = 0.0;
  for (int c = 0; c < L->d; ++c) uu += u[c] * u[c];
  for (int i = 0; i < L->q; ++i) {
    double uc = 0.0;
    for (int c = 0; c < L->d; ++c) uc += u[c] * L->vel[i][c];
    neq[i] = rho * L->a[i] * (1.0 + uc / cs2 + uc * uc / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
  }
  return 0;
}

/* One collision at one site, in place.  Returns 0, -1 if rho <= 0 or rho
 * is not finite (the Gaussian model needs positive local mass), -2 for
 * unusable parameters.
 *
 * Noise: the q - d - 1 non-conserved modes take, in table order, the
 * normals of stream 0 of (seed, site, t): normal s goes to mode d + 1 + s. */
int ora_collide_site(const ora_params* p, double* n, uint32_t site, uint64_t t) {
  const lattice* L = params_lattice(p);
  if (!L) return -2;
  const int q = L->q, d = L->d;
  double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < q; ++i) {
    rho += n[i];
    for (int c = 0; c < d; ++c) j[c] += n[i] * L->vel[i][c];
  }
  if (!(rho > 0.0) || !isfinite(rho)) return -1;
  double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
  double neq[QMAX];
  ora_equilibrium(p->lattice, rho, u, neq);

  double m[QMAX], meq[QMAX], ms[QMAX];
  for (int k = 0; k < q; ++k) {
    double s = 0.0, se = 0.0;
    for (int i = 0; i < q; ++i) {
      s += L->e[k][i] * n[i];
      se += L->e[k][i] * neq[i];
    }
    m[k] = s;
    meq[k] = se;
  }

  const double mu = 3.0 * p->kT; /* mu = kT / c_s^2 in lattice units */
  const int first = d + 1;      /* first non-conserved mode */
  double r[QMAX + 1] = {0};
  if (p->kT > 0.0) ora_normals(p->seed, site, t, 0, q - first, r);

  for (int k = 0; k < q; ++k) {
    const int cls = L->cls[k];
    if (cls == MODE_CONSERVED) {
      ms[k] = m[k];
      continue;
    }
    double g = mode_gamma(p, cls);
    double mk = meq[k] + g * (m[k] - meq[k]);
    if (p->kT > 0.0 && mode_thermalised(p, cls)) {
      /* noise on mode k: sqrt(mu rho w_k (1 - gamma_k^2)) r, local rho */
      mk += sqrt(mu * rho * L->w[k] * (1.0 - g * g)) * r[k - first];
    }
    ms[k] = mk;
  }

  for (int i = 0; i < q; ++i) {
    double s = 0.0;
    for (int k = 0; k < q; ++k) s += L->e[k][i] * ms[k] / L->w[k];
    n[i] = L->a[i] * s;
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
 * sites with rho <= 0 (those sites stream their pre-collision values), or
 * -1 for unusable parameters. */
int64_t ora_step(const ora_params* p, const double* n_in, double* n_out, uint64_t t) {
  const lattice* L = params_lattice(p);
  if (!L) return -1;
  const int q = L->q;
  const int64_t nx = p->nx, ny = p->ny, nz = p->nz;
  const int64_t N = nx * ny * nz;
  int64_t bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
  for (int64_t z = 0; z < nz; ++z) {
    for (int64_t y = 0; y < ny; ++y) {
      for (int64_t x = 0; x < nx; ++x) {
        int64_t s = x + nx * (y + ny * z);
        double n[QMAX];
        for (int i = 0; i < q; ++i) n[i] = n_in[i * N + s];
        if (ora_collide_site(p, n, (uint32_t)s, t) != 0) bad += 1;
        for (int i = 0; i < q; ++i) {
          int64_t xd = wrap(x + L->vel[i][0], nx);
          int64_t yd = wrap(y + L->vel[i][1], ny);
          int64_t zd = wrap(z + L->vel[i][2], nz);
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
  const lattice* L = params_lattice(p);
  if (!L) return -1;
  const int64_t N = p->nx * p->ny * p->nz;
  int64_t bad = 0;
  for (int64_t s = 0; s < nsteps; ++s) {
    bad += ora_step(p, n, tmp, t0 + (uint64_t)s);
    memcpy(n, tmp, sizeof(double) * (size_t)(L->q * N));
  }
  return bad;
}

/* Initial states.  kind 0: rest, n_i = a_i rho0.  kind 1: thermal, every
 * normalised mode (conserved ones included) an independent unit Gaussian,
 * n_i = a_i rho0 + sqrt(mu rho0 a_i) sum_k ehat_ki z_k with
 * ehat_ki = sqrt(a_i / w_k) e_ki (Eqs. xdef, x_s, evectors_orthonormal);
 * normals from stream 1, normal k -> mode k.  kind 2: n_i = n_i^eq(rho, u)
 * from fields[1 + d][N] = (rho, ux, uy[, uz]). */
int ora_init(const ora_params* p, int32_t kind, const double* fields, double* n) {
  const lattice* L = params_lattice(p);
  if (!L) return -1;
  const int q = L->q, d = L->d;
  const int64_t N = p->nx * p->ny * p->nz;
  double mu = 3.0 * p->kT;
  if (kind == 2 && fields == NULL) return -1;
  if (kind < 0 || kind > 2) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < N; ++s) {
    double v[QMAX];
    if (kind == 0) {
      for (int i = 0; i < q; ++i) v[i] = L->a[i] * p->rho0;
    } else if (kind == 1) {
      double z[QMAX + 1];
      ora_normals(p->seed, (uint32_t)s, 0, 1, q, z);
      for (int i = 0; i < q; ++i) {
        double x = 0.0;
        for (int k = 0; k < q; ++k) x += sqrt(L->a[i] / L->w[k]) * L->e[k][i] * z[k];
        v[i] = L->a[i] * p->rho0 + sqrt(mu * p->rho0 * L->a[i]) * x;
      }
    } else {
      double u[3] = {0.0, 0.0, 0.0};
      for (int c = 0; c < d; ++c) u[c] = fields[(c + 1) * N + s];
      ora_equilibrium(p->lattice, fields[s], u, v);
    }
    for (int i = 0; i < q; ++i) n[i * N + s] = v[i];
  }
  return 0;
}

/* rho and j per site (Eqs. defrho, defj): out[1 + d][N]. */
int ora_moments(const ora_params* p, const double* n, double* out) {
  const lattice* L = params_lattice(p);
  if (!L) return -1;
  const int q = L->q, d = L->d;
  const int64_t N = p->nx * p->ny * p->nz;
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < N; ++s) {
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < q; ++i) {
      rho += n[i * N + s];
      for (int c = 0; c < d; ++c) j[c] += n[i * N + s] * L->vel[i][c];
    }
    out[s] = rho;
    for (int c = 0; c < d; ++c) out[(c + 1) * N + s] = j[c];
  }
  return 0;
}

/* Unscaled modes of the deviation from rest, m_k = sum_i e_ki (n_i - a_i rho0),
 * out[q][N] (k = 0 gives rho - rho0; for k >= 1 the rest part vanishes). */
int ora_modes(const ora_params* p, const double* n, double* out) {
  const lattice* L = params_lattice(p);
  if (!L) return -1;
  const int q = L->q;
  const int64_t N = p->nx * p->ny * p->nz;
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < N; ++s) {
    for (int k = 0; k < q; ++k) {
      double acc = 0.0;
      for (int i = 0; i < q; ++i) acc += L->e[k][i] * (n[i * N + s] - L->a[i] * p->rho0);
      out[k * N + s] = acc;
    }
  }
  return 0;
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
