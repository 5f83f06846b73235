/*
 * FP64 CPU oracle for the BPMF sampling hot path (Minh, "Alchemical Grid Dock
 * (AlGDock)", arXiv 1507.03703).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  It shares no code with
 * the GPU path and must never be linked into it; only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark load it.
 *
 * Every quantity is computed by direct definition in double precision:
 *   - grid interaction energy Psi_g = Psi_PBSA + Psi_vdW from one
 *     electrostatic and two van der Waals grids, each trilinearly interpolated
 *     and multiplied by a per-atom scale factor; the repulsive grid is stored
 *     as a quartic root and raised back to the fourth power after
 *     interpolation (Methodology, "Thermodynamic Cycle": grid interaction
 *     energy, electrostatic and van der Waals paragraphs);
 *   - the ligand's intramolecular bonded terms (GAFF functional forms: bonds,
 *     angles, proper torsions) that make up U_s(r_L) in the alchemical
 *     protocol equation (same section);
 *   - the flat-bottom harmonic centre-of-mass restraint, Eq. (binding_site);
 *   - Hamiltonian Monte Carlo with velocity-Verlet trial moves (Sampling);
 *   - Hamiltonian replica exchange with acceptance Eq. (repXacc), attempting
 *     neighbour pairs or all pairs up to a separation (Sampling);
 *   - the reduced potential u_k(x) = U_k(x) / (k_B T_k) evaluated per (k, n)
 *     for MBAR (Thermodynamic Cycle; Estimation).
 *
 * Readings taken where the paper is silent (listed in the design notes):
 *   - trilinear interpolation clamps to the edge outside the grid (value of
 *     the nearest face, zero normal gradient); on a cell face the cell chosen
 *     by floor() supplies the one-sided gradient;
 *   - per-state weights multiply each grid channel (w_kc), T_k per state;
 *   - random numbers come from Philox-4x32-10 (Salmon et al., SC'11) keyed
 *     by the run seed, with the counter (index, ligand<<16|replica, sweep,
 *     purpose|sub<<8); uniforms are (u32 + 1) 2^-32 in (0, 1]; normals by
 *     the Box-Muller transform;
 *   - units: A, fs, amu, kJ/mol, e, K; acceleration F/m * 1e-4 A/fs^2,
 *     kinetic energy m v^2 / 2 * 1e4 kJ/mol.
 *
 * Parity pins for each function live in the test suite (closed forms, exact
 * reproduction of multilinear fields, finite differences, invariants,
 * textbook reductions, known-answer vectors).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_R_GAS 8.314462618e-3 /* kJ/(mol K) */
#define ORA_MAXC 8

enum { ORA_P_MOMENTA = 1, ORA_P_ACCEPT = 2, ORA_P_EXCHANGE = 3 };

typedef struct {
  int nx, ny, nz, nc;
  double ox, oy, oz, h;
  const int* transform; /* per channel: 4 = stored quartic root, 0 = none */
  const float* nodes;   /* nz*ny*nx*nc, x fastest, channel innermost */
} ora_grid;

typedef struct {
  int n;
  const double* mass;  /* n */
  const double* scale; /* n*nc */
  int nb;
  const int* bij;       /* nb*2 */
  const double* bpar;   /* nb*2: K_r, r0 */
  int na;
  const int* aijk;      /* na*3, j = vertex */
  const double* apar;   /* na*2: K_theta, theta0 */
  int nt;
  const int* tijkl;     /* nt*4 */
  const double* tpar;   /* nt*3: V/2, n, gamma */
  double c0[3], d0, krest;
  /* intramolecular nonbonded and OBC generalised-Born / surface-area terms
     of the ligand (pair_on = 0: none); the excluded and 1-4 matrices are
     n*n with 1 marking the pair */
  int pair_on;
  const double* pq;     /* n charges (e) */
  const double* psig;   /* n LJ sigma (A) */
  const double* peps;   /* n LJ epsilon (kJ/mol) */
  const double* prho;   /* n intrinsic radii (A) */
  const double* pS;     /* n descreening scale factors */
  const unsigned char* pexcl;
  const unsigned char* p14;
  double lj14, el14, eps_in, eps_out, gamma, probe;
} ora_ligand;

/* ------------------------------------------------------------------------ */
/* Philox-4x32-10, from the definition in Salmon, Moraes, Dror and Shaw,     */
/* "Parallel random numbers: as easy as 1, 2, 3" (SC'11).                   */
/* ------------------------------------------------------------------------ */
void ora_philox(const uint32_t ctr_in[4], const uint32_t key_in[2],
                uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw(uint64_t seed, uint32_t index, int lig, int rep,
                 uint64_t sweep, uint32_t purpose, uint32_t out[4]) {
  uint32_t ctr[4] = {index, ((uint32_t)lig << 16) | (uint32_t)rep,
                     (uint32_t)sweep, purpose};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  ora_philox(ctr, key, out);
}

static double u01(uint32_t v) { return ((double)v + 1.0) * (1.0 / 4294967296.0); }

/* three standard normals for one atom (Box-Muller on two uniform pairs) */
static void normals3(const uint32_t o[4], double z[3]) {
  const double two_pi = 6.283185307179586476925286766559;
  double r1 = sqrt(-2.0 * log(u01(o[0])));
  z[0] = r1 * cos(two_pi * u01(o[1]));
  z[1] = r1 * sin(two_pi * u01(o[1]));
  double r2 = sqrt(-2.0 * log(u01(o[2])));
  z[2] = r2 * cos(two_pi * u01(o[3]));
}

/* ------------------------------------------------------------------------ */
/* Trilinear interpolation with clamp-to-edge outside the grid.             */
/* ------------------------------------------------------------------------ */
static void ora_axis(double x, double o, double h, int n, int* i, double* t,
                     double* live) {
  double u = (x - o) / h;
  if (isnan(u)) { *i = 0; *t = u; *live = 1.0; return; }
  double uc = u < -1.0 ? -1.0 : (u > (double)n ? (double)n : u);
  int ii = (int)floor(uc);
  if (ii < 0) ii = 0;
  if (ii > n - 2) ii = n - 2;
  double tt = uc - (double)ii;
  if (tt < 0.0) tt = 0.0;
  if (tt > 1.0) tt = 1.0;
  *i = ii;
  *t = tt;
  *live = (u >= 0.0 && u <= (double)(n - 1)) ? 1.0 : 0.0;
}

/* v[c] and dv[c][3] (gradient w.r.t. position) for every channel */
void ora_interp(const ora_grid* g, const double p[3], double* v, double* dv) {
  int ix, iy, iz;
  double tx, ty, tz, lx, ly, lz;
  ora_axis(p[0], g->ox, g->h, g->nx, &ix, &tx, &lx);
  ora_axis(p[1], g->oy, g->h, g->ny, &iy, &ty, &ly);
  ora_axis(p[2], g->oz, g->h, g->nz, &iz, &tz, &lz);
  for (int c = 0; c < g->nc; ++c) {
    v[c] = 0.0;
    dv[3 * c] = dv[3 * c + 1] = dv[3 * c + 2] = 0.0;
  }
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int cc = 0; cc < 2; ++cc) {
        double wx = a ? tx : 1.0 - tx, dwx = a ? 1.0 : -1.0;
        double wy = b ? ty : 1.0 - ty, dwy = b ? 1.0 : -1.0;
        double wz = cc ? tz : 1.0 - tz, dwz = cc ? 1.0 : -1.0;
        size_t node = ((size_t)(iz + cc) * g->ny + (size_t)(iy + b)) * g->nx +
                      (size_t)(ix + a);
        for (int c = 0; c < g->nc; ++c) {
          double gv = (double)g->nodes[node * g->nc + c];
          v[c] += wx * wy * wz * gv;
          dv[3 * c + 0] += dwx * wy * wz * gv;
          dv[3 * c + 1] += wx * dwy * wz * gv;
          dv[3 * c + 2] += wx * wy * dwz * gv;
        }
      }
  for (int c = 0; c < g->nc; ++c) {
    dv[3 * c + 0] *= lx / g->h;
    dv[3 * c + 1] *= ly / g->h;
    dv[3 * c + 2] *= lz / g->h;
  }
}

/* per-atom channel energy e[c] and gradient de[c][3] after the inverse
 * transform and the per-atom scale factor */
void ora_atom_grid(const ora_grid* g, const double p[3], const double* scale,
                   double* e, double* de) {
  double v[ORA_MAXC], dv[3 * ORA_MAXC];
  ora_interp(g, p, v, dv);
  for (int c = 0; c < g->nc; ++c) {
    if (g->transform[c] == 4) {
      double v2 = v[c] * v[c];
      e[c] = scale[c] * v2 * v2;
      double f = 4.0 * scale[c] * v2 * v[c];
      for (int d = 0; d < 3; ++d) de[3 * c + d] = f * dv[3 * c + d];
    } else {
      e[c] = scale[c] * v[c];
      for (int d = 0; d < 3; ++d) de[3 * c + d] = scale[c] * dv[3 * c + d];
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Bonded terms.                                                            */
/* ------------------------------------------------------------------------ */
static void sub3(const double* a, const double* b, double* o) {
  o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2];
}
static double dot3(const double* a, const double* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void cross3(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

/* dihedral angle, IUPAC sign convention, in (-pi, pi] */
double ora_dihedral(const double* xi, const double* xj, const double* xk,
                    const double* xl) {
  double b1[3], b2[3], b3[3], n1[3], n2[3];
  sub3(xj, xi, b1); sub3(xk, xj, b2); sub3(xl, xk, b3);
  cross3(b1, b2, n1); cross3(b2, b3, n2);
  double y = sqrt(dot3(b2, b2)) * dot3(b1, n2);
  return atan2(y, dot3(n1, n2));
}

double ora_angle(const double* xi, const double* xj, const double* xk) {
  double a[3], b[3], c[3];
  sub3(xi, xj, a); sub3(xk, xj, b); cross3(a, b, c);
  return atan2(sqrt(dot3(c, c)), dot3(a, b));
}

/* ------------------------------------------------------------------------ */
/* Intramolecular nonbonded and implicit-solvent energy of the ligand       */
/* (Thermodynamic Cycle: the ligand's force field with an OBC generalised-  */
/* Born / surface-area solvent), by direct definition:                      */
/*   E_LJ  = sum over pairs not excluded of 4 e_ij ((s_ij/r)^12 - (s_ij/r)^6) */
/*           with s_ij = (s_i + s_j)/2, e_ij = sqrt(e_i e_j), 1-4 pairs x lj14;*/
/*   E_C   = the same pairs' k_e q_i q_j / (eps_in r), 1-4 pairs x el14;     */
/*   E_GB  = -(k_e/2)(1/eps_in - 1/eps_out) sum_i sum_j q_i q_j / f_ij, all  */
/*           ordered pairs and i = j, f_ij = sqrt(r^2 + R_i R_j             */
/*           exp(-r^2/(4 R_i R_j))), f_ii = R_i;                            */
/*   Born radii (Onufriev, Bashford, Case 2004, OBC II): 1/R_i = 1/rt_i -    */
/*           tanh(psi - 0.8 psi^2 + 4.85 psi^3)/rho_i, psi = I_i rt_i,       */
/*           rt = rho - 0.09 A, I_i = sum_j of the Hawkins-Cramer-Truhlar    */
/*           descreening integral of |x|^-4/(4 pi) over the ball of radius   */
/*           S_j rt_j at distance r_ij, outside radius rt_i;                 */
/*   E_SA  = sum_i 4 pi gamma (rho_i + probe)^2 (rho_i / R_i)^6.             */
/* mag: the sum of the absolute values of the contributions.               */
/* ------------------------------------------------------------------------ */
#define ORA_KCOUL 1389.35457644382 /* kJ A / (mol e^2) */

/* (1/4pi) x integral of |y|^-4 over the ball of radius s at distance r > 0
   from the origin, outside the ball of radius a about the origin */
static double ora_hct(double r, double a, double s) {
  if (a >= r + s) return 0.0;
  double L = fabs(r - s) > a ? fabs(r - s) : a;
  double U = r + s;
  double l = 1.0 / L, u = 1.0 / U;
  double h = 0.5 * (l - u) + (s * s - r * r) * (l * l - u * u) / (8.0 * r) +
             log(u / l) / (4.0 * r);
  if (a < s - r) h += 1.0 / a - 1.0 / (s - r);
  return h;
}

static double ora_pair_energy(const ora_ligand* L, const double* x,
                              double* mag) {
  const int n = L->n;
  double e = 0.0, m = 0.0;
  /* LJ and Coulomb */
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      if (L->pexcl[(size_t)i * n + j]) continue;
      double d[3];
      sub3(x + 3 * i, x + 3 * j, d);
      double r = sqrt(dot3(d, d));
      double sg = 0.5 * (L->psig[i] + L->psig[j]);
      double ep = sqrt(L->peps[i] * L->peps[j]);
      double sr6 = pow(sg / r, 6.0);
      double lj = 4.0 * ep * (sr6 * sr6 - sr6);
      double cl = ORA_KCOUL * L->pq[i] * L->pq[j] / (L->eps_in * r);
      if (L->p14[(size_t)i * n + j]) {
        lj *= L->lj14;
        cl *= L->el14;
      }
      e += lj + cl;
      m += fabs(lj) + fabs(cl);
    }
  /* Born radii */
  double R[256];
  for (int i = 0; i < n; ++i) {
    double rt = L->prho[i] - 0.09, I = 0.0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      double d[3];
      sub3(x + 3 * i, x + 3 * j, d);
      I += ora_hct(sqrt(dot3(d, d)), rt, L->pS[j] * (L->prho[j] - 0.09));
    }
    double psi = I * rt;
    R[i] = 1.0 / (1.0 / rt -
                  tanh(psi - 0.8 * psi * psi + 4.85 * psi * psi * psi) /
                      L->prho[i]);
  }
  /* generalised Born and surface terms */
  double tau = 1.0 / L->eps_in - 1.0 / L->eps_out;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double f;
      if (i == j) {
        f = R[i];
      } else {
        double d[3];
        sub3(x + 3 * i, x + 3 * j, d);
        double r2 = dot3(d, d), RR = R[i] * R[j];
        f = sqrt(r2 + RR * exp(-r2 / (4.0 * RR)));
      }
      double gb = -0.5 * ORA_KCOUL * tau * L->pq[i] * L->pq[j] / f;
      e += gb;
      m += fabs(gb);
    }
  for (int i = 0; i < n; ++i) {
    double rp = L->prho[i] + L->probe, q = L->prho[i] / R[i];
    double sa = 4.0 * 3.14159265358979323846 * L->gamma * rp * rp * pow(q, 6.0);
    e += sa;
    m += fabs(sa);
  }
  if (mag) *mag = m;
  return e;
}

/* terms: [U_bond, U_angle, U_tors, U_restr, Psi_0 .. Psi_{nc-1}]; with the
 *        ligand's pair terms on, their energy is part of U_restr (the slot
 *        of the state-independent non-bonded energy)
 * mag:   same layout, sum over contributions of |contribution|
 * F:     -grad( U_bond + U_angle + U_tors + U_restr + sum_c w_c Psi_c ),
 *        may be NULL; the pair terms' part by central differences of their
 *        energy (step 1e-5 A) */
void ora_energy(const ora_grid* g, const ora_ligand* L, const double* w,
                const double* x, double* terms, double* mag, double* F) {
  const int n = L->n, nc = g->nc;
  const int nterm = 4 + nc;
  double tl[4 + ORA_MAXC], ml[4 + ORA_MAXC];
  for (int t = 0; t < nterm; ++t) tl[t] = ml[t] = 0.0;
  if (F) memset(F, 0, sizeof(double) * 3 * (size_t)n);

  /* bonds: K_r (r - r0)^2 */
  for (int b = 0; b < L->nb; ++b) {
    int i = L->bij[2 * b], j = L->bij[2 * b + 1];
    double K = L->bpar[2 * b], r0 = L->bpar[2 * b + 1];
    double d[3];
    sub3(x + 3 * i, x + 3 * j, d);
    double r = sqrt(dot3(d, d));
    double E = K * (r - r0) * (r - r0);
    tl[0] += E; ml[0] += fabs(E);
    if (F) {
      double f = -2.0 * K * (r - r0) / r;
      for (int a = 0; a < 3; ++a) {
        F[3 * i + a] += f * d[a];
        F[3 * j + a] -= f * d[a];
      }
    }
  }
  /* angles: K_theta (theta - theta0)^2 */
  for (int t = 0; t < L->na; ++t) {
    int i = L->aijk[3 * t], j = L->aijk[3 * t + 1], k = L->aijk[3 * t + 2];
    double K = L->apar[2 * t], th0 = L->apar[2 * t + 1];
    double a[3], b[3], c[3];
    sub3(x + 3 * i, x + 3 * j, a);
    sub3(x + 3 * k, x + 3 * j, b);
    cross3(a, b, c);
    double la = sqrt(dot3(a, a)), lb = sqrt(dot3(b, b));
    double s = sqrt(dot3(c, c)), co = dot3(a, b);
    double th = atan2(s, co);
    double E = K * (th - th0) * (th - th0);
    tl[1] += E; ml[1] += fabs(E);
    if (F) {
      double dE = 2.0 * K * (th - th0);
      double cth = co / (la * lb), sth = s / (la * lb);
      for (int q = 0; q < 3; ++q) {
        double ah = a[q] / la, bh = b[q] / lb;
        double dti = (cth * ah - bh) / (la * sth);
        double dtk = (cth * bh - ah) / (lb * sth);
        F[3 * i + q] -= dE * dti;
        F[3 * k + q] -= dE * dtk;
        F[3 * j + q] += dE * (dti + dtk);
      }
    }
  }
  /* proper torsions: (V/2) (1 + cos(n phi - gamma)) */
  for (int t = 0; t < L->nt; ++t) {
    int i = L->tijkl[4 * t], j = L->tijkl[4 * t + 1];
    int k = L->tijkl[4 * t + 2], l = L->tijkl[4 * t + 3];
    double V = L->tpar[3 * t], nn = L->tpar[3 * t + 1], gam = L->tpar[3 * t + 2];
    double b1[3], b2[3], b3[3], n1[3], n2[3];
    sub3(x + 3 * j, x + 3 * i, b1);
    sub3(x + 3 * k, x + 3 * j, b2);
    sub3(x + 3 * l, x + 3 * k, b3);
    cross3(b1, b2, n1);
    cross3(b2, b3, n2);
    double lb2 = sqrt(dot3(b2, b2));
    double phi = atan2(lb2 * dot3(b1, n2), dot3(n1, n2));
    double E = V * (1.0 + cos(nn * phi - gam));
    tl[2] += E; ml[2] += fabs(E);
    if (F) {
      double dE = -V * nn * sin(nn * phi - gam);
      double n1sq = dot3(n1, n1), n2sq = dot3(n2, n2);
      double p12 = dot3(b1, b2) / (lb2 * n1sq);
      double p23 = dot3(b2, b3) / (lb2 * n2sq);
      for (int q = 0; q < 3; ++q) {
        double gi = -lb2 / n1sq * n1[q];
        double gl = lb2 / n2sq * n2[q];
        double gj = -gi + p12 * n1[q] + p23 * n2[q];
        double gk = -gl - p12 * n1[q] - p23 * n2[q];
        F[3 * i + q] -= dE * gi;
        F[3 * j + q] -= dE * gj;
        F[3 * k + q] -= dE * gk;
        F[3 * l + q] -= dE * gl;
      }
    }
  }
  /* flat-bottom COM restraint, Eq. (binding_site) */
  {
    double M = 0.0, c[3] = {0, 0, 0};
    for (int i = 0; i < n; ++i) {
      M += L->mass[i];
      for (int a = 0; a < 3; ++a) c[a] += L->mass[i] * x[3 * i + a];
    }
    for (int a = 0; a < 3; ++a) c[a] = c[a] / M - L->c0[a];
    double d = sqrt(dot3(c, c));
    if (d > L->d0) {
      double E = 0.5 * L->krest * (d - L->d0) * (d - L->d0);
      tl[3] += E; ml[3] += fabs(E);
      if (F) {
        double f = -L->krest * (d - L->d0) / d;
        for (int i = 0; i < n; ++i)
          for (int a = 0; a < 3; ++a)
            F[3 * i + a] += f * (L->mass[i] / M) * c[a];
      }
    }
  }
  /* intramolecular nonbonded and implicit-solvent terms */
  if (L->pair_on) {
    double mp = 0.0;
    tl[3] += ora_pair_energy(L, x, &mp);
    ml[3] += mp;
    if (F) {
      const double h = 1e-5;
      double* y = (double*)malloc(sizeof(double) * 3 * (size_t)n);
      memcpy(y, x, sizeof(double) * 3 * (size_t)n);
      for (int q = 0; q < 3 * n; ++q) {
        const double x0 = y[q];
        y[q] = x0 + h;
        const double ep = ora_pair_energy(L, y, NULL);
        y[q] = x0 - h;
        const double em = ora_pair_energy(L, y, NULL);
        y[q] = x0;
        F[q] -= (ep - em) / (2.0 * h);
      }
      free(y);
    }
  }
  /* grid interaction energy */
  for (int i = 0; i < n; ++i) {
    double e[ORA_MAXC], de[3 * ORA_MAXC];
    ora_atom_grid(g, x + 3 * i, L->scale + (size_t)i * nc, e, de);
    for (int c = 0; c < nc; ++c) {
      tl[4 + c] += e[c];
      ml[4 + c] += fabs(e[c]);
      if (F)
        for (int a = 0; a < 3; ++a) F[3 * i + a] -= w[c] * de[3 * c + a];
    }
  }
  for (int t = 0; t < nterm; ++t) {
    if (terms) terms[t] = tl[t];
    if (mag) mag[t] = ml[t];
  }
}

/* total potential energy under grid weights w */
static double total_u(int nc, const double* terms, const double* w) {
  double U = terms[0] + terms[1] + terms[2] + terms[3];
  for (int c = 0; c < nc; ++c) U += w[c] * terms[4 + c];
  return U;
}

/* ------------------------------------------------------------------------ */
/* Velocity Verlet (Sampling: HMC trial moves).                             */
/* x, v in/out (n*3); returns H0 and H1 (kJ/mol) under weights w.           */
/* ------------------------------------------------------------------------ */
void ora_verlet(const ora_grid* g, const ora_ligand* L, const double* w,
                double dt, int nleap, double* x, double* v, double* H,
                double* terms_end) {
  const int n = L->n, nc = g->nc;
  double terms[4 + ORA_MAXC];
  double* F = (double*)malloc(sizeof(double) * 3 * (size_t)n);
  ora_energy(g, L, w, x, terms, NULL, F);
  double ke = 0.0;
  for (int i = 0; i < n; ++i)
    ke += 0.5 * L->mass[i] * dot3(v + 3 * i, v + 3 * i) * 1e4;
  H[0] = total_u(nc, terms, w) + ke;
  for (int s = 0; s < nleap; ++s) {
    for (int i = 0; i < n; ++i)
      for (int a = 0; a < 3; ++a) {
        v[3 * i + a] += 0.5 * dt * F[3 * i + a] / L->mass[i] * 1e-4;
        x[3 * i + a] += dt * v[3 * i + a];
      }
    ora_energy(g, L, w, x, terms, NULL, F);
    for (int i = 0; i < n; ++i)
      for (int a = 0; a < 3; ++a)
        v[3 * i + a] += 0.5 * dt * F[3 * i + a] / L->mass[i] * 1e-4;
  }
  ke = 0.0;
  for (int i = 0; i < n; ++i)
    ke += 0.5 * L->mass[i] * dot3(v + 3 * i, v + 3 * i) * 1e4;
  H[1] = total_u(nc, terms, w) + ke;
  if (terms_end)
    for (int t = 0; t < 4 + nc; ++t) terms_end[t] = terms[t];
  free(F);
}

/* Momenta for one replica: v_i ~ N(0, R T / m_i * 1e-4) per component. */
void ora_momenta(const ora_ligand* L, double T, uint64_t seed, int lig,
                 int rep, uint64_t sweep, double* v) {
  for (int i = 0; i < L->n; ++i) {
    uint32_t o[4];
    double z[3];
    draw(seed, (uint32_t)i, lig, rep, sweep, ORA_P_MOMENTA, o);
    normals3(o, z);
    double sd = sqrt(ORA_R_GAS * T / L->mass[i] * 1e-4);
    for (int a = 0; a < 3; ++a) v[3 * i + a] = sd * z[a];
  }
}

double ora_uniform(uint64_t seed, uint32_t index, int lig, int rep,
                   uint64_t sweep, uint32_t purpose) {
  uint32_t o[4];
  draw(seed, index, lig, rep, sweep, purpose, o);
  return u01(o[0]);
}

/* ------------------------------------------------------------------------ */
/* One HMC move for each of R replicas of one ligand.                       */
/* x: R*n*3 (in/out), comps: R*(1+nc) cached [U_bonded+U_restr, Psi_c]       */
/* (out, only for accepted replicas).  accepted/dH/lnu per replica (out).   */
/* ------------------------------------------------------------------------ */
void ora_hmc_sweep(const ora_grid* g, const ora_ligand* L, int K,
                   const double* T, const double* w, const double* dt,
                   uint64_t seed, int lig, int R, uint64_t sweep, int nleap,
                   double* x, const int* state_of_replica, double* comps,
                   int* accepted, double* dH_out, double* lnu_out) {
  const int n = L->n, nc = g->nc;
  (void)K;
#pragma omp parallel for schedule(dynamic, 1)
  for (int r = 0; r < R; ++r) {
    int k = state_of_replica[r];
    const double* wk = w + (size_t)k * nc;
    double beta = 1.0 / (ORA_R_GAS * T[k]);
    double* xr = x + (size_t)r * n * 3;
    double* xt = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    double* v = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    memcpy(xt, xr, sizeof(double) * 3 * (size_t)n);
    ora_momenta(L, T[k], seed, lig, r, sweep, v);
    double H[2], terms[4 + ORA_MAXC];
    ora_verlet(g, L, wk, dt[k], nleap, xt, v, H, terms);
    double dH = H[1] - H[0];
    double lnu = log(ora_uniform(seed, 0, lig, r, sweep, ORA_P_ACCEPT));
    int acc = isfinite(dH) && (lnu < -beta * dH);
    if (acc) {
      for (int q = 0; q < 3 * n; ++q)
        if (!isfinite(xt[q])) acc = 0;
    }
    if (acc) {
      memcpy(xr, xt, sizeof(double) * 3 * (size_t)n);
      double* cr = comps + (size_t)r * (1 + nc);
      cr[0] = terms[0] + terms[1] + terms[2] + terms[3];
      for (int c = 0; c < nc; ++c) cr[1 + c] = terms[4 + c];
    }
    if (accepted) accepted[r] = acc;
    if (dH_out) dH_out[r] = dH;
    if (lnu_out) lnu_out[r] = lnu;
    free(xt);
    free(v);
  }
}

/* ------------------------------------------------------------------------ */
/* Hamiltonian replica exchange, Eq. (repXacc).  Swaps state labels.         */
/* scheme 0: neighbour pairs, (0,1),(2,3).. on even sweeps, (1,2),.. on odd. */
/* scheme 1: pairs 1..max_sep apart, separation ascending, lower state       */
/*           ascending, applied sequentially (Gibbs sweep).                 */
/* sub: which of the exchange sweeps run back to back at one sweep counter  */
/*      this is (Equilibration and production: an iteration ends with 25);  */
/*      it fills the replica field of the uniforms' counter.                 */
/* ------------------------------------------------------------------------ */
static double state_energy(int nc, const double* w_k, const double* comp) {
  double E = comp[0];
  for (int c = 0; c < nc; ++c) E += w_k[c] * comp[1 + c];
  return E;
}

void ora_exchange(int K, int nc, const double* T, const double* w,
                  uint64_t seed, int lig, uint64_t sweep, int scheme,
                  int max_sep, int sub, const double* comps,
                  int* state_of_replica,
                  int* replica_of_state, int64_t* acc, int64_t* tries) {
  int dmax = scheme == 0 ? 1 : (max_sep < K - 1 ? max_sep : K - 1);
  for (int d = 1; d <= dmax; ++d) {
    int a0 = scheme == 0 ? (int)(sweep & 1u) : 0;
    int step = scheme == 0 ? 2 : 1;
    for (int a = a0; a + d < K; a += step) {
      int b = a + d;
      int ra = replica_of_state[a], rb = replica_of_state[b];
      const double* cx = comps + (size_t)ra * (1 + nc);
      const double* cy = comps + (size_t)rb * (1 + nc);
      double ba = 1.0 / (ORA_R_GAS * T[a]), bb = 1.0 / (ORA_R_GAS * T[b]);
      const double* wa = w + (size_t)a * nc;
      const double* wb = w + (size_t)b * nc;
      double delta = ba * (state_energy(nc, wa, cy) - state_energy(nc, wa, cx)) +
                     bb * (state_energy(nc, wb, cx) - state_energy(nc, wb, cy));
      uint32_t purpose = (uint32_t)ORA_P_EXCHANGE | ((uint32_t)d << 8);
      double lnu =
          log(ora_uniform(seed, (uint32_t)a, lig, sub, sweep, purpose));
      int ok = isfinite(delta) && (lnu < -delta);
      if (d == 1 && tries) tries[a] += 1;
      if (ok) {
        replica_of_state[a] = rb;
        replica_of_state[b] = ra;
        state_of_replica[ra] = b;
        state_of_replica[rb] = a;
        if (d == 1 && acc) acc[a] += 1;
      }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Reduced energies u_k(x_n) = U_k(x_n) / (R T_k), brute force per (k, n).  */
/* ------------------------------------------------------------------------ */
void ora_ukn(const ora_grid* g, const ora_ligand* L, int K, const double* T,
             const double* w, int64_t N, const double* xs, double* ukn) {
  const int n = L->n, nc = g->nc;
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = 0; k < K; ++k)
    for (int64_t s = 0; s < N; ++s) {
      double terms[4 + ORA_MAXC];
      ora_energy(g, L, w + (size_t)k * nc, xs + (size_t)s * n * 3, terms,
                 NULL, NULL);
      ukn[(size_t)k * N + s] = total_u(nc, terms, w + (size_t)k * nc) /
                               (ORA_R_GAS * T[k]);
    }
}

/* per-sample components [U_bonded + U_restr, Psi_c] (factorised form) */
void ora_components(const ora_grid* g, const ora_ligand* L, int64_t N,
                    const double* xs, double* comps, double* mags) {
  const int n = L->n, nc = g->nc;
  double w0[ORA_MAXC] = {0};
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < N; ++s) {
    double terms[4 + ORA_MAXC], mag[4 + ORA_MAXC];
    ora_energy(g, L, w0, xs + (size_t)s * n * 3, terms, mag, NULL);
    double* c = comps + (size_t)s * (1 + nc);
    c[0] = terms[0] + terms[1] + terms[2] + terms[3];
    for (int q = 0; q < nc; ++q) c[1 + q] = terms[4 + q];
    if (mags) {
      double* m = mags + (size_t)s * (1 + nc);
      m[0] = mag[0] + mag[1] + mag[2] + mag[3];
      for (int q = 0; q < nc; ++q) m[1 + q] = mag[4 + q];
    }
  }
}

int ora_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void ora_set_num_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}

/* grid term alone at n points: e (n*nc) = per-channel energies,
 * F (n*3) = -sum_c w_c grad e_c */
void ora_grid_points(const ora_grid* g, int64_t n, const double* pos,
                     const double* scale, const double* w, double* e,
                     double* F) {
  const int nc = g->nc;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double ee[ORA_MAXC], de[3 * ORA_MAXC];
    ora_atom_grid(g, pos + 3 * i, scale + (size_t)i * nc, ee, de);
    for (int a = 0; a < 3; ++a) F[3 * i + a] = 0.0;
    for (int c = 0; c < nc; ++c) {
      e[(size_t)i * nc + c] = ee[c];
      for (int a = 0; a < 3; ++a) F[3 * i + a] -= w[c] * de[3 * c + a];
    }
  }
}

/* energies and forces of many configurations with per-configuration
 * weights: terms (N*(4+nc)), mags (N*(4+nc)), F (N*n*3) */
void ora_energy_batch(const ora_grid* g, const ora_ligand* L, int64_t N,
                      const double* w, const double* xs, double* terms,
                      double* mags, double* F) {
  const int n = L->n, nc = g->nc;
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < N; ++s)
    ora_energy(g, L, w + (size_t)s * nc, xs + (size_t)s * n * 3,
               terms + (size_t)s * (4 + nc), mags + (size_t)s * (4 + nc),
               F + (size_t)s * n * 3);
}

/* three standard normals from the counter-based stream (Box-Muller), the
 * draw the samplers use for any purpose */
/* the four uniforms in (0, 1] of one draw */
void ora_uniform4(uint64_t seed, uint32_t index, int lig, int rep,
                  uint64_t sweep, uint32_t purpose, double* u) {
  uint32_t o[4];
  draw(seed, index, lig, rep, sweep, purpose, o);
  for (int i = 0; i < 4; ++i) u[i] = u01(o[i]);
}

void ora_normals3(uint64_t seed, uint32_t index, int lig, int rep,
                  uint64_t sweep, uint32_t purpose, double* z) {
  uint32_t o[4];
  draw(seed, index, lig, rep, sweep, purpose, o);
  normals3(o, z);
}
