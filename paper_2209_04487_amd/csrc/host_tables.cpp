// Host-side construction of the molecular tables and of the molecule->cell
// maps.  Everything here runs once per init call.
#include "host_tables.h"

#include "mol_jmg.h"

#include <algorithm>
#include <cmath>
#include <complex>

namespace msqd {

// Legendre P_0..P_n at x by the three-term recurrence
// (n+1) P_{n+1} = (2n+1) x P_n - n P_{n-1}.
static void legendre_all(int n, double x, double* p) {
  p[0] = 1.0;
  if (n >= 1) p[1] = x;
  for (int k = 1; k < n; ++k) p[k + 1] = ((2.0 * k + 1.0) * x * p[k] - k * p[k - 1]) / (k + 1.0);
}

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  // Newton iteration on P_n from the Chebyshev-like first guess; nodes are
  // symmetric, so the negative half is mirrored and x = 0 is exact for odd n.
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  std::vector<double> p(n + 1);
  const int half = n / 2;
  for (int i = 0; i < half; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      legendre_all(n, z, p.data());
      const double dp = n * (z * p[n] - p[n - 1]) / (z * z - 1.0);
      const double dz = p[n] / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    legendre_all(n, z, p.data());
    const double dp = n * (z * p[n] - p[n - 1]) / (z * z - 1.0);
    const double wi = 2.0 / ((1.0 - z * z) * dp * dp);
    // ascending order: x[n-1-i] = +z (largest first guess), x[i] = -z
    x[n - 1 - i] = z;
    x[i] = -z;
    w[n - 1 - i] = wi;
    w[i] = wi;
  }
  if (n & 1) {
    legendre_all(n, 0.0, p.data());
    const double dp = n * (-p[n - 1]) / (-1.0);  // n (x P_n - P_{n-1})/(x^2 - 1) at x = 0
    x[half] = 0.0;
    w[half] = 2.0 / (dp * dp);
  }
}

void lift_params(double c, double s, float* p, float* u) {
  // -tan(phi/2) = -s / (1 + c); near phi = pi use (c - 1) / s instead
  const double pd = (c > -0.5) ? -s / (1.0 + c) : (c - 1.0) / s;
  *p = static_cast<float>(pd);
  *u = static_cast<float>(s);
}

void unit_pair_f32(double c, double s, float* cf, float* sf) {
  const bool c_big = std::fabs(c) >= std::fabs(s);
  const double big = c_big ? c : s, small = c_big ? s : c;
  const float bf = static_cast<float>(big);
  const double bb = static_cast<double>(bf);
  const double rest = std::sqrt(std::max(0.0, 1.0 - bb * bb));
  float best = static_cast<float>(std::copysign(rest, small));
  double err = std::fabs(bb * bb + static_cast<double>(best) * best - 1.0);
  // the nearest float of the square root and its two neighbours
  for (int d = -1; d <= 1; d += 2) {
    const float cand = std::nextafter(best, d < 0 ? -2.0f : 2.0f);
    const double e = std::fabs(bb * bb + static_cast<double>(cand) * cand - 1.0);
    if (e < err) {
      err = e;
      best = cand;
    }
  }
  if (small == 0.0) best = 0.0f;
  *cf = c_big ? bf : best;
  *sf = c_big ? best : bf;
}

MolTablesHost build_mol_tables(const qd_desc& d, const double* U_g, const double* U_e,
                               const double* mu12) {
  MolTablesHost t;
  const int nr = d.n_r, nj = d.j_max + 1;
  const double dr = (d.r_max - d.r_min) / nr;
  const double dt = d.dt_au, mass = d.mass_au;
  t.dr = dr;
  t.kin.resize(nr);
  t.tw.resize(nr);
  for (int m = 0; m < nr; ++m) {
    const int ms = (m < nr / 2) ? m : m - nr;
    const double kap = 2.0 * kPi * ms / (nr * dr);
    const double ph = -kap * kap * dt / (4.0 * mass);
    t.kin[m] = std::polar(1.0 / nr, ph);
  }
  // four-step FFT twiddles: tw[x * R1 + y] = exp(-2 pi i x y / n_r), x, y < R1,
  // for the complex128 (tw) and complex64 (tw_f) splits of the grid
  auto twiddles = [&](int r1, std::vector<std::complex<double>>& out) {
    out.assign(static_cast<size_t>(r1) * r1, std::complex<double>(0.0, 0.0));
    for (int x = 0; x < r1; ++x)
      for (int y = 0; y < r1; ++y) {
        const long e = (static_cast<long>(x) * y) % nr;
        out[static_cast<size_t>(x) * r1 + y] = std::polar(1.0, -2.0 * kPi * static_cast<double>(e) / nr);
      }
  };
  twiddles(fft_r1(nr, 8), t.tw);
  twiddles(fft_r1(nr, 4), t.tw_f);
  t.vph.resize(static_cast<size_t>(2) * nj * nr);
  for (int s = 0; s < 2; ++s) {
    const double* U = (s == 0) ? U_g : U_e;
    for (int J = 0; J < nj; ++J) {
      for (int k = 0; k < nr; ++k) {
        const double r = d.r_min + k * dr;
        const double V = U[k] + J * (J + 1.0) / (2.0 * mass * r * r);
        t.vph[(static_cast<size_t>(s) * nj + J) * nr + k] = std::polar(1.0, -V * dt / 2.0);
      }
    }
  }
  std::vector<double> x, w;
  gauss_legendre(nj, x, w);
  t.x = x;
  t.tm.assign(static_cast<size_t>(nj) * nj, 0.0);
  std::vector<double> p(nj + 1);
  for (int k = 0; k < nj; ++k) {
    legendre_all(nj, x[k], p.data());
    for (int J = 0; J < nj; ++J)
      t.tm[static_cast<size_t>(k) * nj + J] = std::sqrt(w[k]) * std::sqrt((2.0 * J + 1.0) / 2.0) * p[J];
  }
  t.mudt.resize(nr);
  t.mu.resize(nr);
  t.mask.assign(nr, 1.0);
  const double ra = d.r_max - d.absorb_width_au;
  t.kdiss = nr;
  for (int k = 0; k < nr; ++k) {
    const double r = d.r_min + k * dr;
    t.mu[k] = mu12[k];
    t.mudt[k] = mu12[k] * dt;
    if (d.absorb_width_au > 0.0 && r >= ra)
      t.mask[k] = std::pow(std::cos(kPi * (r - ra) / (2.0 * d.absorb_width_au)), 0.125);
    if (r > d.r_diss_au && t.kdiss == nr) t.kdiss = k;
  }
  t.cj.assign(nj, 0.0);
  for (int J = 0; J + 1 < nj; ++J)
    t.cj[J] = (J + 1.0) / std::sqrt((2.0 * J + 1.0) * (2.0 * J + 3.0));
  return t;
}

// ------------------------------------------------------------------ maps
namespace {
struct SplitMix64 {
  uint64_t s;
  uint64_t next() {
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
};
inline int32_t scale_index(uint64_t u, int32_t n) {
  const unsigned __int128 prod = static_cast<unsigned __int128>(u >> 11) * static_cast<uint64_t>(n);
  return static_cast<int32_t>(prod >> 53);
}
}  // namespace

void place_slab(int32_t n_mol, int32_t nx, int32_t ny, uint64_t seed, int32_t k0, int32_t nk,
                int32_t* cell_of_mol) {
  SplitMix64 g{seed};
  for (int32_t m = 0; m < n_mol; ++m) {
    const uint64_t ux = g.next(), uy = g.next(), uz = g.next();
    const int64_t i = scale_index(ux, nx), j = scale_index(uy, ny), k = k0 + scale_index(uz, nk);
    cell_of_mol[m] = static_cast<int32_t>((k * ny + j) * nx + i);
  }
}

int32_t build_csr(int32_t n_mol, int32_t n_cells, const int32_t* cell_of_mol, int32_t* occ_cell,
                  int32_t* occ_ptr, int32_t* mol_perm) {
  // stable counting sort by cell
  std::vector<int32_t> count(static_cast<size_t>(n_cells) + 1, 0);
  for (int32_t m = 0; m < n_mol; ++m) count[cell_of_mol[m] + 1]++;
  for (int32_t c = 0; c < n_cells; ++c) count[c + 1] += count[c];
  std::vector<int32_t> pos(count.begin(), count.end() - 1);
  for (int32_t m = 0; m < n_mol; ++m) mol_perm[pos[cell_of_mol[m]]++] = m;
  int32_t n_occ = 0;
  for (int32_t c = 0; c < n_cells; ++c) {
    if (count[c + 1] > count[c]) {
      occ_cell[n_occ] = c;
      occ_ptr[n_occ] = count[c];
      ++n_occ;
    }
  }
  occ_ptr[n_occ] = n_mol;
  return n_occ;
}

// ------------------------------------------------------ (j, m), j_max >= 2
// Eigen-decomposition of a small symmetric matrix a [n x n] (row-major,
// destroyed) by cyclic Jacobi rotations: w ascending, v[i * n + k] the i-th
// component of the k-th eigenvector.  Returns false without convergence.
static bool sym_eig(int n, std::vector<double>& a, std::vector<double>& w, std::vector<double>& v) {
  v.assign(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i) v[i * n + i] = 1.0;
  bool done = false;
  double prev = HUGE_VAL;
  for (int sweep = 0; sweep < 100 && !done; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < n; ++k) (i == k ? diag : off) += a[i * n + k] * a[i * n + k];
    // converged, or stalled at the rounding floor of the sweep
    if (off <= 1e-30 * (diag + 1e-300) || (off >= prev && off <= 1e-24 * (diag + 1e-300))) {
      done = true;
      break;
    }
    prev = off;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a[p * n + q];
        if (apq == 0.0) continue;
        // rotation angle that zeroes a[p][q]
        const double th = (a[q * n + q] - a[p * n + p]) / (2.0 * apq);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {   // columns p, q
          const double akp = a[k * n + p], akq = a[k * n + q];
          a[k * n + p] = c * akp - s * akq;
          a[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {   // rows p, q
          const double apk = a[p * n + k], aqk = a[q * n + k];
          a[p * n + k] = c * apk - s * aqk;
          a[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = v[k * n + p], vkq = v[k * n + q];
          v[k * n + p] = c * vkp - s * vkq;
          v[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  if (!done) return false;
  // sort ascending
  std::vector<int> ord(n);
  for (int i = 0; i < n; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int x, int y) { return a[x * n + x] < a[y * n + y]; });
  std::vector<double> vs(static_cast<size_t>(n) * n);
  w.assign(n, 0.0);
  for (int k = 0; k < n; ++k) {
    w[k] = a[ord[k] * n + ord[k]];
    for (int i = 0; i < n; ++i) vs[i * n + k] = v[i * n + ord[k]];
  }
  v.swap(vs);
  return true;
}

bool fill_jmg_tables(int jm, double* out) {
  const JmgTab tb = jmg_tab(jm);
  std::vector<double> a, w, v;
  // J_x on the block j: <m+1|J_x|m> = sqrt(j(j+1) - m(m+1)) / 2
  for (int j = 0; j <= jm; ++j) {
    const int n = 2 * j + 1;
    a.assign(static_cast<size_t>(n) * n, 0.0);
    for (int i = 0; i + 1 < n; ++i) {
      const double m = i - j;
      a[i * n + i + 1] = a[(i + 1) * n + i] = 0.5 * std::sqrt(j * (j + 1.0) - m * (m + 1.0));
    }
    if (!sym_eig(n, a, w, v)) return false;
    for (int k = 0; k < n; ++k)
      if (std::fabs(w[k] - (k - j)) > 1e-9) return false;   // the spectrum is -j..j
    std::copy(v.begin(), v.end(), out + tb.jx + jmg_jx_off(j));
  }
  // cos(theta) on the block m' = a: <j+1,a|cos|j,a> = sqrt(((j+1)^2 - a^2) / ((2j+1)(2j+3)))
  for (int am = 0; am <= jm; ++am) {
    const int n = jm + 1 - am;
    a.assign(static_cast<size_t>(n) * n, 0.0);
    for (int i = 0; i + 1 < n; ++i) {
      const double j = am + i;
      a[i * n + i + 1] = a[(i + 1) * n + i] =
          std::sqrt(((j + 1.0) * (j + 1.0) - am * am) / ((2.0 * j + 1.0) * (2.0 * j + 3.0)));
    }
    if (!sym_eig(n, a, w, v)) return false;
    std::copy(v.begin(), v.end(), out + tb.q + jmg_q_off(jm, am));
    std::copy(w.begin(), w.end(), out + tb.x + jmg_x_off(jm, am));
  }
  // dipole matrix elements (Condon-Shortley phases)
  for (int j = 0; j <= jm; ++j)
    for (int m = -j; m <= j; ++m) {
      double* e = out + tb.dip + 3 * (j * j + m + j);
      const double jj = j, mm = m;
      e[0] = j < jm ? std::sqrt(((jj + 1.0) * (jj + 1.0) - mm * mm) / ((2.0 * jj + 1.0) * (2.0 * jj + 3.0))) : 0.0;
      e[1] = j < jm ? -std::sqrt((jj + mm + 1.0) * (jj + mm + 2.0) / ((2.0 * jj + 1.0) * (2.0 * jj + 3.0))) : 0.0;
      e[2] = (j >= 1 && m + 1 <= j - 1)
                 ? std::sqrt((jj - mm) * (jj - mm - 1.0) / ((2.0 * jj - 1.0) * (2.0 * jj + 1.0)))
                 : 0.0;
    }
  return true;
}

}  // namespace msqd
