// Host side of the collision library: descriptor validation, direction rules,
// FP64 multiplier tables of the fast spectral method (Sec. 4.4.1), the
// inverse Gram matrix of the collision invariants, device binding and the
// C-ABI entry points of the plan.
#include <dlfcn.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <thread>

#include "bz_internal.hpp"

namespace bz {

static thread_local std::string g_err;

bz_status fail(bz_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}
void clear_error() { g_err.clear(); }
const char* last_error() { return g_err.c_str(); }

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

// ---------------------------------------------------------------- direction rules
// All rules cover the half sphere; the angular integrand of the fast method
// is even in e, and the weights sum to the half-sphere area 2 pi.
void rule_icosa6(std::vector<double>& d, std::vector<double>& w) {
  const double g = (1.0 + std::sqrt(5.0)) / 2.0;
  const double raw[6][3] = {{0, 1, g}, {0, -1, g}, {1, g, 0}, {-1, g, 0}, {g, 0, 1}, {-g, 0, 1}};
  const double s = 1.0 / std::sqrt(1.0 + g * g);
  d.assign(18, 0.0);
  w.assign(6, kPi / 3.0);
  for (int i = 0; i < 6; ++i)
    for (int c = 0; c < 3; ++c) d[3 * i + c] = raw[i][c] * s;
}

void rule_product(int a1, int a2, std::vector<double>& d, std::vector<double>& w) {
  d.clear();
  w.clear();
  double sum = 0.0;
  for (int p = 0; p < a1; ++p) {
    const double th = (p + 0.5) * kPi / a1;
    for (int q = 0; q < a2; ++q) {
      const double ph = q * kPi / a2;
      d.push_back(std::sin(th) * std::cos(ph));
      d.push_back(std::sin(th) * std::sin(ph));
      d.push_back(std::cos(th));
      w.push_back(std::sin(th));
      sum += std::sin(th);
    }
  }
  for (double& x : w) x *= 2.0 * kPi / sum;
}

}  // namespace

void rule_spiral(int m, std::vector<double>& d, std::vector<double>& w) {
  const double g = (1.0 + std::sqrt(5.0)) / 2.0;
  d.resize(3 * m);
  w.assign(m, 2.0 * kPi / m);
  for (int p = 0; p < m; ++p) {
    const double z = (p + 0.5) / m;
    const double az = 2.0 * kPi * p / g;
    const double s = std::sqrt(1.0 - z * z);
    d[3 * p] = s * std::cos(az);
    d[3 * p + 1] = s * std::sin(az);
    d[3 * p + 2] = z;
  }
}

namespace {

// ---------------------------------------------------------------- special functions
// Gauss-Legendre nodes and weights on [-1, 1] by Newton iteration on the
// three-term recurrence of P_n.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

struct PhiEval {
  double R, gamma;
  std::vector<double> t2, wt;  // quadrature in t (rho = R t^2) for gamma not in {0,1}
  explicit PhiEval(double R_, double g_) : R(R_), gamma(g_) {
    if (gamma != 0.0 && gamma != 1.0) {
      std::vector<double> x, w;
      gauss_legendre(256, x, w);
      t2.resize(x.size());
      wt.resize(x.size());
      for (size_t i = 0; i < x.size(); ++i) {
        const double t = 0.5 * (x[i] + 1.0);
        t2[i] = t * t;
        wt[i] = 0.5 * w[i] * std::pow(t, 2.0 * gamma + 1.0);
      }
    }
  }
  static double sinc(double x) { return x == 0.0 ? 1.0 : std::sin(x) / x; }
  // phi_R(s) = 2 int_0^R r^gamma cos(r s) dr
  double operator()(double s) const {
    if (gamma == 1.0) {
      const double a = sinc(R * s), b = sinc(0.5 * R * s);
      return R * R * (2.0 * a - b * b);
    }
    if (gamma == 0.0) return 2.0 * R * sinc(R * s);
    double acc = 0.0;
    for (size_t i = 0; i < t2.size(); ++i) acc += wt[i] * std::cos(R * s * t2[i]);
    return 4.0 * std::pow(R, gamma + 1.0) * acc;
  }
};

// psi_R(r) = 2 pi R J1(R r) / r, pi R^2 at r = 0 (integral over the disc of
// radius R in the plane normal to the direction).
double psi_R(double r, double R) {
  if (r == 0.0) return kPi * R * R;
  return 2.0 * kPi * R * ::j1(R * r) / r;
}

// Inverse of a symmetric positive definite K x K matrix (row-major) by
// Cholesky factorisation; false if G is not positive definite.
template <int K>
bool spd_inverse(const double* G, double* out) {
  double Lc[K * K] = {};
  for (int i = 0; i < K; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = G[K * i + j];
      for (int k = 0; k < j; ++k) s -= Lc[K * i + k] * Lc[K * j + k];
      if (i == j) {
        if (!(s > 0.0)) return false;
        Lc[K * i + i] = std::sqrt(s);
      } else {
        Lc[K * i + j] = s / Lc[K * j + j];
      }
    }
  // columns of the inverse: solve L L^T x = e_c
  for (int c = 0; c < K; ++c) {
    double y[K], x[K];
    for (int i = 0; i < K; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) s -= Lc[K * i + k] * y[k];
      y[i] = s / Lc[K * i + i];
    }
    for (int i = K - 1; i >= 0; --i) {
      double s = y[i];
      for (int k = i + 1; k < K; ++k) s -= Lc[K * k + i] * x[k];
      x[i] = s / Lc[K * i + i];
    }
    for (int i = 0; i < K; ++i) out[K * i + c] = x[i];
  }
  return true;
}

void build_tables(bz_plan* p) {
  const int n = p->n, n3 = n * n * n;
  std::vector<double> kap(n);
  for (int k = 0; k < n; ++k) kap[k] = (kPi / p->L) * double(k < n / 2 ? k : k - n);
  p->mult.assign(size_t(p->m1) * n3 * 2, 0.0);
  PhiEval phi(p->R, p->gamma);
  auto work = [&](int p0, int p1) {
    for (int dir = p0; dir < p1; ++dir) {
      const double e0 = p->dirs[3 * dir], e1 = p->dirs[3 * dir + 1], e2 = p->dirs[3 * dir + 2];
      double* out = &p->mult[size_t(dir) * n3 * 2];
      for (int k2 = 0; k2 < n; ++k2)
        for (int k3 = 0; k3 < n; ++k3)
          for (int k1 = 0; k1 < n; ++k1) {
            const double q1 = kap[k1], q2 = kap[k2], q3 = kap[k3];
            const double s = q1 * e0 + q2 * e1 + q3 * e2;
            const double r1 = q1 - s * e0, r2 = q2 - s * e1, r3 = q3 - s * e2;
            const double r = std::sqrt(r1 * r1 + r2 * r2 + r3 * r3);
            const size_t o = 2 * ((size_t(k2) * n + k3) * n + k1);
            out[o] = phi(s);
            out[o + 1] = psi_R(r, p->R);
          }
    }
  };
  unsigned hw = std::thread::hardware_concurrency();
  int nt = int(std::max(1u, std::min(hw, 16u)));
  nt = std::min(nt, p->m);
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t) th.emplace_back(work, p->m * t / nt, p->m * (t + 1) / nt);
  for (auto& x : th) x.join();
  // loss pass: (Bhat_M, 1), Bhat_M(k) = sum_p w_p alpha_p(k) alpha'_p(k)
  double* loss = &p->mult[size_t(p->m) * n3 * 2];
  for (int dir = 0; dir < p->m; ++dir) {
    const double* a = &p->mult[size_t(dir) * n3 * 2];
    const double wd = p->w[dir];
    for (int i = 0; i < n3; ++i) loss[2 * i] += wd * a[2 * i] * a[2 * i + 1];
  }
  for (int i = 0; i < n3; ++i) loss[2 * i + 1] = 1.0;
  // Balance factors of the packed transforms.  Y = IDFT((a s + i a'/s) fhat)
  // carries s A and A'/s, whose product is A A' for any s; s equalises the
  // two parts so that FP32 rounding of the transform hits both alike.  The
  // loss pass packs Lambda/sL with sL fNyq (the Nyquist part of f):
  // fN Lambda = (f - fNyq) Lambda is then formed with the exact input f,
  // sL = sqrt(Bhat_M(0)) (Lambda/f is scale free, so one sL fits all cells).
  p->pscale.assign(p->m1, 1.0);
  for (int dir = 0; dir < p->m; ++dir) {
    const double* a = &p->mult[size_t(dir) * n3 * 2];
    double ma = 0.0, mb = 0.0;
    for (int i = 0; i < n3; ++i) {
      ma = std::max(ma, std::fabs(a[2 * i]));
      mb = std::max(mb, std::fabs(a[2 * i + 1]));
    }
    p->pscale[dir] = (ma > 0.0 && mb > 0.0) ? std::sqrt(mb / ma) : 1.0;
  }
  p->pscale[p->m] = std::sqrt(std::fabs(loss[0]) > 0.0 ? std::fabs(loss[0]) : 1.0);
  p->wext.assign(p->w.begin(), p->w.end());
  p->wext.push_back(p->pscale[p->m]);
}

// Device form of pass `pass` at table index i ([k2][k3][k1] order): gain
// passes (a s, a'/s), zero on the Nyquist planes; the loss pass
// (Bhat_M/sL, sL [k on a Nyquist plane]).
void device_multiplier(const bz_plan* p, int pass, size_t i, double& re, double& im) {
  const int n = p->n;
  const size_t n3 = p->npts;
  bool nyq;
  if (p->dim == 2) {  // [k2][k1]
    nyq = int(i % n) == n / 2 || int(i / n) == n / 2;
  } else {            // [k2][k3][k1]
    const int k1 = int(i % n), k3 = int((i / n) % n), k2 = int(i / (size_t(n) * n));
    nyq = k1 == n / 2 || k2 == n / 2 || k3 == n / 2;
  }
  const double* a = &p->mult[size_t(pass) * n3 * 2];
  const double s = p->pscale[pass];
  if (pass < p->m) {
    re = nyq ? 0.0 : a[2 * i] * s;
    im = nyq ? 0.0 : a[2 * i + 1] / s;
  } else {
    re = nyq ? 0.0 : a[2 * i] / s;
    im = nyq ? s : 0.0;
  }
}

bool build_gram_inverse(bz_plan* p) {
  const int n = p->n;
  double G[25] = {};
  for (int i1 = 0; i1 < n; ++i1)
    for (int i2 = 0; i2 < n; ++i2)
      for (int i3 = 0; i3 < n; ++i3) {
        const double v1 = (i1 - n / 2) * p->dv, v2 = (i2 - n / 2) * p->dv, v3 = (i3 - n / 2) * p->dv;
        const double c[5] = {1.0, v1, v2, v3, v1 * v1 + v2 * v2 + v3 * v3};
        for (int a = 0; a < 5; ++a)
          for (int b = 0; b < 5; ++b) G[5 * a + b] += c[a] * c[b];
      }
  return spd_inverse<5>(G, p->ginv);
}

// ---------------------------------------------------------------- two velocity dimensions
// Maxwell molecules in two velocity dimensions (Sec. 4.4.1, the 2d case):
// Btilde = C, angles theta_p = pi p / m (p = 1..m) of weight pi/m, and
//   alpha_p(k) = phi(kappa_k . e_p), alpha'_p(k) = phi(kappa_k . e_p'),
//   phi(s) = 2 R sinc(R s), e_p = (cos theta_p, sin theta_p), e_p' = e_p turned by pi/2.
// Host tables [p][k2][k1] x (a, a'), the loss pass (Bhat_M, 1) last.
void build_tables2d(bz_plan* p) {
  const int n = p->n;
  const size_t n2 = size_t(n) * n;
  std::vector<double> kap(n);
  for (int k = 0; k < n; ++k) kap[k] = (kPi / p->L) * double(k < n / 2 ? k : k - n);
  p->w.assign(p->m, kPi / p->m);
  p->dirs.assign(size_t(3) * p->m, 0.0);  // (cos, sin, 0) theta_p
  for (int dir = 0; dir < p->m; ++dir) {
    p->dirs[3 * dir] = std::cos(kPi * double(dir + 1) / p->m);
    p->dirs[3 * dir + 1] = std::sin(kPi * double(dir + 1) / p->m);
  }
  p->mult.assign(size_t(p->m1) * n2 * 2, 0.0);
  auto phi = [&](double x) { const double y = p->R * x; return 2.0 * p->R * (y == 0.0 ? 1.0 : std::sin(y) / y); };
  for (int dir = 0; dir < p->m; ++dir) {
    const double th = kPi * double(dir + 1) / p->m;
    const double c = std::cos(th), sn = std::sin(th);
    double* out = &p->mult[size_t(dir) * n2 * 2];
    for (int k2 = 0; k2 < n; ++k2)
      for (int k1 = 0; k1 < n; ++k1) {
        const size_t o = 2 * (size_t(k2) * n + k1);
        out[o] = phi(kap[k1] * c + kap[k2] * sn);
        out[o + 1] = phi(-kap[k1] * sn + kap[k2] * c);
      }
  }
  double* loss = &p->mult[size_t(p->m) * n2 * 2];
  for (int dir = 0; dir < p->m; ++dir) {
    const double* a = &p->mult[size_t(dir) * n2 * 2];
    for (size_t i = 0; i < n2; ++i) loss[2 * i] += p->w[dir] * a[2 * i] * a[2 * i + 1];
  }
  for (size_t i = 0; i < n2; ++i) loss[2 * i + 1] = 1.0;
  // balance factors as in three dimensions (alpha and alpha' share phi: s = 1)
  p->pscale.assign(p->m1, 1.0);
  for (int dir = 0; dir < p->m; ++dir) {
    const double* a = &p->mult[size_t(dir) * n2 * 2];
    double ma = 0.0, mb = 0.0;
    for (size_t i = 0; i < n2; ++i) {
      ma = std::max(ma, std::fabs(a[2 * i]));
      mb = std::max(mb, std::fabs(a[2 * i + 1]));
    }
    p->pscale[dir] = (ma > 0.0 && mb > 0.0) ? std::sqrt(mb / ma) : 1.0;
  }
  p->pscale[p->m] = std::sqrt(std::fabs(loss[0]) > 0.0 ? std::fabs(loss[0]) : 1.0);
  p->wext.assign(p->w.begin(), p->w.end());
  p->wext.push_back(p->pscale[p->m]);
}

// (C C^T)^-1 of the invariants (1, v1, v2, |v|^2) of two velocity dimensions.
bool build_gram_inverse2d(bz_plan* p) {
  const int n = p->n;
  double G[16] = {};
  for (int i1 = 0; i1 < n; ++i1)
    for (int i2 = 0; i2 < n; ++i2) {
      const double v1 = (i1 - n / 2) * p->dv, v2 = (i2 - n / 2) * p->dv;
      const double c[4] = {1.0, v1, v2, v1 * v1 + v2 * v2};
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) G[4 * a + b] += c[a] * c[b];
    }
  return spd_inverse<4>(G, p->ginv);
}

// One fused kernel keeps every intermediate of a cell on chip: the workspace
// holds only the status word (and a token 256 bytes per cell, so that the
// capacity of a binding still counts cells).
void layout2d(bz_plan* p) {
  const size_t es = p->fp32 ? 4 : 8;
  p->table_mult_bytes = align256(size_t(p->m1) * p->npts * 2 * es);
  p->table_w_off = p->table_mult_bytes;
  p->tables_bytes = p->table_mult_bytes + align256(size_t(p->m1) * es);
  p->table_dft_off = p->tables_bytes;
  if (p->transform == BZ_XF_DFT_GEMM)  // [Re/Im part][N/16 row tiles][N/2 k steps][64 lanes] floats
    p->tables_bytes += align256(size_t(2) * (p->n / 16) * (p->n / 2) * 64 * sizeof(float));
  p->ws = WsLayout{};
  p->ws.fh_cell = spectrum2d_in_workspace(p->n) ? align256(p->npts * 2 * es) : 256;  // the cell's spectrum, [k2][k1]
  p->ws_fixed = kStatusBytes;
  p->ws_per_cell = p->ws.fh_cell;
}

bz_status create_plan2d(const bz_plan_desc& d, bz_plan** out) {
  if (!(d.n == 16 || d.n == 32 || d.n == 64))
    return fail(BZ_ERR_UNSUPPORTED, "bz_plan_create: two-dimensional plans need n in {16,32,64}, got %d", d.n);
  if (d.precision == BZ_FP64 && d.n == 64)
    return fail(BZ_ERR_UNSUPPORTED, "bz_plan_create: two-dimensional FP64 plans need n in {16,32}");
  if (d.gamma != 0.0)
    return fail(BZ_ERR_UNSUPPORTED, "bz_plan_create: two velocity dimensions are Maxwell molecules (gamma = 0)");
  if (d.dir_kind != BZ_DIRS_CIRCLE)
    return fail(BZ_ERR_ARG, "bz_plan_create: two-dimensional plans take dir_kind BZ_DIRS_CIRCLE");
  if (d.transform == BZ_XF_PLAIN)
    return fail(BZ_ERR_UNSUPPORTED, "bz_plan_create: two-dimensional plans have one (fused) kernel");
  if (d.dealias || d.chunks || d.slices)
    return fail(BZ_ERR_ARG, "bz_plan_create: two-dimensional plans take dealias, chunks and slices 0");
  const double R = d.R > 0.0 ? d.R : (std::sqrt(2.0) - 1.0) * d.L;
  bz_plan* p = new bz_plan();
  p->d = d;
  p->d.dirs = nullptr;
  p->d.weights = nullptr;
  p->d.R = R;
  p->dim = 2;
  p->n = d.n;
  p->npts = size_t(d.n) * d.n;
  p->m = d.m;
  p->m1 = d.m + 1;
  p->L = d.L;
  p->R = R;
  p->gamma = 0.0;
  p->C = d.kernel_c;
  p->dv = 2.0 * d.L / d.n;
  p->fp32 = d.precision == BZ_FP32;
  p->project = d.project ? 1 : 0;
  p->transform = BZ_XF_FUSED;
  p->chunks = 1;
  p->slices = 1;
  build_tables2d(p);
  if (!build_gram_inverse2d(p)) {
    delete p;
    return fail(BZ_ERR_NUMERIC, "bz_plan_create: Gram matrix not positive definite");
  }
  layout2d(p);
  *out = p;
  return BZ_OK;
}

// ---------------------------------------------------------------- tune table
std::mutex g_tune_mu;
std::string g_tune_path;
bool g_tune_set = false;

struct TuneChoice {
  int transform = 0, chunks = 0, slices = 0;
  bool found = false;
};

// The table shipped beside the library (tune_gfx950.txt in the directory of
// libbz.so), written by the autotuner on an MI355X.
std::string shipped_tune_table() {
  Dl_info info{};
  if (!dladdr(reinterpret_cast<void*>(&bz_set_tune_table), &info) || !info.dli_fname) return "";
  std::string lib = info.dli_fname;
  const size_t slash = lib.find_last_of('/');
  return (slash == std::string::npos ? std::string(".") : lib.substr(0, slash)) + "/tune_gfx950.txt";
}

TuneChoice tune_lookup(int n, int m, int precision, int max_cells) {
  std::string path;
  bool set = false;
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    set = g_tune_set;
    if (set) path = g_tune_path;
  }
  if (!set) {
    const char* env = std::getenv("BZ_TUNE_TABLE");
    path = env ? std::string(env) : shipped_tune_table();
  }
  TuneChoice best;
  if (path.empty()) return best;
  FILE* fp = std::fopen(path.c_str(), "r");
  if (!fp) return best;
  char line[512];
  int best_cells = -1, smallest_cells = 1 << 30;
  TuneChoice smallest;
  while (std::fgets(line, sizeof line, fp)) {
    char arch[64];
    int tn, tm, tp, tc, tx, tch, ts;
    double us;
    if (std::sscanf(line, "%63s %d %d %d %d %d %d %d %lf", arch, &tn, &tm, &tp, &tc, &tx, &tch, &ts, &us) != 9) continue;
    if (std::strcmp(arch, "gfx950") != 0 || tn != n || tm != m || tp != precision) continue;
    TuneChoice c;
    c.transform = tx;
    c.chunks = tch;
    c.slices = ts;
    c.found = true;
    if (tc <= max_cells && tc > best_cells) {
      best_cells = tc;
      best = c;
    }
    if (tc < smallest_cells) {
      smallest_cells = tc;
      smallest = c;
    }
  }
  std::fclose(fp);
  return best.found ? best : smallest;
}

}  // namespace

// The evaluation strategy of a descriptor at a given capacity (three
// dimensions): the descriptor's knobs, else the tune table's line, else the
// size heuristics.  The server keys its cached plans by it.
// Workspace bytes per cell of the chunked plain path with K directions per
// stage-A launch (the layout below without a dealiased sub-plan).
size_t plain_ws_per_cell(int n, bool fp32, int K) {
  const size_t n3 = size_t(n) * n * n, es = fp32 ? 4 : 8;
  return align256(n3 * 2 * es) + align256(n3 * 2 * es * size_t(K)) + align256(n3 * es) +
         sizeof(double) * bzk::kImexPar * 2;
}

Strategy resolve_strategy(const bz_plan_desc& d, int max_cells, size_t ws_budget) {
  Strategy sg;
  const int fp32 = d.precision == BZ_FP32;
  const bool fused_ok = fused_supported(d.n, fp32);
  const bool gemm_ok = dft_gemm_supported(d.n, fp32);
  int transform = d.transform, chunks = d.chunks, slices = d.slices;
  if (transform == BZ_XF_AUTO && chunks == 0 && slices == 0) {
    const TuneChoice tc = tune_lookup(d.n, d.m, d.precision, max_cells);
    if (tc.found && (tc.transform == BZ_XF_PLAIN || (tc.transform == BZ_XF_DFT_GEMM && gemm_ok) ||
                     (tc.transform == BZ_XF_FUSED && fused_ok && fused_slices_supported(d.n, tc.slices)))) {
      transform = tc.transform;
      chunks = tc.chunks;
      slices = tc.slices;
    }
  }
  if (transform == BZ_XF_DFT_GEMM && gemm_ok) sg.transform = BZ_XF_DFT_GEMM;
  else sg.transform = (transform == BZ_XF_PLAIN || transform == BZ_XF_DFT_GEMM || !fused_ok) ? BZ_XF_PLAIN : BZ_XF_FUSED;
  sg.plain_k = (sg.transform != BZ_XF_FUSED && chunks > 0) ? std::min(chunks, kPlainChunkMax)
                                                           : plain_chunk(d.n, fp32 != 0, max_cells);
  sg.chunks = sg.transform == BZ_XF_FUSED ? (chunks > 0 ? chunks : fused_default_chunks(d.n, max_cells)) : 1;
  if (sg.chunks > d.m + 1) sg.chunks = d.m + 1;
  sg.slices = slices > 0 ? slices : (d.n == 24 ? 1 : 2);
  // fewer stage-A volumes per cell when the workspace of max_cells cells would exceed the budget
  if (sg.transform != BZ_XF_FUSED && !d.dealias)
    while (sg.plain_k > 1 && plain_ws_per_cell(d.n, fp32 != 0, sg.plain_k) * size_t(std::max(1, max_cells)) > ws_budget)
      sg.plain_k /= 2;
  return sg;
}

namespace {

void layout(bz_plan* p) {
  const size_t n3 = size_t(p->n) * p->n * p->n;
  const size_t es = p->fp32 ? 4 : 8;
  p->table_mult_bytes = align256(size_t(p->m1) * n3 * 2 * es);
  p->table_w_off = p->table_mult_bytes;
  p->tables_bytes = p->table_mult_bytes + align256(size_t(p->m1) * es);
  p->table_dft_off = p->tables_bytes;
  if (p->transform == BZ_XF_DFT_GEMM)  // [Re/Im part][N/16 row tiles][N/2 k steps][64 lanes] floats
    p->tables_bytes += align256(size_t(2) * (p->n / 16) * (p->n / 2) * 64 * sizeof(float));
  // fused: the forward transform keeps its intermediate volumes on chip (no y),
  // and with one chunk and the projection on, the products never leave the chip (no acc)
  const bool fused = p->transform == BZ_XF_FUSED;
  const int acc_chunks = fused ? ((p->chunks == 1 && p->project) ? 0 : p->chunks) : 1;
  p->ws.fh_cell = align256(n3 * 2 * es);
  // chunked plain path: a chunk of pchunk directions shares the stage-A output
  // (one volume per direction); fused: an FP32 copy of f in the collision
  // kernel's loss-pass order
  p->pchunk = fused ? 0 : (p->plain_k > 0 ? p->plain_k : plain_chunk(p->n, p->fp32 != 0, p->d.max_cells));
  p->ws.y_cell = fused ? align256(n3 * sizeof(float)) : align256(n3 * 2 * es * p->pchunk);
  p->ws.acc_cell = align256(n3 * es * acc_chunks);
  p->ws.par_cell = sizeof(double) * bzk::kImexPar * 2;  // per-cell IMEX parameters (128 B)
  p->ws_fixed = kStatusBytes;  // the numeric status word of the plan's evaluations
  if (p->pad) {
    // forward at n (fhat, scratch), f and raw Q on the padded grid, padded spectrum,
    // Q resampled back (accumulator region), and the padded plan's own workspace
    const size_t np3 = size_t(p->pad->n) * p->pad->n * p->pad->n;
    p->ws.y_cell = align256(np3 * 2 * es);
    p->ws.acc_cell = align256(n3 * es);
    p->ws.fp_cell = align256(np3 * es);
    p->ws.qp_cell = align256(np3 * es);
    p->ws.gp_cell = align256(np3 * 2 * es);
    p->ws.pad_cell = p->pad->ws_per_cell;
    p->ws_fixed += p->pad->ws_fixed;  // the padded plan's own fixed region sits with its cells
    p->tables_bytes = p->pad->tables_bytes;  // the device tables are the padded operator's
  }
  p->ws_per_cell = p->ws.fh_cell + p->ws.y_cell + p->ws.acc_cell + p->ws.par_cell + p->ws.fp_cell +
                   p->ws.qp_cell + p->ws.gp_cell + p->ws.pad_cell;
}


}  // namespace

Binding make_binding(const bz_plan* p, const void* tables, void* ws, size_t ws_bytes) {
  Binding b;
  b.tables = tables;
  b.ws = ws;
  const size_t cap = ws_bytes >= p->ws_fixed + p->ws_per_cell ? (ws_bytes - p->ws_fixed) / p->ws_per_cell : 0;
  b.capacity = int(std::min<size_t>(cap, size_t(1) << 30));
  b.lay = p->ws;
  b.lay.status_off = 0;
  b.lay.fh_off = kStatusBytes;
  b.lay.y_off = b.lay.fh_off + size_t(b.capacity) * b.lay.fh_cell;
  b.lay.acc_off = b.lay.y_off + size_t(b.capacity) * b.lay.y_cell;
  b.lay.par_off = b.lay.acc_off + size_t(b.capacity) * b.lay.acc_cell;
  b.lay.fp_off = b.lay.par_off + size_t(b.capacity) * b.lay.par_cell;
  b.lay.qp_off = b.lay.fp_off + size_t(b.capacity) * b.lay.fp_cell;
  b.lay.gp_off = b.lay.qp_off + size_t(b.capacity) * b.lay.qp_cell;
  b.lay.pad_off = b.lay.gp_off + size_t(b.capacity) * b.lay.gp_cell;  // padded plan: fixed part, then cells
  return b;
}

void fill_tables_host(const bz_plan* p, unsigned char* host) {
  if (p->pad) {
    fill_tables_host(p->pad, host);
    return;
  }
  const size_t n3 = p->npts;
  std::memset(host, 0, p->tables_bytes);
  const size_t entries = size_t(p->m1) * n3;
  if (p->fp32) {
    // the fused kernels (three and two velocity dimensions) take a gain
    // direction's weight in its multipliers: sqrt|w| on the real part and
    // sign(w) sqrt|w| on the imaginary one, so that Re Y Im Y carries w
    const bool weighted = p->transform == BZ_XF_FUSED;
    float* m = reinterpret_cast<float*>(host);
    for (size_t e = 0; e < entries; ++e) {
      const int pass = int(e / n3);
      double re, im;
      device_multiplier(p, pass, e % n3, re, im);
      if (weighted && pass < p->m) {
        const double w = p->wext[pass], sw = std::sqrt(std::fabs(w));
        re *= sw;
        im *= w < 0.0 ? -sw : sw;
      }
      m[2 * e] = float(re);
      m[2 * e + 1] = float(im);
    }
    float* w = reinterpret_cast<float*>(host + p->table_w_off);
    for (int i = 0; i < p->m1; ++i) w[i] = float(p->wext[i]);
    if (p->transform == BZ_XF_DFT_GEMM) {
      // A operands of Re Y = [Re W | -Im W] [Re X; Im X] and Im Y = [Im W | Re W] [Re X; Im X],
      // W[j1][k1] = exp(+2 pi i j1 k1 / n), in the lane order of the 16x16x4 matrix instruction
      const int n = p->n, mtiles = n / 16, ksteps = n / 2;
      float* fr = reinterpret_cast<float*>(host + p->table_dft_off);
      for (int part = 0; part < 2; ++part)
        for (int mt = 0; mt < mtiles; ++mt)
          for (int ks = 0; ks < ksteps; ++ks)
            for (int l = 0; l < 64; ++l) {
              const int j1 = 16 * mt + l % 16, kk = 4 * ks + l / 16;
              const int k1 = kk < n ? kk : kk - n;
              const double ang = 2.0 * kPi * double((j1 * k1) % n) / double(n);
              const double c = std::cos(ang), sn = std::sin(ang);
              const double v = part == 0 ? (kk < n ? c : -sn) : (kk < n ? sn : c);
              fr[((size_t(part) * mtiles + mt) * ksteps + ks) * 64 + l] = float(v);
            }
    }
  } else {
    const bool weighted = p->transform == BZ_XF_FUSED;  // two velocity dimensions: as above
    double* m = reinterpret_cast<double*>(host);
    for (size_t e = 0; e < entries; ++e) {
      const int pass = int(e / n3);
      device_multiplier(p, pass, e % n3, m[2 * e], m[2 * e + 1]);
      if (weighted && pass < p->m) {
        const double w = p->wext[pass], sw = std::sqrt(std::fabs(w));
        m[2 * e] *= sw;
        m[2 * e + 1] *= w < 0.0 ? -sw : sw;
      }
    }
    std::memcpy(host + p->table_w_off, p->wext.data(), size_t(p->m1) * 8);
  }
}

bz_status upload_tables(const bz_plan* p, void* tables_dev, hipStream_t s) {
  std::vector<unsigned char> host(p->tables_bytes);
  fill_tables_host(p, host.data());
  hipError_t e = hipMemcpyAsync(tables_dev, host.data(), p->tables_bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(BZ_ERR_DEVICE, "table upload failed: %s", hipGetErrorString(e));
  return BZ_OK;
}

namespace {
}  // namespace
}  // namespace bz

using namespace bz;

extern "C" {

int32_t bz_abi_version(void) { return BZ_ABI_VERSION; }

const char* bz_last_error(void) { return bz::last_error(); }

bz_status bz_plan_create(const bz_plan_desc* desc, bz_plan** out) {
  clear_error();
  if (!desc || !out) return fail(BZ_ERR_ARG, "bz_plan_create: null argument");
  *out = nullptr;
  const bz_plan_desc& d = *desc;
  if (d.dim != 0 && d.dim != 2 && d.dim != 3) return fail(BZ_ERR_ARG, "bz_plan_create: dim must be 0, 2 or 3");
  if (d.dim == 2) {
    if (!(d.L > 0.0) || !std::isfinite(d.L)) return fail(BZ_ERR_ARG, "bz_plan_create: L must be > 0");
    const double rmax2 = 4.0 * d.L / (3.0 + std::sqrt(2.0));
    if (d.R > 0.0 && !(d.R <= rmax2 * (1.0 + 1e-12)))
      return fail(BZ_ERR_ARG, "bz_plan_create: R=%.17g exceeds the non-overlap bound 4L/(3+sqrt2)=%.17g", d.R, rmax2);
    if (!(d.kernel_c > 0.0) || !std::isfinite(d.kernel_c)) return fail(BZ_ERR_ARG, "bz_plan_create: kernel_c must be > 0");
    if (d.m < 1 || d.m > 512) return fail(BZ_ERR_ARG, "bz_plan_create: m=%d not in 1..512", d.m);
    if (d.precision != BZ_FP32 && d.precision != BZ_FP64) return fail(BZ_ERR_ARG, "bz_plan_create: bad precision");
    if (d.transform < BZ_XF_AUTO || d.transform > BZ_XF_PLAIN) return fail(BZ_ERR_ARG, "bz_plan_create: bad transform");
    if (d.max_cells < 1) return fail(BZ_ERR_ARG, "bz_plan_create: max_cells must be >= 1");
    return create_plan2d(d, out);
  }
  if (!(d.n == 16 || d.n == 24 || d.n == 32 || d.n == 48))
    return fail(BZ_ERR_UNSUPPORTED, "bz_plan_create: n=%d not in {16,24,32,48}", d.n);
  if (!(d.L > 0.0) || !std::isfinite(d.L)) return fail(BZ_ERR_ARG, "bz_plan_create: L must be > 0");
  const double rmax = 4.0 * d.L / (3.0 + std::sqrt(2.0));
  const double R = d.R > 0.0 ? d.R : (std::sqrt(2.0) - 1.0) * d.L;
  if (!(R <= rmax * (1.0 + 1e-12)))
    return fail(BZ_ERR_ARG, "bz_plan_create: R=%.17g exceeds the non-overlap bound 4L/(3+sqrt2)=%.17g", R, rmax);
  if (!(d.gamma >= 0.0 && d.gamma <= 1.0)) return fail(BZ_ERR_ARG, "bz_plan_create: gamma must be in [0,1]");
  if (!(d.kernel_c > 0.0) || !std::isfinite(d.kernel_c)) return fail(BZ_ERR_ARG, "bz_plan_create: kernel_c must be > 0");
  if (d.m < 1 || d.m > 512) return fail(BZ_ERR_ARG, "bz_plan_create: m=%d not in 1..512", d.m);
  if (d.precision != BZ_FP32 && d.precision != BZ_FP64) return fail(BZ_ERR_ARG, "bz_plan_create: bad precision");
  if (d.transform < BZ_XF_AUTO || d.transform > BZ_XF_DFT_GEMM) return fail(BZ_ERR_ARG, "bz_plan_create: bad transform");
  if (d.max_cells < 1) return fail(BZ_ERR_ARG, "bz_plan_create: max_cells must be >= 1");
  if (d.chunks < 0 || d.chunks > d.m + 1) return fail(BZ_ERR_ARG, "bz_plan_create: chunks must be in 0..m+1");
  if (d.slices < 0 || d.slices > 2) return fail(BZ_ERR_ARG, "bz_plan_create: slices must be 0, 1 or 2");
  if (d.dealias != 0 && d.dealias != 1) return fail(BZ_ERR_ARG, "bz_plan_create: dealias must be 0 or 1");
  if (d.dealias && !(d.n == 16 || d.n == 32))
    return fail(BZ_ERR_UNSUPPORTED, "bz_plan_create: dealiased plans need n = 16 or 32 (padded 24 or 48)");

  bz_plan* p = new bz_plan();
  p->d = d;
  p->d.dirs = nullptr;
  p->d.weights = nullptr;
  p->n = d.n;
  p->npts = size_t(d.n) * d.n * d.n;
  p->d.dim = 3;
  p->m = d.m;
  p->m1 = d.m + 1;
  p->L = d.L;
  p->R = R;
  p->d.R = R;
  p->gamma = d.gamma;
  p->C = d.kernel_c;
  p->dv = 2.0 * d.L / d.n;
  p->fp32 = d.precision == BZ_FP32;
  p->project = d.project ? 1 : 0;
  switch (d.dir_kind) {
    case BZ_DIRS_EXPLICIT:
      if (!d.dirs || !d.weights) { delete p; return fail(BZ_ERR_ARG, "bz_plan_create: explicit rule needs dirs and weights"); }
      p->dirs.assign(d.dirs, d.dirs + 3 * d.m);
      p->w.assign(d.weights, d.weights + d.m);
      break;
    case BZ_DIRS_ICOSA6:
      if (d.m != 6) { delete p; return fail(BZ_ERR_ARG, "bz_plan_create: ICOSA6 needs m=6"); }
      rule_icosa6(p->dirs, p->w);
      break;
    case BZ_DIRS_PRODUCT:
      if (d.a1 < 1 || d.a2 < 1 || d.a1 * d.a2 != d.m) { delete p; return fail(BZ_ERR_ARG, "bz_plan_create: PRODUCT needs a1*a2 == m"); }
      rule_product(d.a1, d.a2, p->dirs, p->w);
      break;
    case BZ_DIRS_SPIRAL:
      rule_spiral(d.m, p->dirs, p->w);
      break;
    case BZ_DIRS_DESIGN:
      if (d.m < 2 || d.m > kDesignMaxM) { delete p; return fail(BZ_ERR_ARG, "bz_plan_create: DESIGN needs 2 <= m <= %d", kDesignMaxM); }
      rule_design(d.m, p->dirs, p->w, &p->rule_t);
      break;
    default:
      delete p;
      return fail(BZ_ERR_ARG, "bz_plan_create: bad dir_kind %d", d.dir_kind);
  }
  double wsum = 0.0;
  for (int i = 0; i < d.m; ++i) {
    const double* e = &p->dirs[3 * i];
    const double nrm = std::sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    if (!(std::fabs(nrm - 1.0) <= 1e-12)) { delete p; return fail(BZ_ERR_ARG, "bz_plan_create: direction %d is not a unit vector", i); }
    if (!std::isfinite(p->w[i])) { delete p; return fail(BZ_ERR_ARG, "bz_plan_create: weight %d not finite", i); }
    wsum += p->w[i];
  }
  if (!(std::fabs(wsum - 2.0 * kPi) <= 1e-12)) { delete p; return fail(BZ_ERR_ARG, "bz_plan_create: weights sum to %.17g, not 2*pi", wsum); }

  const bool fused_ok = fused_supported(p->n, p->fp32);
  if (d.transform == BZ_XF_DFT_GEMM && !dft_gemm_supported(p->n, p->fp32)) {
    delete p;
    return fail(BZ_ERR_UNSUPPORTED, "bz_plan_create: no DFT-as-GEMM stage for n=%d precision=%s (FP32, n in 16, 32, 48)",
                d.n, p->fp32 ? "fp32" : "fp64");
  }
  if (d.transform == BZ_XF_FUSED && !fused_ok) {
    delete p;
    return fail(BZ_ERR_UNSUPPORTED, "bz_plan_create: no fused kernel for n=%d precision=%s", d.n, p->fp32 ? "fp32" : "fp64");
  }
  const Strategy sg = resolve_strategy(d, d.max_cells);
  p->transform = sg.transform;
  p->plain_k = sg.transform != BZ_XF_FUSED ? sg.plain_k : 0;
  p->chunks = sg.chunks;
  p->slices = sg.slices;
  if (p->transform == BZ_XF_FUSED && !fused_slices_supported(p->n, p->slices)) {
    delete p;
    return fail(BZ_ERR_UNSUPPORTED, "bz_plan_create: no fused kernel with %d slices for n=%d", p->slices, d.n);
  }
  if (d.dealias) {
    // the padded operator: same box, R, kernel and rule on 3n/2 points, raw Q in the plan precision
    p->transform = BZ_XF_PLAIN;
    p->chunks = 1;
    bz_plan_desc pd = d;
    pd.n = 3 * d.n / 2;
    pd.R = R;
    pd.dir_kind = BZ_DIRS_EXPLICIT;
    pd.dirs = p->dirs.data();
    pd.weights = p->w.data();
    pd.project = 0;
    pd.transform = BZ_XF_AUTO;
    pd.chunks = 0;
    pd.slices = 0;
    pd.dealias = 0;
    const bz_status st = bz_plan_create(&pd, &p->pad);
    if (st != BZ_OK) {
      delete p;
      return st;
    }
  }
  build_tables(p);
  if (!build_gram_inverse(p)) { bz_plan_destroy(p->pad); delete p; return fail(BZ_ERR_NUMERIC, "bz_plan_create: Gram matrix not positive definite"); }
  layout(p);
  *out = p;
  return BZ_OK;
}

bz_status bz_plan_device_bytes(const bz_plan* p, size_t* tables, size_t* ws_fixed, size_t* ws_per_cell) {
  clear_error();
  if (!p) return fail(BZ_ERR_ARG, "bz_plan_device_bytes: null plan");
  if (tables) *tables = p->tables_bytes;
  if (ws_fixed) *ws_fixed = p->ws_fixed;
  if (ws_per_cell) *ws_per_cell = p->ws_per_cell;
  return BZ_OK;
}

bz_status bz_plan_bind(bz_plan* p, void* tables_dev, void* ws_dev, size_t ws_bytes, void* stream) {
  clear_error();
  if (!p || !tables_dev) return fail(BZ_ERR_ARG, "bz_plan_bind: null argument");
  if (!ws_dev && ws_bytes) return fail(BZ_ERR_ARG, "bz_plan_bind: null workspace with ws_bytes > 0");
  if ((uintptr_t(tables_dev) & 255) || (uintptr_t(ws_dev) & 255))
    return fail(BZ_ERR_ARG, "bz_plan_bind: buffers must be 256-byte aligned");
  if (ws_dev && ws_bytes < p->ws_fixed + p->ws_per_cell)
    return fail(BZ_ERR_NOMEM, "bz_plan_bind: workspace %zu bytes < one cell (%zu)", ws_bytes, p->ws_fixed + p->ws_per_cell);
  const bz_status st = upload_tables(p, tables_dev, static_cast<hipStream_t>(stream));
  if (st != BZ_OK) return st;
  if (!ws_dev) {  // tables only (bz_collide_batch_noalloc brings its own workspace)
    p->capacity = 0;
    p->tables_dev = tables_dev;
    p->ws_dev = nullptr;
    p->ws_bytes = 0;
    return BZ_OK;
  }
  const Binding b = make_binding(p, tables_dev, ws_dev, ws_bytes);
  static const int32_t kZero = 0;
  if (hipMemcpy(static_cast<char*>(ws_dev) + b.lay.status_off, &kZero, sizeof(kZero), hipMemcpyHostToDevice) != hipSuccess)
    return fail(BZ_ERR_DEVICE, "bz_plan_bind: clearing the status word failed");
  p->capacity = b.capacity;
  p->ws = b.lay;
  p->tables_dev = tables_dev;
  p->ws_dev = ws_dev;
  p->ws_bytes = ws_bytes;
  return BZ_OK;
}

bz_status bz_plan_sync(bz_plan* p, void* stream) {
  clear_error();
  if (!p) return fail(BZ_ERR_ARG, "bz_plan_sync: null plan");
  if (!p->ws_dev) return fail(BZ_ERR_STATE, "bz_plan_sync: plan not bound");
  if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess)
    return fail(BZ_ERR_DEVICE, "bz_plan_sync: stream synchronisation failed");
  int32_t h = 0;
  char* w = static_cast<char*>(p->ws_dev) + p->ws.status_off;
  if (hipMemcpy(&h, w, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(BZ_ERR_DEVICE, "bz_plan_sync: reading the status word failed");
  if (h != 0) {
    static const int32_t kZero = 0;
    (void)hipMemcpy(w, &kZero, sizeof(kZero), hipMemcpyHostToDevice);
    return fail(BZ_ERR_NUMERIC, "bz_plan_sync: non-finite values in the output of an evaluation since the last sync");
  }
  return BZ_OK;
}

bz_status bz_plan_destroy(bz_plan* p) {
  clear_error();
  if (!p) return BZ_OK;
  for (auto& e : p->evs) (void)hipEventDestroy(e);
  if (p->pad) bz_plan_destroy(p->pad);
  delete p;
  return BZ_OK;
}

bz_status bz_plan_capacity(const bz_plan* p, int32_t* cells) {
  clear_error();
  if (!p || !cells) return fail(BZ_ERR_ARG, "bz_plan_capacity: null argument");
  if (!p->tables_dev) return fail(BZ_ERR_STATE, "bz_plan_capacity: plan not bound");
  *cells = p->ws_dev ? p->capacity : 0;
  return BZ_OK;
}

bz_status bz_plan_transform(const bz_plan* p, int32_t* transform) {
  clear_error();
  if (!p || !transform) return fail(BZ_ERR_ARG, "bz_plan_transform: null argument");
  *transform = p->transform;
  return BZ_OK;
}

bz_status bz_set_tune_table(const char* path) {
  clear_error();
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune_set = path != nullptr;  // NULL: back to BZ_TUNE_TABLE or the shipped table; "": none
  g_tune_path = path ? path : "";
  return BZ_OK;
}

bz_status bz_plan_strategy(const bz_plan* p, int32_t* transform, int32_t* chunks, int32_t* slices) {
  clear_error();
  if (!p) return fail(BZ_ERR_ARG, "bz_plan_strategy: null plan");
  if (transform) *transform = p->transform;
  if (chunks) *chunks = p->transform != BZ_XF_FUSED ? p->pchunk : p->chunks;
  if (slices) *slices = p->slices;
  return BZ_OK;
}

bz_status bz_plan_get_rule(const bz_plan* p, double* dirs, double* weights) {
  clear_error();
  if (!p || !dirs || !weights) return fail(BZ_ERR_ARG, "bz_plan_get_rule: null argument");
  std::memcpy(dirs, p->dirs.data(), sizeof(double) * 3 * p->m);
  std::memcpy(weights, p->w.data(), sizeof(double) * p->m);
  return BZ_OK;
}

bz_status bz_plan_rule_degree(const bz_plan* p, int32_t* t) {
  clear_error();
  if (!p || !t) return fail(BZ_ERR_ARG, "bz_plan_rule_degree: null argument");
  if (p->dim == 2) return fail(BZ_ERR_UNSUPPORTED, "bz_plan_rule_degree: two-dimensional plans use the circle rule");
  *t = p->rule_t > 0 ? p->rule_t : rule_degree(p->dirs, p->w);
  return BZ_OK;
}

bz_status bz_plan_get_multipliers(const bz_plan* p, int32_t pass, double* out) {
  clear_error();
  if (!p || !out) return fail(BZ_ERR_ARG, "bz_plan_get_multipliers: null argument");
  if (pass < 0 || pass > p->m) return fail(BZ_ERR_ARG, "bz_plan_get_multipliers: pass %d not in 0..m", pass);
  const size_t n3 = p->npts;
  std::memcpy(out, &p->mult[size_t(pass) * n3 * 2], sizeof(double) * n3 * 2);
  return BZ_OK;
}

bz_status bz_plan_set_timing(bz_plan* p, int32_t enable) {
  clear_error();
  if (!p) return fail(BZ_ERR_ARG, "bz_plan_set_timing: null plan");
  if (enable && !p->events_ready) {
    p->evs.resize(4 * bz_plan::kTimingSlots);
    for (auto& e : p->evs) {
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return fail(BZ_ERR_DEVICE, "bz_plan_set_timing: %s", hipGetErrorString(r));
    }
    p->events_ready = true;
  }
  p->timing = enable != 0;
  p->timed_calls = 0;
  return BZ_OK;
}

bz_status bz_plan_last_times(bz_plan* p, float* ms, int32_t n) {
  clear_error();
  if (!p || !ms || n < 1) return fail(BZ_ERR_ARG, "bz_plan_last_times: bad argument");
  if (p->timed_calls < 1) return fail(BZ_ERR_STATE, "bz_plan_last_times: no timed call recorded");
  const int calls = std::min(p->timed_calls, bz_plan::kTimingSlots);
  double acc[4] = {0, 0, 0, 0};
  for (int c = 0; c < calls; ++c) {
    hipEvent_t* e = &p->evs[4 * c];
    hipError_t r = hipEventSynchronize(e[3]);
    if (r != hipSuccess) return fail(BZ_ERR_DEVICE, "bz_plan_last_times: %s", hipGetErrorString(r));
    float t[4] = {};
    (void)hipEventElapsedTime(&t[0], e[0], e[1]);
    (void)hipEventElapsedTime(&t[1], e[1], e[2]);
    (void)hipEventElapsedTime(&t[2], e[2], e[3]);
    (void)hipEventElapsedTime(&t[3], e[0], e[3]);
    for (int i = 0; i < 4; ++i) acc[i] += t[i];
  }
  for (int i = 0; i < n && i < 4; ++i) ms[i] = float(acc[i] / calls);
  if (n > 4) ms[4] = float(calls);
  p->timed_calls = 0;
  return BZ_OK;
}

bz_status bz_collide_batch(const bz_plan* p, const void* f, int32_t f_dtype, const int32_t* idx,
                           int32_t ncells, const int32_t* ncells_dev, void* q, int32_t flags,
                           void* stream) {
  clear_error();
  if (!p) return fail(BZ_ERR_ARG, "bz_collide_batch: null plan");
  if (!p->ws_dev) return fail(BZ_ERR_STATE, "bz_collide_batch: plan not bound");
  if (ncells < 0) return fail(BZ_ERR_ARG, "bz_collide_batch: ncells < 0");
  if (ncells == 0) return BZ_OK;
  if (!f || !q) return fail(BZ_ERR_ARG, "bz_collide_batch: null f or q");
  if (f_dtype != BZ_FP32 && f_dtype != BZ_FP64) return fail(BZ_ERR_ARG, "bz_collide_batch: bad f_dtype");
  if (flags & ~int32_t(BZ_SCATTER)) return fail(BZ_ERR_ARG, "bz_collide_batch: unknown flags");
  if ((flags & BZ_SCATTER) && !idx) return fail(BZ_ERR_ARG, "bz_collide_batch: BZ_SCATTER needs idx");
  if (ncells > p->capacity)
    return fail(BZ_ERR_NOMEM, "bz_collide_batch: %d cells exceed the bound capacity %d", ncells, p->capacity);
  Binding b;
  b.tables = p->tables_dev;
  b.ws = p->ws_dev;
  b.capacity = p->capacity;
  b.lay = p->ws;
  return launch_collide(p, b, f, f_dtype == BZ_FP32, idx, ncells, ncells_dev, q,
                        (flags & BZ_SCATTER) != 0, static_cast<hipStream_t>(stream), p->timing);
}

bz_status bz_imex_euler(const bz_plan* p, const bz_imex_desc* d, const double* f, const double* tr,
                        const int32_t* idx, int32_t ncells, const int32_t* ncells_dev, double* f_out,
                        int32_t flags, void* stream) {
  clear_error();
  if (!p) return fail(BZ_ERR_ARG, "bz_imex_euler: null plan");
  if (p->dim == 2) return fail(BZ_ERR_UNSUPPORTED, "bz_imex_euler: three velocity dimensions only");
  if (!d) return fail(BZ_ERR_ARG, "bz_imex_euler: null descriptor");
  if (!p->ws_dev) return fail(BZ_ERR_STATE, "bz_imex_euler: plan not bound");
  if (!(d->dt > 0.0) || !std::isfinite(d->dt)) return fail(BZ_ERR_ARG, "bz_imex_euler: dt must be > 0");
  if (!d->eps_cells && !(d->eps > 0.0)) return fail(BZ_ERR_ARG, "bz_imex_euler: eps must be > 0");
  if (ncells < 0) return fail(BZ_ERR_ARG, "bz_imex_euler: ncells < 0");
  if (flags & ~int32_t(BZ_SCATTER)) return fail(BZ_ERR_ARG, "bz_imex_euler: unknown flags");
  if ((flags & BZ_SCATTER) && !idx) return fail(BZ_ERR_ARG, "bz_imex_euler: BZ_SCATTER needs idx");
  if (ncells == 0) return BZ_OK;
  if (!f || !tr || !f_out) return fail(BZ_ERR_ARG, "bz_imex_euler: null f, tr or f_out");
  if (f_out == f && idx && !(flags & BZ_SCATTER))
    return fail(BZ_ERR_ARG, "bz_imex_euler: in place with idx needs BZ_SCATTER");
  if (!p->project && p->fp32) return fail(BZ_ERR_UNSUPPORTED, "bz_imex_euler: an FP32 plan must project (FP64 output)");
  if (ncells > p->capacity)
    return fail(BZ_ERR_NOMEM, "bz_imex_euler: %d cells exceed the bound capacity %d", ncells, p->capacity);
  Binding b;
  b.tables = p->tables_dev;
  b.ws = p->ws_dev;
  b.capacity = p->capacity;
  b.lay = p->ws;
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* par = reinterpret_cast<double*>(static_cast<char*>(b.ws) + b.lay.par_off);
  bz_status st = launch_imex_params(p->n, p->dv, idx, ncells, ncells_dev, f, tr, d->dt, par, s);
  if (st != BZ_OK) return st;
  bzk::ImexDev im{par, f, tr, d->eps_cells, d->eps, d->dt};
  return launch_collide(p, b, f, 0, idx, ncells, ncells_dev, f_out, (flags & BZ_SCATTER) != 0, s, p->timing, &im);
}

}  // extern "C"
