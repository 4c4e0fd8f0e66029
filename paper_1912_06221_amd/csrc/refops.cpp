// Reference operators of the nodal DG method and the constant operators of the
// affine reconstruction, built in FP64 on the host.
//
// Nodal DG part (section "Nodal discontinuous Galerkin method"): LGL points,
// warp-and-blend triangle nodes (blend parameter 0), orthonormal collapsed
// Jacobi basis psi, Vandermonde V (eq. Vandermonde), Dr = Vr V^-1, Ds,
// M = (V V^T)^-1 and LIFT_f = M^-1 E_f with E_f the 1D LGL mass matrix.
//
// Reconstruction part (subsection "Reconstruction", Algorithm aRDG): the
// 2Np x (N+1)^2 least-squares system with orthonormal test functions on each
// sub-triangle and tensor Legendre unknowns on the square, and its
// pseudo-inverse.  Because the parallelogram map is affine, these combine with
// the diagonal evaluation into operators that are the same for every edge; the
// only per-edge inputs left are the sub-triangle apex (applied as a de
// Casteljau subdivision of Bernstein coefficients) and two gradient factors.
#include "refops.hpp"

#include <cmath>
#include <stdexcept>

namespace ardg {

namespace {

// Orthonormal Jacobi polynomial p_n^{(a,b)} by its three-term recurrence
// x p_n = a_{n+1} p_{n+1} + b_n p_n + a_n p_{n-1}.
double jacobi_rec(double x, int n, double al, double be) {
  const double h0 = std::pow(2.0, al + be + 1.0) * std::tgamma(al + 1.0) * std::tgamma(be + 1.0) /
                    std::tgamma(al + be + 2.0);
  double pm1 = 0.0, p = 1.0 / std::sqrt(h0);
  if (n == 0) return p;
  auto acoef = [&](int k) {
    const double s = 2.0 * k + al + be;
    return 2.0 / s * std::sqrt(k * (k + al + be) * (k + al) * (k + be) / ((s - 1.0) * (s + 1.0)));
  };
  auto bcoef = [&](int k) {
    if (k == 0) return (be - al) / (al + be + 2.0);
    const double s = 2.0 * k + al + be;
    return (be * be - al * al) / (s * (s + 2.0));
  };
  for (int k = 0; k < n; ++k) {
    const double pn = ((x - bcoef(k)) * p - (k > 0 ? acoef(k) * pm1 : 0.0)) / acoef(k + 1);
    pm1 = p;
    p = pn;
  }
  return p;
}

double jacobi_deriv(double x, int n, double al, double be) {
  if (n == 0) return 0.0;
  return std::sqrt(n * (n + al + be + 1.0)) * jacobi_rec(x, n - 1, al + 1.0, be + 1.0);
}

double legendre_raw(double x, int n) {  // unnormalised P_n, P_n(1) = 1
  double pm1 = 1.0, p = x;
  if (n == 0) return 1.0;
  for (int k = 1; k < n; ++k) {
    const double pn = ((2.0 * k + 1.0) * x * p - k * pm1) / (k + 1.0);
    pm1 = p;
    p = pn;
  }
  return p;
}

// Gauss-Legendre points and weights by Newton iteration.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    double z = -std::cos(pi * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      const double pn = legendre_raw(z, n), pn1 = legendre_raw(z, n - 1);
      const double dp = n * (z * pn - pn1) / (z * z - 1.0);
      const double dz = pn / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    const double pn1 = legendre_raw(z, n - 1), pn = legendre_raw(z, n);
    const double dp = n * (z * pn - pn1) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

struct Mode { int i, j; };

std::vector<Mode> modes(int N) {
  std::vector<Mode> m;
  for (int i = 0; i <= N; ++i)
    for (int j = 0; j <= N - i; ++j) m.push_back({i, j});
  return m;
}

void to_collapsed(double r, double s, double& a, double& b) {
  b = s;
  a = (std::fabs(1.0 - s) < 1e-14) ? -1.0 : 2.0 * (1.0 + r) / (1.0 - s) - 1.0;
}

double psi(double r, double s, int i, int j) {
  double a, b;
  to_collapsed(r, s, a, b);
  return std::sqrt(2.0) * jacobi_rec(a, i, 0, 0) * jacobi_rec(b, j, 2.0 * i + 1.0, 0) *
         std::pow(1.0 - b, i);
}

void grad_psi(double r, double s, int i, int j, double& dr, double& ds) {
  double a, b;
  to_collapsed(r, s, a, b);
  const double fa = jacobi_rec(a, i, 0, 0), dfa = jacobi_deriv(a, i, 0, 0);
  const double gb = jacobi_rec(b, j, 2.0 * i + 1.0, 0), dgb = jacobi_deriv(b, j, 2.0 * i + 1.0, 0);
  const double pw1 = (i >= 1) ? std::pow(1.0 - b, i - 1) : 0.0;
  const double pw = std::pow(1.0 - b, i);
  dr = 2.0 * std::sqrt(2.0) * dfa * gb * pw1;
  ds = std::sqrt(2.0) * (dfa * (1.0 + a) * gb * pw1 + fa * dgb * pw - i * fa * gb * pw1);
}

Mat vandermonde(int N, const std::vector<double>& r, const std::vector<double>& s) {
  auto md = modes(N);
  Mat V((int)r.size(), (int)md.size());
  for (size_t p = 0; p < r.size(); ++p)
    for (size_t q = 0; q < md.size(); ++q) V((int)p, (int)q) = psi(r[p], s[p], md[q].i, md[q].j);
  return V;
}

// Tensor Legendre basis of Q_N on [-1,1]^2, mode q = a*(N+1) + b -> L_a(R) L_b(S).
void qbasis(int N, double R, double S, double* val, double* dR, double* dS) {
  const int n1 = N + 1;
  double LR[16], LS[16], dLR[16], dLS[16];
  for (int a = 0; a <= N; ++a) {
    LR[a] = jacobi_rec(R, a, 0, 0);
    LS[a] = jacobi_rec(S, a, 0, 0);
    dLR[a] = jacobi_deriv(R, a, 0, 0);
    dLS[a] = jacobi_deriv(S, a, 0, 0);
  }
  for (int a = 0; a <= N; ++a)
    for (int b = 0; b <= N; ++b) {
      const int q = a * n1 + b;
      if (val) val[q] = LR[a] * LS[b];
      if (dR) dR[q] = dLR[a] * LS[b];
      if (dS) dS[q] = LR[a] * dLS[b];
    }
}

double factorial(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

}  // namespace

double jacobi_p(double x, int n, double alpha, double beta) { return jacobi_rec(x, n, alpha, beta); }

// LGL points as the roots of P_{N+1} - P_{N-1} (proportional to (1-x^2) P'_N),
// Newton from Chebyshev-Lobatto guesses; q' = (2N+1) P_N.
std::vector<double> lgl_points(int N) {
  std::vector<double> x(N + 1);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i <= N; ++i) {
    double z = -std::cos(pi * i / N);
    if (i == 0 || i == N) { x[i] = z; continue; }
    for (int it = 0; it < 100; ++it) {
      const double q = legendre_raw(z, N + 1) - legendre_raw(z, N - 1);
      const double dq = (2.0 * N + 1.0) * legendre_raw(z, N);
      const double dz = q / dq;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = z;
  }
  return x;
}

RefOps build_refops(int N, bool* rank_ok) {
  RefOps o;
  o.N = N;
  o.Np = (N + 1) * (N + 2) / 2;
  o.Nfp = N + 1;
  o.Mp = (N + 1) * (N + 1);
  const int Np = o.Np, Nfp = o.Nfp, Mp = o.Mp;
  o.lgl = lgl_points(N);

  // ---- warp-and-blend nodes in barycentric form ----------------------------
  std::vector<double> eq(N + 1);
  for (int k = 0; k <= N; ++k) eq[k] = -1.0 + 2.0 * k / N;
  auto warp = [&](double r) {
    double w = 0.0;
    for (int k = 0; k <= N; ++k) {
      double l = 1.0;
      for (int m = 0; m <= N; ++m)
        if (m != k) l *= (r - eq[m]) / (eq[k] - eq[m]);
      w += (o.lgl[k] - eq[k]) * l;
    }
    return w;
  };
  o.r.resize(Np);
  o.s.resize(Np);
  for (int j = 0; j <= N; ++j)
    for (int i = 0; i <= N - j; ++i) {
      const double lam0[3] = {double(N - i - j) / N, double(i) / N, double(j) / N};
      double lam[3] = {lam0[0], lam0[1], lam0[2]};
      const int pairs[3][2] = {{0, 1}, {1, 2}, {2, 0}};
      for (auto& pr : pairs) {
        const double la = lam0[pr[0]], lb = lam0[pr[1]];
        const double rr = lb - la;
        const double den = 1.0 - rr * rr;
        const double wf = (std::fabs(den) > 1e-12) ? warp(rr) / den : 0.0;
        const double d = 4.0 * la * lb * wf;
        lam[pr[0]] -= 0.5 * d;
        lam[pr[1]] += 0.5 * d;
      }
      const int n = lattice_index(N, i, j);
      o.r[n] = -lam[0] + lam[1] - lam[2];
      o.s[n] = -lam[0] - lam[1] + lam[2];
    }

  // ---- modal basis and reference matrices ----------------------------------
  o.V = vandermonde(N, o.r, o.s);
  o.Vinv = inverse(o.V);
  auto md = modes(N);
  Mat Vr(Np, Np), Vs(Np, Np);
  for (int p = 0; p < Np; ++p)
    for (int q = 0; q < Np; ++q) grad_psi(o.r[p], o.s[p], md[q].i, md[q].j, Vr(p, q), Vs(p, q));
  o.Dr = matmul(Vr, o.Vinv);
  o.Ds = matmul(Vs, o.Vinv);
  o.Minv = matmul(o.V, transpose(o.V));
  o.M = inverse(o.Minv);

  // face nodes, counter-clockwise, from the lattice
  for (int k = 0; k <= N; ++k) {
    o.fmask[0][k] = lattice_index(N, k, 0);          // s = -1, r increasing
    o.fmask[1][k] = lattice_index(N, N - k, k);      // hypotenuse, s increasing
    o.fmask[2][k] = lattice_index(N, 0, N - k);      // r = -1, s decreasing
  }
  // 1D mass matrix on the LGL points: M1 = (V1 V1^T)^-1
  Mat V1(Nfp, Nfp);
  for (int p = 0; p < Nfp; ++p)
    for (int n = 0; n <= N; ++n) V1(p, n) = jacobi_rec(o.lgl[p], n, 0, 0);
  const Mat M1 = inverse(matmul(V1, transpose(V1)));
  Mat E(Np, 3 * Nfp);
  for (int f = 0; f < 3; ++f)
    for (int a = 0; a < Nfp; ++a)
      for (int b = 0; b < Nfp; ++b) E(o.fmask[f][a], f * Nfp + b) = M1(a, b);
  o.LIFT = matmul(o.Minv, E);

  // ---- node reorderings: rotated lattice (i,j) -> own lattice --------------
  for (int j = 0; j <= N; ++j)
    for (int i = 0; i <= N - j; ++i) {
      const int n = lattice_index(N, i, j);
      o.rot[0][n] = lattice_index(N, j, N - i - j);  // w = (v3, v1, v2)
      o.rot[1][n] = n;                               // w = (v1, v2, v3)
      o.rot[2][n] = lattice_index(N, N - i - j, i);  // w = (v2, v3, v1)
    }

  // ---- Bernstein basis on I (multi-index (N-i-j, i, j) in lattice order) ---
  o.Bv = Mat(Np, Np);
  for (int p = 0; p < Np; ++p) {
    const double l1 = -(o.r[p] + o.s[p]) / 2.0, l2 = (o.r[p] + 1.0) / 2.0, l3 = (o.s[p] + 1.0) / 2.0;
    for (int j = 0; j <= N; ++j)
      for (int i = 0; i <= N - j; ++i) {
        const int a1 = N - i - j;
        const double c = factorial(N) / (factorial(a1) * factorial(i) * factorial(j));
        o.Bv(p, lattice_index(N, i, j)) = c * std::pow(l1, a1) * std::pow(l2, i) * std::pow(l3, j);
      }
  }
  o.N2B = inverse(o.Bv);
  o.B2psi = matmul(o.Vinv, o.Bv);

  // ---- least-squares system on the parallelogram ---------------------------
  // Duffy map of a Gauss-Legendre tensor rule: int_I f = int int f (1-b)/2 da db
  const int nq = 2 * N + 3;
  std::vector<double> gx, gw;
  gauss_legendre(nq, gx, gw);
  o.A = Mat(2 * Np, Mp);
  std::vector<double> ph1(Mp), ph2(Mp);
  for (int ia = 0; ia < nq; ++ia)
    for (int ib = 0; ib < nq; ++ib) {
      const double a = gx[ia], b = gx[ib];
      const double rr = 0.5 * (1.0 + a) * (1.0 - b) - 1.0, ss = b;
      const double w = gw[ia] * gw[ib] * 0.5 * (1.0 - b);
      qbasis(N, rr, ss, ph1.data(), nullptr, nullptr);
      qbasis(N, -rr, -ss, ph2.data(), nullptr, nullptr);
      for (int m = 0; m < Np; ++m) {
        const double pm = psi(rr, ss, md[m].i, md[m].j) * w;
        for (int q = 0; q < Mp; ++q) {
          o.A(m, q) += pm * ph1[q];
          o.A(Np + m, q) += pm * ph2[q];
        }
      }
    }
  bool ok = pinv_tall(o.A, o.Rop, 1e-10, &o.recon_cond);
  if (rank_ok) *rank_ok = ok;
  if (!ok) return o;

  // ---- evaluation of Q_N at the diagonal nodes d_j = (t_j, -t_j), t: +1 -> -1
  Mat E0(Nfp, Mp), ER(Nfp, Mp), ES(Nfp, Mp);
  for (int jn = 0; jn < Nfp; ++jn) {
    const double t = o.lgl[N - jn];
    qbasis(N, t, -t, &E0(jn, 0), &ER(jn, 0), &ES(jn, 0));
  }
  // Q_N at the sub-triangle nodes: frame 1 = square frame, frame 2 = reflected
  Mat Phi1(Np, Mp), Phi2(Np, Mp);
  for (int p = 0; p < Np; ++p) {
    qbasis(N, o.r[p], o.s[p], &Phi1(p, 0), nullptr, nullptr);
    qbasis(N, -o.r[p], -o.s[p], &Phi2(p, 0), nullptr, nullptr);
  }
  const Mat Bblk = blockdiag(o.B2psi, o.B2psi);
  const Mat Vblk = blockdiag(o.Vinv, o.Vinv);
  const Mat RB = matmul(o.Rop, Bblk);   // Bernstein sub-triangle data -> Q_N coefficients
  const Mat RV = matmul(o.Rop, Vblk);   // nodal sub-triangle data -> Q_N coefficients
  o.KR = matmul(ER, RB);
  o.KS = matmul(ES, RB);
  o.recon_grad_nodal = vcat(matmul(ER, RV), matmul(ES, RV));
  o.KV = matmul(E0, RB);
  o.recon_value_nodal = matmul(E0, RV);

  // Algorithm 1: separate u~ onto the sub-triangles, differentiate in each
  // sub-triangle frame, reconstruct again from the nodal data (no second
  // projection), evaluate on the diagonal.
  const Mat R1 = sub(o.Rop, 0, 0, Mp, Np), R2 = sub(o.Rop, 0, Np, Mp, Np);
  const Mat G1 = matmul(matmul(E0, R1), o.Vinv);   // side-1 nodal data -> diagonal values
  const Mat G2 = matmul(matmul(E0, R2), o.Vinv);
  auto alg1 = [&](const Mat& G, const Mat& Dm, const Mat& Phi, const Mat& Rin) {
    return matmul(matmul(matmul(G, Dm), Phi), Rin);
  };
  o.U1R = alg1(G1, o.Dr, Phi1, RB);
  o.U1S = alg1(G1, o.Ds, Phi1, RB);
  o.U2R = alg1(G2, o.Dr, Phi2, RB);
  o.U2S = alg1(G2, o.Ds, Phi2, RB);
  o.alg1_nodal = vcat(vcat(alg1(G1, o.Dr, Phi1, RV), alg1(G1, o.Ds, Phi1, RV)),
                      vcat(alg1(G2, o.Dr, Phi2, RV), alg1(G2, o.Ds, Phi2, RV)));

  // Algorithm 1 with a nodal coefficient: separation + reference gradient on
  // each sub-triangle, and each sub-triangle's part of the second
  // reconstruction on the diagonal
  o.TR1 = matmul(matmul(o.Dr, Phi1), RB);
  o.TS1 = matmul(matmul(o.Ds, Phi1), RB);
  o.TR2 = matmul(matmul(o.Dr, Phi2), RB);
  o.TS2 = matmul(matmul(o.Ds, Phi2), RB);
  o.G1 = G1;
  o.G2 = G2;

  // Algorithm 2: a constant coefficient is the same constant on the
  // sub-triangle (all nodal values equal), so its reconstruction at the
  // diagonal is G1 1 (side 1) and G2 1 (side 2)
  o.alg2_w1.assign(Nfp, 0.0);
  o.alg2_w2.assign(Nfp, 0.0);
  for (int j = 0; j < Nfp; ++j)
    for (int p = 0; p < Np; ++p) {
      o.alg2_w1[j] += G1(j, p);
      o.alg2_w2[j] += G2(j, p);
    }

  // Boundary faces: the ghost's sub-triangle data is minus side 1's data with
  // (r, s) swapped, i.e. Bernstein multi-index (a1, a2, a3) -> (a1, a3, a2).
  Mat Sw(Np, Np);
  for (int j = 0; j <= N; ++j)
    for (int i = 0; i <= N - j; ++i) Sw(lattice_index(N, i, j), lattice_index(N, j, i)) = 1.0;
  auto fold = [&](const Mat& K) {
    return add(sub(K, 0, 0, K.r, Np), matmul(sub(K, 0, Np, K.r, Np), Sw), -1.0);
  };
  o.KBR = fold(o.KR);
  o.KBS = fold(o.KS);
  o.UBR = add(fold(o.U1R), fold(o.U2R), -1.0);
  o.UBS = add(fold(o.U1S), fold(o.U2S), -1.0);
  return o;
}

}  // namespace ardg
