"""Two-level convergence analysis of Section 3.3 (Lemmas 3.1-3.3, Theorems 3.1-3.2).

TEST INFRASTRUCTURE ONLY (plain FP64 CPU oracle; not part of the product path).

* eq. (equ-03-04): sigma_k are the eigenvalues of M_h^{-1} A_h, here obtained
  from the symmetric-definite pencil (A_h, M_h);
* eq. (equ-03-05): lambda = (2 - tau sigma)/(2 + tau sigma) for the fine
  steps and mu = (2 - tau~ sigma)/(2 + tau~ sigma) for the coarse steps;
* eq. (equ-03-03)/(equ-03-11): the theoretical upper bound (T.U.B.)
  max_w (lam_w)^m |(lam_w)^m - mu''_w| (1 - (mu*_w)^(Nc-1)) / (1 - mu*_w)
  with lam_w = max_j |lambda_w^(j)|, mu''_w = min_k mu_w^(k),
  mu*_w = max_k |mu_w^(k)|;
* Lemma 3.1: after one two-level iteration the C-point error is
  E~_0 = E~_m = 0 and E~_km = sum_{i=0}^{k-2} B_{PsiD,k}^{k-2-i}
  (B_{Psi,(i+2)m}^m - PsiD_{i+2}) B_{Psi,(i+1)m}^m E_im, where
  B_{Psi,s}^l = Psi_s Psi_{s-1} ... Psi_{s-l+1}.
"""
import numpy as np
import scipy.linalg


def generalized_sigma(op):
    """Eigenvalues sigma of M_h^{-1} A_h (dense, small grids)."""
    return scipy.linalg.eigh(op.assembled_A(), op.assembled_M(), eigvals_only=True)


def cn_factor(tau, sigma):
    return (2.0 - tau * sigma) / (2.0 + tau * sigma)


def tub(sigma, t, m):
    """Theoretical upper bound of eq. (equ-03-03) for the paper's coarse propagator (equ-03-02)."""
    t = np.asarray(t, dtype=np.float64)
    N = len(t) - 1
    Nc = N // m
    tau = np.diff(t)
    tc = t[: Nc * m + 1: m]
    tauc = np.diff(tc)
    sigma = np.asarray(sigma)[:, None]
    lam = np.abs(cn_factor(tau[None, :], sigma)).max(axis=1)
    mu = cn_factor(tauc[None, :], sigma)
    mu_min = mu.min(axis=1)
    mu_star = np.abs(mu).max(axis=1)
    lm = lam ** m
    geo = (1.0 - mu_star ** (Nc - 1)) / (1.0 - mu_star)
    return float(np.max(lm * np.abs(lm - mu_min) * geo))


def dense_propagators(op, t, m):
    """Dense fine Psi_n (n = 1..N) and coarse Psi^Delta_j (j = 1..Nc) of eqs. (equ-03-01), (equ-03-02)."""
    M, A = op.assembled_M(), op.assembled_A()
    t = np.asarray(t, dtype=np.float64)

    def psi(tau):
        return np.linalg.solve(M + 0.5 * tau * A, M - 0.5 * tau * A)

    N = len(t) - 1
    fine = [None] + [psi(t[n] - t[n - 1]) for n in range(1, N + 1)]
    tc = t[:: m]
    coarse = [None] + [psi(tc[j] - tc[j - 1]) for j in range(1, len(tc))]
    return fine, coarse


def lemma31_error(fine, coarse, m, E_C):
    """C-point error after one two-level iteration, from the formula of Lemma 3.1.

    fine[s] = Psi_s, coarse[j] = Psi^Delta_j, E_C[k] = error at C-point km (k = 0..Nc).
    """
    n = fine[1].shape[0]
    I = np.eye(n)

    def Bpsi(s, l):                 # Psi_s Psi_{s-1} ... Psi_{s-l+1}
        P = I
        for q in range(s - l + 1, s + 1):
            P = fine[q] @ P
        return P

    def Bcoarse(k, l):              # PsiD_k ... PsiD_{k-l+1}
        P = I
        for q in range(k - l + 1, k + 1):
            P = coarse[q] @ P
        return P

    Nc = len(E_C) - 1
    out = np.zeros_like(E_C)
    for k in range(2, Nc + 1):
        acc = np.zeros(n)
        for i in range(0, k - 1):
            acc += Bcoarse(k, k - 2 - i) @ ((Bpsi((i + 2) * m, m) - coarse[i + 2]) @ (Bpsi((i + 1) * m, m) @ E_C[i]))
        out[k] = acc
    return out
