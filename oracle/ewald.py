"""The potential tensor M of regularized charges in a periodic box (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Parity unpinned: none
-- every function here is pinned by the CPU tests (Wigner self-potential,
NaCl Madelung constant, split-parameter independence, agreement of the two
independent evaluations, closed-form real-space kernels).

Definition (section "Background / Grand Potential Matrix derivation",
Fourier form of the potential tensor; generalised from the paper's shell form
factor j0(ka) to a per-particle form factor s_hat):

    M_ab = 1/(eps V) * sum_{k != 0} s_hat_a(k) s_hat_b(k) exp(i k.(x_a - x_b)) / k^2

with k = 2 pi n / L over all integer n != 0.  The k = 0 term is dropped
(electroneutrality through the surface at infinity).  Two profiles:

* Gaussian charges of standard deviation sigma: s_hat(k) = exp(-sigma^2 k^2 / 2),
  so s_hat_a s_hat_b = exp(-s^2 k^2 / 2) with s^2 = sigma_a^2 + sigma_b^2, and in
  free space M(r) = erf(r / (sqrt(2) s)) / (4 pi eps r).
* Uniformly charged shells of radius a (the paper's own regularization):
  s_hat = j0(ka); in free space M(r) = 1/(4 pi eps r) for r >= 2a and
  (4a - r)/(16 pi eps a^2) for r < 2a (the printed real-space form with its
  stray factors of a removed; this is the shell-shell potential).

Two independent evaluations are provided:

``potential_matrix_ksum``  the definition above summed directly over k
                           (possible only for wide Gaussians in small boxes);
``potential_matrix`` etc.  an Ewald split (section "Spectrally-accurate Ewald
                           summation", splitting function h = exp(-k^2/4 xi^2)):
    M_ab = sum_n R_ab(|x_a - x_b + n L|)          (n=0, a=b: R_aa(0))
         + 1/(eps V) sum_{k != 0} h(k)/k^2 cos(k.(x_a - x_b))
         - R_hat_ab(0)/(eps V)
  with R = M_free - erf(xi r)/(4 pi eps r), i.e. the regularization lives in
  the real-space part and the wave-space part is that of point charges.
  R_hat_ab(0) = lim_{k->0} (s_hat_a s_hat_b - h)/k^2 is the k=0 value of the
  Fourier transform of R, which the image sum of R contains and the
  definition excludes.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf, erfc

FOUR_PI = 4.0 * math.pi
SQRT_PI = math.sqrt(math.pi)


# --------------------------------------------------------------------------
# Regularization profiles: real-space kernel R, its derivative, self value,
# and the k = 0 constant R_hat(0).
# --------------------------------------------------------------------------


class Gaussian:
    """Gaussian charges; ``s2`` is sigma_a^2 + sigma_b^2 of the pair."""

    name = "gauss"

    @staticmethod
    def pair_s2(sig_a, sig_b):
        return sig_a * sig_a + sig_b * sig_b

    @staticmethod
    def free(r, s2, eps=1.0):
        b = 1.0 / np.sqrt(2.0 * s2)
        return erf(b * r) / (FOUR_PI * eps * r)

    @staticmethod
    def real(r, s2, xi, eps=1.0):
        b = 1.0 / np.sqrt(2.0 * s2)
        return (erfc(xi * r) - erfc(b * r)) / (FOUR_PI * eps * r)

    @staticmethod
    def real_deriv(r, s2, xi, eps=1.0):
        """dR/dr."""
        b = 1.0 / np.sqrt(2.0 * s2)
        t1 = -(2.0 * xi / SQRT_PI) * np.exp(-(xi * r) ** 2) * r - erfc(xi * r)
        t2 = -(2.0 * b / SQRT_PI) * np.exp(-(b * r) ** 2) * r - erfc(b * r)
        return (t1 - t2) / (FOUR_PI * eps * r * r)

    @staticmethod
    def real_self(s2, xi, eps=1.0):
        """lim_{r->0} R(r)."""
        b = 1.0 / np.sqrt(2.0 * s2)
        return (2.0 / SQRT_PI) * (b - xi) / (FOUR_PI * eps)

    @staticmethod
    def rhat0(s2, xi):
        return 1.0 / (4.0 * xi * xi) - 0.5 * s2

    @staticmethod
    def shat2(k, s2):
        return np.exp(-0.5 * s2 * k * k)

    @staticmethod
    def reach(s2_max):
        """Distance beyond which the regularization is invisible (1e-17)."""
        return math.sqrt(2.0 * s2_max) * 6.0


class Shell:
    """Uniformly charged spherical shells, all of radius ``a``."""

    name = "shell"

    def __init__(self, a):
        self.a = float(a)

    def pair_s2(self, sig_a, sig_b):  # widths are ignored: one radius for all
        return np.zeros(np.broadcast(sig_a, sig_b).shape)

    def free(self, r, s2=None, eps=1.0):
        a = self.a
        r = np.asarray(r, dtype=np.float64)
        out = np.empty_like(r)
        far = r >= 2 * a
        out[far] = 1.0 / (FOUR_PI * eps * r[far])
        out[~far] = (4 * a - r[~far]) / (16.0 * math.pi * eps * a * a)
        return out

    def real(self, r, s2, xi, eps=1.0):
        r = np.asarray(r, dtype=np.float64)
        return self.free(r, eps=eps) - erf(xi * r) / (FOUR_PI * eps * r)

    def real_deriv(self, r, s2, xi, eps=1.0):
        a = self.a
        r = np.asarray(r, dtype=np.float64)
        dfree = np.where(r >= 2 * a, -1.0 / (FOUR_PI * eps * r * r),
                         -1.0 / (16.0 * math.pi * eps * a * a))
        derf = ((2.0 * xi / SQRT_PI) * np.exp(-(xi * r) ** 2) * r - erf(xi * r)) / (FOUR_PI * eps * r * r)
        return dfree - derf

    def real_self(self, s2, xi, eps=1.0):
        return (1.0 / (FOUR_PI * self.a) - xi / (2.0 * math.pi ** 1.5)) / eps + 0.0 * s2

    def rhat0(self, s2, xi):
        return 1.0 / (4.0 * xi * xi) - self.a ** 2 / 3.0 + 0.0 * s2

    def shat2(self, k, s2=None):
        ka = k * self.a
        j0 = np.where(ka == 0, 1.0, np.sin(ka) / np.where(ka == 0, 1.0, ka))
        return j0 * j0

    def reach(self, s2_max=0.0):
        return 2.0 * self.a


class ShellPaperSplit(Shell):
    """Shells of radius ``a`` with the paper's own placement of the
    regularization in the split (section "Spectrally-accurate Ewald
    summation", the splitting equation): the form factor j0^2(ka) multiplies
    both parts, so the wave part is h(k) j0^2(ka) / k^2 and the real-space
    part the inverse transform of (1 - h(k)) j0^2(ka) / k^2, for which the
    section "Real-space sum" prints a closed form.  The printed Heaviside term
    is read with the sign of its second part flipped,
    -(1/(4 pi r) - (4a - r)/(16 pi a^2)) H(2a - r): only with that sign does the
    closed form equal the inverse transform (and M stay continuous at r = 2a).
    The potential tensor M itself is the same as with the other split."""

    name = "shell_paper"

    def __init__(self, a):
        super().__init__(a)
        self.real_shift = 2.0 * self.a   # the real part decays like erfc(xi (r - 2a))

    def real(self, r, s2, xi, eps=1.0):
        a = self.a
        r = np.asarray(r, dtype=np.float64)
        sp, sm = r + 2 * a, r - 2 * a
        pi32 = math.pi ** 1.5
        out = (-sp / (32 * pi32 * a * a * xi * r) * np.exp(-(sp * xi) ** 2)
               - sm / (32 * pi32 * a * a * xi * r) * np.exp(-(sm * xi) ** 2)
               + 1.0 / (16 * pi32 * a * a * xi) * np.exp(-(r * xi) ** 2)
               + (2 * xi * xi * sp * sp + 1) / (64 * math.pi * a * a * xi * xi * r) * erfc(sp * xi)
               + (2 * xi * xi * sm * sm + 1) / (64 * math.pi * a * a * xi * xi * r) * erfc(sm * xi)
               - (2 * xi * xi * r * r + 1) / (32 * math.pi * a * a * xi * xi * r) * erfc(r * xi))
        heav = np.where(r < 2 * a, 1.0 / (FOUR_PI * r) - (4 * a - r) / (16 * math.pi * a * a), 0.0)
        return (out - heav) / eps

    @staticmethod
    def _g1(s, xi):
        """d/ds of g(s) = (2 xi^2 s^2 + 1) erfc(xi s) / (64 pi xi^2)
        - s exp(-xi^2 s^2) / (32 pi^1.5 xi), the function whose second
        difference (g(r+2a) + g(r-2a) - 2 g(r)) / (a^2 r) is the printed sum of
        erfc and exponential terms: g'(s) = (s erfc(xi s) - exp(-xi^2 s^2) /
        (sqrt(pi) xi)) / (16 pi)."""
        return (s * erfc(xi * s) - np.exp(-(xi * s) ** 2) / (SQRT_PI * xi)) / (16 * math.pi)

    @staticmethod
    def _g(s, xi):
        return ((2 * xi * xi * s * s + 1) * erfc(xi * s) / (64 * math.pi * xi * xi)
                - s * np.exp(-(xi * s) ** 2) / (32 * math.pi ** 1.5 * xi))

    def real_deriv(self, r, s2, xi, eps=1.0):
        a = self.a
        r = np.asarray(r, dtype=np.float64)
        G = self._g(r + 2 * a, xi) + self._g(r - 2 * a, xi) - 2 * self._g(r, xi)
        G1 = self._g1(r + 2 * a, xi) + self._g1(r - 2 * a, xi) - 2 * self._g1(r, xi)
        d = G1 / (a * a * r) - G / (a * a * r * r)
        dheav = np.where(r < 2 * a, -1.0 / (FOUR_PI * r * r) + 1.0 / (16 * math.pi * a * a), 0.0)
        return (d - dheav) / eps

    def real_self(self, s2, xi, eps=1.0):
        a = self.a
        v = (1 - math.exp(-4 * a * a * xi * xi)) / (8 * math.pi ** 1.5 * a * a * xi) + \
            math.erfc(2 * a * xi) / (FOUR_PI * a)
        return v / eps + 0.0 * s2

    def rhat0(self, s2, xi):
        return 1.0 / (4.0 * xi * xi) + 0.0 * s2

    def wave_form(self, kk):
        ka = np.sqrt(kk) * self.a
        j0 = np.where(ka == 0, 1.0, np.sin(ka) / np.where(ka == 0, 1.0, ka))
        return j0 * j0


def _wave_form(profile, kk):
    """Extra factor of the wave-space Green's function: 1 when the whole
    regularization sits in the real-space kernel."""
    f = getattr(profile, "wave_form", None)
    return 1.0 if f is None else f(kk)


def _profile(profile):
    return Gaussian() if profile is None else profile


# --------------------------------------------------------------------------
# Geometry helpers
# --------------------------------------------------------------------------


def volume(box):
    return float(np.prod(box))


def min_image(d, box):
    return d - box * np.round(d / box)


def image_shifts(r_o, box):
    """Integer image vectors n that can bring a minimum-image displacement
    within r_o."""
    nmax = [int(math.ceil(r_o / L + 0.5)) for L in box]
    g = [np.arange(-m, m + 1) for m in nmax]
    n = np.stack(np.meshgrid(*g, indexing="ij"), -1).reshape(-1, 3)
    return n.astype(np.float64) * np.asarray(box)


def k_half_space(box, k_max):
    """Wave vectors k = 2 pi n / L with 0 < |k| <= k_max, one of each +-k
    pair (the sum over the full set is twice the real part of this one)."""
    box = np.asarray(box, dtype=np.float64)
    nmax = [int(math.floor(k_max * L / (2 * math.pi))) for L in box]
    g = [np.arange(-m, m + 1) for m in nmax]
    n = np.stack(np.meshgrid(*g, indexing="ij"), -1).reshape(-1, 3)
    pos = (n[:, 0] > 0) | ((n[:, 0] == 0) & (n[:, 1] > 0)) | \
          ((n[:, 0] == 0) & (n[:, 1] == 0) & (n[:, 2] > 0))
    n = n[pos]
    k = 2 * math.pi * n / box
    kk = np.einsum("ij,ij->i", k, k)
    keep = kk <= k_max * k_max
    return k[keep], kk[keep]


def default_cutoffs(xi, s2_max, profile, tol=1e-16):
    """Real- and wave-space cutoffs that make each truncated tail < tol."""
    lt = math.sqrt(math.log(1.0 / tol))
    r_o = max(lt / xi + getattr(profile, "real_shift", 0.0), profile.reach(s2_max)) * 1.05
    k_o = 2.0 * xi * lt * 1.05
    return r_o, k_o


# --------------------------------------------------------------------------
# Plain definition: the Fourier sum itself (no split).
# --------------------------------------------------------------------------


def potential_matrix_ksum(pos, sig, box, eps=1.0, rel_tail=1e-18):
    """M by the defining Fourier sum for Gaussian charges.

    Feasible only when the narrowest pair width s_min makes
    exp(-s_min^2 k^2 / 2) negligible at a k_max the box can afford.
    """
    pos = np.asarray(pos, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    s2 = Gaussian.pair_s2(sig[:, None], sig[None, :])
    k_max = math.sqrt(2.0 * math.log(1.0 / rel_tail) / s2.min())
    k, kk = k_half_space(box, k_max)
    M = np.zeros((len(pos), len(pos)))
    V = volume(box)
    for c0 in range(0, len(k), 20000):
        kc, kkc = k[c0:c0 + 20000], kk[c0:c0 + 20000]
        ph = pos @ kc.T                                 # (n, nk)
        C, S = np.cos(ph), np.sin(ph)
        for a in range(len(pos)):
            w = np.exp(-0.5 * s2[a][:, None] * kkc[None, :]) / kkc[None, :]   # (n, nk)
            M[a] += 2.0 * np.sum(w * (C[a][None, :] * C + S[a][None, :] * S), axis=1)
    return M / (eps * V)


# --------------------------------------------------------------------------
# Ewald split.
# --------------------------------------------------------------------------


def _real_block(pos_t, sig_t, pos_s, sig_s, box, xi, eps, profile, r_o,
                want_field=False, q_s=None):
    """Real-space part for a block of targets: the matrix block (and the
    gradient block) or, if q_s is given, the potential and field.

    A coincident pair (r = 0: a particle with itself, n = 0) takes the limit
    value R(0), which is the self term; its gradient there is zero."""
    shifts = image_shifts(r_o, box)
    d0 = min_image(pos_t[:, None, :] - pos_s[None, :, :], box)      # (nt, ns, 3)
    s2 = profile.pair_s2(sig_t[:, None], sig_s[None, :])
    Mr = np.zeros(d0.shape[:2])
    Fr = np.zeros(d0.shape) if want_field else None
    tiny = 1e-12 * r_o
    for sh in shifts:
        d = d0 + sh
        r = np.sqrt(np.einsum("ijk,ijk->ij", d, d))
        m = (r < r_o) & (r >= tiny)
        if m.any():
            rr = r[m]
            Mr[m] += profile.real(rr, s2[m], xi, eps)
            if want_field:
                dR = profile.real_deriv(rr, s2[m], xi, eps)
                Fr[m] += (dR / rr)[:, None] * d[m]            # grad_t R
        z = r < tiny
        if z.any():
            Mr[z] += profile.real_self(s2[z], xi, eps)
    if q_s is None:
        return Mr, Fr
    phi = Mr @ q_s
    E = None if not want_field else -np.einsum("ijk,j->ik", Fr, q_s)
    return phi, E


def _rhat0_dot(profile, sig_t, sig_s, q_s, xi):
    """sum_s R_hat_ts(0) q_s for every target (chunked over targets)."""
    out = np.zeros(len(sig_t))
    step = max(1, 4_000_000 // max(len(sig_s), 1))
    for t0 in range(0, len(sig_t), step):
        s2 = profile.pair_s2(sig_t[t0:t0 + step, None], sig_s[None, :])
        out[t0:t0 + step] = profile.rhat0(s2, xi) @ q_s
    return out


def potential_matrix(pos, sig, box, xi, eps=1.0, profile=None, tol=1e-16):
    """Dense M (n x n) of one particle set, by the Ewald split."""
    profile = _profile(profile)
    pos = np.asarray(pos, dtype=np.float64)
    sig = np.asarray(sig, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    n = len(pos)
    s2 = profile.pair_s2(sig[:, None], sig[None, :])
    r_o, k_o = default_cutoffs(xi, float(np.max(s2)) if n else 0.0, profile, tol)
    V = volume(box)
    M = np.zeros((n, n))
    chunk = max(1, 2_000_000 // max(n, 1))
    for t0 in range(0, n, chunk):
        t1 = min(n, t0 + chunk)
        Mr, _ = _real_block(pos[t0:t1], sig[t0:t1], pos, sig, box, xi, eps, profile, r_o)
        M[t0:t1] = Mr
    k, kk = k_half_space(box, k_o)
    g = np.exp(-kk / (4 * xi * xi)) / kk * _wave_form(profile, kk)
    for c0 in range(0, len(k), 8192):
        ph = pos @ k[c0:c0 + 8192].T
        C, S = np.cos(ph), np.sin(ph)
        gc = g[c0:c0 + 8192]
        M += (2.0 / (eps * V)) * ((C * gc) @ C.T + (S * gc) @ S.T)
    M -= profile.rhat0(s2, xi) / (eps * V)
    return M


def potential_field(pos_t, sig_t, pos_s, sig_s, q_s, box, xi, eps=1.0, profile=None,
                    want_field=True, tol=1e-16):
    """Potential phi_t = sum_s M_ts q_s and field E_t = -sum_s grad_t M_ts q_s
    at targets, matrix-free.  A target that coincides with a source (the
    particle itself) picks up the self term M_tt."""
    profile = _profile(profile)
    pos_t = np.asarray(pos_t, dtype=np.float64)
    pos_s = np.asarray(pos_s, dtype=np.float64)
    sig_t = np.asarray(sig_t, dtype=np.float64)
    sig_s = np.asarray(sig_s, dtype=np.float64)
    q_s = np.asarray(q_s, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    nt, ns = len(pos_t), len(pos_s)
    s2max = float(np.max(sig_t) ** 2 + np.max(sig_s) ** 2) if nt and ns else 0.0
    r_o, k_o = default_cutoffs(xi, s2max, profile, tol)
    V = volume(box)
    phi = np.zeros(nt)
    E = np.zeros((nt, 3))
    chunk = max(1, 1_000_000 // max(ns, 1))
    for t0 in range(0, nt, chunk):
        t1 = min(nt, t0 + chunk)
        p, e = _real_block(pos_t[t0:t1], sig_t[t0:t1], pos_s, sig_s, box, xi, eps, profile,
                           r_o, want_field=want_field, q_s=q_s)
        phi[t0:t1] += p
        if want_field:
            E[t0:t1] += e
    k, kk = k_half_space(box, k_o)
    g = np.exp(-kk / (4 * xi * xi)) / kk * _wave_form(profile, kk)
    for c0 in range(0, len(k), 4096):
        kc, gc = k[c0:c0 + 4096], g[c0:c0 + 4096]
        Cs = np.zeros(len(kc))
        Ss = np.zeros(len(kc))
        for s0 in range(0, ns, 16384):
            ph = pos_s[s0:s0 + 16384] @ kc.T
            Cs += q_s[s0:s0 + 16384] @ np.cos(ph)
            Ss += q_s[s0:s0 + 16384] @ np.sin(ph)
        for t0 in range(0, nt, 16384):
            ph = pos_t[t0:t0 + 16384] @ kc.T
            Ct, St = np.cos(ph), np.sin(ph)
            phi[t0:t0 + 16384] += (2.0 / (eps * V)) * ((Ct * Cs + St * Ss) @ gc)
            if want_field:
                # E = -grad_t: d/dx_t cos(k.(x_t-x_s)) = -k sin(k.(x_t-x_s))
                E[t0:t0 + 16384] += (2.0 / (eps * V)) * (((St * Cs - Ct * Ss) * gc) @ kc)
    # constant: -(1/(eps V)) sum_s R_hat_ts(0) q_s
    if ns:
        phi -= _rhat0_dot(profile, sig_t, sig_s, q_s, xi) / (eps * V)
    return phi, E


def cross_matrix(pos_t, sig_t, pos_s, sig_s, box, xi, eps=1.0, profile=None, tol=1e-16):
    """Dense M_ts between two disjoint particle sets."""
    profile = _profile(profile)
    ns = len(pos_s)
    out = np.zeros((len(pos_t), ns))
    for j in range(ns):
        e = np.zeros(ns)
        e[j] = 1.0
        out[:, j], _ = potential_field(pos_t, sig_t, pos_s, sig_s, e, box, xi, eps, profile,
                                       want_field=False, tol=tol)
    return out
