"""Regularised integrals S(alpha, beta, gamma) by direct quadrature (oracle).

Test infrastructure only.

Eq. (sila): S(alpha, beta, gamma) = R int_0^inf x^alpha exp(beta x - gamma x^2) dx,
where for alpha <= -1 "R" keeps the epsilon-independent part of the
integral from epsilon to infinity (singular terms in epsilon are dropped).
This module evaluates it with mpmath by Taylor subtraction: with
g(x) = exp(beta x - gamma x^2) = sum_k g_k x^k,
  R int_0^inf x^a g = int_0^1 x^a (g - sum_{k<=K} g_k x^k) dx
                      + sum_{k<=K, a+k != -1} g_k / (a+k+1)
                      + int_1^inf x^a g dx,
with K = ceil(-a) - 1 (so the subtracted integrand is integrable).  The
term a+k = -1 (integer alpha only) contributes log(1) - log(eps); its
singular log(eps) is dropped and its finite part on [eps, 1] is 0.
"""
import mpmath as mp


def taylor_g(beta, gamma, K):
    """Coefficients g_k of exp(beta x - gamma x^2), k = 0..K."""
    beta, gamma = mp.mpf(beta), mp.mpf(gamma)
    out = []
    for k in range(K + 1):
        s = mp.mpf(0)
        for l in range(k // 2 + 1):
            s += beta ** (k - 2 * l) * (-gamma) ** l / (mp.factorial(k - 2 * l) * mp.factorial(l))
        out.append(s)
    return out


def S_finite_part(alpha, beta, gamma, dps=40):
    """S(alpha, beta, gamma) of Eq. (sila), with the finite part for alpha <= -1.

    On [0, 1] the integrand is expanded in the Taylor series of
    exp(beta x - gamma x^2) and integrated term by term: every term
    g_k x^(alpha+k) contributes g_k / (alpha + k + 1), its finite part (for
    alpha + k + 1 = 0 the finite part of int_eps^1 dx/x is 0).  The series
    converges like g_k (factorially); its terms alternate and grow up to about
    e^{beta^2/(4 gamma)} or e^{|beta|}, so it is summed with 60 extra digits.
    The rest, int_1^inf, is a regular integral.  (Subtracting the Taylor
    polynomial inside a quadrature instead loses all digits when -alpha is
    more than about 2.)"""
    with mp.workdps(dps):
        a = mp.mpf(alpha)
        beta, gamma = mp.mpf(beta), mp.mpf(gamma)
        if a > -1:
            return mp.quad(lambda x: x ** a * mp.exp(beta * x - gamma * x * x), [0, 1, mp.inf])
    with mp.workdps(dps + 60):
        a = mp.mpf(alpha)
        b, c = mp.mpf(beta), mp.mpf(gamma)
        # g_k by (k+1) g_{k+1} = b g_k - 2 c g_{k-1}
        g0, g1 = mp.mpf(1), b
        val = mp.mpf(0)
        k, small = 0, 0
        while True:
            gk = g0 if k == 0 else g1
            if a + k + 1 != 0:
                val += gk / (a + k + 1)
            if k >= 1:
                g0, g1 = g1, (b * g1 - 2 * c * g0) / (k + 1)
            small = small + 1 if (k > 10 and abs(gk) < mp.mpf(10) ** (-(dps + 30)) * (1 + abs(val))) else 0
            if small > 4 or k > 20000:
                break
            k += 1
        val += mp.quad(lambda x: x ** a * mp.exp(b * x - c * x * x), [1, 2, 4, mp.inf])
    with mp.workdps(dps):
        return +val
