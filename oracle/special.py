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
    with mp.workdps(dps):
        a = mp.mpf(alpha)
        beta, gamma = mp.mpf(beta), mp.mpf(gamma)
        g = lambda x: mp.exp(beta * x - gamma * x * x)
        if a > -1:
            return mp.quad(lambda x: x ** a * g(x), [0, 1, mp.inf])
        K = int(mp.ceil(-a)) - 1
        gk = taylor_g(beta, gamma, K)

        def sub(x):
            return x ** a * (g(x) - sum(gk[k] * x ** k for k in range(K + 1)))

        val = mp.quad(sub, [0, 1])
        for k in range(K + 1):
            if a + k + 1 != 0:
                val += gk[k] / (a + k + 1)
        val += mp.quad(lambda x: x ** a * g(x), [1, mp.inf])
        return val
