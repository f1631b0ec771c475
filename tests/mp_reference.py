"""Independent 50-digit evaluation of the Hawkes rate and compensator.

Written from the *rate functions* of Sec. 2.1 evaluated at arbitrary points
(x, t), not from the pair form of the likelihood equation, so that it checks
the oracle's pair terms, constants and indicators from a different angle.
Only for tiny N (pure-Python loops).
"""
import mpmath as mp

mp.mp.dps = 50


def phi_vec(z):
    """D-variate standard normal density of the vector z."""
    d = len(z)
    return (2 * mp.pi) ** (-mp.mpf(d) / 2) * mp.exp(-sum(zi * zi for zi in z) / 2)


def phi1(z):
    return mp.exp(-z * z / 2) / mp.sqrt(2 * mp.pi)


def background_rate(x, t, X, T, p):
    """mu(x, t) = mu0/(tau_x^D tau_t) sum_n phi((x-x_n)/tau_x) phi((t-t_n)/tau_t) I[t != t_n]."""
    mu0, tx, tt = mp.mpf(p[0]), mp.mpf(p[1]), mp.mpf(p[2])
    d = len(x)
    s = mp.mpf(0)
    for xn, tn in zip(X, T):
        if t != tn:
            s += phi_vec([(mp.mpf(a) - mp.mpf(b)) / tx for a, b in zip(x, xn)]) * phi1((mp.mpf(t) - mp.mpf(tn)) / tt)
    return mu0 / (tx ** d * tt) * s


def excitation_rate(x, t, X, T, p):
    """xi(x, t) = theta omega/h^D sum_{t_n < t} exp(-omega (t - t_n)) phi((x - x_n)/h)."""
    th, om, h = mp.mpf(p[3]), mp.mpf(p[4]), mp.mpf(p[5])
    d = len(x)
    s = mp.mpf(0)
    for xn, tn in zip(X, T):
        if tn < t:
            s += mp.exp(-om * (mp.mpf(t) - mp.mpf(tn))) * phi_vec([(mp.mpf(a) - mp.mpf(b)) / h for a, b in zip(x, xn)])
    return th * om / h ** d * s


def rates_at_events(X, T, p):
    return [background_rate(X[n], T[n], X, T, p) + excitation_rate(X[n], T[n], X, T, p) for n in range(len(T))]


def compensator_by_time_quadrature(X, T, p):
    """Integral over [0, t_N] of the spatially integrated rate.  The spatial
    integral of each normalised Gaussian kernel is 1, leaving
    mu0/tau_t sum_n phi((t-t_n)/tau_t) + theta omega sum_{t_n<t} exp(-omega (t-t_n)),
    which is integrated numerically in time (split at the event times)."""
    mu0, tt, th, om = mp.mpf(p[0]), mp.mpf(p[2]), mp.mpf(p[3]), mp.mpf(p[4])
    tN = max(mp.mpf(v) for v in T)

    def f(t):
        s = mp.mpf(0)
        for tn in T:
            s += mu0 / tt * phi1((t - mp.mpf(tn)) / tt)
            if mp.mpf(tn) < t:
                s += th * om * mp.exp(-om * (t - mp.mpf(tn)))
        return s

    pts = sorted(set([mp.mpf(0)] + [mp.mpf(v) for v in T if 0 < v < tN] + [tN]))
    return mp.quad(f, pts)


def loglik(X, T, p):
    lam = rates_at_events(X, T, p)
    return sum(mp.log(v) for v in lam) - compensator_by_time_quadrature(X, T, p)
