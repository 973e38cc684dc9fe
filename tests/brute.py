"""Independent 50-digit brute force of the LOO likelihood (test helper).

Written from the definitions only (scaled Gaussian kernel, Section 2;
eq. (1); eq. (3) with the A_i expansion of Section 3.2; the Epanechnikov
kernel of Section 4 in its multivariate radial form): every kernel value is
formed in full, constants included, with Python's ``decimal`` arithmetic and
its own exp/ln, and summed directly -- no log-sum-exp, no shifts.  It shares
nothing with the C oracle and is used only on tiny inputs.
"""
from decimal import Decimal, getcontext

getcontext().prec = 50
PI = Decimal("3.14159265358979323846264338327950288419716939937510582097494459")
SQRT_2PI = (2 * PI).sqrt()


def _d(v):
    return Decimal(repr(float(v)))


def gauss_kernel(delta, h):
    """Product Gaussian K_h(delta) = prod_k exp(-(d_k/h_k)^2/2) / (h_k sqrt(2 pi))."""
    out = Decimal(1)
    for dk, hk in zip(delta, h):
        t = dk / hk
        out *= (-(t * t) / 2).exp() / (hk * SQRT_2PI)
    return out


def ell(x, y, hx, hy, criterion="cond"):
    """Per-point LOO log-likelihood as a list of Decimals."""
    n = len(x)
    X = [[_d(v) for v in row] for row in x]
    Y = [[_d(v) for v in row] for row in y]
    HX = [_d(v) for v in hx]
    HY = [_d(v) for v in hy]
    out = []
    for i in range(n):
        num = Decimal(0)
        den = Decimal(0)
        for j in range(n):
            if j == i:
                continue
            kx = gauss_kernel([a - b for a, b in zip(X[i], X[j])], HX)
            ky = gauss_kernel([a - b for a, b in zip(Y[i], Y[j])], HY)
            num += kx * ky
            den += kx
        if criterion == "cond":
            out.append((num / den).ln())
        else:
            out.append((num / (n - 1)).ln())
    return out


def density(x, y, hx, hy, xq, yq):
    """f(yq | xq) of eq. (1) over all training points, as a Decimal."""
    X = [[_d(v) for v in row] for row in x]
    Y = [[_d(v) for v in row] for row in y]
    HX = [_d(v) for v in hx]
    HY = [_d(v) for v in hy]
    XQ = [_d(v) for v in xq]
    YQ = [_d(v) for v in yq]
    num = Decimal(0)
    den = Decimal(0)
    for i in range(len(X)):
        kx = gauss_kernel([a - b for a, b in zip(XQ, X[i])], HX)
        num += kx * gauss_kernel([a - b for a, b in zip(YQ, Y[i])], HY)
        den += kx
    return num / den


def unit_ball_volume(d):
    """Volume of the unit d-ball by the recurrence V_d = (2 pi / d) V_{d-2},
    V_0 = 1, V_1 = 2."""
    v = [Decimal(1), Decimal(2)]
    for k in range(2, d + 1):
        v.append(2 * PI / k * v[k - 2])
    return v[d]


def epan_kernel(delta, h):
    """Radial Epanechnikov K_h(delta) = (d+2)/(2 V_d) / prod_k h_k *
    max(0, 1 - sum_k (d_k/h_k)^2)."""
    d = len(delta)
    u = Decimal(0)
    scale = Decimal(1)
    for dk, hk in zip(delta, h):
        t = dk / hk
        u += t * t
        scale *= hk
    if u >= 1:
        return Decimal(0)
    return (Decimal(d + 2) / (2 * unit_ball_volume(d))) / scale * (1 - u)


def ell_epan(x, y, hx, hy, criterion="cond"):
    """Per-point LOO log-likelihood with the Epanechnikov kernel, as floats
    (-inf where no j has a non-zero product kernel)."""
    n = len(x)
    X = [[_d(v) for v in row] for row in x]
    Y = [[_d(v) for v in row] for row in y]
    HX = [_d(v) for v in hx]
    HY = [_d(v) for v in hy]
    out = []
    for i in range(n):
        num = Decimal(0)
        den = Decimal(0)
        for j in range(n):
            if j == i:
                continue
            kx = epan_kernel([a - b for a, b in zip(X[i], X[j])], HX)
            ky = epan_kernel([a - b for a, b in zip(Y[i], Y[j])], HY)
            num += kx * ky
            den += kx
        if num == 0:
            out.append(float("-inf"))
        elif criterion == "cond":
            out.append(float((num / den).ln()))
        else:
            out.append(float((num / (n - 1)).ln()))
    return out


def cond_mean(x, y, hx, xq):
    """E[y | xq] = sum_i K_hx(xq - x_i) y_i / sum_i K_hx(xq - x_i) (first y
    column), every kernel value formed in full."""
    X = [[_d(v) for v in row] for row in x]
    Y = [_d(row[0]) for row in y]
    HX = [_d(v) for v in hx]
    XQ = [_d(v) for v in xq]
    num = Decimal(0)
    den = Decimal(0)
    for i in range(len(X)):
        k = gauss_kernel([a - b for a, b in zip(XQ, X[i])], HX)
        num += k * Y[i]
        den += k
    return float(num / den)


def loo_density_curve(x, y, hx, hy, i, ypts):
    """f^{-i}(y | x_i) of eq. (1) with point i left out, at each row of ypts
    [m, dy], in float64 with scipy's normal density (an independent
    evaluation for quadrature pins)."""
    import numpy as np
    from scipy.stats import norm
    x, y = np.asarray(x, float), np.asarray(y, float)
    hx, hy = np.asarray(hx, float), np.asarray(hy, float)
    keep = np.arange(len(x)) != i
    w = np.prod(norm.pdf((x[i] - x[keep]) / hx) / hx, axis=1)
    ky = np.prod(norm.pdf((np.asarray(ypts, float)[:, None, :] - y[keep][None, :, :]) / hy) / hy,
                 axis=2)
    return ky @ w / w.sum()
