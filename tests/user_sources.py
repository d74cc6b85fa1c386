"""Decomposition functions written as user source text (C, `real` = the
run's floating type).  The same text is compiled by the GPU library (hipRTC)
and by the oracle (host C compiler).

LIN3, CTM and RD restate the built-in systems with the oracle's own operation
order, so the oracle gives bitwise the built-in results for them.  SINE is a
nonlinear chain that is neither cooperative nor linear:
    f_i = -a x_i + b sin(x_{i-1}) + c u,   b > 0, c > 0,
with the tight decomposition of the scalar sine: for the lower argument y and
the upper argument yh of the neighbour, the minimum of sin over [y, yh] when
y <= yh, else its maximum over [yh, y].  It is nondecreasing in y,
nonincreasing in yh and equals sin(y) on the diagonal.
"""

LIN3 = r"""
REACH_DEVICE real lin3_pos(real a) { return a > 0.0 ? a : 0.0; }
REACH_DEVICE real lin3_neg(real a) { return a < 0.0 ? a : 0.0; }
REACH_DEVICE real reach_d(real xm, real x, real xp, real hm, real h, real hp, real u, real uh,
                          const real* prm, long long i, long long n)
{
    const real aL = prm[0], aD = prm[1], aR = prm[2], b = prm[3];
    return aD * x + lin3_pos(aL) * xm + lin3_neg(aL) * hm + lin3_pos(aR) * xp
         + lin3_neg(aR) * hp + lin3_pos(b) * u + lin3_neg(b) * uh;
}
"""

CTM = r"""
REACH_DEVICE real ctm_min(real a, real b) { return a < b ? a : b; }
REACH_DEVICE real ctm_flux(real yi, real yn, int last, const real* prm)
{
    const real v = prm[0], w = prm[1], c = prm[2], q = prm[3];
    if (last) return ctm_min(v * yi, q);
    return ctm_min(ctm_min(v * yi, w * (c - yn)), q);
}
REACH_DEVICE real reach_d(real xm, real x, real xp, real hm, real h, real hp, real u, real uh,
                          const real* prm, long long i, long long n)
{
    const real fin = (i == 0) ? 0.0 : ctm_flux(xm, x, 0, prm);
    return fin - ctm_flux(x, xp, i == n - 1, prm);
}
"""

RD = r"""
REACH_DEVICE real reach_d(real xm, real x, real xp, real hm, real h, real hp, real u, real uh,
                          const real* prm, long long i, long long n)
{
    const real sp = prm[0];
    const real lap = (xm - 2.0 * x + xp) / (sp * sp);
    return lap - x * x * x + u;
}
"""

# RD in the built-in kernel's fused operation order, with prm[0] = 1/h^2 and
# prm[1] = 2/h^2: the user kernel then runs the same arithmetic per cell as
# the built-in one, so the two agree bit for bit.
RD_FUSED = r"""
REACH_DEVICE real reach_d(real xm, real x, real xp, real hm, real h, real hp, real u, real uh,
                          const real* prm, long long i, long long n)
{
    return fma(xm + xp, prm[0], fma(-x, fma(x, x, prm[1]), u));
}
"""

SINE = r"""
/* extremes of sin over [lo, hi]: -1 / +1 when a trough / crest lies inside */
REACH_DEVICE real sine_min(real lo, real hi)
{
    const real twopi = 6.283185307179586, trough = 4.71238898038469;
    const real c = trough + ceil((lo - trough) / twopi) * twopi;
    if (c <= hi) return -1.0;
    return fmin(sin(lo), sin(hi));
}
REACH_DEVICE real sine_max(real lo, real hi)
{
    const real twopi = 6.283185307179586, crest = 1.5707963267948966;
    const real c = crest + ceil((lo - crest) / twopi) * twopi;
    if (c <= hi) return 1.0;
    return fmax(sin(lo), sin(hi));
}
REACH_DEVICE real reach_d(real xm, real x, real xp, real hm, real h, real hp, real u, real uh,
                          const real* prm, long long i, long long n)
{
    const real a = prm[0], b = prm[1], c = prm[2];
    const real s = (xm <= hm) ? sine_min(xm, hm) : sine_max(hm, xm);
    return -a * x + b * s + c * u;
}
"""

SINE_PRM = (1.0, 0.8, 0.5)
