"""Independent checks ("pins") for C(n) and its factorisation.

Each function here computes a property of C(n) = (2n)!/(n!(n+1)!) (Sec. 1) by
a route that shares nothing with either implementation under test: brute
force, Kummer's theorem, Lucas' theorem, product formulas modulo a prime,
2-adic products and the log-gamma function.  They pin the CPU oracle first
and, at sizes the oracle cannot reach, the device result.
"""
from __future__ import annotations

import math

import numpy as np


# ---------------------------------------------------------------- small n
def dyck_bruteforce(n: int) -> int:
    """Count Dyck paths of semilength n by enumerating every valid path."""
    count = 0

    def walk(up: int, down: int):
        nonlocal count
        if up == n and down == n:
            count += 1
            return
        if up < n:
            walk(up + 1, down)
        if down < up:
            walk(up, down + 1)

    walk(0, 0)
    return count


def dyck_dp(n: int) -> int:
    """Count lattice paths of 2n unit steps that never go below zero and end at 0."""
    ways = [1] + [0] * (2 * n + 1)
    for _ in range(2 * n):
        nxt = [0] * (2 * n + 2)
        for h, w in enumerate(ways):
            if not w:
                continue
            nxt[h + 1] += w
            if h > 0:
                nxt[h - 1] += w
        ways = nxt
    return ways[0]


# ---------------------------------------------------------------- exponents
def vp_int(x: int, p: int) -> int:
    v = 0
    while x % p == 0:
        x //= p
        v += 1
    return v


def kummer_exponent(n: int, p: int) -> int:
    """v_p(C(n)) by Kummer's theorem: v_p(binom(2n, n)) is the number of carries
    when adding n + n in base p; C(n) = binom(2n, n)/(n+1)."""
    carries, c, x = 0, 0, n
    while x or c:
        d = x % p
        s = 2 * d + c
        c = 1 if s >= p else 0
        carries += c
        x //= p
    return carries - vp_int(n + 1, p)


# ---------------------------------------------------------------- residues
def _binom_small_mod(a: int, b: int, q: int) -> int:
    """binom(a, b) mod prime q for 0 <= a, b < q (product formula)."""
    if b < 0 or b > a:
        return 0
    b = min(b, a - b)
    num, den = 1, 1
    for i in range(1, b + 1):
        num = num * (a - b + i) % q
        den = den * i % q
    return num * pow(den, q - 2, q) % q


def lucas_binom_mod(N: int, K: int, q: int) -> int:
    """binom(N, K) mod prime q by Lucas' theorem."""
    r = 1
    while N or K:
        r = r * _binom_small_mod(N % q, K % q, q) % q
        if r == 0:
            return 0
        N //= q
        K //= q
    return r


def catalan_mod_prime_lucas(n: int, q: int) -> int:
    """C(n) mod prime q using C(n) = binom(2n, n) - binom(2n, n+1)."""
    return (lucas_binom_mod(2 * n, n, q) - lucas_binom_mod(2 * n, n + 1, q)) % q


def catalan_mod_composite(n: int, factors) -> int:
    """C(n) mod prod(factors) for distinct primes, by Lucas per prime and CRT."""
    m = 1
    for f in factors:
        m *= f
    x = 0
    for f in factors:
        r = catalan_mod_prime_lucas(n, f)
        mf = m // f
        x = (x + r * mf * pow(mf, -1, f)) % m
    return x


def catalan_mod_prime_product(n: int, q: int) -> int:
    """C(n) mod a prime q > 2n as (prod_{k=n+2}^{2n} k) * (n!)^{-1} mod q."""
    assert q > 2 * n
    num = 1
    for k in range(n + 2, 2 * n + 1):
        num = num * k % q
    den = 1
    for k in range(2, n + 1):
        den = den * k % q
    return num * pow(den, q - 2, q) % q


def catalan_low64(n: int) -> int:
    """C(n) mod 2^64: 2^{v_2} times the odd parts of (2n)!/(n!(n+1)!) mod 2^64,
    with v_2(C(n)) = popcount(n+1) - 1."""
    mod = 1 << 64
    v2 = bin(n + 1).count("1") - 1
    num = 1
    for k in range(n + 2, 2 * n + 1):
        while k % 2 == 0:
            k //= 2
        num = num * k % mod
    den = 1
    for k in range(2, n + 1):
        while k % 2 == 0:
            k //= 2
        den = den * k % mod
    odd = num * pow(den, -1, mod) % mod
    return (odd << v2) % mod


# ---------------------------------------------------------------- size pins
def log_pins(n: int, dps: int = 60):
    """bit length, decimal digits and the top 64 bits (limbs L-1, L-2 joined) of
    C(n) from the log-gamma function at `dps` digits.  Returns
    (bits, digits, top64, top64_margin): margin is the distance of the real
    value from the nearest integer, so callers can tell a safe floor."""
    import mpmath

    mpmath.mp.dps = dps
    if n <= 1:
        return 1, 1, None, None
    lnC = mpmath.loggamma(2 * n + 1) - mpmath.loggamma(n + 1) - mpmath.loggamma(n + 2)
    log2C = lnC / mpmath.log(2)
    log10C = lnC / mpmath.log(10)
    bits = int(mpmath.floor(log2C)) + 1
    digits = int(mpmath.floor(log10C)) + 1
    L = (bits + 31) // 32
    top = None
    margin = None
    if L >= 2:
        t = mpmath.power(2, log2C - 32 * (L - 2))
        top = int(mpmath.floor(t))
        margin = float(min(t - top, top + 1 - t))
    return bits, digits, top, margin


def limbs_int(limbs) -> int:
    a = np.ascontiguousarray(limbs, dtype="<u4")
    return int.from_bytes(a.tobytes(), "little")


def limbs_mod(limbs, q: int) -> int:
    """Value of LE uint32 limbs modulo q (Horner from the top)."""
    a = np.ascontiguousarray(limbs, dtype=np.uint64)
    r = 0
    base = (1 << 32) % q
    # Horner in chunks keeps the Python loop short for large inputs
    for x in a[::-1].tolist():
        r = (r * base + x) % q
    return r


def limbs_mod_small(limbs, q: int, chunk: int = 1 << 20) -> int:
    """Value of LE uint32 limbs modulo a small q (q < 2^20), vectorised:
    per chunk sum(limb_i * B^i) mod q with B = 2^32 mod q, chunks joined by
    Horner steps with B^chunk."""
    assert q < (1 << 20)
    x = np.ascontiguousarray(limbs, dtype=np.uint64) % q
    base = (1 << 32) % q
    pw = np.empty(chunk, dtype=np.uint64)
    v = 1
    for i in range(chunk):
        pw[i] = v
        v = v * base % q
    step = pow(base, chunk, q)
    acc = 0
    nch = (len(x) + chunk - 1) // chunk
    for c in range(nch - 1, -1, -1):
        part = x[c * chunk:(c + 1) * chunk]
        r = int(np.sum((part * pw[: len(part)]) % q) % q)
        acc = (acc * step + r) % q
    return acc


def catalan_comb(n: int) -> int:
    return math.comb(2 * n, n) // (n + 1)


# ---------------------------------------------------------------- factorial ratios
def legendre_digits(n: int, p: int) -> int:
    """v_p(n!) = (n - s_p(n)) / (p - 1), s_p the base-p digit sum (Legendre's
    digit-sum form; independent of the repeated-division sums)."""
    s, m = 0, n
    while m:
        s += m % p
        m //= p
    return (n - s) // (p - 1)


def ratio_exponents(num, den, primes_list):
    """v_p(prod num! / prod den!) for every p in primes_list, by digit sums."""
    return [sum(legendre_digits(a, p) for a in num) - sum(legendre_digits(b, p) for b in den) for p in primes_list]


def ratio_value(num, den=()):
    """prod num! / prod den! with Python integers (exact division checked)."""
    import math

    top = 1
    for a in num:
        top *= math.factorial(a)
    bot = 1
    for b in den:
        bot *= math.factorial(b)
    q, r = divmod(top, bot)
    if r:
        raise ValueError("not an integer")
    return q


def limbs_mod_vec(limbs, m: int, chunk: int = 4096) -> int:
    """Value of LE uint32 limbs modulo m < 2^31: per chunk sum((limb_i mod m) *
    (2^32i mod m) mod m), chunks joined by Horner steps with 2^(32 chunk)."""
    assert 1 < m < (1 << 31)
    x = np.ascontiguousarray(limbs, dtype=np.uint64) % m
    base = (1 << 32) % m
    pw = np.empty(chunk, dtype=np.uint64)
    v = 1
    for i in range(chunk):
        pw[i] = v
        v = v * base % m
    step = pow(base, chunk, m)
    pad = (-len(x)) % chunk
    xs = np.concatenate([x, np.zeros(pad, dtype=np.uint64)]).reshape(-1, chunk)
    part = ((xs * pw[None, :]) % m).sum(axis=1) % m
    acc = 0
    for c in range(len(part) - 1, -1, -1):
        acc = (acc * step + int(part[c])) % m
    return acc


def decimal_group_residues(text, rows: int = 1 << 22) -> tuple:
    """From decimal text (a torch uint8 tensor of ASCII digits, any device):
    the nine-digit groups g_i (least significant first) reduced as
    (sum g_i mod 10^9-1, sum (-1)^i g_i mod 10^9+1, g_0), i.e. the number
    modulo 10^9-1, 10^9+1 and 10^9.  Works through the groups in slices."""
    import torch

    pad = (-text.numel()) % 9
    t = torch.cat([torch.full((pad,), 48, dtype=torch.uint8, device=text.device), text]).reshape(-1, 9)
    ng = t.shape[0]
    w = torch.tensor([10**k for k in range(8, -1, -1)], dtype=torch.int64, device=text.device)
    m1, m2 = 10**9 - 1, 10**9 + 1
    s1 = s2 = 0
    for r0 in range(0, ng, rows):
        d = t[r0:r0 + rows].to(torch.int64) - 48
        assert bool(((d >= 0) & (d <= 9)).all())
        g = (d * w).sum(dim=1)                 # most significant first
        idx = ng - 1 - (r0 + torch.arange(g.numel(), device=g.device))   # group index from the bottom
        s1 = (s1 + int(g.sum().item())) % m1
        sign = 1 - 2 * (idx & 1)
        s2 = (s2 + int((g * sign).sum().item())) % m2
    g0 = int(((t[-1].to(torch.int64) - 48) * w).sum().item())
    return s1, s2, g0


def limbs_mod_torch(t, m: int, chunk: int = 4096) -> int:
    """limbs_mod_vec for a torch int32 limb tensor (on its own device)."""
    import torch

    assert 1 < m < (1 << 31)
    x = t.to(torch.int64) & 0xFFFFFFFF
    pad = (-x.numel()) % chunk
    x = torch.cat([x, torch.zeros(pad, dtype=torch.int64, device=x.device)]).reshape(-1, chunk) % m
    base = (1 << 32) % m
    pw, v = [], 1
    for _ in range(chunk):
        pw.append(v)
        v = v * base % m
    pwt = torch.tensor(pw, dtype=torch.int64, device=x.device)
    part = ((x * pwt[None, :]) % m).sum(dim=1).remainder(m).cpu().tolist()
    step = pow(base, chunk, m)
    acc = 0
    for c in range(len(part) - 1, -1, -1):
        acc = (acc * step + part[c]) % m
    return acc


def leading_decimal(n: int, k: int = 30, dps: int = 80):
    """The first k decimal digits of C(n) from log-gamma at `dps` digits, and
    the distance of 10^(frac(log10 C) + k - 1) from the nearest integer (a
    safe floor needs a margin well above 10^(k - dps + 12))."""
    import mpmath

    mpmath.mp.dps = dps
    lnC = mpmath.loggamma(2 * n + 1) - mpmath.loggamma(n + 1) - mpmath.loggamma(n + 2)
    log10C = lnC / mpmath.log(10)
    f = log10C - mpmath.floor(log10C)
    v = mpmath.power(10, f + k - 1)
    lead = int(mpmath.floor(v))
    return str(lead), float(min(v - lead, lead + 1 - v))


def catalan_valuation(n: int, p: int) -> int:
    """v_p(C(n)) = v_p((2n)!) - 2 v_p(n!) - v_p(n+1) (Legendre)."""
    def vf(m):
        s, q = 0, m
        while q:
            q //= p
            s += q
        return s
    m, vn1 = n + 1, 0
    while m % p == 0:
        m //= p
        vn1 += 1
    return vf(2 * n) - 2 * vf(n) - vn1
