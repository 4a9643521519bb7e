"""Pure-Python big-integer definitions used to pin the C oracle.

TEST INFRASTRUCTURE ONLY. Each function is the textbook definition of a quantity, written with
Python integers and no shortcuts, so that the C oracle can be checked against something other
than itself. Sizes are tiny (N <= 256 for the quadratic definitions).
"""
from __future__ import annotations

from typing import List, Sequence


def is_prime(n: int) -> bool:
    """Miller-Rabin with the 7-base set that is deterministic below 2^64 (Jaeschke/Sinclair)."""
    if n < 2:
        return False
    small = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47]
    for p in small:
        if n % p == 0:
            return n == p
    d, r = n - 1, 0
    while d % 2 == 0:
        d //= 2
        r += 1
    for a in (2, 325, 9375, 28178, 450775, 9780504, 1795265022):
        a %= n
        if a == 0:
            continue
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(r - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def brv(x: int, bits: int) -> int:
    return int(format(x, "0%db" % bits)[::-1], 2) if bits else 0


def ntt_definition(a: Sequence[int], q: int, psi: int) -> List[int]:
    """NTT(a)[i] = sum_k a_k psi^{(2 brv(i) + 1) k} mod q, quadratic time."""
    n = len(a)
    bits = n.bit_length() - 1
    out = []
    for i in range(n):
        e = 2 * brv(i, bits) + 1
        w = pow(psi, e, q)
        acc, wk = 0, 1
        for k in range(n):
            acc += a[k] * wk
            wk = wk * w % q
        out.append(acc % q)
    return out


def negacyclic_product(a: Sequence[int], b: Sequence[int], q: int) -> List[int]:
    """Schoolbook product in Z_q[X]/(X^N + 1)."""
    n = len(a)
    out = [0] * n
    for i in range(n):
        for j in range(n):
            k = i + j
            if k < n:
                out[k] += a[i] * b[j]
            else:
                out[k - n] -= a[i] * b[j]
    return [x % q for x in out]


def automorph_definition(a: Sequence[int], g: int, q: int) -> List[int]:
    """a(X^g) reduced mod X^N + 1, by substituting X^k -> X^{gk} and folding with X^N = -1."""
    n = len(a)
    out = [0] * n
    for k in range(n):
        e = g * k
        sign = -1 if (e // n) % 2 else 1
        out[e % n] += sign * a[k]
    return [x % q for x in out]


def crt(residues: Sequence[int], moduli: Sequence[int]) -> int:
    """The unique x in [0, prod moduli) with x = r_i mod m_i."""
    m = 1
    for mi in moduli:
        m *= mi
    x = 0
    for r, mi in zip(residues, moduli):
        mh = m // mi
        x += r * mh * pow(mh, -1, mi)
    return x % m


def centered(x: int, m: int) -> int:
    x %= m
    return x - m if x > (m - 1) // 2 else x


def round_div(x: int, d: int) -> int:
    """Nearest integer to x / d for odd d (no ties)."""
    return (x - centered(x, d)) // d
