"""Index identities the FFT's LDS exchange relies on (fft.hpp).

The exchange buffer holds one pad slot every 16 entries, pad(i) = i + i // 16.
The kernels form the padded index of element e of team lane t as
pad(t) + (T + T/16) e when T is a multiple of 16, and a Stockham stage's
write of output m as pad(base) + m NS (+ m NS / 16 when NS is a multiple of
16) when NS R <= 16 or NS is a multiple of 16.  Both are checked here for
every stage of every transform length and radix the library instantiates.
"""

import pytest


def pad(i):
    return i + (i >> 4)


def stages(L, E):
    ns = 1
    while ns < L:
        r = E if L // ns >= E else L // ns
        yield ns, r
        ns *= r


@pytest.mark.parametrize("E", [4, 8, 16])
def test_exchange_index_identities(E):
    for lg in range(4, 14):
        L = 1 << lg
        if L < E:
            continue
        T = L // E
        for ns, r in stages(L, E):
            if ns * r == L:
                continue  # the last stage stays in registers
            if not (ns % 16 == 0 or ns * r <= 16):
                continue  # the general form is used
            for t in range(T):
                for b in range(E // r):
                    j = t + T * b
                    k = j & (ns - 1)
                    base = (j - k) * r + k
                    for m in range(r):
                        extra = m * ns // 16 if ns % 16 == 0 else 0
                        assert pad(base + m * ns) == pad(base) + m * ns + extra, (L, E, ns, r, t, b, m)
        if T % 16 == 0:
            for t in range(T):
                for e in range(E):
                    assert pad(t + T * e) == pad(t) + (T + T // 16) * e


def test_identity_fails_where_not_used():
    # a stage with NS R > 16 and NS not a multiple of 16 does cross groups
    # unaccounted: the condition is needed (span 4, radix 16)
    ns, r, base = 4, 16, 3
    assert any(pad(base + m * ns) != pad(base) + m * ns for m in range(r))
