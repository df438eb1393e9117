"""Independent big-integer arithmetic used by the oracle's pin tests: direct
definitions (O(n^2) DFT, Horner evaluation, Gauss-Jordan inverse, the inverse
Poseidon permutation) computed with Python integers."""
P = 0xFFFFFFFF00000001
D_INV7 = pow(7, -1, P - 1)          # x -> x^D_INV7 inverts x -> x^7 (gcd(7, p-1) = 1)


def root(log_n):
    return pow(7, (P - 1) >> log_n, P)


def dft(x, inverse=False):
    n = len(x)
    w = root(n.bit_length() - 1)
    if inverse:
        w = pow(w, P - 2, P)
    out = [sum(x[j] * pow(w, j * k, P) for j in range(n)) % P for k in range(n)]
    if inverse:
        ninv = pow(n, P - 2, P)
        out = [v * ninv % P for v in out]
    return out


def horner(coeffs, x):
    acc = 0
    for c in reversed(coeffs):
        acc = (acc * x + c) % P
    return acc


def mat_inv(m):
    n = len(m)
    a = [[m[i][j] % P for j in range(n)] + [1 if i == j else 0 for j in range(n)] for i in range(n)]
    for col in range(n):
        piv = next(r for r in range(col, n) if a[r][col] != 0)
        a[col], a[piv] = a[piv], a[col]
        inv = pow(a[col][col], P - 2, P)
        a[col] = [v * inv % P for v in a[col]]
        for r in range(n):
            if r != col and a[r][col]:
                f = a[r][col]
                a[r] = [(vr - f * vc) % P for vr, vc in zip(a[r], a[col])]
    return [row[n:] for row in a]


def det(m):
    """Determinant mod p by Gaussian elimination with row swaps."""
    a = [[v % P for v in row] for row in m]
    n = len(a)
    d = 1
    for col in range(n):
        piv = next((r for r in range(col, n) if a[r][col] != 0), None)
        if piv is None:
            return 0
        if piv != col:
            a[col], a[piv] = a[piv], a[col]
            d = -d
        d = d * a[col][col] % P
        inv = pow(a[col][col], P - 2, P)
        for r in range(col + 1, n):
            f = a[r][col] * inv % P
            if f:
                a[r] = [(vr - f * vc) % P for vr, vc in zip(a[r], a[col])]
    return d % P


class InversePoseidon:
    """Undo one width-12 permutation with round constants rc[30][12] and matrix m:
    rounds in reverse order, each undoing the linear layer (M^-1), then the x^7
    S-box (x^(7^-1 mod p-1)) on the lanes it touched, then the constant addition."""

    def __init__(self, rc, m, full_half=4, rounds=30):
        self.rc = [[int(v) for v in row] for row in rc]
        self.minv = mat_inv([[int(v) for v in row] for row in m])
        self.full_half, self.rounds = full_half, rounds

    def __call__(self, state):
        s = [int(v) % P for v in state]
        for r in reversed(range(self.rounds)):
            full = r < self.full_half or r >= self.rounds - self.full_half
            s = [sum(self.minv[i][j] * s[j] for j in range(12)) % P for i in range(12)]
            for i in range(12 if full else 1):
                s[i] = pow(s[i], D_INV7, P)
            s = [(s[i] - self.rc[r][i]) % P for i in range(12)]
        return s


# ---------------------------------------------------------------- forward permutation

MASK64 = (1 << 64) - 1
SM_GAMMA = 0x9E3779B97F4A7C15
SM_M1, SM_M2 = 0xBF58476D1CE4E5B9, 0x94D049BB133111EB


def splitmix64(seed, i):
    """Output i (0-based) of SplitMix64 started at seed (Steele, Lea, Flood 2014): the
    state advances by the golden-ratio increment before each output, then the
    published finaliser (xor-shift 30, multiply, xor-shift 27, multiply, xor-shift 31)."""
    z = (seed + (i + 1) * SM_GAMMA) & MASK64
    z = ((z ^ (z >> 30)) * SM_M1) & MASK64
    z = ((z ^ (z >> 27)) * SM_M2) & MASK64
    return z ^ (z >> 31)


def splitmix64_seed_for(target, index):
    """A seed whose stream has output `target` at `index`: the finaliser is a bijection
    (xor-shifts and multiplications by odd constants undo), so the state that yields
    target is found by running it backwards, and the seed is that state minus
    (index + 1) increments."""
    def unxorshift(y, s):
        x = y
        for _ in range(64 // s + 1):
            x = y ^ (x >> s)
        return x
    x = unxorshift(target, 31)
    x = (x * pow(SM_M2, -1, 1 << 64)) & MASK64
    x = unxorshift(x, 27)
    x = (x * pow(SM_M1, -1, 1 << 64)) & MASK64
    x = unxorshift(x, 30)
    return (x - (index + 1) * SM_GAMMA) & MASK64


class ForwardPoseidon:
    """The width-12 permutation written directly from its definition with Python
    integers: for each of the 30 rounds, add the round's constants to every lane, raise
    every lane (rounds 0-3 and 26-29) or lane 0 only (the 22 partial rounds) to the 7th
    power, then replace the state by M times it, M[i][j] = circ[(j - i) mod 12]."""

    def __init__(self, rc, circ, full_half=4, rounds=30):
        self.rc = [[int(v) for v in row] for row in rc]
        self.circ = [int(v) for v in circ]
        self.full_half, self.rounds = full_half, rounds

    def __call__(self, state):
        s = [int(v) % P for v in state]
        for r in range(self.rounds):
            full = r < self.full_half or r >= self.rounds - self.full_half
            s = [(s[i] + self.rc[r][i]) % P for i in range(12)]
            for i in range(12 if full else 1):
                s[i] = pow(s[i], 7, P)
            s = [sum(self.circ[(j - i) % 12] * s[j] for j in range(12)) % P for i in range(12)]
        return s

    def sponge(self, row):
        """Zero state; each chunk of up to 8 elements overwrites lanes 0..k-1, then one
        permutation. Returns the whole final state (digest = lanes 0..3)."""
        s = [0] * 12
        for q in range(0, len(row), 8):
            chunk = [int(v) for v in row[q:q + 8]]
            s[:len(chunk)] = chunk
            s = self(s)
        return s

    def compress(self, left, right):
        return self([int(v) for v in left] + [int(v) for v in right] + [0, 0, 0, 0])[:4]
