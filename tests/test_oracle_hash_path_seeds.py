"""The seeds the matrix-core linear layer is tested with: it holds each circulant
entry C as the signed byte C - 128 (so every entry 1..255 fits) and gives the
byte sums of each limb from two all-ones rows. The default seed's entries lie
well inside that range; seed 53's circulant has the largest entry, 255 (C - 128 =
127, the signed-byte maximum), and seed 293's both extremes, 1 and 255 (-127 and
127). Constants from the oracle's own derivation."""


def test_default_seed_entries_fit_a_signed_byte_after_the_shift(poseidon):
    circ = [int(a) for a in poseidon.circ]
    assert all(-128 <= a - 128 <= 127 for a in circ) and max(circ) < 255


def test_seed_53_has_an_entry_of_255(oracle_mod):
    circ = [int(a) for a in oracle_mod.Poseidon(53).circ]
    assert 255 in circ and max(a - 128 for a in circ) == 127


def test_seed_293_has_both_extreme_entries(oracle_mod):
    circ = [int(a) for a in oracle_mod.Poseidon(293).circ]
    assert min(circ) == 1 and max(circ) == 255
