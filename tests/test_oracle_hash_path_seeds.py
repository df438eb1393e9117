"""The seeds the two linear-layer forms are tested with: the default seed's
circulant has every entry at most 254 (each splits into two signed bytes, so the
bulk hashing kernels use the int8 matrix cores), and seed 53's has an entry of
255 (so they keep the VALU form). Constants from the oracle's own derivation."""


def test_default_seed_entries_split_into_two_signed_bytes(poseidon):
    circ = [int(a) for a in poseidon.circ]
    assert max(circ) <= 254 and all((a + 1) // 2 <= 127 and a // 2 <= 127 and (a + 1) // 2 + a // 2 == a
                                     for a in circ)


def test_seed_53_has_an_entry_of_255(oracle_mod):
    assert 255 in [int(a) for a in oracle_mod.Poseidon(53).circ]
