"""Self-contact and self-friction of a rod (App. A.1, Self-collision and
Friction).  Filled in with the self-contact configuration."""


def candidates(rods, sim, p):
    raise NotImplementedError("self-contact oracle not written yet")


def project_pairs(rods, p, pairs, rec):
    raise NotImplementedError("self-contact oracle not written yet")


def friction(rods, sim, x, v, pairs, rec):
    raise NotImplementedError("self-contact oracle not written yet")
