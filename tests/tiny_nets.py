"""Tiny hand-built networks with closed-form behaviour, used as pins."""
import synth
from synth import COSMIC_RAY, CR_PHOTON, PHOTO, TWO_BODY


def decay(alpha=2.0):
    """A -> B (isomers), cosmic-ray type: k = alpha * zeta."""
    return synth.make_network(
        "decay",
        [("A", {"C": 1, "O": 1}, 0), ("B", {"C": 1, "O": 1}, 0)],
        [(COSMIC_RAY, ["A"], ["B"], alpha, 0.0, 0.0)],
    )


def association(alpha=1e-10, beta=0.0, gamma=0.0):
    """A + B -> C, two-body type."""
    return synth.make_network(
        "assoc",
        [("A", {"C": 1}, 0), ("B", {"O": 1}, 0), ("C", {"C": 1, "O": 1}, 0)],
        [(TWO_BODY, ["A", "B"], ["C"], alpha, beta, gamma)],
    )


def dimer(alpha_f=1e-10, alpha_d=1e-10, gamma_d=1.0):
    """H + H -> H2 (two-body) and H2 -> H + H (photo); steady state in closed form."""
    return synth.make_network(
        "dimer",
        [("H", {"H": 1}, 0), ("H2", {"H": 2}, 0)],
        [(TWO_BODY, ["H", "H"], ["H2"], alpha_f, 0.0, 0.0),
         (PHOTO, ["H2"], ["H", "H"], alpha_d, 0.0, gamma_d)],
    )


def first_order():
    """Only one-body (cosmic-ray and photo) reactions: a linear ODE x' = K x."""
    sp = [("e-", {}, -1), ("H", {"H": 1}, 0), ("H+", {"H": 1}, 1), ("H2", {"H": 2}, 0),
          ("H2+", {"H": 2}, 1), ("CO", {"C": 1, "O": 1}, 0), ("C", {"C": 1}, 0),
          ("O", {"O": 1}, 0), ("C+", {"C": 1}, 1)]
    rx = [
        (COSMIC_RAY, ["H"], ["H+", "e-"], 1.0, 0, 0),
        (COSMIC_RAY, ["H2"], ["H2+", "e-"], 0.9, 0, 0),
        (COSMIC_RAY, ["H2"], ["H", "H"], 0.2, 0, 0),
        (PHOTO, ["H2"], ["H", "H"], 3e-11, 0, 2.5),
        (PHOTO, ["CO"], ["C", "O"], 2e-10, 0, 3.0),
        (PHOTO, ["C"], ["C+", "e-"], 3e-10, 0, 3.0),
        (COSMIC_RAY, ["CO"], ["C+", "O", "e-"], 0.5, 0, 0),
        (PHOTO, ["H2+"], ["H", "H+"], 1e-10, 0, 1.0),
    ]
    return synth.make_network("first-order", sp, rx)


def four_types(albedo=0.6):
    """All four rate laws, cosmic-ray-induced photodissociation among them."""
    sp = [("e-", {}, -1), ("H", {"H": 1}, 0), ("H2", {"H": 2}, 0), ("H+", {"H": 1}, 1), ("CO", {"C": 1, "O": 1}, 0),
          ("C", {"C": 1}, 0), ("O", {"O": 1}, 0), ("C+", {"C": 1}, 1), ("OH", {"H": 1, "O": 1}, 0)]
    rx = [
        (TWO_BODY, ["H", "H"], ["H2"], 3e-17, 0.5, 0.0),
        (TWO_BODY, ["C", "O"], ["CO"], 1e-10, -0.2, 20.0),
        (TWO_BODY, ["O", "H"], ["OH"], 5e-11, 0.3, 10.0),
        (TWO_BODY, ["C+", "e-"], ["C"], 2e-12, -0.6, 0.0),
        (COSMIC_RAY, ["H"], ["H+", "e-"], 0.46, 0.0, 0.0),
        (PHOTO, ["CO"], ["C", "O"], 2e-10, 0.0, 3.5),
        (PHOTO, ["C"], ["C+", "e-"], 3e-10, 0.0, 3.0),
        (CR_PHOTON, ["CO"], ["C", "O"], 1.0, 0.5, 105.0),
        (CR_PHOTON, ["OH"], ["O", "H"], 1.3, 0.0, 509.0),
        (CR_PHOTON, ["C"], ["C+", "e-"], 1.0, 0.0, 1020.0),
    ]
    return synth.make_network("four-types", sp, rx, albedo=albedo)


def hub(n_rx=2100, n_iso=40):
    """One species (H) in n_rx two-body reactions H + A_i -> B_j, more than a
    wave's 64 lanes of 32 entries hold, and one species (Z) in none."""
    sp = ([("H", {"H": 1}, 0), ("Z", {"O": 1}, 0)] + [(f"A{i}", {"C": 1}, 0) for i in range(n_iso)]
          + [(f"B{i}", {"C": 1, "H": 1}, 0) for i in range(n_iso)])
    rx = [(TWO_BODY, ["H", f"A{j % n_iso}"], [f"B{(j // n_iso) % n_iso}"], 1e-10 * (1.0 + 0.37 * (j % 7)),
           0.1 * (j % 3), 5.0 * (j % 5)) for j in range(n_rx)]
    return synth.make_network("hub", sp, rx)
