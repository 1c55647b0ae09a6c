"""Writes closed_forms.json: constants that follow from Eq. (1) of the paper
(Morlet wavelet psi(t) = exp(-t^2/2) cos(5t), 1/sqrt(a) normalisation) by
exact integration, evaluated with mpmath at 40 digits.  It calls neither the
oracle nor the library.

  tap_energy      = int psi(u)^2 du            = (sqrt(pi)/2) (1 + e^-25)
  dc_gain_unit    = int psi(u) du              = sqrt(2 pi) e^-12.5
                    (sum of the taps at scale s -> sqrt(s) * dc_gain_unit)
  tone_gain_unit  = sqrt(pi/2): the response to cos(W n + phi) at scale s is
                    sqrt(s) * tone_gain_unit * [e^{-(sW-5)^2/2} + e^{-(sW+5)^2/2}]
                    * cos(W b + phi)
  peak_y          = (5 + sqrt 27)/2: |W| over s peaks where s*W = peak_y
"""
import json
import os

import mpmath as mp

mp.mp.dps = 40


def main():
    psi = lambda u: mp.exp(-u * u / 2) * mp.cos(5 * u)
    out = {
        "tap_energy": {
            "value": mp.nstr(mp.sqrt(mp.pi) / 2 * (1 + mp.exp(-25)), 30),
            "quad": mp.nstr(mp.quad(lambda u: psi(u) ** 2, [-mp.inf, 0, mp.inf]), 30),
            "source": "Eq. (1), Sec. II-A: energy of the 1/sqrt(a)-normalised Morlet",
        },
        "dc_gain_unit": {
            "value": mp.nstr(mp.sqrt(2 * mp.pi) * mp.exp(-mp.mpf(25) / 2), 30),
            "quad": mp.nstr(mp.quad(psi, [-mp.inf, 0, mp.inf]), 30),
            "source": "Eq. (1): response to a constant signal",
        },
        "tone_gain_unit": {
            "value": mp.nstr(mp.sqrt(mp.pi / 2), 30),
            "source": "Eq. (1): Fourier transform of psi, evaluated for a sinusoid",
        },
        "peak_y": {
            "value": mp.nstr((5 + mp.sqrt(27)) / 2, 30),
            "source": "stationary point of sqrt(s) exp(-(s W - 5)^2 / 2) over s",
        },
        "peak_example_500hz_16khz": {
            "value": mp.nstr((5 + mp.sqrt(27)) / 2 / (2 * mp.pi * 500 / 16000), 30),
            "source": "s* for a 500 Hz tone sampled at 16 kHz (fs of Sec. III-A)",
        },
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "closed_forms.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
