"""The Box-Muller radius's square root on the GPU is the hardware root
(within one ulp of the exact root) moved to a neighbour where that
neighbour's FMA residual says it is closer.  The noise contract needs the
IEEE round-to-nearest root, because the oracle takes the correctly rounded
sqrt.  This checks the correction on the CPU, exhaustively: for every FP32
argument the radius can take (-0, +0 and [2^-24, 34], i.e. -2 ln u for
u in [2^-24, 1]) and each starting value the hardware may return (the
correctly rounded root and its two neighbours), the corrected value is the
correctly rounded root.  A C model of the correction runs the ~2.4e8
arguments in a few seconds."""
import os
import subprocess
import tempfile

SRC = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>
static float u2f(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }
static uint32_t f2u(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
/* the correction: s within one ulp of sqrt(x); move to a neighbour whose
   residual x - n s says it is closer (rd <= 0: the lower neighbour is at or
   above the root's lower half-way point; ru > 0: the upper one is below) */
static float corrected(float x, float s) {
  const float sd = u2f(f2u(s) - 1u), su = u2f(f2u(s) + 1u);
  const float rd = fmaf(-sd, s, x), ru = fmaf(-su, s, x);
  const float r = (rd <= 0.0f) ? sd : s;
  return (ru > 0.0f) ? su : r;
}
int main(void) {
  long bad = 0, n = 0;
  const uint32_t lo = f2u(0x1p-24f), hi = f2u(34.0f);
  for (uint32_t b = lo; b <= hi; ++b) {
    const float x = u2f(b), t = sqrtf(x);
    const float st[3] = {t, u2f(f2u(t) - 1u), u2f(f2u(t) + 1u)};
    for (int i = 0; i < 3; ++i) {
      ++n;
      if (f2u(corrected(x, st[i])) != f2u(t)) {
        if (bad < 5) printf("x=%a start=%a got=%a want=%a\n", x, st[i], corrected(x, st[i]), t);
        ++bad;
      }
    }
  }
  /* the two zeros keep their sign from the hardware root of a zero */
  if (f2u(corrected(0.0f, 0.0f)) != f2u(0.0f) || f2u(corrected(-0.0f, -0.0f)) != f2u(-0.0f)) ++bad;
  printf("checked %ld bad %ld\n", n, bad);
  return bad != 0;
}
"""


def test_radius_sqrt_correction_is_round_to_nearest():
    with tempfile.TemporaryDirectory() as td:
        c, exe = os.path.join(td, "r.c"), os.path.join(td, "r")
        open(c, "w").write(SRC)
        subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-o", exe, c, "-lm"], check=True)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:]
    assert "bad 0" in r.stdout
