"""Builds the oracle's shared library (test infrastructure only).

``python -m oracle.build`` compiles ``aes_ref.c`` and ``par_run.c`` with gcc
into ``oracle/liboracle.so``.  ``build(out, defines)`` is also used by the
tests that plant a mistake in a private copy of the oracle, to show that the
pins catch it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ("aes_ref.c", "par_run.c")
DEFAULT_LIB = os.path.join(HERE, "liboracle.so")


def build(out=DEFAULT_LIB, defines=(), extra_flags=()):
    """Compile the oracle into the shared library ``out``; returns its path."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
           "-pthread", "-D_POSIX_C_SOURCE=200809L"]
    cmd += ["-D" + d for d in defines]
    cmd += list(extra_flags)
    cmd += [os.path.join(HERE, s) for s in SOURCES]
    tmp = out + ".tmp%d" % os.getpid()
    cmd += ["-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(*sys.argv[1:2]))
