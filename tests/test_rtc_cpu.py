"""Runtime compilation of user models, host side (no GPU): the library
compiles a user model with hipRTC for gfx950, reports compiler errors with
their log, and checks the model's M against nvars at compile time."""

import os

import pytest

from paper_2409_12483_amd import abi

HERE = os.path.dirname(os.path.abspath(__file__))

pytestmark = pytest.mark.skipif(not os.path.exists(abi.LIBPATH), reason="libaderdg.so not built")


def _model(name):
    with open(os.path.join(HERE, "models", name)) as f:
        return f.read()


@pytest.mark.parametrize("name,nvars,N,prec", [("burgers.hpp", 1, 3, abi.FP64), ("euler.hpp", 3, 5, abi.FP64),
                                               ("burgers.hpp", 1, 9, abi.FP32_PREDICTOR)])
def test_user_model_compiles_for_gfx950(name, nvars, N, prec):
    ok, log = abi.aderdg_user_compile_check(_model(name), nvars, N, prec)
    assert ok, log


def test_compile_errors_come_back_with_the_log():
    broken = _model("burgers.hpp").replace("q[0] * q[0]", "q[0] * undefined_symbol")
    ok, log = abi.aderdg_user_compile_check(broken, 1, 2)
    assert not ok and "undefined_symbol" in log


def test_nvars_is_checked_against_the_model():
    ok, log = abi.aderdg_user_compile_check(_model("euler.hpp"), 2, 2)
    assert not ok and "nvars" in log


def test_bad_arguments_are_rejected_before_compiling():
    lib = abi.load()
    assert lib.aderdg_user_compile_check(b"struct X {};", 1, 0, 0, None, 0) == abi.ADERDG_E_INVAL
    assert lib.aderdg_user_compile_check(b"struct X {};", 9, 2, 0, None, 0) == abi.ADERDG_E_INVAL
