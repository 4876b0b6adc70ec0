"""The Python binding refuses, before any pointer reaches the library, the
tensors the C ABI cannot check itself: host tensors, groups whose streams
differ in length, outputs shorter than the operation's result. A short or
host buffer passed through would be an out-of-bounds device access instead
of an error. CPU only: no call here reaches a kernel."""
import pytest
import torch

from paper_1509_03838_amd import ne


def host(n, dt=torch.int32):
    return torch.zeros(n, dtype=dt)


@pytest.mark.parametrize("call", [
    lambda: ne.entangle([host(8)] * 3, [host(8, torch.int64)] * 3, 22),
    lambda: ne.entangle_inplace([host(8, torch.int64)] * 3, 22),
    lambda: ne.entangle_operand(host(8), host(8, torch.int64), 22),
    lambda: ne.lsb_apply("conv", [host(8, torch.int64)] * 3, host(4), [host(11, torch.int64)] * 3),
    lambda: ne.extract_recover([host(8, torch.int64)] * 3, 0, [host(8, torch.int64)] * 3, 22),
    lambda: ne.entangle32([host(8)] * 3, [host(8)] * 3, 11),
    lambda: ne.lsb_apply32("scale", [host(8)] * 3, None, [host(8)] * 3, scalar=2),
    lambda: ne.extract_recover32([host(8)] * 3, 1, [host(8)] * 3, 11),
    lambda: ne.plain_apply("conv", [host(8)] * 3, host(4), [host(11, torch.int64)] * 3),
    lambda: ne.checksum([host(8)] * 3, host(8, torch.int64)),
    lambda: ne.checksum_recover([host(8, torch.int64)] * 3, host(8, torch.int64), 1,
                                host(8, torch.int64)),
    lambda: ne.GroupSpec("conv", [host(8)] * 3, host(4), [host(11, torch.int64)] * 3).to_c(),
    lambda: ne.gemm([host(16).view(4, 4)] * 3, host(16).view(4, 4),
                    [host(16, torch.int64).view(4, 4)] * 3),
])
def test_host_tensors_are_refused(call):
    with pytest.raises(ValueError, match="on the GPU"):
        call()


def test_unequal_stream_lengths_are_refused():
    with pytest.raises(ValueError, match="exactly 8"):
        ne._n_of([host(8), host(8), host(7)], None, "c")
    assert ne._n_of([host(8), None, host(8)], None, "c") == 8


def test_explicit_length_needs_every_buffer_that_long():
    assert ne._n_of([host(9), host(8)], 8, "c") == 8
    with pytest.raises(ValueError, match="at least 8"):
        ne._n_of([host(9), host(7)], 8, "c")


def test_short_outputs_are_refused():
    ne._lengths("out", [host(11), host(12)], 11, exact=False)
    with pytest.raises(ValueError, match=r"out\[1\] holds 10"):
        ne._lengths("out", [host(11), host(10)], 11, exact=False)


def test_other_devices_are_refused():
    meta = torch.empty(8, dtype=torch.int32, device="meta")
    with pytest.raises(ValueError):
        ne._on_device("c", [meta])


def test_raw_addresses_and_none_are_left_to_the_caller():
    assert ne._on_device("c", [None, 0x1000]) is None
    ne._lengths("d", [None, 0x1000], 5, exact=True)


def test_group_needs_one_output_per_stream():
    with pytest.raises(ValueError, match="one output per input"):
        ne.GroupSpec("scale", [host(8)] * 3, None, [host(8, torch.int64)] * 2).to_c()


def test_operand_dtype_follows_the_operation():
    # add and sub on entangled words take the entangled int64 operand
    with pytest.raises(TypeError, match="operand must be torch.int64"):
        ne.lsb_apply("add", [host(8, torch.int64)] * 3, host(8), [host(8, torch.int64)] * 3)
    with pytest.raises(TypeError, match="operand must be torch.int32"):
        ne.lsb_apply("conv", [host(8, torch.int64)] * 3, host(4, torch.int64),
                     [host(11, torch.int64)] * 3)
