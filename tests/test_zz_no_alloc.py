"""The allocation-free prediction entry point against the allocating one, through the C ABI:
identical ladders and cutoffs on two calls in a row (the second smaller, so that stale
staging contents would show), and a clear refusal above the size limit."""
import numpy as np
import pytest

from paper_2503_10302_amd import ladder, sg

pytestmark = pytest.mark.gpu


def test_noalloc_prediction_equals_the_allocating_entry_point():
    m = ladder.Predictor(ladder.default_params())
    big = ladder._instances(range(300), (8, 10, 12, 15), 98000)
    small = ladder._instances(range(37), (15, 6), 99000)
    for inst in (big, small):
        b_ref, c_ref = m.predict(inst)
        b, c = m.predict_noalloc(inst)
        np.testing.assert_array_equal(b, b_ref)
        np.testing.assert_array_equal(c, c_ref)
        assert np.all(np.diff(b, axis=1) > 0)
    with pytest.raises(sg.SGError) as e:
        m.predict_noalloc([big[0]] * (sg.PREDICT_NOALLOC_MAX + 1))
    assert e.value.code == sg.SG_EINVAL and "exceeds" in str(e.value)
    # the refused call left nothing behind: a valid call after it still matches
    b, c = m.predict_noalloc(small[:5])
    b_ref, c_ref = m.predict(small[:5])
    np.testing.assert_array_equal(b, b_ref)
    np.testing.assert_array_equal(c, c_ref)
    m.close()
